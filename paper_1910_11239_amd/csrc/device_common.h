// Device helpers shared by the HIP kernels: tensor line geometry, the
// "one thread per 1-D line" contractions, launch configurations, and the
// (dimension, degree) dispatch to template instances.
#pragma once

#include "fts_internal.h"

namespace fts {

constexpr int ipow(int b, int e) {
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}
constexpr int rup64(int x) { return (x + 63) / 64 * 64; }

// Offset of the first element and stride of line l along axis a of a
// D-dimensional tensor with extent N per axis (x fastest).  Lines enumerate
// the remaining coordinates with the lower axis fastest.
template <int D, int N>
__device__ __forceinline__ int line_base(int a, int l) {
    if constexpr (D == 2) {
        return a == 0 ? l * N : l;
    } else {
        const int u = l % N, v = l / N;
        if (a == 0) return u * N + v * N * N;
        if (a == 1) return u + v * N * N;
        return u + v * N;
    }
}
template <int N>
__device__ __forceinline__ int line_stride(int a) {
    return a == 0 ? 1 : (a == 1 ? N : N * N);
}

__device__ __forceinline__ void cell_coords(int64_t cell, const int *m, int *c) {
    c[0] = (int)(cell % m[0]);
    const int64_t r = cell / m[0];
    c[1] = (int)(r % m[1]);
    c[2] = (int)(r / m[1]);
}

// ---------------------------------------------------------------------------
// SIPG operator (Sec. 3.2, eq. KDseparable / bulkcart / 1Dsipg): on a
// rectilinear mesh the operator restricted to the rows of cell K is
//   (A x)_K = sum_t (prod_{s != t} h_s) (Mhat x..x W_t x..x Mhat)
//   W_t = A_t^K x_K + B_t(K, K+e_t) x_{K+e_t} + B_t(K-e_t, K)^T x_{K-e_t}
// with the 1-D cell operator A_t^K (both faces' Nitsche terms) and the
// interface blocks B_t.  Each block of PPB cells: 1) every thread applies the
// 1-D operator along one line of its cell for each axis, reading the
// neighbour lines from global memory; 2) the transverse mass matrices are
// applied line by line in LDS.
template <int D, int N1>
struct OpCfg {
    static constexpr int NC = ipow(N1, D);
    static constexpr int LINES = ipow(N1, D - 1);
    static constexpr int THREADS = LINES <= 64 ? 64 : rup64(LINES);
    static constexpr int PPB = THREADS / LINES;
};

template <int D, int N1>
__device__ __forceinline__ void mass_line(const double *src, double *dst, int a, int l, double scale,
                                          const double *Mh, bool acc) {
    const int base = line_base<D, N1>(a, l), st = line_stride<N1>(a);
    double in[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) in[i] = src[base + i * st];
#pragma unroll
    for (int o = 0; o < N1; ++o) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < N1; ++i) s = fma(Mh[o * N1 + i], in[i], s);
        s *= scale;
        dst[base + o * st] = acc ? dst[base + o * st] + s : s;
    }
}

template <int D, int N1, int KIND>
struct SwCfg {
    static constexpr int N = KIND ? 2 * N1 : N1;
    static constexpr int NT = ipow(N, D);
    static constexpr int NC1 = ipow(N1, D);
    static constexpr int NSC = KIND ? (1 << D) : 1;
    static constexpr int LINES = ipow(N, D - 1);
    static constexpr int THREADS = LINES <= 64 ? 64 : rup64(LINES);
    static constexpr int PPB = THREADS / LINES;
};

struct SubGrid {
    int cnt[3];    // subdomains per axis in this launch
    int first[3];  // position of the first subdomain per axis
    int step;      // 1 (cells) or 2 (one parquet color of vertex patches)
    int64_t nsub;
};

template <typename T>
struct EigTab;
template <>
struct EigTab<double> {
    static __device__ __forceinline__ const double *S(const EigView &e, int a) { return e.S[a]; }
    static __device__ __forceinline__ const double *ST(const EigView &e, int a) { return e.ST[a]; }
    static __device__ __forceinline__ const double *L(const EigView &e, int a) { return e.lam[a]; }
};
template <>
struct EigTab<float> {
    static __device__ __forceinline__ const float *S(const EigView &e, int a) { return e.S32[a]; }
    static __device__ __forceinline__ const float *ST(const EigView &e, int a) { return e.ST32[a]; }
    static __device__ __forceinline__ const float *L(const EigView &e, int a) { return e.lam32[a]; }
};

// Read-only tables addressed uniformly by a whole workgroup are read through
// the constant address space, so the compiler issues scalar loads and the
// FMAs take their matrix operand from scalar registers.
template <typename T>
using cptr = const T __attribute__((address_space(4))) *;
template <typename T>
__device__ __forceinline__ cptr<T> uniform_table(const T *p) {
    return (cptr<T>)(p);
}

// out[o] = sum_j Mat[o][j] in[j] on one line (Mat row-major, rows contiguous).
template <int N, typename T, typename P>
__device__ __forceinline__ void matvec_regs(const T *in, T *out, P Mat) {
#pragma unroll
    for (int o = 0; o < N; ++o) {
        T s = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) s = fma((T)Mat[o * N + j], in[j], s);
        out[o] = s;
    }
}

template <int D, int N, typename T, typename P>
__device__ __forceinline__ void contract_line(T *Tq, int a, int l, P Mat) {
    const int base = line_base<D, N>(a, l), st = line_stride<N>(a);
    T in[N], out[N];
#pragma unroll
    for (int i = 0; i < N; ++i) in[i] = Tq[base + i * st];
    matvec_regs<N>(in, out, Mat);
#pragma unroll
    for (int i = 0; i < N; ++i) Tq[base + i * st] = out[i];
}

// Last axis: forward transform, eigenvalue scaling and backward transform of
// the same line, kept in registers.  lam_rest = lambda of the other axes at
// this line's fixed mode indices.
template <int D, int N, typename T, typename P, typename Q>
__device__ __forceinline__ void last_axis_solve(T *Tq, int l, P ST, P S, Q lam_last, T lam_rest, T omega) {
    constexpr int a = D - 1;
    const int base = line_base<D, N>(a, l), st = line_stride<N>(a);
    T in[N], mid[N];
#pragma unroll
    for (int i = 0; i < N; ++i) in[i] = Tq[base + i * st];
    matvec_regs<N>(in, mid, ST);
#pragma unroll
    for (int m = 0; m < N; ++m) mid[m] = mid[m] * (omega / (lam_rest + (T)lam_last[m]));
    matvec_regs<N>(mid, in, S);
#pragma unroll
    for (int i = 0; i < N; ++i) Tq[base + i * st] = in[i];
}

// ---------------------------------------------------------------------------
// Dispatch on (dim, degree) to the template instances.
template <template <int, int> class F, typename... Args>
fts_status dispatch(int dim, int n1, Args &&...args) {
#define FTS_CASE(DD, NN) \
    if (dim == DD && n1 == NN) return F<DD, NN>::run(args...);
    FTS_CASE(2, 2) FTS_CASE(2, 3) FTS_CASE(2, 4) FTS_CASE(2, 5) FTS_CASE(2, 6) FTS_CASE(2, 7)
    FTS_CASE(2, 8) FTS_CASE(2, 9) FTS_CASE(2, 10)
    FTS_CASE(3, 2) FTS_CASE(3, 3) FTS_CASE(3, 4) FTS_CASE(3, 5) FTS_CASE(3, 6) FTS_CASE(3, 7)
    FTS_CASE(3, 8) FTS_CASE(3, 9) FTS_CASE(3, 10)
#undef FTS_CASE
    return fail(FTS_E_UNSUPPORTED, "dimension/degree combination not built");
}

inline fts_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return FTS_OK;
}


// Body of the operator for the PPB cells cell0.. of the mesh described by g
// (x, b, y: that mesh's vectors).  Shared by the single-mesh and the batched kernels.
template <int D, int N1, bool RES>
__device__ __forceinline__ void operator_block(const LevelView &g, int64_t cell0, const double *__restrict__ x,
                                               const double *__restrict__ b, double *__restrict__ y) {
    using C = OpCfg<D, N1>;
    constexpr int NC = C::NC, LINES = C::LINES, PPB = C::PPB, TH = C::THREADS;
    __shared__ double X[PPB * NC];
    __shared__ double W[D][PPB * NC];
    __shared__ double U[PPB * NC];
    const int t = threadIdx.x;
    const int q = t / LINES, l = t % LINES;
    for (int p = t; p < PPB * NC; p += TH) {
        const int64_t cc = cell0 + p / NC;
        X[p] = cc < g.ncells ? x[cc * NC + p % NC] : 0.0;
    }
    __syncthreads();
    const int64_t cell = cell0 + q;
    const bool act = (q < PPB) && (cell < g.ncells);
    int c[3] = {0, 0, 0};
    if (act) cell_coords(cell, g.m, c);
    const int64_t cs[3] = {1, g.m[0], (int64_t)g.m[0] * g.m[1]};
    const double hx = act ? g.h[0][c[0]] : 0.0, hy = act ? g.h[1][c[1]] : 0.0;
    const double hz = (D == 3 && act) ? g.h[2][c[2]] : 1.0;
    const int qo = q * NC;
    if (act) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int base = line_base<D, N1>(a, l), st = line_stride<N1>(a);
            double in[N1], out[N1];
#pragma unroll
            for (int i = 0; i < N1; ++i) in[i] = X[qo + base + i * st];
            const double *A = g.cellop[a] + (size_t)c[a] * N1 * N1;
#pragma unroll
            for (int o = 0; o < N1; ++o) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < N1; ++i) s = fma(A[o * N1 + i], in[i], s);
                out[o] = s;
            }
            if (c[a] + 1 < g.m[a]) {
                const double *nb = x + (cell + cs[a]) * NC;
#pragma unroll
                for (int i = 0; i < N1; ++i) in[i] = nb[base + i * st];
                const double *B = g.iface[a] + (size_t)c[a] * N1 * N1;
#pragma unroll
                for (int o = 0; o < N1; ++o)
#pragma unroll
                    for (int i = 0; i < N1; ++i) out[o] = fma(B[o * N1 + i], in[i], out[o]);
            }
            if (c[a] > 0) {
                const double *nb = x + (cell - cs[a]) * NC;
#pragma unroll
                for (int i = 0; i < N1; ++i) in[i] = nb[base + i * st];
                const double *B = g.iface[a] + (size_t)(c[a] - 1) * N1 * N1;
#pragma unroll
                for (int o = 0; o < N1; ++o)
#pragma unroll
                    for (int i = 0; i < N1; ++i) out[o] = fma(B[i * N1 + o], in[i], out[o]);
            }
#pragma unroll
            for (int o = 0; o < N1; ++o) W[a][qo + base + o * st] = out[o];
        }
    }
    __syncthreads();
    const double *Mh = g.Mhat;
    double *Y;
    if constexpr (D == 2) {
        if (act) mass_line<D, N1>(W[0] + qo, U + qo, 1, l, hy, Mh, false);
        __syncthreads();
        if (act) mass_line<D, N1>(W[1] + qo, U + qo, 0, l, hx, Mh, true);
        __syncthreads();
        Y = U;
    } else {
        // U = hy hz (Mhat_y W_x) + hx hz (Mhat_x W_y);  X = Mhat_y W_z
        if (act) mass_line<D, N1>(W[0] + qo, U + qo, 1, l, hy * hz, Mh, false);
        __syncthreads();
        if (act) {
            mass_line<D, N1>(W[1] + qo, U + qo, 0, l, hx * hz, Mh, true);
            mass_line<D, N1>(W[2] + qo, X + qo, 1, l, 1.0, Mh, false);
        }
        __syncthreads();
        // W0 = Mhat_z U
        if (act) mass_line<D, N1>(U + qo, W[0] + qo, 2, l, 1.0, Mh, false);
        __syncthreads();
        // W0 += hx hy Mhat_x X
        if (act) mass_line<D, N1>(X + qo, W[0] + qo, 0, l, hx * hy, Mh, true);
        __syncthreads();
        Y = W[0];
    }
    for (int p = t; p < PPB * NC; p += TH) {
        const int64_t cc = cell0 + p / NC;
        if (cc < g.ncells) {
            const int64_t gi = cc * NC + p % NC;
            y[gi] = RES ? b[gi] - Y[p] : Y[p];
        }
    }
}

}  // namespace fts
