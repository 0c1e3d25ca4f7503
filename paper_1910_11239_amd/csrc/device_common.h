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
// interface blocks B_t.  One cell per workgroup (operator_block below): the
// cell and its face neighbours are staged in LDS, every thread applies the
// 1-D operators along one line of the cell for each axis, then the transverse
// mass matrices are applied line by line in LDS.
template <int D, int N1>
struct OpCfg {
    static constexpr int NC = ipow(N1, D);
    static constexpr int LINES = ipow(N1, D - 1);
    // one cell per workgroup: every 1-D table address is uniform (scalar loads)
    static constexpr int THREADS = LINES <= 64 ? 64 : rup64(LINES);
    static constexpr int PPB = 1;
};

template <int D, int N1, typename P>
__device__ __forceinline__ void mass_line(const double *src, double *dst, int a, int l, double scale, P Mh,
                                          bool acc) {
    const int base = line_base<D, N1>(a, l), st = line_stride<N1>(a);
    double in[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) in[i] = src[base + i * st];
#pragma unroll
    for (int o = 0; o < N1; ++o) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < N1; ++i) s = fma((double)Mh[o * N1 + i], in[i], s);
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
// (x, b, y: that mesh's vectors).  Shared by the single-mesh and the batched
// kernels.  The block's cells and their 2d face neighbours are first copied
// into LDS with coalesced whole-cell loads (slot 0 = the cell, slots 1..2d =
// neighbours -x, +x, -y, +y, -z, +z; absent neighbours are skipped); each
// thread then applies the 1-D operators along its line of each axis
// (cell block + the two interface blocks), keeps the d results in registers,
// and after a barrier the transverse mass matrices are applied in LDS reusing
// the neighbour slots.
template <int D, int N1, bool RES>
__device__ __forceinline__ void operator_block(const LevelView &g, int64_t cell0, const double *__restrict__ x,
                                               const double *__restrict__ b, double *__restrict__ y) {
    using C = OpCfg<D, N1>;
    constexpr int NC = C::NC, LINES = C::LINES, PPB = C::PPB, TH = C::THREADS;
    constexpr int NS = 2 * D + 1;  // LDS slots per cell
    __shared__ double S[PPB][NS][NC];
    __shared__ int64_t src_cell[PPB][NS];  // -1: absent
    const int t = threadIdx.x;
    const int q = t / LINES, l = t % LINES;
    const int64_t cs[3] = {1, g.m[0], (int64_t)g.m[0] * g.m[1]};
    for (int e = t; e < PPB * NS; e += TH) {
        const int qq = e / NS, slot = e % NS;
        const int64_t cc = cell0 + qq;
        int64_t src = cc < g.ncells ? cc : -1;
        if (src >= 0 && slot > 0) {
            int c3[3];
            cell_coords(cc, g.m, c3);
            const int a = (slot - 1) >> 1, dir = (slot - 1) & 1;  // dir 0: -e_a, 1: +e_a
            const int nb = c3[a] + (dir ? 1 : -1);
            src = (nb < 0 || nb >= g.m[a]) ? -1 : cc + (dir ? cs[a] : -cs[a]);
        }
        src_cell[qq][slot] = src;
    }
    __syncthreads();
    // stage cells and neighbours (whole cells, coalesced); loads are issued in
    // chunks of independent registers before the LDS stores
    constexpr int TOT = PPB * NS * NC, ITER = (TOT + TH - 1) / TH, CH = 8;
#pragma unroll
    for (int k0 = 0; k0 < ITER; k0 += CH) {
        double v[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int p = t + (k0 + k) * TH;
            v[k] = 0.0;
            if (k0 + k < ITER && p < TOT) {
                const int qs = p / NC, i = p % NC;
                const int64_t src = src_cell[qs / NS][qs % NS];
                if (src >= 0) v[k] = x[src * NC + i];
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int p = t + (k0 + k) * TH;
            if (k0 + k < ITER && p < TOT) {
                const int qs = p / NC, i = p % NC;
                S[qs / NS][qs % NS][i] = v[k];
            }
        }
    }
    __syncthreads();
    const int64_t cell = cell0 + q;
    const bool act = (q < PPB) && (cell < g.ncells);
    // PPB == 1: the cell, its coordinates and all table addresses are uniform
    int c[3] = {0, 0, 0};
    cell_coords(cell0 < g.ncells ? cell0 : 0, g.m, c);
    for (int a = 0; a < 3; ++a) c[a] = __builtin_amdgcn_readfirstlane(c[a]);
    const double hx = uniform_table(g.h[0])[c[0]], hy = uniform_table(g.h[1])[c[1]];
    const double hz = D == 3 ? (double)uniform_table(g.h[2])[c[2]] : 1.0;
    double w[D][N1];
    if (act) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int base = line_base<D, N1>(a, l), st = line_stride<N1>(a);
            double in[N1];
#pragma unroll
            for (int i = 0; i < N1; ++i) in[i] = S[q][0][base + i * st];
            cptr<double> A = uniform_table(g.cellop[a] + (size_t)c[a] * N1 * N1);
#pragma unroll
            for (int o = 0; o < N1; ++o) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < N1; ++i) s = fma((double)A[o * N1 + i], in[i], s);
                w[a][o] = s;
            }
            if (c[a] + 1 < g.m[a]) {
#pragma unroll
                for (int i = 0; i < N1; ++i) in[i] = S[q][2 + 2 * a][base + i * st];
                cptr<double> B = uniform_table(g.iface[a] + (size_t)c[a] * N1 * N1);
#pragma unroll
                for (int o = 0; o < N1; ++o)
#pragma unroll
                    for (int i = 0; i < N1; ++i) w[a][o] = fma((double)B[o * N1 + i], in[i], w[a][o]);
            }
            if (c[a] > 0) {
#pragma unroll
                for (int i = 0; i < N1; ++i) in[i] = S[q][1 + 2 * a][base + i * st];
                cptr<double> B = uniform_table(g.iface[a] + (size_t)(c[a] - 1) * N1 * N1);
#pragma unroll
                for (int o = 0; o < N1; ++o)
#pragma unroll
                    for (int i = 0; i < N1; ++i) w[a][o] = fma((double)B[i * N1 + o], in[i], w[a][o]);
            }
        }
    }
    __syncthreads();  // neighbour slots are free from here on
    double *W0 = S[q][1], *W1 = S[q][2], *U = D == 3 ? S[q][4] : S[q][3];
    if (act) {
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int base = line_base<D, N1>(a, l), st = line_stride<N1>(a);
            double *Wa = S[q][1 + a];
#pragma unroll
            for (int o = 0; o < N1; ++o) Wa[base + o * st] = w[a][o];
        }
    }
    __syncthreads();
    cptr<double> Mh = uniform_table(g.Mhat);
    double *Y;
    if constexpr (D == 2) {
        if (act) mass_line<D, N1>(W0, U, 1, l, hy, Mh, false);
        __syncthreads();
        if (act) mass_line<D, N1>(W1, U, 0, l, hx, Mh, true);
        __syncthreads();
        Y = U;
    } else {
        double *W2 = S[q][3], *X2 = S[q][5];
        // U = hy hz (Mhat_y W_x) + hx hz (Mhat_x W_y);  X2 = Mhat_y W_z
        if (act) mass_line<D, N1>(W0, U, 1, l, hy * hz, Mh, false);
        __syncthreads();
        if (act) {
            mass_line<D, N1>(W1, U, 0, l, hx * hz, Mh, true);
            mass_line<D, N1>(W2, X2, 1, l, 1.0, Mh, false);
        }
        __syncthreads();
        // W0 = Mhat_z U;  W0 += hx hy Mhat_x X2
        if (act) mass_line<D, N1>(U, W0, 2, l, 1.0, Mh, false);
        __syncthreads();
        if (act) mass_line<D, N1>(X2, W0, 0, l, hx * hy, Mh, true);
        __syncthreads();
        Y = W0;
    }
    (void)Y;
    for (int p = t; p < PPB * NC; p += TH) {
        const int qq = p / NC, i = p % NC;
        const int64_t cc = cell0 + qq;
        if (cc < g.ncells) {
            const int64_t gi = cc * NC + i;
            const double v = S[qq][1][i];  // W0 of cell qq holds the result (U for 2-D)
            const double yv = D == 3 ? v : S[qq][3][i];
            y[gi] = RES ? b[gi] - yv : yv;
        }
    }
}

}  // namespace fts
