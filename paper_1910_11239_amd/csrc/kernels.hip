// HIP kernels for gfx950: matrix-free SIPG operator, fast-diagonalisation
// Schwarz local solves on cells and vertex patches (FP64 / FP32 on the vector
// units, FP64 and 16-bit variants on MFMA), grid transfers, the slab-blocked
// assembly of the coarse matrix and the BLAS-1 kernels of CG and GMRES.
//
// Data layout: vectors are cell-major (cells lexicographic, x fastest), each
// cell holding (k+1)^d FP64 coefficients lexicographic with x fastest.  A
// subdomain tensor of extent N per axis lives in LDS with x fastest.
// Contractions are "one thread per 1-D line": a thread owns a line of the
// tensor along one axis, keeps it in registers and applies the N x N 1-D
// matrix, so each LDS value is read once per contraction.
#include "device_common.h"

namespace fts {

template <int D, int N1, bool RES, bool PEN, typename TY = double>
__global__ void __launch_bounds__((OpCfg<D, N1>::THREADS))
k_operator(LevelView g, OpRuns runs, const double *__restrict__ x, const double *__restrict__ b,
           TY *__restrict__ y) {
    int64_t cell0;
    int nact;
    op_run_of_block(runs, blockIdx.x, &cell0, &nact);
    operator_cells<D, N1, RES, PEN, TY>(g, cell0, nact, x, b, y);
}

// ---------------------------------------------------------------------------
// Schwarz local solves (Sec. 3.2, eq. fastinverse / eigenvectormatvec):
//   x += omega * R_j^T (S x..x S) diag(1/Lambda) (S x..x S)^T R_j r
// for a batch of subdomains (cells, or vertex patches of one parquet color).
// KIND 0: cells, tensor extent N = k+1; KIND 1: vertex patches, N = 2(k+1),
// local index a_t = (cell offset)_t (k+1) + i_t.  T is the contraction type.
// STAGE = false: x += correction (the subdomains of one launch must not share
// cells: cells, or one parquet color of vertex patches).  STAGE = true: the
// correction of subdomain s is written to W[s][cell of the subdomain][DoF] in
// the contraction type T and k_patch_gather adds the contributions to x in
// FP64 in a fixed order.
template <int D, int N1, int KIND, typename T, bool STAGE>
__device__ __forceinline__ void schwarz_generic(const LevelView &g, const EigView &e, const SubGrid &sg,
                                                const double *__restrict__ r, double *__restrict__ x,
                                                T *__restrict__ W, double omega, T *Ts) {
    using C = SwCfg<D, N1, KIND>;
    constexpr int N = C::N, NT = C::NT, NC1 = C::NC1, NSC = C::NSC, LINES = C::LINES, PPB = C::PPB,
                  TH = C::THREADS;
    const int t = threadIdx.x;
    const int q = t / LINES, l = t % LINES;
    const int64_t s0 = (int64_t)blockIdx.x * PPB;

    // subdomain -> per-axis position (anchor cell of a patch = vertex - 1)
    auto position = [&](int64_t s, int *p) {
        const int j0 = (int)(s % sg.cnt[0]);
        const int64_t rr = s / sg.cnt[0];
        const int j1 = (int)(rr % sg.cnt[1]);
        const int j2 = (int)(rr / sg.cnt[1]);
        p[0] = sg.first[0] + sg.step * j0;
        p[1] = sg.first[1] + sg.step * j1;
        p[2] = D == 3 ? sg.first[2] + sg.step * j2 : 0;
    };
    const int64_t cs1 = g.m[0], cs2 = (int64_t)g.m[0] * g.m[1];
    // gather R_j r: flat over (subdomain, cell of the subdomain, local DoF)
    for (int p = t; p < PPB * NSC * NC1; p += TH) {
        const int qq = p / (NSC * NC1), rem = p % (NSC * NC1), sc = rem / NC1, i = rem % NC1;
        const int64_t s = s0 + qq;
        if (s >= sg.nsub || !sub_in_color(sg, s)) continue;
        int pos[3];
        position(s, pos);
        const int o0 = sc & 1, o1 = (sc >> 1) & 1, o2 = (sc >> 2) & 1;
        const int64_t cell = (pos[0] + o0) + (pos[1] + o1) * cs1 + (D == 3 ? (pos[2] + o2) * cs2 : 0);
        const int i0 = i % N1, i1 = (i / N1) % N1, i2 = D == 3 ? i / (N1 * N1) : 0;
        const int lds = (o0 * N1 + i0) + (o1 * N1 + i1) * N + (D == 3 ? (o2 * N1 + i2) * N * N : 0);
        Ts[qq * NT + lds] = (T)r[cell * NC1 + i];
    }
    __syncthreads();
    const int64_t s = s0 + q;
    const bool act = (q < PPB) && (s < sg.nsub) && sub_in_color(sg, s);
    T *Tq = Ts + q * NT;
    const T om = (T)omega;
    // mode indices of this thread's line along the last axis (fixed coordinates of the other axes)
    const int ml0 = l % N, ml1 = (l / N) % N;
    if constexpr (PPB == 1) {
        // one subdomain per workgroup: every table address is uniform
        int pos[3];
        position(s0, pos);
        for (int a = 0; a < 3; ++a) pos[a] = __builtin_amdgcn_readfirstlane(pos[a]);
        int tp[3] = {0, 0, 0};  // table positions (EigView::cls)
        for (int a = 0; a < D; ++a) tp[a] = __builtin_amdgcn_readfirstlane(e.cls[a][pos[a]]);
        const int nn = N * N;
        if (act) contract_line<D, N, T>(Tq, 0, l, uniform_table(EigTab<T>::ST(e, 0) + (size_t)tp[0] * nn));
        __syncthreads();
        if constexpr (D == 3) {
            if (act) contract_line<D, N, T>(Tq, 1, l, uniform_table(EigTab<T>::ST(e, 1) + (size_t)tp[1] * nn));
            __syncthreads();
        }
        if (act) {
            constexpr int a = D - 1;
            cptr<T> L0 = uniform_table(EigTab<T>::L(e, 0) + (size_t)tp[0] * N);
            T lr = (T)L0[ml0];
            if constexpr (D == 3) lr += (T)uniform_table(EigTab<T>::L(e, 1) + (size_t)tp[1] * N)[ml1];
            last_axis_solve<D, N, T>(Tq, l, uniform_table(EigTab<T>::ST(e, a) + (size_t)tp[a] * nn),
                                     uniform_table(EigTab<T>::S(e, a) + (size_t)tp[a] * nn),
                                     uniform_table(EigTab<T>::L(e, a) + (size_t)tp[a] * N), lr, om);
        }
        __syncthreads();
        if constexpr (D == 3) {
            if (act) contract_line<D, N, T>(Tq, 1, l, uniform_table(EigTab<T>::S(e, 1) + (size_t)tp[1] * nn));
            __syncthreads();
        }
        if (act) contract_line<D, N, T>(Tq, 0, l, uniform_table(EigTab<T>::S(e, 0) + (size_t)tp[0] * nn));
        __syncthreads();
    } else {
        int pos[3] = {0, 0, 0};
        if (act) position(s, pos);
        int tp[3] = {0, 0, 0};
        if (act)
            for (int a = 0; a < D; ++a) tp[a] = e.cls[a][pos[a]];
        const int nn = N * N;
        if (act) contract_line<D, N, T>(Tq, 0, l, EigTab<T>::ST(e, 0) + (size_t)tp[0] * nn);
        __syncthreads();
        if constexpr (D == 3) {
            if (act) contract_line<D, N, T>(Tq, 1, l, EigTab<T>::ST(e, 1) + (size_t)tp[1] * nn);
            __syncthreads();
        }
        if (act) {
            constexpr int a = D - 1;
            T lr = EigTab<T>::L(e, 0)[(size_t)tp[0] * N + ml0];
            if constexpr (D == 3) lr += EigTab<T>::L(e, 1)[(size_t)tp[1] * N + ml1];
            last_axis_solve<D, N, T>(Tq, l, EigTab<T>::ST(e, a) + (size_t)tp[a] * nn,
                                     EigTab<T>::S(e, a) + (size_t)tp[a] * nn,
                                     EigTab<T>::L(e, a) + (size_t)tp[a] * N, lr, om);
        }
        __syncthreads();
        if constexpr (D == 3) {
            if (act) contract_line<D, N, T>(Tq, 1, l, EigTab<T>::S(e, 1) + (size_t)tp[1] * nn);
            __syncthreads();
        }
        if (act) contract_line<D, N, T>(Tq, 0, l, EigTab<T>::S(e, 0) + (size_t)tp[0] * nn);
        __syncthreads();
    }
    // scatter-add R_j^T
    for (int p = t; p < PPB * NSC * NC1; p += TH) {
        const int qq = p / (NSC * NC1), rem = p % (NSC * NC1), sc = rem / NC1, i = rem % NC1;
        const int64_t ss = s0 + qq;
        if (ss >= sg.nsub || !sub_in_color(sg, ss)) continue;
        int ps[3];
        position(ss, ps);
        const int o0 = sc & 1, o1 = (sc >> 1) & 1, o2 = (sc >> 2) & 1;
        const int64_t cell = (ps[0] + o0) + (ps[1] + o1) * cs1 + (D == 3 ? (ps[2] + o2) * cs2 : 0);
        const int i0 = i % N1, i1 = (i / N1) % N1, i2 = D == 3 ? i / (N1 * N1) : 0;
        const int lds = (o0 * N1 + i0) + (o1 * N1 + i1) * N + (D == 3 ? (o2 * N1 + i2) * N * N : 0);
        if constexpr (STAGE) {
            W[ss * (NSC * NC1) + rem] = Ts[qq * NT + lds];
        } else {
            const int64_t gi = cell * NC1 + i;
            x[gi] = x[gi] + (double)Ts[qq * NT + lds];
        }
    }
}

// 3-D, one subdomain per workgroup: thread l < N^2 owns the line along the
// first axis with the other two local indices (a1, a2) = (l % N, l / N).  It
// reads its line of the residual straight from global memory (2 runs of k+1
// contiguous values for a patch, one for a cell), applies the first forward
// contraction in registers and only then goes through LDS for the other
// axes; the last backward contraction also ends in registers and is written
// to the staging buffer (or added to x) directly.  Index arithmetic happens
// once per thread, not once per element.
//
// Tables of one subdomain: S and S^T per axis, the eigenvalues along z and
// the sum of the x and y eigenvalues of this thread's z-line.
template <typename T>
struct PatchTabs {
    cptr<T> S[3], ST[3], lam2;
    T lr;
};

template <typename T, int N>
__device__ __forceinline__ PatchTabs<T> patch_tabs(const EigView &e, const int *tp, bool act, int a1, int a2) {
    constexpr int nn = N * N;
    PatchTabs<T> pt;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pt.S[a] = uniform_table(EigTab<T>::S(e, a) + (size_t)tp[a] * nn);
        pt.ST[a] = uniform_table(EigTab<T>::ST(e, a) + (size_t)tp[a] * nn);
    }
    pt.lam2 = uniform_table(EigTab<T>::L(e, 2) + (size_t)tp[2] * N);
    // the z-line l has mode indices (l % N, l / N) along x and y (idle
    // threads l >= N^2 read mode 0)
    pt.lr = (T)uniform_table(EigTab<T>::L(e, 0) + (size_t)tp[0] * N)[act ? a1 : 0] +
            (T)uniform_table(EigTab<T>::L(e, 1) + (size_t)tp[1] * N)[act ? a2 : 0];
    return pt;
}

// The local solve of one subdomain: src = this thread's line of the residual
// (NO runs of N1 values, NC1 apart); on return w holds the thread's line of
// the correction.  EO: even-odd contractions (mirror-symmetric eigenbases
// along all three axes, EigView::sym).  Ts: N^3 values of LDS; the function
// starts and ends with every thread free to use its own part of Ts.
template <int N, int N1, int NO, int NC1, typename T, bool EO>
__device__ __forceinline__ void lines3_solve(const double *__restrict__ src, bool act, int l, const PatchTabs<T> &pt,
                                             T om, T *Ts, T *w) {
    constexpr int nn = N * N;
    auto fwd = [&](const T *in, T *out, int a) {
        if constexpr (EO) eo_fwd<N>(in, out, pt.ST[a]);
        else matvec_regs<N>(in, out, pt.ST[a]);
    };
    auto bwd = [&](const T *in, T *out, int a) {
        if constexpr (EO) eo_bwd<N>(in, out, pt.S[a]);
        else matvec_regs<N>(in, out, pt.S[a]);
    };
    T v[N];
    if (act) {
#pragma unroll
        for (int o0 = 0; o0 < NO; ++o0)
#pragma unroll
            for (int i0 = 0; i0 < N1; ++i0) v[o0 * N1 + i0] = (T)src[o0 * NC1 + i0];
        fwd(v, w, 0);
#pragma unroll
        for (int a = 0; a < N; ++a) Ts[N * l + a] = w[a];
    }
    __syncthreads();
    const int yb = line_base<3, N>(1, l), zb = line_base<3, N>(2, l);
    if (act) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = Ts[yb + i * N];
        fwd(v, w, 1);
#pragma unroll
        for (int i = 0; i < N; ++i) Ts[yb + i * N] = w[i];
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = Ts[zb + i * nn];
        fwd(v, w, 2);
#pragma unroll
        for (int m = 0; m < N; ++m) w[m] = w[m] * (om * recip(pt.lr + (T)pt.lam2[m]));
        bwd(w, v, 2);
#pragma unroll
        for (int i = 0; i < N; ++i) Ts[zb + i * nn] = v[i];
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = Ts[yb + i * N];
        bwd(v, w, 1);
#pragma unroll
        for (int i = 0; i < N; ++i) Ts[yb + i * N] = w[i];
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int a = 0; a < N; ++a) v[a] = Ts[N * l + a];
        bwd(v, w, 0);
    }
}

template <int N, int N1, int NO, int NC1, typename T>
__device__ __forceinline__ void lines3_solve_any(bool eo, const double *__restrict__ src, bool act, int l,
                                                 const PatchTabs<T> &pt, T om, T *Ts, T *w) {
    if constexpr (N % 2 == 0) {
        if (eo) {
            lines3_solve<N, N1, NO, NC1, T, true>(src, act, l, pt, om, Ts, w);
            return;
        }
    }
    lines3_solve<N, N1, NO, NC1, T, false>(src, act, l, pt, om, Ts, w);
}

template <int N1, int KIND, typename T, bool STAGE>
__device__ __forceinline__ void schwarz_lines3(const LevelView &g, const EigView &e, const SubGrid &sg,
                                               const double *__restrict__ r, double *__restrict__ x,
                                               T *__restrict__ W, double omega, T *Ts) {
    using C = SwCfg<3, N1, KIND>;
    constexpr int N = C::N, NC1 = C::NC1, NSC = C::NSC, LINES = C::LINES, NO = KIND ? 2 : 1;
    const int l = threadIdx.x;
    const int s = blockIdx.x;
    if (!sub_in_color(sg, s)) return;  // uniform: the whole workgroup leaves before any barrier
    int pos[3];
    {
        const int j0 = s % sg.cnt[0], rr = s / sg.cnt[0];
        pos[0] = __builtin_amdgcn_readfirstlane(sg.first[0] + sg.step * j0);
        pos[1] = __builtin_amdgcn_readfirstlane(sg.first[1] + sg.step * (rr % sg.cnt[1]));
        pos[2] = __builtin_amdgcn_readfirstlane(sg.first[2] + sg.step * (rr / sg.cnt[1]));
    }
    int tp[3];  // table positions (EigView::cls)
    for (int a = 0; a < 3; ++a) tp[a] = __builtin_amdgcn_readfirstlane(e.cls[a][pos[a]]);
    const bool act = l < LINES;
    const int a1 = l % N, a2 = l / N;
    const int o1 = a1 / N1, i1 = a1 % N1, o2 = a2 / N1, i2 = a2 % N1;
    const int64_t cs1 = g.m[0], cs2 = (int64_t)g.m[0] * g.m[1];
    const int64_t cell0 = pos[0] + (pos[1] + o1) * cs1 + (pos[2] + o2) * cs2;
    const int iofs = i1 * N1 + i2 * N1 * N1;
    const PatchTabs<T> pt = patch_tabs<T, N>(e, tp, act, a1, a2);
    const bool eo = __builtin_amdgcn_readfirstlane(e.sym[0][tp[0]] & e.sym[1][tp[1]] & e.sym[2][tp[2]]) != 0;
    T w[N];
    lines3_solve_any<N, N1, NO, NC1, T>(eo, r + cell0 * NC1 + iofs, act, l, pt, (T)omega, Ts, w);
    if (act) {
        if constexpr (STAGE) {
            T *dst = W + (int64_t)s * (NSC * NC1) + (2 * o1 + 4 * o2) * NC1 + iofs;
#pragma unroll
            for (int o0 = 0; o0 < NO; ++o0)
#pragma unroll
                for (int i0 = 0; i0 < N1; ++i0) dst[o0 * NC1 + i0] = w[o0 * N1 + i0];
        } else {
            double *dst = x + cell0 * NC1 + iofs;
#pragma unroll
            for (int o0 = 0; o0 < NO; ++o0)
#pragma unroll
                for (int i0 = 0; i0 < N1; ++i0) dst[o0 * NC1 + i0] += (double)w[o0 * N1 + i0];
        }
    }
}

// Staged vertex patches (3-D, direct-line configuration), a run of up to cz
// patches consecutive along z per workgroup.  Patches j and j+1 of a run
// share the cell layer above patch j: its correction from patch j is kept
// in LDS and added to that of patch j+1 before patch j+1 writes its lower
// layer, and patch j writes no upper layer.  The staging buffer then holds
// 4 + 4 / cz cell blocks per patch instead of 8; k_patch_gather skips the
// upper-layer blocks that were merged (the same rule, cz).  Deterministic.
template <int N1, typename T>
__global__ void __launch_bounds__((SwCfg<3, N1, 1>::THREADS))
k_schwarz_zrun(LevelView g, EigView e, SubGrid sg, int cz, const double *__restrict__ r, T *__restrict__ W,
               double omega) {
    using C = SwCfg<3, N1, 1>;
    constexpr int N = C::N, NC1 = C::NC1, NSC = C::NSC, LINES = C::LINES, HALF = N1 * N * N;
    static_assert(C::PPB == 1, "one patch per workgroup");
    __shared__ T Ts[N * N * N];
    __shared__ T carry[2][HALF];  // [k][i2][a1]: the upper layer of the previous patch
    const int l = threadIdx.x;
    const int nxy = sg.cnt[0] * sg.cnt[1];
    const int b = blockIdx.x;
    const int j0 = b % sg.cnt[0], j1 = (b / sg.cnt[0]) % sg.cnt[1], run = b / nxy;
    const int jz0 = run * cz, jz1 = min(sg.cnt[2], jz0 + cz);
    int tp[3];
    tp[0] = __builtin_amdgcn_readfirstlane(e.cls[0][j0]);
    tp[1] = __builtin_amdgcn_readfirstlane(e.cls[1][j1]);
    const bool act = l < LINES;
    const int a1 = l % N, a2 = l / N;
    const int o1 = a1 / N1, i1 = a1 % N1, o2 = a2 / N1, i2 = a2 % N1;
    const int64_t cs1 = g.m[0], cs2 = (int64_t)g.m[0] * g.m[1];
    const int iofs = i1 * N1 + i2 * N1 * N1;
    const int ci = i2 * N + a1;  // this thread's place in a carry layer
    for (int jz = jz0; jz < jz1; ++jz) {
        tp[2] = __builtin_amdgcn_readfirstlane(e.cls[2][jz]);
        const PatchTabs<T> pt = patch_tabs<T, N>(e, tp, act, a1, a2);
        const bool eo = __builtin_amdgcn_readfirstlane(e.sym[0][tp[0]] & e.sym[1][tp[1]] & e.sym[2][tp[2]]) != 0;
        const int64_t cell0 = j0 + (j1 + o1) * cs1 + (jz + o2) * cs2;
        T w[N];
        lines3_solve_any<N, N1, 2, NC1, T>(eo, r + cell0 * NC1 + iofs, act, l, pt, (T)omega, Ts, w);
        if (act) {
            const int64_t s = j0 + (int64_t)sg.cnt[0] * (j1 + (int64_t)sg.cnt[1] * jz);
            T *dst = W + s * (NSC * NC1) + (2 * o1 + 4 * o2) * NC1 + iofs;
            if (o2 == 1 && jz + 1 < jz1) {
#pragma unroll
                for (int k = 0; k < N; ++k) carry[jz & 1][k * (N1 * N) + ci] = w[k];
            } else {
                if (o2 == 0 && jz > jz0) {
#pragma unroll
                    for (int k = 0; k < N; ++k) w[k] += carry[(jz - 1) & 1][k * (N1 * N) + ci];
                }
#pragma unroll
                for (int o0 = 0; o0 < 2; ++o0)
#pragma unroll
                    for (int i0 = 0; i0 < N1; ++i0) dst[o0 * NC1 + i0] = w[o0 * N1 + i0];
            }
        }
    }
}

template <int D, int N1, int KIND, typename T, bool STAGE>
__global__ void __launch_bounds__((SwCfg<D, N1, KIND>::THREADS))
k_schwarz(LevelView g, EigView e, SubGrid sg, const double *__restrict__ r, double *__restrict__ x,
          T *__restrict__ W, double omega) {
    using C = SwCfg<D, N1, KIND>;
    constexpr bool LINES3 = D == 3 && C::PPB == 1;
    __shared__ T Ts[C::PPB * C::NT];
    if constexpr (LINES3) schwarz_lines3<N1, KIND, T, STAGE>(g, e, sg, r, x, W, omega, Ts);
    else schwarz_generic<D, N1, KIND, T, STAGE>(g, e, sg, r, x, W, omega, Ts);
}

// x += sum over the 2^d vertex patches containing each cell of that patch's
// staged correction (Sec. 2.3, eq. additiveschwarz), in the fixed order of the
// cell's position inside the patch: deterministic, no write conflicts.  The
// staged values are FP64 or FP32 (the contraction type); SCALED: each patch's
// FP32 values carry one FP64 factor, multiplied in here.
template <typename WT, int V>
struct VecOf;
template <> struct VecOf<double, 1> { typedef double type; };
template <> struct VecOf<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<double, 4> { typedef double type __attribute__((ext_vector_type(4))); };
template <> struct VecOf<float, 1> { typedef float type; };
template <> struct VecOf<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct VecOf<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };

template <int D, int N1>
struct GatherCfg {
    static constexpr int NC1 = ipow(N1, D);
    // consecutive DoFs of one cell per thread (vector loads stay aligned)
    static constexpr int V = NC1 % 4 == 0 ? 4 : (NC1 % 2 == 0 ? 2 : 1);
};

template <int D, int N1, typename WT, bool SCALED, int V>
__global__ void __launch_bounds__(256) k_patch_gather(LevelView g, const WT *__restrict__ W,
                                                      const double *__restrict__ Wsc, double *__restrict__ x,
                                                      int cz) {
    constexpr int NC1 = ipow(N1, D), NSC = 1 << D;
    static_assert(NC1 % V == 0, "a thread's DoFs must lie in one cell");
    using WV = typename VecOf<WT, V>::type;
    using XV = typename VecOf<double, V>::type;
    const int64_t gid = ((int64_t)blockIdx.x * 256 + threadIdx.x) * V;  // first DoF of this thread
    if (gid >= g.ncells * NC1) return;
    const int cell = (int)(gid / NC1);
    const int i = (int)(gid - (int64_t)cell * NC1);
    const int r0 = cell / g.m[0];
    const int c0 = cell - r0 * g.m[0], c1 = D == 3 ? r0 % g.m[1] : r0, c2 = D == 3 ? r0 / g.m[1] : 0;
    const int cnt0 = g.m[0] - 1, cnt1 = g.m[1] - 1;
    XV acc = (XV)0.0;
#pragma unroll
    for (int o = 0; o < NSC; ++o) {
        const int a0 = c0 - (o & 1), a1 = c1 - ((o >> 1) & 1), a2 = D == 3 ? c2 - ((o >> 2) & 1) : 0;
        const bool in = a0 >= 0 && a0 < cnt0 && a1 >= 0 && a1 < cnt1 && (D == 2 || (a2 >= 0 && a2 < g.m[2] - 1));
        // upper layer of a patch whose successor along z is in the same run
        // of cz patches: merged into the successor's lower layer
        const bool merged = D == 3 && (o >> 2) && a2 + 1 < g.m[2] - 1 && (a2 + 1) % cz != 0;
        if (in && !merged) {
            const int64_t sidx = a0 + (int64_t)cnt0 * (a1 + (int64_t)cnt1 * a2);
            const WV w = *(const WV *)(W + sidx * (NSC * NC1) + o * NC1 + i);
            XV wd;
            if constexpr (V == 1) wd = (double)w;
            else wd = __builtin_convertvector(w, XV);
            if constexpr (SCALED) acc += Wsc[sidx] * wd;
            else acc += wd;
        }
    }
    XV *xp = (XV *)(x + gid);
    *xp += acc;
}

// Vector width V when x is aligned for it (a caller may pass a view of a
// larger vector), else one DoF per thread.
template <int D, int N1, typename WT, bool SCALED>
static void launch_gather(const fts_level *lv, const WT *W, const double *Wsc, double *x, hipStream_t st,
                          int cz = 1) {
    constexpr int V = GatherCfg<D, N1>::V;
    const int64_t n = lv->ndofs;
    if (reinterpret_cast<uintptr_t>(x) % (V * sizeof(double)) == 0) {
        const int64_t nt = n / V;
        k_patch_gather<D, N1, WT, SCALED, V><<<dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st>>>(lv->view, W,
                                                                                                       Wsc, x, cz);
    } else {
        k_patch_gather<D, N1, WT, SCALED, 1><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(lv->view, W,
                                                                                                      Wsc, x, cz);
    }
}

// ---------------------------------------------------------------------------
// Local solves with 16-bit MFMA contractions (3-D, n <= 16, tensor padded to
// 16^3).  Each 1-D contraction of 16 lines is one v_mfma_f32_16x16x16 in the
// orientation Out^T = Mat * In^T: lane l holds Mat[l%16][4(l/16)+v] (A), the
// line l%16 at indices 4(l/16)+v (B) and receives the output line l%16 at
// indices 4(l/16)+v (D).  Because D has the layout of B, the last axis runs
// forward transform, eigenvalue scaling and backward transform in registers.
// Range control (FP16): the gathered residual is divided by its max-norm, the
// 1-D matrices are stored divided by s = max|S|, and the eigenvalue scaling
// uses Lambda_min / Lambda(m) <= 1; the factor
// F = |r|_max * omega * (s_x s_y s_z)^2 / Lambda_min is applied in FP64 when
// the correction is written.  Accumulation in FP32, update of x in FP64.
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPy = 20, kPz = 324;  // padded LDS pitches (conflict-free strided reads)

__device__ __forceinline__ int mline_base(int a, int L) {
    const int u = L & 15, v = L >> 4;
    if (a == 0) return u * kPy + v * kPz;
    if (a == 1) return u + v * kPz;
    return u + v * kPy;
}
__device__ __forceinline__ int mline_stride(int a) { return a == 0 ? 1 : (a == 1 ? kPy : kPz); }

__device__ __forceinline__ short f32_to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

template <int BF>
struct Mfma16;
template <>
struct Mfma16<0> {
    typedef f16x4 vec;
    static __device__ __forceinline__ vec pack(const float *v) {
        vec r;
        r[0] = (_Float16)v[0];
        r[1] = (_Float16)v[1];
        r[2] = (_Float16)v[2];
        r[3] = (_Float16)v[3];
        return r;
    }
    static __device__ __forceinline__ vec load(const uint16_t *p) {
        const uint2 u = *reinterpret_cast<const uint2 *>(p);
        vec r;
        __builtin_memcpy(&r, &u, 8);
        return r;
    }
    static __device__ __forceinline__ f32x4 mma(vec a, vec b) {
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, z, 0, 0, 0);
    }
};
template <>
struct Mfma16<1> {
    typedef s16x4 vec;
    static __device__ __forceinline__ vec pack(const float *v) {
        vec r;
        r[0] = f32_to_bf16(v[0]);
        r[1] = f32_to_bf16(v[1]);
        r[2] = f32_to_bf16(v[2]);
        r[3] = f32_to_bf16(v[3]);
        return r;
    }
    static __device__ __forceinline__ vec load(const uint16_t *p) {
        const uint2 u = *reinterpret_cast<const uint2 *>(p);
        vec r;
        __builtin_memcpy(&r, &u, 8);
        return r;
    }
    static __device__ __forceinline__ f32x4 mma(vec a, vec b) {
        const f32x4 z = {0.f, 0.f, 0.f, 0.f};
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, z, 0, 0, 0);
    }
};

// RUN (staged vertex patches only): a run of up to cz patches along z per
// workgroup as in k_schwarz_mfma64, the shared cell layer carried in
// registers; the staged values then carry their factor F already (FP32),
// so that two patches' values can be added, and Wsc is not written.
template <int N1, int KIND, int BF, bool STAGE, bool RUN = false>
__global__ void __launch_bounds__(256)
k_schwarz_mfma(LevelView g, EigView e, SubGrid sg, const double *__restrict__ r, double *__restrict__ x,
               float *__restrict__ W, double *__restrict__ Wsc, double omega, int cz = 1) {
    using M = Mfma16<BF>;
    constexpr int N = KIND ? 2 * N1 : N1;
    static_assert(N <= 16, "MFMA path needs n <= 16");
    constexpr int NC1 = N1 * N1 * N1, NSC = KIND ? 8 : 1;
    __shared__ float Ts[16 * kPz];
    __shared__ float wmax[4];
    static_assert(!RUN || (KIND == 1 && STAGE), "runs along z: staged vertex patches");
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int64_t s;
    int jz0 = 0, jz1 = 1;
    if constexpr (RUN) {
        const int nxy = sg.cnt[0] * sg.cnt[1];
        const int run = (int)(blockIdx.x / nxy);
        jz0 = run * cz;
        jz1 = min(sg.cnt[2], jz0 + cz);
        s = blockIdx.x % nxy + (int64_t)nxy * jz0;
    } else {
        s = blockIdx.x;
        if (!sub_in_color(sg, s)) return;  // uniform: the whole workgroup leaves before any barrier
    }
    if (N < 16) {
        for (int p = t; p < 16 * kPz; p += 256) Ts[p] = 0.f;  // padding stays zero through the contractions
        __syncthreads();
    }
    float carry[N];
    for (int jz = jz0; jz < jz1; ++jz) {
    if (RUN && jz > jz0) {
        s += (int64_t)sg.cnt[0] * sg.cnt[1];
        __syncthreads();  // every thread has read its previous line from Ts
    }
    int pos[3];
    {
        const int j0 = (int)(s % sg.cnt[0]);
        const int64_t rr = s / sg.cnt[0];
        const int j1 = (int)(rr % sg.cnt[1]);
        const int j2 = (int)(rr / sg.cnt[1]);
        pos[0] = __builtin_amdgcn_readfirstlane(sg.first[0] + sg.step * j0);
        pos[1] = __builtin_amdgcn_readfirstlane(sg.first[1] + sg.step * j1);
        pos[2] = __builtin_amdgcn_readfirstlane(sg.first[2] + sg.step * j2);
    }
    int tp[3];  // table positions (EigView::cls)
    for (int a = 0; a < 3; ++a) tp[a] = __builtin_amdgcn_readfirstlane(e.cls[a][pos[a]]);
    const int64_t cs1 = g.m[0], cs2 = (int64_t)g.m[0] * g.m[1];
    // thread t < N^2 owns the patch line along x with (a1, a2) = (t % N, t / N)
    // (in a run, with the halves along z swapped on odd patches): NO runs of
    // k+1 contiguous residual values, all loads issued together
    constexpr int NO = KIND ? 2 : 1;
    const bool own = t < N * N;
    const int a1 = t % N, a2 = (RUN && own && ((jz - jz0) & 1)) ? (t / N + N1) % N : t / N;
    const int o1 = a1 / N1, i1 = a1 % N1, o2 = a2 / N1, i2 = a2 % N1;
    const int64_t cell0 = pos[0] + (pos[1] + o1) * cs1 + (pos[2] + o2) * cs2;
    const int iofs = i1 * N1 + i2 * N1 * N1;
    const int lbase = a1 * kPy + a2 * kPz;
    float amax = 0.f;
    if (own) {
        const double *src = r + cell0 * NC1 + iofs;
        double rv[N];
#pragma unroll
        for (int o0 = 0; o0 < NO; ++o0)
#pragma unroll
            for (int i0 = 0; i0 < N1; ++i0) rv[o0 * N1 + i0] = src[o0 * NC1 + i0];
#pragma unroll
        for (int a0 = 0; a0 < N; ++a0) {
            const float v = (float)rv[a0];
            Ts[lbase + a0] = v;
            amax = fmaxf(amax, fabsf(v));
        }
    }
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off, 64));
    if (lane == 0) wmax[wv] = amax;
    __syncthreads();
    const float rmax = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    const float inv = rmax > 0.f ? 1.f / rmax : 0.f;
    const int c4 = 4 * (lane >> 4), j = lane & 15;
    auto mat = [&](const uint16_t *const *tab, int a) {
        return M::load(tab[a] + (size_t)tp[a] * 256 + j * 16 + c4);
    };
    const uint16_t *const *Ftab = BF ? e.Fbf16 : e.Ff16;
    const uint16_t *const *Btab = BF ? e.Bbf16 : e.Bf16;
    // forward transforms along x and y
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const typename M::vec A = mat(Ftab, a);
        const int st = mline_stride(a);
        for (int tt = wv; tt < 16; tt += 4) {
            const int base = mline_base(a, 16 * tt + j) + c4 * st;
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = Ts[base + q * st] * (a == 0 ? inv : 1.f);
            const f32x4 d = M::mma(A, M::pack(v));
#pragma unroll
            for (int q = 0; q < 4; ++q) Ts[base + q * st] = d[q];
        }
        __syncthreads();
    }
    // z: forward, scaling Lambda_min / Lambda(m), backward, in registers
    {
        const typename M::vec Af = mat(Ftab, 2), Ab = mat(Btab, 2);
        const float *lx = e.lam32[0] + (size_t)tp[0] * N, *ly = e.lam32[1] + (size_t)tp[1] * N;
        const float *lz = e.lam32[2] + (size_t)tp[2] * N;
        const float lmin = e.lmin[0][tp[0]] + e.lmin[1][tp[1]] + e.lmin[2][tp[2]];
        for (int tt = wv; tt < 16; tt += 4) {
            const int base = mline_base(2, 16 * tt + j) + c4 * kPz;
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = Ts[base + q * kPz];
            f32x4 d = M::mma(Af, M::pack(v));
            const int mx = j, my = tt;  // this line's fixed mode indices
            const bool inxy = mx < N && my < N;
            const float lxy = inxy ? lx[mx] + ly[my] : 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int mz = c4 + q;
                v[q] = (inxy && mz < N) ? d[q] * (lmin / (lxy + lz[mz])) : 0.f;
            }
            d = M::mma(Ab, M::pack(v));
#pragma unroll
            for (int q = 0; q < 4; ++q) Ts[base + q * kPz] = d[q];
        }
        __syncthreads();
    }
    // backward transforms along y and x
#pragma unroll
    for (int a = 1; a >= 0; --a) {
        const typename M::vec A = mat(Btab, a);
        const int st = mline_stride(a);
        for (int tt = wv; tt < 16; tt += 4) {
            const int base = mline_base(a, 16 * tt + j) + c4 * st;
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = Ts[base + q * st];
            const f32x4 d = M::mma(A, M::pack(v));
#pragma unroll
            for (int q = 0; q < 4; ++q) Ts[base + q * st] = d[q];
        }
        __syncthreads();
    }
    const double sx = e.mscale[0][tp[0]], sy = e.mscale[1][tp[1]], sz = e.mscale[2][tp[2]];
    const double lmin = (double)e.lmin[0][tp[0]] + e.lmin[1][tp[1]] + e.lmin[2][tp[2]];
    const double F = (double)rmax * omega * (sx * sy * sz) * (sx * sy * sz) / lmin;
    if (STAGE && !RUN && t == 0) Wsc[s] = F;
    if (own) {
        float c[N];
#pragma unroll
        for (int a0 = 0; a0 < N; ++a0) c[a0] = Ts[lbase + a0];
        if constexpr (STAGE && RUN) {
            float *dst = W + s * (NSC * NC1) + (2 * o1 + 4 * o2) * NC1 + iofs;  // F applied here
#pragma unroll
            for (int a0 = 0; a0 < N; ++a0) c[a0] = (float)(F * (double)c[a0]);
            if (o2 == 1 && jz + 1 < jz1) {
#pragma unroll
                for (int a0 = 0; a0 < N; ++a0) carry[a0] = c[a0];
            } else {
                if (o2 == 0 && jz > jz0) {
#pragma unroll
                    for (int a0 = 0; a0 < N; ++a0) c[a0] += carry[a0];
                }
#pragma unroll
                for (int o0 = 0; o0 < NO; ++o0)
#pragma unroll
                    for (int i0 = 0; i0 < N1; ++i0) dst[o0 * NC1 + i0] = c[o0 * N1 + i0];
            }
        } else if constexpr (STAGE) {
            float *dst = W + s * (NSC * NC1) + (2 * o1 + 4 * o2) * NC1 + iofs;  // F applied by the gather
#pragma unroll
            for (int o0 = 0; o0 < NO; ++o0)
#pragma unroll
                for (int i0 = 0; i0 < N1; ++i0) dst[o0 * NC1 + i0] = c[o0 * N1 + i0];
        } else {
            double *dst = x + cell0 * NC1 + iofs;
#pragma unroll
            for (int o0 = 0; o0 < NO; ++o0)
#pragma unroll
                for (int i0 = 0; i0 < N1; ++i0) dst[o0 * NC1 + i0] += F * (double)c[o0 * N1 + i0];
        }
    }
    }
}

// ---------------------------------------------------------------------------
// FP64 local solves on MFMA (v_mfma_f64_16x16x4f64) for 3-D vertex patches of
// extent N = 16 (k = 7), the shape where each 1-D contraction of 16 lines is
// a dense 16 x 16 x 16 product.  Same algorithm and arithmetic type as
// k_schwarz (only the summation order differs).  Operand layout of the
// instruction: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16] and
// receives D[4 v + l / 16][l % 16] in slot v.  A contraction Out^T = Mat In^T
// of 16 lines runs as 4 instructions; in step c lane group q = l / 16
// supplies k = 4 c + q, so the result (mode 4 v + q in slot v) is already the
// B operand of a following contraction along the same lines: the last axis
// runs forward transform, eigenvalue scaling and backward transform in
// registers.  The tensor lives in LDS with the pitches of the 16-bit path.
typedef double d4 __attribute__((ext_vector_type(4)));

// LDS pitches of the FP64 tile (in doubles): lanes (j, q) of a contraction
// touch element (line j, index 4 c + q); with a line pitch of 17 and a plane
// pitch of 272 = 16 (mod 32) the 64 addresses of each access spread over the
// 32 double-wide bank pairs for lines along x, y and z alike.
constexpr int kQy = 17, kQz = 272;
__device__ __forceinline__ int qline_base(int a, int L) {
    const int u = L & 15, v = L >> 4;
    if (a == 0) return u * kQy + v * kQz;
    if (a == 1) return u + v * kQz;
    return u + v * kQy;
}
__device__ __forceinline__ int qline_stride(int a) { return a == 0 ? 1 : (a == 1 ? kQy : kQz); }

// RUN (staged only): the workgroup takes a run of up to cz patches along z
// as k_schwarz_zrun does, and the cell layer two neighbours share stays in
// registers: thread t owns the line with o2 flipped on every other patch, so
// the thread that holds patch j's upper layer owns the same lines as the
// lower layer of patch j+1.
template <int N1, bool STAGE, bool RUN = false>
__global__ void __launch_bounds__(256)
k_schwarz_mfma64(LevelView g, EigView e, SubGrid sg, const double *__restrict__ r, double *__restrict__ x,
                 double *__restrict__ W, double omega, int cz = 1) {
    constexpr int N = 2 * N1, NC1 = N1 * N1 * N1, NSC = 8;
    static_assert(N == 16, "one 16 x 16 tile per contraction");
    __shared__ double Ts[16 * kQz];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int64_t s;
    int jz0 = 0, jz1 = 1;
    if constexpr (RUN) {
        const int nxy = sg.cnt[0] * sg.cnt[1];
        const int run = (int)(blockIdx.x / nxy);
        jz0 = run * cz;
        jz1 = min(sg.cnt[2], jz0 + cz);
        s = blockIdx.x % nxy + (int64_t)nxy * jz0;
    } else {
        s = blockIdx.x;
        if (!sub_in_color(sg, s)) return;  // uniform: the whole workgroup leaves before any barrier
    }
    const int64_t cs1 = g.m[0], cs2 = (int64_t)g.m[0] * g.m[1];
    double carry[2 * N1];
    for (int jz = jz0; jz < jz1; ++jz) {
    if (RUN && jz > jz0) {
        s += (int64_t)sg.cnt[0] * sg.cnt[1];
        __syncthreads();  // every thread has read its previous line from Ts
    }
    int pos[3];
    {
        const int j0 = (int)(s % sg.cnt[0]);
        const int64_t rr = s / sg.cnt[0];
        pos[0] = __builtin_amdgcn_readfirstlane(sg.first[0] + sg.step * j0);
        pos[1] = __builtin_amdgcn_readfirstlane(sg.first[1] + sg.step * (int)(rr % sg.cnt[1]));
        pos[2] = __builtin_amdgcn_readfirstlane(sg.first[2] + sg.step * (int)(rr / sg.cnt[1]));
    }
    int tp[3];  // table positions (EigView::cls)
    for (int a = 0; a < 3; ++a) tp[a] = __builtin_amdgcn_readfirstlane(e.cls[a][pos[a]]);
    // thread t owns the patch line along x with (a1, a2) = (t % 16, t / 16),
    // in a run with the upper and lower half along z swapped on odd patches
    const int a1 = t % N, a2 = (RUN && ((jz - jz0) & 1)) ? (t / N + N1) % N : t / N;
    const int o1 = a1 / N1, i1 = a1 % N1, o2 = a2 / N1, i2 = a2 % N1;
    const int64_t cell0 = pos[0] + (pos[1] + o1) * cs1 + (pos[2] + o2) * cs2;
    const int iofs = i1 * N1 + i2 * N1 * N1;
    const int lbase = a1 * kQy + a2 * kQz;
    {
        const double *src = r + cell0 * NC1 + iofs;
        double rv[N];
#pragma unroll
        for (int o0 = 0; o0 < 2; ++o0)
#pragma unroll
            for (int i0 = 0; i0 < N1; ++i0) rv[o0 * N1 + i0] = src[o0 * NC1 + i0];
#pragma unroll
        for (int a0 = 0; a0 < N; ++a0) Ts[lbase + a0] = rv[a0];
    }
    __syncthreads();
    const int q = lane >> 4, j = lane & 15;
    constexpr int nn = N * N;
    // A operand of step c: Mat[j][4 c + q]
    auto amat = [&](const double *M, double *A) {
#pragma unroll
        for (int c = 0; c < 4; ++c) A[c] = M[j * N + 4 * c + q];
    };
    auto tiles = [&](int a, const double *A) {
        const int st = qline_stride(a);
        for (int tt = wv; tt < 16; tt += 4) {
            const int base = qline_base(a, 16 * tt + j);
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[c], Ts[base + st * (4 * c + q)], acc, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) Ts[base + st * (4 * v + q)] = acc[v];
        }
    };
    double A[4];
    // forward transforms along x and y: Mat = S^T
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        amat(e.ST[a] + (size_t)tp[a] * nn, A);
        tiles(a, A);
        __syncthreads();
    }
    {
        double Af[4], Ab[4];
        amat(e.ST[2] + (size_t)tp[2] * nn, Af);
        amat(e.S[2] + (size_t)tp[2] * nn, Ab);
        const double *lx = e.lam[0] + (size_t)tp[0] * N, *ly = e.lam[1] + (size_t)tp[1] * N;
        const double *lz = e.lam[2] + (size_t)tp[2] * N;
        for (int tt = wv; tt < 16; tt += 4) {
            const int base = qline_base(2, 16 * tt + j);
            d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Af[c], Ts[base + kQz * (4 * c + q)], acc, 0, 0, 0);
            // this z-line has modes (j, tt) along x and y; slot v holds mode 4 v + q along z
            const double lxy = lx[j] + ly[tt];
            d4 acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double sc = acc[c] * (omega * recip(lxy + lz[4 * c + q]));
                acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ab[c], sc, acc2, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) Ts[base + kQz * (4 * v + q)] = acc2[v];
        }
        __syncthreads();
    }
    // backward transforms along y and x: Mat = S
#pragma unroll
    for (int a = 1; a >= 0; --a) {
        amat(e.S[a] + (size_t)tp[a] * nn, A);
        tiles(a, A);
        __syncthreads();
    }
    double cv[N];
#pragma unroll
    for (int a0 = 0; a0 < N; ++a0) cv[a0] = Ts[lbase + a0];
    if constexpr (STAGE) {
        double *dst = W + s * (NSC * NC1) + (2 * o1 + 4 * o2) * NC1 + iofs;
        if (RUN && o2 == 1 && jz + 1 < jz1) {
#pragma unroll
            for (int a0 = 0; a0 < N; ++a0) carry[a0] = cv[a0];
        } else {
            if (RUN && o2 == 0 && jz > jz0) {
#pragma unroll
                for (int a0 = 0; a0 < N; ++a0) cv[a0] += carry[a0];
            }
#pragma unroll
            for (int o0 = 0; o0 < 2; ++o0)
#pragma unroll
                for (int i0 = 0; i0 < N1; ++i0) dst[o0 * NC1 + i0] = cv[o0 * N1 + i0];
        }
    } else {
        double *dst = x + cell0 * NC1 + iofs;
#pragma unroll
        for (int o0 = 0; o0 < 2; ++o0)
#pragma unroll
            for (int i0 = 0; i0 < N1; ++i0) dst[o0 * NC1 + i0] += cv[o0 * N1 + i0];
    }
    }
}

// ---------------------------------------------------------------------------
// Transfers (Sec. 2.2).  Child c of a coarse cell sits at offset o in
// {0,1}^d; its coefficients are (E_{o_d} x..x E_{o_1}) applied to the coarse
// coefficients, E_o[i][j] = phi_j((xi_i + o)/2).  Restriction applies the
// transposes and sums over the 2^d children.  All 2^d children at once:
// with the stacked 1-D matrix Es = [E_0; E_1] (2 n1 x n1, the level table E)
// the children of a cell form one (2 n1)^d tensor, Es x..x Es times the
// coarse coefficients, so prolongation is d contractions that each double
// one axis (n1 -> 2 n1) and restriction d transposed contractions that
// halve one, one workgroup per coarse cell and one thread per line.
template <int D, int N1>
struct XferCfg {
    static constexpr int N2 = 2 * N1;
    static constexpr int NC = ipow(N1, D);
    static constexpr int NT = ipow(N2, D);
    static constexpr int MAXL = ipow(N2, D - 1);  // lines of the widest stage
    static constexpr int THREADS = MAXL <= 64 ? 64 : rup64(MAXL);
};

// Stage a works along axis a of the (2 n1)^d tensor (strides 1, 2 n1,
// (2 n1)^2) while the axes below a have extent 2 n1 and those above n1:
// N2^a N1^(d-1-a) lines; line l's first element.
template <int D, int N1>
__device__ __forceinline__ int xfer_line_base(int a, int l) {
    constexpr int N2 = 2 * N1;
    if constexpr (D == 2) {
        return a == 0 ? l * N2 : l;
    } else {
        if (a == 0) return (l % N1) * N2 + (l / N1) * N2 * N2;
        if (a == 1) return (l % N2) + (l / N2) * N2 * N2;
        return (l % N2) + (l / N2) * N2;
    }
}
template <int D, int N1>
__device__ __forceinline__ int xfer_lines(int a) {
    return ipow(2 * N1, a) * ipow(N1, D - 1 - a);
}

template <int D, int N1, bool RESTRICT>
__global__ void __launch_bounds__((XferCfg<D, N1>::THREADS))
k_transfer(LevelView gc, LevelView gf, const double *__restrict__ src, double *__restrict__ dst) {
    using C = XferCfg<D, N1>;
    constexpr int N2 = C::N2, NC = C::NC, NT = C::NT, TH = C::THREADS;
    __shared__ double T[NT];
    const int t = threadIdx.x;
    const int64_t cc = blockIdx.x;
    int c[3];
    cell_coords(cc, gc.m, c);
    const int64_t fs1 = gf.m[0], fs2 = (int64_t)gf.m[0] * gf.m[1];
    const cptr<double> Es = uniform_table(gc.E);  // [2 n1][n1]
    // global index of element p of the children's tensor
    auto fine_index = [&](int p) {
        const int f0 = p % N2, f1 = (p / N2) % N2, f2 = D == 3 ? p / (N2 * N2) : 0;
        const int64_t cell = (2 * c[0] + f0 / N1) + (2 * c[1] + f1 / N1) * fs1 +
                             (D == 3 ? (int64_t)(2 * c[2] + f2 / N1) * fs2 : 0);
        return cell * NC + (f0 % N1) + N1 * (f1 % N1) + (D == 3 ? N1 * N1 * (f2 % N1) : 0);
    };
    // the coarse cell's coefficients sit in the corner [0, n1)^d of the tensor
    auto corner = [&](int p) {
        const int i0 = p % N1, i1 = (p / N1) % N1, i2 = D == 3 ? p / (N1 * N1) : 0;
        return i0 + N2 * i1 + N2 * N2 * i2;
    };
    if constexpr (!RESTRICT) {
        for (int p = t; p < NC; p += TH) T[corner(p)] = src[cc * NC + p];
        __syncthreads();
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const int st = a == 0 ? 1 : (a == 1 ? N2 : N2 * N2);
            for (int l = t; l < xfer_lines<D, N1>(a); l += TH) {
                const int base = xfer_line_base<D, N1>(a, l);
                double in[N1];
#pragma unroll
                for (int i = 0; i < N1; ++i) in[i] = T[base + i * st];
#pragma unroll
                for (int o = 0; o < N2; ++o) {
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < N1; ++i) s = fma((double)Es[o * N1 + i], in[i], s);
                    T[base + o * st] = s;
                }
            }
            __syncthreads();
        }
        for (int p = t; p < NT; p += TH) {
            const int64_t gi = fine_index(p);
            dst[gi] += T[p];
        }
    } else {
        for (int p = t; p < NT; p += TH) T[p] = src[fine_index(p)];
        __syncthreads();
#pragma unroll
        for (int a = D - 1; a >= 0; --a) {
            const int st = a == 0 ? 1 : (a == 1 ? N2 : N2 * N2);
            for (int l = t; l < xfer_lines<D, N1>(a); l += TH) {
                const int base = xfer_line_base<D, N1>(a, l);
                double in[N2];
#pragma unroll
                for (int o = 0; o < N2; ++o) in[o] = T[base + o * st];
#pragma unroll
                for (int i = 0; i < N1; ++i) {
                    double s = 0.0;
#pragma unroll
                    for (int o = 0; o < N2; ++o) s = fma((double)Es[o * N1 + i], in[o], s);
                    T[base + i * st] = s;
                }
            }
            __syncthreads();
        }
        for (int p = t; p < NC; p += TH) dst[cc * NC + p] = T[corner(p)];
    }
}

// ---------------------------------------------------------------------------
// Coarse matrix in slab blocks (SlabBlocks): entry (row, col) from the same
// 1-D tables as the operator.  One thread per row; for a fixed column the
// rows of a wave are consecutive, so the stores coalesce.
__device__ __forceinline__ double &slab_entry(const SlabBlocks &s, int64_t row, int64_t col) {
    const int64_t bi = row / s.B, bj = col / s.B;
    const int64_t off = (row - bi * s.B) + (col - bj * s.B) * s.B;
    double *blk = bj == bi ? s.D + bi * s.B * s.B : (bj < bi ? s.Lo + (bi - 1) * s.B * s.B : s.Up + bi * s.B * s.B);
    return blk[off];
}

template <int D, int N1>
__global__ void __launch_bounds__(256) k_assemble_slabs(LevelView g, SlabBlocks A, int64_t N) {
    constexpr int NC = ipow(N1, D);
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= N) return;
    const int64_t cell = row / NC;
    const int iota = (int)(row % NC);
    int c[3];
    cell_coords(cell, g.m, c);
    int ii[3] = {iota % N1, (iota / N1) % N1, D == 3 ? iota / (N1 * N1) : 0};
    const int64_t cs[3] = {1, g.m[0], (int64_t)g.m[0] * g.m[1]};
    double h[3] = {g.h[0][c[0]], g.h[1][c[1]], D == 3 ? g.h[2][c[2]] : 1.0};
    const double *Mh = g.Mhat;
    for (int j = 0; j < NC; ++j) {
        int jj[3] = {j % N1, (j / N1) % N1, D == 3 ? j / (N1 * N1) : 0};
        double mass[3];
        for (int a = 0; a < D; ++a) mass[a] = h[a] * Mh[ii[a] * N1 + jj[a]];
        // diagonal block
        double v = 0.0;
        for (int tt = 0; tt < D; ++tt) {
            double term = g.cellop[tt][(size_t)c[tt] * N1 * N1 + ii[tt] * N1 + jj[tt]];
            for (int a = 0; a < D; ++a)
                if (a != tt) term *= mass[a];
            v += term;
        }
        slab_entry(A, row, cell * NC + j) = v;
        for (int tt = 0; tt < D; ++tt) {
            double tr = 1.0;
            for (int a = 0; a < D; ++a)
                if (a != tt) tr *= mass[a];
            if (c[tt] + 1 < g.m[tt]) {
                const double bv = g.iface[tt][(size_t)c[tt] * N1 * N1 + ii[tt] * N1 + jj[tt]];
                slab_entry(A, row, (cell + cs[tt]) * NC + j) = bv * tr;
            }
            if (c[tt] > 0) {
                const double bv = g.iface[tt][(size_t)(c[tt] - 1) * N1 * N1 + jj[tt] * N1 + ii[tt]];
                slab_entry(A, row, (cell - cs[tt]) * NC + j) = bv * tr;
            }
        }
    }
}

__global__ void k_fill(double *__restrict__ p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <int D, int N1>
struct RunOperator {
    static fts_status run(const fts_level *lv, const double *x, const double *b, double *y, bool res,
                          hipStream_t st) {
        using C = OpCfg<D, N1>;
        if (lv->ncells > INT_MAX) return fail(FTS_E_SIZE, "too many cells for one launch");
        const OpRuns runs = op_runs(lv->view.m, D, C::CPW);
        const int64_t blocks = runs.nblocks;
        if (blocks == 0) return FTS_OK;
        if (blocks > INT_MAX) return fail(FTS_E_SIZE, "too many cells for one launch");
        if (res)
            k_operator<D, N1, true, false><<<dim3((unsigned)blocks), dim3(C::THREADS), 0, st>>>(lv->view, runs, x, b, y);
        else
            k_operator<D, N1, false, false><<<dim3((unsigned)blocks), dim3(C::THREADS), 0, st>>>(lv->view, runs, x, b, y);
        return check_launch("k_operator");
    }
};

fts_status launch_operator(const fts_level *lv, const double *x, const double *b, double *y, bool residual,
                           hipStream_t stream) {
    return dispatch<RunOperator>(lv->dim, lv->n1, lv, x, b, y, residual, stream);
}

// r = b - A x computed in FP64 and stored rounded to FP32 (the residual the
// 16-bit local solves of the owner tiles read).
template <int D, int N1>
struct RunResidual32 {
    static fts_status run(const fts_level *lv, const double *x, const double *b, float *r, hipStream_t st) {
        using C = OpCfg<D, N1>;
        if (lv->ncells > INT_MAX) return fail(FTS_E_SIZE, "too many cells for one launch");
        const OpRuns runs = op_runs(lv->view.m, D, C::CPW);
        const int64_t blocks = runs.nblocks;
        if (blocks == 0) return FTS_OK;
        if (blocks > INT_MAX) return fail(FTS_E_SIZE, "too many cells for one launch");
        k_operator<D, N1, true, false, float><<<dim3((unsigned)blocks), dim3(C::THREADS), 0, st>>>(lv->view, runs, x, b, r);
        return check_launch("k_operator (FP32 residual)");
    }
};

fts_status smooth_additive(const fts_level *lv, const fts_eigs *eg, double omega, fts_prec prec, const double *b,
                           double *x, void *rbuf, bool x_zero, hipStream_t stream) {
    if (x_zero) return launch_schwarz(lv, eg, omega, prec, b, x, stream);  // r = b - A 0 = b
    const bool f32r = (prec == FTS_PREC_BF16 || prec == FTS_PREC_F16) && lv->dim == 3 &&
                      eg->kind == FTS_VERTEX_PATCH && effective_schedule(eg->schedule, lv->ncells) == FTS_SCHEDULE_OWNER &&
                      lv->n1 <= 8 &&
                      reinterpret_cast<uintptr_t>(rbuf) % 16 == 0;
    if (!f32r) {
        double *r = static_cast<double *>(rbuf);
        fts_status st = launch_operator(lv, x, b, r, true, stream);
        return st == FTS_OK ? launch_schwarz(lv, eg, omega, prec, r, x, stream) : st;
    }
    float *r = static_cast<float *>(rbuf);
    fts_status st = dispatch<RunResidual32>(lv->dim, lv->n1, lv, x, b, r, stream);
    return st == FTS_OK ? launch_schwarz_mfma_tile(lv, eg, omega, prec == FTS_PREC_BF16, r, true, x, stream) : st;
}

template <int D, int N1>
struct RunSchwarz {
    template <int KIND, typename T>
    static fts_status go(const fts_level *lv, const fts_eigs *eg, double omega, const double *r, double *x,
                         hipStream_t st) {
        using C = SwCfg<D, N1, KIND>;
        const bool staged = KIND == 1 && eg->schedule != FTS_SCHEDULE_COLORED;
        const int ncolor = (KIND && !staged) ? (1 << D) : 1;
        int cz = 1;  // patches per run along z in the staging buffer (k_schwarz_zrun)
        for (int color = 0; color < ncolor; ++color) {
            SubGrid sg{};
            sg.parity = -1;
            sg.step = (KIND && !staged) ? 2 : 1;
            sg.nsub = 1;
            for (int a = 0; a < 3; ++a) {
                if (a >= D) {
                    sg.cnt[a] = 1;
                    sg.first[a] = 0;
                    continue;
                }
                const int npos = eg->count[a];  // positions along the axis
                sg.first[a] = (KIND && !staged) ? ((color >> a) & 1) : 0;
                sg.cnt[a] = npos > sg.first[a] ? (npos - sg.first[a] + sg.step - 1) / sg.step : 0;
                sg.nsub *= sg.cnt[a];
            }
            if (sg.nsub == 0) continue;
            const int64_t blocks = (sg.nsub + C::PPB - 1) / C::PPB;
            if (blocks > INT_MAX) return fail(FTS_E_SIZE, "too many subdomains for one launch");
            if constexpr (D == 3 && KIND == 1 && C::PPB == 1) {
                // runs of cz patches along z, as long as enough workgroups remain
                cz = 1;
                while (cz < 8 && sg.nsub / (2 * cz) >= 6144) cz *= 2;
                if (staged && cz > 1) {
                    const int64_t runs = (sg.cnt[2] + cz - 1) / cz;
                    k_schwarz_zrun<N1, T><<<dim3((unsigned)((int64_t)sg.cnt[0] * sg.cnt[1] * runs)),
                                            dim3(C::THREADS), 0, st>>>(lv->view, eg->view, sg, cz, r,
                                                                       reinterpret_cast<T *>(eg->d_stage), omega);
                    fts_status s = check_launch("k_schwarz_zrun");
                    if (s != FTS_OK) return s;
                    continue;
                }
                cz = 1;
            }
            if (staged)
                k_schwarz<D, N1, KIND, T, true><<<dim3((unsigned)blocks), dim3(C::THREADS), 0, st>>>(
                    lv->view, eg->view, sg, r, x, reinterpret_cast<T *>(eg->d_stage), omega);
            else
                k_schwarz<D, N1, KIND, T, false><<<dim3((unsigned)blocks), dim3(C::THREADS), 0, st>>>(
                    lv->view, eg->view, sg, r, x, nullptr, omega);
            fts_status s = check_launch("k_schwarz");
            if (s != FTS_OK) return s;
        }
        if (staged) {
            launch_gather<D, N1, T, false>(lv, reinterpret_cast<const T *>(eg->d_stage), nullptr, x, st, cz);
            return check_launch("k_patch_gather");
        }
        return FTS_OK;
    }
    template <int KIND, int BF>
    static fts_status go_mfma(const fts_level *lv, const fts_eigs *eg, double omega, const double *r, double *x,
                              hipStream_t st) {
        if constexpr (D != 3 || (KIND ? 2 * N1 : N1) > 16) {
            return fail(FTS_E_UNSUPPORTED, "16-bit MFMA contractions need d = 3 and n <= 16");
        } else {
            if constexpr (KIND == 1) {
                if (effective_schedule(eg->schedule, lv->ncells) == FTS_SCHEDULE_OWNER &&
                    reinterpret_cast<uintptr_t>(r) % 16 == 0)
                    return launch_schwarz_mfma_tile(lv, eg, omega, BF, r, false, x, st);
            }
            const bool staged = KIND == 1 && eg->schedule != FTS_SCHEDULE_COLORED;
            const int ncolor = (KIND && !staged) ? 8 : 1;
            int cz = 1;
            for (int color = 0; color < ncolor; ++color) {
                SubGrid sg{};
                sg.parity = -1;
                sg.step = (KIND && !staged) ? 2 : 1;
                sg.nsub = 1;
                for (int a = 0; a < 3; ++a) {
                    sg.first[a] = (KIND && !staged) ? ((color >> a) & 1) : 0;
                    const int npos = eg->count[a];
                    sg.cnt[a] = npos > sg.first[a] ? (npos - sg.first[a] + sg.step - 1) / sg.step : 0;
                    sg.nsub *= sg.cnt[a];
                }
                if (sg.nsub == 0) continue;
                if (staged) {
                    // runs of cz patches along z, as long as enough workgroups remain
                    while (cz < 8 && sg.nsub / (2 * cz) >= 6144) cz *= 2;
                    if constexpr (KIND == 1) {
                        if (cz > 1)
                            k_schwarz_mfma<N1, KIND, BF, true, true>
                                <<<dim3((unsigned)((int64_t)sg.cnt[0] * sg.cnt[1] * ((sg.cnt[2] + cz - 1) / cz))),
                                   dim3(256), 0, st>>>(lv->view, eg->view, sg, r, x,
                                                       reinterpret_cast<float *>(eg->d_stage), nullptr, omega, cz);
                    }
                    if (cz == 1)
                        k_schwarz_mfma<N1, KIND, BF, true><<<dim3((unsigned)sg.nsub), dim3(256), 0, st>>>(
                            lv->view, eg->view, sg, r, x, reinterpret_cast<float *>(eg->d_stage),
                            eg->d_stage_scale, omega);
                } else
                    k_schwarz_mfma<N1, KIND, BF, false><<<dim3((unsigned)sg.nsub), dim3(256), 0, st>>>(
                        lv->view, eg->view, sg, r, x, nullptr, nullptr, omega);
                fts_status s = check_launch("k_schwarz_mfma");
                if (s != FTS_OK) return s;
            }
            if (staged) {
                if (cz > 1)  // the run kernel stores the values with their factor applied
                    launch_gather<D, N1, float, false>(lv, reinterpret_cast<const float *>(eg->d_stage), nullptr,
                                                       x, st, cz);
                else
                    launch_gather<D, N1, float, true>(lv, reinterpret_cast<const float *>(eg->d_stage),
                                                      eg->d_stage_scale, x, st);
                return check_launch("k_patch_gather");
            }
            return FTS_OK;
        }
    }
    // One color of the multiplicative smoother (Alg. multsmoother, Sec. 2.3):
    // red-black cells (color 0 / 1), or the 2^(d+1) vertex-patch colors with
    // the parquet color in the low d bits and the red-black parity inside the
    // parquet sub-lattice in bit d.  Subdomains of one color share no DoF (and
    // their local problems do not couple), so x is updated in place.
    template <int KIND>
    static SubGrid color_grid(const fts_eigs *eg, int color) {
        SubGrid sg{};
        sg.step = KIND ? 2 : 1;
        sg.nsub = 1;
        for (int a = 0; a < 3; ++a) {
            if (a >= D) {
                sg.cnt[a] = 1;
                sg.first[a] = 0;
                continue;
            }
            sg.first[a] = KIND ? ((color >> a) & 1) : 0;
            const int npos = eg->count[a];
            sg.cnt[a] = npos > sg.first[a] ? (npos - sg.first[a] + sg.step - 1) / sg.step : 0;
            sg.nsub *= sg.cnt[a];
        }
        sg.parity = KIND ? ((color >> D) & 1) : (color & 1);
        return sg;
    }
    template <int KIND, typename T>
    static fts_status go_color(const fts_level *lv, const fts_eigs *eg, double omega, const double *r, double *x,
                               int color, hipStream_t st) {
        using C = SwCfg<D, N1, KIND>;
        const SubGrid sg = color_grid<KIND>(eg, color);
        if (sg.nsub == 0) return FTS_OK;
        const int64_t blocks = (sg.nsub + C::PPB - 1) / C::PPB;
        if (blocks > INT_MAX) return fail(FTS_E_SIZE, "too many subdomains for one launch");
        k_schwarz<D, N1, KIND, T, false><<<dim3((unsigned)blocks), dim3(C::THREADS), 0, st>>>(
            lv->view, eg->view, sg, r, x, nullptr, omega);
        return check_launch("k_schwarz (color)");
    }
    template <int KIND, int BF>
    static fts_status go_color_mfma(const fts_level *lv, const fts_eigs *eg, double omega, const double *r,
                                    double *x, int color, hipStream_t st) {
        if constexpr (D != 3 || (KIND ? 2 * N1 : N1) > 16) {
            return fail(FTS_E_UNSUPPORTED, "16-bit MFMA contractions need d = 3 and n <= 16");
        } else {
            const SubGrid sg = color_grid<KIND>(eg, color);
            if (sg.nsub == 0) return FTS_OK;
            if (sg.nsub > INT_MAX) return fail(FTS_E_SIZE, "too many subdomains for one launch");
            k_schwarz_mfma<N1, KIND, BF, false><<<dim3((unsigned)sg.nsub), dim3(256), 0, st>>>(
                lv->view, eg->view, sg, r, x, nullptr, nullptr, omega);
            return check_launch("k_schwarz_mfma (color)");
        }
    }
    static fts_status run_color(const fts_level *lv, const fts_eigs *eg, double omega, fts_prec prec,
                                const double *r, double *x, int color, hipStream_t st) {
        const bool cell = eg->kind == FTS_CELL;
        if (prec == FTS_PREC_F16 || prec == FTS_PREC_BF16) {
            if (!eg->d_mfma) return fail(FTS_E_UNSUPPORTED, "16-bit MFMA contractions need n <= 16");
            if (prec == FTS_PREC_BF16)
                return cell ? go_color_mfma<0, 1>(lv, eg, omega, r, x, color, st)
                            : go_color_mfma<1, 1>(lv, eg, omega, r, x, color, st);
            return cell ? go_color_mfma<0, 0>(lv, eg, omega, r, x, color, st)
                        : go_color_mfma<1, 0>(lv, eg, omega, r, x, color, st);
        }
        if (prec == FTS_PREC_F64) {
            if constexpr (D == 3 && N1 == 8)
                if (!cell) {
                    const SubGrid sg = color_grid<1>(eg, color);
                    if (sg.nsub == 0) return FTS_OK;
                    if (sg.nsub > INT_MAX) return fail(FTS_E_SIZE, "too many subdomains for one launch");
                    k_schwarz_mfma64<N1, false><<<dim3((unsigned)sg.nsub), dim3(256), 0, st>>>(
                        lv->view, eg->view, sg, r, x, nullptr, omega);
                    return check_launch("k_schwarz_mfma64 (color)");
                }
            return cell ? go_color<0, double>(lv, eg, omega, r, x, color, st)
                        : go_color<1, double>(lv, eg, omega, r, x, color, st);
        }
        if (prec == FTS_PREC_F32)
            return cell ? go_color<0, float>(lv, eg, omega, r, x, color, st)
                        : go_color<1, float>(lv, eg, omega, r, x, color, st);
        return fail(FTS_E_UNSUPPORTED, "precision not built");
    }
    // FP64 vertex patches of extent 16 (3-D, k = 7): the MFMA kernel
    static fts_status go_mfma64(const fts_level *lv, const fts_eigs *eg, double omega, const double *r, double *x,
                                hipStream_t st) {
        if constexpr (D != 3 || N1 != 8) {
            return fail(FTS_E_UNSUPPORTED, "FP64 MFMA local solves need d = 3 and k = 7");
        } else {
            const bool staged = eg->schedule != FTS_SCHEDULE_COLORED;
            const int ncolor = staged ? 1 : 8;
            int cz = 1;
            for (int color = 0; color < ncolor; ++color) {
                SubGrid sg{};
                sg.parity = -1;
                sg.step = staged ? 1 : 2;
                sg.nsub = 1;
                for (int a = 0; a < 3; ++a) {
                    sg.first[a] = staged ? 0 : ((color >> a) & 1);
                    const int npos = eg->count[a];
                    sg.cnt[a] = npos > sg.first[a] ? (npos - sg.first[a] + sg.step - 1) / sg.step : 0;
                    sg.nsub *= sg.cnt[a];
                }
                if (sg.nsub == 0) continue;
                if (sg.nsub > INT_MAX) return fail(FTS_E_SIZE, "too many subdomains for one launch");
                if (staged) {
                    // runs of cz patches along z, as long as enough workgroups remain
                    while (cz < 8 && sg.nsub / (2 * cz) >= 6144) cz *= 2;
                    if (cz > 1)
                        k_schwarz_mfma64<N1, true, true>
                            <<<dim3((unsigned)((int64_t)sg.cnt[0] * sg.cnt[1] * ((sg.cnt[2] + cz - 1) / cz))),
                               dim3(256), 0, st>>>(lv->view, eg->view, sg, r, x, eg->d_stage, omega, cz);
                    else
                        k_schwarz_mfma64<N1, true><<<dim3((unsigned)sg.nsub), dim3(256), 0, st>>>(
                            lv->view, eg->view, sg, r, x, eg->d_stage, omega);
                } else
                    k_schwarz_mfma64<N1, false><<<dim3((unsigned)sg.nsub), dim3(256), 0, st>>>(
                        lv->view, eg->view, sg, r, x, nullptr, omega);
                fts_status s = check_launch("k_schwarz_mfma64");
                if (s != FTS_OK) return s;
            }
            if (staged) {
                launch_gather<D, N1, double, false>(lv, eg->d_stage, nullptr, x, st, cz);
                return check_launch("k_patch_gather");
            }
            return FTS_OK;
        }
    }
    static fts_status run(const fts_level *lv, const fts_eigs *eg, double omega, fts_prec prec, const double *r,
                          double *x, hipStream_t st) {
        if (prec == FTS_PREC_F16 || prec == FTS_PREC_BF16) {
            if (!eg->d_mfma) return fail(FTS_E_UNSUPPORTED, "16-bit MFMA contractions need n <= 16");
            const bool bf = prec == FTS_PREC_BF16;
            if (eg->kind == FTS_CELL)
                return bf ? go_mfma<0, 1>(lv, eg, omega, r, x, st) : go_mfma<0, 0>(lv, eg, omega, r, x, st);
            return bf ? go_mfma<1, 1>(lv, eg, omega, r, x, st) : go_mfma<1, 0>(lv, eg, omega, r, x, st);
        }
        if (prec == FTS_PREC_F64) {
            if constexpr (D == 3 && N1 == 8)
                if (eg->kind == FTS_VERTEX_PATCH) return go_mfma64(lv, eg, omega, r, x, st);
            return eg->kind == FTS_CELL ? go<0, double>(lv, eg, omega, r, x, st) : go<1, double>(lv, eg, omega, r, x, st);
        }
        if (prec == FTS_PREC_F32)
            return eg->kind == FTS_CELL ? go<0, float>(lv, eg, omega, r, x, st) : go<1, float>(lv, eg, omega, r, x, st);
        return fail(FTS_E_UNSUPPORTED, "precision not built");
    }
};

fts_status launch_schwarz(const fts_level *lv, const fts_eigs *eg, double omega, fts_prec prec, const double *r,
                          double *x, hipStream_t stream) {
    return dispatch<RunSchwarz>(lv->dim, lv->n1, lv, eg, omega, prec, r, x, stream);
}

template <int D, int N1>
struct RunSchwarzColor {
    static fts_status run(const fts_level *lv, const fts_eigs *eg, double omega, fts_prec prec, const double *r,
                          double *x, int color, hipStream_t st) {
        return RunSchwarz<D, N1>::run_color(lv, eg, omega, prec, r, x, color, st);
    }
};

int schwarz_mult_colors(const fts_eigs *eg) {
    return eg->kind == FTS_CELL ? 2 : 2 << eg->level->dim;
}

fts_status launch_schwarz_color(const fts_level *lv, const fts_eigs *eg, double omega, fts_prec prec,
                                const double *r, double *x, int color, hipStream_t stream) {
    if (color < 0 || color >= schwarz_mult_colors(eg)) return fail(FTS_E_INVAL, "Schwarz color out of range");
    return dispatch<RunSchwarzColor>(lv->dim, lv->n1, lv, eg, omega, prec, r, x, color, stream);
}

template <int D, int N1>
struct RunTransfer {
    static fts_status run(const fts_level *c, const fts_level *f, const double *src, double *dst, bool restrict_,
                          hipStream_t st) {
        using C = XferCfg<D, N1>;
        const int64_t blocks = c->ncells;
        if (blocks == 0) return FTS_OK;
        if (blocks > INT_MAX) return fail(FTS_E_SIZE, "too many cells for one launch");
        if (restrict_)
            k_transfer<D, N1, true><<<dim3((unsigned)blocks), dim3(C::THREADS), 0, st>>>(c->view, f->view, src, dst);
        else
            k_transfer<D, N1, false><<<dim3((unsigned)blocks), dim3(C::THREADS), 0, st>>>(c->view, f->view, src, dst);
        return check_launch("k_transfer");
    }
};

fts_status launch_restrict(const fts_level *coarse, const fts_level *fine, const double *rf, double *bc,
                           hipStream_t stream) {
    return dispatch<RunTransfer>(coarse->dim, coarse->n1, coarse, fine, rf, bc, true, stream);
}

fts_status launch_prolongate(const fts_level *coarse, const fts_level *fine, const double *ec, double *xf,
                             hipStream_t stream) {
    return dispatch<RunTransfer>(coarse->dim, coarse->n1, coarse, fine, ec, xf, false, stream);
}

template <int D, int N1>
struct RunAssemble {
    static fts_status run(const fts_level *lv, const SlabBlocks &A, hipStream_t st) {
        const int64_t N = lv->ndofs;
        k_assemble_slabs<D, N1><<<dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st>>>(lv->view, A, N);
        return check_launch("k_assemble_slabs");
    }
};

fts_status launch_assemble_slabs(const fts_level *lv, const SlabBlocks &A, hipStream_t stream) {
    return dispatch<RunAssemble>(lv->dim, lv->n1, lv, A, stream);
}

fts_status launch_fill(double *p, int64_t n, double v, hipStream_t stream) {
    if (n <= 0) return FTS_OK;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
    k_fill<<<dim3((unsigned)blocks), dim3(256), 0, stream>>>(p, n, v);
    return check_launch("k_fill");
}

}  // namespace fts

namespace fts {

// ---------------------------------------------------------------------------
// Level-1 vector kernels for the outer CG.  Dot products are deterministic
// two-stage reductions: fixed grid of kRedBlocks partial sums, then one block
// sums the partials in a fixed order.
constexpr int kRedBlocks = 1024;

__device__ __forceinline__ double block_sum(double v, double *sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    return s;
}

// partial[b][0] = sum x.y, partial[b][1] = sum x.z (z may be null)
__global__ void __launch_bounds__(256) k_dot2_partial(const double *__restrict__ x, const double *__restrict__ y,
                                                      const double *__restrict__ z, int64_t n, double *__restrict__ part) {
    __shared__ double sh[8];
    double a = 0.0, c = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        a = fma(x[i], y[i], a);
        if (z) c = fma(x[i], z[i], c);
    }
    const double sa = block_sum(a, sh);
    __syncthreads();
    const double sc = block_sum(c, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa;
        part[2 * blockIdx.x + 1] = sc;
    }
}

__global__ void __launch_bounds__(256) k_dot2_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
    __shared__ double sh[8];
    double a = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        a += part[2 * i];
        c += part[2 * i + 1];
    }
    const double sa = block_sum(a, sh);
    __syncthreads();
    const double sc = block_sum(c, sh);
    if (threadIdx.x == 0) {
        out[0] = sa;
        out[1] = sc;
    }
}

// x += alpha p; r -= alpha q
__global__ void __launch_bounds__(256) k_cg_update(double *__restrict__ x, double *__restrict__ r,
                                                   const double *__restrict__ p, const double *__restrict__ q,
                                                   double alpha, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        x[i] = fma(alpha, p[i], x[i]);
        r[i] = fma(-alpha, q[i], r[i]);
    }
}

// p = z + beta p
__global__ void __launch_bounds__(256) k_xpby(double *__restrict__ p, const double *__restrict__ z, double beta,
                                              int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = fma(beta, p[i], z[i]);
}

static unsigned vec_grid(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 8192); }

fts_status launch_dot2(const double *x, const double *y, const double *z, int64_t n, double *part, double *out,
                       hipStream_t st) {
    k_dot2_partial<<<kRedBlocks, 256, 0, st>>>(x, y, z, n, part);
    k_dot2_final<<<1, 256, 0, st>>>(part, kRedBlocks, out);
    return check_launch("dot products");
}

fts_status launch_cg_update(double *x, double *r, const double *p, const double *q, double alpha, int64_t n,
                            hipStream_t st) {
    k_cg_update<<<vec_grid(n), 256, 0, st>>>(x, r, p, q, alpha, n);
    return check_launch("k_cg_update");
}

__global__ void __launch_bounds__(256) k_scale(double *__restrict__ p, double a, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] *= a;
}

fts_status launch_scale(double *p, double a, int64_t n, hipStream_t st) {
    k_scale<<<vec_grid(n), 256, 0, st>>>(p, a, n);
    return check_launch("k_scale");
}

fts_status launch_xpby(double *p, const double *z, double beta, int64_t n, hipStream_t st) {
    k_xpby<<<vec_grid(n), 256, 0, st>>>(p, z, beta, n);
    return check_launch("k_xpby");
}

int red_partials() { return kRedBlocks; }

}  // namespace fts

namespace fts {

// ---------------------------------------------------------------------------
// Adjoint helper: derivative of the local solvers with respect to gamma_hat.
// For every subdomain j: u~ = Lambda^-1 Z^T R_j u, v~ = Lambda^-1 Z^T R_j v and
//   c_j = u~^T (sum_t I x..x D_t x..x I) v~,  D_t = Z_t^T (dA_t/dgamma_hat) Z_t,
// which equals (A_j^-1 R_j u)^T (dA_j/dgamma_hat) (A_j^-1 R_j v) because
// Z_t^T M_t Z_t = I (eq. generalizedEVP, eq. localsolverEVP).  One partial sum
// per workgroup.
template <int D, int N1, int KIND>
__global__ void __launch_bounds__((SwCfg<D, N1, KIND>::THREADS))
k_schwarz_dgamma(LevelView g, EigView e, SubGrid sg, const double *__restrict__ u, const double *__restrict__ v,
                 double *__restrict__ partials) {
    using C = SwCfg<D, N1, KIND>;
    constexpr int N = C::N, NT = C::NT, NC1 = C::NC1, NSC = C::NSC, LINES = C::LINES, PPB = C::PPB,
                  TH = C::THREADS;
    __shared__ double Tu[PPB * NT];
    __shared__ double Tv[PPB * NT];
    __shared__ double red[TH / 64];
    const int t = threadIdx.x;
    const int q = t / LINES, l = t % LINES;
    const int64_t s0 = (int64_t)blockIdx.x * PPB;
    auto position = [&](int64_t s, int *p) {
        const int j0 = (int)(s % sg.cnt[0]);
        const int64_t rr = s / sg.cnt[0];
        const int j1 = (int)(rr % sg.cnt[1]);
        const int j2 = (int)(rr / sg.cnt[1]);
        p[0] = sg.first[0] + sg.step * j0;
        p[1] = sg.first[1] + sg.step * j1;
        p[2] = D == 3 ? sg.first[2] + sg.step * j2 : 0;
    };
    const int64_t cs1 = g.m[0], cs2 = (int64_t)g.m[0] * g.m[1];
    for (int p = t; p < PPB * NSC * NC1; p += TH) {
        const int qq = p / (NSC * NC1), rem = p % (NSC * NC1), sc = rem / NC1, i = rem % NC1;
        const int64_t s = s0 + qq;
        if (s >= sg.nsub) continue;
        int pos[3];
        position(s, pos);
        const int o0 = sc & 1, o1 = (sc >> 1) & 1, o2 = (sc >> 2) & 1;
        const int64_t cell = (pos[0] + o0) + (pos[1] + o1) * cs1 + (D == 3 ? (pos[2] + o2) * cs2 : 0);
        const int i0 = i % N1, i1 = (i / N1) % N1, i2 = D == 3 ? i / (N1 * N1) : 0;
        const int lds = (o0 * N1 + i0) + (o1 * N1 + i1) * N + (D == 3 ? (o2 * N1 + i2) * N * N : 0);
        Tu[qq * NT + lds] = u[cell * NC1 + i];
        Tv[qq * NT + lds] = v[cell * NC1 + i];
    }
    __syncthreads();
    const int64_t s = s0 + q;
    const bool act = (q < PPB) && (s < sg.nsub);
    int pos[3] = {0, 0, 0};
    if (act) position(s, pos);
    for (int a = 0; a < D; ++a) {
        if (act) {
            contract_line<D, N, double>(Tu + q * NT, a, l, e.ST[a] + (size_t)pos[a] * N * N);
            contract_line<D, N, double>(Tv + q * NT, a, l, e.ST[a] + (size_t)pos[a] * N * N);
        }
        __syncthreads();
    }
    for (int p = t; p < PPB * NT; p += TH) {
        const int qq = p / NT, mm = p % NT;
        const int64_t ss = s0 + qq;
        if (ss >= sg.nsub) continue;
        int ps[3];
        position(ss, ps);
        const int m0 = mm % N, m1 = (mm / N) % N, m2 = D == 3 ? mm / (N * N) : 0;
        double lam = e.lam[0][(size_t)ps[0] * N + m0] + e.lam[1][(size_t)ps[1] * N + m1];
        if constexpr (D == 3) lam += e.lam[2][(size_t)ps[2] * N + m2];
        Tu[p] /= lam;
        Tv[p] /= lam;
    }
    __syncthreads();
    double acc = 0.0;
    if (act) {
        for (int a = 0; a < D; ++a) {
            const int base = line_base<D, N>(a, l), st = line_stride<N>(a);
            const double *Dt = e.DG[a] + (size_t)pos[a] * N * N;
            double in[N], out[N];
#pragma unroll
            for (int i = 0; i < N; ++i) in[i] = Tv[q * NT + base + i * st];
            matvec_regs<N>(in, out, Dt);
#pragma unroll
            for (int i = 0; i < N; ++i) acc = fma(Tu[q * NT + base + i * st], out[i], acc);
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((t & 63) == 0) red[t >> 6] = acc;
    __syncthreads();
    if (t == 0) {
        double sum = 0.0;
        for (int w = 0; w < TH / 64; ++w) sum += red[w];
        partials[blockIdx.x] = sum;
    }
}

template <int D, int N1>
struct RunDgamma {
    template <int KIND>
    static fts_status go(const fts_level *lv, const fts_eigs *eg, const double *u, const double *v, double *part,
                         int64_t *npart, hipStream_t st) {
        using C = SwCfg<D, N1, KIND>;
        SubGrid sg{};
        sg.parity = -1;
        sg.step = 1;
        sg.nsub = 1;
        for (int a = 0; a < 3; ++a) {
            sg.first[a] = 0;
            sg.cnt[a] = a < D ? eg->count[a] : 1;
            sg.nsub *= sg.cnt[a];
        }
        const int64_t blocks = (sg.nsub + C::PPB - 1) / C::PPB;
        *npart = blocks;
        if (blocks == 0) return FTS_OK;
        k_schwarz_dgamma<D, N1, KIND><<<dim3((unsigned)blocks), dim3(C::THREADS), 0, st>>>(lv->view, eg->view, sg,
                                                                                            u, v, part);
        return check_launch("k_schwarz_dgamma");
    }
    static fts_status run(const fts_level *lv, const fts_eigs *eg, const double *u, const double *v, double *part,
                          int64_t *npart, hipStream_t st) {
        return eg->kind == FTS_CELL ? go<0>(lv, eg, u, v, part, npart, st) : go<1>(lv, eg, u, v, part, npart, st);
    }
};

fts_status launch_schwarz_dgamma(const fts_level *lv, const fts_eigs *eg, const double *u, const double *v,
                                 double *partials, int64_t *npart, hipStream_t stream) {
    return dispatch<RunDgamma>(lv->dim, lv->n1, lv, eg, u, v, partials, npart, stream);
}

template <int D, int N1>
struct RunOperatorPen {
    static fts_status run(const fts_level *lv, const double *x, double *y, hipStream_t st) {
        using C = OpCfg<D, N1>;
        if (lv->ncells > INT_MAX) return fail(FTS_E_SIZE, "too many cells for one launch");
        const OpRuns runs = op_runs(lv->view.m, D, C::CPW);
        const int64_t blocks = runs.nblocks;
        if (blocks == 0) return FTS_OK;
        if (blocks > INT_MAX) return fail(FTS_E_SIZE, "too many cells for one launch");
        k_operator<D, N1, false, true><<<dim3((unsigned)blocks), dim3(C::THREADS), 0, st>>>(lv->view, runs, x, nullptr, y);
        return check_launch("k_operator (penalty)");
    }
};

fts_status launch_operator_penalty(const fts_level *lv, const double *x, double *y, hipStream_t stream) {
    return dispatch<RunOperatorPen>(lv->dim, lv->n1, lv, x, y, stream);
}

template <int D, int N1>
struct OpCells {
    static int run() { return OpCfg<D, N1>::CPW; }
};
int operator_cells_per_block(int dim, int n1) {
    const int r = dispatch<OpCells>(dim, n1);
    return r > 0 ? r : 1;
}

__global__ void __launch_bounds__(256) k_dot2_final_acc(const double *__restrict__ part, int nb, double scale,
                                                        double *__restrict__ out) {
    __shared__ double sh[8];
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) a += part[2 * i];
    const double sa = block_sum(a, sh);
    if (threadIdx.x == 0) out[0] += scale * sa;
}

__global__ void __launch_bounds__(256) k_sum_partial(const double *__restrict__ x, int64_t n, double *__restrict__ part) {
    __shared__ double sh[8];
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a += x[i];
    const double sa = block_sum(a, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sa;
        part[2 * blockIdx.x + 1] = 0.0;
    }
}

__global__ void __launch_bounds__(256) k_axpy(double a, const double *__restrict__ x, double *__restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        y[i] = fma(a, x[i], y[i]);
}

fts_status launch_dot_acc(const double *x, const double *y, int64_t n, double scale, double *part, double *out,
                          hipStream_t st) {
    k_dot2_partial<<<kRedBlocks, 256, 0, st>>>(x, y, nullptr, n, part);
    k_dot2_final_acc<<<1, 256, 0, st>>>(part, kRedBlocks, scale, out);
    return check_launch("dot (accumulate)");
}

fts_status launch_sum_acc(const double *x, int64_t n, double scale, double *part, double *out, hipStream_t st) {
    k_sum_partial<<<kRedBlocks, 256, 0, st>>>(x, n, part);
    k_dot2_final_acc<<<1, 256, 0, st>>>(part, kRedBlocks, scale, out);
    return check_launch("sum (accumulate)");
}

fts_status launch_axpy(double a, const double *x, double *y, int64_t n, hipStream_t st) {
    k_axpy<<<vec_grid(n), 256, 0, st>>>(a, x, y, n);
    return check_launch("k_axpy");
}

}  // namespace fts
