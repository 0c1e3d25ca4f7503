// Device helpers shared by the HIP kernels: tensor line geometry, the
// "one thread per 1-D line" contractions, launch configurations, and the
// (dimension, degree) dispatch to template instances.
#pragma once

#include <type_traits>

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
//   (A x)_K = sum_t (prod_{s != t} h_s Mhat_s) W_t
//   W_t = A_t^K x_K + B_t(K, K+e_t) x_{K+e_t} + B_t(K-e_t, K)^T x_{K-e_t}
// with the 1-D cell operator A_t^K = Lhat / h + (Nitsche terms of both faces)
// and the interface blocks B_t.  With the nodal Gauss-Lobatto basis the value
// at an end of the cell is the end coefficient, so every face term is rank one
// or two in the end values and the end derivatives d0, d1 (eq. 1Dnitsche,
// eq. 1Dsipginterface): the kernels need only the reference tables Lhat,
// Mhat, d0, d1 (the same for every cell) and a few widths per cell.  That
// frees the mapping of cells to lanes: a workgroup takes CPW cells so that
// its lanes are nearly all busy.
template <int D, int N1>
struct OpCfg {
    static constexpr int NC = ipow(N1, D);
    static constexpr int LINES = ipow(N1, D - 1);
    // workgroup size (64..256) wasting the fewest lanes on whole cells
    static constexpr int pick_threads() {
        int best = 64, best_used = 0;
        for (int th = 64; th <= 256; th += 64) {
            const int used = (th / LINES) * LINES;
            if (used * best > best_used * th) best = th, best_used = used;
        }
        return best;
    }
    static constexpr int THREADS = pick_threads();
    static constexpr int CPW = THREADS / LINES;  // cells per workgroup
    // LDS pitch of a line along x: odd, so that lanes reading consecutive
    // x-lines hit different banks
    static constexpr int P = N1 | 1;
    static constexpr int SLOT = D == 3 ? P * N1 * N1 : P * N1;
};

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
    int parity;    // -1: every subdomain; 0 / 1: only those with j0 + j1 + j2 of this parity
                   // (j = index inside this launch's grid; red-black colors)
    int64_t nsub;
};

// Is subdomain s (index within the launch) part of it under sg.parity?
__device__ __forceinline__ bool sub_in_color(const SubGrid &sg, int64_t s) {
    if (sg.parity < 0) return true;
    const int j0 = (int)(s % sg.cnt[0]);
    const int64_t rr = s / sg.cnt[0];
    const int j1 = (int)(rr % sg.cnt[1]), j2 = (int)(rr / sg.cnt[1]);
    return ((j0 + j1 + j2) & 1) == sg.parity;
}

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

// Contractions with a mirror-symmetric eigenbasis (EigView::sym): S (N x N,
// N even, row-major [i][m]) has its N/2 even columns first (S[N-1-i][m] =
// S[i][m]) and its N/2 odd ones last (S[N-1-i][m] = -S[i][m]), so only the
// rows i < N/2 are read and each product costs half the FMAs.
// out = S^T in, with ST = S^T (row-major [m][i]: each output reads N/2
// contiguous coefficients, so few scalar registers are live at a time):
template <int N, typename T, typename P>
__device__ __forceinline__ void eo_fwd(const T *in, T *out, P ST) {
    constexpr int H = N / 2;
    T ue[H], uo[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        ue[j] = in[j] + in[N - 1 - j];
        uo[j] = in[j] - in[N - 1 - j];
    }
#pragma unroll
    for (int m = 0; m < H; ++m) {
        T se = 0, so = 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            se = fma((T)ST[m * N + i], ue[i], se);
            so = fma((T)ST[(H + m) * N + i], uo[i], so);
        }
        out[m] = se;
        out[H + m] = so;
    }
}
// out = S c:
template <int N, typename T, typename P>
__device__ __forceinline__ void eo_bwd(const T *c, T *out, P S) {
    constexpr int H = N / 2;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        T ve = 0, vo = 0;
#pragma unroll
        for (int m = 0; m < H; ++m) {
            ve = fma((T)S[i * N + m], c[m], ve);
            vo = fma((T)S[i * N + H + m], c[H + m], vo);
        }
        out[i] = ve + vo;
        out[N - 1 - i] = ve - vo;
    }
}

// Line of N values at Tq[base + i st] <- Mat * line.
template <int N, typename T, typename P>
__device__ __forceinline__ void contract_at(T *Tq, int base, int st, P Mat) {
    T in[N], out[N];
#pragma unroll
    for (int i = 0; i < N; ++i) in[i] = Tq[base + i * st];
    matvec_regs<N>(in, out, Mat);
#pragma unroll
    for (int i = 0; i < N; ++i) Tq[base + i * st] = out[i];
}

template <int D, int N, typename T, typename P>
__device__ __forceinline__ void contract_line(T *Tq, int a, int l, P Mat) {
    contract_at<N>(Tq, line_base<D, N>(a, l), line_stride<N>(a), Mat);
}

// 1/d from the hardware reciprocal refined by Newton steps, each of which
// squares the relative error: within a few units in the last place of the
// correctly rounded quotient, at a third of the instructions of IEEE division.
__device__ __forceinline__ double recip(double d) {
    double y = __builtin_amdgcn_rcp(d);
    y = fma(y, fma(-d, y, 1.0), y);
    return fma(y, fma(-d, y, 1.0), y);
}
__device__ __forceinline__ float recip(float d) {
    const float y = __builtin_amdgcn_rcpf(d);
    return fmaf(y, fmaf(-d, y, 1.0f), y);
}

// Last axis: forward transform, eigenvalue scaling and backward transform of
// the same line, kept in registers.  lam_rest = lambda of the other axes at
// this line's fixed mode indices.
template <int N, typename T, typename P, typename Q>
__device__ __forceinline__ void last_axis_solve_at(T *Tq, int base, int st, P ST, P S, Q lam_last, T lam_rest,
                                                   T omega) {
    T in[N], mid[N];
#pragma unroll
    for (int i = 0; i < N; ++i) in[i] = Tq[base + i * st];
    matvec_regs<N>(in, mid, ST);
#pragma unroll
    for (int m = 0; m < N; ++m) mid[m] = mid[m] * (omega * recip(lam_rest + (T)lam_last[m]));
    matvec_regs<N>(mid, in, S);
#pragma unroll
    for (int i = 0; i < N; ++i) Tq[base + i * st] = in[i];
}

template <int D, int N, typename T, typename P, typename Q>
__device__ __forceinline__ void last_axis_solve(T *Tq, int l, P ST, P S, Q lam_last, T lam_rest, T omega) {
    constexpr int a = D - 1;
    last_axis_solve_at<N>(Tq, line_base<D, N>(a, l), line_stride<N>(a), ST, S, lam_last, lam_rest, omega);
}

// ---------------------------------------------------------------------------
// Dispatch on (dim, degree) to the template instances.
template <template <int, int> class F, typename... Args>
fts_status dispatch(int dim, int n1, Args &&...args) {
#define FTS_CASE(DD, NN) \
    if (dim == DD && n1 == NN) return F<DD, NN>::run(args...);
    FTS_CASE(2, 2) FTS_CASE(2, 3) FTS_CASE(2, 4) FTS_CASE(2, 5) FTS_CASE(2, 6) FTS_CASE(2, 7)
    FTS_CASE(2, 8) FTS_CASE(2, 9) FTS_CASE(2, 10) FTS_CASE(2, 11) FTS_CASE(2, 12) FTS_CASE(2, 13)
    FTS_CASE(2, 14) FTS_CASE(2, 15) FTS_CASE(2, 16)
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


// One 1-D operator along axis t on a line of cell K (eq. 1Dsipg with the
// interface blocks of eq. 1Dsipginterface): in = the line of K, nl / nr = the
// same line in the neighbours K - e_t / K + e_t (used when present), ih, ihl,
// ihr = inverse widths, gk = gamma_hat k (k+1).  PEN: only the penalty terms,
// i.e. dA/dgamma_hat with gk = k (k+1).
// out = scale * Mat in on one line, Mat centro-symmetric (Mat[i][j] =
// Mat[n-1-i][n-1-j], true of the reference mass and stiffness because the
// nodes are symmetric about the cell centre), from its even-odd form: with
// h = n / 2 and he = (n + 1) / 2, E (he x he) acts on the sums
// in_j + in_{n-1-j} (and the middle value for odd n), O (h x h) on the
// differences in_j - in_{n-1-j}, and out_i, out_{n-1-i} are the sum and the
// difference of the two results.  Half the multiplications of a plain
// matrix-vector product, and half the table.
template <int N, typename P>
__device__ __forceinline__ void eo_matvec(const double *in, double *out, double scale, P E, P O) {
    constexpr int H = N / 2, HE = (N + 1) / 2;
    double ue[HE], uo[H > 0 ? H : 1];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        ue[j] = in[j] + in[N - 1 - j];
        uo[j] = in[j] - in[N - 1 - j];
    }
    if constexpr (N % 2) ue[H] = in[H];
    // E and O are symmetric (so are Mhat and Lhat): only their upper triangles
    // are read, which keeps fewer of their entries in scalar registers
#pragma unroll
    for (int i = 0; i < HE; ++i) {
        double se = 0.0;
#pragma unroll
        for (int j = 0; j < HE; ++j) se = fma((double)E[i <= j ? i * HE + j : j * HE + i], ue[j], se);
        if (i < H) {
            double so = 0.0;
#pragma unroll
            for (int j = 0; j < H; ++j) so = fma((double)O[i <= j ? i * H + j : j * H + i], uo[j], so);
            out[i] = (se + so) * scale;
            out[N - 1 - i] = (se - so) * scale;
        } else {
            out[i] = se * scale;
        }
    }
}

template <int N1, bool PEN, typename P>
__device__ __forceinline__ void sipg_line(const double *in, const double *nl, const double *nr, bool hasl, bool hasr,
                                          double ih, double ihl, double ihr, double gk, P LE, P LO, P d0,
                                          double *out) {
    // derivatives of the basis at the right end: phi_j'(1) = -phi_{n-1-j}'(0)
    // (Gauss-Lobatto nodes symmetric about the midpoint), so only d0 is read
    auto d1 = [&](int j) { return -(double)d0[N1 - 1 - j]; };
    const double eta0 = hasl ? 0.5 : 1.0, eta1 = hasr ? 0.5 : 1.0;
    const double g0 = hasl ? gk * (ih + ihl) : 2.0 * gk * ih;
    const double g1 = hasr ? gk * (ih + ihr) : 2.0 * gk * ih;
    const double x0 = in[0], xn = in[N1 - 1];
    if constexpr (PEN) {
#pragma unroll
        for (int o = 0; o < N1; ++o) out[o] = 0.0;
        out[0] = eta0 * g0 * x0;
        out[N1 - 1] += eta1 * g1 * xn;
        if (hasl) out[0] -= 0.5 * g0 * nl[N1 - 1];
        if (hasr) out[N1 - 1] -= 0.5 * g1 * nr[0];
    } else {
        eo_matvec<N1>(in, out, ih, LE, LO);
        double dx0 = 0.0, dxn = 0.0;
#pragma unroll
        for (int j = 0; j < N1; ++j) {
            dx0 = fma((double)d0[j], in[j], dx0);
            dxn = fma(d1(j), in[j], dxn);
        }
        double e0 = eta0 * (g0 * x0 + ih * dx0);   // added to out[0]
        double en = eta1 * (g1 * xn - ih * dxn);   // added to out[N1-1]
        double c0 = eta0 * ih * x0, c1 = -eta1 * ih * xn;  // coefficients of d0, d1
        if (hasl) {
            double dl = 0.0;
#pragma unroll
            for (int j = 0; j < N1; ++j) dl = fma(d1(j), nl[j], dl);
            const double xl = nl[N1 - 1];
            e0 += 0.5 * (dl * ihl - g0 * xl);
            c0 -= 0.5 * ih * xl;
        }
        if (hasr) {
            double dr = 0.0;
#pragma unroll
            for (int j = 0; j < N1; ++j) dr = fma((double)d0[j], nr[j], dr);
            const double xr = nr[0];
            en -= 0.5 * (dr * ihr + g1 * xr);
            c1 += 0.5 * ih * xr;
        }
        out[0] += e0;
        out[N1 - 1] += en;
#pragma unroll
        for (int o = 0; o < N1; ++o) out[o] = fma((double)d0[o], c0, fma(d1(o), c1, out[o]));
    }
}

// y = A x (RES: y = b - A x) on the nact <= CPW cells cell0, cell0+1, ... of the mesh
// described by g (x, b, y: that mesh's vectors).  Shared by the single-mesh
// and the batched kernels.  Thread (q, l) works on cell cell0 + q and is in
// turn the owner of line l along x, along y and along z; it reads the lines
// of the neighbours (and, for k >= 5, of its own cell) straight from global
// memory (every such read is a coalesced run along x or a set of them).  LDS
// per cell: two work slots U, V (and the cell's coefficients X for k <= 4),
// lines along x padded to an odd pitch.  Sequence (3-D),
// M = the reference mass (even-odd form) times the widths named:
//   x-lines: W_x -> U                       y-lines: U <- h_y h_z M U, W_y -> V
//   x-lines: U += h_x h_z M V               z-lines: U <- M U,         W_z -> V
//   y-lines: V <- h_x h_y M V               x-lines: y = U + M V (or b - ...)
template <int D, int N1, bool RES, bool PEN = false, typename TY = double>
__device__ __forceinline__ void operator_cells(const LevelView &g, int64_t cell0, int nact,
                                               const double *__restrict__ x, const double *__restrict__ b,
                                               TY *__restrict__ y) {
    using C = OpCfg<D, N1>;
    constexpr int NC = C::NC, LINES = C::LINES, CPW = C::CPW, P = C::P, SL = C::SLOT;
    constexpr int HE = (N1 + 1) / 2;
    // XL: the cell's own coefficients are staged in LDS (slot X) instead of
    // being read from global memory once per axis.  Pays for small cells; from
    // k = 5 on, the third slot costs more occupancy than the re-reads cost.
    constexpr bool XL = N1 <= 5;
    __shared__ double S[CPW][XL ? 3 : 2][SL];
    const int t = threadIdx.x;
    const int q = t / LINES, l = t % LINES;
    const int64_t cell = cell0 + q;
    const bool act = q < nact;
    const cptr<double> LE = uniform_table(g.Leo), ME = uniform_table(g.Meo);
    const cptr<double> LO = LE + HE * HE, MO = ME + HE * HE;
    const cptr<double> d0 = uniform_table(g.d0);
    const double gk = PEN ? g.pk : g.gk;
    // padded LDS index of cell-local coefficient (i0, i1, i2)
    auto li = [](int i0, int i1, int i2) { return i0 + P * (i1 + N1 * i2); };
    constexpr int X = 2;
    if constexpr (XL) {
        const int ncopy = nact * NC;
        const double *src = x + cell0 * NC;
        for (int e = t; e < ncopy; e += C::THREADS) {
            const int qq = e / NC, i = e % NC;
            const int i0 = i % N1, rest = i / N1;
            S[qq][X][i0 + P * rest] = src[e];
        }
        __syncthreads();
    }
    int c[3] = {0, 0, 0};
    double h[3] = {1.0, 1.0, 1.0};
    const int64_t cs[3] = {1, g.m[0], (int64_t)g.m[0] * g.m[1]};
    if (act) {
        const int cc = (int)cell, r0 = cc / g.m[0];
        c[0] = cc - r0 * g.m[0];
        c[1] = D == 3 ? r0 % g.m[1] : r0;
        c[2] = D == 3 ? r0 / g.m[1] : 0;
#pragma unroll
        for (int a = 0; a < D; ++a) h[a] = g.h[a][c[a]];
    }
    // line l along axis a: its fixed cell-local indices
    auto line_idx = [&](int a, int j) {  // global offset (within a cell) of element j of line l along a
        if constexpr (D == 3) {
            const int u = l % N1, v = l / N1;
            return a == 0 ? j + N1 * (u + N1 * v) : (a == 1 ? u + N1 * (j + N1 * v) : u + N1 * (v + N1 * j));
        } else {
            return a == 0 ? j + N1 * l : l + N1 * j;
        }
    };
    auto lds_idx = [&](int a, int j) {
        if constexpr (D == 3) {
            const int u = l % N1, v = l / N1;
            return a == 0 ? li(j, u, v) : (a == 1 ? li(u, j, v) : li(u, v, j));
        } else {
            return a == 0 ? li(j, l, 0) : li(l, j, 0);
        }
    };
    // W_a on this thread's line along axis a
    auto w_line = [&](int a, double *w) {
        double in[N1], nl[N1], nr[N1];
        if constexpr (XL) {
#pragma unroll
            for (int j = 0; j < N1; ++j) in[j] = S[q][X][lds_idx(a, j)];
        } else {
            const double *own = x + cell * NC;
#pragma unroll
            for (int j = 0; j < N1; ++j) in[j] = own[line_idx(a, j)];
        }
        const bool hasl = c[a] > 0, hasr = c[a] + 1 < g.m[a];
        double ihl = 1.0, ihr = 1.0;
        if (hasl) {
            const double *src = x + (cell - cs[a]) * NC;
#pragma unroll
            for (int j = 0; j < N1; ++j) nl[j] = src[line_idx(a, j)];
            ihl = g.ih[a][c[a] - 1];
        }
        if (hasr) {
            const double *src = x + (cell + cs[a]) * NC;
#pragma unroll
            for (int j = 0; j < N1; ++j) nr[j] = src[line_idx(a, j)];
            ihr = g.ih[a][c[a] + 1];
        }
        sipg_line<N1, PEN>(in, nl, nr, hasl, hasr, g.ih[a][c[a]], ihl, ihr, gk, LE, LO, d0, w);
    };
    auto ld = [&](int slot, int a, double *v) {
#pragma unroll
        for (int j = 0; j < N1; ++j) v[j] = S[q][slot][lds_idx(a, j)];
    };
    auto st = [&](int slot, int a, const double *v) {
#pragma unroll
        for (int j = 0; j < N1; ++j) S[q][slot][lds_idx(a, j)] = v[j];
    };
    auto mass = [&](const double *in, double *out, double scale) { eo_matvec<N1>(in, out, scale, ME, MO); };
    constexpr int U = 0, V = 1;
    double w[N1], v[N1], m[N1];
    if constexpr (D == 3) {
        if (act) {
            w_line(0, w);
            st(U, 0, w);
        }
        __syncthreads();
        if (act) {
            ld(U, 1, v);
            mass(v, m, h[1] * h[2]);
            st(U, 1, m);
            w_line(1, w);
            st(V, 1, w);
        }
        __syncthreads();
        if (act) {
            ld(V, 0, v);
            mass(v, m, h[0] * h[2]);
            ld(U, 0, v);
#pragma unroll
            for (int j = 0; j < N1; ++j) v[j] += m[j];
            st(U, 0, v);
        }
        __syncthreads();
        if (act) {
            ld(U, 2, v);
            mass(v, m, 1.0);
            st(U, 2, m);
            w_line(2, w);
            st(V, 2, w);
        }
        __syncthreads();
        if (act) {
            ld(V, 1, v);
            mass(v, m, h[0] * h[1]);
            st(V, 1, m);
        }
        __syncthreads();
        if (act) {
            ld(V, 0, v);
            mass(v, m, 1.0);
            ld(U, 0, v);
            TY *dst = y + cell * NC + line_idx(0, 0);
            if constexpr (RES) {
                const double *bb = b + cell * NC + line_idx(0, 0);
#pragma unroll
                for (int j = 0; j < N1; ++j) dst[j] = (TY)(bb[j] - (v[j] + m[j]));
            } else {
#pragma unroll
                for (int j = 0; j < N1; ++j) dst[j] = (TY)(v[j] + m[j]);
            }
        }
    } else {
        if (act) {
            w_line(0, w);
            st(U, 0, w);
        }
        __syncthreads();
        if (act) {
            ld(U, 1, v);
            mass(v, m, h[1]);
            st(U, 1, m);
            w_line(1, w);
            st(V, 1, w);
        }
        __syncthreads();
        if (act) {
            ld(V, 0, v);
            mass(v, m, h[0]);
            ld(U, 0, v);
            TY *dst = y + cell * NC + line_idx(0, 0);
            if constexpr (RES) {
                const double *bb = b + cell * NC + line_idx(0, 0);
#pragma unroll
                for (int j = 0; j < N1; ++j) dst[j] = (TY)(bb[j] - (v[j] + m[j]));
            } else {
#pragma unroll
                for (int j = 0; j < N1; ++j) dst[j] = (TY)(v[j] + m[j]);
            }
        }
    }
}

}  // namespace fts
