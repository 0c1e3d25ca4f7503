// Direct solver of the coarsest level (Alg. gmg, level 0): LU factorisation
// of A_0 without pivoting, applied by forward and backward substitution.  A_0
// is symmetric positive definite, for which elimination without pivoting is
// stable.
//
// Structure.  Unknowns are numbered cell by cell with the last axis slowest,
// so each slab of cells (one coordinate along the last axis) is a contiguous
// range of B unknowns and couples only to its two neighbouring slabs: A_0 is
// block tridiagonal over the nb slabs (SlabBlocks).  Elimination creates no
// fill outside that band, so the factors are block bidiagonal,
//     L: diagonal L_ii, below it Lo_i = A_{i+1,i} U_ii^-1,
//     U: diagonal U_ii, above it Up_i = L_ii^-1 A_{i,i+1},
// the same numbers a dense LU of A_0 produces, with the exact zeros left out.
//
// Low rank between slabs.  A cell couples to the cell across its face on the
// next slab only through face terms (eq. bfsipg), and every face quantity of
// a cell at its top face (the trace and the gradient at any point of the
// face, on Cartesian and on mapped cells alike) is a linear function of the
// r = 2 (k+1)^(d-1) numbers T u: for every node line along the last axis,
// the nodal value at the top end and the derivative of the line's 1-D
// interpolant there.  Hence, with T = diag over the cells of a slab,
//     A_{i+1,i} = P_i T,   P_i = A_{i+1,i} T^+   (block diagonal over cells)
//     A_{i,i+1} = T^T R_i, R_i = (T^+)^T A_{i,i+1}
// (T T^T = G x I with the 2 x 2 Gram matrix G of the two end functionals, so
// T^+ = T^T (G^-1 x I) in closed form), and the blocks of the factors are
//     Lo_i = P_i W_i with W_i = T inv(U_ii): row (cell c, j) zero left of c,
//     Up_i = V_i R_i with V_i = inv(L_ii) T^T: row of cell c zero right of
//                                              the columns of cell c.
// W_i and V_i have r instead of (k+1)^d rows (resp. columns) per cell, so
// the substitution reads 2 r / (k+1)^d of the bytes of Lo_i and Up_i (0.4 at
// k = 4 in 3-D).  Lo_i and Up_i themselves are needed only for the Schur
// updates of the setup.
//
// Setup (once): P_i and R_i from the assembled off-diagonal blocks; block
// elimination over the slabs with library BLAS-3 (GEMM, TRSM) and a
// one-workgroup kernel for the small diagonal panels; then the diagonal
// factors are replaced by their inverses (strict lower part inv(L_ii) with
// unit diagonal implied, upper part inv(U_ii)), W_i and V_i are formed from
// them, and Lo_i, Up_i are released.
//
// Solve (every V-cycle), every step a matrix-vector product:
//     forward   y_0 = inv(L_00) b_0,
//               y_{i+1} = inv(L_{i+1,i+1}) (b_{i+1} - P_i (W_i y_i))
//     backward  x_last = inv(U) y_last,
//               x_i = inv(U_ii) (y_i - V_i (R_i x_{i+1}))
// The diagonal blocks are read once in full (their lower half forward, upper
// half backward), W_i and V_i in their nonzero parts, P_i and R_i (r (k+1)^d
// numbers per cell) once each.
#include <rocblas/rocblas.h>

#include <climits>

#include "device_common.h"

namespace fts {

struct CoarseLU {
    int64_t N = 0;
    int B = 0, nb = 0, nc = 0;   // slab size, number of slabs, unknowns per cell
    int ncs = 0, rc = 0, Rl = 0;  // cells per slab, face numbers per cell, Rl = ncs rc
    double *D = nullptr;          // nb blocks B x B: packed inv(L_ii), inv(U_ii)
    double *Lo = nullptr;         // setup only: nb - 1 blocks A_{i+1,i}, then Lo_i
    double *Up = nullptr;         // setup only: nb - 1 blocks A_{i,i+1}, then Up_i
    double *W = nullptr;          // nb - 1 blocks Rl x B: W_i = T inv(U_ii)
    double *V = nullptr;          // nb - 1 blocks B x Rl: V_i = inv(L_ii) T^T
    double *Pt = nullptr;         // nb - 1 blocks: P_i per cell, [cell][unknown][face number]
    double *Rt = nullptr;         // nb - 1 blocks: R_i per cell, [cell][face number][unknown]
    double *y = nullptr;          // N: result of the forward substitution
    double *t = nullptr;          // B: right-hand side of the current diagonal step
    double *s = nullptr;          // Rl: face numbers of the current off-diagonal step
};

// The face functionals of the top face (last axis, xi = 1) of a cell: face
// number a = kind * nxy + q takes sum_z f[kind][z] u[q + z nxy] over the node
// line q (f[0] = phi(1), f[1] = phi'(1)); ginv = G^-1 of their Gram matrix.
struct FaceMap {
    double f[2][kMaxN1Any];
    double ginv[2][2];
    int n1, nxy, nc, rc;
};

constexpr int kNB = 256;  // panel width of the factorisation

#define COARSE_TRY(expr)                  \
    do {                                  \
        const fts_status s_ = (expr);     \
        if (s_ != FTS_OK) return s_;      \
    } while (0)

__global__ void __launch_bounds__(1024) k_lu_diag(double *__restrict__ A, int64_t lda, int kb) {
    const int tid = threadIdx.x;
    for (int j = 0; j < kb; ++j) {
        __syncthreads();
        const double piv = A[j + j * lda];
        for (int i = j + 1 + tid; i < kb; i += blockDim.x) A[i + j * lda] /= piv;
        __syncthreads();
        const int w = kb - j - 1;
        for (int e = tid; e < w * w; e += blockDim.x) {
            const int i = j + 1 + e % w, c = j + 1 + e / w;
            A[i + (int64_t)c * lda] -= A[i + j * lda] * A[j + (int64_t)c * lda];
        }
    }
}

// ---------------------------------------------------------------------------
// Block mat-vec out = base + sgn * (M v) over one R x C block M stored
// row-major, restricted to the block's nonzero part.  Row r of each part
// occupies one contiguous column range:
//     kLowerInv  strict lower part of a packed diagonal block (R = C = B):
//                [0, r)  (the unit diagonal comes in through base = v)
//     kUpperInv  upper part of a packed diagonal block:    [r, B)
//     kBelowLR   W_i (R = Rl, C = B), row of cell c:        [c nc, B)
//     kAboveLR   V_i (R = B, C = Rl), row of cell c:        [0, (c + 1) rc)
// The rows are cut into groups of ROWS; a workgroup owns group g and group
// G-1-g, a short and a long range, so every workgroup streams about the same
// number of bytes.  Its waves take interleaved passes of 64 lanes x two
// columns over each range (16-byte non-temporal loads, one per row and
// lane, the loads of kUnroll passes issued before their FMAs), keep one
// partial per row and lane, and reduce across lanes with shuffles and across
// waves in LDS in a fixed order: no atomics, and the result does not depend
// on timing.
constexpr int kMvWaves = 8, kUnroll = 2;
typedef double dvec2 __attribute__((ext_vector_type(2)));

enum BlockPart { kLowerInv = 0, kUpperInv = 1, kBelowLR = 2, kAboveLR = 3 };

// Rows per group: the low-rank blocks have fewer rows (W_i) or shorter ones
// (V_i); two rows keep enough workgroups in flight for W_i, and spread the
// short rows of V_i over more workgroups (1.5 % faster coarse solve at 8^3 Q4
// than four).
template <int PART>
constexpr int part_rows() { return PART == kBelowLR || PART == kAboveLR ? 2 : 4; }

// Column range [lo, hi) covering the nonzero parts of rows [r0, r1].
template <int PART>
__device__ __forceinline__ void group_range(int r0, int r1, int C, int nc, int rc, int &lo, int &hi) {
    if (PART == kLowerInv) lo = 0, hi = r1;
    else if (PART == kUpperInv) lo = r0, hi = C;
    else if (PART == kBelowLR) lo = (r0 / rc) * nc, hi = C;
    else lo = 0, hi = (r1 / nc + 1) * rc;
}

// Entry (row, col) of the union range that lies outside the row's own part.
// Only the packed diagonal blocks need this: the low-rank blocks store their
// zeros.
template <int PART>
__device__ __forceinline__ bool outside(int row, int col) {
    if (PART == kLowerInv) return col >= row;
    if (PART == kUpperInv) return col < row;
    return false;
}

// acc[q] += sum over this lane's columns of row r0 + q (rows past r1 are
// loaded from row r1 and their sums dropped by the caller).  Passes
// p = wave, wave + kMvWaves, ... < np; pass p covers PC columns from lo + p PC.
template <int PART, bool PAIR, int ROWS>
__device__ __forceinline__ void stream_group(const double *__restrict__ M, int C, const double *__restrict__ v,
                                             int r0, int r1, int lo, int hi, int np, int wave, int lane,
                                             double *acc) {
    constexpr int CPL = PAIR ? 2 : 1, PC = 64 * CPL;
    const double *rowp[ROWS];
#pragma unroll
    for (int q = 0; q < ROWS; ++q) rowp[q] = M + (int64_t)min(r0 + q, r1) * C;
    int p = wave;
    for (; p + (kUnroll - 1) * kMvWaves < np; p += kUnroll * kMvWaves) {
        int jj[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int j = lo + (p + u * kMvWaves) * PC + CPL * lane;
            ok[u] = j < hi;
            jj[u] = ok[u] ? j : lo;
        }
        if constexpr (PAIR) {
            dvec2 x[kUnroll], m[kUnroll][ROWS];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                x[u] = *(const dvec2 *)(v + jj[u]);
#pragma unroll
                for (int q = 0; q < ROWS; ++q) m[u][q] = __builtin_nontemporal_load((const dvec2 *)(rowp[q] + jj[u]));
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int q = 0; q < ROWS; ++q) {
                    const double mx = (ok[u] && !outside<PART>(r0 + q, jj[u])) ? m[u][q].x : 0.0;
                    const double my = (ok[u] && !outside<PART>(r0 + q, jj[u] + 1)) ? m[u][q].y : 0.0;
                    acc[q] = fma(my, x[u].y, fma(mx, x[u].x, acc[q]));
                }
        } else {
            double x[kUnroll], m[kUnroll][ROWS];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                x[u] = v[jj[u]];
#pragma unroll
                for (int q = 0; q < ROWS; ++q) m[u][q] = rowp[q][jj[u]];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int q = 0; q < ROWS; ++q)
                    acc[q] = fma((ok[u] && !outside<PART>(r0 + q, jj[u])) ? m[u][q] : 0.0, x[u], acc[q]);
        }
    }
    for (; p < np; p += kMvWaves) {
        const int j = lo + p * PC + CPL * lane;
        const bool ok = j < hi;
        const int jj = ok ? j : lo;
        if constexpr (PAIR) {
            const dvec2 x = *(const dvec2 *)(v + jj);
            dvec2 m[ROWS];
#pragma unroll
            for (int q = 0; q < ROWS; ++q) m[q] = __builtin_nontemporal_load((const dvec2 *)(rowp[q] + jj));
#pragma unroll
            for (int q = 0; q < ROWS; ++q) {
                const double mx = (ok && !outside<PART>(r0 + q, jj)) ? m[q].x : 0.0;
                const double my = (ok && !outside<PART>(r0 + q, jj + 1)) ? m[q].y : 0.0;
                acc[q] = fma(my, x.y, fma(mx, x.x, acc[q]));
            }
        } else {
            const double x = v[jj];
            double m[ROWS];
#pragma unroll
            for (int q = 0; q < ROWS; ++q) m[q] = rowp[q][jj];
#pragma unroll
            for (int q = 0; q < ROWS; ++q) acc[q] = fma((ok && !outside<PART>(r0 + q, jj)) ? m[q] : 0.0, x, acc[q]);
        }
    }
}

template <int PART, bool PAIR>
__global__ void __launch_bounds__(64 * kMvWaves) k_slab_mv(const double *__restrict__ M, int R, int C, int nc, int rc,
                                                           int G, const double *__restrict__ v, const double *base,
                                                           double sgn, double *__restrict__ out) {
    constexpr int ROWS = part_rows<PART>();
    constexpr int PC = PAIR ? 128 : 64;  // columns per wave pass
    __shared__ double red[kMvWaves][2 * ROWS];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ga = blockIdx.x, gb = G - 1 - blockIdx.x;  // gb == ga: a single group
    int r0[2], r1[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        r0[s] = (s == 0 ? ga : gb) * ROWS;
        r1[s] = min(r0[s] + ROWS, R) - 1;
        int lo, hi;
        group_range<PART>(r0[s], r1[s], C, nc, rc, lo, hi);
        if (PAIR) lo &= ~1, hi = min(C, (hi + 1) & ~1);
        const int np = (s == 1 && gb == ga) || hi <= lo ? 0 : (hi - lo + PC - 1) / PC;
        double acc[ROWS];
#pragma unroll
        for (int q = 0; q < ROWS; ++q) acc[q] = 0.0;
        stream_group<PART, PAIR, ROWS>(M, C, v, r0[s], r1[s], lo, hi, np, wave, lane, acc);
#pragma unroll
        for (int q = 0; q < ROWS; ++q) {
            double t = acc[q];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
            if (lane == 0) red[wave][s * ROWS + q] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * ROWS) {
        const int s = threadIdx.x / ROWS, q = threadIdx.x % ROWS;
        const int row = r0[s] + q;
        if ((s == 0 || gb != ga) && row <= r1[s]) {
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < kMvWaves; ++w) sum += red[w][threadIdx.x];
            out[row] = (base ? base[row] : 0.0) + sgn * sum;
        }
    }
}

template <int PART>
static void slab_mv(const CoarseLU *c, const double *M, int R, int C, const double *v, const double *base, double sgn,
                    double *out, hipStream_t s) {
    constexpr int ROWS = part_rows<PART>();
    const int G = (R + ROWS - 1) / ROWS;
    const dim3 grid((G + 1) / 2);
    if (C % 2 == 0) k_slab_mv<PART, true><<<grid, 64 * kMvWaves, 0, s>>>(M, R, C, c->nc, c->rc, G, v, base, sgn, out);
    else k_slab_mv<PART, false><<<grid, 64 * kMvWaves, 0, s>>>(M, R, C, c->nc, c->rc, G, v, base, sgn, out);
}

// out[j] = base[j] - sum_a P_c[j][a] s[c rc + a] for the B unknowns j of a
// slab (c the cell of j): the expansion of the face numbers s by P_i.  One
// wave per unknown.
__global__ void __launch_bounds__(256) k_lr_expand(const double *__restrict__ Pt, const double *__restrict__ s,
                                                   const double *__restrict__ base, int nc, int rc, int B,
                                                   double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= B) return;  // whole waves leave together
    const int c = j / nc;
    const double *p = Pt + (int64_t)j * rc;
    const double *sc = s + (int64_t)c * rc;
    double acc = 0.0;
    for (int a = lane; a < rc; a += 64) acc = fma(p[a], sc[a], acc);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) out[j] = base[j] - acc;
}

// s[c rc + a] = sum_l R_c[a][l] x[c nc + l]: one wave per face number.
__global__ void __launch_bounds__(256) k_lr_reduce(const double *__restrict__ Rt, const double *__restrict__ x, int nc,
                                                   int rc, int Rl, double *__restrict__ s) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= Rl) return;  // whole waves leave together
    const int c = row / rc;
    const double *r = Rt + (int64_t)row * nc;
    const double *xc = x + (int64_t)c * nc;
    double acc = 0.0;
    for (int l = lane; l < nc; l += 64) acc = fma(r[l], xc[l], acc);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) s[row] = acc;
}

fts_status coarse_solve(CoarseLU *c, const double *b, double *x, hipStream_t s) {
    const int64_t B = c->B, BB = B * B, BR = B * (int64_t)c->Rl, PR = (int64_t)c->ncs * c->rc * c->nc;
    const unsigned gexp = (unsigned)((B + 3) / 4), gred = (unsigned)((c->Rl + 3) / 4);
    for (int i = 0; i < c->nb; ++i) {
        const double *rhs = i == 0 ? b : c->t;
        slab_mv<kLowerInv>(c, c->D + i * BB, c->B, c->B, rhs, rhs, 1.0, c->y + i * B, s);
        if (i + 1 < c->nb) {
            slab_mv<kBelowLR>(c, c->W + i * BR, c->Rl, c->B, c->y + i * B, nullptr, 1.0, c->s, s);
            k_lr_expand<<<gexp, 256, 0, s>>>(c->Pt + i * PR, c->s, b + (i + 1) * B, c->nc, c->rc, c->B, c->t);
        }
    }
    for (int i = c->nb - 1; i >= 0; --i) {
        const double *rhs = i == c->nb - 1 ? c->y + i * B : c->t;
        slab_mv<kUpperInv>(c, c->D + i * BB, c->B, c->B, rhs, nullptr, 1.0, x + i * B, s);
        if (i > 0) {
            k_lr_reduce<<<gred, 256, 0, s>>>(c->Rt + (i - 1) * PR, x + i * B, c->nc, c->rc, c->Rl, c->s);
            slab_mv<kAboveLR>(c, c->V + (i - 1) * BR, c->B, c->Rl, c->s, c->y + (i - 1) * B, -1.0, c->t, s);
        }
    }
    return check_launch("coarse substitution mat-vecs");
}

// ---------------------------------------------------------------------------
// Setup.
__global__ void k_set_identity(double *__restrict__ X, int64_t N) {
    const int64_t nn = N * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x)
        X[e] = (e % N == e / N) ? 1.0 : 0.0;
}

// LU[i + jN] <- X[i + jN] on the strict lower (LOWER) or upper-with-diagonal part.
template <bool LOWER>
__global__ void k_pack_triangle(double *__restrict__ LU, const double *__restrict__ X, int64_t N) {
    const int64_t nn = N * N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % N, j = e / N;
        if (LOWER ? (i > j) : (i <= j)) LU[e] = X[e];
    }
}

// out = in^T for B x B blocks: the column-major factors become row-major.
__global__ void __launch_bounds__(256) k_transpose(const double *__restrict__ in, double *__restrict__ out, int B) {
    __shared__ double tile[32][33];
    const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32, tx = threadIdx.x, ty = threadIdx.y;
    for (int k = 0; k < 32; k += 8) {
        const int r = r0 + tx, c = c0 + ty + k;
        if (r < B && c < B) tile[ty + k][tx] = in[r + (int64_t)c * B];
    }
    __syncthreads();
    for (int k = 0; k < 32; k += 8) {
        const int r = r0 + ty + k, c = c0 + tx;
        if (r < B && c < B) out[(int64_t)r * B + c] = tile[tx][ty + k];
    }
}

// Pt_i, Rt_i of one pair of slabs from the assembled blocks (column-major
// B x B): Aplus = A_{i+1,i}, Aminus = A_{i,i+1}.  Both are block diagonal
// over the cells, K_c = Aplus[cell c, cell c] and K'_c = Aminus[cell c, cell c]:
//     P_c = K_c T_c^T (G^-1 x I),  R_c = (G^-1 x I) T_c K'_c.
// One thread per (cell, face number, unknown); Pt is stored
// [cell][unknown][face number], Rt [cell][face number][unknown].
__global__ void k_lr_split(const double *__restrict__ Aplus, const double *__restrict__ Aminus, int B, FaceMap f,
                           int ncs, double *__restrict__ Pt, double *__restrict__ Rt) {
    const int64_t total = (int64_t)ncs * f.rc * f.nc;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(e % f.nc);
        const int64_t ca = e / f.nc;
        const int a = (int)(ca % f.rc), c = (int)(ca / f.rc);
        const int kind = a / f.nxy, q = a - kind * f.nxy;
        const int64_t o = (int64_t)c * f.nc;
        double kt[2] = {0.0, 0.0}, tk[2] = {0.0, 0.0};
        for (int z = 0; z < f.n1; ++z) {
            const int64_t col = o + q + (int64_t)z * f.nxy;  // unknown on node line q of cell c
            const double kp = Aplus[(o + l) + col * B];      // K_c[l][q + z nxy]
            const double km = Aminus[col + (o + l) * B];     // K'_c[q + z nxy][l]
            for (int w = 0; w < 2; ++w) {
                kt[w] = fma(kp, f.f[w][z], kt[w]);
                tk[w] = fma(f.f[w][z], km, tk[w]);
            }
        }
        Pt[(o + l) * f.rc + a] = kt[0] * f.ginv[0][kind] + kt[1] * f.ginv[1][kind];
        Rt[e] = f.ginv[kind][0] * tk[0] + f.ginv[kind][1] * tk[1];
    }
}

// W_i = T inv(U_ii) and V_i = inv(L_ii) T^T from the packed, row-major
// inverted factors D (B x B).  W: Rl x B row-major, row (c, a); V: B x Rl
// row-major.
__global__ void k_lr_w(const double *__restrict__ D, int B, FaceMap f, int Rl, double *__restrict__ W) {
    const int64_t total = (int64_t)Rl * B;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int col = (int)(e % B), row = (int)(e / B);
        const int c = row / f.rc, a = row - c * f.rc;
        const int kind = a / f.nxy, q = a - kind * f.nxy;
        double acc = 0.0;
        for (int z = 0; z < f.n1; ++z) {
            const int r = c * f.nc + q + z * f.nxy;  // row of inv(U): zero left of the diagonal
            if (col >= r) acc = fma(f.f[kind][z], D[(int64_t)r * B + col], acc);
        }
        W[e] = acc;
    }
}

__global__ void k_lr_v(const double *__restrict__ D, int B, FaceMap f, int Rl, double *__restrict__ V) {
    const int64_t total = (int64_t)B * Rl;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int ca = (int)(e % Rl), r = (int)(e / Rl);
        const int c = ca / f.rc, a = ca - c * f.rc;
        const int kind = a / f.nxy, q = a - kind * f.nxy;
        double acc = 0.0;
        for (int z = 0; z < f.n1; ++z) {
            const int j = c * f.nc + q + z * f.nxy;  // column of inv(L): unit diagonal, zero right of it
            const double lij = j < r ? D[(int64_t)r * B + j] : (j == r ? 1.0 : 0.0);
            acc = fma(lij, f.f[kind][z], acc);
        }
        V[e] = acc;
    }
}

static fts_status rb_check(rocblas_status st, const char *what) {
    // (the size statuses answer calls made during a workspace-size query)
    if (st != rocblas_status_success && st != rocblas_status_size_increased && st != rocblas_status_size_unchanged)
        return fail(FTS_E_HIP, std::string("rocBLAS failure in ") + what + ": " + rocblas_status_to_string(st));
    return FTS_OK;
}

// Blocked LU without pivoting of the n x n matrix A (column-major, lda = n), in place.
static fts_status lu_inplace(rocblas_handle h, double *A, int n, hipStream_t stream, bool query) {
    const double one = 1.0, mone = -1.0;
    for (int k0 = 0; k0 < n; k0 += kNB) {
        const int kb = std::min(kNB, n - k0), n2 = n - k0 - kb;
        double *A11 = A + k0 + (int64_t)k0 * n;
        if (!query) {
            k_lu_diag<<<1, 1024, 0, stream>>>(A11, n, kb);
            COARSE_TRY(check_launch("k_lu_diag"));
        }
        if (n2 == 0) break;
        double *A12 = A + k0 + (int64_t)(k0 + kb) * n;
        double *A21 = A + (k0 + kb) + (int64_t)k0 * n;
        double *A22 = A + (k0 + kb) + (int64_t)(k0 + kb) * n;
        COARSE_TRY(rb_check(rocblas_dtrsm(h, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                                       rocblas_diagonal_unit, kb, n2, &one, A11, n, A12, n),
                         "dtrsm (L panel)"));
        COARSE_TRY(rb_check(rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                       rocblas_diagonal_non_unit, n2, kb, &one, A11, n, A21, n),
                         "dtrsm (U panel)"));
        COARSE_TRY(rb_check(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n2, n2, kb, &mone, A21,
                                       n, A12, n, &one, A22, n),
                         "dgemm (trailing update)"));
    }
    return FTS_OK;
}

// Replace the factors L, U stored in A (n x n) by inv(L) (strict lower part)
// and inv(U) (upper part); X is an n x n temporary.
static fts_status invert_factors(rocblas_handle h, double *A, int n, double *X, hipStream_t stream, bool query) {
    const double one = 1.0;
    const int64_t nn = (int64_t)n * n;
    const int grid = (int)std::min<int64_t>((nn + 255) / 256, 1 << 20);
    for (int pass = 0; pass < 2; ++pass) {
        const bool lower = pass == 0;
        if (!query) {
            k_set_identity<<<grid, 256, 0, stream>>>(X, n);
            COARSE_TRY(check_launch("k_set_identity"));
        }
        COARSE_TRY(rb_check(rocblas_dtrsm(h, rocblas_side_left, lower ? rocblas_fill_lower : rocblas_fill_upper,
                                       rocblas_operation_none,
                                       lower ? rocblas_diagonal_unit : rocblas_diagonal_non_unit, n, n, &one, A, n,
                                       X, n),
                         "dtrsm (triangular inverse)"));
        if (query) continue;
        if (lower) k_pack_triangle<true><<<grid, 256, 0, stream>>>(A, X, n);
        else k_pack_triangle<false><<<grid, 256, 0, stream>>>(A, X, n);
        COARSE_TRY(check_launch("k_pack_triangle"));
    }
    return FTS_OK;
}

// Block elimination over the slabs (see the top of this file).  query: only
// the BLAS calls, inside a rocBLAS workspace-size query (nothing computed).
static fts_status factor_slabs(rocblas_handle h, CoarseLU *c, double *X, hipStream_t stream, bool query) {
    const int B = c->B;
    const int64_t BB = (int64_t)B * B;
    const double one = 1.0, mone = -1.0;
    COARSE_TRY(rb_check(rocblas_set_stream(h, stream), "rocblas_set_stream"));
    for (int i = 0; i < c->nb; ++i) {
        double *Di = c->D + i * BB;
        if (i > 0)  // D_i <- A_ii - Lo_{i-1} Up_{i-1}
            COARSE_TRY(rb_check(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, B, B, B, &mone,
                                           c->Lo + (i - 1) * BB, B, c->Up + (i - 1) * BB, B, &one, Di, B),
                             "dgemm (slab update)"));
        COARSE_TRY(lu_inplace(h, Di, B, stream, query));
        if (i + 1 < c->nb) {
            COARSE_TRY(rb_check(rocblas_dtrsm(h, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                                           rocblas_diagonal_unit, B, B, &one, Di, B, c->Up + i * BB, B),
                             "dtrsm (Up)"));
            COARSE_TRY(rb_check(rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                           rocblas_diagonal_non_unit, B, B, &one, Di, B, c->Lo + i * BB, B),
                             "dtrsm (Lo)"));
        }
        COARSE_TRY(invert_factors(h, Di, B, X, stream, query));
    }
    if (query) return FTS_OK;
    // The substitution kernels read rows: store the diagonal blocks row-major
    // (Lo_i and Up_i are not read by the solve).
    const dim3 tgrid((B + 31) / 32, (B + 31) / 32), tblock(32, 8);
    for (int blk = 0; blk < c->nb; ++blk) {
        double *Mb = c->D + blk * BB;
        k_transpose<<<tgrid, tblock, 0, stream>>>(Mb, X, B);
        COARSE_TRY(check_launch("k_transpose"));
        FTS_HIP_CHECK(hipMemcpyAsync(Mb, X, BB * sizeof(double), hipMemcpyDeviceToDevice, stream));
    }
    return FTS_OK;
}

void coarse_destroy(CoarseLU *c) {
    if (!c) return;
    for (double *p : {c->D, c->Lo, c->Up, c->W, c->V, c->Pt, c->Rt, c->y, c->t, c->s})
        if (p) dev_free(p);
    delete c;
}

fts_status coarse_create(const fts_level *l0, hipStream_t stream, CoarseLU **out) {
    return coarse_create_with(l0, [&](const SlabBlocks &blk) { return launch_assemble_slabs(l0, blk, stream); },
                              stream, out);
}

fts_status coarse_create_with(const fts_level *l0, const std::function<fts_status(const SlabBlocks &)> &fill,
                              hipStream_t stream, CoarseLU **out) {
    *out = nullptr;
    const int d = l0->dim;
    int64_t nc = 1;
    for (int a = 0; a < d; ++a) nc *= l0->n1;
    const int64_t B = nc * l0->m[0] * (d == 3 ? l0->m[1] : 1);
    const int nb = l0->m[d - 1];
    if (B > INT_MAX || (int64_t)B * nb != l0->ndofs)
        return fail(FTS_E_SIZE, "coarse slab too large for the BLAS interface");
    CoarseLU *c = new CoarseLU;
    c->N = l0->ndofs;
    c->B = (int)B;
    c->nb = nb;
    c->nc = (int)nc;
    // the face functionals of the top face along the slab axis
    FaceMap fm{};
    fm.n1 = l0->n1;
    fm.nc = (int)nc;
    fm.nxy = (int)(nc / l0->n1);
    fm.rc = 2 * fm.nxy;
    double g[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int z = 0; z < l0->n1; ++z) {
        fm.f[0][z] = l0->ref.v1[z];
        fm.f[1][z] = l0->ref.d1[z];
    }
    for (int u = 0; u < 2; ++u)
        for (int w = 0; w < 2; ++w)
            for (int z = 0; z < l0->n1; ++z) g[u][w] += fm.f[u][z] * fm.f[w][z];
    const double det = g[0][0] * g[1][1] - g[0][1] * g[1][0];
    fm.ginv[0][0] = g[1][1] / det;
    fm.ginv[1][1] = g[0][0] / det;
    fm.ginv[0][1] = -g[0][1] / det;
    fm.ginv[1][0] = -g[1][0] / det;
    c->ncs = (int)(B / nc);
    c->rc = fm.rc;
    c->Rl = c->ncs * c->rc;
    const int64_t nblk = (int64_t)B * B, nlr = (int64_t)B * c->Rl, npr = (int64_t)c->ncs * c->rc * nc;
    const size_t blk = (size_t)nblk * sizeof(double);
    double *X = nullptr;
    fts_status st = FTS_OK;
    if (dev_malloc(&c->D, nb * blk) != hipSuccess ||
        (nb > 1 && (dev_malloc(&c->Lo, (nb - 1) * blk) != hipSuccess ||
                    dev_malloc(&c->Up, (nb - 1) * blk) != hipSuccess ||
                    dev_malloc(&c->W, (nb - 1) * nlr * sizeof(double)) != hipSuccess ||
                    dev_malloc(&c->V, (nb - 1) * nlr * sizeof(double)) != hipSuccess ||
                    dev_malloc(&c->Pt, (nb - 1) * npr * sizeof(double)) != hipSuccess ||
                    dev_malloc(&c->Rt, (nb - 1) * npr * sizeof(double)) != hipSuccess)) ||
        dev_malloc(&c->y, c->N * sizeof(double)) != hipSuccess || dev_malloc(&c->t, B * sizeof(double)) != hipSuccess ||
        dev_malloc(&c->s, c->Rl * sizeof(double)) != hipSuccess || dev_malloc(&X, blk) != hipSuccess)
        st = fail(FTS_E_HIP, "device allocation of the coarse factors failed");
    if (st == FTS_OK) st = launch_fill(c->D, nb * nblk, 0.0, stream);
    if (st == FTS_OK && nb > 1) st = launch_fill(c->Lo, (nb - 1) * nblk, 0.0, stream);
    if (st == FTS_OK && nb > 1) st = launch_fill(c->Up, (nb - 1) * nblk, 0.0, stream);
    if (st == FTS_OK) st = fill(SlabBlocks{c->D, c->Lo, c->Up, B});
    // P_i, R_i from the assembled off-diagonal blocks, before the
    // elimination overwrites them
    const unsigned gsplit = (unsigned)std::min<int64_t>((npr + 255) / 256, 1 << 16);
    for (int i = 0; st == FTS_OK && i + 1 < nb; ++i) {
        k_lr_split<<<gsplit, 256, 0, stream>>>(c->Lo + i * nblk, c->Up + i * nblk, (int)B, fm, c->ncs,
                                               c->Pt + i * npr, c->Rt + i * npr);
        st = check_launch("k_lr_split");
    }
    rocblas_handle h = nullptr;
    void *bws = nullptr;
    if (st == FTS_OK && rocblas_create_handle(&h) != rocblas_status_success)
        st = fail(FTS_E_HIP, "rocblas_create_handle failed");
    if (st == FTS_OK) st = rb_check(rocblas_set_stream(h, stream), "rocblas_set_stream");
    // the BLAS workspace of the factorisation comes from the registered
    // allocator: size it with a query pass, then hand it to rocBLAS
    if (st == FTS_OK) st = rb_check(rocblas_start_device_memory_size_query(h), "workspace query");
    if (st == FTS_OK) {
        fts_status sq = factor_slabs(h, c, X, stream, true);
        size_t wsz = 0;
        const fts_status se = rb_check(rocblas_stop_device_memory_size_query(h, &wsz), "workspace query");
        st = sq != FTS_OK ? sq : se;
        if (st == FTS_OK && wsz > 0 && dev_malloc(&bws, wsz) != hipSuccess)
            st = fail(FTS_E_HIP, "device allocation of the BLAS workspace failed");
        if (st == FTS_OK && wsz > 0) st = rb_check(rocblas_set_workspace(h, bws, wsz), "rocblas_set_workspace");
    }
    if (st == FTS_OK) st = factor_slabs(h, c, X, stream, false);
    // W_i, V_i from the inverted diagonal factors; Lo_i, Up_i are then done
    const unsigned glr = (unsigned)std::min<int64_t>((nlr + 255) / 256, 1 << 20);
    for (int i = 0; st == FTS_OK && i + 1 < nb; ++i) {
        k_lr_w<<<glr, 256, 0, stream>>>(c->D + i * nblk, (int)B, fm, c->Rl, c->W + i * nlr);
        k_lr_v<<<glr, 256, 0, stream>>>(c->D + i * nblk, (int)B, fm, c->Rl, c->V + i * nlr);
        st = check_launch("k_lr_w / k_lr_v");
    }
    if (hipStreamSynchronize(stream) != hipSuccess && st == FTS_OK) st = fail(FTS_E_HIP, "coarse factorisation failed");
    if (h) rocblas_destroy_handle(h);
    dev_free(bws);
    if (X) dev_free(X);
    if (c->Lo) dev_free(c->Lo);
    if (c->Up) dev_free(c->Up);
    c->Lo = c->Up = nullptr;
    if (st != FTS_OK) {
        coarse_destroy(c);
        return st;
    }
    *out = c;
    return FTS_OK;
}

}  // namespace fts
