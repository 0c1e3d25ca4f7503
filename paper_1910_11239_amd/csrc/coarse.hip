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
// Between two slabs a cell couples only to the cell at the same position, so
// Lo_i is zero where the column's cell precedes the row's cell and Up_i is
// zero where it follows it.
//
// Setup (once): block elimination over the slabs with library BLAS-3 (GEMM,
// TRSM) and a one-workgroup kernel for the small diagonal panels; then the
// diagonal factors are replaced by their inverses (strict lower part
// inv(L_ii) with unit diagonal implied, upper part inv(U_ii)), so every step
// of the substitution is a matrix-vector product.
//
// Solve (every V-cycle): 2 (2 nb - 1) mat-vec launches
//     forward   y_0 = inv(L_00) b_0,          y_i = inv(L_ii) (b_i - Lo_{i-1} y_{i-1})
//     backward  x_last = inv(U) y_last,       x_i = inv(U_ii) (y_i - Up_i x_{i+1})
// each reading the live part of its block once: 8 B^2 (2 nb - 1) bytes per
// solve instead of the 8 N^2 of dense triangular factors (N = nb B).
#include <rocblas/rocblas.h>

#include <climits>

#include "device_common.h"

namespace fts {

struct CoarseLU {
    int64_t N = 0;
    int B = 0, nb = 0, nc = 0;  // slab size, number of slabs, unknowns per cell
    double *D = nullptr;         // nb blocks: packed inv(L_ii), inv(U_ii)
    double *Lo = nullptr;        // nb - 1 blocks Lo_i
    double *Up = nullptr;        // nb - 1 blocks Up_i
    double *y = nullptr;         // N: result of the forward substitution
    double *t = nullptr;         // B: right-hand side of the current diagonal step
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
// Block mat-vec out = base + sgn * (M v) over one B x B block M stored
// row-major, restricted to the block's nonzero part.  Row r of each part
// occupies one contiguous column range:
//     kLowerInv  strict lower part of a packed diagonal block: [0, r)
//                (the unit diagonal comes in through base = v)
//     kUpperInv  upper part of a packed diagonal block:        [r, B)
//     kBelow     Lo_i, zero left of the row's cell:             [cell(r) nc, B)
//     kAbove     Up_i, zero right of the row's cell:            [0, (cell(r) + 1) nc)
// The rows are cut into groups of kRows; a workgroup owns group g and group
// G-1-g, a short and a long range, so every workgroup streams about the same
// number of bytes.  Its waves take interleaved passes of 64 lanes x two
// columns over each range (16-byte non-temporal loads, one per row and
// lane, the loads of kUnroll passes issued before their FMAs), keep one
// partial per row and lane, and reduce across lanes with shuffles and across
// waves in LDS in a fixed order: no atomics, and the result does not depend
// on timing.
constexpr int kRows = 4, kMvWaves = 8, kUnroll = 2;
typedef double dvec2 __attribute__((ext_vector_type(2)));

enum BlockPart { kLowerInv = 0, kUpperInv = 1, kBelow = 2, kAbove = 3 };

// Column range [lo, hi) covering the nonzero parts of rows [r0, r1].
template <int PART>
__device__ __forceinline__ void group_range(int r0, int r1, int B, int nc, int &lo, int &hi) {
    if (PART == kLowerInv) lo = 0, hi = r1;
    else if (PART == kUpperInv) lo = r0, hi = B;
    else if (PART == kBelow) lo = (r0 / nc) * nc, hi = B;
    else lo = 0, hi = (r1 / nc + 1) * nc;
}

// Entry (row, col) of the union range that lies outside the row's own part.
// Only the packed diagonal blocks need this: the off-diagonal blocks store
// their zeros.
template <int PART>
__device__ __forceinline__ bool outside(int row, int col) {
    if (PART == kLowerInv) return col >= row;
    if (PART == kUpperInv) return col < row;
    return false;
}

// acc[q] += sum over this lane's columns of row r0 + q (rows past r1 are
// loaded from row r1 and their sums dropped by the caller).  Passes
// p = wave, wave + kMvWaves, ... < np; pass p covers PC columns from lo + p PC.
template <int PART, bool PAIR>
__device__ __forceinline__ void stream_group(const double *__restrict__ M, int B, const double *__restrict__ v,
                                             int r0, int r1, int lo, int hi, int np, int wave, int lane,
                                             double *acc) {
    constexpr int CPL = PAIR ? 2 : 1, PC = 64 * CPL;
    const double *rowp[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) rowp[q] = M + (int64_t)min(r0 + q, r1) * B;
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
            dvec2 x[kUnroll], m[kUnroll][kRows];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                x[u] = *(const dvec2 *)(v + jj[u]);
#pragma unroll
                for (int q = 0; q < kRows; ++q) m[u][q] = __builtin_nontemporal_load((const dvec2 *)(rowp[q] + jj[u]));
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int q = 0; q < kRows; ++q) {
                    const double mx = (ok[u] && !outside<PART>(r0 + q, jj[u])) ? m[u][q].x : 0.0;
                    const double my = (ok[u] && !outside<PART>(r0 + q, jj[u] + 1)) ? m[u][q].y : 0.0;
                    acc[q] = fma(my, x[u].y, fma(mx, x[u].x, acc[q]));
                }
        } else {
            double x[kUnroll], m[kUnroll][kRows];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                x[u] = v[jj[u]];
#pragma unroll
                for (int q = 0; q < kRows; ++q) m[u][q] = rowp[q][jj[u]];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int q = 0; q < kRows; ++q)
                    acc[q] = fma((ok[u] && !outside<PART>(r0 + q, jj[u])) ? m[u][q] : 0.0, x[u], acc[q]);
        }
    }
    for (; p < np; p += kMvWaves) {
        const int j = lo + p * PC + CPL * lane;
        const bool ok = j < hi;
        const int jj = ok ? j : lo;
        if constexpr (PAIR) {
            const dvec2 x = *(const dvec2 *)(v + jj);
            dvec2 m[kRows];
#pragma unroll
            for (int q = 0; q < kRows; ++q) m[q] = __builtin_nontemporal_load((const dvec2 *)(rowp[q] + jj));
#pragma unroll
            for (int q = 0; q < kRows; ++q) {
                const double mx = (ok && !outside<PART>(r0 + q, jj)) ? m[q].x : 0.0;
                const double my = (ok && !outside<PART>(r0 + q, jj + 1)) ? m[q].y : 0.0;
                acc[q] = fma(my, x.y, fma(mx, x.x, acc[q]));
            }
        } else {
            const double x = v[jj];
            double m[kRows];
#pragma unroll
            for (int q = 0; q < kRows; ++q) m[q] = rowp[q][jj];
#pragma unroll
            for (int q = 0; q < kRows; ++q) acc[q] = fma((ok && !outside<PART>(r0 + q, jj)) ? m[q] : 0.0, x, acc[q]);
        }
    }
}

template <int PART, bool PAIR>
__global__ void __launch_bounds__(64 * kMvWaves) k_slab_mv(const double *__restrict__ M, int B, int nc, int G,
                                                           const double *__restrict__ v, const double *base,
                                                           double sgn, double *__restrict__ out) {
    constexpr int PC = PAIR ? 128 : 64;  // columns per wave pass
    __shared__ double red[kMvWaves][2 * kRows];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ga = blockIdx.x, gb = G - 1 - blockIdx.x;  // gb == ga: a single group
    int r0[2], r1[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        r0[s] = (s == 0 ? ga : gb) * kRows;
        r1[s] = min(r0[s] + kRows, B) - 1;
        int lo, hi;
        group_range<PART>(r0[s], r1[s], B, nc, lo, hi);
        if (PAIR) lo &= ~1, hi = min(B, (hi + 1) & ~1);
        const int np = (s == 1 && gb == ga) || hi <= lo ? 0 : (hi - lo + PC - 1) / PC;
        double acc[kRows];
#pragma unroll
        for (int q = 0; q < kRows; ++q) acc[q] = 0.0;
        stream_group<PART, PAIR>(M, B, v, r0[s], r1[s], lo, hi, np, wave, lane, acc);
#pragma unroll
        for (int q = 0; q < kRows; ++q) {
            double t = acc[q];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
            if (lane == 0) red[wave][s * kRows + q] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kRows) {
        const int s = threadIdx.x / kRows, q = threadIdx.x % kRows;
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
static void slab_mv(const CoarseLU *c, const double *M, const double *v, const double *base, double sgn,
                    double *out, hipStream_t s) {
    const int G = (c->B + kRows - 1) / kRows;
    const dim3 grid((G + 1) / 2);
    if (c->B % 2 == 0) k_slab_mv<PART, true><<<grid, 64 * kMvWaves, 0, s>>>(M, c->B, c->nc, G, v, base, sgn, out);
    else k_slab_mv<PART, false><<<grid, 64 * kMvWaves, 0, s>>>(M, c->B, c->nc, G, v, base, sgn, out);
}

fts_status coarse_solve(CoarseLU *c, const double *b, double *x, hipStream_t s) {
    const int64_t B = c->B, BB = B * B;
    for (int i = 0; i < c->nb; ++i) {
        const double *rhs = i == 0 ? b : c->t;
        slab_mv<kLowerInv>(c, c->D + i * BB, rhs, rhs, 1.0, c->y + i * B, s);
        if (i + 1 < c->nb) slab_mv<kBelow>(c, c->Lo + i * BB, c->y + i * B, b + (i + 1) * B, -1.0, c->t, s);
    }
    for (int i = c->nb - 1; i >= 0; --i) {
        const double *rhs = i == c->nb - 1 ? c->y + i * B : c->t;
        slab_mv<kUpperInv>(c, c->D + i * BB, rhs, nullptr, 1.0, x + i * B, s);
        if (i > 0) slab_mv<kAbove>(c, c->Up + (i - 1) * BB, x + i * B, c->y + (i - 1) * B, -1.0, c->t, s);
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
    // The substitution kernels read rows: store every block row-major.
    const dim3 tgrid((B + 31) / 32, (B + 31) / 32), tblock(32, 8);
    for (int blk = 0; blk < 3 * c->nb - 2; ++blk) {
        double *Mb = blk < c->nb ? c->D + blk * BB
                                 : (blk < 2 * c->nb - 1 ? c->Lo + (blk - c->nb) * BB : c->Up + (blk - 2 * c->nb + 1) * BB);
        k_transpose<<<tgrid, tblock, 0, stream>>>(Mb, X, B);
        COARSE_TRY(check_launch("k_transpose"));
        FTS_HIP_CHECK(hipMemcpyAsync(Mb, X, BB * sizeof(double), hipMemcpyDeviceToDevice, stream));
    }
    return FTS_OK;
}

void coarse_destroy(CoarseLU *c) {
    if (!c) return;
    for (void *p : {(void *)c->D, (void *)c->Lo, (void *)c->Up, (void *)c->y, (void *)c->t})
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
    const size_t blk = (size_t)B * B * sizeof(double);
    double *X = nullptr;
    fts_status st = FTS_OK;
    if (dev_malloc(&c->D, nb * blk) != hipSuccess ||
        (nb > 1 && (dev_malloc(&c->Lo, (nb - 1) * blk) != hipSuccess ||
                    dev_malloc(&c->Up, (nb - 1) * blk) != hipSuccess)) ||
        dev_malloc(&c->y, c->N * sizeof(double)) != hipSuccess || dev_malloc(&c->t, B * sizeof(double)) != hipSuccess ||
        dev_malloc(&X, blk) != hipSuccess)
        st = fail(FTS_E_HIP, "device allocation of the coarse factors failed");
    const int64_t nblk = (int64_t)B * B;
    if (st == FTS_OK) st = launch_fill(c->D, nb * nblk, 0.0, stream);
    if (st == FTS_OK && nb > 1) st = launch_fill(c->Lo, (nb - 1) * nblk, 0.0, stream);
    if (st == FTS_OK && nb > 1) st = launch_fill(c->Up, (nb - 1) * nblk, 0.0, stream);
    if (st == FTS_OK) st = fill(SlabBlocks{c->D, c->Lo, c->Up, B});
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
    if (hipStreamSynchronize(stream) != hipSuccess && st == FTS_OK) st = fail(FTS_E_HIP, "coarse factorisation failed");
    if (h) rocblas_destroy_handle(h);
    dev_free(bws);
    if (X) dev_free(X);
    if (st != FTS_OK) {
        coarse_destroy(c);
        return st;
    }
    *out = c;
    return FTS_OK;
}

}  // namespace fts
