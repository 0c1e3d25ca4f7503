// Dense LU of the coarsest-level matrix and the two triangular solves of the
// coarse solve (Alg. gmg, level 0).  The factor is column-major with leading
// dimension N, overwritten in place: unit lower L below the diagonal, U on
// and above it.  No pivoting: A_0 is symmetric positive definite, for which
// Gaussian elimination without pivoting is stable.
//
// Factorisation (setup, once): blocks of NB columns; the diagonal block is
// factored by one workgroup, the two panels by triangular solves and the
// trailing matrix by a GEMM (library BLAS-3, setup only).  Afterwards the
// inverses of all diagonal blocks of L and U are formed, so that each step
// of the triangular solves is a matrix-vector product.
//
// Triangular solve (every V-cycle): one launch per block step.  Step s of
// the forward solve finalises block s (head workgroup: subtract column block
// s-1, then multiply by inv(L_ss)) while the other workgroups subtract column
// block s-1 from all rows below block s.  The backward solve mirrors it.
// Every launch streams its column panel once with coalesced column-major
// reads, so a full solve reads the factor once (8 N^2 bytes).
#include <rocblas/rocblas.h>

#include "fts_internal.h"

namespace fts {

constexpr int kNB = 256;         // block size of factor and solves
constexpr int kRowsPerWG = 64;   // rows per non-head workgroup in a solve step
constexpr int kColGroups = 4;    // column groups per workgroup (256 threads)

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

// Triangular matrix-vector products with the inverted factors stored in the
// LU buffer: strictly below the diagonal inv(L) (unit diagonal implied), on
// and above it inv(U).  Tiles of TR rows x TC columns; a workgroup owns one
// tile, each thread two consecutive rows (16-byte loads), columns streamed
// with non-temporal coalesced column-major reads and independent partial
// sums; tile results go to P[column block][row] and are summed in a fixed
// order by k_tri_reduce (deterministic).  A tile is live when it holds an
// entry of the triangle; both kernels use the same column-block range.
constexpr int kTR = 512, kTC = 1024, kUnroll = 8;
typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int live_lo(bool lower, int64_t rb0) { return lower ? 0 : (int)(rb0 / kTC); }
__device__ __forceinline__ int live_hi(bool lower, int64_t rb0, int ncb) {
    return lower ? (int)std::min<int64_t>(ncb, (rb0 + kTR + kTC - 1) / kTC) : ncb;
}

template <bool LOWER>
__global__ void __launch_bounds__(256) k_tri_partial(const double *__restrict__ F, int64_t N,
                                                     const double *__restrict__ v, double *__restrict__ P) {
    __shared__ double vs[kTC];
    const int64_t r0 = (int64_t)blockIdx.y * kTR;
    const int cb = blockIdx.x;
    if (cb < live_lo(LOWER, r0) || cb >= live_hi(LOWER, r0, gridDim.x)) return;
    const int64_t c0 = (int64_t)cb * kTC;
    for (int j = threadIdx.x; j < kTC; j += 256) vs[j] = (c0 + j < N) ? v[c0 + j] : 0.0;
    __syncthreads();
    const int64_t i = r0 + 2 * threadIdx.x;  // rows i, i+1
    if (i >= N) return;
    const bool pair = (i + 1 < N) && ((N & 1) == 0);  // 16-byte aligned row pairs
    // Column range (tile-relative) shared by rows i and i+1, and the one column
    // jd = i - c0 that belongs to only one of them (row i+1 for the strict
    // lower part, row i for the upper part including the diagonal).
    const int ncol = (int)std::min<int64_t>(kTC, N - c0);
    int jlo, jhi;
    if (LOWER) {
        jlo = 0;
        jhi = (int)std::min<int64_t>(ncol, std::max<int64_t>(0, i - c0));
    } else {
        jlo = (int)std::min<int64_t>(ncol, std::max<int64_t>(0, i + 1 - c0));
        jhi = ncol;
    }
    const int64_t jd = i - c0;
    const bool extra = jd >= 0 && jd < ncol;
    double a0[kUnroll], a1[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) a0[u] = a1[u] = 0.0;
    const double *col = F + i + c0 * N;
    if (pair) {
        int j = jlo;
        for (; j + kUnroll <= jhi; j += kUnroll) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const dvec2 m = __builtin_nontemporal_load((const dvec2 *)(col + (int64_t)(j + u) * N));
                a0[u] = fma(m.x, vs[j + u], a0[u]);
                a1[u] = fma(m.y, vs[j + u], a1[u]);
            }
        }
        for (; j < jhi; ++j) {
            const dvec2 m = *(const dvec2 *)(col + (int64_t)j * N);
            a0[0] = fma(m.x, vs[j], a0[0]);
            a1[0] = fma(m.y, vs[j], a1[0]);
        }
    } else {
        for (int j = jlo; j < jhi; ++j) {
            a0[0] = fma(col[(int64_t)j * N], vs[j], a0[0]);
            if (i + 1 < N) a1[0] = fma(col[(int64_t)j * N + 1], vs[j], a1[0]);
        }
    }
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        s0 += a0[u];
        s1 += a1[u];
    }
    if (extra) {
        if (LOWER) {
            if (i + 1 < N) s1 = fma(col[jd * N + 1], vs[jd], s1);
        } else {
            s0 = fma(col[jd * N], vs[jd], s0);
        }
    }
    P[(int64_t)cb * N + i] = s0;
    if (i + 1 < N) P[(int64_t)cb * N + i + 1] = s1;
}

template <bool LOWER>
__global__ void __launch_bounds__(256) k_tri_reduce(const double *__restrict__ P, int64_t N, int ncb,
                                                    const double *__restrict__ v, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int64_t rb0 = (i / kTR) * kTR;  // first row of this row tile
    const int lo = live_lo(LOWER, rb0), hi = live_hi(LOWER, rb0, ncb);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int cb = lo;
    for (; cb + 4 <= hi; cb += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += P[(int64_t)(cb + u) * N + i];
    }
    for (; cb < hi; ++cb) acc[0] += P[(int64_t)cb * N + i];
    out[i] = (LOWER ? v[i] : 0.0) + ((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

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

static fts_status rb_check(rocblas_status st, const char *what) {
    if (st != rocblas_status_success)
        return fail(FTS_E_HIP, std::string("rocBLAS failure in ") + what + ": " + rocblas_status_to_string(st));
    return FTS_OK;
}

// Factor A (N x N, column-major, lda = N) in place, then replace the factors
// by their inverses: strict lower part inv(L), upper part inv(U).  Needs one
// temporary N x N buffer (allocated and freed here, setup only).
fts_status coarse_factor(double *A, int64_t N, hipStream_t stream) {
    if (N > 2147483647LL) return fail(FTS_E_SIZE, "coarse matrix too large for the BLAS interface");
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return fail(FTS_E_HIP, "rocblas_create_handle failed");
    fts_status st = rb_check(rocblas_set_stream(h, stream), "rocblas_set_stream");
    const double one = 1.0, mone = -1.0;
    for (int64_t k0 = 0; k0 < N && st == FTS_OK; k0 += kNB) {
        const int kb = (int)std::min<int64_t>(kNB, N - k0);
        const int n2 = (int)(N - k0 - kb);
        double *A11 = A + k0 + k0 * N;
        k_lu_diag<<<1, 1024, 0, stream>>>(A11, N, kb);
        if (hipGetLastError() != hipSuccess) {
            st = fail(FTS_E_HIP, "k_lu_diag launch failed");
            break;
        }
        if (n2 == 0) break;
        double *A12 = A + k0 + (k0 + kb) * N;
        double *A21 = A + (k0 + kb) + k0 * N;
        double *A22 = A + (k0 + kb) + (k0 + kb) * N;
        st = rb_check(rocblas_dtrsm(h, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                                    rocblas_diagonal_unit, kb, n2, &one, A11, (int)N, A12, (int)N),
                      "dtrsm (L panel)");
        if (st != FTS_OK) break;
        st = rb_check(rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                    rocblas_diagonal_non_unit, n2, kb, &one, A11, (int)N, A21, (int)N),
                      "dtrsm (U panel)");
        if (st != FTS_OK) break;
        st = rb_check(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, n2, n2, kb, &mone, A21,
                                    (int)N, A12, (int)N, &one, A22, (int)N),
                      "dgemm (trailing update)");
    }
    double *X = nullptr;
    if (st == FTS_OK && hipMalloc(&X, (size_t)N * N * sizeof(double)) != hipSuccess)
        st = fail(FTS_E_HIP, "hipMalloc of the inversion buffer failed");
    const int grid = (int)std::min<int64_t>((N * N + 255) / 256, 1 << 20);
    for (int pass = 0; pass < 2 && st == FTS_OK; ++pass) {
        const bool lower = pass == 0;
        k_set_identity<<<grid, 256, 0, stream>>>(X, N);
        st = rb_check(rocblas_dtrsm(h, rocblas_side_left, lower ? rocblas_fill_lower : rocblas_fill_upper,
                                    rocblas_operation_none, lower ? rocblas_diagonal_unit : rocblas_diagonal_non_unit,
                                    (int)N, (int)N, &one, A, (int)N, X, (int)N),
                      "dtrsm (triangular inverse)");
        if (st != FTS_OK) break;
        if (lower) k_pack_triangle<true><<<grid, 256, 0, stream>>>(A, X, N);
        else k_pack_triangle<false><<<grid, 256, 0, stream>>>(A, X, N);
        if (hipGetLastError() != hipSuccess) st = fail(FTS_E_HIP, "packing of the inverse factors failed");
    }
    if (hipStreamSynchronize(stream) != hipSuccess && st == FTS_OK) st = fail(FTS_E_HIP, "coarse factorisation failed");
    if (X) hipFree(X);
    rocblas_destroy_handle(h);
    return st;
}

int coarse_ncb(int64_t N) { return (int)((N + kTC - 1) / kTC); }

// x = inv(U) (inv(L) b): two tiled triangular mat-vecs, each reading its
// triangle of the stored inverse factors once.  P: workspace of ncb * N
// doubles; y: workspace of N doubles.  x must not alias y or P.
fts_status coarse_solve(const double *F, int64_t N, const double *b, double *x, double *y, double *P,
                        hipStream_t stream) {
    const int ncb = coarse_ncb(N);
    const int nrb = (int)((N + kTR - 1) / kTR);
    const dim3 grid(ncb, nrb);
    const int rgrid = (int)((N + 255) / 256);
    k_tri_partial<true><<<grid, 256, 0, stream>>>(F, N, b, P);
    k_tri_reduce<true><<<rgrid, 256, 0, stream>>>(P, N, ncb, b, y);
    k_tri_partial<false><<<grid, 256, 0, stream>>>(F, N, y, P);
    k_tri_reduce<false><<<rgrid, 256, 0, stream>>>(P, N, ncb, y, x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "coarse triangular mat-vecs");
    return FTS_OK;
}

}  // namespace fts
