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
// tile, thread = row, columns streamed with coalesced column-major reads and
// independent partial sums; tile results go to P[column block][row] and are
// summed in a fixed order by k_tri_reduce (deterministic).
constexpr int kTR = 256, kTC = 1024, kUnroll = 8;

template <bool LOWER>
__global__ void __launch_bounds__(kTR) k_tri_partial(const double *__restrict__ F, int64_t N,
                                                     const double *__restrict__ v, double *__restrict__ P) {
    __shared__ double vs[kTC];
    const int64_t r0 = (int64_t)blockIdx.y * kTR, c0 = (int64_t)blockIdx.x * kTC;
    // tiles outside the triangle do nothing; k_tri_reduce uses the same test
    if (LOWER ? (c0 >= r0 + kTR) : (c0 + kTC <= r0)) return;
    for (int j = threadIdx.x; j < kTC; j += kTR) vs[j] = (c0 + j < N) ? v[c0 + j] : 0.0;
    __syncthreads();
    const int64_t i = r0 + threadIdx.x;
    if (i >= N) return;
    // column range of this row inside the tile
    int jlo = 0, jhi = (int)std::min<int64_t>(kTC, N - c0);
    if (LOWER) jhi = (int)std::min<int64_t>(jhi, std::max<int64_t>(0, i - c0));      // j < i
    else jlo = (int)std::min<int64_t>(kTC, std::max<int64_t>(0, i - c0));           // j >= i
    const double *col = F + i + c0 * N;
    double acc[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc[u] = 0.0;
    int j = jlo;
    for (; j + kUnroll <= jhi; j += kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc[u] = fma(col[(int64_t)(j + u) * N], vs[j + u], acc[u]);
    }
    for (; j < jhi; ++j) acc[0] = fma(col[(int64_t)j * N], vs[j], acc[0]);
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) s += acc[u];
    P[(int64_t)blockIdx.x * N + i] = s;
}

template <bool LOWER>
__global__ void __launch_bounds__(256) k_tri_reduce(const double *__restrict__ P, int64_t N, int ncb,
                                                    const double *__restrict__ v, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int64_t rb0 = (i / kTR) * kTR;  // first row of this row tile
    double s = LOWER ? v[i] : 0.0;
    for (int cb = 0; cb < ncb; ++cb) {
        const int64_t c0 = (int64_t)cb * kTC;
        const bool live = LOWER ? (c0 < rb0 + kTR) : (c0 + kTC > rb0);
        if (live) s += P[(int64_t)cb * N + i];
    }
    out[i] = s;
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
    k_tri_partial<true><<<grid, kTR, 0, stream>>>(F, N, b, P);
    k_tri_reduce<true><<<rgrid, 256, 0, stream>>>(P, N, ncb, b, y);
    k_tri_partial<false><<<grid, kTR, 0, stream>>>(F, N, y, P);
    k_tri_reduce<false><<<rgrid, 256, 0, stream>>>(P, N, ncb, y, x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "coarse triangular mat-vecs");
    return FTS_OK;
}

}  // namespace fts
