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

// Inverses of the diagonal blocks: thread c computes column c of inv(L_ss)
// (unit lower) and inv(U_ss) by substitution.  Stored column-major nb x nb.
__global__ void __launch_bounds__(kNB) k_tri_inv(const double *__restrict__ LU, int64_t N, double *__restrict__ Linv,
                                                  double *__restrict__ Uinv) {
    const int s = blockIdx.x, c = threadIdx.x;
    const int64_t k0 = (int64_t)s * kNB;
    const int kb = (int)std::min<int64_t>(kNB, N - k0);
    double *X = Linv + (size_t)s * kNB * kNB + (size_t)c * kNB;
    double *Y = Uinv + (size_t)s * kNB * kNB + (size_t)c * kNB;
    auto at = [&](int i, int j) { return LU[(k0 + i) + (k0 + j) * N]; };
    if (c >= kb) {
        for (int i = 0; i < kNB; ++i) X[i] = Y[i] = 0.0;
        return;
    }
    for (int i = 0; i < c; ++i) X[i] = 0.0;
    X[c] = 1.0;
    for (int i = c + 1; i < kb; ++i) {
        double sum = 0.0;
        for (int p = c; p < i; ++p) sum += at(i, p) * X[p];
        X[i] = -sum;
    }
    for (int i = kb; i < kNB; ++i) X[i] = 0.0;
    for (int i = c + 1; i < kNB; ++i) Y[i] = 0.0;
    Y[c] = 1.0 / at(c, c);
    for (int i = c - 1; i >= 0; --i) {
        double sum = 0.0;
        for (int p = i + 1; p <= c; ++p) sum += at(i, p) * Y[p];
        Y[i] = -sum / at(i, i);
    }
}

// Forward step s: see file comment.
__global__ void __launch_bounds__(256) k_trsv_fwd(const double *__restrict__ LU, int64_t N,
                                                   const double *__restrict__ Linv, double *__restrict__ y, int s) {
    __shared__ double yp[kNB];
    __shared__ double red[kColGroups][kRowsPerWG];
    __shared__ double ys[kNB];
    const int tid = threadIdx.x;
    const int64_t k0 = (int64_t)s * kNB;
    const int kb = (int)std::min<int64_t>(kNB, N - k0);
    const int64_t p0 = k0 - kNB;  // previous column block (valid when s > 0)
    if (s > 0) {
        yp[tid] = y[p0 + tid];  // previous block is always full
    }
    __syncthreads();
    if (blockIdx.x == 0) {
        double v = 0.0;
        if (tid < kb) {
            v = y[k0 + tid];
            if (s > 0) {
                const double *col = LU + (k0 + tid) + p0 * N;
                double acc = 0.0;
                for (int c = 0; c < kNB; ++c) acc = fma(col[c * N], yp[c], acc);
                v -= acc;
            }
        }
        ys[tid] = v;
        __syncthreads();
        if (tid < kb) {
            const double *Li = Linv + (size_t)s * kNB * kNB + tid;
            double out = 0.0;
            for (int c = 0; c < kb; ++c) out = fma(Li[(size_t)c * kNB], ys[c], out);
            y[k0 + tid] = out;
        }
        return;
    }
    // rows below block s, column block s-1
    const int r = tid % kRowsPerWG, g = tid / kRowsPerWG;
    const int64_t row = k0 + kNB + (int64_t)(blockIdx.x - 1) * kRowsPerWG + r;
    double acc = 0.0;
    if (row < N) {
        const double *col = LU + row + p0 * N;
        for (int c = g; c < kNB; c += kColGroups) acc = fma(col[c * N], yp[c], acc);
    }
    red[g][r] = acc;
    __syncthreads();
    if (g == 0 && row < N) y[row] -= red[0][r] + red[1][r] + red[2][r] + red[3][r];
}

// Backward step s (s from the last block down to 0).
__global__ void __launch_bounds__(256) k_trsv_bwd(const double *__restrict__ LU, int64_t N,
                                                   const double *__restrict__ Uinv, double *__restrict__ x, int s,
                                                   int nblk) {
    __shared__ double xn[kNB];
    __shared__ double red[kColGroups][kRowsPerWG];
    __shared__ double xs[kNB];
    const int tid = threadIdx.x;
    const int64_t k0 = (int64_t)s * kNB;
    const int kb = (int)std::min<int64_t>(kNB, N - k0);
    const int64_t n0 = k0 + kNB;  // next column block
    const int kn = s + 1 < nblk ? (int)std::min<int64_t>(kNB, N - n0) : 0;
    xn[tid] = tid < kn ? x[n0 + tid] : 0.0;
    __syncthreads();
    if (blockIdx.x == 0) {
        double v = 0.0;
        if (tid < kb) {
            v = x[k0 + tid];
            if (kn > 0) {
                const double *col = LU + (k0 + tid) + n0 * N;
                double acc = 0.0;
                for (int c = 0; c < kn; ++c) acc = fma(col[c * N], xn[c], acc);
                v -= acc;
            }
        }
        xs[tid] = v;
        __syncthreads();
        if (tid < kb) {
            const double *Ui = Uinv + (size_t)s * kNB * kNB + tid;
            double out = 0.0;
            for (int c = 0; c < kb; ++c) out = fma(Ui[(size_t)c * kNB], xs[c], out);
            x[k0 + tid] = out;
        }
        return;
    }
    const int r = tid % kRowsPerWG, g = tid / kRowsPerWG;
    const int64_t row = (int64_t)(blockIdx.x - 1) * kRowsPerWG + r;
    double acc = 0.0;
    if (row < k0) {
        const double *col = LU + row + n0 * N;
        for (int c = g; c < kn; c += kColGroups) acc = fma(col[c * N], xn[c], acc);
    }
    red[g][r] = acc;
    __syncthreads();
    if (g == 0 && row < k0) x[row] -= red[0][r] + red[1][r] + red[2][r] + red[3][r];
}

static fts_status rb_check(rocblas_status st, const char *what) {
    if (st != rocblas_status_success)
        return fail(FTS_E_HIP, std::string("rocBLAS failure in ") + what + ": " + rocblas_status_to_string(st));
    return FTS_OK;
}

// Factor A (N x N, column-major, lda = N) in place and form the diagonal-block
// inverses.  Linv, Uinv: nblk * NB * NB doubles each.
fts_status coarse_factor(double *A, int64_t N, double *Linv, double *Uinv, hipStream_t stream) {
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
    if (st == FTS_OK) {
        const int nblk = (int)((N + kNB - 1) / kNB);
        k_tri_inv<<<nblk, kNB, 0, stream>>>(A, N, Linv, Uinv);
        if (hipGetLastError() != hipSuccess) st = fail(FTS_E_HIP, "k_tri_inv launch failed");
    }
    if (st == FTS_OK && hipStreamSynchronize(stream) != hipSuccess) st = fail(FTS_E_HIP, "coarse factorisation failed");
    rocblas_destroy_handle(h);
    return st;
}

int coarse_nblk(int64_t N) { return (int)((N + kNB - 1) / kNB); }
int coarse_nb() { return kNB; }

// x = A^-1 b with the stored factors; x may alias b.
fts_status coarse_solve(const double *LU, int64_t N, const double *Linv, const double *Uinv, const double *b,
                        double *x, hipStream_t stream) {
    const int nblk = coarse_nblk(N);
    if (x != b) FTS_HIP_CHECK(hipMemcpyAsync(x, b, N * sizeof(double), hipMemcpyDeviceToDevice, stream));
    for (int s = 0; s < nblk; ++s) {
        const int64_t below = s == 0 ? 0 : std::max<int64_t>(0, N - (int64_t)(s + 1) * kNB);
        const int grid = 1 + (int)((below + kRowsPerWG - 1) / kRowsPerWG);
        k_trsv_fwd<<<grid, 256, 0, stream>>>(LU, N, Linv, x, s);
    }
    for (int s = nblk - 1; s >= 0; --s) {
        const int64_t above = s + 1 < nblk ? (int64_t)s * kNB : 0;
        const int grid = 1 + (int)((above + kRowsPerWG - 1) / kRowsPerWG);
        k_trsv_bwd<<<grid, 256, 0, stream>>>(LU, N, Uinv, x, s, nblk);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "coarse triangular solves");
    return FTS_OK;
}

}  // namespace fts
