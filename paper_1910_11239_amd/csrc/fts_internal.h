// Internal declarations of libfts: handle layouts, kernel argument structs,
// host setup helpers and the launchers of the HIP kernels.
#pragma once

#include <functional>

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fts.h"

namespace fts {

constexpr int kMaxDegree = 9;     // 3-D
constexpr int kMaxDegree2D = 15;  // 2-D (a patch of n = 32 lines still fits a workgroup)
constexpr int kMaxN1 = kMaxDegree + 1;
constexpr int kMaxN1Any = kMaxDegree2D + 1;

void set_error(const std::string &msg);

// Device memory of the library comes from the allocator registered with
// fts_set_allocator (the caller's, e.g. torch's); without one every
// allocation fails.  dev_free returns memory to it.
hipError_t dev_malloc_raw(void **p, size_t bytes);
void dev_free(void *p);
template <typename T>
inline hipError_t dev_malloc(T **p, size_t bytes) {
    return dev_malloc_raw(reinterpret_cast<void **>(p), bytes);
}
fts_status fail(fts_status code, const std::string &msg);
fts_status hip_fail(hipError_t err, const char *what);

#define FTS_HIP_CHECK(call)                                   \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return ::fts::hip_fail(e_, #call); \
    } while (0)

// ---------------------------------------------------------------------------
// Host 1-D reference data on [0, 1] (Sec. 2.1, Sec. 3 intro): Gauss-Lobatto
// nodes, exact mass / stiffness matrices, endpoint values and derivatives,
// and the two child-embedding matrices of the midpoint refinement.
struct Ref1D {
    int k = 0, n1 = 0;
    std::vector<double> nodes;   // n1
    std::vector<double> Mhat;    // n1 x n1, [test][trial]
    std::vector<double> Lhat;    // n1 x n1
    std::vector<double> v0, v1;  // phi_i(0), phi_i(1)
    std::vector<double> d0, d1;  // phi_i'(0), phi_i'(1)
    std::vector<double> E[2];    // E_c[i][j] = phi_j((xi_i + c)/2)
    void build(int degree);
    // 1-D SIPG matrices (Sec. 3.2), row = test function, column = trial function.
    // Neighbour widths <= 0 mean "boundary face".
    void cell_operator(double h, double h_left, double h_right, double gamma_hat,
                       double *A) const;
    void interface_block(double hl, double hr, double gamma_hat, double *B) const;
    // Derivatives with respect to gamma_hat (the operators are affine in it):
    // the penalty terms alone, evaluated at gamma_hat = 1.
    void cell_penalty(double h, double h_left, double h_right, double *A) const;
    void interface_penalty(double hl, double hr, double *B) const;
};

// (k+1)-point Gauss rule on [0, 1] (points xq, weights wq) and the values
// V[q][i] = phi_i(xq_q) and derivatives D[q][i] = phi_i'(xq_q) of the
// Gauss-Lobatto Lagrange basis of degree k there.
void gauss_basis(int k, std::vector<double> &xq, std::vector<double> &wq, std::vector<double> &V,
                 std::vector<double> &D);

// Generalised symmetric-definite eigenproblem A S = M S diag(lam), S^T M S = I,
// by Cholesky of M and cyclic Jacobi on L^-1 A L^-T (FP64, host).
// Returns FTS_E_NOT_SPD if M is not positive definite or an eigenvalue <= 0.
fts_status sym_gen_eig(int n, const double *A, const double *M, double *S, double *lam);

// ---------------------------------------------------------------------------
// Device-side views passed to kernels by value.
struct LevelView {
    int m[3];                 // cells per axis (m[2] = 1 in 2-D)
    int64_t ncells;
    const double *cellop[3];  // per axis: m[a] blocks of n1 x n1 (A_cell, eq. 1Dsipg)
    const double *iface[3];   // per axis: m[a]-1 blocks, coupling cell c (test) to c+1 (trial)
    const double *h[3];       // per axis widths
    const double *ih[3];      // per axis 1 / widths
    const double *Mhat;       // n1 x n1
    const double *E;          // 2 x n1 x n1 embedding matrices
    const double *Lhat;       // n1 x n1 reference stiffness
    const double *d0, *d1;    // derivatives of the basis at 0 and at 1
    const double *Meo, *Leo;  // Mhat, Lhat in even-odd form: E ((n1+1)/2)^2 then O (n1/2)^2, row-major
    double gk, pk;            // gamma_hat k (k+1) and k (k+1)
};

// Levels of at least this many cells use the owner tiles under FTS_SCHEDULE_AUTO.
constexpr int64_t kOwnerMinCells = 4096;

// The schedule a call of the 16-bit vertex-patch smoother actually runs:
// FTS_SCHEDULE_AUTO resolved by the level size.
inline int effective_schedule(int schedule, int64_t ncells) {
    if (schedule != FTS_SCHEDULE_AUTO) return schedule;
    return ncells >= kOwnerMinCells ? FTS_SCHEDULE_OWNER : FTS_SCHEDULE_STAGED;
}

// Cell runs of the matrix-free operator launch.  Workgroups are handed to the
// 8 XCDs round-robin (block b to XCD b % 8), and each XCD has its own L2.  The
// rows (y, z) are split into min(8, m_y) groups of consecutive y; at fixed z
// the rows of a group are one contiguous range of cells (a segment), cut into
// runs of cpw cells (the last run of a segment may be shorter).  XCD j takes a
// contiguous range of the order (group, z, run), so the x-, y- and
// z-neighbours whose lines a cell reads were read shortly before on the same
// XCD (within one segment of its group).
struct OpRuns {
    int m0, m1, m2, cpw, groups;
    int64_t nblocks;
};

// first row and row count of group gi
__host__ __device__ inline void op_group_rows(const OpRuns &o, int gi, int *y0, int *sy) {
    const int a = (int)((int64_t)gi * o.m1 / o.groups), e = (int)((int64_t)(gi + 1) * o.m1 / o.groups);
    *y0 = a;
    *sy = e - a;
}

inline OpRuns op_runs(const int m[3], int dim, int cpw) {
    OpRuns o;
    o.m0 = m[0];
    o.m1 = m[1];
    o.m2 = dim == 3 ? m[2] : 1;
    o.cpw = cpw;
    o.groups = o.m1 < 8 ? o.m1 : 8;
    o.nblocks = 0;
    for (int gi = 0; gi < o.groups; ++gi) {
        int y0, sy;
        op_group_rows(o, gi, &y0, &sy);
        o.nblocks += ((int64_t)sy * o.m0 + cpw - 1) / cpw * o.m2;
    }
    return o;
}

// block b -> first cell and number of cells (1..cpw) of its run
__host__ __device__ inline void op_run_of_block(const OpRuns &o, int64_t b, int64_t *cell0, int *nact) {
    const int64_t q = o.nblocks / 8, r = o.nblocks % 8;
    const int64_t xcd = b % 8, i = b / 8;
    int64_t L = xcd * q + (xcd < r ? xcd : r) + i;  // position in the (group, z, run) order
    int y0 = 0, sy = o.m1;
    int64_t seg = 0, nrun = 1;
    for (int gi = 0; gi < o.groups; ++gi) {
        op_group_rows(o, gi, &y0, &sy);
        seg = (int64_t)sy * o.m0;
        nrun = (seg + o.cpw - 1) / o.cpw;
        if (L < nrun * o.m2) break;
        L -= nrun * o.m2;
    }
    const int64_t run = L % nrun, z = L / nrun;
    *cell0 = (z * o.m1 + y0) * o.m0 + run * o.cpw;
    const int64_t left = seg - run * o.cpw;
    *nact = left < o.cpw ? (int)left : o.cpw;
}

// The coarse matrix stored by slabs of cells (all cells sharing their
// coordinate along the last axis).  Unknowns are numbered cell by cell with
// the last axis slowest, so a slab is a contiguous range of B unknowns, and
// the face couplings of SIPG reach only the two neighbouring slabs: A_0 is
// block tridiagonal.  Block (i, i) is D + i B^2, block (i, i-1) is
// Lo + (i-1) B^2 and block (i, i+1) is Up + i B^2, each B x B column-major.
struct SlabBlocks {
    double *D, *Lo, *Up;
    int64_t B;
};

struct EigView {
    int count[3];             // positions per axis
    const double *S[3];       // per axis: count blocks of n x n, row-major [i][m]
    const double *ST[3];      // transposes, row-major [m][i]
    const double *lam[3];     // per axis: count blocks of n
    const float *S32[3];
    const float *ST32[3];
    const float *lam32[3];
    // 16-bit operands of the MFMA path (n <= 16, padded to 16 x 16): for each
    // axis and position the forward matrix F[o][k] = S[k][o] / s and the
    // backward matrix B[o][k] = S[o][k] / s with s = max |S|; FP16 and BF16
    // bit patterns.  mscale = s, lmin = smallest eigenvalue (FP32).
    const uint16_t *Ff16[3], *Bf16[3], *Fbf16[3], *Bbf16[3];
    const float *mscale[3], *lmin[3];
    // S^T (dA/dgamma_hat) S per axis position (n x n, FP64), for the adjoint
    const double *DG[3];
    // per axis and position: the first position with the same tables (the
    // kernels read their tables there, so that a uniform mesh touches only
    // a few distinct tables)
    const int *cls[3];
    // per axis and position: 1 if its modes are ordered even-then-odd about
    // the centre and S is exactly even / odd in them (contractions may use
    // the even-odd form with the first n/2 rows of S), else 0
    const int *sym[3];
};

}  // namespace fts

struct fts_level {
    int dim = 0, k = 0, n1 = 0;
    int m[3] = {1, 1, 1};
    std::vector<double> h[3];
    double gamma_hat = 1.0;
    int64_t ncells = 0, ndofs = 0;
    fts::Ref1D ref;
    std::vector<double> host_cellop[3], host_iface[3];
    double *d_tab = nullptr;  // single device allocation holding every table
    fts::LevelView view{};
};

struct fts_eigs {
    const fts_level *level = nullptr;
    int kind = 0, n = 0;
    int count[3] = {0, 0, 0};
    std::vector<double> A[3], M[3], S[3], lam[3], DG[3];
    std::vector<int> cls[3], sym[3];
    int *d_cls = nullptr;
    double *d_tab = nullptr;
    float *d_tab32 = nullptr;
    double *d_stage = nullptr;  // staged corrections of all vertex patches (one per cell of each;
                                // FP64 or FP32 values, sized for FP64)
    double *d_stage_scale = nullptr;  // one FP64 factor per patch for the 16-bit path
    void *d_mfma = nullptr;     // 16-bit MFMA tables (n <= 16 only)
    int schedule = FTS_SCHEDULE_AUTO;  // owner tiles for 16-bit 3-D vertex patches on large levels, else staged
    fts::EigView view{};
};

namespace fts {
// Launchers (kernels.hip).  All asynchronous on `stream`.
fts_status launch_operator(const fts_level *lv, const double *x, const double *b, double *y,
                           bool residual, hipStream_t stream);
// y = (dA/dgamma_hat) x on the level (penalty terms at gamma_hat = 1)
fts_status launch_operator_penalty(const fts_level *lv, const double *x, double *y, hipStream_t stream);
// out[blockIdx] partial sums of sum_j (L^-1 Z^T R_j u)^T (sum_t I x D_t x I) (L^-1 Z^T R_j v)
// over the subdomains; returns the number of partials in *npart.  FP64.
fts_status launch_schwarz_dgamma(const fts_level *lv, const fts_eigs *eg, const double *u, const double *v,
                                 double *partials, int64_t *npart, hipStream_t stream);
// out[0] += scale * sum_i x[i] y[i]  (deterministic; part: 2 * red_partials())
fts_status launch_dot_acc(const double *x, const double *y, int64_t n, double scale, double *part, double *out,
                          hipStream_t stream);
// out[0] += scale * sum_i x[i]
fts_status launch_sum_acc(const double *x, int64_t n, double scale, double *part, double *out, hipStream_t stream);
// y += a x
fts_status launch_axpy(double a, const double *x, double *y, int64_t n, hipStream_t stream);
fts_status launch_schwarz(const fts_level *lv, const fts_eigs *eg, double omega, fts_prec prec,
                          const double *r, double *x, hipStream_t stream);
// 16-bit local solves of 3-D vertex patches by owner-computes tiles (tile.hip):
// x += omega sum_j R_j^T A_j^-1 R_j r; r (FP64, or FP32 if r_f32) must be
// 16-byte aligned.
fts_status launch_schwarz_mfma_tile(const fts_level *lv, const fts_eigs *eg, double omega, int bf, const void *r,
                                    bool r_f32, double *x, hipStream_t stream);
// One additive smoothing step x <- x + omega C (b - A x) (Alg. addsmoother);
// x_zero: x is zero, r = b.  rbuf: ndofs doubles of space for the residual,
// which is stored in FP32 when the local solves are 16-bit owner tiles.
fts_status smooth_additive(const fts_level *lv, const fts_eigs *eg, double omega, fts_prec prec, const double *b,
                           double *x, void *rbuf, bool x_zero, hipStream_t stream);
// Colors of the multiplicative smoother: 2 (red-black cells) or 2^(d+1)
// (vertex patches); one color's local solves added to x in place.
int schwarz_mult_colors(const fts_eigs *eg);
fts_status launch_schwarz_color(const fts_level *lv, const fts_eigs *eg, double omega, fts_prec prec,
                                const double *r, double *x, int color, hipStream_t stream);
fts_status launch_restrict(const fts_level *coarse, const fts_level *fine, const double *rf,
                           double *bc, hipStream_t stream);
fts_status launch_prolongate(const fts_level *coarse, const fts_level *fine, const double *ec,
                             double *xf, hipStream_t stream);
fts_status launch_assemble_slabs(const fts_level *lv, const SlabBlocks &blk, hipStream_t stream);
fts_status launch_fill(double *p, int64_t n, double v, hipStream_t stream);
// out[0] = x.y, out[1] = x.z (z may be NULL); part: 2 * red_partials() doubles
fts_status launch_dot2(const double *x, const double *y, const double *z, int64_t n, double *part, double *out,
                       hipStream_t stream);
fts_status launch_cg_update(double *x, double *r, const double *p, const double *q, double alpha, int64_t n,
                            hipStream_t stream);
fts_status launch_xpby(double *p, const double *z, double beta, int64_t n, hipStream_t stream);
// p *= a
fts_status launch_scale(double *p, double a, int64_t n, hipStream_t stream);
int red_partials();
// cells per workgroup of the operator kernels (the batched residual's blocks)
int operator_cells_per_block(int dim, int n1);

// Direct solver of the coarsest level (coarse.hip).
struct CoarseLU;
fts_status coarse_create(const fts_level *l0, hipStream_t stream, CoarseLU **out);
// The same factorisation of a matrix with the slab structure of l0 (cell
// counts, degree, DoF numbering), whose blocks `fill` writes into the zeroed
// slab storage (launch_assemble_slabs for the Cartesian A_0).
fts_status coarse_create_with(const fts_level *l0, const std::function<fts_status(const SlabBlocks &)> &fill,
                              hipStream_t stream, CoarseLU **out);
void coarse_destroy(CoarseLU *c);
// x = A_0^-1 b; x must not alias b.  Uses the solver's own workspaces, so
// solves with one CoarseLU must not overlap.
fts_status coarse_solve(CoarseLU *c, const double *b, double *x, hipStream_t stream);
}  // namespace fts
