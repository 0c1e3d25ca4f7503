// Batched additive vertex-patch smoothing of many independent 3-D meshes of
// mixed degree and anisotropic (rectilinear) cells: every patch has its own
// per-axis 1-D eigen-data (Sec. 3.2, eq. generalizedEVP), and all patches of
// all meshes are processed by one persistent launch.
//
// Work queue: the meshes are listed in decreasing degree (largest local
// solves first) and each mesh's patches are cut into chunks; persistent
// workgroups take chunks with a 64-bit atomic counter until none is left
// (every workgroup reaches the exit).  A chunk lies inside one mesh, so a
// workgroup runs one degree's body for the whole chunk.  The body is the
// direct-line form of the single-mesh kernel (residual lines read straight
// into the first contraction, the last one written straight to the staging
// buffer, scalar-loaded 1-D tables, last axis fused in registers),
// the same for every degree.  A batched gather adds the staged corrections of
// each cell in a fixed order.
// The FP64 residual runs as one launch per degree present.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>

#include "device_common.h"

namespace fts {
fts_status setup_eigs_internal(const fts_level *lv, fts_patch_kind kind, bool staging, fts_eigs **out);
}

namespace fts {

struct BatchMesh {
    LevelView lv;
    EigView ev;
    int64_t dof_off, stage_off;
    int n1, pad;
    int cnt[3], pad2;
};

struct BatchBlock {
    int mesh, pad;
    int64_t first;  // first cell (residual) or first DoF (gather) of the block
};

constexpr int kBatchMaxN = 20;  // vertex patch of degree 9

// The local solve of one vertex patch with TH threads: thread t owns the
// x-lines t, t + TH, ... (at most two: N^2 <= 2 TH), taken one after the
// other.  The first forward contraction reads the thread's residual line
// straight from global memory (two runs of k+1 values), y and z go through
// LDS (z forward, eigenvalue scaling and z backward fused in registers), and
// the last backward contraction writes the staged correction straight from
// registers: no separate gather and scatter passes through LDS.
template <int N1, int TH, typename T>
__device__ __forceinline__ void batch_patch_lines(const BatchMesh &M, int64_t p, const double *__restrict__ r,
                                                  T *__restrict__ W, T om, T *Ts) {
    constexpr int N = 2 * N1, NC1 = N1 * N1 * N1, NN = N * N, LINES = NN;
    constexpr int BL = (LINES + TH - 1) / TH;
    static_assert(BL <= 2, "at most two lines per thread");
    const int t = threadIdx.x;
    int pos[3];
    pos[0] = __builtin_amdgcn_readfirstlane((int)(p % M.cnt[0]));
    pos[1] = __builtin_amdgcn_readfirstlane((int)((p / M.cnt[0]) % M.cnt[1]));
    pos[2] = __builtin_amdgcn_readfirstlane((int)(p / ((int64_t)M.cnt[0] * M.cnt[1])));
    const EigView &e = M.ev;
    const int64_t cs1 = M.lv.m[0], cs2 = (int64_t)M.lv.m[0] * M.lv.m[1];
    T v[N], w[N];
    // x forward, from global memory
    for (int k = 0; k < BL; ++k) {
        const int l = t + k * TH;
        if (l < LINES) {
            const int a1 = l % N, a2 = l / N;
            const int o1 = a1 / N1, i1 = a1 % N1, o2 = a2 / N1, i2 = a2 % N1;
            const int64_t cell0 = pos[0] + (pos[1] + o1) * cs1 + (pos[2] + o2) * cs2;
            const double *src = r + M.dof_off + cell0 * NC1 + i1 * N1 + i2 * N1 * N1;
#pragma unroll
            for (int o0 = 0; o0 < 2; ++o0)
#pragma unroll
                for (int i0 = 0; i0 < N1; ++i0) v[o0 * N1 + i0] = (T)src[o0 * NC1 + i0];
            matvec_regs<N>(v, w, uniform_table(EigTab<T>::ST(e, 0) + (size_t)pos[0] * NN));
#pragma unroll
            for (int a = 0; a < N; ++a) Ts[N * l + a] = w[a];
        }
    }
    __syncthreads();
    // y forward
    for (int k = 0; k < BL; ++k) {
        const int l = t + k * TH;
        if (l < LINES) contract_at<N, T>(Ts, line_base<3, N>(1, l), N,
                                         uniform_table(EigTab<T>::ST(e, 1) + (size_t)pos[1] * NN));
    }
    __syncthreads();
    // z: forward, scaling by omega / (lambda_x + lambda_y + lambda_z), backward
    {
        cptr<T> L0 = uniform_table(EigTab<T>::L(e, 0) + (size_t)pos[0] * N);
        cptr<T> L1 = uniform_table(EigTab<T>::L(e, 1) + (size_t)pos[1] * N);
        cptr<T> L2 = uniform_table(EigTab<T>::L(e, 2) + (size_t)pos[2] * N);
        for (int k = 0; k < BL; ++k) {
            const int l = t + k * TH;
            if (l < LINES) {
                const int base = line_base<3, N>(2, l);
#pragma unroll
                for (int i = 0; i < N; ++i) v[i] = Ts[base + i * NN];
                matvec_regs<N>(v, w, uniform_table(EigTab<T>::ST(e, 2) + (size_t)pos[2] * NN));
                const T lr = (T)L0[l % N] + (T)L1[l / N];
#pragma unroll
                for (int m = 0; m < N; ++m) w[m] = w[m] * (om * recip(lr + (T)L2[m]));
                matvec_regs<N>(w, v, uniform_table(EigTab<T>::S(e, 2) + (size_t)pos[2] * NN));
#pragma unroll
                for (int i = 0; i < N; ++i) Ts[base + i * NN] = v[i];
            }
        }
    }
    __syncthreads();
    // y backward
    for (int k = 0; k < BL; ++k) {
        const int l = t + k * TH;
        if (l < LINES) contract_at<N, T>(Ts, line_base<3, N>(1, l), N,
                                         uniform_table(EigTab<T>::S(e, 1) + (size_t)pos[1] * NN));
    }
    __syncthreads();
    // x backward, to the staging buffer
    T *Wm = W + M.stage_off + p * (8 * NC1);
    for (int k = 0; k < BL; ++k) {
        const int l = t + k * TH;
        if (l < LINES) {
#pragma unroll
            for (int a = 0; a < N; ++a) v[a] = Ts[N * l + a];
            matvec_regs<N>(v, w, uniform_table(EigTab<T>::S(e, 0) + (size_t)pos[0] * NN));
            const int a1 = l % N, a2 = l / N;
            const int o1 = a1 / N1, i1 = a1 % N1, o2 = a2 / N1, i2 = a2 % N1;
            T *dst = Wm + (2 * o1 + 4 * o2) * NC1 + i1 * N1 + i2 * N1 * N1;
#pragma unroll
            for (int o0 = 0; o0 < 2; ++o0)
#pragma unroll
                for (int i0 = 0; i0 < N1; ++i0) dst[o0 * NC1 + i0] = w[o0 * N1 + i0];
        }
    }
    __syncthreads();  // Ts is reused by the next patch
}

template <int TH, typename T>
__global__ void __launch_bounds__(TH) __attribute__((amdgpu_waves_per_eu(4)))
k_batch_smooth(const BatchMesh *__restrict__ meshes, const int64_t *__restrict__ prefix,
               const int *__restrict__ order, int nslot, int chunk,
               unsigned long long *__restrict__ counter, const double *__restrict__ r, T *__restrict__ W,
               double omega) {
    __shared__ T Ts[kBatchMaxN * kBatchMaxN * kBatchMaxN];
    __shared__ unsigned long long item_s;
    const T om = (T)omega;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(counter, 1ull);
        __syncthreads();
        // the same value in every lane; readfirstlane tells the compiler so, and
        // the chunk bounds and the degree switch below stay scalar branches
        const unsigned long long it = item_s;
        int64_t item = (int64_t)(((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(it >> 32)) << 32) |
                                 (unsigned)__builtin_amdgcn_readfirstlane((unsigned)it));
        __syncthreads();
        // work item -> (queue slot, chunk of that slot's patches): slot s has
        // ceil(np_s / chunk) chunks, the slots in queue order
        int slot = 0;
        int64_t np = 0;
        for (; slot < nslot; ++slot) {
            np = prefix[slot + 1] - prefix[slot];
            const int64_t nch = (np + chunk - 1) / chunk;
            if (item < nch) break;
            item -= nch;
        }
        if (slot >= nslot) break;  // every item taken: all workgroups leave here
        const int mi = __builtin_amdgcn_readfirstlane(order[slot]);
        const BatchMesh &M = meshes[mi];
        const int64_t p0 = item * chunk, p1 = p0 + chunk < np ? p0 + chunk : np;
        switch (M.n1) {
#define FTS_BATCH_CASE(N1) \
    case N1:               \
        for (int64_t p = p0; p < p1; ++p) batch_patch_lines<N1, TH, T>(M, p, r, W, om, Ts); \
        break;
            FTS_BATCH_CASE(2)
            FTS_BATCH_CASE(3)
            FTS_BATCH_CASE(4)
            FTS_BATCH_CASE(5)
            FTS_BATCH_CASE(6)
            FTS_BATCH_CASE(7)
            FTS_BATCH_CASE(8)
            FTS_BATCH_CASE(9)
            FTS_BATCH_CASE(10)
#undef FTS_BATCH_CASE
            default: break;
        }
    }
}

__global__ void k_batch_reset(unsigned long long *counter) { *counter = 0ull; }

// x += the staged corrections (FP64 or FP32, the contraction type) of the
// 8 patches around each cell, in FP64 and in a fixed order.  One launch per
// degree present (compile-time cell size: the index arithmetic is a few
// multiplications); a block covers kGatherPer x 256 consecutive DoFs of one
// mesh.  Where (k+1)^3 is a multiple of 4 a thread takes 4 consecutive DoFs of
// one cell and reads each patch's 4 staged values with one vector load (the
// staging blocks of a mesh start at multiples of 8 (k+1)^3 values); otherwise
// consecutive threads take consecutive DoFs, kGatherPer rounds.
constexpr int kGatherPer = 4;

template <typename WT, int V>
struct GVec;
template <> struct GVec<float, 1> { typedef float type; };
template <> struct GVec<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct GVec<double, 1> { typedef double type; };
template <> struct GVec<double, 4> { typedef double type __attribute__((ext_vector_type(4))); };

template <int N1, typename WT>
__global__ void __launch_bounds__(256)
k_batch_gather(const BatchMesh *__restrict__ meshes, const BatchBlock *__restrict__ blocks,
               const WT *__restrict__ W, double *__restrict__ x) {
    constexpr int NC1 = N1 * N1 * N1;
    constexpr int V = NC1 % 4 == 0 ? 4 : 1;
    constexpr int ROUNDS = kGatherPer / V;
    using WV = typename GVec<WT, V>::type;
    const BatchBlock B = blocks[blockIdx.x];
    const BatchMesh &M = meshes[B.mesh];
    // per mesh: at most 24^3 cells of (k+1)^3 <= 1000 DoFs and 23^3 patches of
    // 8 (k+1)^3 staged values, so 32-bit offsets suffice inside a mesh
    const int nd = (int)(M.lv.ncells * NC1);
    const int m0 = M.lv.m[0], m1 = M.lv.m[1];
    const int cnt0 = M.cnt[0], cnt1 = M.cnt[1], cnt2 = M.cnt[2];
    const WT *Wm = W + M.stage_off;
    double *xm = x + M.dof_off;
#pragma unroll
    for (int u = 0; u < ROUNDS; ++u) {
        const int gid = (int)B.first + (u * 256 + (int)threadIdx.x) * V;  // first DoF of this thread
        if (gid < nd) {
            const int cell = gid / NC1, i = gid - cell * NC1;
            const int r0 = cell / m0;
            const int c0 = cell - r0 * m0, c1 = r0 % m1, c2 = r0 / m1;
            WV acc[8];
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int a0 = c0 - (o & 1), a1 = c1 - ((o >> 1) & 1), a2 = c2 - ((o >> 2) & 1);
                const bool in = a0 >= 0 && a0 < cnt0 && a1 >= 0 && a1 < cnt1 && a2 >= 0 && a2 < cnt2;
                acc[o] = in ? *(const WV *)(Wm + (a0 + cnt0 * (a1 + cnt1 * a2)) * (8 * NC1) + o * NC1 + i)
                               : (WV)0;
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                double sum = 0.0;
#pragma unroll
                for (int o = 0; o < 8; ++o) {
                    if constexpr (V == 1) sum += (double)acc[o];
                    else sum += (double)acc[o][v];
                }
                xm[gid + v] += sum;
            }
        }
    }
}

template <int D, int N1>
struct RunBatchGather {
    template <typename WT>
    static fts_status run(const BatchMesh *meshes, const BatchBlock *blocks, int64_t nblocks, const WT *W, double *x,
                          hipStream_t st) {
        if constexpr (D != 3) {
            return fail(FTS_E_UNSUPPORTED, "batches are 3-D");
        } else {
            k_batch_gather<N1, WT><<<dim3((unsigned)nblocks), dim3(256), 0, st>>>(meshes, blocks, W, x);
            return check_launch("k_batch_gather");
        }
    }
};

template <int N1>
__global__ void __launch_bounds__((OpCfg<3, N1>::THREADS))
k_batch_residual(const BatchMesh *__restrict__ meshes, const BatchBlock *__restrict__ blocks,
                 const double *__restrict__ x, const double *__restrict__ b, double *__restrict__ r) {
    const BatchBlock B = blocks[blockIdx.x];
    const LevelView g = meshes[B.mesh].lv;
    const int64_t off = meshes[B.mesh].dof_off;
    const int64_t left = g.ncells - B.first;
    const int nact = left < OpCfg<3, N1>::CPW ? (int)left : OpCfg<3, N1>::CPW;
    operator_cells<3, N1, true>(g, B.first, nact, x + off, b + off, r + off);
}

template <int D, int N1>
struct RunBatchResidual {
    static fts_status run(const BatchMesh *meshes, const BatchBlock *blocks, int64_t nblocks, const double *x,
                          const double *b, double *r, hipStream_t st) {
        if constexpr (D != 3) {
            return fail(FTS_E_UNSUPPORTED, "batches are 3-D");
        } else {
            k_batch_residual<N1><<<dim3((unsigned)nblocks), dim3(OpCfg<3, N1>::THREADS), 0, st>>>(meshes, blocks, x,
                                                                                                   b, r);
            return check_launch("k_batch_residual");
        }
    }
};

}  // namespace fts

using namespace fts;

struct fts_batch {
    int nmesh = 0;
    std::vector<fts_level *> levels;
    std::vector<fts_eigs *> eigs;
    std::vector<int64_t> dof_off, ndofs;
    int64_t ndofs_total = 0, patches_total = 0;
    BatchMesh *d_meshes = nullptr;
    int64_t *d_prefix = nullptr;
    int *d_order = nullptr;
    int nslot = 0;
    unsigned long long *d_counter = nullptr;
    double *d_stage = nullptr;
    struct Group {
        int n1;
        BatchBlock *blocks;
        int64_t nblocks;
    };
    std::vector<Group> res_groups;
    std::vector<Group> gather_groups;  // per degree present: blocks of kGatherPer x 256 DoFs
    int threads = 256, grid = 0, chunk = 4;  // launch shape (autotuned)
    int ncu = 256;
};

static fts_status batch_launch_smooth(fts_batch *bt, int threads, int grid, int chunk, fts_prec prec,
                                      const double *r, double omega, hipStream_t s) {
    k_batch_reset<<<1, 1, 0, s>>>(bt->d_counter);
    const bool f32 = prec == FTS_PREC_F32;
#define FTS_BATCH_LAUNCH(TH)                                                                            \
    if (f32)                                                                                           \
        k_batch_smooth<TH, float><<<grid, TH, 0, s>>>(bt->d_meshes, bt->d_prefix, bt->d_order, bt->nslot, \
                                                      chunk, bt->d_counter, r,                          \
                                                      reinterpret_cast<float *>(bt->d_stage), omega);    \
    else                                                                                               \
        k_batch_smooth<TH, double><<<grid, TH, 0, s>>>(bt->d_meshes, bt->d_prefix, bt->d_order,           \
                                                       bt->nslot, chunk, bt->d_counter, r, bt->d_stage,   \
                                                       omega);
    if (threads == 256) {
        FTS_BATCH_LAUNCH(256)
    } else if (threads == 512) {
        FTS_BATCH_LAUNCH(512)
    } else {
        return fail(FTS_E_INVAL, "batch: threads must be 256 or 512");
    }
#undef FTS_BATCH_LAUNCH
    return check_launch("k_batch_smooth");
}

extern "C" {

fts_status fts_batch_destroy(fts_batch *bt) {
    if (!bt) return FTS_OK;
    for (auto *e : bt->eigs) fts_eigs_destroy(e);
    for (auto *l : bt->levels) fts_level_destroy(l);
    if (bt->d_meshes) dev_free(bt->d_meshes);
    if (bt->d_prefix) dev_free(bt->d_prefix);
    if (bt->d_order) dev_free(bt->d_order);
    if (bt->d_counter) dev_free(bt->d_counter);
    if (bt->d_stage) dev_free(bt->d_stage);
    for (auto &g : bt->res_groups)
        if (g.blocks) dev_free(g.blocks);
    for (auto &g : bt->gather_groups)
        if (g.blocks) dev_free(g.blocks);
    delete bt;
    return FTS_OK;
}

fts_status fts_batch_create(const fts_mesh_desc *meshes, int32_t nmesh, fts_batch **out) {
    if (!meshes || !out || nmesh < 1) return fail(FTS_E_INVAL, "fts_batch_create: invalid arguments");
    *out = nullptr;
    fts_batch *bt = new fts_batch();
    bt->nmesh = nmesh;
    fts_status st = FTS_OK;
    std::vector<BatchMesh> host(nmesh);
    int64_t stage_total = 0;
    for (int i = 0; i < nmesh && st == FTS_OK; ++i) {
        if (meshes[i].dim != 3) {
            st = fail(FTS_E_UNSUPPORTED, "batched meshes must be 3-D");
            break;
        }
        fts_level *lv = nullptr;
        st = fts_level_create(&meshes[i], &lv);
        if (st != FTS_OK) break;
        bt->levels.push_back(lv);
        fts_eigs *eg = nullptr;
        st = setup_eigs_internal(lv, FTS_VERTEX_PATCH, false, &eg);
        if (st != FTS_OK) break;
        bt->eigs.push_back(eg);
        BatchMesh &M = host[i];
        M.lv = lv->view;
        M.ev = eg->view;
        M.dof_off = bt->ndofs_total;
        M.stage_off = stage_total;
        M.n1 = lv->n1;
        int64_t np = 1;
        for (int a = 0; a < 3; ++a) {
            M.cnt[a] = eg->count[a];
            np *= eg->count[a];
        }
        bt->dof_off.push_back(bt->ndofs_total);
        bt->ndofs.push_back(lv->ndofs);
        bt->ndofs_total += lv->ndofs;
        stage_total += np * 8 * (int64_t)lv->n1 * lv->n1 * lv->n1;
        bt->patches_total += np;
    }
    if (st != FTS_OK) {
        fts_batch_destroy(bt);
        return st;
    }
    // queue order: decreasing degree (stable), prefix sums of patch counts
    std::vector<int> order(nmesh);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return host[a].n1 > host[b].n1; });
    std::vector<int64_t> prefix(nmesh + 1, 0);
    for (int s = 0; s < nmesh; ++s)
        prefix[s + 1] = prefix[s] + (int64_t)host[order[s]].cnt[0] * host[order[s]].cnt[1] * host[order[s]].cnt[2];
    bt->nslot = nmesh;
    // residual and gather blocks, grouped by degree (one launch per degree)
    auto upload_group = [&](std::vector<fts_batch::Group> &groups, int n1, const std::vector<BatchBlock> &blocks) {
        if (blocks.empty() || st != FTS_OK) return;
        fts_batch::Group g{n1, nullptr, (int64_t)blocks.size()};
        if (dev_malloc(&g.blocks, blocks.size() * sizeof(BatchBlock)) != hipSuccess ||
            hipMemcpy(g.blocks, blocks.data(), blocks.size() * sizeof(BatchBlock), hipMemcpyHostToDevice) != hipSuccess)
            st = fail(FTS_E_HIP, "batch: upload of launch blocks failed");
        groups.push_back(g);
    };
    for (int n1 = 2; n1 <= kMaxN1 && st == FTS_OK; ++n1) {
        std::vector<BatchBlock> rblocks, gblocks;
        for (int i = 0; i < nmesh; ++i) {
            if (host[i].n1 != n1) continue;
            const int cpw = operator_cells_per_block(3, n1);
            for (int64_t c = 0; c < bt->levels[i]->ncells; c += cpw) rblocks.push_back({i, 0, c});
            for (int64_t d = 0; d < bt->ndofs[i]; d += kGatherPer * 256) gblocks.push_back({i, 0, d});
        }
        upload_group(bt->res_groups, n1, rblocks);
        upload_group(bt->gather_groups, n1, gblocks);
    }
    auto up = [&](void **dst, const void *src, size_t bytes) {
        if (st != FTS_OK) return;
        if (dev_malloc(dst, std::max<size_t>(bytes, 8)) != hipSuccess ||
            (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess))
            st = fail(FTS_E_HIP, "batch: upload failed");
    };
    up((void **)&bt->d_meshes, host.data(), host.size() * sizeof(BatchMesh));
    up((void **)&bt->d_prefix, prefix.data(), prefix.size() * sizeof(int64_t));
    up((void **)&bt->d_order, order.data(), order.size() * sizeof(int));
    if (st == FTS_OK && (dev_malloc(&bt->d_counter, sizeof(unsigned long long)) != hipSuccess ||
                         dev_malloc(&bt->d_stage, (size_t)std::max<int64_t>(stage_total, 1) * sizeof(double)) != hipSuccess))
        st = fail(FTS_E_HIP, "batch: allocation of the staging buffer failed");
    if (st == FTS_OK) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            bt->ncu = prop.multiProcessorCount;
        bt->grid = 4 * bt->ncu;
    }
    if (st != FTS_OK) {
        fts_batch_destroy(bt);
        return st;
    }
    *out = bt;
    return FTS_OK;
}

int64_t fts_batch_ndofs(const fts_batch *bt) { return bt ? bt->ndofs_total : -1; }

fts_status fts_batch_mesh_offset(const fts_batch *bt, int32_t mesh, int64_t *offset, int64_t *ndofs) {
    if (!bt || mesh < 0 || mesh >= bt->nmesh) return fail(FTS_E_INVAL, "fts_batch_mesh_offset: bad mesh index");
    if (offset) *offset = bt->dof_off[mesh];
    if (ndofs) *ndofs = bt->ndofs[mesh];
    return FTS_OK;
}

fts_status fts_batch_residual(fts_batch *bt, const double *b, const double *x, double *r, void *stream) {
    if (!bt || !b || !x || !r) return fail(FTS_E_INVAL, "fts_batch_residual: NULL argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (auto &g : bt->res_groups) {
        fts_status st = dispatch<RunBatchResidual>(3, g.n1, bt->d_meshes, g.blocks, g.nblocks, x, b, r, s);
        if (st != FTS_OK) return st;
    }
    return FTS_OK;
}

fts_status fts_batch_apply(fts_batch *bt, double omega, fts_prec prec, const double *r, double *x, void *stream) {
    if (!bt || !r || !x) return fail(FTS_E_INVAL, "fts_batch_apply: NULL argument");
    if (prec != FTS_PREC_F64 && prec != FTS_PREC_F32)
        return fail(FTS_E_UNSUPPORTED, "batched smoothing supports FP64 and FP32 contractions");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    fts_status st = batch_launch_smooth(bt, bt->threads, bt->grid, bt->chunk, prec, r, omega, s);
    if (st != FTS_OK) return st;
    for (auto &g : bt->gather_groups) {
        st = prec == FTS_PREC_F32
                 ? dispatch<RunBatchGather>(3, g.n1, bt->d_meshes, g.blocks, g.nblocks,
                                            reinterpret_cast<const float *>(bt->d_stage), x, s)
                 : dispatch<RunBatchGather>(3, g.n1, bt->d_meshes, g.blocks, g.nblocks,
                                            static_cast<const double *>(bt->d_stage), x, s);
        if (st != FTS_OK) return st;
    }
    return FTS_OK;
}

size_t fts_batch_ws_bytes(const fts_batch *bt) { return bt ? (size_t)bt->ndofs_total * sizeof(double) : 0; }

fts_status fts_batch_smooth(fts_batch *bt, double omega, fts_prec prec, const double *b, double *x, int32_t nsweeps,
                            void *ws, size_t ws_bytes, void *stream) {
    if (!bt || !b || !x || !ws) return fail(FTS_E_INVAL, "fts_batch_smooth: NULL argument");
    if (ws_bytes < fts_batch_ws_bytes(bt)) return fail(FTS_E_SIZE, "fts_batch_smooth: workspace too small");
    double *r = static_cast<double *>(ws);
    for (int i = 0; i < nsweeps; ++i) {
        fts_status st = fts_batch_residual(bt, b, x, r, stream);
        if (st == FTS_OK) st = fts_batch_apply(bt, omega, prec, r, x, stream);
        if (st != FTS_OK) return st;
    }
    return FTS_OK;
}

fts_status fts_batch_set_launch(fts_batch *bt, int32_t threads, int32_t grid, int32_t chunk) {
    if (!bt || (threads != 256 && threads != 512) || grid < 1 || chunk < 1)
        return fail(FTS_E_INVAL, "fts_batch_set_launch: invalid launch shape");
    bt->threads = threads;
    bt->grid = grid;
    bt->chunk = chunk;
    return FTS_OK;
}

fts_status fts_batch_get_launch(const fts_batch *bt, int32_t *threads, int32_t *grid, int32_t *chunk) {
    if (!bt) return fail(FTS_E_INVAL, "fts_batch_get_launch: NULL handle");
    if (threads) *threads = bt->threads;
    if (grid) *grid = bt->grid;
    if (chunk) *chunk = bt->chunk;
    return FTS_OK;
}

fts_status fts_batch_autotune(fts_batch *bt, fts_prec prec, const double *r, void *stream, char *report,
                              size_t report_len) {
    if (!bt || !r) return fail(FTS_E_INVAL, "fts_batch_autotune: NULL argument");
    if (prec != FTS_PREC_F64 && prec != FTS_PREC_F32)
        return fail(FTS_E_UNSUPPORTED, "batched smoothing supports FP64 and FP32 contractions");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    FTS_HIP_CHECK(hipEventCreate(&e0));
    FTS_HIP_CHECK(hipEventCreate(&e1));
    std::string rep;
    float best = 1e30f;
    int bt_th = bt->threads, bt_gr = bt->grid, bt_ch = bt->chunk;
    fts_status st = FTS_OK;
    for (int th : {256, 512}) {
        for (int mult : {1, 2, 4, 8}) {
            for (int ch : {1, 4, 16}) {
                const int grid = mult * bt->ncu;
                st = batch_launch_smooth(bt, th, grid, ch, prec, r, 0.1, s);  // warm-up
                if (st != FTS_OK) break;
                if (hipEventRecord(e0, s) != hipSuccess) st = fail(FTS_E_HIP, "autotune timing failed");
                for (int rep_i = 0; rep_i < 2 && st == FTS_OK; ++rep_i)
                    st = batch_launch_smooth(bt, th, grid, ch, prec, r, 0.1, s);
                float ms = 0.f;
                if (st == FTS_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                     hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    st = fail(FTS_E_HIP, "autotune timing failed");
                if (st != FTS_OK) break;
                ms *= 0.5f;
                char line[128];
                std::snprintf(line, sizeof line, "threads=%d grid=%d chunk=%d: %.3f ms\n", th, grid, ch, ms);
                rep += line;
                if (ms < best) {
                    best = ms;
                    bt_th = th;
                    bt_gr = grid;
                    bt_ch = ch;
                }
            }
            if (st != FTS_OK) break;
        }
        if (st != FTS_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FTS_OK) return st;
    bt->threads = bt_th;
    bt->grid = bt_gr;
    bt->chunk = bt_ch;
    char line[160];
    std::snprintf(line, sizeof line, "chosen: threads=%d grid=%d chunk=%d (%.3f ms)\n", bt_th, bt_gr, bt_ch, best);
    rep += line;
    if (report && report_len) {
        std::strncpy(report, rep.c_str(), report_len - 1);
        report[report_len - 1] = '\0';
    }
    return FTS_OK;
}

}  // extern "C"
