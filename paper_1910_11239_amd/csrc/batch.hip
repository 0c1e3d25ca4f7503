// Batched additive vertex-patch smoothing of many independent 3-D meshes of
// mixed degree and anisotropic (rectilinear) cells: every patch has its own
// per-axis 1-D eigen-data (Sec. 3.2, eq. generalizedEVP), and all patches of
// all meshes are processed by one persistent launch.
//
// Work queue: the global patch index space lists the meshes in decreasing
// degree (largest local solves first); persistent workgroups take chunks of
// patches with a 64-bit atomic counter until the space is exhausted (every
// workgroup reaches the exit).  Per patch a switch on the mesh's degree runs
// the same fast-diagonalisation body as the single-mesh kernel (scalar-loaded
// 1-D tables, last axis fused in registers) and stages the correction; a
// batched gather adds the corrections of each cell in a fixed order.  The
// FP64 residual runs as one launch per degree present.
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
// lines per thread and pass of the contractions (measured: 2 beats 1, 3, 4, 6)
constexpr int kBatchLines = 2;

template <int N1, int TH, typename T>
__device__ __forceinline__ void batch_patch(const BatchMesh &M, int64_t p, const double *__restrict__ r,
                                            T *__restrict__ W, T om, T *Ts) {
    constexpr int D = 3, N = 2 * N1, NC1 = N1 * N1 * N1, NSC = 8, LINES = N * N, NN = N * N;
    constexpr int BL = kBatchLines;
    const int t = threadIdx.x;
    int pos[3];
    pos[0] = __builtin_amdgcn_readfirstlane((int)(p % M.cnt[0]));
    pos[1] = __builtin_amdgcn_readfirstlane((int)((p / M.cnt[0]) % M.cnt[1]));
    pos[2] = __builtin_amdgcn_readfirstlane((int)(p / ((int64_t)M.cnt[0] * M.cnt[1])));
    const int64_t cs1 = M.lv.m[0], cs2 = (int64_t)M.lv.m[0] * M.lv.m[1];
    const double *rm = r + M.dof_off;
    for (int q = t; q < NSC * NC1; q += TH) {
        const int sc = q / NC1, i = q % NC1;
        const int o0 = sc & 1, o1 = (sc >> 1) & 1, o2 = (sc >> 2) & 1;
        const int64_t cell = (pos[0] + o0) + (pos[1] + o1) * cs1 + (pos[2] + o2) * cs2;
        const int i0 = i % N1, i1 = (i / N1) % N1, i2 = i / (N1 * N1);
        Ts[(o0 * N1 + i0) + (o1 * N1 + i1) * N + (o2 * N1 + i2) * NN] = (T)rm[cell * NC1 + i];
    }
    __syncthreads();
    const EigView &e = M.ev;
    // BL lines per thread and pass (contract_lines): the 1-D matrices of the
    // larger degrees do not fit in scalar registers
    for (int l = t; l < LINES; l += BL * TH)
        contract_lines<D, N, BL, T>(Ts, 0, l, TH, LINES, uniform_table(EigTab<T>::ST(e, 0) + (size_t)pos[0] * NN));
    __syncthreads();
    for (int l = t; l < LINES; l += BL * TH)
        contract_lines<D, N, BL, T>(Ts, 1, l, TH, LINES, uniform_table(EigTab<T>::ST(e, 1) + (size_t)pos[1] * NN));
    __syncthreads();
    {
        cptr<T> L0 = uniform_table(EigTab<T>::L(e, 0) + (size_t)pos[0] * N);
        cptr<T> L1 = uniform_table(EigTab<T>::L(e, 1) + (size_t)pos[1] * N);
        cptr<T> ST2 = uniform_table(EigTab<T>::ST(e, 2) + (size_t)pos[2] * NN);
        cptr<T> S2 = uniform_table(EigTab<T>::S(e, 2) + (size_t)pos[2] * NN);
        cptr<T> L2 = uniform_table(EigTab<T>::L(e, 2) + (size_t)pos[2] * N);
        for (int l = t; l < LINES; l += BL * TH) {
            T lr[BL];
#pragma unroll
            for (int k = 0; k < BL; ++k) {
                const int lk = l + k * TH < LINES ? l + k * TH : l;
                lr[k] = (T)L0[lk % N] + (T)L1[lk / N];
            }
            last_axis_solves<D, N, BL, T>(Ts, l, TH, LINES, ST2, S2, L2, lr, om);
        }
    }
    __syncthreads();
    for (int l = t; l < LINES; l += BL * TH)
        contract_lines<D, N, BL, T>(Ts, 1, l, TH, LINES, uniform_table(EigTab<T>::S(e, 1) + (size_t)pos[1] * NN));
    __syncthreads();
    for (int l = t; l < LINES; l += BL * TH)
        contract_lines<D, N, BL, T>(Ts, 0, l, TH, LINES, uniform_table(EigTab<T>::S(e, 0) + (size_t)pos[0] * NN));
    __syncthreads();
    T *Wm = W + M.stage_off + p * (NSC * NC1);
    for (int q = t; q < NSC * NC1; q += TH) {
        const int sc = q / NC1, i = q % NC1;
        const int o0 = sc & 1, o1 = (sc >> 1) & 1, o2 = (sc >> 2) & 1;
        const int i0 = i % N1, i1 = (i / N1) % N1, i2 = i / (N1 * N1);
        Wm[q] = Ts[(o0 * N1 + i0) + (o1 * N1 + i1) * N + (o2 * N1 + i2) * NN];
    }
    __syncthreads();  // Ts is reused by the next patch
}

template <int TH, typename T>
__global__ void __launch_bounds__(TH)
k_batch_smooth(const BatchMesh *__restrict__ meshes, const int64_t *__restrict__ prefix,
               const int *__restrict__ order, int nslot, int64_t total, int chunk,
               unsigned long long *__restrict__ counter, const double *__restrict__ r, T *__restrict__ W,
               double omega) {
    __shared__ T Ts[kBatchMaxN * kBatchMaxN * kBatchMaxN];
    __shared__ unsigned long long start_s;
    const T om = (T)omega;
    for (;;) {
        if (threadIdx.x == 0) start_s = atomicAdd(counter, (unsigned long long)chunk);
        __syncthreads();
        const int64_t start = (int64_t)start_s;
        __syncthreads();
        if (start >= total) break;
        const int64_t end = start + chunk < total ? start + chunk : total;
        int lo = 0, hi = nslot;  // prefix[lo] <= start < prefix[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (prefix[mid] <= start) lo = mid;
            else hi = mid;
        }
        int slot = lo;
        for (int64_t gidx = start; gidx < end; ++gidx) {
            while (gidx >= prefix[slot + 1]) ++slot;
            const int mi = __builtin_amdgcn_readfirstlane(order[slot]);
            const BatchMesh &M = meshes[mi];
            const int64_t p = gidx - prefix[slot];
            switch (M.n1) {
                case 2: batch_patch<2, TH, T>(M, p, r, W, om, Ts); break;
                case 3: batch_patch<3, TH, T>(M, p, r, W, om, Ts); break;
                case 4: batch_patch<4, TH, T>(M, p, r, W, om, Ts); break;
                case 5: batch_patch<5, TH, T>(M, p, r, W, om, Ts); break;
                case 6: batch_patch<6, TH, T>(M, p, r, W, om, Ts); break;
                case 7: batch_patch<7, TH, T>(M, p, r, W, om, Ts); break;
                case 8: batch_patch<8, TH, T>(M, p, r, W, om, Ts); break;
                case 9: batch_patch<9, TH, T>(M, p, r, W, om, Ts); break;
                case 10: batch_patch<10, TH, T>(M, p, r, W, om, Ts); break;
                default: break;
            }
        }
    }
}

__global__ void k_batch_reset(unsigned long long *counter) { *counter = 0ull; }

// x += the staged corrections (FP64 or FP32, the contraction type) of the
// 8 patches around each cell, in FP64 and in a fixed order.
template <typename WT>
__global__ void __launch_bounds__(256)
k_batch_gather(const BatchMesh *__restrict__ meshes, const BatchBlock *__restrict__ blocks,
               const WT *__restrict__ W, double *__restrict__ x) {
    const BatchBlock B = blocks[blockIdx.x];
    const BatchMesh &M = meshes[B.mesh];
    const int n1 = M.n1, NC1 = n1 * n1 * n1;
    const int64_t nd = M.lv.ncells * NC1;
    const int64_t gid = B.first + threadIdx.x;
    if (gid >= nd) return;
    const int64_t cell = gid / NC1;
    const int i = (int)(gid % NC1);
    int c[3];
    cell_coords(cell, M.lv.m, c);
    double acc = 0.0;
    for (int o = 0; o < 8; ++o) {
        const int a0 = c[0] - (o & 1), a1 = c[1] - ((o >> 1) & 1), a2 = c[2] - ((o >> 2) & 1);
        if (a0 >= 0 && a0 < M.cnt[0] && a1 >= 0 && a1 < M.cnt[1] && a2 >= 0 && a2 < M.cnt[2]) {
            const int64_t sidx = a0 + (int64_t)M.cnt[0] * (a1 + (int64_t)M.cnt[1] * a2);
            acc += (double)W[M.stage_off + sidx * (8 * NC1) + o * NC1 + i];
        }
    }
    x[M.dof_off + gid] += acc;
}

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
    BatchBlock *d_gather = nullptr;
    int64_t ngather = 0;
    int threads = 256, grid = 0, chunk = 4;  // launch shape (autotuned)
    int ncu = 256;
};

static fts_status batch_launch_smooth(fts_batch *bt, int threads, int grid, int chunk, fts_prec prec,
                                      const double *r, double omega, hipStream_t s) {
    k_batch_reset<<<1, 1, 0, s>>>(bt->d_counter);
    const bool f32 = prec == FTS_PREC_F32;
#define FTS_BATCH_LAUNCH(TH)                                                                                  \
    if (f32)                                                                                                 \
        k_batch_smooth<TH, float><<<grid, TH, 0, s>>>(bt->d_meshes, bt->d_prefix, bt->d_order, bt->nslot,   \
                                                      bt->patches_total, chunk, bt->d_counter, r,           \
                                                      reinterpret_cast<float *>(bt->d_stage), omega);        \
    else                                                                                                     \
        k_batch_smooth<TH, double><<<grid, TH, 0, s>>>(bt->d_meshes, bt->d_prefix, bt->d_order, bt->nslot,  \
                                                       bt->patches_total, chunk, bt->d_counter, r,           \
                                                       bt->d_stage, omega);
    if (threads == 64) {
        FTS_BATCH_LAUNCH(64)
    } else if (threads == 128) {
        FTS_BATCH_LAUNCH(128)
    } else if (threads == 256) {
        FTS_BATCH_LAUNCH(256)
    } else {
        return fail(FTS_E_INVAL, "batch: threads must be 64, 128 or 256");
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
    if (bt->d_gather) dev_free(bt->d_gather);
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
    // residual blocks per degree, gather blocks
    std::vector<BatchBlock> gblocks;
    for (int n1 = 2; n1 <= kMaxN1 && st == FTS_OK; ++n1) {
        std::vector<BatchBlock> blocks;
        for (int i = 0; i < nmesh; ++i) {
            if (host[i].n1 != n1) continue;
            const int cpw = operator_cells_per_block(3, n1);
            for (int64_t c = 0; c < bt->levels[i]->ncells; c += cpw) blocks.push_back({i, 0, c});
        }
        if (blocks.empty()) continue;
        fts_batch::Group g{n1, nullptr, (int64_t)blocks.size()};
        if (dev_malloc(&g.blocks, blocks.size() * sizeof(BatchBlock)) != hipSuccess ||
            hipMemcpy(g.blocks, blocks.data(), blocks.size() * sizeof(BatchBlock), hipMemcpyHostToDevice) != hipSuccess)
            st = fail(FTS_E_HIP, "batch: upload of residual blocks failed");
        bt->res_groups.push_back(g);
    }
    for (int i = 0; i < nmesh; ++i)
        for (int64_t d = 0; d < bt->ndofs[i]; d += 256) gblocks.push_back({i, 0, d});
    bt->ngather = (int64_t)gblocks.size();
    auto up = [&](void **dst, const void *src, size_t bytes) {
        if (st != FTS_OK) return;
        if (dev_malloc(dst, std::max<size_t>(bytes, 8)) != hipSuccess ||
            (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess))
            st = fail(FTS_E_HIP, "batch: upload failed");
    };
    up((void **)&bt->d_meshes, host.data(), host.size() * sizeof(BatchMesh));
    up((void **)&bt->d_prefix, prefix.data(), prefix.size() * sizeof(int64_t));
    up((void **)&bt->d_order, order.data(), order.size() * sizeof(int));
    up((void **)&bt->d_gather, gblocks.data(), gblocks.size() * sizeof(BatchBlock));
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
    if (prec == FTS_PREC_F32)
        k_batch_gather<float><<<dim3((unsigned)bt->ngather), dim3(256), 0, s>>>(
            bt->d_meshes, bt->d_gather, reinterpret_cast<const float *>(bt->d_stage), x);
    else
        k_batch_gather<double><<<dim3((unsigned)bt->ngather), dim3(256), 0, s>>>(bt->d_meshes, bt->d_gather,
                                                                                 bt->d_stage, x);
    return check_launch("k_batch_gather");
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
    if (!bt || (threads != 64 && threads != 128 && threads != 256) || grid < 1 || chunk < 1)
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
    for (int th : {64, 128, 256}) {
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
