// Allocation-free variant of the additive Schwarz smoother
// (fts_schwarz_smooth_noalloc): the residual workspace that fts_schwarz_smooth
// takes as an argument lives in a file-scope device array instead, so that the
// call allocates nothing.
#include <mutex>

#include "fts_internal.h"

using namespace fts;

namespace {

// Residual workspace of the allocation-free smoother: one FP64 vector of up to
// FTS_NOALLOC_SCRATCH_BYTES / 8 entries.  Each device the library runs on holds
// its own copy until the process ends.
static __device__ __align__(256) double scratch[FTS_NOALLOC_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of this device's copy of `scratch`, looked up once per
// device (with that device current) and kept.
fts_status scratch_ptr(double **out) {
    int dev = -1;
    FTS_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FTS_E_UNSUPPORTED, "fts_schwarz_smooth_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        FTS_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(FTS_E_HIP, "fts_schwarz_smooth_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return FTS_OK;
}

}  // namespace

extern "C" {

fts_status fts_schwarz_smooth_noalloc(const fts_level *level, const fts_eigs *eigs, double omega, fts_prec prec,
                                      const double *b, double *x, int32_t nsweeps, void *stream) {
    if (!level || !eigs || !b || !x) return fail(FTS_E_INVAL, "fts_schwarz_smooth_noalloc: NULL argument");
    if (eigs->level != level) return fail(FTS_E_INVAL, "fts_schwarz_smooth_noalloc: eigs belong to another level");
    if ((size_t)level->ndofs * sizeof(double) > (size_t)FTS_NOALLOC_SCRATCH_BYTES)
        return fail(FTS_E_SIZE, "fts_schwarz_smooth_noalloc: the level has " + std::to_string(level->ndofs) +
                                    " DoFs, more than the " + std::to_string(FTS_NOALLOC_SCRATCH_BYTES / 8) +
                                    " the static residual workspace holds");
    if (nsweeps < 0) return fail(FTS_E_INVAL, "fts_schwarz_smooth_noalloc: nsweeps < 0");
    double *r = nullptr;
    fts_status st = scratch_ptr(&r);
    if (st != FTS_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // r is written in full by the residual kernel before the local solves read
    // it (in FP64, or FP32 for the 16-bit owner tiles), so nothing carried
    // over from an earlier call is ever read
    for (int it = 0; it < nsweeps; ++it) {
        st = smooth_additive(level, eigs, omega, prec, b, x, r, false, s);
        if (st != FTS_OK) return st;
    }
    return FTS_OK;
}

}  // extern "C"
