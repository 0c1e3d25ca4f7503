// C entry points for the hot calls and the multigrid hierarchy (Alg. gmg).
#include <algorithm>
#include <cmath>

#include "fts_internal.h"

using namespace fts;

struct fts_hierarchy {
    int nlevels = 0;
    int kind = 0;
    int m_pre = 1, m_post = 1;
    std::vector<double> omega;
    std::vector<fts_level *> levels;  // 0 = coarsest
    std::vector<fts_eigs *> eigs;     // eigs[0] = nullptr
    std::vector<double *> vb, vx, vr;  // per-level vectors (b, x for l < L; r for every l)
    CoarseLU *coarse = nullptr;  // direct solver of A_0 (coarse.hip)
    int smoother = FTS_SMOOTHER_ADDITIVE;
    int64_t N0 = 0;
    double *host_scalars = nullptr;       // pinned readback buffer of the CG reductions
    // adjoint workspaces (fts_hierarchy_enable_adjoint)
    bool adj = false;
    std::vector<std::vector<double *>> xs;  // per level: inputs of every smoothing step and the output
    std::vector<double *> lam, lamb, aq, atr, at;
    double *apart = nullptr, *ared = nullptr, *agrad = nullptr;
    double *host_grad = nullptr;
};

static hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" {

fts_status fts_apply_operator(const fts_level *level, const double *x, double *y, void *stream) {
    if (!level || !x || !y) return fail(FTS_E_INVAL, "fts_apply_operator: NULL argument");
    return launch_operator(level, x, nullptr, y, false, S(stream));
}

fts_status fts_residual(const fts_level *level, const double *b, const double *x, double *r, void *stream) {
    if (!level || !b || !x || !r) return fail(FTS_E_INVAL, "fts_residual: NULL argument");
    if (r == x) return fail(FTS_E_INVAL, "fts_residual: r must not alias x");
    return launch_operator(level, x, b, r, true, S(stream));
}

size_t fts_smooth_ws_bytes(const fts_level *level) { return level ? (size_t)level->ndofs * sizeof(double) : 0; }

fts_status fts_schwarz_apply(const fts_level *level, const fts_eigs *eigs, double omega, fts_prec prec,
                             const double *r, double *x, void *stream) {
    if (!level || !eigs || !r || !x) return fail(FTS_E_INVAL, "fts_schwarz_apply: NULL argument");
    if (eigs->level != level) return fail(FTS_E_INVAL, "fts_schwarz_apply: eigs belong to another level");
    return launch_schwarz(level, eigs, omega, prec, r, x, S(stream));
}

fts_status fts_schwarz_smooth(const fts_level *level, const fts_eigs *eigs, double omega, fts_prec prec,
                              const double *b, double *x, int32_t nsweeps, void *ws, size_t ws_bytes,
                              void *stream) {
    if (!level || !eigs || !b || !x || !ws) return fail(FTS_E_INVAL, "fts_schwarz_smooth: NULL argument");
    if (eigs->level != level) return fail(FTS_E_INVAL, "fts_schwarz_smooth: eigs belong to another level");
    if (ws_bytes < fts_smooth_ws_bytes(level)) return fail(FTS_E_SIZE, "fts_schwarz_smooth: workspace too small");
    for (int it = 0; it < nsweeps; ++it) {
        const fts_status st = smooth_additive(level, eigs, omega, prec, b, x, ws, false, S(stream));
        if (st != FTS_OK) return st;
    }
    return FTS_OK;
}

fts_status fts_schwarz_smooth_mult(const fts_level *level, const fts_eigs *eigs, double omega, fts_prec prec,
                                   const double *b, double *x, int32_t nsweeps, void *ws, size_t ws_bytes,
                                   void *stream) {
    if (!level || !eigs || !b || !x || !ws) return fail(FTS_E_INVAL, "fts_schwarz_smooth_mult: NULL argument");
    if (eigs->level != level) return fail(FTS_E_INVAL, "fts_schwarz_smooth_mult: eigs belong to another level");
    if (ws_bytes < fts_smooth_ws_bytes(level))
        return fail(FTS_E_SIZE, "fts_schwarz_smooth_mult: workspace too small");
    double *r = static_cast<double *>(ws);
    const int nc = schwarz_mult_colors(eigs);
    for (int it = 0; it < nsweeps; ++it)
        for (int c = 0; c < nc; ++c) {
            fts_status st = launch_operator(level, x, b, r, true, S(stream));
            if (st != FTS_OK) return st;
            st = launch_schwarz_color(level, eigs, omega, prec, r, x, c, S(stream));
            if (st != FTS_OK) return st;
        }
    return FTS_OK;
}

static fts_status check_pair(const fts_level *c, const fts_level *f) {
    if (!c || !f) return fail(FTS_E_INVAL, "transfer: NULL level");
    if (c->dim != f->dim || c->k != f->k) return fail(FTS_E_INVAL, "transfer: levels differ in dim or degree");
    for (int a = 0; a < c->dim; ++a) {
        if (f->m[a] != 2 * c->m[a]) return fail(FTS_E_INVAL, "transfer: fine level is not the refinement");
        for (int i = 0; i < c->m[a]; ++i) {
            const double w = f->h[a][2 * i] + f->h[a][2 * i + 1];
            if (std::fabs(w - c->h[a][i]) > 1e-12 * c->h[a][i] ||
                std::fabs(f->h[a][2 * i] - f->h[a][2 * i + 1]) > 1e-12 * c->h[a][i])
                return fail(FTS_E_INVAL, "transfer: children must be equal halves of the parent");
        }
    }
    return FTS_OK;
}

fts_status fts_restrict(const fts_level *coarse, const fts_level *fine, const double *rf, double *bc,
                        void *stream) {
    fts_status st = check_pair(coarse, fine);
    if (st != FTS_OK) return st;
    if (!rf || !bc) return fail(FTS_E_INVAL, "fts_restrict: NULL vector");
    return launch_restrict(coarse, fine, rf, bc, S(stream));
}

fts_status fts_prolongate_add(const fts_level *coarse, const fts_level *fine, const double *ec, double *xf,
                              void *stream) {
    fts_status st = check_pair(coarse, fine);
    if (st != FTS_OK) return st;
    if (!ec || !xf) return fail(FTS_E_INVAL, "fts_prolongate_add: NULL vector");
    return launch_prolongate(coarse, fine, ec, xf, S(stream));
}

fts_status fts_hierarchy_destroy(fts_hierarchy *h) {
    if (!h) return FTS_OK;
    for (auto *e : h->eigs) fts_eigs_destroy(e);
    for (auto *l : h->levels) fts_level_destroy(l);
    for (auto *p : h->vb) if (p) dev_free(p);
    for (auto *p : h->vx) if (p) dev_free(p);
    for (auto *p : h->vr) if (p) dev_free(p);
    coarse_destroy(h->coarse);
    if (h->host_scalars) (void)hipHostFree(h->host_scalars);
    for (auto &v : h->xs)
        for (auto *p : v) if (p) dev_free(p);
    for (auto *vv : {&h->lam, &h->lamb, &h->aq, &h->atr, &h->at})
        for (auto *p : *vv) if (p) dev_free(p);
    if (h->apart) dev_free(h->apart);
    if (h->ared) dev_free(h->ared);
    if (h->agrad) dev_free(h->agrad);
    if (h->host_grad) (void)hipHostFree(h->host_grad);
    delete h;
    return FTS_OK;
}

fts_status fts_hierarchy_create(const fts_mesh_desc *finest, int32_t nlevels, fts_patch_kind kind,
                                const double *omega_per_level, const double *penalty_per_level, int32_t m_pre,
                                int32_t m_post, fts_hierarchy **out) {
    if (!finest || !out || !omega_per_level) return fail(FTS_E_INVAL, "fts_hierarchy_create: NULL argument");
    *out = nullptr;
    if (nlevels < 1 || nlevels > 16) return fail(FTS_E_INVAL, "nlevels must be in 1..16");
    if (m_pre < 0 || m_post < 0) return fail(FTS_E_INVAL, "negative smoothing step count");
    if (finest->dim != 2 && finest->dim != 3) return fail(FTS_E_UNSUPPORTED, "dim must be 2 or 3");
    fts_hierarchy *h = new fts_hierarchy();
    h->nlevels = nlevels;
    h->kind = kind;
    h->m_pre = m_pre;
    h->m_post = m_post;
    h->omega.assign(omega_per_level, omega_per_level + nlevels);
    // widths of every level, finest last
    std::vector<std::vector<double>> w[3];
    for (int a = 0; a < finest->dim; ++a) {
        if (!finest->h[a] || finest->ncells[a] < 1) {
            delete h;
            return fail(FTS_E_INVAL, "invalid finest mesh");
        }
        w[a].assign(nlevels, {});
        w[a][nlevels - 1].assign(finest->h[a], finest->h[a] + finest->ncells[a]);
        for (int l = nlevels - 2; l >= 0; --l) {
            const auto &f = w[a][l + 1];
            if (f.size() % 2) {
                delete h;
                return fail(FTS_E_INVAL, "cannot coarsen an odd number of cells");
            }
            for (size_t i = 0; i < f.size(); i += 2) {
                if (std::fabs(f[i] - f[i + 1]) > 1e-12 * f[i]) {
                    delete h;
                    return fail(FTS_E_INVAL, "children of a coarse cell must be equal halves");
                }
                w[a][l].push_back(f[i] + f[i + 1]);
            }
        }
    }
    fts_status st = FTS_OK;
    for (int l = 0; l < nlevels && st == FTS_OK; ++l) {
        fts_mesh_desc d = *finest;
        for (int a = 0; a < finest->dim; ++a) {
            d.ncells[a] = (int32_t)w[a][l].size();
            d.h[a] = w[a][l].data();
        }
        d.penalty_factor = penalty_per_level ? penalty_per_level[l] : finest->penalty_factor;
        fts_level *lv = nullptr;
        st = fts_level_create(&d, &lv);
        if (st != FTS_OK) break;
        h->levels.push_back(lv);
        fts_eigs *eg = nullptr;
        if (l > 0) {
            st = fts_setup_1d_eigs(lv, kind, &eg);
            if (st != FTS_OK) break;
        }
        h->eigs.push_back(eg);
        double *pb = nullptr, *px = nullptr, *pr = nullptr;
        const size_t bytes = (size_t)lv->ndofs * sizeof(double);
        if (l < nlevels - 1 && (dev_malloc(&pb, bytes) != hipSuccess || dev_malloc(&px, bytes) != hipSuccess))
            st = fail(FTS_E_HIP, "device allocation of level vectors failed");
        if (st == FTS_OK && dev_malloc(&pr, bytes) != hipSuccess) st = fail(FTS_E_HIP, "device allocation of level vectors failed");
        h->vb.push_back(pb);
        h->vx.push_back(px);
        h->vr.push_back(pr);
    }
    if (st == FTS_OK) {
        const fts_level *l0 = h->levels[0];
        const int64_t N = l0->ndofs;
        h->N0 = N;
        st = coarse_create(l0, nullptr, &h->coarse);
        if (st == FTS_OK && hipHostMalloc(&h->host_scalars, 4 * sizeof(double)) != hipSuccess)
            st = fail(FTS_E_HIP, "hipHostMalloc of the readback buffer failed");
    }
    if (st != FTS_OK) {
        fts_hierarchy_destroy(h);
        return st;
    }
    *out = h;
    return FTS_OK;
}

const fts_level *fts_hierarchy_level(const fts_hierarchy *h, int32_t l) {
    return (h && l >= 0 && l < h->nlevels) ? h->levels[l] : nullptr;
}
const fts_eigs *fts_hierarchy_eigs(const fts_hierarchy *h, int32_t l) {
    return (h && l >= 0 && l < h->nlevels) ? h->eigs[l] : nullptr;
}

fts_status fts_coarse_solve(fts_hierarchy *h, const double *b0, double *x0, void *stream) {
    if (!h || !b0 || !x0) return fail(FTS_E_INVAL, "fts_coarse_solve: NULL argument");
    return coarse_solve(h->coarse, b0, x0, S(stream));
}

// One smoothing step x <- S(x, b) on level l: Alg. addsmoother (one
// residual, all local solves) or Alg. multsmoother (a residual before each
// color; with FTS_SMOOTHER_MULTIPLICATIVE_SYMMETRIC the colors of a
// post-smoothing step (post = true) run in reverse order).  x_zero: x is
// known to be zero on entry, so the first residual is b itself (A 0 = 0) and
// is not computed.
static fts_status smooth_step(fts_hierarchy *h, int l, fts_prec prec, const double *b, double *x, hipStream_t s,
                              bool x_zero = false, bool post = false) {
    const fts_level *lv = h->levels[l];
    const fts_eigs *eg = h->eigs[l];
    double *r = h->vr[l];
    fts_status st = FTS_OK;
    if (h->smoother != FTS_SMOOTHER_ADDITIVE) {
        const int nc = schwarz_mult_colors(eg);
        const bool reverse = post && h->smoother == FTS_SMOOTHER_MULTIPLICATIVE_SYMMETRIC;
        for (int i = 0; i < nc && st == FTS_OK; ++i) {
            const int c = reverse ? nc - 1 - i : i;
            const bool first = x_zero && i == 0;
            if (!first) st = launch_operator(lv, x, b, r, true, s);
            if (st == FTS_OK) st = launch_schwarz_color(lv, eg, h->omega[l], prec, first ? b : r, x, c, s);
        }
        return st;
    }
    return smooth_additive(lv, eg, h->omega[l], prec, b, x, r, x_zero, s);
}

// x <- MG_l(x, b) (Alg. gmg).  x_zero: x is zero on entry (the coarser
// levels of a V-cycle, and the preconditioner calls of PCG and GMRES).
static fts_status vcycle_level(fts_hierarchy *h, int l, fts_prec prec, const double *b, double *x, hipStream_t s,
                               bool x_zero = false) {
    if (l == 0) return coarse_solve(h->coarse, b, x, s);
    const fts_level *lv = h->levels[l];
    double *r = h->vr[l];
    fts_status st = FTS_OK;
    for (int i = 0; i < h->m_pre && st == FTS_OK; ++i) st = smooth_step(h, l, prec, b, x, s, x_zero && i == 0);
    if (st == FTS_OK) st = launch_operator(lv, x, b, r, true, s);
    if (st == FTS_OK) st = launch_restrict(h->levels[l - 1], lv, r, h->vb[l - 1], s);
    if (st == FTS_OK && l - 1 > 0) st = launch_fill(h->vx[l - 1], h->levels[l - 1]->ndofs, 0.0, s);
    if (st == FTS_OK) st = vcycle_level(h, l - 1, prec, h->vb[l - 1], h->vx[l - 1], s, true);
    if (st == FTS_OK) st = launch_prolongate(h->levels[l - 1], lv, h->vx[l - 1], x, s);
    for (int i = 0; i < h->m_post && st == FTS_OK; ++i) st = smooth_step(h, l, prec, b, x, s, false, true);
    return st;
}

size_t fts_pcg_ws_bytes(const fts_hierarchy *h) {
    if (!h) return 0;
    return (size_t)(5 * h->levels.back()->ndofs + 2 * red_partials() + 2) * sizeof(double);
}

static fts_status readback(fts_hierarchy *h, const double *dev, hipStream_t s, double *out2) {
    FTS_HIP_CHECK(hipMemcpyAsync(h->host_scalars, dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    FTS_HIP_CHECK(hipStreamSynchronize(s));
    out2[0] = h->host_scalars[0];
    out2[1] = h->host_scalars[1];
    return FTS_OK;
}

fts_status fts_pcg(fts_hierarchy *h, fts_prec prec, const double *b, double *x, double rtol, int32_t maxit,
                   void *ws, size_t ws_bytes, int32_t *iters, double *relres, double *history, void *stream) {
    if (!h || !b || !x || !ws) return fail(FTS_E_INVAL, "fts_pcg: NULL argument");
    if (ws_bytes < fts_pcg_ws_bytes(h)) return fail(FTS_E_SIZE, "fts_pcg: workspace too small");
    if (!(rtol >= 0.0) || maxit < 0) return fail(FTS_E_INVAL, "fts_pcg: invalid rtol or maxit");
    hipStream_t s = S(stream);
    const fts_level *lv = h->levels.back();
    const int64_t N = lv->ndofs;
    double *r = static_cast<double *>(ws), *z = r + N, *zo = z + N, *p = zo + N, *q = p + N;
    double *part = q + N, *dout = part + 2 * red_partials();
    double v[2];
    fts_status st;
#define FTS_TRY(expr)        \
    do {                     \
        st = (expr);         \
        if (st != FTS_OK) return st; \
    } while (0)
    FTS_TRY(launch_operator(lv, x, b, r, true, s));
    FTS_TRY(launch_dot2(b, b, nullptr, N, part, dout, s));
    FTS_TRY(readback(h, dout, s, v));
    const double bb = v[0];
    FTS_TRY(launch_dot2(r, r, nullptr, N, part, dout, s));
    FTS_TRY(readback(h, dout, s, v));
    double rel = bb > 0.0 ? std::sqrt(v[0] / bb) : 0.0;
    if (history) history[0] = rel;
    int it = 0;
    if (rel > rtol && maxit > 0) {
        FTS_TRY(launch_fill(z, N, 0.0, s));
        FTS_TRY(vcycle_level(h, h->nlevels - 1, prec, r, z, s, true));
        FTS_HIP_CHECK(hipMemcpyAsync(p, z, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        FTS_TRY(launch_dot2(r, z, nullptr, N, part, dout, s));
        FTS_TRY(readback(h, dout, s, v));
        double rz = v[0];
        while (it < maxit) {
            FTS_TRY(launch_operator(lv, p, nullptr, q, false, s));
            FTS_TRY(launch_dot2(p, q, nullptr, N, part, dout, s));
            FTS_TRY(readback(h, dout, s, v));
            const double alpha = rz / v[0];
            FTS_TRY(launch_cg_update(x, r, p, q, alpha, N, s));
            FTS_TRY(launch_dot2(r, r, nullptr, N, part, dout, s));
            FTS_TRY(readback(h, dout, s, v));
            rel = std::sqrt(v[0] / bb);
            ++it;
            if (history) history[it] = rel;
            if (!(rel > rtol)) break;
            std::swap(z, zo);
            FTS_TRY(launch_fill(z, N, 0.0, s));
            FTS_TRY(vcycle_level(h, h->nlevels - 1, prec, r, z, s, true));
            FTS_TRY(launch_dot2(r, z, zo, N, part, dout, s));
            FTS_TRY(readback(h, dout, s, v));
            // flexible (Polak-Ribiere) update: beta = r.(z - z_old) / rz_old
            const double beta = (v[0] - v[1]) / rz;
            rz = v[0];
            FTS_TRY(launch_xpby(p, z, beta, N, s));
        }
    }
#undef FTS_TRY

    if (iters) *iters = it;
    if (relres) *relres = rel;
    return FTS_OK;
}

size_t fts_gmres_ws_bytes(const fts_hierarchy *h, int32_t restart) {
    if (!h || restart < 1) return 0;
    return (size_t)((2 * (int64_t)restart + 2) * h->levels.back()->ndofs + 2 * red_partials() + 2) * sizeof(double);
}

fts_status fts_gmres(fts_hierarchy *h, fts_prec prec, const double *b, double *x, double rtol, int32_t restart,
                     int32_t maxit, void *ws, size_t ws_bytes, int32_t *iters, double *relres, double *history,
                     void *stream) {
    if (!h || !b || !x || !ws) return fail(FTS_E_INVAL, "fts_gmres: NULL argument");
    if (restart < 1 || maxit < 0) return fail(FTS_E_INVAL, "fts_gmres: restart >= 1 and maxit >= 0 required");
    if (ws_bytes < fts_gmres_ws_bytes(h, restart)) return fail(FTS_E_SIZE, "fts_gmres: workspace too small");
    hipStream_t s = S(stream);
    const int L = h->nlevels - 1;
    const fts_level *lv = h->levels[L];
    const int64_t N = lv->ndofs;
    const int m = restart;
    double *V = static_cast<double *>(ws);  // m + 1 vectors
    double *Z = V + (int64_t)(m + 1) * N;   // m vectors
    double *w = Z + (int64_t)m * N;
    double *part = w + N, *dout = part + 2 * red_partials();
    double v2[2];
    fts_status st;
#define GM_TRY(expr)                   \
    do {                               \
        st = (expr);                   \
        if (st != FTS_OK) return st;   \
    } while (0)
    auto dot = [&](const double *a, const double *c, double *out) -> fts_status {
        fts_status e = launch_dot2(a, c, nullptr, N, part, dout, s);
        if (e != FTS_OK) return e;
        e = readback(h, dout, s, v2);
        *out = v2[0];
        return e;
    };
    double bb, rr;
    GM_TRY(dot(b, b, &bb));
    const double nb = std::sqrt(bb) > 0.0 ? std::sqrt(bb) : 1.0;
    GM_TRY(launch_operator(lv, x, b, V, true, s));  // r = b - A x in V_0
    GM_TRY(dot(V, V, &rr));
    double beta = std::sqrt(rr);
    double rel = beta / nb;
    if (history) history[0] = rel;
    int it = 0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto Hij = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };
    while (rel > rtol && it < maxit && beta > 0.0) {
        GM_TRY(launch_scale(V, 1.0 / beta, N, s));  // v_1 = r / |r|
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            double *Vj = V + (int64_t)j * N, *Zj = Z + (int64_t)j * N;
            GM_TRY(launch_fill(Zj, N, 0.0, s));
            GM_TRY(vcycle_level(h, L, prec, Vj, Zj, s, true));  // z_j = MG(0, v_j)
            GM_TRY(launch_operator(lv, Zj, nullptr, w, false, s));
            for (int i = 0; i <= j; ++i) {  // modified Gram-Schmidt
                double hij;
                GM_TRY(dot(w, V + (int64_t)i * N, &hij));
                Hij(i, j) = hij;
                GM_TRY(launch_axpy(-hij, V + (int64_t)i * N, w, N, s));
            }
            double ww;
            GM_TRY(dot(w, w, &ww));
            const double hn = std::sqrt(ww);
            // Givens rotations: triangularise column j, residual = |g[j+1]|
            for (int i = 0; i < j; ++i) {
                const double t0 = Hij(i, j), t1 = Hij(i + 1, j);
                Hij(i, j) = cs[i] * t0 + sn[i] * t1;
                Hij(i + 1, j) = -sn[i] * t0 + cs[i] * t1;
            }
            const double a = Hij(j, j), r2 = std::hypot(a, hn);
            cs[j] = r2 > 0.0 ? a / r2 : 1.0;
            sn[j] = r2 > 0.0 ? hn / r2 : 0.0;
            Hij(j, j) = r2;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            ++it;
            rel = std::fabs(g[j + 1]) / nb;
            if (history) history[it] = rel;
            if (rel <= rtol || it >= maxit || hn == 0.0) break;
            double *Vn = V + (int64_t)(j + 1) * N;
            GM_TRY(launch_fill(Vn, N, 0.0, s));
            GM_TRY(launch_axpy(1.0 / hn, w, Vn, N, s));
        }
        for (int i = k - 1; i >= 0; --i) {  // R y = g
            double t = g[i];
            for (int c = i + 1; c < k; ++c) t -= Hij(i, c) * y[c];
            y[i] = t / Hij(i, i);
        }
        for (int i = 0; i < k; ++i) GM_TRY(launch_axpy(y[i], Z + (int64_t)i * N, x, N, s));
        GM_TRY(launch_operator(lv, x, b, V, true, s));
        GM_TRY(dot(V, V, &rr));
        beta = std::sqrt(rr);
        rel = beta / nb;
        if (history) history[it] = rel;
    }
#undef GM_TRY
    if (iters) *iters = it;
    if (relres) *relres = rel;
    return FTS_OK;
}

fts_status fts_hierarchy_set_smoother(fts_hierarchy *h, int32_t smoother) {
    if (!h) return fail(FTS_E_INVAL, "fts_hierarchy_set_smoother: NULL handle");
    if (smoother != FTS_SMOOTHER_ADDITIVE && smoother != FTS_SMOOTHER_MULTIPLICATIVE &&
        smoother != FTS_SMOOTHER_MULTIPLICATIVE_SYMMETRIC)
        return fail(FTS_E_INVAL, "fts_hierarchy_set_smoother: unknown smoother");
    h->smoother = smoother;
    return FTS_OK;
}

fts_status fts_hierarchy_set_omega(fts_hierarchy *h, const double *omega_per_level) {
    if (!h || !omega_per_level) return fail(FTS_E_INVAL, "fts_hierarchy_set_omega: NULL argument");
    h->omega.assign(omega_per_level, omega_per_level + h->nlevels);
    return FTS_OK;
}

fts_status fts_hierarchy_enable_adjoint(fts_hierarchy *h) {
    if (!h) return fail(FTS_E_INVAL, "fts_hierarchy_enable_adjoint: NULL handle");
    if (h->adj) return FTS_OK;
    const int L = h->nlevels;
    h->xs.assign(L, {});
    int64_t maxcells = 1;
    auto alloc = [&](int64_t n, double **p) {
        return dev_malloc(p, (size_t)std::max<int64_t>(n, 1) * sizeof(double)) == hipSuccess;
    };
    bool ok = true;
    for (int l = 0; l < L && ok; ++l) {
        const int64_t n = h->levels[l]->ndofs;
        maxcells = std::max(maxcells, h->levels[l]->ncells);
        const int nstates = l == 0 ? 1 : h->m_pre + h->m_post + 2;
        for (int i = 0; i < nstates && ok; ++i) {
            double *p = nullptr;
            ok = alloc(n, &p);
            h->xs[l].push_back(p);
        }
        for (auto *vv : {&h->lam, &h->lamb, &h->aq, &h->atr, &h->at}) {
            double *p = nullptr;
            if (ok) ok = alloc(n, &p);
            vv->push_back(p);
        }
    }
    if (ok) ok = alloc(maxcells, &h->apart) && alloc(2 * red_partials(), &h->ared) && alloc(2 * L, &h->agrad);
    if (ok) ok = hipHostMalloc(&h->host_grad, 2 * L * sizeof(double)) == hipSuccess;
    if (!ok) return fail(FTS_E_HIP, "allocation of the adjoint workspaces failed");
    h->adj = true;
    return FTS_OK;
}

// Forward V-cycle on level l from x_in (NULL = zero) recording the input of
// every smoothing step and the output in h->xs[l]; b_l is b (finest) or vb.
static fts_status adj_forward(fts_hierarchy *h, int l, const double *x_in, const double *b, hipStream_t s) {
    const fts_level *lv = h->levels[l];
    const int64_t n = lv->ndofs;
    auto &X = h->xs[l];
    fts_status st = FTS_OK;
    if (l == 0) return coarse_solve(h->coarse, b, X[0], s);
    if (x_in) {
        FTS_HIP_CHECK(hipMemcpyAsync(X[0], x_in, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
        st = launch_fill(X[0], n, 0.0, s);
    }
    const fts_eigs *eg = h->eigs[l];
    double *r = h->atr[l];
    int k = 0;
    for (int i = 0; i < h->m_pre && st == FTS_OK; ++i, ++k) {
        FTS_HIP_CHECK(hipMemcpyAsync(X[k + 1], X[k], n * sizeof(double), hipMemcpyDeviceToDevice, s));
        st = launch_operator(lv, X[k], b, r, true, s);
        if (st == FTS_OK) st = launch_schwarz(lv, eg, h->omega[l], FTS_PREC_F64, r, X[k + 1], s);
    }
    if (st == FTS_OK) st = launch_operator(lv, X[k], b, r, true, s);
    if (st == FTS_OK) st = launch_restrict(h->levels[l - 1], lv, r, h->vb[l - 1], s);
    if (st == FTS_OK) st = adj_forward(h, l - 1, nullptr, h->vb[l - 1], s);
    if (st == FTS_OK) {
        FTS_HIP_CHECK(hipMemcpyAsync(X[k + 1], X[k], n * sizeof(double), hipMemcpyDeviceToDevice, s));
        st = launch_prolongate(h->levels[l - 1], lv, h->xs[l - 1].back(), X[k + 1], s);
        ++k;
    }
    for (int i = 0; i < h->m_post && st == FTS_OK; ++i, ++k) {
        FTS_HIP_CHECK(hipMemcpyAsync(X[k + 1], X[k], n * sizeof(double), hipMemcpyDeviceToDevice, s));
        st = launch_operator(lv, X[k], b, r, true, s);
        if (st == FTS_OK) st = launch_schwarz(lv, eg, h->omega[l], FTS_PREC_F64, r, X[k + 1], s);
    }
    return st;
}

// Reverse of one smoothing step x' = x + omega C (b - A x) on level l, with
// lam[l] = adjoint of x' on entry and of x on exit; accumulates the adjoint
// of b in lamb[l], d omega_l and d gamma_l in agrad.
static fts_status adj_smooth_step(fts_hierarchy *h, int l, const double *xin, const double *b, hipStream_t s) {
    const fts_level *lv = h->levels[l];
    const fts_eigs *eg = h->eigs[l];
    const int64_t n = lv->ndofs;
    const double om = h->omega[l];
    double *lam = h->lam[l], *q = h->aq[l], *r = h->atr[l], *t = h->at[l];
    double *dom = h->agrad + 2 * l, *dga = h->agrad + 2 * l + 1;
    fts_status st = launch_operator(lv, xin, b, r, true, s);        // r = b - A x
    if (st == FTS_OK) st = launch_fill(q, n, 0.0, s);
    if (st == FTS_OK) st = launch_schwarz(lv, eg, 1.0, FTS_PREC_F64, lam, q, s);  // q = C lam
    if (st == FTS_OK) st = launch_dot_acc(q, r, n, 1.0, h->ared, dom, s);        // d omega += q.r
    if (st == FTS_OK) st = launch_axpy(om, q, h->lamb[l], n, s);                  // lam_b += omega q
    int64_t np = 0;
    if (st == FTS_OK) st = launch_schwarz_dgamma(lv, eg, lam, r, h->apart, &np, s);
    if (st == FTS_OK) st = launch_sum_acc(h->apart, np, -om, h->ared, dga, s);    // -omega sum_j u~ D v~
    if (st == FTS_OK) st = launch_operator_penalty(lv, xin, t, s);                // t = A1 x
    if (st == FTS_OK) st = launch_dot_acc(q, t, n, -om, h->ared, dga, s);         // -omega q.(A1 x)
    if (st == FTS_OK) st = launch_operator(lv, q, nullptr, t, false, s);          // t = A q
    if (st == FTS_OK) st = launch_axpy(-om, t, lam, n, s);                        // lam -= omega A q
    return st;
}

// Reverse of MG_l(x, b): lam[l] = adjoint of the output on entry, of x on exit;
// lamb[l] = adjoint of b (overwritten).
static fts_status adj_reverse(fts_hierarchy *h, int l, const double *b, hipStream_t s) {
    const fts_level *lv = h->levels[l];
    const int64_t n = lv->ndofs;
    fts_status st = FTS_OK;
    if (l == 0) {
        // x0 = A0^-1 b0: lam_b0 = A0^-1 lam; d gamma_0 -= lam_b0 . (A1 x0); lam_x = 0
        st = coarse_solve(h->coarse, h->lam[0], h->lamb[0], s);
        if (st == FTS_OK) st = launch_operator_penalty(lv, h->xs[0][0], h->at[0], s);
        if (st == FTS_OK) st = launch_dot_acc(h->lamb[0], h->at[0], n, -1.0, h->ared, h->agrad + 1, s);
        if (st == FTS_OK) st = launch_fill(h->lam[0], n, 0.0, s);
        return st;
    }
    auto &X = h->xs[l];
    st = launch_fill(h->lamb[l], n, 0.0, s);
    const int kc = h->m_pre;  // index of the state before the coarse correction
    for (int i = h->m_post; i >= 1 && st == FTS_OK; --i) st = adj_smooth_step(h, l, X[kc + i], b, s);
    // x_{kc+1} = x_kc + P e
    if (st == FTS_OK) st = launch_restrict(h->levels[l - 1], lv, h->lam[l], h->lam[l - 1], s);
    if (st == FTS_OK) st = adj_reverse(h, l - 1, h->vb[l - 1], s);
    // b_{l-1} = P^T (b - A x_kc)
    double *tr = h->atr[l];
    if (st == FTS_OK) st = launch_fill(tr, n, 0.0, s);
    if (st == FTS_OK) st = launch_prolongate(h->levels[l - 1], lv, h->lamb[l - 1], tr, s);
    if (st == FTS_OK) st = launch_axpy(1.0, tr, h->lamb[l], n, s);
    if (st == FTS_OK) st = launch_operator(lv, tr, nullptr, h->at[l], false, s);
    if (st == FTS_OK) st = launch_axpy(-1.0, h->at[l], h->lam[l], n, s);
    if (st == FTS_OK) st = launch_operator_penalty(lv, X[kc], h->aq[l], s);
    if (st == FTS_OK) st = launch_dot_acc(tr, h->aq[l], n, -1.0, h->ared, h->agrad + 2 * l + 1, s);
    for (int i = h->m_pre; i >= 1 && st == FTS_OK; --i) st = adj_smooth_step(h, l, X[i - 1], b, s);
    return st;
}

fts_status fts_vcycle_adjoint(fts_hierarchy *h, const double *b, const double *x_in, const double *lambda_out,
                              double *lambda_b, double *lambda_x, double *d_omega, double *d_penalty, void *stream) {
    if (!h || !b || !x_in || !lambda_out) return fail(FTS_E_INVAL, "fts_vcycle_adjoint: NULL argument");
    if (!h->adj) return fail(FTS_E_INVAL, "fts_vcycle_adjoint: call fts_hierarchy_enable_adjoint first");
    if (h->smoother != FTS_SMOOTHER_ADDITIVE)
        return fail(FTS_E_UNSUPPORTED, "fts_vcycle_adjoint: the adjoint is built for the additive smoother");
    if (h->kind != FTS_VERTEX_PATCH && h->kind != FTS_CELL) return fail(FTS_E_INVAL, "bad hierarchy");
    hipStream_t s = S(stream);
    const int L = h->nlevels - 1;
    const int64_t n = h->levels[L]->ndofs;
    fts_status st = launch_fill(h->agrad, 2 * h->nlevels, 0.0, s);
    if (st == FTS_OK) st = adj_forward(h, L, x_in, b, s);
    if (st == FTS_OK)
        FTS_HIP_CHECK(hipMemcpyAsync(h->lam[L], lambda_out, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (st == FTS_OK) st = adj_reverse(h, L, b, s);
    if (st == FTS_OK && lambda_b) st = launch_axpy(1.0, h->lamb[L], lambda_b, n, s);
    if (st == FTS_OK && lambda_x)
        FTS_HIP_CHECK(hipMemcpyAsync(lambda_x, h->lam[L], n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (st != FTS_OK) return st;
    FTS_HIP_CHECK(hipMemcpyAsync(h->host_grad, h->agrad, 2 * h->nlevels * sizeof(double), hipMemcpyDeviceToHost, s));
    FTS_HIP_CHECK(hipStreamSynchronize(s));
    for (int l = 0; l < h->nlevels; ++l) {
        if (d_omega) d_omega[l] += h->host_grad[2 * l];
        if (d_penalty) d_penalty[l] += h->host_grad[2 * l + 1];
    }
    return FTS_OK;
}

fts_status fts_vcycle(fts_hierarchy *h, fts_prec prec, const double *b, double *x, void *stream) {
    if (!h || !b || !x) return fail(FTS_E_INVAL, "fts_vcycle: NULL argument");
    if (b == x) return fail(FTS_E_INVAL, "fts_vcycle: b must not alias x");
    return vcycle_level(h, h->nlevels - 1, prec, b, x, S(stream));
}

}  // extern "C"
