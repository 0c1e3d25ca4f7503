// Host FP64 setup: 1-D reference data, 1-D SIPG operators of cells and vertex
// patches, generalised eigenproblems, and the level / eigen tables uploaded to
// the device.  (Sec. 2.1, Sec. 3.2 of Witte, Arndt, Kanschat.)
#include <algorithm>
#include <array>
#include <map>
#include <cmath>
#include <mutex>
#include <cstring>

#include "fts_internal.h"

namespace fts {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

namespace {
std::mutex g_alloc_mutex;
fts_alloc_fn g_alloc_fn = nullptr;
fts_free_fn g_free_fn = nullptr;
void *g_alloc_ctx = nullptr;
}  // namespace

hipError_t dev_malloc_raw(void **p, size_t bytes) {
    fts_alloc_fn fn;
    void *ctx;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mutex);
        fn = g_alloc_fn;
        ctx = g_alloc_ctx;
    }
    *p = nullptr;
    if (!fn) {
        set_error("no device allocator registered (fts_set_allocator)");
        return hipErrorInvalidValue;
    }
    *p = fn(bytes > 0 ? bytes : 1, ctx);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

void dev_free(void *p) {
    if (!p) return;
    fts_free_fn fn;
    void *ctx;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mutex);
        fn = g_free_fn;
        ctx = g_alloc_ctx;
    }
    if (fn) fn(p, ctx);
}

fts_status fail(fts_status code, const std::string &msg) {
    set_error(msg);
    return code;
}

fts_status hip_fail(hipError_t err, const char *what) {
    set_error(std::string("HIP error in ") + what + ": " + hipGetErrorString(err));
    return FTS_E_HIP;
}

// Legendre polynomial P_n and its derivative at x in [-1, 1] by the
// three-term recurrence.
static void legendre(int n, double x, double &p, double &dp) {
    double p0 = 1.0, p1 = x;
    if (n == 0) {
        p = 1.0;
        dp = 0.0;
        return;
    }
    for (int j = 1; j < n; ++j) {
        double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    // derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n)
    dp = (std::fabs(1.0 - x * x) > 1e-300) ? n * (p0 - x * p1) / (1.0 - x * x) : 0.0;
}

// Interior Gauss-Lobatto nodes: roots of P_k' found by Newton's method on
// q(x) = (1 - x^2) P_k'(x) / k = P_{k-1}(x) - x P_k(x), whose roots in (-1,1) are
// those of P_k'.  Start: Chebyshev-Gauss-Lobatto points.
static std::vector<double> gll_nodes_unit(int k) {
    std::vector<double> z(k + 1);
    z[0] = -1.0;
    z[k] = 1.0;
    for (int j = 1; j < k; ++j) {
        double x = -std::cos(M_PI * j / k);
        for (int it = 0; it < 100; ++it) {
            // f(x) = P_k'(x); f'(x) = P_k''(x) = (2x P_k' - k(k+1) P_k) / (1 - x^2)
            double p, dp;
            legendre(k, x, p, dp);
            double ddp = (2.0 * x * dp - k * (k + 1.0) * p) / (1.0 - x * x);
            double dx = dp / ddp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        z[j] = x;
    }
    std::sort(z.begin(), z.end());
    std::vector<double> out(k + 1);
    for (int j = 0; j <= k; ++j) out[j] = 0.5 * (z[j] + 1.0);
    out[0] = 0.0;
    out[k] = 1.0;
    return out;
}

// nq-point Gauss-Legendre rule on [0, 1] (Newton on P_nq, weights 2/((1-x^2)P'^2)).
static void gauss_unit(int nq, std::vector<double> &x, std::vector<double> &w) {
    x.assign(nq, 0.0);
    w.assign(nq, 0.0);
    for (int j = 0; j < nq; ++j) {
        double t = std::cos(M_PI * (j + 0.75) / (nq + 0.5));
        double p = 0, dp = 1;
        for (int it = 0; it < 100; ++it) {
            legendre(nq, t, p, dp);
            double dt = p / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        legendre(nq, t, p, dp);
        x[j] = 0.5 * (1.0 - t);
        w[j] = 1.0 / ((1.0 - t * t) * dp * dp);  // 2/(...) scaled by 1/2 for [0,1]
    }
}

// Barycentric Lagrange evaluation: values and first derivatives of all
// basis polynomials of `nodes` at the point x.
static void lagrange_at(const std::vector<double> &nodes, double x, double *val, double *der) {
    const int n = (int)nodes.size();
    std::vector<double> wb(n, 1.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (j != i) wb[i] /= (nodes[i] - nodes[j]);
    int hit = -1;
    for (int i = 0; i < n; ++i)
        if (std::fabs(x - nodes[i]) < 1e-15) hit = i;
    if (hit >= 0) {
        // at a node: delta values; derivative from the differentiation matrix row
        for (int j = 0; j < n; ++j) val[j] = (j == hit) ? 1.0 : 0.0;
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == hit) continue;
            der[j] = (wb[j] / wb[hit]) / (nodes[hit] - nodes[j]);
            diag -= der[j];
        }
        der[hit] = diag;
        return;
    }
    double ell = 1.0;
    for (int i = 0; i < n; ++i) ell *= (x - nodes[i]);
    for (int j = 0; j < n; ++j) {
        val[j] = ell * wb[j] / (x - nodes[j]);
        // phi_j' / phi_j = sum_{i != j} 1/(x - x_i), summed without the j term
        double s = 0.0;
        for (int i = 0; i < n; ++i)
            if (i != j) s += 1.0 / (x - nodes[i]);
        der[j] = val[j] * s;
    }
}

void gauss_basis(int k, std::vector<double> &xq, std::vector<double> &wq, std::vector<double> &V,
                 std::vector<double> &D) {
    const int n1 = k + 1;
    const std::vector<double> nodes = gll_nodes_unit(k);
    gauss_unit(n1, xq, wq);
    V.assign(n1 * n1, 0.0);
    D.assign(n1 * n1, 0.0);
    for (int q = 0; q < n1; ++q) lagrange_at(nodes, xq[q], &V[q * n1], &D[q * n1]);
}

void Ref1D::build(int degree) {
    k = degree;
    n1 = k + 1;
    nodes = gll_nodes_unit(k);
    std::vector<double> xq, wq;
    gauss_unit(n1, xq, wq);  // exact for the degree-2k integrands
    Mhat.assign(n1 * n1, 0.0);
    Lhat.assign(n1 * n1, 0.0);
    std::vector<double> val(n1), der(n1);
    for (int q = 0; q < n1; ++q) {
        lagrange_at(nodes, xq[q], val.data(), der.data());
        for (int a = 0; a < n1; ++a)
            for (int b = 0; b < n1; ++b) {
                Mhat[a * n1 + b] += wq[q] * val[a] * val[b];
                Lhat[a * n1 + b] += wq[q] * der[a] * der[b];
            }
    }
    v0.assign(n1, 0.0);
    v1.assign(n1, 0.0);
    d0.assign(n1, 0.0);
    d1.assign(n1, 0.0);
    lagrange_at(nodes, 0.0, v0.data(), d0.data());
    lagrange_at(nodes, 1.0, v1.data(), d1.data());
    for (int c = 0; c < 2; ++c) {
        E[c].assign(n1 * n1, 0.0);
        for (int i = 0; i < n1; ++i) {
            lagrange_at(nodes, 0.5 * (nodes[i] + c), val.data(), der.data());
            for (int j = 0; j < n1; ++j) E[c][i * n1 + j] = val[j];
        }
    }
}

// Cell operator A = L/h + N_0 + N_1 (eq. 1Dsipg).  A face term for the face
// at reference point p with outward sign s (= -1 left, +1 right) and weight
// eta (1 on the boundary, 1/2 inside, from the 1/sqrt(2) average):
//   N_p = eta*gamma v_p v_p^T - (s*eta/h) (v_p d_p^T + d_p v_p^T)
// with gamma = gamma_hat k (k+1) (1/h + 1/h_neighbour) (eq. penalty).
void Ref1D::cell_operator(double h, double h_left, double h_right, double gamma_hat,
                          double *A) const {
    const double kk = gamma_hat * k * (k + 1.0);
    for (int a = 0; a < n1; ++a)
        for (int b = 0; b < n1; ++b) A[a * n1 + b] = Lhat[a * n1 + b] / h;
    for (int p = 0; p < 2; ++p) {
        const double hn = p == 0 ? h_left : h_right;
        const bool bdry = !(hn > 0.0);
        const double eta = bdry ? 1.0 : 0.5;
        const double gamma = bdry ? kk * 2.0 / h : kk * (1.0 / h + 1.0 / hn);
        const double s = p == 0 ? -1.0 : 1.0;
        const std::vector<double> &v = p == 0 ? v0 : v1;
        const std::vector<double> &d = p == 0 ? d0 : d1;
        for (int a = 0; a < n1; ++a)
            for (int b = 0; b < n1; ++b)
                A[a * n1 + b] += eta * gamma * v[a] * v[b] - (s * eta / h) * (v[a] * d[b] + d[a] * v[b]);
    }
}

// Coupling of the left cell (test functions, width hl) to the right cell
// (trial functions, width hr) through their common face, from eq. (bfsipg)
// with the 1/sqrt(2) average: penalty -gamma/2 u_r v_l, consistency
// -1/2 d_n u_r v_l, adjoint consistency +1/2 u_r d_n v_l (n from left to right).
void Ref1D::interface_block(double hl, double hr, double gamma_hat, double *B) const {
    const double gamma = gamma_hat * k * (k + 1.0) * (1.0 / hl + 1.0 / hr);
    for (int a = 0; a < n1; ++a)
        for (int b = 0; b < n1; ++b)
            B[a * n1 + b] = -0.5 * gamma * v1[a] * v0[b] - v1[a] * d0[b] / (2.0 * hr) +
                            d1[a] * v0[b] / (2.0 * hl);
}

void Ref1D::cell_penalty(double h, double h_left, double h_right, double *A) const {
    const double kk = k * (k + 1.0);
    for (int a = 0; a < n1 * n1; ++a) A[a] = 0.0;
    for (int p = 0; p < 2; ++p) {
        const double hn = p == 0 ? h_left : h_right;
        const bool bdry = !(hn > 0.0);
        const double eta = bdry ? 1.0 : 0.5;
        const double gamma = bdry ? kk * 2.0 / h : kk * (1.0 / h + 1.0 / hn);
        const std::vector<double> &v = p == 0 ? v0 : v1;
        for (int a = 0; a < n1; ++a)
            for (int b = 0; b < n1; ++b) A[a * n1 + b] += eta * gamma * v[a] * v[b];
    }
}

void Ref1D::interface_penalty(double hl, double hr, double *B) const {
    const double gamma = k * (k + 1.0) * (1.0 / hl + 1.0 / hr);
    for (int a = 0; a < n1; ++a)
        for (int b = 0; b < n1; ++b) B[a * n1 + b] = -0.5 * gamma * v1[a] * v0[b];
}

fts_status sym_gen_eig(int n, const double *A, const double *M, double *S, double *lam) {
    // Cholesky M = L L^T
    std::vector<double> L(n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        double s = M[j * n + j];
        for (int p = 0; p < j; ++p) s -= L[j * n + p] * L[j * n + p];
        if (!(s > 0.0)) return fail(FTS_E_NOT_SPD, "1-D mass matrix is not positive definite");
        L[j * n + j] = std::sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double t = M[i * n + j];
            for (int p = 0; p < j; ++p) t -= L[i * n + p] * L[j * n + p];
            L[i * n + j] = t / L[j * n + j];
        }
    }
    // Linv by forward substitution
    std::vector<double> Li(n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) {
            double t = (i == c) ? 1.0 : 0.0;
            for (int p = 0; p < i; ++p) t -= L[i * n + p] * Li[p * n + c];
            Li[i * n + c] = t / L[i * n + i];
        }
    }
    // C = Linv A Linv^T (symmetrised)
    std::vector<double> T(n * n, 0.0), C(n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double t = 0.0;
            for (int p = 0; p < n; ++p) t += Li[i * n + p] * A[p * n + j];
            T[i * n + j] = t;
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double t = 0.0;
            for (int p = 0; p < n; ++p) t += T[i * n + p] * Li[j * n + p];
            C[i * n + j] = t;
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) C[i * n + j] = C[j * n + i] = 0.5 * (C[i * n + j] + C[j * n + i]);
    // cyclic Jacobi: C = Q diag Q^T
    std::vector<double> Q(n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
    double fro = 0.0;
    for (int i = 0; i < n * n; ++i) fro += C[i] * C[i];
    fro = std::sqrt(fro);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += C[i * n + j] * C[i * n + j];
        if (std::sqrt(off) <= 1e-17 * fro) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = C[p * n + q];
                if (std::fabs(apq) <= 1e-300) continue;
                const double theta = (C[q * n + q] - C[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < n; ++r) {  // columns p, q
                    const double crp = C[r * n + p], crq = C[r * n + q];
                    C[r * n + p] = c * crp - s * crq;
                    C[r * n + q] = s * crp + c * crq;
                }
                for (int r = 0; r < n; ++r) {  // rows p, q
                    const double cpr = C[p * n + r], cqr = C[q * n + r];
                    C[p * n + r] = c * cpr - s * cqr;
                    C[q * n + r] = s * cpr + c * cqr;
                }
                for (int r = 0; r < n; ++r) {
                    const double qrp = Q[r * n + p], qrq = Q[r * n + q];
                    Q[r * n + p] = c * qrp - s * qrq;
                    Q[r * n + q] = s * qrp + c * qrq;
                }
            }
    }
    // sort ascending, S = Linv^T Q
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return C[a * n + a] < C[b * n + b]; });
    for (int m = 0; m < n; ++m) {
        const int o = order[m];
        lam[m] = C[o * n + o];
        if (!(lam[m] > 0.0)) return fail(FTS_E_NOT_SPD, "1-D SIPG operator is not positive definite");
        for (int i = 0; i < n; ++i) {
            double t = 0.0;
            for (int p = 0; p < n; ++p) t += Li[p * n + i] * Q[p * n + o];
            S[i * n + m] = t;
        }
    }
    return FTS_OK;
}

}  // namespace fts

using namespace fts;

// Even-odd form of a centro-symmetric n x n matrix M (M[i][j] = M[n-1-i][n-1-j];
// the reference mass and stiffness are, up to rounding, because the nodes are
// symmetric about the cell centre; M is symmetrised first).  With h = n / 2 and
// he = (n + 1) / 2: E (he x he) maps the sums u_j + u_{n-1-j}, j < h, and for odd
// n the middle value u_h, to the half sums (y_i + y_{n-1-i}) / 2 (i < h) and to
// y_h; O (h x h) maps the differences u_j - u_{n-1-j} to the half differences.
// Stored E then O, row-major.
static std::vector<double> even_odd(const std::vector<double> &M, int n) {
    const int h = n / 2, he = (n + 1) / 2;
    auto sym = [&](int i, int j) { return 0.5 * (M[i * n + j] + M[(n - 1 - i) * n + (n - 1 - j)]); };
    std::vector<double> out((size_t)he * he + (size_t)h * h, 0.0);
    for (int i = 0; i < he; ++i)
        for (int j = 0; j < he; ++j) {
            double e;
            if (i < h && j < h) e = 0.5 * (sym(i, j) + sym(i, n - 1 - j));
            else e = sym(i, j);  // middle row or column (odd n)
            out[(size_t)i * he + j] = e;
        }
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < h; ++j) out[(size_t)he * he + (size_t)i * h + j] = 0.5 * (sym(i, j) - sym(i, n - 1 - j));
    return out;
}

extern "C" {

const char *fts_version(void) { return "fts 0.1.0 (gfx950)"; }

fts_status fts_last_error(char *buf, size_t len) {
    if (!buf || len == 0) return FTS_E_INVAL;
    std::strncpy(buf, g_last_error.c_str(), len - 1);
    buf[len - 1] = '\0';
    return FTS_OK;
}

fts_status fts_level_create(const fts_mesh_desc *mesh, fts_level **out) {
    if (!mesh || !out) return fail(FTS_E_INVAL, "fts_level_create: NULL argument");
    *out = nullptr;
    if (mesh->dim != 2 && mesh->dim != 3) return fail(FTS_E_UNSUPPORTED, "dim must be 2 or 3");
    if (mesh->degree < 1 || mesh->degree > (mesh->dim == 2 ? kMaxDegree2D : kMaxDegree))
        return fail(FTS_E_UNSUPPORTED, mesh->dim == 2 ? "degree must be in 1..15 in 2-D" : "degree must be in 1..9 in 3-D");
    if (!(mesh->penalty_factor > 0.0) || !std::isfinite(mesh->penalty_factor))
        return fail(FTS_E_INVAL, "penalty_factor must be positive");
    fts_level *lv = new fts_level();
    lv->dim = mesh->dim;
    lv->k = mesh->degree;
    lv->n1 = mesh->degree + 1;
    lv->gamma_hat = mesh->penalty_factor;
    lv->ncells = 1;
    for (int a = 0; a < 3; ++a) {
        if (a >= lv->dim) {
            lv->m[a] = 1;
            lv->h[a].assign(1, 1.0);
            continue;
        }
        if (mesh->ncells[a] < 1 || !mesh->h[a]) {
            delete lv;
            return fail(FTS_E_INVAL, "ncells must be >= 1 and h non-NULL on every axis");
        }
        lv->m[a] = mesh->ncells[a];
        lv->h[a].assign(mesh->h[a], mesh->h[a] + mesh->ncells[a]);
        for (double w : lv->h[a])
            if (!(w > 0.0) || !std::isfinite(w)) {
                delete lv;
                return fail(FTS_E_INVAL, "cell widths must be positive and finite");
            }
        lv->ncells *= lv->m[a];
    }
    int64_t cd = 1;
    for (int a = 0; a < lv->dim; ++a) cd *= lv->n1;
    lv->ndofs = lv->ncells * cd;
    lv->ref.build(lv->k);
    const int n1 = lv->n1, nn = n1 * n1;
    // host tables
    size_t total = 0;
    for (int a = 0; a < 3; ++a) {
        const int m = lv->m[a];
        lv->host_cellop[a].assign((size_t)m * nn, 0.0);
        lv->host_iface[a].assign((size_t)std::max(m - 1, 0) * nn, 0.0);
        for (int c = 0; c < m; ++c) {
            const double hl = c > 0 ? lv->h[a][c - 1] : -1.0;
            const double hr = c + 1 < m ? lv->h[a][c + 1] : -1.0;
            lv->ref.cell_operator(lv->h[a][c], hl, hr, lv->gamma_hat, &lv->host_cellop[a][(size_t)c * nn]);
            if (c + 1 < m)
                lv->ref.interface_block(lv->h[a][c], lv->h[a][c + 1], lv->gamma_hat,
                                        &lv->host_iface[a][(size_t)c * nn]);
        }
        total += lv->host_cellop[a].size() + lv->host_iface[a].size() + 2 * lv->h[a].size();
    }
    total += nn + 2 * nn + nn + 2 * lv->n1 + 2 * nn;
    if (dev_malloc(&lv->d_tab, total * sizeof(double)) != hipSuccess) {
        delete lv;
        return fail(FTS_E_HIP, "device allocation of level tables failed");
    }
    std::vector<double> host(total);
    size_t off = 0;
    auto put = [&](const std::vector<double> &v) {
        std::copy(v.begin(), v.end(), host.begin() + off);
        const double *p = lv->d_tab + off;
        off += v.size();
        return p;
    };
    for (int a = 0; a < 3; ++a) {
        lv->view.cellop[a] = put(lv->host_cellop[a]);
        lv->view.iface[a] = put(lv->host_iface[a]);
        lv->view.h[a] = put(lv->h[a]);
        std::vector<double> ih(lv->h[a].size());
        for (size_t c = 0; c < ih.size(); ++c) ih[c] = 1.0 / lv->h[a][c];
        lv->view.ih[a] = put(ih);
        lv->view.m[a] = lv->m[a];
    }
    lv->view.Mhat = put(lv->ref.Mhat);
    std::vector<double> E(2 * nn);
    std::copy(lv->ref.E[0].begin(), lv->ref.E[0].end(), E.begin());
    std::copy(lv->ref.E[1].begin(), lv->ref.E[1].end(), E.begin() + nn);
    lv->view.E = put(E);
    lv->view.Lhat = put(lv->ref.Lhat);
    lv->view.d0 = put(lv->ref.d0);
    lv->view.d1 = put(lv->ref.d1);
    lv->view.Meo = put(even_odd(lv->ref.Mhat, lv->n1));
    lv->view.Leo = put(even_odd(lv->ref.Lhat, lv->n1));
    lv->view.gk = lv->gamma_hat * lv->k * (lv->k + 1.0);
    lv->view.pk = lv->k * (lv->k + 1.0);
    lv->view.ncells = lv->ncells;
    if (hipMemcpy(lv->d_tab, host.data(), total * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        dev_free(lv->d_tab);
        delete lv;
        return fail(FTS_E_HIP, "upload of level tables failed");
    }
    *out = lv;
    return FTS_OK;
}

fts_status fts_level_destroy(fts_level *level) {
    if (!level) return FTS_OK;
    if (level->d_tab) dev_free(level->d_tab);
    delete level;
    return FTS_OK;
}

int64_t fts_level_ndofs(const fts_level *level) { return level ? level->ndofs : -1; }

}  // extern "C"

namespace fts {
fts_status setup_eigs_internal(const fts_level *lv, fts_patch_kind kind, bool staging, fts_eigs **out) {
    if (!lv || !out) return fail(FTS_E_INVAL, "fts_setup_1d_eigs: NULL argument");
    *out = nullptr;
    if (kind != FTS_CELL && kind != FTS_VERTEX_PATCH) return fail(FTS_E_INVAL, "unknown patch kind");
    const int n1 = lv->n1;
    const int n = kind == FTS_CELL ? n1 : 2 * n1;
    for (int a = 0; a < lv->dim; ++a)
        if (kind == FTS_VERTEX_PATCH && lv->m[a] < 2)
            return fail(FTS_E_INVAL, "vertex patches need at least 2 cells per axis");
    fts_eigs *eg = new fts_eigs();
    eg->level = lv;
    eg->kind = kind;
    eg->n = n;
    const int nn = n * n, c2 = n1 * n1;
    std::vector<double> tmp(c2);
    size_t total = 0;
    for (int a = 0; a < 3; ++a) {
        const int m = lv->m[a];
        const int cnt = (a >= lv->dim) ? 0 : (kind == FTS_CELL ? m : m - 1);
        eg->count[a] = cnt;
        eg->A[a].assign((size_t)cnt * nn, 0.0);
        eg->M[a].assign((size_t)cnt * nn, 0.0);
        eg->S[a].assign((size_t)cnt * nn, 0.0);
        eg->lam[a].assign((size_t)cnt * n, 0.0);
        eg->cls[a].assign(cnt, 0);
        const std::vector<double> &h = lv->h[a];
        // The 1-D problem of a position is a function of the widths of the
        // cells it covers and of their outer neighbours (-1: boundary).
        // Positions with the same widths bit for bit share one table.
        std::map<std::array<double, 4>, int> seen;
        for (int s = 0; s < cnt; ++s) {
            std::array<double, 4> key;
            if (kind == FTS_CELL)
                key = {s > 0 ? h[s - 1] : -1.0, h[s], s + 1 < m ? h[s + 1] : -1.0, 0.0};
            else
                key = {s > 0 ? h[s - 1] : -1.0, h[s], h[s + 1], s + 2 < m ? h[s + 2] : -1.0};
            const auto hit = seen.find(key);
            if (hit != seen.end()) {
                const int r = hit->second;
                eg->cls[a][s] = r;
                std::copy_n(&eg->A[a][(size_t)r * nn], nn, &eg->A[a][(size_t)s * nn]);
                std::copy_n(&eg->M[a][(size_t)r * nn], nn, &eg->M[a][(size_t)s * nn]);
                std::copy_n(&eg->S[a][(size_t)r * nn], nn, &eg->S[a][(size_t)s * nn]);
                std::copy_n(&eg->lam[a][(size_t)r * n], n, &eg->lam[a][(size_t)s * n]);
                const std::vector<double> dg(eg->DG[a].begin() + (size_t)r * nn,
                                             eg->DG[a].begin() + (size_t)(r + 1) * nn);
                eg->DG[a].insert(eg->DG[a].end(), dg.begin(), dg.end());
                continue;
            }
            seen.emplace(key, s);
            eg->cls[a][s] = s;
            double *A = &eg->A[a][(size_t)s * nn];
            double *M = &eg->M[a][(size_t)s * nn];
            if (kind == FTS_CELL) {
                lv->ref.cell_operator(h[s], s > 0 ? h[s - 1] : -1.0, s + 1 < m ? h[s + 1] : -1.0,
                                      lv->gamma_hat, A);
                for (int i = 0; i < c2; ++i) M[i] = h[s] * lv->ref.Mhat[i];
            } else {
                // two cells s (left, "+") and s+1 (right, "-") around vertex s+1 (eq. 1DsipgVP)
                const int cl = s, cr = s + 1;
                lv->ref.cell_operator(h[cl], cl > 0 ? h[cl - 1] : -1.0, h[cr], lv->gamma_hat, tmp.data());
                for (int i = 0; i < n1; ++i)
                    for (int j = 0; j < n1; ++j) A[i * n + j] = tmp[i * n1 + j];
                lv->ref.cell_operator(h[cr], h[cl], cr + 1 < m ? h[cr + 1] : -1.0, lv->gamma_hat, tmp.data());
                for (int i = 0; i < n1; ++i)
                    for (int j = 0; j < n1; ++j) A[(n1 + i) * n + n1 + j] = tmp[i * n1 + j];
                lv->ref.interface_block(h[cl], h[cr], lv->gamma_hat, tmp.data());
                for (int i = 0; i < n1; ++i)
                    for (int j = 0; j < n1; ++j) {
                        A[i * n + n1 + j] = tmp[i * n1 + j];
                        A[(n1 + j) * n + i] = tmp[i * n1 + j];
                    }
                for (int i = 0; i < n1; ++i)
                    for (int j = 0; j < n1; ++j) {
                        M[i * n + j] = h[cl] * lv->ref.Mhat[i * n1 + j];
                        M[(n1 + i) * n + n1 + j] = h[cr] * lv->ref.Mhat[i * n1 + j];
                    }
            }
            fts_status st = sym_gen_eig(n, A, M, &eg->S[a][(size_t)s * nn], &eg->lam[a][(size_t)s * n]);
            if (st != FTS_OK) {
                delete eg;
                return st;
            }
            // dA/dgamma_hat of the same 1-D operator, then S^T (dA/dgamma_hat) S
            std::vector<double> A1(nn, 0.0);
            if (kind == FTS_CELL) {
                lv->ref.cell_penalty(h[s], s > 0 ? h[s - 1] : -1.0, s + 1 < m ? h[s + 1] : -1.0, A1.data());
            } else {
                const int cl = s, cr = s + 1;
                lv->ref.cell_penalty(h[cl], cl > 0 ? h[cl - 1] : -1.0, h[cr], tmp.data());
                for (int i = 0; i < n1; ++i)
                    for (int j = 0; j < n1; ++j) A1[i * n + j] = tmp[i * n1 + j];
                lv->ref.cell_penalty(h[cr], h[cl], cr + 1 < m ? h[cr + 1] : -1.0, tmp.data());
                for (int i = 0; i < n1; ++i)
                    for (int j = 0; j < n1; ++j) A1[(n1 + i) * n + n1 + j] = tmp[i * n1 + j];
                lv->ref.interface_penalty(h[cl], h[cr], tmp.data());
                for (int i = 0; i < n1; ++i)
                    for (int j = 0; j < n1; ++j) {
                        A1[i * n + n1 + j] = tmp[i * n1 + j];
                        A1[(n1 + j) * n + i] = tmp[i * n1 + j];
                    }
            }
            const double *Sd = &eg->S[a][(size_t)s * nn];
            std::vector<double> T1(nn, 0.0);
            for (int i = 0; i < n; ++i)
                for (int m2 = 0; m2 < n; ++m2) {
                    double t = 0.0;
                    for (int p = 0; p < n; ++p) t += A1[i * n + p] * Sd[p * n + m2];
                    T1[i * n + m2] = t;
                }
            for (int o = 0; o < n; ++o)
                for (int m2 = 0; m2 < n; ++m2) {
                    double t = 0.0;
                    for (int p = 0; p < n; ++p) t += Sd[p * n + o] * T1[p * n + m2];
                    eg->DG[a].push_back(t);
                }
        }
        total += 3 * eg->S[a].size() + eg->lam[a].size();
    }
    // Device copies of the tables.  A position whose 1-D problem is mirror
    // symmetric about its centre (equal widths on both sides, n even) has
    // eigenvectors that are even or odd about the centre (Sec. 3.2: S is
    // determined up to the order and sign of its columns).  Its modes are
    // reordered, the n/2 even ones first, and each vector is made exactly
    // even or odd, so that the kernels can contract it in even-odd form with
    // the first n/2 rows of S.  fts_eigs_get returns the eigen-solver's order.
    std::vector<double> Sd[3], lamd[3], DGd[3];
    for (int a = 0; a < 3; ++a) {
        Sd[a] = eg->S[a];
        lamd[a] = eg->lam[a];
        DGd[a] = eg->DG[a];
        eg->sym[a].assign(eg->count[a], 0);
        if (n % 2) continue;
        const int m = lv->m[a], h2 = n / 2;
        const std::vector<double> &h = lv->h[a];
        for (int p = 0; p < eg->count[a]; ++p) {
            const int r = eg->cls[a][p];
            if (r != p) {
                std::copy_n(&Sd[a][(size_t)r * nn], nn, &Sd[a][(size_t)p * nn]);
                std::copy_n(&lamd[a][(size_t)r * n], n, &lamd[a][(size_t)p * n]);
                std::copy_n(&DGd[a][(size_t)r * nn], nn, &DGd[a][(size_t)p * nn]);
                eg->sym[a][p] = eg->sym[a][r];
                continue;
            }
            const bool mirror = kind == FTS_CELL
                                    ? (p > 0 ? h[p - 1] : -1.0) == (p + 1 < m ? h[p + 1] : -1.0)
                                    : h[p] == h[p + 1] && (p > 0 ? h[p - 1] : -1.0) == (p + 2 < m ? h[p + 2] : -1.0);
            if (!mirror) continue;
            const double *S0 = &eg->S[a][(size_t)p * nn];
            std::vector<int> even, odd;
            for (int c = 0; c < n; ++c) {
                double sc = 0.0, ep = 0.0, em = 0.0;
                for (int i = 0; i < n; ++i) {
                    sc = std::max(sc, std::fabs(S0[i * n + c]));
                    ep = std::max(ep, std::fabs(S0[i * n + c] - S0[(n - 1 - i) * n + c]));
                    em = std::max(em, std::fabs(S0[i * n + c] + S0[(n - 1 - i) * n + c]));
                }
                if (ep <= 1e-10 * sc) even.push_back(c);
                else if (em <= 1e-10 * sc) odd.push_back(c);
            }
            if ((int)even.size() != h2 || (int)odd.size() != h2) continue;  // e.g. a repeated eigenvalue
            std::vector<int> perm(even);
            perm.insert(perm.end(), odd.begin(), odd.end());
            double *Sp = &Sd[a][(size_t)p * nn];
            for (int c = 0; c < n; ++c) {
                const int q = perm[c];
                const double sg = c < h2 ? 1.0 : -1.0;
                for (int i = 0; i < h2; ++i) {
                    const double v = 0.5 * (S0[i * n + q] + sg * S0[(n - 1 - i) * n + q]);
                    Sp[i * n + c] = v;
                    Sp[(n - 1 - i) * n + c] = sg * v;
                }
                lamd[a][(size_t)p * n + c] = eg->lam[a][(size_t)p * n + q];
                for (int c2 = 0; c2 < n; ++c2)
                    DGd[a][(size_t)p * nn + c * n + c2] = eg->DG[a][(size_t)p * nn + q * n + perm[c2]];
            }
            eg->sym[a][p] = 1;
        }
    }
    if (dev_malloc(&eg->d_tab, std::max<size_t>(total, 1) * sizeof(double)) != hipSuccess ||
        dev_malloc(&eg->d_tab32, std::max<size_t>(total, 1) * sizeof(float)) != hipSuccess) {
        if (eg->d_tab) dev_free(eg->d_tab);
        delete eg;
        return fail(FTS_E_HIP, "device allocation of eigen tables failed");
    }
    std::vector<double> host(total);
    std::vector<float> host32(total);
    size_t off = 0;
    for (int a = 0; a < 3; ++a) {
        eg->view.count[a] = eg->count[a];
        eg->view.S[a] = eg->d_tab + off;
        eg->view.S32[a] = eg->d_tab32 + off;
        for (double v : Sd[a]) host[off++] = v;
        eg->view.ST[a] = eg->d_tab + off;
        eg->view.ST32[a] = eg->d_tab32 + off;
        for (int s = 0; s < eg->count[a]; ++s)
            for (int m = 0; m < n; ++m)
                for (int i = 0; i < n; ++i) host[off++] = Sd[a][(size_t)s * nn + i * n + m];
        eg->view.DG[a] = eg->d_tab + off;
        for (double v : DGd[a]) host[off++] = v;
        eg->view.lam[a] = eg->d_tab + off;
        eg->view.lam32[a] = eg->d_tab32 + off;
        for (double v : lamd[a]) host[off++] = v;
    }
    for (size_t i = 0; i < total; ++i) host32[i] = (float)host[i];
    if (total && (hipMemcpy(eg->d_tab, host.data(), total * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
                  hipMemcpy(eg->d_tab32, host32.data(), total * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)) {
        dev_free(eg->d_tab);
        dev_free(eg->d_tab32);
        delete eg;
        return fail(FTS_E_HIP, "upload of eigen tables failed");
    }
    {
        std::vector<int> hc;
        for (int a = 0; a < 3; ++a) hc.insert(hc.end(), eg->cls[a].begin(), eg->cls[a].end());
        for (int a = 0; a < 3; ++a) hc.insert(hc.end(), eg->sym[a].begin(), eg->sym[a].end());
        if (dev_malloc(&eg->d_cls, std::max<size_t>(hc.size(), 1) * sizeof(int)) != hipSuccess ||
            (!hc.empty() &&
             hipMemcpy(eg->d_cls, hc.data(), hc.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)) {
            if (eg->d_cls) dev_free(eg->d_cls);
            dev_free(eg->d_tab);
            dev_free(eg->d_tab32);
            delete eg;
            return fail(FTS_E_HIP, "upload of the table classes failed");
        }
        size_t co = 0;
        for (int a = 0; a < 3; ++a) {
            eg->view.cls[a] = eg->d_cls + co;
            co += eg->cls[a].size();
        }
        for (int a = 0; a < 3; ++a) {
            eg->view.sym[a] = eg->d_cls + co;
            co += eg->sym[a].size();
        }
    }
    if (n <= 16) {
        // 16-bit MFMA tables: 4 matrices of 256 entries per (axis, position), plus 2 floats
        size_t cnt_all = 0;
        for (int a = 0; a < 3; ++a) cnt_all += eg->count[a];
        const size_t mats = cnt_all * 4 * 256 * sizeof(uint16_t);
        const size_t flts = cnt_all * 2 * sizeof(float);
        std::vector<unsigned char> host16(std::max<size_t>(mats + flts, 4));
        uint16_t *m16 = reinterpret_cast<uint16_t *>(host16.data());
        float *f32 = reinterpret_cast<float *>(host16.data() + mats);
        if (dev_malloc(&eg->d_mfma, host16.size()) != hipSuccess) {
            dev_free(eg->d_tab);
            dev_free(eg->d_tab32);
            dev_free(eg->d_cls);
            delete eg;
            return fail(FTS_E_HIP, "device allocation of the MFMA tables failed");
        }
        const uint16_t *dm = static_cast<const uint16_t *>(eg->d_mfma);
        const float *df = reinterpret_cast<const float *>(static_cast<const unsigned char *>(eg->d_mfma) + mats);
        size_t mo = 0, fo = 0;
        auto to_f16 = [](double v) {
            _Float16 hv = (_Float16)(float)v;
            uint16_t u;
            std::memcpy(&u, &hv, 2);
            return u;
        };
        auto to_bf16 = [](double v) {
            float f = (float)v;
            uint32_t u;
            std::memcpy(&u, &f, 4);
            u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
            return (uint16_t)(u >> 16);
        };
        for (int a = 0; a < 3; ++a) {
            const int cnt = eg->count[a];
            eg->view.Ff16[a] = dm + mo;
            eg->view.Bf16[a] = dm + mo + (size_t)cnt * 256;
            eg->view.Fbf16[a] = dm + mo + (size_t)cnt * 512;
            eg->view.Bbf16[a] = dm + mo + (size_t)cnt * 768;
            eg->view.mscale[a] = df + fo;
            eg->view.lmin[a] = df + fo + cnt;
            for (int s = 0; s < cnt; ++s) {
                const double *S = &Sd[a][(size_t)s * nn];
                double smax = 0.0, lmn = lamd[a][(size_t)s * n];
                for (int i = 0; i < nn; ++i) smax = std::max(smax, std::fabs(S[i]));
                for (int i = 0; i < n; ++i) lmn = std::min(lmn, lamd[a][(size_t)s * n + i]);
                for (int o = 0; o < 16; ++o)
                    for (int k2 = 0; k2 < 16; ++k2) {
                        const double fv = (o < n && k2 < n) ? S[k2 * n + o] / smax : 0.0;
                        const double bv = (o < n && k2 < n) ? S[o * n + k2] / smax : 0.0;
                        const size_t e = (size_t)s * 256 + o * 16 + k2;
                        m16[mo + e] = to_f16(fv);
                        m16[mo + (size_t)cnt * 256 + e] = to_f16(bv);
                        m16[mo + (size_t)cnt * 512 + e] = to_bf16(fv);
                        m16[mo + (size_t)cnt * 768 + e] = to_bf16(bv);
                    }
                f32[fo + s] = (float)smax;
                f32[fo + cnt + s] = (float)lmn;
            }
            mo += (size_t)cnt * 1024;
            fo += (size_t)cnt * 2;
        }
        if (hipMemcpy(eg->d_mfma, host16.data(), host16.size(), hipMemcpyHostToDevice) != hipSuccess) {
            dev_free(eg->d_tab);
            dev_free(eg->d_tab32);
            dev_free(eg->d_mfma);
            dev_free(eg->d_cls);
            delete eg;
            return fail(FTS_E_HIP, "upload of the MFMA tables failed");
        }
    }
    if (kind == FTS_VERTEX_PATCH && staging) {
        int64_t nsub = 1;
        for (int a = 0; a < lv->dim; ++a) nsub *= eg->count[a];
        const size_t bytes = (size_t)nsub * (1u << lv->dim) * (lv->ndofs / lv->ncells) * sizeof(double);
        if (dev_malloc(&eg->d_stage, std::max<size_t>(bytes, 8)) != hipSuccess ||
            dev_malloc(&eg->d_stage_scale, (size_t)std::max<int64_t>(nsub, 1) * sizeof(double)) != hipSuccess) {
            if (eg->d_stage) dev_free(eg->d_stage);
            dev_free(eg->d_tab);
            dev_free(eg->d_tab32);
            if (eg->d_mfma) dev_free(eg->d_mfma);
            dev_free(eg->d_cls);
            delete eg;
            return fail(FTS_E_HIP, "device allocation of the patch staging buffer failed");
        }
    }
    *out = eg;
    return FTS_OK;
}

}  // namespace fts

extern "C" {

fts_status fts_set_allocator(fts_alloc_fn alloc, fts_free_fn release, void *ctx) {
    if (!alloc != !release) return fail(FTS_E_INVAL, "fts_set_allocator: give both functions or neither");
    std::lock_guard<std::mutex> lock(g_alloc_mutex);
    g_alloc_fn = alloc;
    g_free_fn = release;
    g_alloc_ctx = ctx;
    return FTS_OK;
}

fts_status fts_setup_1d_eigs(const fts_level *lv, fts_patch_kind kind, fts_eigs **out) {
    return setup_eigs_internal(lv, kind, true, out);
}

fts_status fts_eigs_set_schedule(fts_eigs *eigs, int32_t schedule) {
    if (!eigs) return fail(FTS_E_INVAL, "fts_eigs_set_schedule: NULL handle");
    if (schedule != FTS_SCHEDULE_STAGED && schedule != FTS_SCHEDULE_COLORED && schedule != FTS_SCHEDULE_OWNER &&
        schedule != FTS_SCHEDULE_AUTO)
        return fail(FTS_E_INVAL, "fts_eigs_set_schedule: unknown schedule");
    if (schedule != FTS_SCHEDULE_COLORED && eigs->kind == FTS_VERTEX_PATCH && !eigs->d_stage)
        return fail(FTS_E_INVAL, "fts_eigs_set_schedule: these eigen-data have no staging buffer");
    eigs->schedule = schedule;
    return FTS_OK;
}

fts_status fts_eigs_destroy(fts_eigs *eigs) {
    if (!eigs) return FTS_OK;
    if (eigs->d_tab) dev_free(eigs->d_tab);
    if (eigs->d_tab32) dev_free(eigs->d_tab32);
    if (eigs->d_stage) dev_free(eigs->d_stage);
    if (eigs->d_stage_scale) dev_free(eigs->d_stage_scale);
    if (eigs->d_mfma) dev_free(eigs->d_mfma);
    if (eigs->d_cls) dev_free(eigs->d_cls);
    delete eigs;
    return FTS_OK;
}

int32_t fts_eigs_n(const fts_eigs *eigs) { return eigs ? eigs->n : -1; }

fts_status fts_eigs_get(const fts_eigs *eg, int32_t axis, int32_t index, double *A, double *M,
                        double *S, double *lambda) {
    if (!eg) return fail(FTS_E_INVAL, "fts_eigs_get: NULL handle");
    if (axis < 0 || axis >= eg->level->dim || index < 0 || index >= eg->count[axis])
        return fail(FTS_E_INVAL, "fts_eigs_get: axis or index out of range");
    const int n = eg->n, nn = n * n;
    if (A) std::copy_n(&eg->A[axis][(size_t)index * nn], nn, A);
    if (M) std::copy_n(&eg->M[axis][(size_t)index * nn], nn, M);
    if (S) std::copy_n(&eg->S[axis][(size_t)index * nn], nn, S);
    if (lambda) std::copy_n(&eg->lam[axis][(size_t)index * n], n, lambda);
    return FTS_OK;
}

}  // extern "C"
