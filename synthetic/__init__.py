"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle checks.

This module holds no arithmetic of the method: only mesh geometry (per-axis
cell widths), random vectors and the named workload configurations.  Random
numbers come from numpy's PCG64 ``default_rng(seed)``.

Workloads (the paper measures on the unit square/cube with uniform
refinement, Sec. 2.4; nothing here stands in for a dataset):

* ``acs_2d_q3``      2-D, Q3, 16 x 16 uniform cells of [0,1]^2, additive cell
                     smoother, omega = 0.7, penalty 2.5 k(k+1)/h on every face.
* ``avs_3d_q4``      3-D, Q4, 32^3 uniform cells of [0,1]^3, additive vertex-patch
                     smoother omega = 0.5 in a 3-level V-cycle, 2 pre/post sweeps,
                     dense LU on the 8^3 coarse mesh.
* ``mixed_3d_q7``    3-D, Q7, 48^3 uniform cells, vertex patches, FP64 CG to 1e-10.
* ``batched``        64 meshes, cube counts m ~ U{8..24}, degrees k ~ U{2..9},
                     per-slab widths log-uniform in [0.25, 4].
* ``adjoint_3d_q5``  3-D, Q5, 32^3, 4 V-cycles, smooth product-of-sines target.

The penalty factor gamma_hat of eq. (penalty) is 1 (the paper's choice for
Cartesian meshes) except for ``acs_2d_q3``, whose stated penalty 2.5 k(k+1)/h
on a uniform mesh means gamma_hat (1/h + 1/h) = 2.5/h, i.e. gamma_hat = 1.25.
"""
import numpy as np

CONFIGS = {
    "acs_2d_q3": dict(dim=2, k=3, m=16, gamma_hat=1.25, kind="cell", omega=0.7,
                      seed_b=0, seed_x=1),
    "avs_3d_q4": dict(dim=3, k=4, m=32, gamma_hat=1.0, kind="vertex", omega=0.5,
                      nlevels=3, m_pre=2, m_post=2, seed_b=0, seed_x=1),
    "mixed_3d_q7": dict(dim=3, k=7, m=48, gamma_hat=1.0, kind="vertex", omega=0.125,
                        nlevels=5, m_pre=2, m_post=2, rtol=1e-10, seed_b=0),
    "batched": dict(dim=3, nmesh=64, m_range=(8, 24), k_range=(2, 9),
                    width_range=(0.25, 4.0), seed=0),
    "adjoint_3d_q5": dict(dim=3, k=5, m=32, gamma_hat=1.0, kind="vertex", omega=0.125,
                          nlevels=4, m_pre=2, m_post=2, ncycles=4, seed=0),
}


def uniform_widths(dim, m, length=1.0):
    ms = (m,) * dim if np.isscalar(m) else tuple(m)
    return tuple(np.full(mm, length / mm) for mm in ms)


def loguniform_widths(rng, dim, m, lo, hi, paired=False):
    """Per-axis slab widths, log-uniform in [lo, hi].  paired=True repeats each
    width twice (halved) so the mesh can be coarsened by merging pairs."""
    ms = (m,) * dim if np.isscalar(m) else tuple(m)
    out = []
    for mm in ms:
        if paired:
            if mm % 2:
                raise ValueError("paired widths need an even cell count")
            w = np.exp(rng.uniform(np.log(lo), np.log(hi), mm // 2))
            out.append(np.repeat(w / 2.0, 2))
        else:
            out.append(np.exp(rng.uniform(np.log(lo), np.log(hi), mm)))
    return tuple(out)


def random_vector(n, seed):
    """i.i.d. uniform[-1, 1] entries, PCG64 seeded."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def batched_meshes(cfg=None):
    """The mixed-degree anisotropic batch: list of (k, widths) in mesh order."""
    cfg = cfg or CONFIGS["batched"]
    rng = np.random.default_rng(cfg["seed"])
    out = []
    lo_m, hi_m = cfg["m_range"]
    lo_k, hi_k = cfg["k_range"]
    for _ in range(cfg["nmesh"]):
        m = int(rng.integers(lo_m, hi_m + 1))
        k = int(rng.integers(lo_k, hi_k + 1))
        w = loguniform_widths(rng, cfg["dim"], m, *cfg["width_range"])
        out.append((k, w))
    return out


def grid_vertices(widths):
    """Vertex coordinates (prod(m+1), d) of the rectilinear grid with these
    per-axis cell widths, x fastest (origin at 0)."""
    coords = [np.concatenate(([0.0], np.cumsum(np.asarray(w, dtype=np.float64)))) for w in widths]
    grids = np.meshgrid(*reversed(coords), indexing="ij")
    return np.stack([g.ravel() for g in reversed(grids)], axis=1)


def distorted_vertices(dim, m, levels, distortion, seed):
    """Distorted meshes of the unit square / cube (the test meshes of Sec. 4):
    a uniform grid of m cells per axis whose interior vertices are moved by
    distortion * h_v in a random direction (h_v the shortest edge at the
    vertex, directions uniform on the sphere, numpy PCG64 from seed), then
    refined `levels` times by splitting every cell at the midpoints of its
    reference cell (new vertices on the multilinear cell map).  Returns the
    cells per axis and the vertex array (prod(m+1), d), x fastest."""
    rng = np.random.default_rng(seed)
    ms = (m,) * dim
    X = grid_vertices([np.full(m, 1.0 / m)] * dim).reshape(tuple(mm + 1 for mm in reversed(ms)) + (dim,))
    shape = X.shape[:-1]
    out = X.copy()
    for idx in np.ndindex(*shape):
        if any(i == 0 or i == n - 1 for i, n in zip(idx, shape)):
            continue
        hv = np.inf
        for a in range(dim):
            for s in (-1, 1):
                nb = list(idx)
                nb[a] += s
                hv = min(hv, float(np.linalg.norm(X[tuple(nb)] - X[idx])))
        direction = rng.normal(size=dim)
        out[idx] = X[idx] + distortion * hv * direction / np.linalg.norm(direction)
    X = out
    for _ in range(levels):
        shape = X.shape[:-1]
        fine_shape = tuple(2 * (n - 1) + 1 for n in shape)
        F = np.zeros(fine_shape + (dim,))
        for fidx in np.ndindex(*fine_shape):
            c = [min(f // 2, n - 2) for f, n in zip(fidx, shape)]
            xi = [(f - 2 * cc) / 2.0 for f, cc in zip(fidx, c)]
            p = np.zeros(dim)
            for corner in np.ndindex(*([2] * dim)):
                wgt = np.prod([xi[a] if corner[a] else 1.0 - xi[a] for a in range(dim)])
                p += wgt * X[tuple(c[a] + corner[a] for a in range(dim))]
            F[fidx] = p
        X = F
        ms = tuple(2 * mm for mm in ms)
    # X is indexed [v_{d-1}, ..., v_0]: flatten with v_0 fastest
    return ms, X.reshape(-1, dim)


def sine_modes(seed, dim):
    """Integer frequencies m_t in 1..4 of the smooth target prod_t sin(pi m_t x_t)."""
    return tuple(int(v) for v in np.random.default_rng(seed).integers(1, 5, dim))
