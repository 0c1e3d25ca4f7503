"""Pin the oracle's tangent-linear V-cycle against central finite differences of
the oracle's forward map (rebuilt with perturbed damping / penalty)."""
import numpy as np
import pytest

from oracle.mesh import uniform_mesh, refine
from oracle import multigrid, tangent
from synthetic import random_vector


def _setup(kind, d, k, m0, nl, omega, gamma):
    fine = uniform_mesh(d, k, m0)
    for _ in range(nl - 1):
        fine = refine(fine)
    return fine


def _loss(fine, nl, kind, omegas, gammas, b, ustar, ncycles):
    h = multigrid.Hierarchy(fine, nl, kind, omegas, m_pre=2, m_post=2, gamma_hats=gammas)
    u = np.zeros_like(b)
    for _ in range(ncycles):
        u = h.vcycle(u, b)
    return float(np.sum((u - ustar) ** 2)), u


@pytest.mark.parametrize("kind,d,k,m0,nl", [("vertex", 2, 2, 2, 2), ("cell", 2, 3, 2, 3)])
def test_tangent_matches_central_differences(kind, d, k, m0, nl):
    fine = _setup(kind, d, k, m0, nl, 0.2, 1.0)
    omegas = np.array([0.0] + [0.2 if kind == "vertex" else 0.6] * (nl - 1))
    gammas = np.array([1.1, 1.3, 0.9][:nl])
    b = random_vector(fine.ndofs, 0)
    ustar = random_vector(fine.ndofs, 1)
    ncycles = 2
    h = multigrid.Hierarchy(fine, nl, kind, omegas, m_pre=2, m_post=2, gamma_hats=gammas)
    th = tangent.TangentHierarchy(h)
    L0, u = _loss(fine, nl, kind, omegas, gammas, b, ustar, ncycles)
    eps = 1e-6
    # directions: one per parameter and a random b direction
    dirs = [("b", random_vector(fine.ndofs, 2), np.zeros(nl), np.zeros(nl))]
    for l in range(1, nl):
        e = np.zeros(nl)
        e[l] = 1.0
        dirs.append((f"omega{l}", np.zeros(fine.ndofs), e, np.zeros(nl)))
    for l in range(nl):
        e = np.zeros(nl)
        e[l] = 1.0
        dirs.append((f"gamma{l}", np.zeros(fine.ndofs), np.zeros(nl), e))
    for name, db, dom, dga in dirs:
        uu, du = th.iterate(b, db, dom, dga, ncycles)
        assert np.allclose(uu, u, rtol=1e-13, atol=1e-13)
        dL = 2 * (uu - ustar) @ du
        Lp, _ = _loss(fine, nl, kind, omegas + eps * dom, gammas + eps * dga, b + eps * db, ustar, ncycles)
        Lm, _ = _loss(fine, nl, kind, omegas - eps * dom, gammas - eps * dga, b - eps * db, ustar, ncycles)
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - dL) <= 1e-6 * max(1.0, abs(dL)), (name, fd, dL)
