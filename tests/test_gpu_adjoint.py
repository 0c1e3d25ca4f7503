"""GPU adjoint of the V-cycle (fts_vcycle_adjoint) and the differentiable
V-cycle iteration, against the oracle's tangent-linear V-cycle and central
finite differences of the GPU forward map (h = 1e-6)."""
import numpy as np
import pytest

from oracle.mesh import Mesh, uniform_mesh, refine
from oracle import sipg, multigrid, tangent
from synthetic import random_vector, loguniform_widths, sine_modes, CONFIGS, uniform_widths
from gpu_util import dev, host, rel, announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1910_11239_amd as fts  # noqa: E402


def _fine(d, k, ms_coarse, nl, seed):
    rng = np.random.default_rng(seed)
    m = Mesh(d, k, loguniform_widths(rng, d, ms_coarse, 0.5, 2.0), 1.0)
    for _ in range(nl - 1):
        m = refine(m)
    return m


@pytest.mark.parametrize("kind,d,k,msc,nl,om", [("vertex", 3, 2, (2, 1, 1), 3, 0.125), ("cell", 2, 3, (2, 2), 3, 0.6),
                                                ("vertex", 2, 4, (1, 2), 3, 0.25), ("vertex", 3, 5, (2, 1, 1), 2, 0.125),
                                                ("cell", 3, 5, (1, 1, 2), 2, 0.6), ("vertex", 2, 8, (1, 2), 3, 0.25)])
def test_vcycle_adjoint_against_oracle_tangents(kind, d, k, msc, nl, om):
    """For a linear functional c.x_out of one V-cycle, the adjoint outputs
    (dL/dx_in, dL/db, dL/domega_l, dL/dgamma_l) contracted with a direction equal
    the oracle's directional derivative along that direction."""
    announce("adjoint one cycle", kind, d, k, msc, nl)
    fine = _fine(d, k, msc, nl, 3)
    omegas = np.array([0.0] + [om] * (nl - 1))
    gammas = np.array([1.2, 0.9, 1.1][:nl])
    oh = multigrid.Hierarchy(fine, nl, kind, omegas, m_pre=2, m_post=2, gamma_hats=gammas)
    th = tangent.TangentHierarchy(oh)
    gh = fts.Hierarchy(d, k, fine.widths, nl, kind, omegas, gammas, 2, 2)
    N = fine.ndofs
    b, x, c = random_vector(N, 0), random_vector(N, 1), random_vector(N, 2)
    lam_b = dev(np.zeros(N))
    lam_x = dev(np.zeros(N))
    dom, dga = gh.vcycle_adjoint(dev(b), dev(x), dev(c), lam_b, lam_x)
    lb, lx = host(lam_b), host(lam_x)
    z = np.zeros(nl)
    # x direction
    dx_dir = random_vector(N, 3)
    _, dxo = th.vcycle(x, dx_dir, b, np.zeros(N), z, z)
    assert abs(lx @ dx_dir - c @ dxo) <= 1e-10 * abs(c @ dxo)
    # b direction
    db_dir = random_vector(N, 4)
    _, dxo = th.vcycle(x, np.zeros(N), b, db_dir, z, z)
    assert abs(lb @ db_dir - c @ dxo) <= 1e-10 * abs(c @ dxo)
    for l in range(nl):
        e = np.zeros(nl)
        e[l] = 1.0
        if l > 0:
            _, dxo = th.vcycle(x, np.zeros(N), b, np.zeros(N), e, z)
            assert abs(dom[l] - c @ dxo) <= 1e-10 * max(1e-300, abs(c @ dxo)), ("omega", l, dom[l], c @ dxo)
        _, dxo = th.vcycle(x, np.zeros(N), b, np.zeros(N), z, e)
        assert abs(dga[l] - c @ dxo) <= 1e-9 * max(1e-300, abs(c @ dxo)), ("gamma", l, dga[l], c @ dxo)


def test_autograd_iterations_small():
    """4 V-cycles, loss ||u_4 - u*||^2 through torch.autograd: gradient in b,
    omega_l, gamma_l vs the oracle tangent and vs central differences (h = 1e-6)
    of the GPU forward map."""
    announce("autograd small")
    d, k, nl = 3, 2, 3
    fine = _fine(d, k, (2, 1, 1), nl, 5)
    N = fine.ndofs
    solver = fts.VCycleIterations(d, k, fine.widths, nl, "vertex", 2, 2, ncycles=4)
    b = dev(random_vector(N, 0)).requires_grad_(True)
    ustar = dev(random_vector(N, 1))
    omegas = torch.tensor([0.0, 0.125, 0.125], dtype=torch.float64, requires_grad=True)
    gammas = torch.tensor([1.0, 1.0, 1.0], dtype=torch.float64, requires_grad=True)
    u = solver(b, omegas, gammas)
    loss = torch.sum((u - ustar) ** 2)
    loss.backward()
    gb, gom, gga = b.grad.detach().cpu().numpy(), omegas.grad.numpy(), gammas.grad.numpy()

    oh = multigrid.Hierarchy(fine, nl, "vertex", omegas.detach().numpy(), m_pre=2, m_post=2,
                             gamma_hats=gammas.detach().numpy())
    th = tangent.TangentHierarchy(oh)
    bn, us = host(b.detach()), host(ustar)
    z = np.zeros(nl)
    db_dir = random_vector(N, 7)
    uu, du = th.iterate(bn, db_dir, z, z, 4)
    assert abs(gb @ db_dir - 2 * (uu - us) @ du) <= 1e-10 * abs(2 * (uu - us) @ du)
    for l in range(nl):
        e = np.zeros(nl)
        e[l] = 1.0
        if l > 0:
            uu, du = th.iterate(bn, np.zeros(N), e, z, 4)
            ref = 2 * (uu - us) @ du
            assert abs(gom[l] - ref) <= 1e-9 * abs(ref), ("omega", l)
        uu, du = th.iterate(bn, np.zeros(N), z, e, 4)
        ref = 2 * (uu - us) @ du
        assert abs(gga[l] - ref) <= 1e-9 * abs(ref), ("gamma", l)

    def L(bv, om, ga):
        with torch.no_grad():
            uu = solver(bv, torch.as_tensor(om), torch.as_tensor(ga))
            return float(torch.sum((uu - ustar) ** 2))

    h = 1e-6
    om0, ga0 = omegas.detach().numpy(), gammas.detach().numpy()
    for l in range(1, nl):
        e = np.zeros(nl)
        e[l] = h
        fd = (L(b.detach(), om0 + e, ga0) - L(b.detach(), om0 - e, ga0)) / (2 * h)
        assert abs(fd - gom[l]) <= 1e-6 * abs(gom[l]) + 1e-9
    e = np.full(nl, h)  # shared penalty factor: sum of the per-level gradients
    fd = (L(b.detach(), om0, ga0 + e) - L(b.detach(), om0, ga0 - e)) / (2 * h)
    assert abs(fd - gga.sum()) <= 1e-6 * abs(gga.sum()) + 1e-9


def test_autograd_interleaved_forwards_keep_their_damping():
    """Two forwards that share a hierarchy (same penalties) but use different
    damping, then the two backwards in reverse order: each gradient is that of
    its own forward map (oracle tangent), and parameters on the GPU get their
    gradients on the GPU."""
    announce("autograd interleaved")
    d, k, nl = 3, 2, 3
    fine = _fine(d, k, (2, 1, 1), nl, 6)
    N = fine.ndofs
    solver = fts.VCycleIterations(d, k, fine.widths, nl, "vertex", 2, 2, ncycles=2)
    ustar = dev(random_vector(N, 1))
    runs = []
    for om in (0.125, 0.08):
        b = dev(random_vector(N, 0)).requires_grad_(True)
        omegas = torch.tensor([0.0, om, om], dtype=torch.float64, device="cuda", requires_grad=True)
        gammas = torch.tensor([1.0, 1.0, 1.0], dtype=torch.float64, device="cuda", requires_grad=True)
        loss = torch.sum((solver(b, omegas, gammas) - ustar) ** 2)
        runs.append((om, b, omegas, gammas, loss))
    for om, b, omegas, gammas, loss in reversed(runs):
        loss.backward()
        assert omegas.grad.device.type == "cuda" and gammas.grad.device.type == "cuda"
        oh = multigrid.Hierarchy(fine, nl, "vertex", [0.0, om, om], m_pre=2, m_post=2, gamma_hats=[1.0] * nl)
        th = tangent.TangentHierarchy(oh)
        bn, us = host(b.detach()), host(ustar)
        z = np.zeros(nl)
        gom = omegas.grad.detach().cpu().numpy()
        for l in range(1, nl):
            e = np.zeros(nl)
            e[l] = 1.0
            uu, du = th.iterate(bn, np.zeros(N), e, z, 2)
            ref = 2 * (uu - us) @ du
            assert abs(gom[l] - ref) <= 1e-9 * abs(ref), ("omega", om, l, gom[l], ref)
        db_dir = random_vector(N, 7)
        uu, du = th.iterate(bn, db_dir, z, z, 2)
        gb = b.grad.detach().cpu().numpy()
        assert abs(gb @ db_dir - 2 * (uu - us) @ du) <= 1e-10 * abs(2 * (uu - us) @ du)


@pytest.mark.slow
def test_adjoint_q5_32_cubed_workload():
    """The 3-D Q5 32^3 workload: 4 V-cycles (32^3/16^3/8^3/4^3, vertex patches,
    omega 2^-3), b = int f phi_i for -Lap u* = f, u* = prod_t sin(pi m_t x_t)
    interpolated, loss ||u_4 - u*||^2.  Gradients in omega_l and the shared
    penalty factor against central differences of the forward map (h = 1e-6),
    and in b along a random direction."""
    cfg = CONFIGS["adjoint_3d_q5"]
    announce("adjoint_3d_q5 full size")
    d, k, m, nl = cfg["dim"], cfg["k"], cfg["m"], cfg["nlevels"]
    mesh = uniform_mesh(d, k, m)
    ms = sine_modes(cfg["seed"], d)
    us_fun = lambda X: np.prod([np.sin(np.pi * ms[a] * X[:, a]) for a in range(d)], axis=0)
    f_fun = lambda X: np.pi ** 2 * sum(mm ** 2 for mm in ms) * us_fun(X)
    ustar = dev(sipg.interpolate(mesh, us_fun))
    b = dev(sipg.rhs(mesh, f_fun)).requires_grad_(True)
    solver = fts.VCycleIterations(d, k, mesh.widths, nl, "vertex", cfg["m_pre"], cfg["m_post"], cfg["ncycles"])
    omegas = torch.tensor([0.0] + [cfg["omega"]] * (nl - 1), dtype=torch.float64, requires_grad=True)
    gammas = torch.full((nl,), cfg["gamma_hat"], dtype=torch.float64, requires_grad=True)
    u = solver(b, omegas, gammas)
    loss = torch.sum((u - ustar) ** 2)
    loss.backward()
    gom, gga = omegas.grad.numpy(), gammas.grad.numpy()

    def L(bv, om, ga):
        with torch.no_grad():
            uu = solver(bv, torch.as_tensor(om), torch.as_tensor(ga))
            return float(torch.sum((uu - ustar) ** 2))

    h = 1e-6
    om0, ga0 = omegas.detach().numpy(), gammas.detach().numpy()
    for l in range(1, nl):
        e = np.zeros(nl)
        e[l] = h
        fd = (L(b.detach(), om0 + e, ga0) - L(b.detach(), om0 - e, ga0)) / (2 * h)
        print("omega", l, "adjoint", gom[l], "fd", fd)
        assert abs(fd - gom[l]) <= 1e-5 * abs(gom[l]) + 1e-12
    e = np.full(nl, h)
    fd = (L(b.detach(), om0, ga0 + e) - L(b.detach(), om0, ga0 - e)) / (2 * h)
    print("gamma (shared)", "adjoint", gga.sum(), "fd", fd)
    assert abs(fd - gga.sum()) <= 1e-5 * abs(gga.sum()) + 1e-12
    dbv = dev(random_vector(mesh.ndofs, 9)) * torch.linalg.norm(b.detach()) / np.sqrt(mesh.ndofs)
    fd = (L(b.detach() + h * dbv, om0, ga0) - L(b.detach() - h * dbv, om0, ga0)) / (2 * h)
    gd = float(torch.dot(b.grad, dbv))
    print("b direction", "adjoint", gd, "fd", fd)
    assert abs(fd - gd) <= 1e-5 * abs(gd) + 1e-12
