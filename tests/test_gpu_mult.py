"""GPU parity of the multiplicative Schwarz smoothers (Alg. multsmoother with
red-black cells and the 2^(d+1) vertex-patch colors), the V-cycle built on
them, and GMRES with that V-cycle as preconditioner, against the FP64 oracle
on the same seeded inputs.  Bar: 1e-12 relative in FP64 for smoother and
V-cycle; GMRES: same iteration count, residual histories equal to 1e-9 and
the solution of the discrete system."""
import numpy as np
import pytest

from oracle.mesh import Mesh, uniform_mesh, refine
from oracle import sipg, onedim, schwarz, multigrid, krylov
from synthetic import loguniform_widths, random_vector
from gpu_util import dev, host, rel, rel2, announce

pytestmark = pytest.mark.gpu
TOL = 1e-12

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1910_11239_amd as fts  # noqa: E402


def omesh(d, k, ms, seed):
    rng = np.random.default_rng(seed)
    return Mesh(d, k, loguniform_widths(rng, d, ms, 0.25, 4.0))


def oracle_colors(kind, m):
    return schwarz.cell_red_black(m) if kind == "cell" else schwarz.vertex_patch_mult_colors(m)


# kernel paths: 2-D and 3-D cells with several subdomains per workgroup, 2-D
# patches, 3-D patches one per workgroup (k = 2, 3, 7), ragged subdomain grids
MULT_CASES = [("cell", 2, 3, (5, 4)), ("cell", 3, 2, (3, 4, 3)), ("cell", 3, 7, (2, 3, 2)),
              ("vertex", 2, 2, (5, 6)), ("vertex", 3, 2, (4, 5, 3)), ("vertex", 3, 3, (5, 4, 4)),
              ("vertex", 3, 7, (3, 3, 4))]


@pytest.mark.parametrize("kind,d,k,ms", MULT_CASES)
def test_mult_smoother_parity(kind, d, k, ms):
    announce("mult smoother", kind, d, k, ms)
    m = omesh(d, k, ms, 31)
    A = sipg.assemble(m)
    subs = schwarz.cell_subdomains(m) if kind == "cell" else schwarz.vertex_patch_subdomains(m)
    sol = schwarz.ExactLocalSolvers(A, subs, cache=False)
    x, b = random_vector(m.ndofs, 1), random_vector(m.ndofs, 0)
    omega = 0.9
    ref = schwarz.multiplicative_smooth(A, sol, x, b, omega, oracle_colors(kind, m))
    ref2 = schwarz.multiplicative_smooth(A, sol, ref, b, omega, oracle_colors(kind, m))
    lv = fts.Level(d, k, m.widths, m.gamma_hat)
    eg = fts.Eigs(lv, kind)
    xg = dev(x)
    fts.schwarz_smooth_mult(lv, eg, omega, dev(b), xg, nsweeps=1)
    assert rel(host(xg), ref) < TOL
    fts.schwarz_smooth_mult(lv, eg, omega, dev(b), xg, nsweeps=1)
    assert rel(host(xg), ref2) < TOL


@pytest.mark.parametrize("prec,bound", [("f32", 1e-4), ("f16", 1.5e-3), ("bf16", 1.2e-2)])
def test_mult_smoother_reduced_precision(prec, bound):
    """Reduced-precision contractions in the multiplicative vertex-patch smoother:
    error of the correction against the FP64 oracle within the bounds of the
    additive smoother's tests."""
    announce("mult smoother", prec)
    m = omesh(3, 4, (4, 3, 4), 32)
    A = sipg.assemble(m)
    sol = schwarz.ExactLocalSolvers(A, schwarz.vertex_patch_subdomains(m), cache=False)
    x, b = random_vector(m.ndofs, 1), random_vector(m.ndofs, 0)
    ref = schwarz.multiplicative_smooth(A, sol, x, b, 0.8, schwarz.vertex_patch_mult_colors(m))
    lv = fts.Level(3, 4, m.widths, m.gamma_hat)
    eg = fts.Eigs(lv, "vertex")
    xg = dev(x)
    fts.schwarz_smooth_mult(lv, eg, 0.8, dev(b), xg, nsweeps=1, prec=prec)
    err = rel2(host(xg) - x, ref - x)
    print(prec, "relative error of the correction", err)
    assert err < bound


def hierarchies(kind, d, k, ms, nl, omega, seed, smoother="multiplicative"):
    fine = omesh(d, k, tuple(mm >> (nl - 1) for mm in ms), seed)
    for _ in range(nl - 1):
        fine = refine(fine)
    omegas = [0.0] + [omega] * (nl - 1)
    oh = multigrid.Hierarchy(fine, nl, kind, omegas, m_pre=1, m_post=1, cache=False, smoother=smoother)
    gh = fts.Hierarchy(d, k, fine.widths, nl, kind, omegas, fine.gamma_hat, m_pre=1, m_post=1)
    gh.set_smoother(smoother)
    return fine, oh, gh


@pytest.mark.parametrize("smoother", ["multiplicative", "multiplicative_symmetric"])
@pytest.mark.parametrize("kind,d,k,ms,nl", [("vertex", 3, 2, (8, 4, 4), 3), ("cell", 2, 3, (8, 12), 3),
                                            ("vertex", 2, 4, (8, 8), 3)])
def test_vcycle_mult_parity(kind, d, k, ms, nl, smoother):
    announce("mult vcycle", smoother, kind, d, k, ms, nl)
    fine, oh, gh = hierarchies(kind, d, k, ms, nl, 1.0, 33, smoother)
    b, x = random_vector(fine.ndofs, 0), random_vector(fine.ndofs, 1)
    ref = oh.vcycle(x.copy(), b)
    xg = dev(x)
    gh.vcycle(dev(b), xg)
    assert rel(host(xg), ref) < TOL


@pytest.mark.parametrize("kind,d,k,ms,nl,restart", [("vertex", 3, 2, (8, 8, 8), 3, 30), ("cell", 2, 3, (16, 16), 3, 5)])
def test_gmres_mult_vcycle(kind, d, k, ms, nl, restart):
    """GMRES preconditioned by the multiplicative V-cycle (Sec. 2.4): same
    iteration count and residual history as the oracle's GMRES with the
    oracle's V-cycle, and the solution of the discrete system (exact solution
    by global fast diagonalisation on a uniform mesh)."""
    announce("gmres", kind, d, k, ms, nl, restart)
    fine = uniform_mesh(d, k, tuple(mm >> (nl - 1) for mm in ms))
    for _ in range(nl - 1):
        fine = refine(fine)
    omegas = [0.0] + [1.0] * (nl - 1)
    oh = multigrid.Hierarchy(fine, nl, kind, omegas, m_pre=1, m_post=1, smoother="multiplicative")
    b = random_vector(fine.ndofs, 0)
    xo, ito, histo = krylov.gmres(oh.A[-1], b, lambda v: oh.vcycle(np.zeros_like(v), v), restart=restart,
                                  rtol=1e-10, maxit=200)
    gh = fts.Hierarchy(d, k, fine.widths, nl, kind, omegas, fine.gamma_hat, m_pre=1, m_post=1)
    gh.set_smoother("multiplicative")
    xg = dev(np.zeros(fine.ndofs))
    it, relres, hist = gh.gmres(dev(b), xg, rtol=1e-10, restart=restart, maxit=200)
    print("gmres iterations gpu", it, "oracle", ito, "final", relres)
    assert it == ito and relres <= 1e-10
    nh = min(8, len(hist), len(histo))
    assert np.allclose(hist[:nh], histo[:nh], rtol=1e-9, atol=1e-14)
    xs = onedim.global_fastdiag_solve(fine, b)
    assert rel(host(xg), xs) < 1e-8
    assert rel(host(xg), xo) < 1e-8


def test_gmres_additive_vcycle_agrees_with_pcg():
    """With the additive V-cycle GMRES and PCG solve the same system."""
    fine = uniform_mesh(3, 3, (4, 4, 4))
    fine = refine(fine)
    gh = fts.Hierarchy(3, 3, fine.widths, 2, "vertex", [0.0, 0.125], 1.0, m_pre=2, m_post=2)
    b = dev(random_vector(fine.ndofs, 0))
    xg = dev(np.zeros(fine.ndofs))
    xc = dev(np.zeros(fine.ndofs))
    itg, relg, _ = gh.gmres(b, xg, rtol=1e-10, restart=30, maxit=200)
    itc, relc, _ = gh.pcg(b, xc, rtol=1e-10, maxit=200)
    assert relg <= 1e-10 and relc <= 1e-10
    assert rel(host(xg), host(xc)) < 1e-8


@pytest.mark.parametrize("kind,d,k,ms,nl", [("cell", 3, 3, (8, 8, 8), 3), ("vertex", 3, 2, (8, 8, 8), 3),
                                            ("cell", 2, 4, (16, 16), 3)])
def test_pcg_with_symmetrised_multiplicative_vcycle(kind, d, k, ms, nl):
    """The symmetrised multiplicative V-cycle (colors reversed in
    post-smoothing) preconditions CG: the library's PCG reaches 1e-10 with
    the oracle's iteration count and residual history (oracle PCG with the
    oracle's symmetrised V-cycle), and the solution is the discrete one."""
    announce("pcg symmetric mult", kind, d, k, ms, nl)
    fine = uniform_mesh(d, k, tuple(mm >> (nl - 1) for mm in ms))
    for _ in range(nl - 1):
        fine = refine(fine)
    omegas = [0.0] + [1.0] * (nl - 1)
    oh = multigrid.Hierarchy(fine, nl, kind, omegas, m_pre=1, m_post=1, smoother="multiplicative_symmetric")
    b = random_vector(fine.ndofs, 0)
    xo, ito, histo = krylov.pcg(oh.A[-1], b, lambda v: oh.vcycle(np.zeros_like(v), v), rtol=1e-10, maxit=200,
                                flexible=True)
    gh = fts.Hierarchy(d, k, fine.widths, nl, kind, omegas, fine.gamma_hat, m_pre=1, m_post=1)
    gh.set_smoother("multiplicative_symmetric")
    xg = dev(np.zeros(fine.ndofs))
    it, relres, hist = gh.pcg(dev(b), xg, rtol=1e-10, maxit=200)
    print("pcg iterations gpu", it, "oracle", ito, "final", relres)
    assert relres <= 1e-10 and abs(it - ito) <= 1
    nh = min(6, len(hist), len(histo))
    assert np.allclose(hist[:nh], histo[:nh], rtol=1e-8, atol=1e-14)
    xs = onedim.global_fastdiag_solve(fine, b)
    assert rel(host(xg), xs) < 1e-8
