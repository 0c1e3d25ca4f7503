"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded inputs.

Bar (FP64): ||gpu - oracle||_2 / ||oracle||_2 <= 1e-12 per output vector; the
oracle assembles the SIPG matrix by quadrature and solves local problems by
dense LU, the GPU uses sum factorisation and fast diagonalisation.  Meshes are
rectilinear with log-uniform random widths in [0.25, 4] and cell counts that
leave ragged tails for the per-block batching of the kernels.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.mesh import Mesh, uniform_mesh
from oracle import sipg, onedim, schwarz, multigrid
from synthetic import loguniform_widths, random_vector, uniform_widths, CONFIGS
from gpu_util import dev, host, rel, rel2, announce

pytestmark = pytest.mark.gpu
TOL = 1e-12

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1910_11239_amd as fts  # noqa: E402


def omesh(d, k, ms, seed, gamma_hat=1.0, paired=False):
    rng = np.random.default_rng(seed)
    return Mesh(d, k, loguniform_widths(rng, d, ms, 0.25, 4.0, paired=paired), gamma_hat)


def glevel(m):
    return fts.Level(m.dim, m.k, m.widths, m.gamma_hat)


OP_CASES = [(2, 1, (5, 3)), (2, 3, (5, 4)), (2, 5, (4, 3)), (2, 8, (3, 4)), (2, 9, (3, 2)), (2, 12, (3, 2)),
            (2, 15, (2, 3)), (3, 1, (4, 3, 5)),
            (3, 2, (3, 4, 3)), (3, 4, (4, 3, 5)), (3, 5, (3, 4, 2)), (3, 6, (2, 3, 3)), (3, 7, (3, 2, 3)),
            (3, 8, (2, 3, 2)), (3, 9, (2, 2, 3))]


@pytest.mark.parametrize("d,k,ms", OP_CASES)
def test_operator_and_residual(d, k, ms):
    announce("operator", d, k, ms)
    m = omesh(d, k, ms, 11, gamma_hat=1.3)
    A = sipg.assemble(m)
    x, b = random_vector(m.ndofs, 1), random_vector(m.ndofs, 0)
    lv = glevel(m)
    y = dev(np.zeros(m.ndofs))
    lv.apply(dev(x), y)
    assert rel(host(y), A @ x) < TOL
    r = dev(np.zeros(m.ndofs))
    lv.residual(dev(b), dev(x), r)
    assert rel(host(r), b - A @ x) < TOL


@pytest.mark.parametrize("kind", ["cell", "vertex"])
@pytest.mark.parametrize("d,k,ms", [(2, 3, (4, 3)), (3, 2, (3, 4, 3)), (3, 4, (2, 3, 2))])
def test_setup_1d_eigs(kind, d, k, ms):
    announce("eigs", kind, d, k, ms)
    m = omesh(d, k, ms, 12, gamma_hat=1.25)
    lv = glevel(m)
    eg = fts.Eigs(lv, kind)
    ref = onedim.Ref1D(k)
    for a in range(d):
        npos = m.ncells[a] if kind == "cell" else m.ncells[a] - 1
        for s in range(npos):
            A, M, S, lam = eg.get(a, s)
            ws, lo, hi = onedim.axis_chain(m, a, s, 1 if kind == "cell" else 2)
            A0, M0 = onedim.chain_operator(ref, ws, lo, hi, m.gamma_hat)
            assert np.abs(A - A0).max() <= 1e-13 * np.abs(A0).max()
            assert np.abs(M - M0).max() <= 1e-14 * np.abs(M0).max()
            assert np.abs(S.T @ M0 @ S - np.eye(len(lam))).max() < 1e-12
            assert np.abs(S.T @ A0 @ S - np.diag(lam)).max() < 1e-12 * lam.max()
            assert np.allclose(lam, sla.eigh(A0, M0, eigvals_only=True), rtol=1e-12, atol=0)


SMOOTH_CASES = [("cell", 2, 3, (5, 4)), ("cell", 3, 4, (3, 4, 3)), ("cell", 3, 5, (3, 2, 3)),
                ("cell", 3, 8, (2, 3, 2)), ("cell", 3, 9, (2, 2, 1)),
                ("vertex", 2, 3, (5, 4)), ("vertex", 2, 5, (4, 3)), ("vertex", 2, 8, (3, 4)),
                ("vertex", 2, 9, (3, 3)), ("cell", 2, 11, (3, 2)), ("cell", 2, 15, (2, 3)),
                ("vertex", 2, 13, (3, 3)), ("vertex", 2, 15, (3, 2)), ("vertex", 3, 1, (5, 4, 3)),
                ("vertex", 3, 2, (4, 3, 5)), ("vertex", 3, 4, (3, 4, 3)), ("vertex", 3, 5, (3, 4, 3)),
                ("vertex", 3, 6, (3, 3, 2)), ("vertex", 3, 7, (3, 4, 3)),  # k = 7: FP64 MFMA local solves
                ("vertex", 3, 8, (3, 2, 3))]


@pytest.mark.parametrize("kind,d,k,ms", SMOOTH_CASES)
def test_schwarz_smooth(kind, d, k, ms):
    announce("smooth", kind, d, k, ms)
    m = omesh(d, k, ms, 13)
    A = sipg.assemble(m)
    subs = schwarz.cell_subdomains(m) if kind == "cell" else schwarz.vertex_patch_subdomains(m)
    sol = schwarz.ExactLocalSolvers(A, subs, cache=False)
    x, b = random_vector(m.ndofs, 1), random_vector(m.ndofs, 0)
    omega = 0.7 if kind == "cell" else 0.3
    x1 = schwarz.additive_smooth(A, sol, x, b, omega)
    x2 = schwarz.additive_smooth(A, sol, x1, b, omega)
    lv = glevel(m)
    eg = fts.Eigs(lv, kind)
    r = b - A @ x
    for schedule in (("staged", "colored") if kind == "vertex" else ("staged",)):
        eg.set_schedule(schedule)
        xg = dev(x)
        fts.schwarz_smooth(lv, eg, omega, dev(b), xg, nsweeps=1)
        assert rel(host(xg), x1) < TOL, schedule
        fts.schwarz_smooth(lv, eg, omega, dev(b), xg, nsweeps=1)
        assert rel(host(xg), x2) < TOL, schedule
        # local-solver part alone
        xa = dev(np.zeros(m.ndofs))
        fts.schwarz_apply(lv, eg, 1.0, dev(r), xa)
        assert rel(host(xa), sol.apply(r)) < TOL, schedule


@pytest.mark.parametrize("kind,k,widths", [("vertex", 3, "uniform"), ("vertex", 3, "mirrored"),
                                            ("vertex", 4, "uniform"), ("vertex", 4, "mirrored"),
                                            ("cell", 7, "uniform")])
def test_schwarz_mirror_symmetric_positions(kind, k, widths):
    """Positions whose 1-D problem is mirror symmetric (equal widths on both
    sides) are contracted in even-odd form: on a uniform mesh every interior
    position; on the mirrored widths (x, y: 1 1 2 2 1 1, z: 0.5 1 1 0.5) one
    position per axis, next to positions that are not.  Same bar as every
    FP64 smoother result, and the FP32 contractions within the FP32 bound."""
    announce("mirror", kind, k, widths)
    if widths == "uniform":
        m = uniform_mesh(3, k, (5, 4, 5) if kind == "vertex" else (3, 3, 3))
    else:
        wx, wz = np.array([1.0, 1.0, 2.0, 2.0, 1.0, 1.0]), np.array([0.5, 1.0, 1.0, 0.5])
        m = Mesh(3, k, (wx / wx.sum(), wx / wx.sum(), wz / wz.sum()), 1.0)
    A = sipg.assemble(m)
    subs = schwarz.cell_subdomains(m) if kind == "cell" else schwarz.vertex_patch_subdomains(m)
    sol = schwarz.ExactLocalSolvers(A, subs, cache=False)
    x, b = random_vector(m.ndofs, 1), random_vector(m.ndofs, 0)
    omega = 0.7 if kind == "cell" else 0.3
    ref = schwarz.additive_smooth(A, sol, x, b, omega)
    lv = glevel(m)
    eg = fts.Eigs(lv, kind)
    xg = dev(x)
    fts.schwarz_smooth(lv, eg, omega, dev(b), xg, nsweeps=1)
    assert rel(host(xg), ref) < TOL
    xg = dev(x)
    fts.schwarz_smooth(lv, eg, omega, dev(b), xg, nsweeps=1, prec="f32")
    assert rel2(host(xg) - x, ref - x) < 1e-4


@pytest.mark.parametrize("k,m,cz,widths", [(3, 25, 2, "random"), (4, 32, 4, "uniform"), (3, 48, 8, "random"),
                                           (7, 26, 2, "uniform"), (7, 34, 4, "random"), (6, 17, 1, "random")])
def test_staged_runs_along_z_match_colored(k, m, cz, widths):
    """Launches with many vertex patches stage runs of cz patches along z and
    merge the cell layer two neighbours of a run share (cz = 2, 4, 8 at these
    sizes, which are too large for the oracle; k = 7 in FP64 runs on the FP64
    MFMA kernel): the staged result equals the colored schedule, which adds
    each patch to x directly, up to rounding order; the same with FP32 and
    16-bit MFMA contractions (whose run kernel stores the values with their
    scale factor applied).  The owner-computes tiles (16-bit only; other
    precisions fall back to staging) agree as well, here with ragged tiles
    and z-segments.  All schedules are checked against the oracle on small
    meshes above."""
    announce("zrun", k, m, cz, widths)
    rng = np.random.default_rng(23)
    ws = uniform_widths(3, (m, m, m)) if widths == "uniform" else loguniform_widths(rng, 3, (m, m, m), 0.25, 4.0)
    lv = fts.Level(3, k, ws, 1.0)
    eg = fts.Eigs(lv, "vertex")
    r = dev(random_vector(lv.ndofs, 2))
    for prec, tol in (("f64", 1e-13), ("f32", 1e-6), ("f16", 1e-6), ("bf16", 1e-6)):
        out = {}
        for schedule in ("staged", "colored", "owner"):
            eg.set_schedule(schedule)
            xa = dev(np.zeros(lv.ndofs))
            fts.schwarz_apply(lv, eg, 0.5, r, xa, prec)
            out[schedule] = host(xa)
        assert rel2(out["staged"], out["colored"]) < tol, prec
        # the owner tiles contract in the transposed orientation (other FP32
        # summation order inside the MFMA), so a 16-bit rounding of an
        # intermediate value comes out one unit apart now and then: about
        # 1e-5 in the 2-norm, far below the 16-bit error against the oracle
        # (checked on small meshes and at full size)
        tol_owner = tol if prec in ("f64", "f32") else 1e-4
        assert rel2(out["owner"], out["colored"]) < tol_owner, prec


def test_staged_schedule_is_deterministic():
    """Repeated staged applications give bit-identical results."""
    m = omesh(3, 3, (5, 4, 3), 19)
    lv = glevel(m)
    eg = fts.Eigs(lv, "vertex")
    r = dev(random_vector(m.ndofs, 2))
    outs = []
    for _ in range(3):
        xa = dev(np.zeros(m.ndofs))
        fts.schwarz_apply(lv, eg, 0.5, r, xa)
        outs.append(host(xa))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_staged_gather_with_unaligned_x(prec):
    """x given as a view one element into a larger buffer (no longer aligned for
    the gather's vector loads): same result as an aligned x (same arithmetic in
    the same order; compared to 1e-14 in case the compiler contracts the two
    variants differently), and the neighbouring entries untouched."""
    announce("unaligned x", prec)
    m = omesh(3, 3, (4, 3, 3), 23)  # (k+1)^3 = 64 DoFs per cell: vector width 4
    lv = glevel(m)
    eg = fts.Eigs(lv, "vertex")
    r = dev(random_vector(m.ndofs, 2))
    x0 = random_vector(m.ndofs, 3)
    xa = dev(x0)
    fts.schwarz_apply(lv, eg, 0.5, r, xa, prec=prec)
    buf = dev(np.concatenate([[7.0], x0, [9.0]]))
    xv = buf[1:m.ndofs + 1]
    assert xv.data_ptr() % 16 != 0
    fts.schwarz_apply(lv, eg, 0.5, r, xv, prec=prec)
    hb = host(buf)
    assert rel(hb[1:m.ndofs + 1], host(xa)) < 1e-14
    assert hb[0] == 7.0 and hb[-1] == 9.0


@pytest.mark.parametrize("d,k", [(2, 4), (3, 9)])
def test_one_patch_mesh_is_exact_solve(d, k):
    """2^d-cell mesh: one vertex patch, omega = 1 gives A^-1 b (largest degree)."""
    announce("one patch", d, k)
    m = omesh(d, k, (2,) * d, 14)
    A = sipg.assemble(m)
    b = random_vector(m.ndofs, 0)
    lv = glevel(m)
    eg = fts.Eigs(lv, "vertex")
    xg = dev(random_vector(m.ndofs, 1))
    fts.schwarz_smooth(lv, eg, 1.0, dev(b), xg, nsweeps=1)
    xs = host(xg)
    assert np.linalg.norm(A @ xs - b) < 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("d,k,ms", [(2, 5, (1, 1)), (3, 3, (1, 1, 1))])
def test_one_cell_mesh_is_exact_solve(d, k, ms):
    """Degenerate mesh of one cell (every face on the boundary): the cell
    smoother with omega = 1 is the exact solve A^-1 b, and the residual is
    the assembled one."""
    announce("one cell", d, k)
    m = omesh(d, k, ms, 15)
    A = sipg.assemble(m)
    b, x0 = random_vector(m.ndofs, 0), random_vector(m.ndofs, 1)
    lv = glevel(m)
    r = dev(np.zeros(m.ndofs))
    lv.residual(dev(b), dev(x0), r)
    assert rel(host(r), b - A @ x0) < 1e-12
    eg = fts.Eigs(lv, "cell")
    xg = dev(x0)
    fts.schwarz_smooth(lv, eg, 1.0, dev(b), xg, nsweeps=1)
    assert np.linalg.norm(A @ host(xg) - b) < 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("d,k,ms", [(3, 2, (1, 3, 3)), (2, 3, (5, 1))])
def test_vertex_patches_need_two_cells_per_axis(d, k, ms):
    """A mesh with a single cell along some axis has no interior vertex (the
    oracle finds no vertex patch): the library refuses vertex-patch tables
    for it with an error instead of returning an empty smoother, and the
    cell smoother on the same mesh works."""
    announce("no patches", d, k, ms)
    m = omesh(d, k, ms, 16)
    assert len(schwarz.vertex_patch_subdomains(m)) == 0
    lv = glevel(m)
    with pytest.raises(fts.FtsError, match="at least 2 cells"):
        fts.Eigs(lv, "vertex")
    eg = fts.Eigs(lv, "cell")
    A = sipg.assemble(m)
    sol = schwarz.ExactLocalSolvers(A, schwarz.cell_subdomains(m), cache=False)
    b, x0 = random_vector(m.ndofs, 0), random_vector(m.ndofs, 1)
    ref = schwarz.additive_smooth(A, sol, x0, b, 0.7)
    xg = dev(x0)
    fts.schwarz_smooth(lv, eg, 0.7, dev(b), xg, nsweeps=1)
    assert rel(host(xg), ref) < 1e-12


@pytest.mark.parametrize("d,k,ms", [(2, 3, (3, 2)), (3, 2, (2, 3, 2)), (3, 4, (1, 2, 2)), (3, 9, (1, 1, 2)),
                                    (2, 11, (2, 3)), (2, 15, (2, 2))])
def test_transfers(d, k, ms):
    announce("transfer", d, k, ms)
    mc = omesh(d, k, ms, 15)
    from oracle.mesh import refine
    mf = refine(mc)
    P = multigrid.prolongation(mc, mf)
    lc, lf = glevel(mc), glevel(mf)
    ec, rf = random_vector(mc.ndofs, 2), random_vector(mf.ndofs, 3)
    xf0 = random_vector(mf.ndofs, 4)
    xg = dev(xf0)
    fts.prolongate_add(lc, lf, dev(ec), xg)
    assert rel(host(xg), xf0 + P @ ec) < TOL
    bc = dev(np.zeros(mc.ndofs))
    fts.restrict(lc, lf, dev(rf), bc)
    assert rel(host(bc), P.T @ rf) < TOL


@pytest.mark.parametrize("kind,d,k,ms,nl", [("vertex", 3, 2, (8, 4, 4), 3), ("cell", 2, 3, (8, 8), 3),
                                            ("vertex", 2, 4, (8, 4), 3), ("vertex", 3, 4, (4, 4, 4), 2),
                                            ("vertex", 3, 5, (4, 4, 4), 2), ("cell", 3, 5, (4, 4, 2), 2),
                                            ("vertex", 2, 8, (8, 4), 3), ("vertex", 3, 8, (4, 2, 2), 2),
                                            ("vertex", 2, 15, (4, 4), 2), ("cell", 2, 13, (4, 4), 3)])
def test_vcycle(kind, d, k, ms, nl):
    announce("vcycle", kind, d, k, ms, nl)
    from oracle.mesh import refine
    fine = omesh(d, k, tuple(mm >> (nl - 1) for mm in ms), 16)
    for _ in range(nl - 1):
        fine = refine(fine)
    omegas = [0.0] + [0.7 if kind == "cell" else 0.25] * (nl - 1)
    oh = multigrid.Hierarchy(fine, nl, kind, omegas, m_pre=2, m_post=2, cache=False)
    gh = fts.Hierarchy(d, k, fine.widths, nl, kind, omegas, fine.gamma_hat, m_pre=2, m_post=2)
    b, x = random_vector(fine.ndofs, 0), random_vector(fine.ndofs, 1)
    ref = oh.vcycle(x.copy(), b)
    xg = dev(x)
    gh.vcycle(dev(b), xg)
    assert rel(host(xg), ref) < TOL
    # preconditioner form: zero initial guess
    ref0 = oh.vcycle(np.zeros_like(b), b)
    x0 = dev(np.zeros_like(b))
    gh.vcycle(dev(b), x0)
    assert rel(host(x0), ref0) < TOL


@pytest.mark.parametrize("d,k,ms", [(3, 2, (2, 2, 2)), (3, 4, (4, 3, 2)), (2, 3, (9, 10)), (3, 2, (3, 3, 3)),
                                    (3, 1, (3, 2, 4)), (2, 2, (5, 4))])
def test_coarse_lu_solve(d, k, ms):
    """Dense LU of the coarse matrix (several 256-blocks and a ragged last
    block), against scipy's pivoted LU of the assembled matrix.  The cases
    cover even and odd slab sizes (paired and single-column loads of the
    substitution mat-vecs), k = 1 (as many face numbers as unknowns per cell)
    and several slabs in 2-D and 3-D."""
    announce("coarse", d, k, ms)
    m = omesh(d, k, ms, 17)
    gh = fts.Hierarchy(d, k, m.widths, 1, "vertex", [0.0], m.gamma_hat)
    A = sipg.assemble(m).toarray()
    b = random_vector(m.ndofs, 5)
    xs = sla.lu_solve(sla.lu_factor(A), b)
    xg = dev(np.zeros(m.ndofs))
    gh.coarse_solve(dev(b), xg)
    assert rel(host(xg), xs) < 1e-12 * max(1.0, np.linalg.cond(A) / 1e3)


def test_acs_2d_q3_workload():
    """The 2-D Q3 16x16 workload in full: one damped cell-smoother step plus one
    residual, against the oracle."""
    cfg = CONFIGS["acs_2d_q3"]
    announce("acs_2d_q3 full")
    m = Mesh(2, cfg["k"], uniform_widths(2, cfg["m"]), cfg["gamma_hat"])
    A = sipg.assemble(m)
    sol = schwarz.ExactLocalSolvers(A, schwarz.cell_subdomains(m), cache=False)
    b, x0 = random_vector(m.ndofs, cfg["seed_b"]), random_vector(m.ndofs, cfg["seed_x"])
    x1 = schwarz.additive_smooth(A, sol, x0, b, cfg["omega"])
    r1 = b - A @ x1
    lv = glevel(m)
    eg = fts.Eigs(lv, "cell")
    xg = dev(x0)
    fts.schwarz_smooth(lv, eg, cfg["omega"], dev(b), xg, 1)
    rg = dev(np.zeros(m.ndofs))
    lv.residual(dev(b), xg, rg)
    assert rel(host(xg), x1) < TOL
    assert rel(host(rg), r1) < TOL


def test_avs_3d_q4_full_size_sampled():
    """The 3-D Q4 32^3 fine level at full size, as the benchmark launches it:
    one residual + vertex-patch sweep; the oracle recomputes sampled cells
    (corners, faces, interior) exactly from their neighbourhoods."""
    cfg = CONFIGS["avs_3d_q4"]
    announce("avs_3d_q4 full-size sampled")
    m = Mesh(3, cfg["k"], uniform_widths(3, cfg["m"]), cfg["gamma_hat"])
    b, x0 = random_vector(m.ndofs, cfg["seed_b"]), random_vector(m.ndofs, cfg["seed_x"])
    lv = glevel(m)
    eg = fts.Eigs(lv, "vertex")
    rg = dev(np.zeros(m.ndofs))
    lv.residual(dev(b), dev(x0), rg)
    xg = dev(x0)
    fts.schwarz_smooth(lv, eg, cfg["omega"], dev(b), xg, 1)
    r_h, x_h = host(rg), host(xg)
    from oracle import sampled
    mm = cfg["m"] - 1
    cells = [(0, 0, 0), (mm, mm, mm), (0, 5, mm), (16, 16, 16), (1, 30, 7), (31, 0, 15), (13, 1, 29)]
    rs = sampled.residual_cells(m, x0, b, cells)
    for c, rv in rs.items():
        assert rel(r_h[m.cell_dofs(c)], rv) < TOL
    xs = sampled.smooth_cells(m, x0, b, cfg["omega"], "vertex", cells[:5])
    for c, xv in xs.items():
        assert rel(x_h[m.cell_dofs(c)], xv) < TOL


def _full_size_sampled(m, omega, res_cells, smooth_cells, precs):
    """One residual and one vertex-patch sweep of the full-size mesh `m` on the
    GPU (the launch configuration the benchmark uses), against the oracle's
    values recomputed exactly on sampled cells from their neighbourhoods:
    FP64 at the parity bar, reduced-precision corrections within their bounds."""
    from oracle import sampled
    b, x0 = random_vector(m.ndofs, 0), random_vector(m.ndofs, 1)
    lv = glevel(m)
    eg = fts.Eigs(lv, "vertex")
    bg = dev(b)
    x0g = dev(x0)
    rg = torch.empty_like(bg)
    lv.residual(bg, x0g, rg)
    r_h = host(rg)
    del rg
    outs = {}
    for prec in precs:
        xg = x0g.clone()
        fts.schwarz_smooth(lv, eg, omega, bg, xg, 1, prec=prec)
        outs[prec] = {c: host(xg[m.cell_dofs(c)[0]:m.cell_dofs(c)[-1] + 1]) for c in smooth_cells}
        del xg
    rs = sampled.residual_cells(m, x0, b, res_cells)
    for c, rv in rs.items():
        assert rel(r_h[m.cell_dofs(c)], rv) < TOL, c
    xs = sampled.smooth_cells(m, x0, b, omega, "vertex", smooth_cells)
    for c, xv in xs.items():
        d0 = m.cell_dofs(c)
        for prec, bound in precs.items():
            got = outs[prec][c]
            if prec == "f64":
                assert rel(got, xv) < TOL, (prec, c)
            else:
                err = rel2(got - x0[d0], xv - x0[d0])
                print(prec, "cell", c, "correction error vs oracle", err)
                assert err < bound, (prec, c, err)


def test_mixed_3d_q7_full_size_sampled():
    """The 48^3 Q7 fine level (56,623,104 DoFs) at full size: residual and one
    vertex-patch sweep with FP64 contractions (FP64 MFMA local solves in runs
    along z) at the parity bar, and FP32 / FP16 / BF16 contractions within
    their error bounds, against sampled oracle cells (corner, edge, interior)."""
    cfg = CONFIGS["mixed_3d_q7"]
    announce("mixed_3d_q7 full-size sampled")
    m = Mesh(3, cfg["k"], uniform_widths(3, cfg["m"]), cfg["gamma_hat"])
    mm = cfg["m"] - 1
    _full_size_sampled(m, cfg["omega"], [(0, 0, 0), (mm, mm, mm), (0, 7, mm), (24, 24, 24), (47, 3, 20)],
                       [(0, 0, 0), (mm, 0, 11), (23, 30, 17)],
                       {"f64": None, "f32": 1e-4, "f16": 1.5e-3, "bf16": 1.2e-2})


def test_adjoint_3d_q5_full_size_sampled():
    """The 32^3 Q5 fine level (7,077,888 DoFs): residual and one FP64
    vertex-patch sweep against sampled oracle cells."""
    cfg = CONFIGS["adjoint_3d_q5"]
    announce("adjoint_3d_q5 fine level full-size sampled")
    m = Mesh(3, cfg["k"], uniform_widths(3, cfg["m"]), cfg["gamma_hat"])
    mm = cfg["m"] - 1
    _full_size_sampled(m, cfg["omega"], [(0, 0, 0), (mm, mm, mm), (0, 5, mm), (16, 16, 16), (1, 30, 7)],
                       [(0, 0, 0), (mm, 9, 0), (16, 16, 16), (5, 1, 30)], {"f64": None, "f32": 1e-4})


def test_q8_26_cubed_full_size_sampled():
    """k = 8 on 26^3 random rectilinear cells (12,812,904 DoFs): enough patches
    (15,625) for runs of 2 patches along z; residual and FP64 / FP32 sweep
    against sampled oracle cells."""
    announce("q8 26^3 sampled")
    rng = np.random.default_rng(29)
    m = Mesh(3, 8, loguniform_widths(rng, 3, (26, 26, 26), 0.25, 4.0), 1.0)
    _full_size_sampled(m, 0.125, [(0, 0, 0), (25, 25, 25), (12, 0, 5), (11, 13, 12)],
                       [(0, 0, 0), (25, 0, 25), (0, 12, 7)], {"f64": None, "f32": 1e-4})


@pytest.mark.parametrize("d,k,ms", [(3, 4, (4, 3, 3))])
def test_f32_contractions_error_bound(d, k, ms):
    """FP32 contractions (FP64 residual and accumulation): error of one sweep
    against the FP64 oracle within a few FP32 unit roundoffs times the local
    condition number; reported, not exact."""
    announce("f32", d, k, ms)
    m = omesh(d, k, ms, 18)
    A = sipg.assemble(m)
    sol = schwarz.ExactLocalSolvers(A, schwarz.vertex_patch_subdomains(m), cache=False)
    x, b = random_vector(m.ndofs, 1), random_vector(m.ndofs, 0)
    ref = schwarz.additive_smooth(A, sol, x, b, 0.3)
    lv = glevel(m)
    eg = fts.Eigs(lv, "vertex")
    xg = dev(x)
    fts.schwarz_smooth(lv, eg, 0.3, dev(b), xg, 1, prec="f32")
    err = rel2(host(xg) - x, ref - x)
    print("f32 relative error of the correction", err)
    assert err < 1e-4


@pytest.mark.parametrize("kind,d,k,ms,nl,omega", [("vertex", 3, 3, (8, 8, 8), 3, 0.125), ("cell", 2, 4, (16, 16), 4, 0.7)])
def test_pcg(kind, d, k, ms, nl, omega):
    """FP64 flexible PCG with the V-cycle preconditioner: residual history of
    the first iterations equals the oracle's (same algorithm), the iteration
    counts agree and the final iterate solves the system (checked against the
    exact discrete solution by global fast diagonalisation)."""
    announce("pcg", kind, d, k, ms, nl)
    from oracle import krylov
    from oracle.mesh import refine
    fine = uniform_mesh(d, k, tuple(mm >> (nl - 1) for mm in ms))
    for _ in range(nl - 1):
        fine = refine(fine)
    omegas = [0.0] + [omega] * (nl - 1)
    oh = multigrid.Hierarchy(fine, nl, kind, omegas, m_pre=2, m_post=2)
    b = random_vector(fine.ndofs, 0)
    xo, ito, histo = krylov.pcg(oh.A[-1], b, lambda r: oh.vcycle(np.zeros_like(r), r), rtol=1e-10, flexible=True)
    gh = fts.Hierarchy(d, k, fine.widths, nl, kind, omegas, fine.gamma_hat, m_pre=2, m_post=2)
    xg = dev(np.zeros(fine.ndofs))
    it, relres, hist = gh.pcg(dev(b), xg, rtol=1e-10, maxit=200)
    print("pcg iterations gpu", it, "oracle", ito, "final", relres)
    assert abs(it - ito) <= 1 and relres <= 1e-10
    nh = min(6, len(hist), len(histo))
    assert np.allclose(hist[:nh], histo[:nh], rtol=1e-9, atol=0)
    xs = onedim.global_fastdiag_solve(fine, b)
    assert rel(host(xg), xs) < 1e-8
    assert rel(host(xg), xo) < 1e-8


def test_pcg_mixed_precision_reaches_fp64_residual():
    """FP32 contractions in the preconditioner, FP64 CG: reaches 1e-10 with at
    most a few more iterations than the FP64 preconditioner."""
    announce("pcg mixed")
    from oracle.mesh import refine
    fine = refine(refine(uniform_mesh(3, 3, 2)))
    omegas = [0.0, 0.125, 0.125]
    gh = fts.Hierarchy(3, 3, fine.widths, 3, "vertex", omegas, 1.0, 2, 2)
    b = dev(random_vector(fine.ndofs, 0))
    x64 = dev(np.zeros(fine.ndofs))
    it64, r64, _ = gh.pcg(b, x64, rtol=1e-10)
    x32 = dev(np.zeros(fine.ndofs))
    it32, r32, _ = gh.pcg(b, x32, rtol=1e-10, prec="f32")
    print("iterations f64", it64, "f32", it32)
    assert r32 <= 1e-10 and it32 <= it64 + 3
    assert rel(host(x32), host(x64)) < 1e-8


@pytest.mark.parametrize("kind,k,ms", [("vertex", 3, (4, 3, 5)), ("vertex", 4, (3, 4, 3)), ("vertex", 7, (3, 2, 2)),
                                       ("vertex", 5, (5, 4, 3)), ("vertex", 7, (5, 7, 4)), ("vertex", 2, (8, 4, 5)),
                                       ("cell", 4, (3, 2, 3)), ("cell", 9, (2, 2, 1))])
@pytest.mark.parametrize("prec,bound", [("f16", 1.5e-3), ("bf16", 1.2e-2)])
def test_mfma_contractions_error_bound(kind, k, ms, prec, bound):
    """16-bit MFMA contractions (FP32 accumulation, FP64 update of x): the
    correction of one local-solver application against the FP64 oracle, in
    both schedules; bounded by a few units of the 16-bit roundoff."""
    announce("mfma", prec, kind, k, ms)
    m = omesh(3, k, ms, 20)
    A = sipg.assemble(m)
    subs = schwarz.cell_subdomains(m) if kind == "cell" else schwarz.vertex_patch_subdomains(m)
    sol = schwarz.ExactLocalSolvers(A, subs, cache=False)
    r = random_vector(m.ndofs, 3) * 1e-7  # small residuals must not underflow FP16
    ref = 0.4 * sol.apply(r)
    lv = glevel(m)
    eg = fts.Eigs(lv, kind)
    for schedule in (("staged", "colored", "owner") if kind == "vertex" else ("staged",)):
        eg.set_schedule(schedule)
        xa = dev(np.zeros(m.ndofs))
        fts.schwarz_apply(lv, eg, 0.4, dev(r), xa, prec=prec)
        err = rel2(host(xa), ref)
        print(prec, kind, k, schedule, "relative error", err)
        assert err < bound


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_pcg_mfma_preconditioner_reaches_fp64_residual(prec):
    announce("pcg", prec)
    from oracle.mesh import refine
    fine = refine(refine(uniform_mesh(3, 3, 2)))
    gh = fts.Hierarchy(3, 3, fine.widths, 3, "vertex", [0.0, 0.125, 0.125], 1.0, 2, 2)
    b = dev(random_vector(fine.ndofs, 0))
    x64 = dev(np.zeros(fine.ndofs))
    it64, _, _ = gh.pcg(b, x64, rtol=1e-10)
    xl = dev(np.zeros(fine.ndofs))
    itl, rl, _ = gh.pcg(b, xl, rtol=1e-10, prec=prec)
    print("iterations f64", it64, prec, itl)
    assert rl <= 1e-10 and itl <= it64 + 8
    assert rel(host(xl), host(x64)) < 1e-8


def test_mixed_3d_q7_cg_error_vs_oracle():
    """The 48^3 Q7 workload end to end: FP64 CG preconditioned by the 5-level
    vertex-patch V-cycle to ||r|| <= 1e-10 ||b||, with the smoother's
    contractions in FP64, FP32, FP16 and BF16; each solution against the exact
    discrete solution from the oracle's global fast diagonalisation."""
    cfg = CONFIGS["mixed_3d_q7"]
    announce("mixed_3d_q7 CG vs oracle")
    d, k, mm, nl = cfg["dim"], cfg["k"], cfg["m"], cfg["nlevels"]
    m = uniform_mesh(d, k, mm, gamma_hat=cfg["gamma_hat"])
    b = random_vector(m.ndofs, cfg["seed_b"])
    xs = onedim.global_fastdiag_solve(m, b)
    h = fts.Hierarchy(d, k, m.widths, nl, "vertex", [0.0] + [cfg["omega"]] * (nl - 1), cfg["gamma_hat"],
                      cfg["m_pre"], cfg["m_post"])
    bg = dev(b)
    xsg = dev(xs)
    nxs = float(torch.linalg.norm(xsg))
    for prec in ("f64", "f32", "f16", "bf16"):
        xg = torch.zeros_like(bg)
        it, relres, _ = h.pcg(bg, xg, rtol=cfg["rtol"], maxit=200, prec=prec)
        err = float(torch.linalg.norm(xg - xsg)) / nxs
        print(prec, "iterations", it, "final relres", relres, "error vs oracle", err)
        assert relres <= cfg["rtol"]
        assert err < 1e-8, (prec, err)
