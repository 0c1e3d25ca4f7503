"""Batched mixed-degree smoothing (fts_batch_*): one persistent launch over the
vertex patches of several anisotropic meshes of different degrees, against the
oracle mesh by mesh."""
import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle import sipg, schwarz
from synthetic import loguniform_widths, random_vector, batched_meshes
from gpu_util import dev, host, rel, rel2, announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1910_11239_amd as fts  # noqa: E402

SPECS = [(2, (4, 3, 5)), (3, (3, 3, 3)), (4, (2, 3, 2)), (5, (3, 2, 3)), (1, (3, 2, 2)), (6, (2, 2, 3)),
         (7, (3, 2, 2)), (8, (2, 3, 2)), (9, (2, 2, 2))]


def _meshes():
    rng = np.random.default_rng(42)
    return [Mesh(3, k, loguniform_widths(rng, 3, ms, 0.25, 4.0), 1.0) for k, ms in SPECS]


def _oracle_sweeps(meshes, omega, b, x):
    outs = []
    for i, m in enumerate(meshes):
        A = sipg.assemble(m)
        if m.k == 9:
            outs.append(("exact", A, b[i]))
            continue
        sol = schwarz.ExactLocalSolvers(A, schwarz.vertex_patch_subdomains(m), cache=False)
        outs.append(("ref", schwarz.additive_smooth(A, sol, x[i], b[i], omega), None))
    return outs


@pytest.mark.parametrize("launch", [None, (512, 512, 16), (256, 1024, 1)])
def test_batch_fp64_parity(launch):
    announce("batch fp64", launch)
    meshes = _meshes()
    batch = fts.Batch([(m.k, m.widths, m.gamma_hat) for m in meshes])
    if launch:
        batch.set_launch(*launch)
    bs = [random_vector(m.ndofs, 10 + i) for i, m in enumerate(meshes)]
    xs = [random_vector(m.ndofs, 20 + i) for i, m in enumerate(meshes)]
    omega = 1.0  # the one-patch Q9 mesh is then an exact solve
    xg = dev(np.concatenate(xs))
    batch.smooth(omega, dev(np.concatenate(bs)), xg, nsweeps=1, prec="f64")
    out = host(xg)
    for i, (kind, ref, extra) in enumerate(_oracle_sweeps(meshes, omega, bs, xs)):
        off, n = batch.offsets[i]
        got = out[off:off + n]
        if kind == "exact":
            assert np.linalg.norm(ref @ got - extra) < 1e-10 * np.linalg.norm(extra), i
        else:
            assert rel(got, ref) < 1e-12, (i, meshes[i].k)


def test_batch_fp32_error_and_autotune():
    announce("batch fp32 + autotune")
    meshes = _meshes()[:-1]
    batch = fts.Batch([(m.k, m.widths, m.gamma_hat) for m in meshes])
    bs = [random_vector(m.ndofs, 10 + i) for i, m in enumerate(meshes)]
    xs = [random_vector(m.ndofs, 20 + i) for i, m in enumerate(meshes)]
    b, x = dev(np.concatenate(bs)), dev(np.concatenate(xs))
    r = torch.empty_like(b)
    batch.residual(b, x, r)
    report = batch.autotune(r, prec="f32")
    print(report)
    assert "chosen" in report
    xg = x.clone()
    batch.smooth(0.4, b, xg, nsweeps=1, prec="f32")
    out = host(xg)
    for i, (kind, ref, _) in enumerate(_oracle_sweeps(meshes, 0.4, bs, xs)):
        off, n = batch.offsets[i]
        err = rel2(out[off:off + n] - xs[i], ref - xs[i])
        print("mesh", i, "k", meshes[i].k, "fp32 correction error", err)
        assert err < 1e-5


def test_batched_workload_runs_and_is_consistent():
    """The 64-mesh workload (k ~ U{2..9}, m ~ U{8..24}, per-slab widths
    log-uniform in [0.25, 4]): the batched FP64 sweep equals the single-mesh
    FP64 path within 1e-12 on the first mesh of every degree present and on the
    last mesh (the single-mesh path is parity-tested against the oracle at
    every degree), and FP32 stays within 1e-5."""
    announce("batched workload")
    specs = batched_meshes()
    batch = fts.Batch([(k, w, 1.0) for k, w in specs])
    N = batch.ndofs
    b = dev(random_vector(N, 0))
    x0 = dev(random_vector(N, 1))
    x64 = x0.clone()
    batch.smooth(0.125, b, x64, nsweeps=1, prec="f64")
    x32 = x0.clone()
    batch.smooth(0.125, b, x32, nsweeps=1, prec="f32")
    d64, d32 = x64 - x0, x32 - x0
    err = float(torch.linalg.norm(d32 - d64) / torch.linalg.norm(d64))
    print("FP32 vs FP64 correction, whole batch:", err)
    assert err < 1e-5
    first = {}
    for i, (k, _) in enumerate(specs):
        first.setdefault(k, i)
    assert set(first) == set(range(2, 10))
    for i in sorted(set(first.values()) | {len(specs) - 1}):
        k, w = specs[i]
        announce("batched workload mesh", i, "k", k, "m", len(w[0]))
        off, n = batch.offsets[i]
        lv = fts.Level(3, k, w, 1.0)
        eg = fts.Eigs(lv, "vertex")
        xs = x0[off:off + n].clone()
        fts.schwarz_smooth(lv, eg, 0.125, b[off:off + n].clone(), xs, 1)
        assert rel(host(xs), host(x64[off:off + n])) < 1e-12, (i, k)
