"""The allocation-free smoother (fts_schwarz_smooth_noalloc) against the
workspace form (fts_schwarz_smooth), both through the C ABI: two calls in a
row on different levels, the second with a smaller level, so the static
residual array holds the first call's values when the second starts; and a
level above the array's size is refused."""
import ctypes

import numpy as np
import pytest

from oracle.mesh import Mesh
from synthetic import loguniform_widths, random_vector, uniform_widths
from gpu_util import dev, host, rel, announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1910_11239_amd as fts  # noqa: E402


def _case(d, k, ms, seed, kind, prec, omega, nsweeps):
    rng = np.random.default_rng(seed)
    m = Mesh(d, k, loguniform_widths(rng, d, ms, 0.25, 4.0), 1.0)
    lv = fts.Level(d, k, m.widths, 1.0)
    eg = fts.Eigs(lv, kind)
    b, x0 = dev(random_vector(m.ndofs, seed)), dev(random_vector(m.ndofs, seed + 1))
    ref = x0.clone()
    fts.schwarz_smooth(lv, eg, omega, b, ref, nsweeps=nsweeps, prec=prec)
    got = x0.clone()
    st = fts.lib().fts_schwarz_smooth_noalloc(lv._h, eg._h, ctypes.c_double(omega), fts.PREC[prec],
                                              ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(got.data_ptr()),
                                              nsweeps, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, fts.last_error()
    return host(got), host(ref)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_matches_workspace_form_twice(prec):
    announce("noalloc", prec)
    got, ref = _case(3, 4, (9, 8, 7), 3, "vertex", prec, 0.3, 2)
    assert rel(got, ref) < 1e-12
    # second call: a smaller level, the array still holds the first residual
    got, ref = _case(3, 3, (4, 3, 5), 5, "vertex", prec, 0.3, 1)
    assert rel(got, ref) < 1e-12
    got, ref = _case(2, 5, (6, 5), 7, "cell", prec, 0.7, 1)
    assert rel(got, ref) < 1e-12


def test_noalloc_full_size_q4_and_refuses_larger_level():
    """The 3-D Q4 32^3 fine level (4,096,000 DoFs) fits the array; a level
    above 4,194,304 DoFs is refused with FTS_E_SIZE and x is left unchanged."""
    announce("noalloc q4 32^3 + size limit")
    lv = fts.Level(3, 4, uniform_widths(3, 32), 1.0)
    eg = fts.Eigs(lv, "vertex")
    b, x0 = dev(random_vector(lv.ndofs, 0)), dev(random_vector(lv.ndofs, 1))
    ref = x0.clone()
    fts.schwarz_smooth(lv, eg, 0.5, b, ref, 1)
    got = x0.clone()
    fts.schwarz_smooth_noalloc(lv, eg, 0.5, b, got, 1)
    assert rel(host(got), host(ref)) < 1e-12
    big = fts.Level(3, 4, uniform_widths(3, (33, 32, 32)), 1.0)
    egb = fts.Eigs(big, "vertex")
    xb = torch.zeros(big.ndofs, dtype=torch.float64, device="cuda")
    bb = torch.ones_like(xb)
    with pytest.raises(fts.FtsError, match="static residual workspace"):
        fts.schwarz_smooth_noalloc(big, egb, 0.5, bb, xb, 1)
    assert float(torch.count_nonzero(xb)) == 0
