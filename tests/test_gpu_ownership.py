"""Ownership of device memory: every table, level vector, staging buffer,
coarse factor and batch queue the library's handles hold is torch memory
obtained through the allocator the binding registers (fts_set_allocator), and
it goes back to torch when the handle is destroyed."""
import gc

import numpy as np
import pytest

from synthetic import uniform_widths, batched_meshes, distorted_vertices, random_vector
from gpu_util import dev, host, announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1910_11239_amd as fts  # noqa: E402


def _held():
    torch.cuda.synchronize()
    return fts.device_bytes_held(), torch.cuda.memory_allocated()


@pytest.mark.parametrize("what", ["hierarchy", "level+eigs", "batch", "mapped"])
def test_handles_hold_torch_memory_and_return_it(what):
    announce("ownership", what)
    gc.collect()
    h0, t0 = _held()
    if what == "hierarchy":
        obj = fts.Hierarchy(3, 3, uniform_widths(3, 8), 3, "vertex", [0.0, 0.125, 0.125], 1.0, 2, 2)
        b = dev(random_vector(obj.ndofs, 0))
        x = torch.zeros_like(b)
        obj.vcycle(b, x)
        assert float(torch.linalg.norm(x)) > 0
    elif what == "level+eigs":
        obj = [fts.Level(3, 4, uniform_widths(3, 6), 1.0)]
        obj.append(fts.Eigs(obj[0], "vertex"))
    elif what == "batch":
        obj = fts.Batch([(k, w, 1.0) for k, w in batched_meshes()[:4]])
    else:
        ms, V = distorted_vertices(3, 2, 1, 0.25, 1)
        obj = fts.MappedLevel(3, 3, ms, V, 4.0)
    h1, t1 = _held()
    print(what, "library bytes held", h1 - h0, "torch allocated grew by", t1 - t0)
    assert h1 > h0
    assert t1 - t0 >= h1 - h0  # all of it is torch memory
    del obj
    gc.collect()
    h2, t2 = _held()
    assert h2 == h0
    assert t2 <= t0 + (t1 - t0) - (h1 - h0)
