"""Pin the FLOP model used for the rooflines against the paper's printed counts."""
import json
import os

import numpy as np

from paper_1910_11239_amd import workmodel as wm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "flop_tables.json")))


def test_flop_model_reproduces_table_flop_additive():
    d = GOLD["dim"]
    for k, mflop in GOLD["acs_local_solvers_mflop"].items():
        model = GOLD["cells"] * wm.local_solver_flops(d, int(k) + 1) / 1e6
        assert abs(model - mflop) / mflop < 0.01, (k, model, mflop)
    for k, mflop in GOLD["avs_local_solvers_mflop"].items():
        model = GOLD["patches"] * wm.local_solver_flops(d, 2 * (int(k) + 1)) / 1e6
        assert abs(model - mflop) / mflop < 0.01, (k, model, mflop)


def test_flop_model_constants_table_cmplxconstant():
    d = GOLD["dim"]
    for k, acs, avs in zip(GOLD["cmplx_degrees"], GOLD["cmplx_acs_local_solvers"], GOLD["cmplx_avs_local_solvers"]):
        n1 = k + 1
        assert abs(wm.local_solver_flops(d, n1) / n1 ** (d + 1) - acs) < 0.5
        assert abs(wm.local_solver_flops(d, 2 * n1) / n1 ** (d + 1) - avs) / avs < 0.02


def test_counts():
    assert wm.n_subdomains((16, 16, 16), "vertex") == 3375
    assert wm.ndofs(3, 4, (32, 32, 32)) == 4096000
    assert wm.ndofs(3, 7, (48, 48, 48)) == 56623104


def test_coarse_solve_bytes_count_the_rows_the_kernels_read():
    """Brute force over rows: the diagonal blocks' strict lower and upper
    halves, W_i rows (cell c, face number a) over [c nc, B), V_i rows of cell
    c over [0, (c + 1) rc), and P_i, R_i in full."""
    for dim, k, ncells in ((3, 4, (8, 8, 8)), (2, 3, (5, 3)), (3, 1, (2, 3, 4))):
        n1 = k + 1
        nc, rc = n1 ** dim, 2 * n1 ** (dim - 1)
        nb, ncs = ncells[-1], int(np.prod(ncells[:-1]))
        B = ncs * nc
        diag = sum(r for r in range(B)) + sum(B - r for r in range(B))
        w = sum(B - (row // rc) * nc for row in range(ncs * rc))
        v = sum((r // nc + 1) * rc for r in range(B))
        count = nb * diag + (nb - 1) * (w + v + 2 * ncs * rc * nc)
        assert wm.coarse_solve_bytes(dim, k, ncells) == 8 * count
    # the 8^3 Q4 coarse level: 5.60 GB against 7.68 GB for the full triangular off-diagonal blocks
    assert abs(wm.coarse_solve_bytes(3, 4, (8, 8, 8)) / 1e9 - 5.597) < 0.001
