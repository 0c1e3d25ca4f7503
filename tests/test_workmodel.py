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
