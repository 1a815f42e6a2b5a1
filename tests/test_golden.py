"""Regression pins: the oracle's Alg. 1 and Alg. 2 results on the seeded 4^4
workloads, stored by tests/golden/make_golden.py (which calls only the oracle
and the input generator). They catch an unintended change of the oracle or of
the generator; the mathematical pins are in test_oracle_*_pins.py."""
import json
import os

import pytest

from oracle import sdfft

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "oracle_4x4.json")) as fh:
        return json.load(fh)


@pytest.mark.parametrize("name,gauge", [("landau", 0), ("coulomb", 1)])
def test_oracle_matches_stored_results(oracle_lib, field_cache, golden, name, gauge):
    dims = (4, 4, 4, 4)
    g = golden[name]
    U = field_cache(dims, 0.3, 0)
    F0, th0 = oracle_lib.quality(U, dims, gauge)
    assert abs(F0 - g["initial_F"]) < 1e-15 and abs(th0 - g["initial_theta"]) < 1e-13
    r = oracle_lib.fix(U, dims, 1.7, 1e-12, 2000, gauge, reunit_every=20)
    ref = g["or_omega_1p7"]
    assert r["converged"] and r["iters"] == ref["iters"] and abs(r["F"] - ref["F"]) < 1e-14
    _, rs = sdfft.sd_fix(field_cache(dims, 0.3, 0), dims, 0.08, 1e-12, 2000, gauge)
    ref = g["sd_fourier_alpha_0p08"]
    assert rs["converged"] and rs["iters"] == ref["iters"] and abs(rs["F"] - ref["F"]) < 1e-14
