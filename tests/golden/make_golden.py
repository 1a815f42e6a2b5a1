"""Write the oracle's results on the 4^4 workloads to oracle_4x4.json.

Uses only the oracle and the seeded input generator (no GPU code). The paper
prints no worked example, so these stored values are regression pins of the
oracle itself (Alg. 1 and Alg. 2 on seeded synthetic fields), not values from
the paper. Run from the repository root: python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import sdfft  # noqa: E402
from paper_1412_1498_amd import synth  # noqa: E402


def main():
    dims = (4, 4, 4, 4)
    out = {}
    for name, gauge in (("landau", 0), ("coulomb", 1)):
        U = synth.random_gauge_field(dims, 0.3, 0).numpy().copy()
        F0, th0 = oracle.quality(U, dims, gauge)
        r = oracle.fix(U, dims, 1.7, 1e-12, 2000, gauge, reunit_every=20)
        V = synth.random_gauge_field(dims, 0.3, 0).numpy().copy()
        _, rs = sdfft.sd_fix(V, dims, 0.08, 1e-12, 2000, gauge)
        out[name] = dict(initial_F=F0, initial_theta=th0, or_omega_1p7=r, sd_fourier_alpha_0p08=rs)
    out["recipe"] = ("4^4 lattice, amp 0.3, seed 0 (paper_1412_1498_amd.synth.random_gauge_field); "
                     "overrelaxation omega 1.7, reunitarisation every 20 sweeps, theta < 1e-12; "
                     "Fourier-accelerated steepest descent alpha 0.08, theta < 1e-12")
    with open(os.path.join(HERE, "oracle_4x4.json"), "w") as fh:
        json.dump(out, fh, indent=1, default=float)


if __name__ == "__main__":
    main()
