"""Writes the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py

dcut4_beta01497_16steps.json: the 4D flow at beta = 0.1497, h = 0, Dcut = 4,
16 steps along x, y, z, t (one site coarse-grained to a 16^4 lattice), with
both impurity tensors: per step lnZ/N (Eqs. (2.3)-(2.5)), the impurity energy
and magnetisation (Eqs. (2.10), (2.12)) and X^(n) (Eqs. (3.2)-(3.3)), the
bond dimensions and c_n.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import hotrg as OH  # noqa: E402


def dcut4_flow():
    beta, h, dcut, n = 0.1497, 0.0, 4, 16
    f = OH.run(beta, h, dcut, 4, n)
    steps = [{"n": r.n, "axis": r.axis, "dims": list(r.dims), "c_n": r.c, "lnz_per_site": r.lnz_per_site,
              "e_imp": r.e_imp, "m_imp": r.m_imp, "nn_imp": r.nn_imp, "X": r.X} for r in f.records]
    return {"workload": "4D Ising HOTRG, beta = 0.1497, h = 0, Dcut = 4, 16 steps (x, y, z, t cycle), impurities",
            "source": "oracle/hotrg.py run(); written by tests/golden/make_golden.py",
            "beta": beta, "h": h, "dcut": dcut, "steps": steps}


if __name__ == "__main__":
    out = os.path.join(HERE, "dcut4_beta01497_16steps.json")
    with open(out, "w") as fh:
        json.dump(dcut4_flow(), fh, indent=1)
    print(out)
