"""Writes the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py

dcut4_beta01497_16steps.json: the 4D flow at beta = 0.1497, h = 0, Dcut = 4,
16 steps along x, y, z, t (one site coarse-grained to a 16^4 lattice), with
both impurity tensors: per step lnZ/N (Eqs. (2.3)-(2.5)), the impurity energy
and magnetisation (Eqs. (2.10), (2.12)) and X^(n) (Eqs. (3.2)-(3.3)), the
bond dimensions and c_n.

dcut8_beta01497_h1e-5_6steps.json: the flow at beta = 0.1497, h = 1e-5,
Dcut = 8, 6 steps (steps 4-6 at the steady-state dims 8^4, environments of
64 x 64), with both impurity tensors: the same per-step values plus, for every
truncated transverse axis, the kept dimension, the chosen side and the chosen
side's environment spectrum (descending).  About an hour of CPU time.

    python tests/golden/make_golden.py [dcut4] [dcut8]     # default: both
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


def dcut8_flow():
    beta, h, dcut, n = 0.1497, 1e-5, 8, 6
    f = OH.start(beta, h, dcut, 4)
    steps = []
    for k in range(n):
        r = OH.step(f, k % 4)
        decs = [{"axis": d.nu, "k": d.k, "side": d.side, "spectrum": [float(v) for v in d.spectra[d.side]]}
                for d in r.decisions if d.truncated]
        steps.append({"n": r.n, "axis": r.axis, "dims": list(r.dims), "c_n": r.c, "lnz_per_site": r.lnz_per_site,
                      "e_imp": r.e_imp, "m_imp": r.m_imp, "nn_imp": r.nn_imp, "X": r.X, "truncated": decs})
        print(f"dcut8 step {r.n} done: dims {r.dims}", flush=True)
    return {"workload": "4D Ising HOTRG, beta = 0.1497, h = 1e-5, Dcut = 8, 6 steps (x, y, z, t cycle), impurities",
            "source": "oracle/hotrg.py start()/step(); written by tests/golden/make_golden.py",
            "beta": beta, "h": h, "dcut": dcut, "steps": steps}


FIXTURES = {"dcut4": ("dcut4_beta01497_16steps.json", dcut4_flow),
            "dcut8": ("dcut8_beta01497_h1e-5_6steps.json", dcut8_flow)}

if __name__ == "__main__":
    for name in sys.argv[1:] or list(FIXTURES):
        fname, make = FIXTURES[name]
        data = make()
        out = os.path.join(HERE, fname)
        with open(out, "w") as fh:
            json.dump(data, fh, indent=1)
        print(out, flush=True)
