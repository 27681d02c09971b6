"""Writes the stored expected values under tests/golden/ from the oracle only.

c0_narrow_e2.json: the deterministic second-order energy of Eq. FinalMP2
(direct and exchange parts and total) of the tiny two-nucleus workload with
basis exponents in [0.3, 1.2] (seeded synthetic inputs, four-component
spinors), from McMurchie-Davidson integrals and an explicit four-index
transformation.  The GPU chain test and the redundant-walker convergence
study compare stochastic estimates with it.

Run from the repository root:  python tests/golden/make_references.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mp2  # noqa: E402
from synth import make_inputs  # noqa: E402


def c0_narrow():
    inp = make_inputs("C0", exp_range=(0.3, 1.2))
    eri = mp2.spinor_eri(inp, mp2.ao_eri(inp))
    d, x = (complex(v) for v in mp2.mp2_final_parts(eri, inp.eps, inp.n_occ))
    return {"workload": "C0 with basis exponents in [0.3, 1.2] (synth.make_inputs('C0', exp_range=(0.3, 1.2)), "
                        "seed 0, four-component spinors)",
            "definition": "Eq. FinalMP2 from McMurchie-Davidson ERIs and an explicit four-index transformation "
                          "(oracle.mp2), direct and exchange parts",
            "direct": d.real, "exchange": x.real, "total": d.real + x.real,
            "imag_total": d.imag + x.imag}


if __name__ == "__main__":
    out = os.path.join(HERE, "c0_narrow_e2.json")
    with open(out, "w") as fh:
        json.dump(c0_narrow(), fh, indent=1)
        fh.write("\n")
    print(out)
