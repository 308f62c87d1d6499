"""Write the stored oracle values the GPU tests and the benchmark compare against.

Calls only the FP64 oracle (oracle/) and the shared seeded input generator
(structgen/); nothing here touches the HIP path.  Re-run after any change to the
oracle's arithmetic or to the generator:  python tests/golden/make_golden.py"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import structgen as sg  # noqa: E402
from oracle import lbm as O  # noqa: E402


def two_phase_32():
    """The 32^3 two-phase workload: QSGS core probability 0.01, growth 0.02,
    porosity 0.5, tau = 1, C = 1 / 0 at the x faces, D_eff/D0 by the exact fixed point."""
    out = []
    for seed in range(1, 11):
        ph = sg.two_phase(seed, n=32)
        t = time.time()
        s = O.solve(ph, O.Params())
        out.append({"seed": seed, "deff": s.deff, "j_in": s.fluxes.j_in, "j_out": s.fluxes.j_out,
                    "seconds": round(time.time() - t, 2)})
        print(out[-1], flush=True)
    return {"workload": "two-phase QSGS 32^3, porosity 0.5, tau 1, D_eff mode",
            "generator": "structgen.two_phase(seed, n=32)", "solver": "oracle.lbm.solve (sparse direct)",
            "cases": out}


if __name__ == "__main__":
    data = two_phase_32()
    with open(os.path.join(HERE, "oracle_two_phase_32.json"), "w") as fh:
        json.dump(data, fh, indent=1)
