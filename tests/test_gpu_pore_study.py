"""Carved micro- and mesopores in NPMC carbon (Section 5.3): the solver's steady
outputs on such structures against the oracle's exact fixed point (sparse LU),
with Knudsen diffusion in the small carved pores, for the effective-diffusivity
and the reactive problem (every carbon face reactive)."""
import numpy as np
import pytest

import structgen as sg
from oracle import lbm as O

pytestmark = pytest.mark.gpu

CARVED = [
    ("micro", dict(carbon_final=0.45, micro=0.05, meso=0.0, micro_d=(2, 4))),
    ("meso", dict(carbon_final=0.45, micro=0.0, meso=0.05, meso_d=(5, 8))),
]


@pytest.mark.parametrize("name,kw", CARVED)
@pytest.mark.parametrize("mode", [0, 1])
def test_carved_npmc_matches_the_oracle_fixed_point(hip, name, kw, mode):
    ph = sg.npmc_cl(5, shape=(14, 14, 40), ionomer=0.15, **kw)
    k = 1e-3 if mode == 1 else 0.0
    cat = (1 << O.CARBON) | (1 << O.PT)
    prob = O.prepare(ph, O.Params(mode=mode, knudsen=True, voxel_m=1e-9, k_lat=k, catalyst_phases=cat))
    want = O.solve_fixed_point(prob, "direct")
    s = hip.Solver(ph, hip.lbm_params_default(mode=mode, knudsen=1, k_lat=k, catalyst_phases=cat), voxel_m=1e-9)
    st, info = s.run_to_steady()
    assert st == 0
    got, ref = (s.deff()[1], want.deff) if mode == 0 else (s.reaction_rate()[1], want.rate)
    print(f"[carved {name}] mode {mode}: GPU {got:.10e} oracle {ref:.10e} ({info.steps} steps)", flush=True)
    assert np.isfinite(got) and got == pytest.approx(ref, rel=1e-4)
