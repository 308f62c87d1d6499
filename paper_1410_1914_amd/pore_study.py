"""Micro- and mesopores carved inside the carbon of an NPMC catalyst layer
(Chen et al., arXiv 1410.1914, Section 5.3), on synthetic structures.

The same carbon (grown to 0.55 of the volume) and ionomer (0.15) are kept in
three variants; only what is carved inside the carbon, away from its ionomer
faces, differs:

* ``original``: nothing carved (carbon 0.55);
* ``A1``: 0.10 of the volume carved as pores of 5-10 nm (micropores);
* ``A2``: 0.10 of the volume carved as pores of 15-25 nm (mesopores).

For each variant, at 1 nm voxels with Knudsen diffusion: the mean pore size
(13-direction chords, on the device), D_eff/D_b (Section 3.5.1), and, with
every carbon face reactive, the reaction rate per unit area and the mean
concentration on the outlet plane (Section 3.5.2).  The rate constant,
k = 1e-6 per face in lattice units, leaves a measurable concentration across
the layer: at 1e-4 the oxygen is consumed within ~7 voxels of the inlet.

The paper's finding to compare with: micropores change D_eff little, while
mesopores raise it several-fold and lift the outlet concentration.

python -m paper_1410_1914_amd.pore_study [edge] [seed ...]
"""
import json
import sys
import time

import numpy as np

from . import lbm

VOXEL_M = 1e-9
K_LAT = 1e-6
VARIANTS = {
    "original": dict(carbon_final=0.55, micro=0.0, meso=0.0),
    "A1": dict(carbon_final=0.45, micro=0.10, meso=0.0, micro_d=(5, 10)),
    "A2": dict(carbon_final=0.45, micro=0.0, meso=0.10, meso_d=(15, 25)),
}


def structure(name, seed, n):
    import structgen

    return structgen.npmc_cl(seed, n=n, ionomer=0.15, **VARIANTS[name])


def _run(solver, log, label, chunk=200_000):
    t0 = time.perf_counter()
    while True:
        st, info = solver.advance(chunk)
        log(f"  [{label}] {info.steps} steps, residual {info.residual:.1e}, estimate {info.est_error:.1e} "
            f"({time.perf_counter() - t0:.0f}s)")
        if st != lbm.NOT_CONVERGED or info.steps >= solver.params.max_steps:
            return st, info, time.perf_counter() - t0


def study(name, seed, n, log=print):
    import torch

    ph = structure(name, seed, n)
    pore = ph == lbm.PORE
    dp = lbm.pore_size_device(pore)
    mean_dp = float(dp[torch.from_numpy(pore).cuda()].mean()) if pore.any() else 0.0
    out = {"variant": name, "seed": seed, "edge": n, "porosity": float(pore.mean()),
           "mean_pore_size_nm": mean_dp * VOXEL_M * 1e9}

    p = lbm.lbm_params_default(mode=lbm.MODE_DEFF, knudsen=1, check_every=1000, max_steps=20_000_000)
    s = lbm.Solver(ph, p, voxel_m=VOXEL_M)
    st, info, wall = _run(s, log, f"{name} seed {seed} D_eff")
    out.update(deff_over_db=s.deff()[1], deff_status=st, deff_steps=info.steps, deff_wall_s=round(wall, 1))
    s.close()

    p = lbm.lbm_params_default(mode=lbm.MODE_REACT, knudsen=1, k_lat=K_LAT,
                               catalyst_phases=(1 << lbm.CARBON) | (1 << lbm.PT), check_every=1000,
                               max_steps=20_000_000)
    s = lbm.Solver(ph, p, voxel_m=VOXEL_M)
    st, info, wall = _run(s, log, f"{name} seed {seed} reactive")
    act = torch.from_numpy(s.host_fields()[0].astype(bool)).cuda()
    c = s.concentration()
    last = act[:, :, -1]
    out.update(rate_per_area=s.reaction_rate()[1], react_status=st, react_steps=info.steps,
               react_wall_s=round(wall, 1),
               outlet_mean_c=float(c[:, :, -1][last].mean()) if bool(last.any()) else 0.0)
    s.close()
    log(json.dumps(out))
    return out


def main(argv):
    n = int(argv[0]) if argv else 128
    seeds = [int(a) for a in argv[1:]] or [1]
    lbm.require_gpu()
    rows = [study(name, seed, n) for seed in seeds for name in VARIANTS]
    summary = {}
    for name in VARIANTS:
        r = [x for x in rows if x["variant"] == name]
        summary[name] = {k: float(np.mean([x[k] for x in r])) for k in
                         ("porosity", "mean_pore_size_nm", "deff_over_db", "rate_per_area", "outlet_mean_c")}
    base = summary["original"]
    ratio = lambda a, b: a / b if b > 0 else None  # noqa: E731
    for name in ("A1", "A2"):
        summary[name]["deff_ratio_to_original"] = ratio(summary[name]["deff_over_db"], base["deff_over_db"])
        summary[name]["rate_ratio_to_original"] = ratio(summary[name]["rate_per_area"], base["rate_per_area"])
        summary[name]["outlet_c_ratio_to_original"] = ratio(summary[name]["outlet_mean_c"], base["outlet_mean_c"])
    print(json.dumps({"edge": n, "seeds": seeds, "k_lat": K_LAT, "summary": summary, "runs": rows}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
