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


def pt_cl_slab():
    """Four-phase Pt catalyst layers at 2 nm (carbon + Pt 0.35, ionomer 0.20, pores
    0.45), Knudsen pore diffusivity, ionomer 1e-3 D0, as 32 x 32 x 130 slabs (rows of
    130 voxels along the transport axis x): D_eff/D0, and the reaction rate (k = 1e-2
    per Pt face) with the inlet reservoir plane prepended to a 32 x 32 x 129 structure,
    each at the exact fixed point (sparse LU)."""
    out = []
    for seed in (7, 8):
        for mode, shape, k in ((O.MODE_DEFF, (32, 32, 130), 0.0), (O.MODE_REACT, (32, 32, 129), 1e-2)):
            ph = sg.pt_cl(seed, shape=shape)
            t = time.time()
            s = O.solve_fixed_point(O.prepare(ph, O.Params(mode=mode, knudsen=True, voxel_m=2e-9, k_lat=k)),
                                    "direct")
            out.append({"seed": seed, "shape": list(shape), "mode": mode, "k_lat": k, "deff": s.deff,
                        "rate": s.rate, "j_in": s.fluxes.j_in, "seconds": round(time.time() - t, 1)})
            print(out[-1], flush=True)
    return {"workload": "Pt CL slabs at 2 nm, Knudsen, ionomer 1e-3 D0; D_eff and reactive (k 1e-2) problems",
            "generator": "structgen.pt_cl(seed, shape=...)", "solver": "oracle.lbm.solve_fixed_point (sparse LU)",
            "cases": out}


def pt_cl_cube(n, modes=("react", "deff")):
    """Four-phase Pt catalyst layer cubes at 2 nm (the 128^3 layer of the paper's
    Pt workload, and a 64^3 one), seed 1, Knudsen pore diffusivity, ionomer 1e-3 D0:
    the reaction rate (k = 1e-2 per Pt face, inlet reservoir plane prepended) and
    D_eff/D0, each at the exact fixed point.  Too large for the sparse LU, so the
    route is restarted GMRES preconditioned by an incomplete LU of the same matrix,
    to a true residual of 1e-13 of the right-hand side, then certified as a fixed
    point by one plain time step (relative change of C below 1e-12)."""
    out = []
    ph = sg.pt_cl(1, n=n)
    for mode in modes:
        m, k = (O.MODE_REACT, 1e-2) if mode == "react" else (O.MODE_DEFF, 0.0)
        t = time.time()
        prob = O.prepare(ph, O.Params(mode=m, knudsen=True, voxel_m=2e-9, k_lat=k))
        s = O.solve_fixed_point(prob, "gmres", tol=1e-13)
        out.append({"seed": 1, "edge": n, "mode": m, "k_lat": k, "deff": s.deff, "rate": s.rate,
                     "j_in": s.fluxes.j_in, "j_out": s.fluxes.j_out, "n_active": int(prob.active.sum()),
                     "seconds": round(time.time() - t, 1)})
        print(out[-1], flush=True)
    return {"workload": f"Pt CL {n}^3 at 2 nm (structgen.pt_cl(1, n={n})), Knudsen, ionomer 1e-3 D0; "
                        "reactive (k 1e-2 per Pt face) and D_eff problems",
            "generator": f"structgen.pt_cl(1, n={n})",
            "solver": "oracle.lbm.solve_fixed_point(method='gmres', tol=1e-13): ILU-preconditioned GMRES, "
                      "certified by one plain step",
            "cases": out}


def pt_cl_react_64x64x63():
    """The reactive Pt layer on a 64 x 64 x 63 structure (structgen.pt_cl(1, shape=(64,
    64, 63))): with its inlet reservoir plane the simulated grid is 64^3, a grid the
    warm-start network takes (each size a multiple of 8).  Knudsen, 2 nm voxels, k = 1e-2
    per Pt face; the certified GMRES route as for the cubes."""
    ph = sg.pt_cl(1, shape=(64, 64, 63))
    t = time.time()
    prob = O.prepare(ph, O.Params(mode=O.MODE_REACT, knudsen=True, voxel_m=2e-9, k_lat=1e-2))
    s = O.solve_fixed_point(prob, "gmres", tol=1e-13)
    case = {"seed": 1, "shape": [64, 64, 63], "mode": O.MODE_REACT, "k_lat": 1e-2, "rate": s.rate,
            "j_in": s.fluxes.j_in, "n_active": int(prob.active.sum()), "seconds": round(time.time() - t, 1)}
    print(case, flush=True)
    return {"workload": "Pt CL 64 x 64 x 63 at 2 nm (64^3 simulated with the reservoir plane), Knudsen, "
                        "ionomer 1e-3 D0, reactive k 1e-2 per Pt face",
            "generator": "structgen.pt_cl(1, shape=(64, 64, 63))",
            "solver": "oracle.lbm.solve_fixed_point(method='gmres', tol=1e-13), certified by one plain step",
            "cases": [case]}


def coupled_16():
    """The coupled O2 / proton-potential problem (Eqs. 15-18b, Tafel Eq. 17b) on a
    16^3 Pt catalyst layer whose membrane face is ionomer (structgen.pt_cl(5,
    shape=(16, 16, 16)), pores of the x = L plane turned to ionomer), proton source
    gamma = 5e-3 V, other coupling parameters at their defaults: the oracle's Picard
    iteration on exact D3Q19 fixed points to a potential change of 1e-10 V.  The
    potential is stored on the structure grid (phi_m off the potential's voxels)."""
    from oracle import coupled as CO

    ph = sg.pt_cl(5, shape=(16, 16, 16))
    skin = ph[:, :, -1]
    skin[skin == O.PORE] = O.IONOMER
    t = time.time()
    r = CO.solve(ph, O.Params(), CO.Coupling(gamma=5e-3))
    out = {"seed": 5, "shape": [16, 16, 16], "gamma": 5e-3, "iterations": r.iterations, "rate": r.rate,
           "proton_in": r.proton_in, "source": r.source, "phi_min": float(r.phi.min()),
           "phi": [float("%.12g" % v) for v in r.phi.ravel()], "seconds": round(time.time() - t, 1)}
    print({k: v for k, v in out.items() if k != "phi"}, flush=True)
    return {"workload": "coupled O2 / proton potential, Pt CL 16^3 with an ionomer membrane face, gamma 5e-3 V",
            "generator": "structgen.pt_cl(5, shape=(16, 16, 16)) with the x = L plane's pores made ionomer",
            "solver": "oracle.coupled.solve (Picard on exact D3Q19 fixed points, sparse LU)", "cases": [out]}


GOLDEN = {"oracle_two_phase_32.json": two_phase_32, "oracle_pt_cl_slab.json": pt_cl_slab,
          "oracle_coupled_16.json": coupled_16, "oracle_pt_cl_react_64x64x63.json": pt_cl_react_64x64x63,
          "oracle_pt_cl_64.json": lambda: pt_cl_cube(64), "oracle_pt_cl_128.json": lambda: pt_cl_cube(128)}

if __name__ == "__main__":
    names = sys.argv[1:] or list(GOLDEN)
    for name in names:
        data = GOLDEN[name]()
        with open(os.path.join(HERE, name), "w") as fh:
            json.dump(data, fh, indent=1)
