"""What the trained warm-start networks change: the number of LBM steps, never the answer.

The networks are the committed weights. The structures are fresh seeds, unseen in
training (training seeds start at 10000).

* On the effective-diffusivity workload, the learned start must save at least 25%
  of the cold start's steps. Measured at 192^3 the saving is about 1.8x.
* Both workloads must reach the cold start's output.
* A start that is not finite must take the cold fallback.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ws(hip):
    from paper_1410_1914_amd import warmstart

    return warmstart


def _solver(ws, w, seed, shape):
    ph = ws.structure(seed, shape)
    s = ws.lbm.Solver(ph, ws.params(w), voxel_m=ws.VOXEL_M)
    return s, s.host_fields()


def test_learned_start_saves_steps_on_deff(ws):
    w = ws.WORKLOADS["deff"]
    net = ws.unet.UNet.from_file(w.weights)
    s, (act, ncat, om) = _solver(ws, w, 20002, (96, 96, 96))
    cold = ws.solve(s, w, None)
    warm = ws.solve(s, w, ws.predict(net, w, act, ncat, om))
    print(f"[warm] deff 96^3: cold {cold['steps']} steps, learned {warm['steps']} steps, "
          f"D_eff {cold['out']:.8f} vs {warm['out']:.8f}", flush=True)
    assert cold["status"] == 0 and warm["status"] == 0 and not warm["fallback"]
    assert warm["steps"] < 0.75 * cold["steps"]
    assert warm["out"] == pytest.approx(cold["out"], rel=1e-4)


def test_learned_start_keeps_the_reactive_answer(ws):
    w = ws.WORKLOADS["react"]
    net = ws.unet.UNet.from_file(w.weights)
    s, (act, ncat, om) = _solver(ws, w, 20003, (96, 96, 95))
    cold = ws.solve(s, w, None)
    warm = ws.solve(s, w, ws.predict(net, w, act, ncat, om, s.pore_depth()))
    print(f"[warm] react 96^3: cold {cold['steps']} steps, learned {warm['steps']} steps, "
          f"rate {cold['out']:.9e} vs {warm['out']:.9e}", flush=True)
    assert cold["status"] == 0 and warm["status"] == 0
    assert warm["out"] == pytest.approx(cold["out"], rel=1e-4)


def test_non_finite_start_falls_back_to_cold(ws):
    import torch

    w = ws.WORKLOADS["react"]
    s, (act, _, _) = _solver(ws, w, 20004, (16, 16, 63))
    cold = ws.solve(s, w, None)
    bad = torch.full(act.shape, float("nan"), dtype=torch.float32, device="cuda")
    r = ws.solve(s, w, bad)
    assert r["fallback"] and r["status"] == 0
    assert r["steps"] == cold["steps"]
    assert r["out"] == cold["out"]
    assert np.isfinite(r["out"])


def _golden(name):
    """The stored oracle fixed point of a grid the network takes (sizes multiples of
    8): the 64^3 D_eff cube, and the 64 x 64 x 63 reactive layer whose reservoir
    plane makes it 64^3 simulated."""
    import json
    import os

    fname, mode = {"deff": ("oracle_pt_cl_64.json", 0), "react": ("oracle_pt_cl_react_64x64x63.json", 1)}[name]
    with open(os.path.join(os.path.dirname(__file__), "golden", fname)) as fh:
        return next(c for c in json.load(fh)["cases"] if c["mode"] == mode)


@pytest.mark.parametrize("name", ["react", "deff"])
def test_learned_start_reaches_the_oracle_fixed_point(ws, name):
    """A warm-started solve ends at the oracle's exact fixed point, not merely at the
    GPU's own cold solve (the workloads' physics: Knudsen, 2 nm voxels, k 1e-2 per
    Pt face when reactive), within 1e-4."""
    import structgen as sg

    w = ws.WORKLOADS[name]
    case = _golden(name)
    net = ws.unet.UNet.from_file(w.weights)
    ph = sg.pt_cl(case["seed"], shape=tuple(case.get("shape", (64, 64, 64))))
    s = ws.lbm.Solver(ph, ws.params(w, max_steps=20_000_000), voxel_m=ws.VOXEL_M)
    assert s.info.n_active == case["n_active"]
    act, ncat, om = s.host_fields()
    extra = (s.pore_depth(),) if name == "react" else ()
    warm = ws.solve(s, w, ws.predict(net, w, act, ncat, om, *extra))
    want = case["rate"] if name == "react" else case["deff"]
    err = abs(warm["out"] / want - 1)
    print(f"[warm] {name} {s.shape} learned start: {warm['steps']} steps, {warm['out']:.10g} vs oracle "
          f"{want:.10g} (rel {err:.2e}), fallback {warm['fallback']}", flush=True)
    assert warm["status"] == 0
    assert err < 1e-4


@pytest.mark.parametrize("name,seed,shape", [("deff", 20002, (96, 96, 96)), ("react", 20003, (96, 96, 95))])
def test_learned_start_matches_the_better_simple_start(ws, name, seed, shape):
    """What the network gains over the method without it: each simple start is good
    on one problem only (C = 0 on the reactive problem, the linear profile between
    the Dirichlet faces on D_eff), and the learned start, not told which problem it
    faces beyond its inputs, needs at most 15% more steps than the better of the two
    on both (measured at 192^3: 0.98x the linear start on D_eff, 0.90x the cold
    start on the reactive problem)."""
    w = ws.WORKLOADS[name]
    net = ws.unet.UNet.from_file(w.weights)
    s, (act, ncat, om) = _solver(ws, w, seed, shape)
    cold = ws.solve(s, w, None)
    lin = ws.solve(s, w, ws.linear_profile(act.shape))
    extra = (s.pore_depth(),) if name == "react" else ()
    warm = ws.solve(s, w, ws.predict(net, w, act, ncat, om, *extra))
    best = min(cold["steps"], lin["steps"])
    print(f"[warm] {name} {shape}: cold {cold['steps']}, linear {lin['steps']}, learned {warm['steps']} steps "
          f"({best / warm['steps']:.2f}x the better simple start)", flush=True)
    assert cold["status"] == lin["status"] == warm["status"] == 0
    assert warm["steps"] <= 1.15 * best
    assert warm["out"] == pytest.approx(cold["out"], rel=1e-4)
