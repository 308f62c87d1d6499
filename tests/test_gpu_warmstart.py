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
