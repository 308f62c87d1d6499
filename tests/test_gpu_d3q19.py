"""Parity of the D3Q19 HIP path (lbm19_* through the C ABI) with the D3Q19
oracle (Section 4, Eqs. 21-24).

Tolerances: each step rounds the shifted populations to FP32 once, so after a
few steps they agree with the FP64 oracle to a few FP32 ulps of the largest
concentration (absolute 2e-6 of it).  Steady outputs agree with the oracle's
exact fixed point to 1e-4 relative."""
import numpy as np
import pytest

import structgen as sg
from oracle import lbm as L
from oracle import lbm19 as O

pytestmark = pytest.mark.gpu

STEADY_RTOL = 1e-4


def _pair(hip, ph, mode, voxel_m=2e-9, **kw):
    okw = {k: v for k, v in kw.items() if k != "check_every"}
    okw["knudsen"] = bool(okw.get("knudsen", 0))
    prob = O.prepare(ph, L.Params(mode=mode, voxel_m=voxel_m, **okw))
    s = hip.Solver19(ph, hip.lbm_params_default(mode=mode, **kw), voxel_m=voxel_m)
    return prob, s


STEP_CASES = [
    ("pt_cl", 7, (20, 24, 70), L.MODE_DEFF, dict(knudsen=1)),
    ("pt_cl", 8, (20, 24, 70), L.MODE_DEFF, dict(tau_ref=0.7, d_ionomer_rel=0.05)),
    ("pt_cl", 9, (20, 24, 70), L.MODE_REACT, dict(knudsen=1, k_lat=0.05)),
    ("npmc_cl", 4, (16, 20, 45), L.MODE_REACT,
     dict(knudsen=1, k_lat=0.02, catalyst_phases=(1 << L.CARBON) | (1 << L.PT))),
    ("pt_cl", 5, (12, 18, 40), L.MODE_PROTON, {}),
    ("empty", 0, (1, 3, 33), L.MODE_DEFF, dict(tau_ref=1.3)),
    # rows of 64 k + 1 voxels: flat segment windows running on across row ends
    ("pt_cl", 11, (5, 7, 64), L.MODE_REACT, dict(knudsen=1, k_lat=0.05)),
    ("pt_cl", 12, (3, 2, 64), L.MODE_REACT, dict(k_lat=0.02)),
    ("pt_cl", 13, (4, 3, 129), L.MODE_DEFF, dict(knudsen=1)),
    ("pt_cl", 14, (3, 1, 128), L.MODE_REACT, dict(k_lat=0.02)),
]


def _structure(kind, seed, shape):
    if kind == "empty":
        return np.zeros(shape, np.uint8)
    return getattr(sg, kind)(seed, shape=shape)


@pytest.mark.parametrize("kind,seed,shape,mode,kw", STEP_CASES)
def test_steps_match_oracle(hip, kind, seed, shape, mode, kw):
    """The stored post-collision state after n steps, every population of every
    voxel, and the fluxes measured on the last step."""
    import torch

    ph = _structure(kind, seed, shape)
    prob, s = _pair(hip, ph, mode, **kw)
    print(f"[d3q19] steps {kind} seed {seed} {prob.active.shape} mode {mode}", flush=True)
    rng = np.random.default_rng(seed + 100)
    if mode == L.MODE_REACT:
        C0 = np.zeros(prob.active.shape)      # collide(0) = 0: the stored start is the oracle's
    else:
        C0 = (rng.random(prob.active.shape) * prob.active).astype(np.float32).astype(np.float64)
        s.set_initial_concentration(torch.from_numpy(C0.astype(np.float32)).cuda())
    f = O.equilibrium(prob, C0)
    pmap = O.pull_map(prob)
    n = 6
    s.step(n - 1)
    for _ in range(n - 1):
        f = O.step(prob, f, pmap)
    m = s.measure()
    before = O.fluxes(prob, f)
    f = O.step(prob, f, pmap)
    after = O.fluxes(prob, f)
    got = s.populations().cpu().numpy()
    want = O.collide(prob, f)
    scale = max(1.0, float(np.abs(C0).max()))
    err = np.abs(got - want).max()
    print(f"  max |f - f_oracle| = {err:.2e}", flush=True)
    assert err < 2e-6 * scale
    A = prob.ny * prob.nz
    tol = 2e-6 * scale * prob.active.sum() / A
    assert abs(m.j_in - before.j_in) < tol
    assert abs(m.j_out - before.j_out) < tol
    assert abs(m.j_vol - before.j_vol) < tol
    assert abs(m.mass - after.mass) < 2e-6 * scale * prob.active.sum()
    assert abs(m.rate - after.rate) < tol
    conc = s.concentration().cpu().numpy()
    assert np.abs(conc - O.concentration(f)).max() < 4e-6 * scale


STEADY_CASES = [
    (3, L.MODE_DEFF, dict(knudsen=1)),
    (4, L.MODE_DEFF, dict(tau_ref=0.8, d_ionomer_rel=0.05)),
    (3, L.MODE_REACT, dict(knudsen=1, k_lat=1e-2)),
    (5, L.MODE_REACT, dict(k_lat=3e-2, catalyst_phases=(1 << L.CARBON) | (1 << L.PT))),
]


@pytest.mark.parametrize("seed,mode,kw", STEADY_CASES)
def test_steady_state_matches_oracle_fixed_point(hip, seed, mode, kw):
    ph = sg.pt_cl(seed, shape=(10, 12, 20))
    prob, s = _pair(hip, ph, mode, check_every=200, **kw)
    assert prob.percolates
    ref = O.solve_fixed_point(prob)
    st, info = s.run_to_steady()
    assert st == 0, info.as_dict()
    if mode == L.MODE_REACT:
        got, want = s.reaction_rate()[1], ref.rate
    else:
        got, want = s.deff()[1], ref.deff
    print(f"[d3q19] steady seed {seed} mode {mode}: {got:.8g} vs oracle {want:.8g} "
          f"({got / want - 1:+.1e}), {info.steps} steps", flush=True)
    assert abs(got / want - 1) < STEADY_RTOL


def test_empty_box_and_no_percolation(hip):
    s = hip.Solver19(np.zeros((3, 5, 37), np.uint8), hip.lbm_params_default(tau_ref=0.9, check_every=100))
    st, _ = s.run_to_steady()
    assert st == 0
    assert s.deff()[1] == pytest.approx(1.0, rel=1e-5)
    ph = np.zeros((4, 4, 12), np.uint8)
    ph[:, :, 6] = L.CARBON
    s = hip.Solver19(ph, hip.lbm_params_default())
    st, _ = s.run_to_steady()
    assert st == hip.ERR_NO_PERCOLATION
    assert s.deff() == (hip.ERR_NO_PERCOLATION, 0.0)


def test_mass_balance_at_full_size(hip):
    """At the 256^3 NPMC size, where the oracle cannot follow step by step: every
    step changes the total of C by (J_in - J_out - R) times the area, with the
    fluxes of the links it moved and the sink of the state it started from, to
    FP32 rounding of the stored values."""
    ph = sg.npmc_cl(1, n=256)
    p = hip.lbm_params_default(mode=hip.MODE_REACT, knudsen=1, k_lat=1e-4,
                               catalyst_phases=(1 << hip.CARBON) | (1 << hip.PT))
    s = hip.Solver19(ph, p, voxel_m=1e-9)
    A = s.info.ny * s.info.nz
    s.step(200)
    prev = s.measure()
    for _ in range(3):
        # the step's link fluxes, and the sink of the state it started from
        m = s.measure()
        dm = m.mass - prev.mass
        flux = (m.j_in - m.j_out - prev.rate) * A
        print(f"[d3q19] 256^3: dmass {dm:.6e}, (J_in - J_out - R) A {flux:.6e}", flush=True)
        assert abs(dm - flux) < 1e-5 * abs(flux) + 2e-8 * m.mass
        prev = m


def test_steady_state_on_flat_windows_matches_oracle_fixed_point(hip):
    """A reactive layer whose reservoir plane makes 65-voxel rows (flat segment
    windows) against the oracle's exact fixed point."""
    ph = sg.pt_cl(6, shape=(8, 9, 64))
    prob, s = _pair(hip, ph, L.MODE_REACT, check_every=200, knudsen=1, k_lat=1e-2)
    assert prob.percolates
    ref = O.solve_fixed_point(prob)
    st, info = s.run_to_steady()
    assert st == 0
    rate = s.reaction_rate()[1]
    print(f"[d3q19] flat steady: {rate:.10g} vs oracle {ref.rate:.10g}, {info.steps} steps", flush=True)
    assert rate == pytest.approx(ref.rate, rel=1e-4)
