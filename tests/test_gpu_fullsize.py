"""Parity at the full workload sizes, in the launch configuration the benchmark times.

The oracle cannot reach the fixed point of a 128^3 or 256^3 structure in seconds,
but it can take one exact FP64 step.  So each case:

* autotunes the HIP solver (the benchmark's launch configuration);
* writes a seeded random state over every fluid voxel of the grid
  (lbm_set_populations), so that no voxel is near equilibrium: a gather from a
  wrong neighbour, a wrong bounce-back, a wrong relaxation rate or a wrong segment
  offset anywhere in the grid changes the result;
* streams and collides that stored state once with the oracle;
* compares with the GPU's next stored state, element by element over every fluid
  voxel;
* compares the FP64 reductions (fluxes, sink, mass) of a state against the
  oracle's.

The tolerance is that of the small step tests: a few FP32 ulps of the largest
population."""
import numpy as np
import pytest

import structgen as sg
from oracle import lbm as O

pytestmark = pytest.mark.gpu

CASES = [
    # Pt catalyst layer 128^3 at 2 nm: reactive k = 1e-2 on Pt faces, Knudsen, ionomer 1e-3 D0
    ("pt_cl_128", lambda: sg.pt_cl(1, n=128), 2e-9, dict(mode=1, knudsen=1, k_lat=1e-2)),
    # NPMC catalyst layer 256^3 at 1 nm: every carbon/Pt face reactive, k = 1e-4, Knudsen
    ("npmc_cl_256", lambda: sg.npmc_cl(1, n=256), 1e-9,
     dict(mode=1, knudsen=1, k_lat=1e-4, catalyst_phases=(1 << O.CARBON) | (1 << O.PT))),
]


@pytest.mark.parametrize("name,make,voxel,kw", CASES, ids=[c[0] for c in CASES])
def test_full_size_step_and_reductions(hip, name, make, voxel, kw):
    import torch

    print(f"[fullsize] {name}: generating", flush=True)
    ph = make()
    s = hip.Solver(ph, hip.lbm_params_default(check_every=100, **kw), voxel_m=voxel)
    s.autotune(5)  # the benchmark's launch configuration (also advances the state)
    # a random state far from equilibrium on every voxel (populations in [0, 0.5))
    s.set_populations(torch.from_numpy(sg.random_state(41, s.shape, scale=0.5)).cuda())
    torch.cuda.synchronize()
    print(f"[fullsize] {name}: tiling {s.tiling()}, oracle preparation", flush=True)
    okw = dict(kw)
    okw["knudsen"] = bool(okw["knudsen"])
    prob = O.prepare(ph, O.Params(voxel_m=voxel, **okw))
    act = prob.active.ravel()
    assert np.array_equal(s.host_fields()[0].ravel().astype(bool), act)

    g = s.populations().cpu().numpy().reshape(7, -1).astype(np.float64)  # stored post-collision state
    # the state is far from equilibrium everywhere: the non-equilibrium part is of
    # the order of the populations themselves on every fluid voxel
    ceq = g.sum(axis=0)
    w = O.weights(0.25)
    neq = np.abs(g - w[:, None] * ceq[None, :])[:, act].max(axis=0)
    assert np.quantile(neq, 0.01) > 0.02
    s.step(1)
    got = s.populations().cpu().numpy().reshape(7, -1)
    f1 = O.stream(prob, g)
    want = O.collide(prob, f1)
    scale = max(1.0, float(np.abs(want).max()))
    err = float(np.abs(got[:, act] - want[:, act]).max())
    print(f"[fullsize] {name}: one step, max |GPU - oracle| = {err:.2e} (scale {scale:.2f})", flush=True)
    assert err < 2e-6 * scale

    # FP64 reductions of the state whose pre-collision populations are f1
    s.set_populations(torch.from_numpy(want.astype(np.float32)).reshape((7,) + s.shape))
    m = s.measure()
    ref = O.fluxes(prob, f1)
    sc = max(abs(ref.j_in), abs(ref.rate), 1e-30)
    print(f"[fullsize] {name}: j_in {m.j_in:.9e} vs {ref.j_in:.9e}, rate {m.rate:.9e} vs {ref.rate:.9e}", flush=True)
    assert m.j_in == pytest.approx(ref.j_in, abs=1e-6 * sc)
    assert m.rate == pytest.approx(ref.rate, abs=1e-6 * sc)
    assert m.mass == pytest.approx(ref.mass, rel=1e-6)


def test_batched_instances_match_single_solves(hip):
    """Instances of the batched workload (uneven sizes, porosities and rates, one
    launch per step) reach the single-solver answers."""
    import torch

    phases, ks = [], []
    for i, (edge, por, k) in enumerate([(48, 0.45, 3e-2), (64, 0.6, 1e-3), (48, 0.35, 1e-1), (64, 0.5, 1e-4)]):
        phases.append(sg.pt_cl(2024000 + i, shape=(edge, edge, edge), carbon=(1 - por) * 0.35 / 0.55,
                               ionomer=(1 - por) * 0.20 / 0.55))
        ks.append(k)
    params = [hip.lbm_params_default(mode=1, k_lat=k, check_every=200) for k in ks]
    b = hip.Batch(phases, params)
    b.autotune(5)
    st, infos = b.run()
    assert st == 0
    torch.cuda.synchronize()
    for i, ph in enumerate(phases):
        s = hip.Solver(ph, params[i])
        st1, _ = s.run_to_steady()
        assert st1 == 0
        r_single = s.reaction_rate()[1]
        r_batch = b.reaction_rate(i)[1]
        print(f"[batch] instance {i}: rate batched {r_batch:.9e} single {r_single:.9e}", flush=True)
        assert r_batch == pytest.approx(r_single, rel=2e-5)
        cb = b.concentration(i)
        assert torch.allclose(cb, s.concentration(), rtol=0, atol=2e-4)


# The reactive workloads' 129- and 257-voxel rows are cut into flat windows, which
# the two-step kernel does not tile; its full-size cases are the same structures'
# effective-diffusivity problems (128- and 256-voxel rows).
CASES2 = [
    ("pt_cl_128_deff", lambda: sg.pt_cl(1, n=128), 2e-9, dict(mode=0, knudsen=1)),
    ("npmc_cl_256_deff", lambda: sg.npmc_cl(1, n=256), 1e-9, dict(mode=0, knudsen=1)),
]


@pytest.mark.parametrize("name,make,voxel,kw", CASES2, ids=[c[0] for c in CASES2])
def test_full_size_two_step_launch_is_bit_identical(hip, name, make, voxel, kw):
    """One launch of the two-step kernel (the autotuner's other form) against two
    single-step launches, from a seeded random state over the whole full-size
    structure (far from equilibrium on every voxel, so every halo row, chunk-end
    plane and x-edge voxel of every tile matters).  Both runs start from the same
    dense state written with lbm_set_populations."""
    import torch

    ph = make()
    s = hip.Solver(ph, hip.lbm_params_default(check_every=100, **kw), voxel_m=voxel)
    f0 = torch.from_numpy(sg.random_state(43, s.shape, scale=0.5)).cuda()
    s.set_temporal(0)
    s.set_populations(f0)
    g0 = s.populations().cpu().numpy().reshape(7, -1).astype(np.float64)  # the state as stored
    s.step(2)
    ref = s.populations()
    # the two single steps against two exact FP64 oracle steps, over every fluid voxel
    okw = dict(kw)
    okw["knudsen"] = bool(okw["knudsen"])
    prob = O.prepare(ph, O.Params(voxel_m=voxel, **okw))
    act = prob.active.ravel()
    # the stored states are post-collision: each step streams, then collides
    want = O.collide(prob, O.stream(prob, O.collide(prob, O.stream(prob, g0))))
    got2 = ref.cpu().numpy().reshape(7, -1)
    scale = max(1.0, float(np.abs(want).max()))
    err = float(np.abs(got2[:, act] - want[:, act]).max())
    print(f"[fullsize] {name}: two steps, max |GPU - oracle| = {err:.2e} (scale {scale:.2f})", flush=True)
    assert err < 4e-6 * scale
    for by, zc in ((6, 16), (8, 64)):
        s.set_populations(f0)
        s.set_temporal(by, zc)
        s.step(2)
        got = s.populations()
        print(f"[fullsize] {name}: two-step tile {by}x{zc} bit-identical: {bool(torch.equal(got, ref))}", flush=True)
        assert torch.equal(got, ref)
    s.set_temporal(0)
