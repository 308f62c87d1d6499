"""Learned warm start for the catalyst-layer solves.

The structures are four-phase Pt catalyst layers at 2 nm voxels: carbon + Pt 0.35,
ionomer 0.20, Pt on 10% of the carbon-pore faces, pores 0.45. The problems use
Knudsen pore diffusivity and ionomer D = 1e-3 D0 (Chen et al., arXiv 1410.1914,
Sections 3.4-3.5). There are two workloads, each with its own network:

* ``react``: the reactive problem of Section 3.5.2, with a first-order sink
  k = 1e-2 (lattice units) per Pt face. Its boundaries are the inlet reservoir
  plane, Dirichlet inlet, zero-gradient outlet, and periodic y and z. Structures
  are 95 voxels long in x, so the simulated grid, reservoir plane included, is a
  multiple of 8 for the network's three poolings. The network predicts
  ln(C + 1e-3), so its error is relative to C.
* ``deff``: the effective-diffusivity problem of Section 3.5.1 (Eq. 19), Dirichlet
  C = 1 and C = 0 at the x faces. The network predicts the corrector
  N_x (C - linear profile). For a statistically uniform structure that field
  depends on the local structure only, so training on 64^3 transfers to 192^3.

Pipeline:
  1. Training fields are the batched HIP solver's steady states on seeded structures.
  2. The U-Net of ``unet.py`` trains on the GPU with the project's own kernels. The
     loss is a masked MSE weighted by sqrt(D_ref / D) (capped), so slowly relaxing
     ionomer counts more.
  3. To use it: features of a new structure -> predicted field -> equilibrium
     populations (``lbm_set_initial_concentration``) -> the solver refines to its own
     stop rule. If the windowed residual rises between the first two checks, the
     solve falls back to the cold start. The network can never change the answer,
     only the number of steps.

In the reactive problem, the steps a solve needs are set by the voxels that relax
slowest: ionomer films and blobs (D = 1e-3 D0, tau close to 1/2). Their
concentration is small, so the cold start's error there is already small. A
prediction only helps where its error is smaller still. Deep inside the ionomer,
beyond ``depth_max`` voxels from the connected pores (lbm_get_pore_depth), the
trained network's error is not smaller, and the start keeps C = 0 there.
"""
from __future__ import annotations

import json
import os
import sys
import time
from dataclasses import dataclass

import numpy as np

from . import lbm, unet

HERE = os.path.dirname(os.path.abspath(__file__))
VOXEL_M = 2e-9
WEIGHT_POWER = 0.5
WEIGHT_CAP = 32.0
C_MAX = 1.5         # upper clip of a predicted start (the discrete field may exceed C_in slightly)


@dataclass(frozen=True)
class Workload:
    name: str
    mode: int
    k_lat: float
    train_shape: tuple    # structure (nz, ny, nx)
    test_shape: tuple
    target: str           # "log": ln(C + eps); "corrector": N_x (C - linear profile)
    target_eps: float = 0.0
    depth_max: int = -1   # >= 0: keep the prediction up to this pore depth, C = 0 deeper in
    description: str = ""
    chunk: int = 0        # > 0: test solves advance in chunks of this many steps, printing progress

    @property
    def weights(self):
        return os.path.join(HERE, "weights", f"unet_{self.name}_ptcl.npz")


WORKLOADS = {
    "react": Workload("react", lbm.MODE_REACT, 1e-2, (96, 96, 95), (192, 192, 191), "log", target_eps=1e-3,
                      # depth limit chosen on validation structures (seeds 30000 and 30001)
                      depth_max=4,
                      description="Pt CL reactive, k=1e-2 per Pt face, Knudsen"),
    "deff": Workload("deff", lbm.MODE_DEFF, 0.0, (64, 64, 64), (192, 192, 192), "corrector",
                     description="Pt CL effective diffusivity, Knudsen", chunk=400_000),
}


def params(w: Workload, **kw):
    p = lbm.lbm_params_default(mode=w.mode, knudsen=1, k_lat=w.k_lat, check_every=200)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def structure(seed, shape):
    import structgen as sg

    return sg.pt_cl(seed, shape=shape)


def _structures(seeds, shape, workers=16):
    """Generate structures on host processes (done before any GPU work)."""
    from concurrent.futures import ProcessPoolExecutor

    with ProcessPoolExecutor(max_workers=min(workers, len(seeds))) as ex:
        return list(ex.map(structure, seeds, [shape] * len(seeds)))


# ------------------------------------------------------------------ features and prediction

def _ncat_input(w: Workload, ncat):
    # catalyst counts only matter where a sink acts
    return ncat if w.mode == lbm.MODE_REACT else np.zeros_like(ncat)


def features(w: Workload, active, ncat, omega, tau_ref=1.0):
    """BF16 (V, 16) network input from the solver's dense host fields (simulated grid)."""
    import torch

    shape = active.shape
    feat = torch.empty((int(np.prod(shape)), unet.IN_CH), dtype=torch.bfloat16, device="cuda")
    a = torch.from_numpy(np.ascontiguousarray(active)).cuda()
    n = torch.from_numpy(np.ascontiguousarray(_ncat_input(w, ncat))).cuda()
    o = torch.from_numpy(np.ascontiguousarray(omega)).cuda()
    unet.unet_features(a, n, o, tau_ref, feat, shape)
    return feat, a


def predict(net, w: Workload, active, ncat, omega, depth=None, depth_max=None):
    """Start field for the solver (FP32, dense simulated grid, on the GPU), by one
    unet_predict call on the solver's dense fields.

    ``react``: the predicted steady concentration; when the pore-depth map is given,
    the cold value 0 in voxels deeper than depth_max. ``deff``: the linear profile
    plus the predicted corrector."""
    import torch

    a = torch.from_numpy(np.ascontiguousarray(active)).cuda()
    o = torch.from_numpy(np.ascontiguousarray(omega)).cuda()
    n = torch.from_numpy(np.ascontiguousarray(ncat)).cuda() if w.mode == lbm.MODE_REACT else None
    d = torch.from_numpy(np.ascontiguousarray(depth)).cuda() if depth is not None else None
    if w.target == "corrector":
        p = params(w)
        tgt = unet.unet_target(kind=unet.UNET_TARGET_CORRECTOR, eps=1.0, cmax=C_MAX, c_in=p.c_in, c_out=p.c_out)
    else:
        tgt = unet.unet_target(kind=unet.UNET_TARGET_LOG, eps=w.target_eps, cmax=C_MAX,
                               depth=d.data_ptr() if d is not None else None,
                               depth_max=w.depth_max if depth_max is None else depth_max)
    return net.predict(a, n, o, 1.0, tgt)


# ------------------------------------------------------------------ solves

def _output(solver, w: Workload):
    if w.mode == lbm.MODE_REACT:
        return solver.reaction_rate()[1]
    return solver.deff()[1]


def solve(solver, w: Workload, c0=None, fallback=True, chunk=0, log=None):
    """Steady solve from c0 (None: cold start C = 0).  Returns a dict with the steps,
    wall time, status, output (reaction rate or D_eff/D0) and whether the cold
    fallback was taken.  With chunk > 0 the solve runs as successive lbm_advance
    calls of at most that many steps, each followed by a progress line."""
    import torch

    t0 = time.perf_counter()
    solver.set_initial_concentration(c0)
    K = solver.params.check_every
    used_fallback = False
    spent = 0  # steps taken from a rejected start (they count against it)
    if c0 is not None and fallback and not bool(torch.isfinite(c0).all()):
        used_fallback = True
        solver.set_initial_concentration(None)
    elif c0 is not None and fallback:
        _, i1 = solver.advance(K)
        st, i2 = solver.advance(K)
        if st != lbm.OK and i2.residual > i1.residual:
            used_fallback = True
            spent = int(i2.steps)
            solver.set_initial_concentration(None)
    if chunk > 0:
        while True:
            st, info = solver.advance(chunk)
            if log:
                log(f"  ... {info.steps} steps, residual {info.residual:.2e}, estimate {info.est_error:.1e}, "
                    f"status {st} ({time.perf_counter() - t0:.0f}s)")
            if st != lbm.NOT_CONVERGED or info.steps >= solver.params.max_steps:
                break
    else:
        st, info = solver.run_to_steady()
    torch.cuda.synchronize()
    return {"status": st, "steps": int(info.steps) + spent, "wall_s": time.perf_counter() - t0,
            "out": _output(solver, w), "fallback": used_fallback, "steps_before_fallback": spent}


# ------------------------------------------------------------------ training data

def make_dataset(w: Workload, seeds, batch=32, tol_flux=1e-4, tol_change=1e-8, log=print):
    """Steady fields of the batched solver.  Returns a list of per-sample dicts of
    GPU tensors (active u8, ncat u8, omega f32, target f32) and host shape."""
    import torch

    phases = _structures(list(seeds), w.train_shape)
    data = []
    for s0 in range(0, len(phases), batch):
        chunk = phases[s0:s0 + batch]
        t = time.perf_counter()
        b = lbm.Batch(chunk, [params(w, tol_flux=tol_flux, tol_change=tol_change) for _ in chunk], voxel_m=VOXEL_M)
        st, infos = b.run()
        for i in range(len(chunk)):
            act, ncat, om = b.host_fields(i)
            data.append({"active": torch.from_numpy(act).cuda(),
                         "ncat": torch.from_numpy(np.ascontiguousarray(_ncat_input(w, ncat))).cuda(),
                         "omega": torch.from_numpy(om).cuda(), "target": b.concentration(i).clone(),
                         "shape": act.shape, "count": int(act.sum()), "steps": int(infos[i].steps)})
        del b
        torch.cuda.synchronize()
        log(f"[data] {s0 + len(chunk)}/{len(phases)} fields, batch of {len(chunk)} in {time.perf_counter() - t:.1f}s "
            f"(mean steps {np.mean([x['steps'] for x in data[-len(chunk):]]):.0f}, status {st})")
    return data


def _targets(w: Workload, data):
    """The network's target of every sample (kept with the sample)."""
    import torch

    p = params(w)
    for d in data:
        if d.get("y_key") == w.name:
            continue
        t = d["target"].view(-1)
        d["y"] = torch.empty_like(t)
        if w.target == "log":
            unet.unet_log_map(t, d["y"], t.numel(), w.target_eps, False)
        else:
            unet.unet_corrector_map(t, d["y"], t.numel(), d["shape"][2], p.c_in, p.c_out, False)
        d["y_key"] = w.name


def _features_dev(d, weight_power=WEIGHT_POWER, weight_cap=WEIGHT_CAP):
    """Features and per-voxel loss weights of one training sample (on the GPU)."""
    import torch

    shape = d["shape"]
    feat = torch.empty((int(np.prod(shape)), unet.IN_CH), dtype=torch.bfloat16, device="cuda")
    weight = torch.empty(int(np.prod(shape)), dtype=torch.float32, device="cuda")
    unet.unet_features(d["active"], d["ncat"], d["omega"], 1.0, feat, shape, weight, weight_power, weight_cap)
    return feat, weight


def train(net, w: Workload, data, epochs=4, lr=1e-3, log=print, seed=0, weight_power=WEIGHT_POWER,
          weight_cap=WEIGHT_CAP):
    """Adam on the weighted masked MSE, cosine learning-rate decay; returns the loss
    history.  The weight of a voxel is (D_ref / D)^weight_power capped at weight_cap:
    an error left in a low-diffusivity voxel (ionomer) relaxes slowly, so it costs
    the solver far more steps than the same error in a pore."""
    import torch

    rng = np.random.default_rng(seed)
    hist = []
    total = epochs * len(data)
    _targets(w, data)
    if net.t == 0:  # start the output bias at the mean target
        m = float(np.mean([float(d["y"][d["active"].view(-1) > 0].mean()) for d in data[:32]]))
        net.B["head"].fill_(m)
        net.touch()
    net.target_eps = w.target_eps
    step = 0
    for ep in range(epochs):
        order = rng.permutation(len(data))
        t = time.perf_counter()
        losses = []
        for idx in order:
            d = data[idx]
            feat, weight = _features_dev(d, weight_power, weight_cap)
            lr_t = lr * 0.5 * (1 + np.cos(np.pi * step / total))
            loss = net.train_step(feat, d["shape"], d["y"], d["active"].view(-1), d["count"], lr_t, weight)
            losses.append(loss.clone())
            step += 1
        torch.cuda.synchronize()
        ep_loss = float(torch.stack(losses).mean().cpu()) if losses else float("nan")
        hist.append(ep_loss)
        log(f"[train] epoch {ep + 1}/{epochs}: mean loss {ep_loss:.3e} ({time.perf_counter() - t:.1f}s)")
    return hist


# ------------------------------------------------------------------ evaluation

def linear_profile(shape, c_in=1.0):
    """C_in (1 - x / (nx - 1)) on the simulated grid: the linear-profile start."""
    import torch

    nx = shape[2]
    prof = c_in * (1.0 - torch.arange(nx, dtype=torch.float32, device="cuda") / max(nx - 1, 1))
    return prof.expand(shape).contiguous()


def compare(net, w: Workload, seeds, shape=None, log=print, unmasked=True):
    """Cold start (C = 0), linear-profile start and learned start on fresh
    structures: steps, wall time (inference included) and converged output."""
    import torch

    shape = shape or w.test_shape
    phases = [structure(s, shape) for s in seeds]
    rows = []
    for seed, ph in zip(seeds, phases):
        s = lbm.Solver(ph, params(w), voxel_m=VOXEL_M, device_prep=True)
        s.autotune(10)  # one launch form for all three starts (the trial steps are undone by each start)
        act, ncat, om = s.host_fields()
        kw = dict(chunk=w.chunk, log=log)
        cold = solve(s, w, None, **kw)
        log(f"[warm/{w.name}] seed {seed}: cold start done ({cold['steps']} steps)")
        lin = solve(s, w, linear_profile(act.shape), **kw)
        log(f"[warm/{w.name}] seed {seed}: linear-profile start done ({lin['steps']} steps)")
        row = {"seed": seed, "cold": cold, "linear": lin}
        if unmasked and w.depth_max >= 0:
            row["warm_unmasked"] = solve(s, w, predict(net, w, act, ncat, om), **kw)
        t0 = time.perf_counter()
        depth = s.pore_depth() if w.depth_max >= 0 else None
        c0 = predict(net, w, act, ncat, om, depth)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        warm = solve(s, w, c0, **kw)
        warm["wall_s"] += t_inf
        warm["inference_s"] = t_inf
        row["warm"] = warm
        row["out_rel_diff"] = abs(warm["out"] / cold["out"] - 1)
        rows.append(row)
        extra = f" (unmasked prediction {row['warm_unmasked']['steps']})" if "warm_unmasked" in row else ""
        log(f"[warm/{w.name}] seed {seed}: steps cold {cold['steps']} linear {lin['steps']} warm {warm['steps']}"
            f"{extra} (inference {t_inf * 1e3:.1f} ms); wall cold {cold['wall_s']:.2f}s warm {warm['wall_s']:.2f}s; "
            f"output diff {row['out_rel_diff']:.1e}, fallback {warm['fallback']}")
        s.close()
    mean = lambda key, f: float(np.mean([r[key][f] for r in rows]))  # noqa: E731
    nxs = shape[2] + (1 if w.mode == lbm.MODE_REACT else 0)
    summ = {
        "workload": f"{w.description}, {shape[0]}x{shape[1]}x{nxs} simulated",
        "seeds": list(seeds),
        "steps_cold": mean("cold", "steps"), "steps_linear": mean("linear", "steps"),
        "steps_warm": mean("warm", "steps"),
        "wall_cold_s": mean("cold", "wall_s"), "wall_linear_s": mean("linear", "wall_s"),
        "wall_warm_s": mean("warm", "wall_s"),
        "inference_ms": float(np.mean([r["warm"]["inference_s"] for r in rows]) * 1e3),
        "fallbacks": int(sum(r["warm"]["fallback"] for r in rows)),
        "max_output_rel_diff": float(max(r["out_rel_diff"] for r in rows)),
    }
    if "warm_unmasked" in rows[0]:
        summ["steps_warm_unmasked"] = mean("warm_unmasked", "steps")
        summ["depth_max"] = w.depth_max
    summ["speedup_steps"] = summ["steps_cold"] / summ["steps_warm"]
    summ["speedup_wall"] = summ["wall_cold_s"] / summ["wall_warm_s"]
    summ["speedup_steps_vs_linear"] = summ["steps_linear"] / summ["steps_warm"]
    summ["speedup_wall_vs_linear"] = summ["wall_linear_s"] / summ["wall_warm_s"]
    return summ


def bench_warm_vs_cold(names=("react", "deff"), shapes=None, seeds=None):
    """Leg of bench.py: every named workload whose trained weights are present, on
    its test grid (192^3) unless ``shapes`` names another for it, on the test
    structures ``seeds`` names for it (default: seed 20000)."""
    out = {}
    for name in names:
        w = WORKLOADS[name]
        if not os.path.exists(w.weights):
            continue
        net = unet.UNet.from_file(w.weights)
        out[name] = compare(net, w, (seeds or {}).get(name, (20000,)), shape=(shapes or {}).get(name),
                            log=lambda *a: print(*a, file=sys.stderr, flush=True), unmasked=False)
        net.release()
    return out or None


def time_network(w: Workload, reps=10, log=print):
    """Times inference on the test grid and one training step on the training grid
    (HIP events on the network's stream); returns ms and achieved TFLOP/s."""
    import torch

    ph = structure(20000, w.test_shape)
    s = lbm.Solver(ph, params(w), voxel_m=VOXEL_M)
    act, ncat, om = s.host_fields()
    net = unet.UNet.from_file(w.weights) if os.path.exists(w.weights) else unet.UNet(seed=0)
    feat, _ = features(w, act, ncat, om)
    shape = act.shape
    net.forward(feat, shape)  # buffers and first touch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        net.forward(feat, shape)
    e1.record()
    e1.synchronize()
    inf_ms = e0.elapsed_time(e1) / reps
    tf = unet.conv_flops(shape)
    # one training step on the training grid, random target (timing only)
    s.close()
    pt = structure(10000, w.train_shape)
    st = lbm.Solver(pt, params(w), voxel_m=VOXEL_M)
    a2, n2, o2 = st.host_fields()
    d = {"active": torch.from_numpy(a2).cuda(), "ncat": torch.from_numpy(_ncat_input(w, n2)).cuda(),
         "omega": torch.from_numpy(o2).cuda(), "shape": a2.shape, "count": int(a2.sum())}
    f2, wt = _features_dev(d)
    tgt = torch.rand(int(np.prod(a2.shape)), dtype=torch.float32, device="cuda")
    trainer = unet.UNet(seed=1)
    trainer.train_step(f2, a2.shape, tgt, d["active"].view(-1), d["count"], 1e-4, wt)
    e0.record()
    for _ in range(reps):
        trainer.train_step(f2, a2.shape, tgt, d["active"].view(-1), d["count"], 1e-4, wt)
    e1.record()
    e1.synchronize()
    tr_ms = e0.elapsed_time(e1) / reps
    tt = 3 * unet.conv_flops(a2.shape)
    res = {"inference_grid": list(shape), "inference_ms": inf_ms, "inference_conv_tflop": tf / 1e12,
           "inference_tflops": tf / inf_ms / 1e9, "train_grid": list(a2.shape), "train_step_ms": tr_ms,
           "train_step_tflops_approx": tt / tr_ms / 1e9, "peak_bf16_tflops": 2500.0}
    log(json.dumps(res))
    return res


def time_layers(shape, reps=20, log=print):
    """Times each distinct convolution of a forward pass on a (nz, ny, nx) grid on
    its own (random BF16 activations and weights, HIP events over reps launches);
    returns {"n^3 cin->cout": microseconds}."""
    import torch

    level = {"e1": 0, "d1": 0, "e2": 1, "d2": 1, "e3": 2, "d3": 2, "b4": 3}
    g = torch.Generator(device="cuda").manual_seed(0)
    out = {}
    for name, cin, cout in unet.layer_specs():
        dims = tuple(s // 2 ** level[name[:2]] for s in shape)
        key = f"{'x'.join(map(str, dims))} {cin}->{cout}"
        if key in out:
            continue
        nv = int(np.prod(dims))
        x = torch.randn(nv * cin, device="cuda", generator=g).to(torch.bfloat16)
        w = (torch.randn(cout * unet.unet_kpad(cin), device="cuda", generator=g) * 0.05).to(torch.bfloat16)
        b = torch.zeros(cout, device="cuda")
        y = torch.empty(nv * cout, device="cuda", dtype=torch.bfloat16)
        for _ in range(3):
            unet.unet_conv3d_fwd(x, cin, 0, w, b, y, cout, 0, None, dims, cin, cout, True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            unet.unet_conv3d_fwd(x, cin, 0, w, b, y, cout, 0, None, dims, cin, cout, True)
        e1.record()
        e1.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        tflops = 2 * 27 * cin * cout * nv / us / 1e6
        out[key] = us
        log(f"[layer] {key}: {us:.1f} us, {tflops:.0f} TFLOP/s, {tflops / 25:.1f}% of the BF16 peak")
    return out


def main(argv):
    """python -m paper_1410_1914_amd.warmstart train <react|deff> [n_samples] [epochs]
    python -m paper_1410_1914_amd.warmstart eval <react|deff> [seed ...]
    python -m paper_1410_1914_amd.warmstart time <react|deff>"""
    import torch

    if len(argv) < 2 or argv[0] not in ("train", "eval", "time") or argv[1] not in WORKLOADS:
        print(main.__doc__)
        return 2
    w = WORKLOADS[argv[1]]
    log = lambda *a: print(*a, flush=True)  # noqa: E731
    if argv[0] == "train":
        n = int(argv[2]) if len(argv) > 2 else 512
        epochs = int(argv[3]) if len(argv) > 3 else 8
        seeds = range(10000, 10000 + n)
        _structures([10000], w.train_shape)  # start the process pool before the GPU is touched
        lbm.require_gpu()
        t = time.perf_counter()
        data = make_dataset(w, seeds, log=log)
        log(f"[data] {len(data)} fields in {time.perf_counter() - t:.1f}s")
        net = unet.UNet(seed=0)
        t = time.perf_counter()
        hist = train(net, w, data, epochs=epochs, log=log)
        log(f"[train] {epochs} epochs in {time.perf_counter() - t:.1f}s")
        out = os.environ.get("WARMSTART_OUT", w.weights)
        os.makedirs(os.path.dirname(out) or ".", exist_ok=True)
        net.save(out)
        del data
        torch.cuda.empty_cache()
        summ = compare(net, w, (20000, 20001), log=log)
        summ["train"] = {"samples": n, "epochs": epochs, "loss_history": hist, "train_shape": w.train_shape}
        log(json.dumps(summ))
        with open(os.path.splitext(out)[0] + ".json", "w") as fh:
            json.dump(summ, fh, indent=1)
    elif argv[0] == "time":
        lbm.require_gpu()
        time_network(w, log=log)
        time_layers(w.test_shape, log=log)
    else:
        seeds = tuple(int(a) for a in argv[2:]) or (20000, 20001)
        lbm.require_gpu()
        net = unet.UNet.from_file(w.weights)
        log(json.dumps(compare(net, w, seeds, log=log)))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
