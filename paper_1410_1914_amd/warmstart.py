"""Learned warm start for the reactive catalyst-layer problem.

Workload: four-phase Pt catalyst layers (carbon + Pt 0.35, ionomer 0.20, Pt on 10%
of the carbon-pore faces, pores 0.45) at 2 nm voxels, reactive problem of Chen et
al. (arXiv 1410.1914, Section 3.5.2: inlet reservoir plane, Dirichlet inlet,
zero-gradient outlet, periodic y and z) with Knudsen pore diffusivity, ionomer
D = 1e-3 D0 and a first-order sink k = 1e-2 (lattice units) per Pt face.
Structures are 95 voxels long in x so that the simulated grid (with the reservoir
plane) is a multiple of 8 for the network's three poolings.

Pipeline:
  1. training fields: the batched HIP solver's steady states on seeded structures;
  2. training: the U-Net of ``unet.py`` on the GPU with the project's own kernels.
     The target is ln(C + 1e-3), so the error is relative to C, and the masked
     MSE weighs a voxel by sqrt(D_ref / D) (capped), so slowly relaxing ionomer
     counts more;
  3. use: features of a new structure -> predicted concentration, kept where the
     pore depth (lbm_get_pore_depth) is at most DEPTH_MAX and C = 0 deeper in ->
     equilibrium populations (``lbm_set_initial_concentration``) -> the solver
     refines to its own stop rule.  If the windowed residual rises between the
     first two checks the solve falls back to the cold start, so the network can
     never change the answer, only the number of steps.

Why the depth mask: the steps a solve needs are set by the voxels that relax
slowest, which are ionomer films and blobs (D = 1e-3 D0, tau close to 1/2).  Their
concentration is small, so the cold start's error there is already small, and a
prediction only helps where its error is smaller still; deep inside the ionomer
(beyond DEPTH_MAX voxels from the connected pores) the trained network's is not.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import lbm, unet

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "weights", "unet_react_ptcl.npz")
K_LAT = 1e-2
VOXEL_M = 2e-9
TRAIN_SHAPE = (96, 96, 95)    # structure (nz, ny, nx); simulated grid (96, 96, 96)
TEST_SHAPE = (192, 192, 191)  # simulated grid (192, 192, 192)
WEIGHT_POWER = 0.5
WEIGHT_CAP = 32.0
TARGET_EPS = 1e-3   # the network predicts ln(C + TARGET_EPS)
DEPTH_MAX = 4       # the prediction is used up to this pore depth; C = 0 (cold) deeper in (chosen on
                    # validation structures, seeds 30000 and 30001)
C_MAX = 1.5         # upper clip of a predicted start (the discrete field may exceed C_in slightly)


def params(**kw):
    p = lbm.lbm_params_default(mode=lbm.MODE_REACT, knudsen=1, k_lat=K_LAT, check_every=200)
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

def features(active, ncat, omega, tau_ref=1.0):
    """BF16 (V, 16) network input from the solver's dense host fields (simulated grid)."""
    import torch

    shape = active.shape
    feat = torch.empty((int(np.prod(shape)), unet.IN_CH), dtype=torch.bfloat16, device="cuda")
    a = torch.from_numpy(np.ascontiguousarray(active)).cuda()
    n = torch.from_numpy(np.ascontiguousarray(ncat)).cuda()
    o = torch.from_numpy(np.ascontiguousarray(omega)).cuda()
    unet.unet_features(a, n, o, tau_ref, feat, shape)
    return feat, a


def predict(net, active, ncat, omega, depth=None, depth_max=DEPTH_MAX):
    """Start field for the solver (FP32, dense simulated grid, on the GPU): the
    predicted steady concentration, and, when the pore-depth map is given, the cold
    value 0 in voxels deeper than depth_max (ionomer interiors relax slowly and hold
    little oxygen; a wrong guess there costs more steps than C = 0)."""
    import torch

    feat, _ = features(active, ncat, omega)
    out = net.forward(feat, active.shape)
    c = torch.empty(out.numel(), dtype=torch.float32, device=out.device)
    if depth is not None:
        if not net.target_eps > 0:
            raise ValueError("the depth-masked start needs a log-space network")
        d = torch.from_numpy(np.ascontiguousarray(depth)).to(out.device)
        unet.unet_start_field(out, d, depth_max, net.target_eps, C_MAX, c, out.numel())
    elif net.target_eps > 0:
        unet.unet_log_map(out, c, out.numel(), net.target_eps, True, C_MAX)
    else:
        # linear-output network: the same clip through the map's inverse of ln(C + 1)
        unet.unet_log_map(out, c, out.numel(), 1.0, False)
        unet.unet_log_map(c, c, out.numel(), 1.0, True, C_MAX)
    return c.view(active.shape)


# ------------------------------------------------------------------ solves

def solve(solver, c0=None, fallback=True):
    """Steady solve from c0 (None: cold start C = 0).  Returns a dict with the steps,
    wall time, status, reaction rate and whether the cold fallback was taken."""
    import torch

    t0 = time.perf_counter()
    solver.set_initial_concentration(c0)
    K = solver.params.check_every
    used_fallback = False
    if c0 is not None and fallback and not bool(torch.isfinite(c0).all()):
        used_fallback = True
        solver.set_initial_concentration(None)
    elif c0 is not None and fallback:
        _, i1 = solver.advance(K)
        st, i2 = solver.advance(K)
        if st != lbm.OK and i2.residual > i1.residual:
            used_fallback = True
            solver.set_initial_concentration(None)
    st, info = solver.run_to_steady()
    torch.cuda.synchronize()
    _, rate, jin = solver.reaction_rate()
    return {"status": st, "steps": int(info.steps), "wall_s": time.perf_counter() - t0, "rate": rate,
            "fallback": used_fallback}


# ------------------------------------------------------------------ training data

def make_dataset(seeds, shape=TRAIN_SHAPE, batch=32, tol_flux=1e-4, tol_change=1e-8, log=print):
    """Steady fields of the batched solver.  Returns a list of per-sample dicts of
    GPU tensors (active u8, ncat u8, omega f32, target f32) and host shape."""
    import torch

    phases = _structures(list(seeds), shape)
    data = []
    for s0 in range(0, len(phases), batch):
        chunk = phases[s0:s0 + batch]
        t = time.perf_counter()
        b = lbm.Batch(chunk, [params(tol_flux=tol_flux, tol_change=tol_change) for _ in chunk], voxel_m=VOXEL_M)
        st, infos = b.run()
        for i in range(len(chunk)):
            act, ncat, om = b.host_fields(i)
            data.append({"active": torch.from_numpy(act).cuda(), "ncat": torch.from_numpy(ncat).cuda(),
                         "omega": torch.from_numpy(om).cuda(), "target": b.concentration(i).clone(),
                         "shape": act.shape, "count": int(act.sum()), "steps": int(infos[i].steps)})
        del b
        torch.cuda.synchronize()
        log(f"[data] {s0 + len(chunk)}/{len(phases)} fields, batch of {len(chunk)} in {time.perf_counter() - t:.1f}s "
            f"(mean steps {np.mean([x['steps'] for x in data[-len(chunk):]]):.0f}, status {st})")
    return data


def _log_targets(data, eps):
    """ln(C + eps) of every sample's target (kept with the sample)."""
    import torch

    key = ("y", eps)
    for d in data:
        if d.get("y_key") != key:
            t = d["target"].view(-1)
            d["y"] = torch.empty_like(t)
            unet.unet_log_map(t, d["y"], t.numel(), eps, False)
            d["y_key"] = key


def train(net, data, epochs=4, lr=1e-3, log=print, seed=0, weight_power=WEIGHT_POWER, weight_cap=WEIGHT_CAP,
          target_eps=TARGET_EPS):
    """Adam on the weighted masked MSE, cosine learning-rate decay; returns the loss
    history.  The weight of a voxel is (D_ref / D)^weight_power capped at weight_cap: an error
    left in a low-diffusivity voxel (ionomer) relaxes slowly, so it costs the solver
    far more steps than the same error in a pore."""
    import torch

    rng = np.random.default_rng(seed)
    hist = []
    total = epochs * len(data)
    if target_eps > 0:
        _log_targets(data, target_eps)
        if net.t == 0:  # start the output bias at the mean log target
            m = float(np.mean([float(d["y"][d["active"].view(-1) > 0].mean()) for d in data[:32]]))
            net.B["head"].fill_(m)
    net.target_eps = target_eps
    step = 0
    for ep in range(epochs):
        order = rng.permutation(len(data))
        t = time.perf_counter()
        losses = []
        for idx in order:
            d = data[idx]
            feat, weight = _features_dev(d, weight_power, weight_cap)
            lr_t = lr * 0.5 * (1 + np.cos(np.pi * step / total))
            tgt = d["y"] if target_eps > 0 else d["target"].view(-1)
            loss = net.train_step(feat, d["shape"], tgt, d["active"].view(-1), d["count"], lr_t, weight)
            losses.append(loss.clone())
            step += 1
        torch.cuda.synchronize()
        ep_loss = float(torch.stack(losses).mean().cpu()) if losses else float("nan")
        hist.append(ep_loss)
        log(f"[train] epoch {ep + 1}/{epochs}: mean loss {ep_loss:.3e} ({time.perf_counter() - t:.1f}s)")
    return hist


def _features_dev(d, weight_power=WEIGHT_POWER, weight_cap=WEIGHT_CAP):
    """Features and per-voxel loss weights of one training sample (on the GPU)."""
    import torch

    shape = d["shape"]
    feat = torch.empty((int(np.prod(shape)), unet.IN_CH), dtype=torch.bfloat16, device="cuda")
    weight = torch.empty(int(np.prod(shape)), dtype=torch.float32, device="cuda")
    unet.unet_features(d["active"], d["ncat"], d["omega"], 1.0, feat, shape, weight, weight_power, weight_cap)
    return feat, weight


# ------------------------------------------------------------------ evaluation

def linear_profile(shape, c_in=1.0):
    """C_in (1 - x / (nx - 1)) on the simulated grid: the linear-profile start."""
    import torch

    nx = shape[2]
    prof = c_in * (1.0 - torch.arange(nx, dtype=torch.float32, device="cuda") / max(nx - 1, 1))
    return prof.expand(shape).contiguous()


def compare(net, seeds, shape=TEST_SHAPE, log=print):
    """Cold start (C = 0), linear-profile start and learned start on fresh
    structures: steps, wall time (inference included) and converged rate."""
    import torch

    phases = [structure(s, shape) for s in seeds]
    rows = []
    for seed, ph in zip(seeds, phases):
        s = lbm.Solver(ph, params(), voxel_m=VOXEL_M)
        act, ncat, om = s.host_fields()
        cold = solve(s, None)
        lin = solve(s, linear_profile(act.shape))
        unmasked = solve(s, predict(net, act, ncat, om))
        t0 = time.perf_counter()
        depth = s.pore_depth()
        c0 = predict(net, act, ncat, om, depth)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        warm = solve(s, c0)
        warm["wall_s"] += t_inf
        warm["inference_s"] = t_inf
        row = {"seed": seed, "cold": cold, "linear": lin, "warm": warm, "warm_unmasked": unmasked,
               "rate_rel_diff": abs(warm["rate"] / cold["rate"] - 1)}
        rows.append(row)
        log(f"[warm] seed {seed}: steps cold {cold['steps']} linear {lin['steps']} warm {warm['steps']} "
            f"(unmasked prediction {unmasked['steps']}) "
            f"(inference {t_inf * 1e3:.1f} ms); wall cold {cold['wall_s']:.2f}s warm {warm['wall_s']:.2f}s; "
            f"rate diff {row['rate_rel_diff']:.1e}, fallback {warm['fallback']}")
        s.close()
    summ = {
        "workload": f"Pt CL reactive, k={K_LAT}, Knudsen, {shape[0]}x{shape[1]}x{shape[2] + 1} simulated",
        "seeds": list(seeds),
        "steps_cold": float(np.mean([r["cold"]["steps"] for r in rows])),
        "steps_linear": float(np.mean([r["linear"]["steps"] for r in rows])),
        "steps_warm": float(np.mean([r["warm"]["steps"] for r in rows])),
        "steps_warm_unmasked": float(np.mean([r["warm_unmasked"]["steps"] for r in rows])),
        "wall_cold_s": float(np.mean([r["cold"]["wall_s"] for r in rows])),
        "wall_linear_s": float(np.mean([r["linear"]["wall_s"] for r in rows])),
        "wall_warm_s": float(np.mean([r["warm"]["wall_s"] for r in rows])),
        "inference_ms": float(np.mean([r["warm"]["inference_s"] for r in rows]) * 1e3),
        "depth_max": DEPTH_MAX,
        "fallbacks": int(sum(r["warm"]["fallback"] for r in rows)),
        "max_rate_rel_diff": float(max(r["rate_rel_diff"] for r in rows)),
    }
    summ["speedup_steps"] = summ["steps_cold"] / summ["steps_warm"]
    summ["speedup_wall"] = summ["wall_cold_s"] / summ["wall_warm_s"]
    summ["speedup_steps_vs_linear"] = summ["steps_linear"] / summ["steps_warm"]
    summ["speedup_wall_vs_linear"] = summ["wall_linear_s"] / summ["wall_warm_s"]
    return summ


def bench_warm_vs_cold(seeds=(20000, 20001), shape=TEST_SHAPE):
    """Leg of bench.py: needs the trained weights."""
    if not os.path.exists(WEIGHTS):
        return None
    net = unet.UNet.from_file(WEIGHTS)
    return compare(net, seeds, shape, log=lambda *a: print(*a, file=sys.stderr, flush=True))


def main(argv):
    """python -m paper_1410_1914_amd.warmstart train [n_samples] [epochs]"""
    import torch

    if len(argv) < 1 or argv[0] not in ("train", "eval"):
        print(main.__doc__)
        return 2
    log = lambda *a: print(*a, flush=True)  # noqa: E731
    if argv[0] == "train":
        n = int(argv[1]) if len(argv) > 1 else 512
        epochs = int(argv[2]) if len(argv) > 2 else 4
        seeds = range(10000, 10000 + n)
        phases_first = _structures([10000], TRAIN_SHAPE)  # warm the process pool before CUDA
        del phases_first
        lbm.require_gpu()
        t = time.perf_counter()
        data = make_dataset(seeds, log=log)
        log(f"[data] {len(data)} fields in {time.perf_counter() - t:.1f}s")
        net = unet.UNet(seed=0)
        t = time.perf_counter()
        hist = train(net, data, epochs=epochs, log=log)
        log(f"[train] {epochs} epochs in {time.perf_counter() - t:.1f}s")
        os.makedirs(os.path.dirname(WEIGHTS), exist_ok=True)
        out = os.environ.get("WARMSTART_OUT", WEIGHTS)
        net.save(out)
        del data
        torch.cuda.empty_cache()
        summ = compare(net, (20000, 20001), log=log)
        summ["train"] = {"samples": n, "epochs": epochs, "loss_history": hist, "train_shape": TRAIN_SHAPE}
        log(json.dumps(summ))
        with open(os.path.splitext(out)[0] + ".json", "w") as fh:
            json.dump(summ, fh, indent=1)
    else:
        lbm.require_gpu()
        log(json.dumps(bench_warm_vs_cold()))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
