#!/usr/bin/env python3
"""Benchmark of the D3Q7 reactive-diffusion LBM on one MI355X.

Headline (``value``): MLUPS, millions of fluid-voxel updates per second, of the
steady-state loop on the 256^3 non-precious-metal catalyst layer at 1 nm (carbon
0.45 with micro- and mesopores carved inside, ionomer 0.15, pores 0.40; Knudsen
diffusivity in the pores; every carbon face reactive, k = 1e-4 per face; reactive
problem with the inlet reservoir plane).  One bench step is one check window of
the solver: ``--lbm-steps`` fused stream-collide steps (a captured HIP graph),
the FP64 reductions and the host stop-rule evaluation.  Inputs are resident in
HBM before timing starts.

Also reported on the same JSON line:
  * roofline: algorithmic bytes per stream-collide launch / its mean duration
    (HIP events on the solver stream), against the 8 TB/s HBM peak;
  * other_form: kernel time per step of the launch form the autotuner did not
    keep (one step per launch, or two steps per launch with a 6 x 16 tile);
  * cpu_baseline: the FP64 oracle's step rate on a slab of the same structure;
  * characterise: pore size (13 directions) and face reach of the same structure
    on the device, against the host preprocessing of lbm_create;
  * solves: solves/s to D_eff on the 32^3 two-phase workload (seeds 1..10),
    sequential single solves vs one batched solve, with the error against the
    stored oracle values;
  * warm_start: learned start vs cold start (C = 0) and vs a linear-profile start
    on a fresh 192^3 Pt catalyst layer (seed 20000), when the trained networks
    exist: the effective-diffusivity problem (cold solve ~2.5 M steps) and the
    reactive problem;
  * batch64: 64 uneven reactive structures (edges 48..160): one batched solve of
    all 64, and sequential single solves vs one batched solve on the first 12;
  * skipped: optional legs left out because their estimated time did not fit in
    the wall-clock budget (--budget, default 545 s).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed bench steps (check windows)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--lbm-steps", type=int, default=500, help="LBM steps per bench step")
    ap.add_argument("--n", type=int, default=256, help="cube edge of the headline structure")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-solves", action="store_true", help="skip the 32^3 solves/s legs")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start leg")
    ap.add_argument("--no-charz", action="store_true", help="skip the device structure-characterisation leg")
    ap.add_argument("--no-d3q19", action="store_true", help="skip the D3Q19 (paper's lattice) leg")
    ap.add_argument("--coupled", action="store_true", help="add the coupled O2 / proton-potential leg")
    ap.add_argument("--no-batch64", action="store_true", help="skip the 64-structure batch leg")
    ap.add_argument("--budget", type=float, default=545.0,
                    help="wall-clock seconds for the whole run: an optional leg whose estimated time would not fit "
                         "in what is left is skipped and listed under 'skipped'")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="CPU time budget of the oracle sample")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tiling (no autotuning)")
    ap.add_argument("--tiling", default=None,
                    help="segments/wave,waves/workgroup,xcd: use this one-step launch instead of autotuning "
                         "(profiles pin the form the autotuner keeps at 256^3: 1,1,1)")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--batch-max-edge", type=int, default=None)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy three times (calibrates HBM byte counters) and exit")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the step kernel's source and of the engine that orders its work
    (the order of the segment list decides how much of the traffic the L2 keeps)."""
    h = hashlib.sha256()
    for name in ("kernels.hip", "engine.hip"):
        with open(os.path.join(ROOT, "paper_1410_1914_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(info, knudsen: bool) -> float:
    """Bytes one stream-collide launch must move per the method's data: 7 FP32
    reads + 7 FP32 writes per fluid voxel (56 B), plus its metadata: 1 B of flags
    and, with Knudsen diffusivity, its FP32 1/tau (61 B per fluid update)."""
    return info.n_active * (56.0 + 1.0 + (4.0 if knudsen else 0.0))


def metadata_bytes(n_listed: int) -> float:
    """Bytes of the layout's own bookkeeping per launch, reported apart from the
    algorithmic bytes: per listed segment (a window of up to 64 voxels, one wave)
    its 120-byte record and 4-byte list entry."""
    return n_listed * 124.0


def traffic_from_profiles(kernel_sha: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    e = d.get(workload)
    if not e or e.get("kernel_sha") != kernel_sha:
        return None
    return e.get("bytes_per_launch")


def headline(args, lbm, structgen):
    import torch

    n = args.n
    t = time.time()
    ph = structgen.npmc_cl(args.seed, n=n)
    t_gen = time.time() - t
    p = lbm.lbm_params_default(mode=lbm.MODE_REACT, knudsen=1, k_lat=1e-4,
                               catalyst_phases=(1 << lbm.CARBON) | (1 << lbm.PT),
                               check_every=args.lbm_steps, max_steps=1 << 60)
    t = time.time()
    s = lbm.Solver(ph, p, voxel_m=1e-9)
    t_prep = time.time() - t
    info = s.info
    log(f"[bench] {n}^3 NPMC: generated in {t_gen:.1f}s, preprocessed+bound in {t_prep:.1f}s, "
        f"{info.n_active} fluid voxels, {info.n_segments} segments")
    if args.tiling:
        s.set_tiling(*(int(v) for v in args.tiling.split(",")))
        tune_ms = float("nan")
    else:
        tune_ms = s.autotune(10) if not args.no_tune else float("nan")
    tiling, temporal = s.tiling(), s.temporal()
    spl = 2 if temporal[0] else 1  # LBM steps per stream-collide launch
    log(f"[bench] autotuned tiling (segments/wave, waves/workgroup, xcd) = {tiling}, two-step tile "
        f"(rows, planes) = {temporal if spl == 2 else 'off'}: {tune_ms*1e3:.1f} us/step")
    _, r0 = s.advance(0)
    for _ in range(args.warmup):
        _, r0 = s.advance(args.lbm_steps)
    torch.cuda.synchronize()
    ms0, l0 = r0.kernel_ms, r0.kernel_launches
    t0 = time.perf_counter()
    r = r0
    for _ in range(args.steps):
        _, r = s.advance(args.lbm_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps_timed = r.kernel_launches - l0  # counts LBM steps
    kms = r.kernel_ms - ms0
    updates = info.n_active * steps_timed
    mlups = updates / wall / 1e6
    per_launch_s = kms / 1e3 / steps_timed * spl
    # one launch, of either form, must read and write the lattice once
    alg = algorithmic_bytes(info, knudsen=True)
    meta = metadata_bytes(info.n_listed)
    achieved = alg / per_launch_s / 1e9
    log(f"[bench] {steps_timed} LBM steps in {wall:.3f}s: {mlups:.0f} MLUPS; kernel mean {per_launch_s*1e6:.1f} us "
        f"per launch ({spl} step(s)), {achieved:.0f} GB/s algorithmic")
    other = other_form(s, args, temporal if spl == 2 else (0, 0))
    workload = f"npmc_cl_{n}^3_react_knudsen"
    sha = kernel_source_hash()
    tb = traffic_from_profiles(sha, workload) if spl == 1 else None
    kname = (f"k_step2<{temporal[0]},true,true> (two steps per launch, Knudsen, reactive)" if spl == 2 else
             f"k_step<{tiling[1]},{tiling[0]},true,true,true> (fused pull stream-collide, Knudsen, reactive)")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (round(tb / per_launch_s / 1e9, 1) if tb else None),
            "kernel": kname, "steps_per_launch": spl,
            "tiling": {"segs_per_wave": tiling[0], "waves_per_block": tiling[1], "xcd_remap": tiling[2],
                       "two_step_rows": temporal[0] if spl == 2 else 0,
                       "two_step_planes": temporal[1] if spl == 2 else 0},
            "alg_bytes_per_launch": int(alg), "alg_bytes_per_update": 61,
            "metadata_bytes_per_launch": int(meta),
            "traffic_bytes_per_launch": (int(tb) if tb else None),
            "mean_launch_us": round(per_launch_s * 1e6, 2),
            "kernel_source_sha": sha}
    res = {"mlups": mlups, "ms_per_step": 1e3 * wall / args.steps, "roofline": roof, "workload": workload,
           "other_form": other,
           "n_active": info.n_active, "n_voxels": n ** 3, "prep_s": round(t_prep, 2), "gen_s": round(t_gen, 2),
           "kernel_mlups": info.n_active * spl / per_launch_s / 1e6,
           "rate_per_area_after": r.rate, "steps_taken": r.steps}
    return res, ph


def d3q19_leg(lbm, ph, args):
    """The paper's own lattice (D3Q19, compact storage) on the headline structure and
    problem: kernel time per step from HIP events on the solver's stream, and the
    fraction of HBM peak its algorithmic bytes reach."""
    import torch

    p = lbm.lbm_params_default(mode=lbm.MODE_REACT, knudsen=1, k_lat=1e-4,
                               catalyst_phases=(1 << lbm.CARBON) | (1 << lbm.PT))
    s = lbm.Solver19(ph, p, voxel_m=1e-9)
    n_act, N = s.info.n_active, s.N
    s.step(50)
    steps = 200
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    e1.synchronize()
    per_step_s = e0.elapsed_time(e1) / 1e3 / steps
    # per simulated voxel: 19 FP32 reads and writes, 1/tau and k n (152 + 4 + 4 B)
    alg = n_act * (19 * 4 * 2 + 4 + 4)
    gbs = alg / per_step_s / 1e9
    out = {"kernel": "k_d3q19<true,false> (compact pull stream-collide, reactive)",
           "mean_launch_us": round(per_step_s * 1e6, 2), "mlups": round(n_act / per_step_s / 1e6, 1),
           "alg_bytes_per_launch": int(alg), "achieved_gbs": round(gbs, 1),
           "frac": round(gbs / HBM_PEAK_GBS, 4), "steps_timed": steps}
    log(f"[bench] D3Q19 leg: {out['mean_launch_us']} us per step, {out['mlups']} MLUPS, {out['frac']:.3f} of HBM peak")
    s.close()
    return out


def coupled_leg(lbm, structgen, n=64, gamma=2.25e-5):
    """The coupled O2 / proton-potential solve (Eqs. 15-18b) on a Pt layer at 2 nm
    (64^3 by default) with an ionomer skin on the membrane face: Picard iterations,
    O2 lattice steps, conjugate-gradient iterations of the potential solves, wall
    time, potential drop and consumption."""
    import torch

    ph = structgen.pt_cl(7, n=n)
    skin = ph[:, :, -1]
    skin[skin == lbm.PORE] = lbm.IONOMER
    p = lbm.lbm_params_default(mode=lbm.MODE_REACT, knudsen=1, check_every=500, tol_flux=1e-6,
                               max_steps=4_000_000)
    c = lbm.Coupled19(ph, p, lbm.lbm_coupling_default(gamma=gamma, tol_phi=1e-5), voxel_m=2e-9)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, info = c.run()
    wall = time.perf_counter() - t0
    out = {"edge": n, "gamma_V": gamma, "status": st, "iterations": info.iterations, "o2_steps": info.o2_steps,
           "phi_cg_iterations": info.phi_cg_iterations, "wall_s": round(wall, 2),
           "phi_drop_V": round(0.6 - info.phi_min, 5), "rate_per_area": info.rate,
           "proton_in_per_area": info.proton_in}
    log(f"[bench] coupled leg ({n}^3): {info.iterations} Picard iterations, {info.o2_steps} O2 steps, "
        f"{info.phi_cg_iterations} CG iterations, {wall:.1f}s, potential drop {out['phi_drop_V']} V, status {st}")
    c.close()
    return out


def other_form(s, args, chosen):
    """Kernel time per LBM step of the form the autotuner did not keep (two steps per
    launch with a 6-row, 16-plane tile, or one step per launch), on the same state;
    the chosen form is restored afterwards."""
    alt = (0, 0) if chosen[0] else (6, 16)
    try:
        s.set_temporal(*alt)
    except Exception as e:  # the two-step kernel tiles rows: not on flat windows (rows of 64 k + 1)
        log(f"[bench] other form (two steps per launch): not available on this grid ({e})")
        return {"form": "two steps per launch", "available": False,
                "reason": "rows of 64k+1 voxels use flat segment windows, which the two-step tiles do not cover"}
    _, r0 = s.advance(args.lbm_steps)
    _, r1 = s.advance(4 * args.lbm_steps)
    us = (r1.kernel_ms - r0.kernel_ms) * 1e3 / (r1.kernel_launches - r0.kernel_launches)
    s.set_temporal(*chosen)
    form = f"two steps per launch, tile {alt[0]} rows x {alt[1]} planes" if alt[0] else "one step per launch"
    log(f"[bench] other form ({form}): {us:.1f} us per step")
    return {"form": form, "kernel_us_per_step": round(us, 2)}


def charz_leg(lbm, ph):
    """Structure characterisation of the headline structure on the device (pore
    size by 13-direction chords, reach of the transport phases from both x faces),
    against the host preprocessing of lbm_create on the same structure."""
    import numpy as np
    import torch

    pore = torch.from_numpy((ph == lbm.PORE).astype(np.uint8)).cuda()
    transport = torch.from_numpy(((ph == lbm.PORE) | (ph == lbm.IONOMER)).astype(np.uint8)).cuda()
    lbm.pore_size_device(pore)  # first launch
    lbm.reach_device(transport, 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lbm.pore_size_device(pore)
    t1 = time.perf_counter()
    _, cycles = lbm.reach_device(transport, 3)
    t2 = time.perf_counter()
    p = lbm.lbm_params_default(mode=lbm.MODE_DEFF, knudsen=1)
    t3 = time.perf_counter()
    h = lbm.lbm_create(ph, p, 1e-9)
    t4 = time.perf_counter()
    lbm.lbm_destroy(h)
    log(f"[bench] device characterisation: pore size {1e3 * (t1 - t0):.1f} ms, reach {1e3 * (t2 - t1):.1f} ms "
        f"({cycles} cycles); host lbm_create {t4 - t3:.2f} s")
    return {"workload": "pore size (13 directions) and face reach of the headline structure",
            "gpu_pore_size_ms": round(1e3 * (t1 - t0), 2), "gpu_reach_ms": round(1e3 * (t2 - t1), 2),
            "reach_cycles": cycles, "host_lbm_create_s": round(t4 - t3, 3),
            "host_note": "the whole host preprocessing (chords, reach, tau, segment tables), D_eff problem"}


def cpu_baseline(args, ph, structgen):
    """Oracle (plain FP64 C, OpenMP) step rate on a slab of the same structure."""
    import numpy as np
    from oracle import lbm as O

    slab = np.ascontiguousarray(ph[:, :, :64])
    prob = O.prepare(slab, O.Params(mode=O.MODE_REACT, knudsen=True, voxel_m=1e-9, k_lat=1e-4,
                                    catalyst_phases=(1 << O.CARBON) | (1 << O.PT)))
    f = O.equilibrium(prob, 0.0)
    st = O.Stepper(prob)
    g = np.empty_like(f)
    st.step(f, g)  # first touch
    n = 0
    t0 = time.perf_counter()
    while True:
        st.step(f, g)
        f, g = g, f
        n += 1
        if time.perf_counter() - t0 > args.cpu_seconds:
            break
    dt = time.perf_counter() - t0
    act = int(prob.active.sum())
    v = act * n / dt / 1e6
    return {"value": round(v, 2), "unit": "MLUPS", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{n} FP64 steps of the oracle on the first 64 x-planes of the same structure "
                      f"({slab.shape[2]}x{slab.shape[1]}x{slab.shape[0]}, {act} fluid voxels)"}


def solves_leg(lbm, structgen):
    """Solves/s to D_eff on the 32^3 two-phase workload, single vs batched."""
    import torch

    with open(os.path.join(ROOT, "tests", "golden", "oracle_two_phase_32.json")) as fh:
        gold = {c["seed"]: c["deff"] for c in json.load(fh)["cases"]}
    seeds = sorted(gold)
    phases = [structgen.two_phase(sd, n=32) for sd in seeds]
    mk = lambda: lbm.lbm_params_default(check_every=200)  # noqa: E731
    # sequential single solves (each a fresh solver: preprocessing + bind + solve)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    errs, steps = [], []
    for sd, ph in zip(seeds, phases):
        s = lbm.Solver(ph, mk())
        st, r = s.run_to_steady()
        errs.append(abs(s.deff()[1] / gold[sd] - 1))
        steps.append(r.steps)
        s.close()
    t_single = time.perf_counter() - t0
    # one batched solve of the same structures
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = lbm.Batch(phases, [mk() for _ in phases])
    b.autotune(20)
    st, infos = b.run()
    berrs = [abs(b.deff(i)[1] / gold[sd] - 1) for i, sd in enumerate(seeds)]
    t_batch = time.perf_counter() - t0
    return {"workload": "two-phase QSGS 32^3, seeds 1..10, tau 1, D_eff",
            "single_solves_per_s": round(len(seeds) / t_single, 2),
            "batched_solves_per_s": round(len(seeds) / t_batch, 2),
            "batched_speedup": round(t_single / t_batch, 2),
            "max_rel_err_single": max(errs), "max_rel_err_batched": max(berrs),
            "mean_steps": int(sum(steps) / len(steps)), "tiling": list(b.tiling())}


def _batch_instance(i, max_edge):
    import structgen

    return structgen.batch_instances(2024, count=1, max_edge=max_edge, first=i)[0]


def batch64_structures(args):
    """The uneven 64-structure batch, generated on host processes before any GPU work."""
    from concurrent.futures import ProcessPoolExecutor

    n = args.batch_count
    with ProcessPoolExecutor(max_workers=min(16, n)) as ex:
        return list(ex.map(_batch_instance, range(n), [args.batch_max_edge] * n))


def batch64_leg(lbm, insts, n_seq=12):
    """The uneven 64-structure reactive batch: one batched solve of all 64 (solves/s),
    and, on the first n_seq instances (the generator's random order), sequential
    single solves against one batched solve of the same instances (the speed-up).
    Every solver prepares its structures with the device's share of the
    preprocessing."""
    import torch

    params = [lbm.lbm_params_default(mode=lbm.MODE_REACT, k_lat=d["k"], check_every=200) for d in insts]
    phases = [d["phase"] for d in insts]

    def batched(idx, label):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = lbm.Batch([phases[i] for i in idx], [params[i] for i in idx], device_prep=True)
        b.autotune(20)
        while True:  # in budgets of 100k steps, with a progress line each
            st, infos = b.advance(100_000)
            done = sum(1 for r in infos if r.status != lbm.NOT_CONVERGED)
            log(f"[bench] batch leg ({label}): batched solve at {max(r.steps for r in infos)} steps, {done}/{len(infos)} "
                f"instances finished ({time.perf_counter() - t0:.0f}s)")
            if st != lbm.NOT_CONVERGED:
                break
        rates = [b.reaction_rate(k)[1] for k in range(len(idx))]
        t = time.perf_counter() - t0
        upd = sum(r.steps * b.info(k).n_active for k, r in enumerate(infos))
        tiling = list(b.tiling())
        del b
        return t, rates, st, upd, tiling

    t_all, rates_all, st_all, upd_all, tiling = batched(list(range(len(phases))), "all")
    sub = list(range(min(n_seq, len(phases))))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    single, steps, upd_single = [], [], 0
    for i in sub:
        s = lbm.Solver(phases[i], params[i], device_prep=True)
        st, r = s.run_to_steady()
        single.append(s.reaction_rate()[1])
        steps.append(r.steps)
        upd_single += r.steps * s.info.n_active
        s.close()
        log(f"[bench] batch leg: single solve {len(single)}/{len(sub)} ({phases[i].shape[0]}^3, {r.steps} steps, "
            f"status {st})")
    t_single = time.perf_counter() - t0
    t_sub, rates_sub, _, upd_sub, _ = batched(sub, f"first {len(sub)}")
    vox = sum(int(ph.size) for ph in phases)
    return {"workload": f"{len(phases)} reactive Pt-CL structures, edges in {{48..{max(ph.shape[0] for ph in phases)}}}, "
                        f"porosity 0.3-0.7, k log-uniform 1e-4..1e-1 ({vox / 1e6:.1f} M voxels)",
            "batched_solves_per_s": round(len(phases) / t_all, 3), "batched_wall_s": round(t_all, 1),
            "status": st_all, "tiling": list(tiling), "group_bytes": 192 << 20,
            "fluid_updates_batched": int(upd_all),
            "subset": {"instances": len(sub), "edges": [int(phases[i].shape[0]) for i in sub],
                       "single_solves_per_s": round(len(sub) / t_single, 3),
                       "batched_solves_per_s": round(len(sub) / t_sub, 3),
                       "batched_speedup": round(t_single / t_sub, 2),
                       "max_rate_rel_diff": max(abs(a / c - 1) for a, c in zip(rates_sub, single)),
                       "max_steps": int(max(steps)),
                       "fluid_updates_single": int(upd_single), "fluid_updates_batched": int(upd_sub)}}


def warm_leg(name, seeds=(20000,)):
    """Learned start vs cold start (C = 0) and vs a linear-profile start on fresh
    192^3 Pt catalyst layers: ``deff`` the effective-diffusivity problem (cold solve
    ~2.5 M steps), ``react`` the reactive one."""
    from paper_1410_1914_amd import warmstart

    w = warmstart.bench_warm_vs_cold((name,), None, {name: tuple(seeds)})
    return w[name] if w else None


# Estimated wall time of the optional legs (seconds) at the reference stream-collide
# rate of 126 us per 256^3 step, scaled by the rate measured in the run.
LEG_SECONDS = {"cpu_baseline": 5.0, "characterise": 8.0, "d3q19": 8.0, "solves": 6.0, "warm_deff": 320.0,
               "batch64": 140.0, "warm_react": 40.0}


def main():
    t_start = time.perf_counter()
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch  # noqa: F401

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": src.numel() * 4, "copies": 3}))
        return

    import structgen
    from paper_1410_1914_amd import lbm

    # host work before the GPU is touched
    insts = batch64_structures(args) if not args.no_batch64 else None
    lbm.require_gpu()
    head, ph = headline(args, lbm, structgen)
    out = {
        "metric": "D3Q7 MLUPS (% HBM peak); solves/s to D_eff +-1e-4; warm-start vs cold speedup",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "none",
        "vs_baseline": None,
        "dtype": "f64",
        "storage_dtype": "f32",
        "data": "synthetic (seeded QSGS structure)",
        "config": {"workload": head["workload"], "edge": args.n, "voxel_nm": 1.0, "lbm_steps_per_step": args.lbm_steps,
                   "fluid_voxels": head["n_active"], "k_lat": 1e-4, "parallelism": "single GPU"},
        "roofline": head["roofline"],
        "kernel_mlups": round(head["kernel_mlups"], 1),
        "other_form": head["other_form"],
        "prep_s": head["prep_s"],
    }
    # optional legs, in order, each only when its estimated time fits in the budget
    speed = head["roofline"]["mean_launch_us"] / 126.0 if args.n == 256 else 1.0
    skipped = []

    def fits(leg, extra=0.0):
        est = LEG_SECONDS[leg] * (speed if leg.startswith(("warm", "batch")) else 1.0) + extra
        left = args.budget - (time.perf_counter() - t_start)
        if est <= left:
            return True
        skipped.append({"leg": leg, "estimated_s": round(est), "left_s": round(left)})
        log(f"[bench] skipping {leg}: estimated {est:.0f}s, {left:.0f}s of the budget left")
        return False

    if not args.no_cpu and fits("cpu_baseline", args.cpu_seconds):
        log("[bench] CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(args, ph, structgen)
    if not args.no_charz and fits("characterise"):
        out["characterise"] = charz_leg(lbm, ph)
    if not args.no_d3q19 and fits("d3q19"):
        out["d3q19"] = d3q19_leg(lbm, ph, args)
    if args.coupled:
        out["coupled"] = coupled_leg(lbm, structgen)
    del ph
    if not args.no_solves and fits("solves"):
        log("[bench] 32^3 solves/s legs ...")
        out["solves"] = solves_leg(lbm, structgen)
    warm = {}
    if not args.no_warm and fits("warm_deff"):
        log("[bench] warm start, effective diffusivity at 192^3 ...")
        r = warm_leg("deff")
        if r is not None:
            warm["deff"] = r
    if insts is not None and fits("batch64"):
        log("[bench] 64-structure batch leg ...")
        out["batch64"] = batch64_leg(lbm, insts)
    if not args.no_warm and fits("warm_react"):
        log("[bench] warm start, reactive at 192^3 ...")
        r = warm_leg("react")
        if r is not None:
            warm["react"] = r
    if warm:
        out["warm_start"] = warm
    out["skipped"] = skipped
    out["wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
