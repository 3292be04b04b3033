"""Benchmark of the m-mode Teukolsky Lax-Wendroff engine on one MI355X.

A bench step is one complete forced EMRI evolution of the 6400 x 128 Kerr
grid (a = 0.9, s = -2, m = 2, circular orbit at r0 = 10M): 40000 iterations of
the two-step Lax-Wendroff stencil with its compact source passes and the
waveform extracted at r* = 500M after every iteration, from zero data in HBM.
value = grid-point updates per second (GPts/s) over the timed steps.

Also reported on the same JSON line:
  roofline      dominant kernel (the stencil, in the launch configuration
                the autotuner picks before timing): algorithmic HBM bytes per
                launch (64 B per point: read u^n and write u^{n+k}, Phi and
                Pi) over its average launch duration, from HIP events around
                every stencil launch of one extra evolution;
  hbm_grid      the same physics on 25600 x 512 (both state levels 3.3x
                the 256 MB last-level cache, so the traffic is HBM traffic):
                GPts/s and a roofline block like the one above, with the
                HBM bytes from counters when the committed counter summary
                matches the current sources; beside it the achieved
                bandwidth of a plain device copy (a STREAM-copy ceiling);
  batched       64 independent instances of uneven size (seeded m, a, grid
                level, pulse centre), 10000 iterations each, in both batch
                modes (one persistent launch per evolution captured in a HIP
                graph; one launch per iteration over all instances), against
                the plain stepper running the same instances one after another;
  all_m         every m (1..4) of one circular orbit on the 6400 x 128 grid,
                each with its source, 4000 iterations as one batch, against
                the same instances one after another;
  small_batch   64 instances of the 801 x 33 grid, 2000 iterations, both
                batch modes against the plain stepper (short launches);
  adjoint_at_scale
                16 instances on 12800 x 256 with eccentric orbits (seeded a,
                m, p, e), forward + checkpointed adjoint one instance after
                another, 50000 iterations each (snapshots every
                ceil(sqrt N) iterations, every segment recomputed);
  cpu_baseline  the FP64 oracle on the host for a bounded number of
                iterations of the same workload.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_POINT = 64.0


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"lw_step_kernel_{workload}_traffic.json")


def measured_traffic(workload, seg_rows, k_steps):
    """Bytes leaving L2 per stencil launch from the committed counter summary
    of this workload, or None if the stencil sources or the launch
    configuration changed since."""
    import hashlib
    try:
        rec = json.load(open(traffic_file(workload)))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for src in rec["kernel_sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != rec["sources_sha256"] or rec.get("tuning") != [seg_rows, k_steps]:
        return None
    return rec["traffic_bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-hbm", action="store_true",
                    help="skip the HBM-resident 25600 x 512 grid and the device-copy ceiling")
    ap.add_argument("--cpu-iters", type=int, default=16)
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint/forward ratio")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-instance workloads")
    ap.add_argument("--all-m-iterations", type=int, default=None,
                    help="iterations of the all-m batch (default: the workload's 4000)")
    ap.add_argument("--batched-iterations", type=int, default=10000)
    ap.add_argument("--no-scale", action="store_true",
                    help="skip the forward + checkpointed adjoint of the 16 instances on 12800 x 256")
    ap.add_argument("--scale-instances", type=int, default=None,
                    help="run only the first N instances of the 16 x 12800 x 256 workload (profiling)")
    ap.add_argument("--scale-iterations", type=int, default=None,
                    help="iterations per instance of that workload (default its full 50000)")
    ap.add_argument("--workload", default="kerr_emri_6400x128",
                    choices=["kerr_emri_6400x128", "kerr_emri_25600x512"],
                    help="main workload (the second one only for profiling passes)")
    ap.add_argument("--iterations", type=int, default=None,
                    help="override the iterations per evolution (profiling passes only)")
    ap.add_argument("--tuning", default=None,
                    help="SEG,K: fixed launch configuration instead of the autotuner (profiling passes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (counter calibration)")
    return ap.parse_args()


def copy_calibration():
    """A plain elementwise kernel of known traffic: read 256 MiB, write 256 MiB."""
    import torch
    n = 16 * 1024 * 1024                      # complex128 elements = 256 MiB
    a = torch.ones(n, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"kernel": "elementwise mul (torch)", "dispatches": 3,
                                           "read_bytes_per_dispatch": n * 16,
                                           "write_bytes_per_dispatch": n * 16}}), flush=True)


def stream_copy():
    """Achieved bandwidth of a plain device copy (read 1 GiB, write 1 GiB,
    far beyond the last-level cache): the practical ceiling of a kernel that
    streams its data once, timed with events over 20 launches."""
    import torch
    n = 64 * 1024 * 1024                      # complex128 elements = 1 GiB
    a = torch.ones(n, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / 20
    del a, b
    return {"kernel": "device copy (torch copy_)", "bytes_per_launch": 2 * n * 16,
            "avg_launch_us": round(s * 1e6, 1), "GBs": round(2 * n * 16 / s / 1e9, 1),
            "frac_of_peak": round(2 * n * 16 / s / 1e9 / HBM_PEAK_GBS, 4)}


def stencil_roofline(eng, workload, npts, run):
    """Roofline block of the stencil: algorithmic bytes per launch (64 per
    point) over the average launch duration from the launches' own events
    during one more evolution (run()), plus the counter traffic if the
    committed summary matches."""
    tune = eng.tuning
    eng.set_kernel_timing(True)
    run()
    kms, kn = eng.kernel_timing()
    eng.set_kernel_timing(False)
    avg_s = kms / kn * 1e-3
    achieved = npts * BYTES_PER_POINT / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(workload, tune["seg_rows"], tune["k_steps"]),
            "kernel": "lw_step_kernel" if tune["k_steps"] == 1 else "lw_block_kernel",
            "avg_launch_us": round(avg_s * 1e6, 3),
            "bytes_per_launch": int(npts * BYTES_PER_POINT), "launches_timed": kn,
            "tuning": {"seg_rows": tune["seg_rows"], "k_steps": tune["k_steps"]}}


def make_engine(cfg, nsteps):
    from paper_1001_3631_amd.engine import Engine
    g = cfg["grid"]
    eng = Engine(**g)
    src = cfg["source"]
    orbit = eng.orbit_circular(src["r0"], 2 * nsteps + 1, M=g["M"], a=g["a"])
    eng.set_source(orbit, src["amplitude"], src["sigma_r_cells"], src["sigma_th_cells"],
                   src["cutoff_sigmas"])
    return eng


def run_evolution(eng, zero_phi, zero_pi, nsteps, wave):
    eng.set_state(zero_phi, zero_pi)
    eng.step(nsteps, out=wave)


def adjoint_ratio(args):
    """Adjoint/forward time ratio on the 3200 x 64 adjoint workload (20000
    iterations): forward with extraction; reverse sweep driven by the
    waveform residual (no states needed); and the checkpointed pair
    (snapshots every ceil(sqrt(N)) iterations, every segment recomputed)."""
    import torch
    from paper_1001_3631_amd import workloads as W
    cfg = W.ADJOINT
    g = cfg["grid"]
    n = cfg["steps"]
    eng = make_engine(cfg, n)
    eng.autotune(None)                      # the forward at its best launch configuration
    y = torch.zeros((n, g["nth"]), dtype=torch.complex128, device="cuda")

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, out

    def fwd():
        eng.init_pulse(**cfg["pulse"])
        return eng.step(n)

    fwd()                                                   # warm-up
    tf, w = timed(fwd)
    gw = (2.0 * (w - y)).contiguous()

    def adj():
        eng.adjoint_begin(n, gw=gw)
        eng.adjoint_step(n)
        return eng.adjoint_get()

    adj()
    ta, _ = timed(adj)

    def ckpt():
        eng.init_pulse(**cfg["pulse"])
        eng.forward_checkpointed(n, interval=0, force_recompute=True)
        return eng.backward_checkpointed(gw, 0.0)

    tc, _ = timed(ckpt)
    tune = eng.tuning
    eng.close()
    return {"workload": cfg["name"], "iterations": n, "tuning": tune,
            "forward_s": round(tf, 4), "adjoint_s": round(ta, 4),
            "ratio": round(ta / tf, 3), "forward_plus_backward_with_recompute_s": round(tc, 4),
            "ratio_with_recompute": round((tc - tf) / tf, 3)}


HBM_BYTES = 288e9          # MI355X HBM3E per GPU


def adjoint_at_scale(args):
    """Forward + checkpointed adjoint of the 16 eccentric-orbit instances on
    12800 x 256 (seeded a, m, p, e, anomaly), one instance after another:
    each alone fills the GPU (51200 waves per launch) and its state fits the
    last-level cache.  Snapshots: the binomial schedule with the slots that
    fit each instance's share of the HBM (288 GB / 16), i.e. the memory the
    whole batch's snapshots could take if it were held at once; the backward
    runs the schedule's recomputation (forced: this loss needs no forward
    state) while sweeping in reverse.  Loss sum |w - y|^2 against the
    waveform of source amplitude 0.9 (zero initial data, so y = 0.9 w and
    dL/dA = 0.2 |w|^2 exactly: checked).  Also times the forward of all 16
    instances as one batch (one launch per iteration over every instance)
    against the same iterations one instance after another."""
    import torch
    from paper_1001_3631_amd import workloads as W
    from paper_1001_3631_amd.engine import Batch, Engine, checkpoint_schedule
    cfg = W.ADJOINT_AT_SCALE
    n = args.scale_iterations or cfg["steps"]
    src = cfg["source"]
    insts = W.adjoint_at_scale_instances(cfg["seed"], cfg["instances"])
    budget = HBM_BYTES / len(insts)
    if args.scale_instances:
        insts = insts[:args.scale_instances]
    tf = tb = 0.0
    pts = 0
    worst_dA = 0.0
    snap_bytes = peak_used = 0
    w2_max = 0.0
    tuning = None
    snapshots = None
    for k, inst in enumerate(insts):
        g, o = inst["grid"], inst["orbit"]
        free0, _ = torch.cuda.mem_get_info()
        eng = Engine(**g)
        orbit = eng.orbit_eccentric(o["p"], o["e"], 2 * n + 1, M=g["M"], a=g["a"], chi0=o["chi0"])
        eng.set_source(orbit, src["amplitude"], src["sigma_r_cells"], src["sigma_th_cells"],
                       src["cutoff_sigmas"])
        if tuning is None:
            eng.autotune(None)              # same shape for every instance: tune once (untimed)
            tuning = eng.tuning
            snapshots = eng.snapshots_for_budget(n, budget)
        else:
            eng.set_tuning(tuning["seg_rows"], tuning["k_steps"])
        z = torch.zeros((g["nth"], g["nr"]), dtype=torch.complex128, device="cuda")
        eng.set_state(z, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w, _ = eng.forward_checkpointed(n, force_recompute=True, snapshots=snapshots)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        free1, _ = torch.cuda.mem_get_info()
        gw = ((2.0 * (1.0 - cfg["target_amplitude"])) * w).contiguous()
        gp, gq, dA = eng.backward_checkpointed(gw, 0.0)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        eng.check_finite()
        w2 = float(torch.sum(torch.abs(w) ** 2))
        w2_max = max(w2_max, w2)
        ref = 2.0 * (1.0 - cfg["target_amplitude"]) * w2
        worst_dA = max(worst_dA, abs(dA - ref) / max(abs(ref), 1e-300))
        tf += t1 - t0
        tb += t2 - t1
        pts += g["nr"] * g["nth"] * n
        snap_bytes = max(snap_bytes, eng.checkpoint_bytes(n, snapshots=snapshots))
        peak_used = max(peak_used, free0 - free1)
        print(f"[bench] adjoint_at_scale instance {k}: a={g['a']:.3f} m={g['m']} p={o['p']:.2f} "
              f"e={o['e']:.3f} fwd {t1 - t0:.3f} s bwd {t2 - t1:.3f} s dA {dA:.6e}", file=sys.stderr,
              flush=True)
        del gp, gq, gw, w, z
        eng.close()
    _, _, (reps, recomputed, _) = checkpoint_schedule(n, snapshots)
    out = {"workload": cfg["name"], "instances": len(insts), "iterations": n,
           "schedule": "instances one after another (each fills the GPU); binomial checkpoints, "
                       "every recomputation of the schedule run in the backward",
           "snapshots_per_instance": snapshots, "repetitions": reps,
           "backward_recomputed_iterations": recomputed,
           "snapshot_budget_bytes_per_instance": int(budget),
           "tuning": tuning, "forward_s": round(tf, 3), "backward_with_recompute_s": round(tb, 3),
           "ratio_backward_over_forward": round(tb / tf, 3),
           "forward_gpts": round(pts / tf / 1e9, 3),
           "snapshot_bytes_per_instance": int(snap_bytes),
           "snapshot_bytes_all_instances": int(snap_bytes) * len(insts),
           "device_bytes_used_per_instance": int(peak_used),
           # the check is empty (null) when no signal reached the extraction radius
           "dL_dA_worst_rel_vs_closed_form": float(f"{worst_dA:.3e}") if w2_max > 0 else None,
           "waveform_norm2_max": float(f"{w2_max:.6e}")}

    # the same 16 forwards as one batch (its fastest mode and segment length)
    nb = min(n, 1000)
    b = Batch([inst["grid"] for inst in insts])
    for e, inst in zip(b.instances, insts):
        o, g = inst["orbit"], inst["grid"]
        orbit = e.orbit_eccentric(o["p"], o["e"], 2 * nb + 1, M=g["M"], a=g["a"], chi0=o["chi0"])
        e.set_source(orbit, src["amplitude"], src["sigma_r_cells"], src["sigma_th_cells"], src["cutoff_sigmas"])
    b.autotune(None)
    zs = [torch.zeros(e.shape, dtype=torch.complex128, device="cuda") for e in b.instances]
    for e, z0 in zip(b.instances, zs):
        e.set_state(z0, z0)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(nb, waveform=False)
    b.sync()
    t_batch = time.perf_counter() - t0
    mode = "persistent" if b.mode == Batch.PERSISTENT else "per_iteration"
    seg = b.seg_rows
    b.close()
    out["batched_forward_probe"] = {
        "iterations": nb, "mode": mode, "seg_rows": seg, "batch_s": round(t_batch, 3),
        "batch_gpts": round(pts / n * nb / t_batch / 1e9, 3),
        "one_after_another_gpts": out["forward_gpts"],
        "batch_state_bytes": int(sum(2 * 2 * 16 * i["grid"]["nr"] * i["grid"]["nth"] for i in insts))}
    return out


def batched(args):
    """The batched workload: both batch modes (persistent graph launch, one
    launch per iteration) at their best segment lengths vs the plain stepper."""
    import torch
    from paper_1001_3631_amd import workloads as W
    from paper_1001_3631_amd.engine import Batch, Engine
    inst = W.batched_instances()
    n = args.batched_iterations
    grids = [it["grid"] for it in inst]
    pts = sum(g["nr"] * g["nth"] for g in grids)
    b = Batch(grids)
    tune = b.autotune(None)                         # [(seg_rows, mode, us)], fastest first
    best_seg = {}
    for seg, mode, _ in tune:
        best_seg.setdefault(mode, seg)
    waves = [torch.empty((n, g["nth"]), dtype=torch.complex128, device="cuda") for g in grids]

    def evolve():
        for e, it in zip(b.instances, inst):
            e.init_pulse(**it["pulse"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(n, out=waves)
        b.sync()
        return time.perf_counter() - t0

    names = {Batch.PERSISTENT: "persistent", Batch.PER_ITERATION: "per_iteration"}
    times = {}
    for mode in (Batch.PERSISTENT, Batch.PER_ITERATION):
        b.set_tuning(best_seg[mode])
        b.set_mode(mode)
        if mode == Batch.PERSISTENT:
            evolve()                                # captures the graph for n iterations
        times[mode] = evolve()
        for e in b.instances:
            e.check_finite()
    b.close()
    del waves
    mode_b = min(times, key=times.get)
    tb = times[mode_b]

    # plain stepper, one instance after another, same iterations and extraction
    tp = 0.0
    for it in inst:
        eng = Engine(**it["grid"])
        eng.autotune(None)
        w = torch.empty((n, it["grid"]["nth"]), dtype=torch.complex128, device="cuda")
        eng.init_pulse(**it["pulse"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        eng.step(n, out=w)
        torch.cuda.synchronize()
        tp += time.perf_counter() - t1
        eng.close()
    return {"workload": "batched_64_instances_seed3", "instances": len(grids), "points": pts,
            "iterations": n, "mode": names[mode_b], "seg_rows": best_seg[mode_b],
            "batched_s": round(tb, 3), "batched_gpts": round(pts * n / tb / 1e9, 3),
            "by_mode": {names[m]: {"seg_rows": best_seg[m], "s": round(times[m], 3),
                                   "gpts": round(pts * n / times[m] / 1e9, 3)} for m in times},
            "plain_sequential_s": round(tp, 3), "plain_gpts": round(pts * n / tp / 1e9, 3),
            "batched_over_plain": round(tp / tb, 3)}


def small_batch(args):
    """64 instances of the 801 x 33 Schwarzschild pulse grid (26 433 points
    each), 2000 iterations, in both batch modes: a workload where one launch
    per iteration is short, against the plain stepper one instance after
    another."""
    import torch
    from paper_1001_3631_amd import workloads as W
    from paper_1001_3631_amd.engine import Batch, Engine
    cfg = W.SCHWARZSCHILD_PULSE
    grids = [cfg["grid"]] * 64
    n = cfg["steps"]
    pts = sum(g["nr"] * g["nth"] for g in grids)
    b = Batch(grids)
    tune = b.autotune(None)
    best_seg = {}
    for seg, mode, _ in tune:
        best_seg.setdefault(mode, seg)

    def evolve():
        for e in b.instances:
            e.init_pulse(**cfg["pulse"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(n, waveform=False)
        b.sync()
        return time.perf_counter() - t0

    names = {Batch.PERSISTENT: "persistent", Batch.PER_ITERATION: "per_iteration"}
    times = {}
    for mode in (Batch.PERSISTENT, Batch.PER_ITERATION):
        b.set_tuning(best_seg[mode])
        b.set_mode(mode)
        evolve()
        times[mode] = evolve()
    b.close()
    eng = Engine(**cfg["grid"])
    eng.autotune(None)
    eng.init_pulse(**cfg["pulse"])
    eng.step(n, waveform=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(len(grids)):
        eng.init_pulse(**cfg["pulse"])
        eng.step(n, waveform=False)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t1
    eng.close()
    return {"workload": "64 x schwarzschild_pulse_801x33", "instances": len(grids), "points": pts, "iterations": n,
            "by_mode": {names[m]: {"seg_rows": best_seg[m], "s": round(times[m], 3),
                                   "gpts": round(pts * n / times[m] / 1e9, 3)} for m in times},
            "plain_sequential_s": round(tp, 3), "plain_gpts": round(pts * n / tp / 1e9, 3)}


def all_m(args):
    """Every m of one orbit (m = 1..4, each with the orbit's source) as one
    batch against the same instances stepped one after another."""
    import torch
    from paper_1001_3631_amd import workloads as W
    from paper_1001_3631_amd.engine import Batch, Engine
    cfg = W.ALL_M
    grids, src = cfg["grids"], cfg["source"]
    n = args.all_m_iterations or cfg["steps"]
    pts = sum(g["nr"] * g["nth"] for g in grids)

    def attach(e, g):
        orbit = e.orbit_circular(src["r0"], 2 * n + 1, M=g["M"], a=g["a"])
        e.set_source(orbit, src["amplitude"], src["sigma_r_cells"], src["sigma_th_cells"], src["cutoff_sigmas"])

    b = Batch(grids)
    for e, g in zip(b.instances, grids):
        attach(e, g)
    tune = b.autotune(None)                         # sources detached while timing
    waves = [torch.empty((n, g["nth"]), dtype=torch.complex128, device="cuda") for g in grids]
    z = [torch.zeros((g["nth"], g["nr"]), dtype=torch.complex128, device="cuda") for g in grids]

    def evolve():
        for e, zz in zip(b.instances, z):
            e.set_state(zz, zz)                     # zero data, source clock back to 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(n, out=waves)
        b.sync()
        return time.perf_counter() - t0

    evolve()
    tb = evolve()
    for e in b.instances:
        e.check_finite()
    b.close()
    del waves

    tp = 0.0
    for g in grids:
        eng = Engine(**g)
        eng.autotune(None)
        attach(eng, g)
        w = torch.empty((n, g["nth"]), dtype=torch.complex128, device="cuda")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        eng.step(n, out=w)
        torch.cuda.synchronize()
        tp += time.perf_counter() - t1
        eng.check_finite()
        eng.close()
    names = {Batch.PERSISTENT: "persistent", Batch.PER_ITERATION: "per_iteration"}
    return {"workload": cfg["name"], "instances": len(grids), "points": pts, "iterations": n,
            "mode": names[tune[0][1]], "seg_rows": tune[0][0],
            "batched_s": round(tb, 3), "batched_gpts": round(pts * n / tb / 1e9, 3),
            "plain_sequential_s": round(tp, 3), "plain_gpts": round(pts * n / tp / 1e9, 3),
            "batched_over_plain": round(tp / tb, 3)}


def hbm_grid():
    """The stencil on a grid whose state lives in HBM (25600 x 512: both
    levels 3.3x the last-level cache).  The single-step kernel at its best
    segment length gives the roofline block (64 B per point update, HBM
    bound); the autotuner's overall choice (which may fuse k iterations per
    launch, 64/k B per point update) gives the throughput; a plain device
    copy gives the achievable streaming bandwidth."""
    import torch
    from paper_1001_3631_amd import workloads as W
    hc = W.HBM_PLAIN
    hg = hc["grid"]
    hn = hc["steps"]
    hpts = hg["nr"] * hg["nth"]
    heng = make_engine(hc, hn)
    table = heng.autotune(None)              # [(seg, k, us/iteration)], fastest first
    best = table[0]
    single = min((t for t in table if t[1] == 1), key=lambda t: t[2])
    hphi = torch.zeros((hg["nth"], hg["nr"]), dtype=torch.complex128, device="cuda")
    hpi = torch.zeros_like(hphi)
    hwave = torch.empty((hn, hg["nth"]), dtype=torch.complex128, device="cuda")

    def timed():
        run_evolution(heng, hphi, hpi, hn, hwave)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run_evolution(heng, hphi, hpi, hn, hwave)
        torch.cuda.synchronize()
        return time.perf_counter() - t1

    out = {"workload": hc["name"], "iterations": hn, "state_bytes_per_level": hpts * 32}
    heng.set_tuning(single[0], 1)
    t_single = timed()
    out["roofline"] = stencil_roofline(heng, hc["name"], hpts, lambda: run_evolution(heng, hphi, hpi, hn, hwave))
    out["single_step_gpts"] = round(hn * hpts / t_single / 1e9, 3)
    heng.set_tuning(best[0], best[1])
    t_best = timed()
    out["autotuned"] = {"tuning": {"seg_rows": best[0], "k_steps": best[1]},
                        "gpts": round(hn * hpts / t_best / 1e9, 3),
                        "effective_GBs": round(hn * hpts * BYTES_PER_POINT / t_best / 1e9, 1),
                        "table_us_per_iteration": [[t[0], t[1], round(t[2], 2)] for t in table]}
    heng.close()
    del hphi, hpi, hwave
    out["stream_copy"] = stream_copy()
    return out


def cpu_baseline(cfg, iters):
    import numpy as np
    from oracle import teuk_oracle as T
    g = T.Grid(**cfg["grid"])
    src = cfg["source"]
    orbit = T.circular_orbit(g.M, g.a, src["r0"], g.dt, iters)
    s = T.Source(g, orbit, src["amplitude"], src["sigma_r_cells"], src["sigma_th_cells"],
                 src["cutoff_sigmas"])
    z = np.zeros((g.nth, g.nr), np.complex128)
    t0 = time.perf_counter()
    T.evolve(g, z, z, iters, s)
    dt = time.perf_counter() - t0
    return {"value": iters * g.nr * g.nth / dt / 1e9, "unit": "GPts/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{iters} iterations of the {cfg['name']} workload (NumPy FP64, one thread), "
                      f"{dt:.1f} s"}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note only)"}))
        sys.exit(2)
    import torch
    from paper_1001_3631_amd import workloads as W

    assert torch.cuda.is_available(), "bench needs a HIP device"
    cfg = W.KERR_EMRI if args.workload == W.KERR_EMRI["name"] else W.HBM_PLAIN
    g = cfg["grid"]
    n = args.iterations or cfg["steps"]
    npts = g["nr"] * g["nth"]
    eng = make_engine(cfg, n)
    if args.tuning:
        seg, k = (int(v) for v in args.tuning.split(","))
        eng.set_tuning(seg, k)
    else:
        eng.autotune(None)                  # launch configuration by measurement (untimed)
    tune = eng.tuning
    zphi = torch.zeros((g["nth"], g["nr"]), dtype=torch.complex128, device="cuda")
    zpi = torch.zeros_like(zphi)
    wave = torch.empty((n, g["nth"]), dtype=torch.complex128, device="cuda")

    for _ in range(args.warmup):
        run_evolution(eng, zphi, zpi, n, wave)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_evolution(eng, zphi, zpi, n, wave)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    eng.check_finite()
    ms_per_step = elapsed / args.steps * 1e3
    gpts = args.steps * n * npts / elapsed / 1e9
    print(f"[bench] {cfg['name']}: {args.steps} evolutions of {n} iterations in {elapsed:.3f} s "
          f"-> {gpts:.2f} GPts/s", file=sys.stderr, flush=True)

    # dominant kernel: average stencil launch duration from HIP events
    roofline = stencil_roofline(eng, cfg["name"], npts, lambda: run_evolution(eng, zphi, zpi, n, wave))
    print(f"[bench] stencil launch avg {roofline['avg_launch_us']:.2f} us -> {roofline['achieved']:.0f} GB/s "
          f"algorithmic", file=sys.stderr, flush=True)

    extra = {}
    if not args.no_hbm and cfg is not W.HBM_PLAIN:
        eng.close()
        del wave
        extra["hbm_grid"] = hbm_grid()
        print(f"[bench] hbm_grid: {extra['hbm_grid']}", file=sys.stderr, flush=True)

    if not args.no_adjoint:
        extra["adjoint"] = adjoint_ratio(args)
        print(f"[bench] adjoint: {extra['adjoint']}", file=sys.stderr, flush=True)

    if not args.no_batched:
        extra["batched"] = batched(args)
        print(f"[bench] batched: {extra['batched']}", file=sys.stderr, flush=True)
        extra["all_m"] = all_m(args)
        print(f"[bench] all_m: {extra['all_m']}", file=sys.stderr, flush=True)
        extra["small_batch"] = small_batch(args)
        print(f"[bench] small_batch: {extra['small_batch']}", file=sys.stderr, flush=True)

    if not args.no_scale:
        extra["adjoint_at_scale"] = adjoint_at_scale(args)
        print(f"[bench] adjoint_at_scale: {extra['adjoint_at_scale']}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(cfg, args.cpu_iters)
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)

    line = {
        "metric": "grid-point updates/s (GPts/s) + % HBM roofline; adjoint/forward time ratio",
        "value": round(gpts, 4), "unit": "GPts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": [g["nr"], g["nth"]], "iterations": n,
                   "a": g["a"], "m": g["m"], "s": g["s"], "source": "circular r0=10M",
                   "extraction": "every iteration at r*=500M", "parallelism": "single GPU",
                   "tuning": {"seg_rows": tune["seg_rows"], "k_steps": tune["k_steps"]}},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
