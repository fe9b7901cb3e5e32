#!/usr/bin/env python3
"""Leaf-cell updates/s of the MR-LBM hot path on one MI355X.

Workload (the D1Q3 Burgers family at full size): D1Q3 scheme with m2^eq = 0.9 lambda^2 u,
lambda = 1, periodic [-1, 1], J_min = 2, J = 14 (16384 finest cells), gamma = 1,
mu_bar = 0; the sweep s in {1.5, 1.9} x eps in {1e-2, 1e-3, 1e-4}, with ``--seeds``
seeded initial data per pair (Riemann data + sine, see workloads.burgers); the default
85 seeds give 510 runs, about two per compute unit. All runs advance together in the
batched engine (one workgroup per run, persistent over the whole launch); a "step" is one
time step of every run. The runs are checkpointed at t = 0; the built-in tuner picks the
launch shape and the run-to-workgroup schedule with trials of the timed step count from
t = 0 (restored after each); the warmup advances the runs in that configuration (one launch),
they are restored to t = 0 and the timed steps run as one launch. T = 0.4 is 3277 steps: by
default the warmup and the timed region are each the whole run, so the two launches are the
same work in the same configuration.

Reported next to the throughput:
* roofline of the step kernel: algorithmic bytes (2 q s_b + 8 per leaf-cell update: read
  and write the populations once, a 4-byte leaf key read and written) per launch over the
  launch time measured with HIP events on the library's stream; peak 8 TB/s HBM;
* the plain adaptive step: the same kind of run advanced by one launch per time step
  and run, for comparison;
* the error check: delta = ||M_ref - m_hathat||_1 on the conserved moment against an
  eps = 0 run of the same library (the uniform finest-grid scheme, bit for bit), as delta/eps;
* the batched ensemble (FP64 and FP32): 4096 independent D1Q2 advection/Burgers instances
  with J uniform in 8..14 in one launch, against one launch per time step and instance;
* the reconstructed collision (Sec. 4.3.1): the same 510 runs, the first 200 steps with it
  and with the leaves collision in the same launch shape, and delta/eps of two runs;
* the learned-refinement form: on D1Q2^3 Euler Riemann problems (J = 14, eps = 1e-4) the
  network is trained on the rule-(b) pairs the method records, then unseen runs advance with
  and without it: leaf-cell updates/s, delta/eps, misses and redos of the judge;
* the CPU baseline: the FP64 oracle (plain numpy, one thread) on two whole runs of the
  workload (about 14 s).
"""

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
Q = 3  # D1Q3


def b_alg(q, prec):
    sb = 8 if prec == 0 else 4
    return 2 * q * sb + 8


def instances(seeds, prec):
    out = []
    for s in (1.5, 1.9):
        for eps in (1e-2, 1e-3, 1e-4):
            for seed in range(seeds):
                p, mc = W.burgers(seed, jmax=14, eps=eps, s=s)
                p["precision"] = prec
                out.append((p, mc))
    return out


def delta_check(mrlbm, cases, nsteps):
    """delta/eps of a few runs against the eps = 0 run (the uniform scheme)."""
    worst = 0.0
    rows = []
    for p, mc in cases:
        a = mrlbm.MRLBM(p, mc)
        r = mrlbm.MRLBM(dict(p, eps=0.0, precision=0), mc)
        a.step(nsteps)
        r.step(nsteps)
        ma = a.moments(mrlbm.FINEST)
        mr = r.moments(mrlbm.FINEST)
        dx = (p["x_max"] - p["x_min"]) / ma.shape[1]
        d = float(dx * np.sum(np.abs(ma[0] - mr[0])))
        rows.append({"s": p["s"][0], "eps": p["eps"], "delta": d, "delta_over_eps": d / p["eps"],
                     "leaves": a.stats()["leaves"]})
        worst = max(worst, d / p["eps"])
        a.close()
        r.close()
    return worst, rows


def plain_step_rate(mrlbm, cases, nsteps):
    """One launch per time step and run (the plain adaptive step), all runs on one stream."""
    runs = [mrlbm.MRLBM(p, mc) for p, mc in cases]
    for r in runs:
        r.step(5)
    for r in runs:
        r.stats()
    u0 = sum(r.stats()["leaf_updates"] for r in runs)
    t0 = time.perf_counter()
    for _ in range(nsteps):
        for r in runs:
            r.step(1)
    u1 = sum(r.stats()["leaf_updates"] for r in runs)  # stats synchronizes
    dt = time.perf_counter() - t0
    for r in runs:
        r.close()
    return (u1 - u0) / dt, dt


def cpu_baseline(sample_runs):
    """The FP64 oracle, as it stands, on whole runs of the workload (s = 1.9, eps = 1e-4,
    seeds 0 .. sample_runs-1, 3277 steps each): about 7 s of single-core work per run."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle.adaptive import AdaptiveMRLBM
    from oracle.lattice import scheme_from_params
    upd, dt, steps = 0, 0.0, 0
    for seed in range(sample_runs):
        p, mc = W.burgers(seed, jmax=14, eps=1e-4, s=1.9)
        a = AdaptiveMRLBM(scheme_from_params(p), p["jmin"], p["jmax"], p["gamma"], p["eps"], p["mu_bar"],
                          p["bc"], mc)
        t0 = time.perf_counter()
        a.step(p["steps"])
        dt += time.perf_counter() - t0
        upd += a.leaf_updates
        steps = p["steps"]
    return {"value": upd / dt, "unit": "leaf-cell updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample_runs} whole D1Q3 Burgers runs of the workload (J=14, s=1.9, eps=1e-4, "
                      f"seeds 0..{sample_runs - 1}, {steps} steps each), {upd} leaf-cell updates in "
                      f"{dt:.2f} s, single-threaded numpy",
            "host": platform.processor() or platform.machine(), "host_cpus": os.cpu_count()}


def euler_runs(seeds, jmax, eps, steps):
    ps, ms = [], []
    for s in seeds:
        p, mc = W.euler(s, jmax=jmax, eps=eps, steps=steps)
        ps.append(p)
        ms.append(mc)
    return ps, ms


def ensemble_form(mrlbm, n, steps, prec, tune):
    """The batched ensemble: n independent D1Q2 advection/Burgers instances with J uniform
    in 8..14 and eps in {1e-3, 1e-4} (workloads.batch_instance) in one launch, against the
    same instances advanced by one launch per time step and instance (a sample of them)."""
    cases = []
    for seed in range(n):
        p, mc = W.batch_instance(seed, steps=steps)
        p["precision"] = prec
        cases.append((p, mc))
    b = mrlbm.Batch([c[0] for c in cases], [c[1] for c in cases])
    b.checkpoint()
    t = b.tune(steps) if tune else None
    b.step(steps)
    b.restore()
    u0 = b.total_updates()
    ms = b.step_timed(steps)
    upd = b.total_updates() - u0
    shape = [b.get_block(), b.get_capacity(), b.get_schedule()]
    b.close()
    sample = cases[:: max(1, n // 64)]
    rate_plain, _ = plain_step_rate(mrlbm, sample, 100)
    js = [c[0]["jmax"] for c in cases]
    return {"runs": n, "steps": steps, "j_max_range": [min(js), max(js)], "updates_per_s": upd / (ms / 1e3),
            "ms": ms, "leaf_updates": upd, "tuned": t is not None,
            "threads_capacity_schedule": shape,
            "per_instance_launches_updates_per_s": rate_plain,
            "speedup_vs_per_instance_launches": (upd / (ms / 1e3)) / rate_plain,
            "per_instance_sample": len(sample)}


def reconstructed_form(mrlbm, seeds, steps, tune=True, block=0, capacity=-1, schedule=256):
    """The reconstructed collision (Sec. 4.3.1) on the benchmark's workload (the 510-run D1Q3
    Burgers batch, J = 14): the first `steps` steps from t = 0, against the leaves collision
    on the same steps, each in the launch shape the built-in tuner picks for it (or the given
    one), and delta/eps of two runs against the eps = 0 run."""
    out = {"steps": steps}
    for coll in ("leaves", "reconstructed"):
        cases = instances(seeds, 0)
        b = mrlbm.Batch([dict(c[0], collision=coll) for c in cases], [c[1] for c in cases])
        b.checkpoint()
        if tune:
            b.tune(steps)
        else:
            b.set_block(block or 512)
            if capacity >= 0:
                b.set_capacity(capacity)
            b.set_schedule(schedule)
        b.step(steps)
        b.restore()
        u0 = b.total_updates()
        ms = b.step_timed(steps)
        upd = b.total_updates() - u0
        out[coll] = {"updates_per_s": upd / (ms / 1e3), "ms_per_step": ms / steps, "leaf_updates": upd,
                     "threads_capacity_schedule": [b.get_block(), b.get_capacity(), b.get_schedule()],
                     "tuned": tune}
        b.close()
    out["reconstructed_over_leaves"] = out["reconstructed"]["updates_per_s"] / out["leaves"]["updates_per_s"]
    sample = [(dict(p, collision="reconstructed"), mc) for p, mc in instances(1, 0)
              if p["s"][0] == 1.9 and p["eps"] in (1e-3, 1e-4)]
    worst, rows = delta_check(mrlbm, sample, steps)
    out["max_delta_over_eps"] = worst
    out["delta_runs"] = rows
    return out


def learned_form(mrlbm, n_train, n_test, steps, jmax=14, eps=1e-4, pos_weight=16.0, gate=8.0):
    """The learned-refinement form on the D1Q2^3 Euler Riemann problems (J = 14, eps = 1e-4):
    record the rule-(b) pairs of n_train runs, train the network on the GPU, then advance
    n_test unseen runs in the batched engine with and without it (same launch shape)."""
    ps, ms = euler_runs(range(1000, 1000 + n_train), jmax, eps, steps)
    rec = mrlbm.Batch(ps, ms)
    rec.set_predictor(None, mrlbm.PRED_RECORD, sample_capacity=2_000_000)
    rec.step(steps)
    X, y = rec.samples()
    rec.close()
    t0 = time.perf_counter()
    net = mrlbm.MLP(W.mlp_init(0))
    loss = net.train(X, y, epochs=20, batch=512, lr=2e-3, pos_weight=pos_weight, seed=3)
    _, bits = net.params()
    net.close()
    t_train = time.perf_counter() - t0
    ps, ms = euler_runs(range(2000, 2000 + n_test), jmax, eps, steps)
    ref = mrlbm.Batch([dict(p, eps=0.0) for p in ps], ms)
    ref.step(steps)
    fin_ref = [ref.moments(i, mrlbm.FINEST) for i in range(n_test)]
    ref.close()
    out = {"workload": f"D1Q2^3 Euler Riemann problems, J_min=2 J={jmax}, eps={eps}, s=1.9, lambda=3, clamp",
           "train_runs": n_train, "test_runs": n_test, "steps": steps, "samples": int(X.shape[0]),
           "positive_fraction": float(y.mean()), "train_seconds": t_train, "train_loss": loss,
           "pos_weight": pos_weight, "gate": gate}
    for name, mode in (("plain", mrlbm.PRED_OFF), ("learned", mrlbm.PRED_LEARNED)):
        b = mrlbm.Batch(ps, ms)
        if mode != mrlbm.PRED_OFF:
            b.set_predictor(bits, mode, gate)
        ms_run = b.step_timed(steps)
        sts = [b.stats(i) for i in range(n_test)]
        upd = sum(st["leaf_updates"] for st in sts)
        worst = 0.0
        for i in range(n_test):
            m = b.moments(i, mrlbm.FINEST)
            dx = 2.0 / m.shape[1]
            worst = max(worst, max(float(dx * np.sum(np.abs(m[c] - fin_ref[i][c]))) for c in range(m.shape[0])))
        b.close()
        out[name] = {"updates_per_s": upd / (ms_run / 1e3), "leaf_updates": upd, "ms": ms_run,
                     "max_delta_over_eps": worst / eps, "misses": sum(st["misses"] for st in sts),
                     "redos": sum(st["redos"] for st in sts)}
    out["leaf_update_gain"] = 1.0 - out["learned"]["leaf_updates"] / out["plain"]["leaf_updates"]
    out["speed_vs_plain"] = out["learned"]["updates_per_s"] / out["plain"]["updates_per_s"]
    return out


def copy_probe(nbytes):
    """Device-to-device copy of known size through the HIP runtime (its blit kernel), for
    scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters: 3 copies of nbytes."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    n = ctypes.c_size_t(nbytes)
    if hip.hipMalloc(ctypes.byref(a), n) or hip.hipMalloc(ctypes.byref(b), n):
        raise RuntimeError("hipMalloc failed")
    try:
        if hip.hipMemset(a, 1, n) or hip.hipDeviceSynchronize():
            raise RuntimeError("hipMemset failed")
        for _ in range(3):
            if hip.hipMemcpy(b, a, n, 3):  # hipMemcpyDeviceToDevice
                raise RuntimeError("hipMemcpy failed")
        if hip.hipDeviceSynchronize():
            raise RuntimeError("copy failed")
    finally:
        hip.hipFree(a)
        hip.hipFree(b)
    print(json.dumps({"copy_probe_bytes": nbytes, "copies": 3}))


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Device-to-device copy rate through the HIP runtime (read + write bytes per second, GB/s),
    timed with HIP events: a measured ceiling beside the nominal 8 TB/s."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    e0, e1 = ctypes.c_void_p(), ctypes.c_void_p()
    n = ctypes.c_size_t(nbytes)
    if hip.hipMalloc(ctypes.byref(a), n) or hip.hipMalloc(ctypes.byref(b), n):
        raise RuntimeError("hipMalloc failed")
    try:
        if hip.hipEventCreate(ctypes.byref(e0)) or hip.hipEventCreate(ctypes.byref(e1)):
            raise RuntimeError("hipEventCreate failed")
        if hip.hipMemset(a, 1, n) or hip.hipMemcpy(b, a, n, 3) or hip.hipDeviceSynchronize():
            raise RuntimeError("copy warmup failed")
        hip.hipEventRecord(e0, None)
        for _ in range(reps):
            if hip.hipMemcpyAsync(b, a, n, 3, None):
                raise RuntimeError("hipMemcpyAsync failed")
        hip.hipEventRecord(e1, None)
        if hip.hipEventSynchronize(e1):
            raise RuntimeError("copy failed")
        ms = ctypes.c_float()
        hip.hipEventElapsedTime(ctypes.byref(ms), e0, e1)
        hip.hipEventDestroy(e0)
        hip.hipEventDestroy(e1)
    finally:
        hip.hipFree(a)
        hip.hipFree(b)
    return 2.0 * nbytes * reps / (ms.value / 1e3) / 1e9


def profile_summary(path):
    """Text summary of rocprofv3 CSV output under ``path`` (kernel stats, per-dispatch trace
    figures of the step kernel, and counter averages per kernel)."""
    import csv
    import glob
    lines = []
    for f in sorted(glob.glob(os.path.join(path, "**", "*_kernel_stats.csv"), recursive=True)):
        lines.append(f"kernel stats ({os.path.basename(f)}):")
        lines.append(f"  {'calls':>6} {'avg_us':>12} {'total_ms':>10} {'pct':>6}  name")
        with open(f) as fh:
            for r in list(csv.DictReader(fh))[:8]:
                lines.append(f"  {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:12.1f} "
                             f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}  {r['Name'][:90]}")
    for f in sorted(glob.glob(os.path.join(path, "**", "*_kernel_trace.csv"), recursive=True)):
        with open(f) as fh:
            rows = [r for r in csv.DictReader(fh) if "k_steps" in r["Kernel_Name"]]
        for r in rows[:12]:
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            name = r["Kernel_Name"]
            tmpl = name[name.find("k_steps"):name.find(">") + 1] if "<" in name else "k_steps"
            lines.append(f"step kernel dispatch: {dur:.1f} us, grid {r['Grid_Size_X']}, workgroup "
                         f"{r['Workgroup_Size_X']}, LDS {r['LDS_Block_Size']} B, VGPR {r['VGPR_Count']}, "
                         f"AGPR {r['Accum_VGPR_Count']}, SGPR {r['SGPR_Count']}, scratch {r['Scratch_Size']} B"
                         f"  {tmpl}")
    for f in sorted(glob.glob(os.path.join(path, "**", "*_counter_collection.csv"), recursive=True)):
        acc = {}
        with open(f) as fh:
            for r in csv.DictReader(fh):
                k = (r["Kernel_Name"][:70], r["Counter_Name"])
                d = acc.setdefault(k, {})
                d[r["Dispatch_Id"]] = d.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        lines.append(f"counters ({os.path.basename(f)}), average per dispatch:")
        for (kn, cn), d in sorted(acc.items()):
            v = list(d.values())
            lines.append(f"  {cn:>12} {sum(v) / len(v):16.1f} over {len(v):3d} dispatches  {kn}")
    print("\n".join(lines) if lines else f"no rocprofv3 CSV output under {path}")


KERNEL_SOURCES = ("mrlbm_device.h", "mrlbm_kernels.h", "instances.hip")
COUNTER_FILE = os.path.join(ROOT, "profiles", "k_steps_burgers_j14_counters.txt")


def kernel_source_hash():
    """sha256 over the sources of the step kernel: counters taken on other sources are stale."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2102_12163_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counter_avg(path, counter, kernel_substr):
    import csv
    import glob
    per = {}
    for f in glob.glob(os.path.join(path, "**", "*_counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and kernel_substr in r["Kernel_Name"]:
                    per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for {kernel_substr} under {path}")
    return sum(per.values()) / len(per), len(per)


def traffic_summary(dirs, copy_bytes, updates):
    """Machine-readable block of HBM traffic per step-kernel launch from four rocprofv3 --pmc
    folders (step FETCH_SIZE, step WRITE_SIZE, copy FETCH_SIZE, copy WRITE_SIZE); each counter
    is scaled by what it reads for the copy probe of known size (KiB per dispatch)."""
    fd, wd, cfd, cwd = dirs.split(",")
    f, nf = _counter_avg(fd, "FETCH_SIZE", "k_steps")
    w, nw = _counter_avg(wd, "WRITE_SIZE", "k_steps")
    cf, _ = _counter_avg(cfd, "FETCH_SIZE", "copyBuffer")
    cw, _ = _counter_avg(cwd, "WRITE_SIZE", "copyBuffer")
    kib = copy_bytes / 1024.0
    sf, sw = kib / cf, kib / cw
    traffic = (f * sf + w * sw) * 1024.0
    print(f"kernel_source_sha256: {kernel_source_hash()}")
    print(f"fetch_kib_per_dispatch: {f:.1f}  (over {nf} dispatches)")
    print(f"write_kib_per_dispatch: {w:.1f}  (over {nw} dispatches)")
    print(f"copy_probe_bytes: {copy_bytes}  fetch_kib {cf:.1f} -> scale {sf:.4f}  write_kib {cw:.1f} -> scale {sw:.4f}")
    print(f"traffic_bytes_per_launch: {traffic:.6e}")
    print(f"updates_per_launch: {updates:.0f}")
    print(f"traffic_bytes_per_update: {traffic / updates:.3f}")


def traffic_for(upd):
    """HBM bytes of a launch of ``upd`` leaf-cell updates from the committed counter summary
    (bytes per update x updates), or None when the summary is missing or the kernel sources
    changed since it was taken."""
    try:
        with open(COUNTER_FILE) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("kernel_source_sha256", "").strip() != kernel_source_hash():
        return None
    return float(kv["traffic_bytes_per_update"].split()[0]) * upd


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3277, help="timed steps (3277: the whole run to T=0.4)")
    ap.add_argument("--warmup", type=int, default=3277,
                    help="untimed steps before the timed region; the runs are then put back to t=0")
    ap.add_argument("--launch-steps", type=int, default=0,
                    help="steps per kernel launch (0: the warmup and the timed steps as one launch each)")
    ap.add_argument("--seeds", type=int, default=85, help="seeded runs per (s, eps) pair")
    ap.add_argument("--no-tune", action="store_true", help="skip the built-in launch-shape tuner")
    ap.add_argument("--tune-steps", type=int, default=0,
                    help="steps of each tuner trial, from t=0 (0: the timed step count)")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--block", type=int, default=0, help="threads per workgroup (0: tuner)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-runs", type=int, default=2)
    ap.add_argument("--no-extras", action="store_true", help="skip the plain-step and delta checks")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-refinement form")
    ap.add_argument("--learned-steps", type=int, default=2400)
    ap.add_argument("--ensemble-runs", type=int, default=4096, help="instances of the batched ensemble")
    ap.add_argument("--ensemble-steps", type=int, default=512)
    ap.add_argument("--recon-steps", type=int, default=200, help="steps of the reconstructed-collision form")
    ap.add_argument("--recon-only", action="store_true",
                    help="only the reconstructed-collision form (for profiling its launches)")
    ap.add_argument("--capacity", type=int, default=-1, help="on-chip capacity in cells (-1: tuner or default)")
    ap.add_argument("--schedule", type=int, default=-1, help="workgroup schedule stride (-1: tuner or identity)")
    ap.add_argument("--profile-summary", default="", help="only summarize rocprofv3 CSV output in this folder")
    ap.add_argument("--traffic-summary", default="", help="only print the traffic block from four --pmc folders "
                    "(step FETCH, step WRITE, copy FETCH, copy WRITE), comma-separated")
    ap.add_argument("--traffic-updates", type=float, default=0, help="leaf-cell updates per profiled launch")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run a device copy of this many bytes")
    args = ap.parse_args()

    if args.traffic_summary:
        traffic_summary(args.traffic_summary, 1073741824, args.traffic_updates)
        return 0
    if args.profile_summary:
        profile_summary(args.profile_summary)
        return 0
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures a single GPU (asked for {args.gpus}): the batched engine runs on one "
              f"device; across GPUs the independent runs would be split by instance", file=sys.stderr)
        return 2
    if (args.steps <= 0 or args.warmup < 0 or args.seeds <= 0 or args.launch_steps < 0 or args.ensemble_runs <= 0
            or args.ensemble_steps <= 0):
        print("bench.py needs --steps > 0, --warmup >= 0, --seeds > 0, --launch-steps >= 0, --ensemble-runs > 0, "
              "--ensemble-steps > 0", file=sys.stderr)
        return 2

    from paper_2102_12163_amd import mrlbm

    if args.recon_only:
        print(json.dumps({"reconstructed_form": reconstructed_form(
            mrlbm, args.seeds, args.recon_steps, tune=not args.no_tune, block=args.block, capacity=args.capacity,
            schedule=args.schedule if args.schedule >= 0 else 256)}))
        return 0
    prec = 0 if args.precision == "fp64" else 1
    cases = instances(args.seeds, prec)
    print(f"[bench] {len(cases)} runs, warmup {args.warmup}, timed {args.steps}", file=sys.stderr, flush=True)
    batch = mrlbm.Batch([c[0] for c in cases], [c[1] for c in cases])
    batch.set_launch_steps(args.launch_steps)
    tuned = None
    if args.block:
        batch.set_block(args.block)
    if args.capacity >= 0:
        batch.set_capacity(args.capacity)
    batch.checkpoint()  # t = 0
    # launch shape and schedule fixed at t = 0 (tuner trials from t = 0, restored after each),
    # so that the warmup launch runs in the timed configuration
    if not args.block and args.capacity < 0 and not args.no_tune:
        tuned = batch.tune(args.tune_steps or args.steps)
        print(f"[bench] tuner: {tuned[0]} threads per workgroup, on-chip capacity {tuned[1]} cells, "
              f"schedule stride {batch.get_schedule()}", file=sys.stderr, flush=True)
    if args.schedule >= 0:
        batch.set_schedule(args.schedule)
    cap_cells = batch.get_capacity()
    sched = batch.get_schedule()
    if args.warmup:
        batch.step(args.warmup)
    # the timed steps start from t = 0 again: with the default counts the warmup launch and
    # the timed launch do the same work
    batch.restore()
    u0 = batch.total_updates()
    ms = batch.step_timed(args.steps)
    u1 = batch.total_updates()
    upd = u1 - u0
    value = upd / (ms / 1e3)
    leaves_now = [batch.stats(i)["leaves"] for i in range(len(cases))]
    block = batch.get_block()
    print(f"[bench] timed region {ms:.1f} ms, {upd} leaf-cell updates", file=sys.stderr, flush=True)
    chunked = None
    if not args.no_extras and args.launch_steps == 0:
        # the same timed steps as launches of 113 steps (all runs synchronise at every launch)
        batch.restore()
        batch.set_launch_steps(113)
        c0 = batch.total_updates()
        msc = batch.step_timed(args.steps)
        uc = batch.total_updates() - c0
        chunked = {"launch_steps": 113, "updates_per_s": uc / (msc / 1e3), "ms_per_step": msc / args.steps,
                   "note": "timed steps as launches of 113 steps from t=0; every launch waits for its "
                           "slowest run"}
    batch.close()

    bpu = b_alg(Q, prec)
    launches = -(-args.steps // args.launch_steps) if args.launch_steps > 0 else 1
    # algorithmic bytes per launch / average launch duration = total bytes / total time
    achieved = upd * bpu / (ms / 1e3) / 1e9
    result = {
        "metric": "leaf-cell updates/s and % HBM roofline at error<=C*eps vs plain adaptive step",
        "value": value,
        "unit": "leaf-cell updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32",
        "data": "synthetic",
        "config": {
            "workload": "D1Q3 Burgers, J_min=2 J=14 (16384 cells), gamma=1, periodic [-1,1], "
                        "s in {1.5,1.9} x eps in {1e-2,1e-3,1e-4}, batched runs",
            "runs": len(cases), "seeds_per_pair": args.seeds, "finest_cells": 16384,
            "threads_per_workgroup": block, "onchip_capacity_cells": cap_cells, "schedule_stride": sched,
            "tuned": tuned is not None, "launch_steps": args.launch_steps,
            "form": "batched engine, persistent workgroups; timed steps from t=0 (checkpoint restored after "
                    "the warmup), one launch (launch_steps 0) or launches of launch_steps steps",
            "mean_leaves_per_run": float(np.mean(leaves_now)),
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(upd / launches) if prec == 0 else None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-probe scaled)",
            "kernel": "k_steps<double,1,1>" if prec == 0 else "k_steps<float,1,1>",
            "bytes_per_update": bpu, "launches": launches, "avg_launch_ms": ms / launches,
        },
    }
    if chunked is not None:
        result["chunked_launches"] = chunked
    if not args.no_extras:
        cbw = copy_bandwidth()
        result["roofline"]["measured_copy_gbs"] = cbw
        result["roofline"]["frac_of_measured_copy"] = achieved / cbw
    nJ = 16384
    result["compression"] = {
        "mean_cr_pct": 100.0 * (1.0 - float(np.mean(leaves_now)) / nJ),
        "definition": "CR = 100 (1 - #leaves / 2^J) at the end of the timed run, averaged over the runs",
        "paper_context": "the paper's only efficiency figure: CR about 95 % (advection of a Gaussian, J=9) and "
                         "above 90 % (box advection), sequential C++ on an unreported CPU"}
    if not args.no_extras:
        one = [c for c in cases if c[0]["eps"] == 1e-4][:1] * 1
        rate_plain, _ = plain_step_rate(mrlbm, one, 300)
        rate_plain_all, _ = plain_step_rate(mrlbm, cases[:: max(1, len(cases) // 12)], 100)
        result["plain_step"] = {
            "one_run_updates_per_s": rate_plain,
            "per_run_launches_updates_per_s": rate_plain_all,
            "batched_speedup_vs_per_run_launches": value / rate_plain_all,
        }
        sample = [c for c in cases if c[0]["s"][0] == 1.9 and c[0]["eps"] in (1e-3, 1e-4)][:: args.seeds]
        worst, rows = delta_check(mrlbm, sample, args.steps)
        result["error_check"] = {"max_delta_over_eps": worst, "runs": rows,
                                 "reference": "eps=0 run of the same library (uniform finest scheme)"}
    if not args.no_extras and prec == 0:
        print("[bench] FP32-storage form", file=sys.stderr, flush=True)
        c32 = instances(args.seeds, 1)
        b32 = mrlbm.Batch([c[0] for c in c32], [c[1] for c in c32])
        b32.checkpoint()
        t32 = b32.tune(args.tune_steps or args.steps) if not args.no_tune else None
        if args.warmup:
            b32.step(args.warmup)
        b32.restore()
        v0 = b32.total_updates()
        ms32 = b32.step_timed(args.steps)
        u32 = b32.total_updates() - v0
        b32.close()
        sample32 = [c for c in c32 if c[0]["s"][0] == 1.9 and c[0]["eps"] in (1e-3, 1e-4)][:: args.seeds]
        worst32, _ = delta_check(mrlbm, sample32, args.steps)
        result["fp32_form"] = {"updates_per_s": u32 / (ms32 / 1e3), "ms_per_step": ms32 / args.steps,
                               "tuned": list(t32) if t32 else None, "bytes_per_update": b_alg(Q, 1),
                               "speed_vs_fp64": (u32 / (ms32 / 1e3)) / value,
                               "max_delta_over_eps": worst32,
                               "reference": "eps=0 FP64 run of the same library"}
    if not args.no_extras and prec == 0:
        print("[bench] batched ensemble", file=sys.stderr, flush=True)
        result["ensemble_form"] = {
            "fp64": ensemble_form(mrlbm, args.ensemble_runs, args.ensemble_steps, 0, not args.no_tune),
            "fp32": ensemble_form(mrlbm, args.ensemble_runs, args.ensemble_steps, 1, not args.no_tune)}
    if not args.no_extras and prec == 0:
        print("[bench] reconstructed collision", file=sys.stderr, flush=True)
        result["reconstructed_form"] = reconstructed_form(mrlbm, args.seeds, args.recon_steps,
                                                          tune=not args.no_tune, block=args.block,
                                                          capacity=args.capacity,
                                                          schedule=args.schedule if args.schedule >= 0 else 256)
    if not args.no_learned and prec == 0:
        print("[bench] learned-refinement form", file=sys.stderr, flush=True)
        result["learned_form"] = learned_form(mrlbm, 8, 64, args.learned_steps)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args.cpu_sample_runs)
    print(json.dumps(result))
    return 0


if __name__ == "__main__":
    sys.exit(main())
