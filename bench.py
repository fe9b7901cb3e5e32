#!/usr/bin/env python3
"""Leaf-cell updates/s of the MR-LBM hot path on one MI355X.

Headline workload (the batched ensemble): 4096 independent D1Q2 instances, advection
(V = 0.75, s = 1.9) or Burgers (s in {1.5, 1.9}) with probability 1/2, J uniform in 8..14,
eps in {1e-3, 1e-4}, gamma = 1, mu_bar = 0, periodic [-1, 1], seeded step + bump data
(workloads.batch_instance), 512 steps each, FP64. All instances advance together in the
batched engine: one workgroup per instance, persistent over a launch, one launch per call,
replayed from a HIP graph. A "step" is one time step of every instance.

Protocol: the instances start at t = 0 on the full tree (Sec. 4.4); ``--warmup`` W steps
advance them (the first of them, whose adaptation walks the full trees, is timed alone and
reported as ``t0_step_ms``); the timed region is the ``--steps`` K steps that follow, as one
launch (no restore: the timed steps continue the warmed-up runs). The launch shape is fixed
so that the committed rocprofv3 counters describe the launch that
is timed: two launch classes, the runs with J <= 12 in workgroups of 128 threads sized for eight
per compute unit and the J = 13, 14 runs in workgroups of 256 threads sized for four, the
heaviest class first and both grids side by side, heaviest instances first within each (the
step is latency bound: more, smaller workgroups per CU hide more of it); the built-in tuner's
choice for the same steps (which, on this batch, is this shape) is reported beside it.

Reported next to the throughput:
* ``roofline``: algorithmic bytes (2 q s_b + 8 = 40 per leaf-cell update for D1Q2 FP64:
  read and write the populations once, a 4-byte leaf key read and written) per launch over
  the launch time (HIP events on the library's stream), against 8 TB/s; ``traffic`` is the
  HBM bytes rocprofv3 counted for this very launch (FETCH_SIZE + WRITE_SIZE, scaled by a
  copy of known size), null when the committed counters were taken on other kernel sources
  or another launch; ``issue`` is the ceiling the kernel actually meets: its VALU and SALU
  wave instructions per update (SQ counters of the same launch) against the issue rate of
  256 CUs at 2.4 GHz;
* ``error_check``: delta/eps of one sampled instance per J over its whole 512-step run,
  against an eps = 0 run of the same library (the uniform scheme, bit for bit);
* extras: the whole 512-step run from t = 0 as one launch, the tuner's launch shape, the
  instances advanced by one launch per step and instance (the plain adaptive step), FP32
  storage, the D1Q3 Burgers batch (510 runs, J = 14, whole runs to T = 0.4), the
  reconstructed collision, the learned-refinement form;
* ``cpu_baseline``: the FP64 oracle (plain numpy, one thread per process) on whole runs of a
  sample of the same instances, over a pool of host processes.
"""

import os

# one BLAS thread per process, set before numpy loads (the CPU baseline's processes inherit it)
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import argparse  # noqa: E402
import json  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
# issue rates of MI355X: 256 CUs at 2.4 GHz; a CU's four SIMDs each take a wave64 VALU
# instruction every 4 cycles (16 lanes), its scalar unit one SALU instruction per cycle
CUS, CLOCK_HZ = 256, 2.4e9
VALU_ISSUE_PER_S = CUS * 4 * CLOCK_HZ / 4.0
SALU_ISSUE_PER_S = CUS * CLOCK_HZ
LDS_BYTES_PER_S = CUS * 128 * CLOCK_HZ

ENSEMBLE_STEPS = 512
# launch classes of the headline: runs with J <= 12 in workgroups of 128 threads sized for 8 per
# CU, the J = 13, 14 runs in workgroups of 256 threads sized for 4 per CU (heaviest class first)
HEADLINE_CLASSES = ([12, 14], [128, 256], [8, 4])
HEADLINE_SHAPE = {"block": 256, "capacity": 442}  # --no-classes: one launch, heaviest first
KERNEL_SOURCES = ("mrlbm_device.h", "mrlbm_kernels.h", "instances.hip")
COUNTER_FILE = os.path.join(ROOT, "profiles", "k_steps_ensemble4096_counters.txt")


def b_alg(q, prec):
    sb = 8 if prec == 0 else 4
    return 2 * q * sb + 8


def host_cpu():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


# ------------------------------------------------------------------ workloads
def ensemble_cases(n, prec):
    out = []
    for seed in range(n):
        p, mc = W.batch_instance(seed, steps=ENSEMBLE_STEPS)
        p["precision"] = prec
        out.append((p, mc))
    return out


def burgers_cases(seeds, prec):
    out = []
    for s in (1.5, 1.9):
        for eps in (1e-2, 1e-3, 1e-4):
            for seed in range(seeds):
                p, mc = W.burgers(seed, jmax=14, eps=eps, s=s)
                p["precision"] = prec
                out.append((p, mc))
    return out


def make_batch(mrlbm, cases, block=0, capacity=-1, schedule=-1):
    b = mrlbm.Batch([c[0] for c in cases], [c[1] for c in cases])
    if block:
        b.set_block(block)
    if capacity >= 0:
        b.set_capacity(capacity)
    if schedule >= 0:
        b.set_schedule(schedule)
    return b


def timed_region(b, warmup, steps):
    """W warmup steps (the first one timed alone), then K timed steps as one launch."""
    t0 = None
    if warmup > 0:
        t0 = b.step_timed(1)
        if warmup > 1:
            b.step(warmup - 1)
    u0 = b.total_updates()
    ms = b.step_timed(steps)
    upd = b.total_updates() - u0
    return ms, upd, t0


def delta_check(mrlbm, cases, nsteps):
    """delta/eps of each run after nsteps steps against the eps = 0 run of the same data (the
    uniform scheme, bit for bit), on the first conserved moment."""
    a = mrlbm.Batch([c[0] for c in cases], [c[1] for c in cases])
    r = mrlbm.Batch([dict(c[0], eps=0.0, precision=0) for c in cases], [c[1] for c in cases])
    a.step(nsteps)
    r.step(nsteps)
    rows, worst = [], 0.0
    for i, (p, _) in enumerate(cases):
        ma = a.moments(i, mrlbm.FINEST)
        mr = r.moments(i, mrlbm.FINEST)
        dx = (p["x_max"] - p["x_min"]) / ma.shape[1]
        d = float(dx * np.sum(np.abs(ma[0] - mr[0])))
        rows.append({"j_max": p["jmax"], "s": p["s"][0], "eps": p["eps"], "steps": nsteps, "delta": d,
                     "delta_over_eps": d / p["eps"], "leaves": a.stats(i)["leaves"]})
        worst = max(worst, d / p["eps"])
    a.close()
    r.close()
    return worst, rows


def hip_runtime():
    """The HIP runtime the library has loaded (same soname), for the baseline's streams."""
    import ctypes
    return ctypes.CDLL("libamdhip64.so")


def plain_step_rate(mrlbm, cases, nsteps, nstreams):
    """One launch per time step and run (the plain adaptive step), the runs spread round-robin
    over ``nstreams`` non-blocking HIP streams (one stream: every launch in order)."""
    import ctypes
    hip = hip_runtime()
    streams = []
    for _ in range(nstreams):
        sp = ctypes.c_void_p()
        if hip.hipStreamCreateWithFlags(ctypes.byref(sp), ctypes.c_uint(1)) != 0:
            raise RuntimeError("hipStreamCreateWithFlags failed")
        streams.append(sp)
    try:
        runs = [mrlbm.MRLBM(p, mc, stream=streams[i % nstreams]) for i, (p, mc) in enumerate(cases)]
        for r in runs:
            r.step(5)
        u0 = sum(r.stats()["leaf_updates"] for r in runs)  # stats synchronizes
        t0 = time.perf_counter()
        for _ in range(nsteps):
            for r in runs:
                r.step(1)
        u1 = sum(r.stats()["leaf_updates"] for r in runs)
        dt = time.perf_counter() - t0
        for r in runs:
            r.close()
    finally:
        for sp in streams:
            hip.hipStreamDestroy(sp)
    return (u1 - u0) / dt


# ------------------------------------------------------------------ CPU baseline (oracle)
def _oracle_instance(seed):
    from oracle.adaptive import AdaptiveMRLBM
    from oracle.lattice import scheme_from_params
    p, mc = W.batch_instance(seed, steps=ENSEMBLE_STEPS)
    a = AdaptiveMRLBM(scheme_from_params(p), p["jmin"], p["jmax"], p["gamma"], p["eps"], p["mu_bar"], p["bc"], mc)
    t0 = time.perf_counter()
    a.step(ENSEMBLE_STEPS)
    return a.leaf_updates, time.perf_counter() - t0


def cpu_baseline(sample, procs):
    """The FP64 oracle as it stands on whole 512-step runs of the first ``sample`` ensemble
    instances, one instance per task over a pool of ``procs`` single-threaded processes
    (spawned, before this process touches the GPU); updates per second of wall time."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_instance, range(sample), chunksize=1)
    wall = time.perf_counter() - t0
    upd = sum(r[0] for r in res)
    cpu_s = sum(r[1] for r in res)
    return {"value": upd / wall, "unit": "leaf-cell updates/s", "cores": procs, "kind": "oracle",
            "sample": f"whole {ENSEMBLE_STEPS}-step runs of ensemble instances 0..{sample - 1} (the headline's "
                      f"first {sample} instances), {upd} leaf-cell updates, {wall:.1f} s wall over {procs} "
                      f"single-threaded numpy processes ({cpu_s:.1f} s of oracle time in all)",
            "single_core_updates_per_s": upd / cpu_s,
            "host": host_cpu(), "host_cpus": os.cpu_count()}


# ------------------------------------------------------------------ committed counters
def kernel_source_hash():
    """sha256 over the sources of the step kernel: counters taken on other sources are stale."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2102_12163_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def workload_key(runs, steps, warmup, shape, schedule, prec):
    """shape: 'block=B capacity=C' of a single launch, or the launch classes."""
    return (f"ensemble runs={runs} steps={steps} warmup={warmup} {shape} "
            f"schedule={schedule} precision={'fp64' if prec == 0 else 'fp32'}")


def launch_shape(b, classes):
    """The launch shape of a batch as text (workload key) and as a config entry."""
    if not classes:
        return f"block={b.get_block()} capacity={b.get_capacity()}", None
    got = b.get_classes()
    rows = [{"j_max_upper": j, "threads": t, "runs_per_cu": r, "runs": n, "onchip_capacity_cells": c}
            for (j, t, r), (n, c) in zip(zip(*classes), got)]
    return classes_text(classes), rows


def classes_text(classes):
    """Launch classes as requested (j_max bound: threads x runs per CU); the capacities they
    give follow from the device's LDS and are reported beside the key."""
    return "classes=" + ";".join(f"j<={j}:{t}x{r}" for j, t, r in zip(*classes))


def read_counters(path=COUNTER_FILE):
    try:
        with open(path) as fh:
            return dict((k.strip(), v.strip()) for k, v in
                        (line.split(":", 1) for line in fh if ":" in line and not line.startswith("#")))
    except OSError:
        return {}


def counters_for(key):
    """The committed counter block when it was taken on these kernel sources and this very
    launch (workload key), else None."""
    kv = read_counters()
    if kv.get("kernel_source_sha256") != kernel_source_hash() or kv.get("workload_key") != key:
        return None
    return kv


def _rows(path, counter, kernel_substr):
    """Per-dispatch sums of one counter over the rocprofv3 CSV files under path."""
    import csv
    import glob
    per = {}
    for f in glob.glob(os.path.join(path, "**", "*_counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and kernel_substr in r["Kernel_Name"]:
                    d = int(r["Dispatch_Id"])
                    per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for {kernel_substr} under {path}")
    return per


def counters_summary(spec):
    """Counter block of the timed launch from rocprofv3 --pmc folders, printed in the format
    bench.py reads back. spec: comma-separated key=folder items: fetch, write (the bench
    command with FETCH_SIZE / WRITE_SIZE), cfetch, cwrite (the copy probe), sq (any number of
    folders with SQ_* counters), json (the bench line of the profiled run). The timed launch is
    the last step-kernel launch of the run: its last ``grids`` dispatches (one per launch
    class, summed)."""
    items = [kv.split("=", 1) for kv in spec.split(",")]
    ks = "k_steps"
    line = None
    sq = []
    d = {}
    for k, v in items:
        if k == "sq":
            sq.append(v)
        elif k == "json":
            with open(v) as fh:
                line = json.loads([x for x in fh.read().splitlines() if x.startswith("{")][-1])
        else:
            d[k] = v
    f = _rows(d["fetch"], "FETCH_SIZE", ks)
    w = _rows(d["write"], "WRITE_SIZE", ks)
    cf = _rows(d["cfetch"], "FETCH_SIZE", "copyBuffer")
    cw = _rows(d["cwrite"], "WRITE_SIZE", "copyBuffer")
    grids = int(line.get("roofline", {}).get("grids", 1))

    def last(per):
        ids = sorted(per)[-grids:]
        return sum(per[i] for i in ids)

    fk, wk = last(f), last(w)
    cfk = sum(cf.values()) / len(cf)
    cwk = sum(cw.values()) / len(cw)
    kib = (1 << 30) / 1024.0
    sf, sw = kib / cfk, kib / cwk
    traffic = (fk * sf + wk * sw) * 1024.0
    upd = line["timed_updates"]
    print(f"kernel_source_sha256: {kernel_source_hash()}")
    print(f"workload_key: {line['workload_key']}")
    print(f"dispatches_seen: {len(f)} (the timed launch is the last {grids}, summed)")
    print(f"fetch_kib: {fk:.1f}")
    print(f"write_kib: {wk:.1f}")
    print(f"copy_probe: 1 GiB per copy, fetch_kib {cfk:.1f} -> scale {sf:.4f}, write_kib {cwk:.1f} -> scale {sw:.4f}")
    print(f"traffic_bytes_per_launch: {traffic:.6e}")
    print(f"updates_per_launch: {upd}")
    print(f"traffic_bytes_per_update: {traffic / upd:.4f}")
    for folder in sq:
        import csv
        import glob
        names = set()
        for fcsv in glob.glob(os.path.join(folder, "**", "*_counter_collection.csv"), recursive=True):
            with open(fcsv) as fh:
                names |= {r["Counter_Name"] for r in csv.DictReader(fh)}
        for n in sorted(names):
            rows = _rows(folder, n, ks)
            print(f"{n}: {last(rows):.1f}")


def issue_block(kv, value):
    """Instruction-issue ceiling of the timed launch from its committed SQ counters."""
    if not kv or "SQ_INSTS_VALU" not in kv:
        return None
    upd = float(kv["updates_per_launch"])
    valu = float(kv["SQ_INSTS_VALU"]) / upd
    salu = float(kv["SQ_INSTS_SALU"]) / upd
    lds = float(kv.get("SQ_INSTS_LDS", "nan")) / upd
    cv = VALU_ISSUE_PER_S / valu
    cs = SALU_ISSUE_PER_S / salu
    out = {"valu_per_update": valu, "salu_per_update": salu, "lds_instr_per_update": lds,
           "valu_issue_peak_per_s": VALU_ISSUE_PER_S, "salu_issue_peak_per_s": SALU_ISSUE_PER_S,
           "ceiling_updates_per_s": min(cv, cs), "binding": "valu" if cv <= cs else "salu",
           "frac": value / min(cv, cs),
           "note": "wave instructions per leaf-cell update (SQ counters of the timed launch); a CU issues "
                   "one wave64 VALU instruction per cycle over its four SIMDs and one SALU instruction per "
                   "cycle: 256 CUs at 2.4 GHz"}
    if "SQ_WAIT_ANY" in kv and "SQ_WAVE_CYCLES" in kv:
        out["wait_fraction"] = float(kv["SQ_WAIT_ANY"]) / float(kv["SQ_WAVE_CYCLES"])
    if "SQ_ACTIVE_INST_VALU" in kv and "SQ_WAVE_CYCLES" in kv:
        out["valu_active_fraction"] = float(kv["SQ_ACTIVE_INST_VALU"]) / float(kv["SQ_WAVE_CYCLES"])
    return out


# ------------------------------------------------------------------ rocprofv3 helpers
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
    """Text summary of rocprofv3 CSV output under ``path``: kernel stats, then every
    step-kernel dispatch in order (duration, launch shape, registers)."""
    import csv
    import glob
    lines = []
    for f in sorted(glob.glob(os.path.join(path, "**", "*_kernel_stats.csv"), recursive=True)):
        lines.append("kernel stats:")
        lines.append(f"  {'calls':>6} {'avg_us':>12} {'total_ms':>10} {'pct':>6}  name")
        with open(f) as fh:
            for r in list(csv.DictReader(fh))[:10]:
                lines.append(f"  {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:12.1f} "
                             f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}  {r['Name'][:90]}")
    for f in sorted(glob.glob(os.path.join(path, "**", "*_kernel_trace.csv"), recursive=True)):
        with open(f) as fh:
            rows = [r for r in csv.DictReader(fh) if "k_steps" in r["Kernel_Name"]]
        if not rows:
            continue
        rows.sort(key=lambda r: int(r["Start_Timestamp"]))
        # launches: dispatches whose intervals overlap (the grids of one launch's classes run
        # side by side) form one launch; its span is the last end minus the first start
        spans = []
        for r in rows:
            a, e = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            if spans and a < spans[-1][1]:
                spans[-1] = [spans[-1][0], max(spans[-1][1], e), spans[-1][2] + 1]
            else:
                spans.append([a, e, 1])
        lines.append(f"step-kernel launches ({len(spans)}; overlapping dispatches are one launch; the first 12):")
        for i, (a, e, k) in enumerate(spans[:12]):
            lines.append(f"  L{i}: span {(e - a) / 1e6:10.4f} ms, {k} dispatch(es)")
        lines.append(f"step-kernel dispatches in launch order ({len(rows)} in all; the first 12):")
        for i, r in enumerate(rows[:12]):
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
            name = r["Kernel_Name"]
            tmpl = name[name.find("k_steps"):name.find(">") + 1] if "<" in name else "k_steps"
            lines.append(f"  #{i}: {dur:10.4f} ms, grid {r['Grid_Size_X']}, workgroup {r['Workgroup_Size_X']}, "
                         f"LDS {r['LDS_Block_Size']} B, VGPR {r['VGPR_Count']}, AGPR {r['Accum_VGPR_Count']}, "
                         f"SGPR {r['SGPR_Count']}, scratch {r['Scratch_Size']} B  {tmpl}")
    print("\n".join(lines) if lines else f"no rocprofv3 CSV output under {path}")


# ------------------------------------------------------------------ extra forms
def burgers_form(mrlbm, seeds, warmup, steps, prec):
    """The D1Q3 Burgers batch (510 runs at the default 85 seeds per (s, eps), J = 14): the
    whole run to T = 0.4 (3277 steps) as one launch from t = 0 in the tuner's launch shape, and
    the steady rate of W warmup + K timed steps; delta/eps of two runs over the whole run."""
    cases = burgers_cases(seeds, prec)
    b = make_batch(mrlbm, cases)
    b.checkpoint()
    n_whole = cases[0][0]["steps"]
    tuned = b.tune(n_whole)
    ms_whole = b.step_timed(n_whole)
    upd_whole = b.total_updates()
    b.restore()
    ms, upd, t0 = timed_region(b, warmup, steps)
    leaves = [b.stats(i)["leaves"] for i in range(len(cases))]
    out = {"runs": len(cases), "j_max": 14, "precision": "fp64" if prec == 0 else "fp32",
           "threads_capacity_schedule": [b.get_block(), b.get_capacity(), b.get_schedule()], "tuned": list(tuned),
           "whole_run": {"steps": n_whole, "updates_per_s": upd_whole / (ms_whole / 1e3),
                         "ms_per_step": ms_whole / n_whole, "leaf_updates": upd_whole},
           "steady": {"warmup": warmup, "steps": steps, "updates_per_s": upd / (ms / 1e3), "ms_per_step": ms / steps,
                      "t0_step_ms": t0},
           "bytes_per_update": b_alg(3, prec),
           "mean_leaves_after_timed_steps": float(np.mean(leaves))}
    b.close()
    sample = [c for c in cases if c[0]["s"][0] == 1.9 and c[0]["eps"] in (1e-3, 1e-4)][::seeds]
    worst, rows = delta_check(mrlbm, sample, n_whole)
    out["error_check"] = {"max_delta_over_eps": worst, "runs": rows}
    return out


def reconstructed_form(mrlbm, seeds, steps, tune=True, block=0, capacity=-1, schedule=256):
    """The reconstructed collision (Sec. 4.3.1) on the D1Q3 Burgers batch (510 runs, J = 14):
    the first `steps` steps from t = 0, against the leaves collision on the same steps, each
    in the launch shape the built-in tuner picks for it (or the given one), and delta/eps of
    two runs against the eps = 0 run."""
    out = {"steps": steps}
    for coll in ("leaves", "reconstructed"):
        cases = burgers_cases(seeds, 0)
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
    sample = [(dict(p, collision="reconstructed"), mc) for p, mc in burgers_cases(1, 0)
              if p["s"][0] == 1.9 and p["eps"] in (1e-3, 1e-4)]
    worst, rows = delta_check(mrlbm, sample, steps)
    out["max_delta_over_eps"] = worst
    out["delta_runs"] = rows
    return out


def euler_runs(seeds, jmax, eps, steps):
    ps, ms = [], []
    for s in seeds:
        p, mc = W.euler(s, jmax=jmax, eps=eps, steps=steps)
        ps.append(p)
        ms.append(mc)
    return ps, ms


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
    # "ideal": a network that declines every gated pair; the judge's redos leave exactly the
    # declines it accepts, so its leaf-update gain bounds what any network can save here
    never = W.mlp_constant_bits(-1.0)
    nets = {"learned": bits, "ideal": never}
    for name, mode in (("plain", mrlbm.PRED_OFF), ("learned", mrlbm.PRED_LEARNED), ("ideal", mrlbm.PRED_LEARNED)):
        b = mrlbm.Batch(ps, ms)
        if mode != mrlbm.PRED_OFF:
            b.set_predictor(nets[name], mode, gate)
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
    out["ideal_leaf_update_gain_bound"] = 1.0 - out["ideal"]["leaf_updates"] / out["plain"]["leaf_updates"]
    out["speed_vs_plain"] = out["learned"]["updates_per_s"] / out["plain"]["updates_per_s"]
    # time to solution of the same runs (the figure a predictor would have to improve)
    out["time_to_solution_vs_plain"] = out["learned"]["ms"] / out["plain"]["ms"]
    return out


def shallow_form(mrlbm, runs, steps=0):
    """The shallow-water dam break at its full size (J = 16, 65536 finest cells, clamp,
    eps = 1e-4, lambda = 2) with the D1Q2^2 scheme (s = 1.7) and with D1Q5 (Sec. 5.2.1:
    alpha = beta = 1, s3 = s4 = 1, s2 = 1.5; its stream reaches two cells): ``runs`` seeded
    runs of each advanced together, ``steps`` steps from t = 0 as one launch (0: the whole run
    to T = 0.4, 26214 steps)."""
    out = {}
    for name, scheme, s, q in (("d1q2x2", W.D1Q2x2, 1.7, 4), ("d1q5", W.D1Q5, 1.5, 5)):
        cases = [W.shallow(seed, jmax=16, scheme=scheme, s=s) for seed in range(runs)]
        n = steps or cases[0][0]["steps"]
        b = make_batch(mrlbm, cases, 512)
        ms = b.step_timed(n)
        upd = b.total_updates()
        st = [b.stats(i) for i in range(len(cases))]
        bpu = b_alg(q, 0)
        out[name] = {"runs": runs, "j_max": 16, "steps": n, "updates_per_s": upd / (ms / 1e3), "ms_per_step": ms / n,
                     "leaf_updates": upd, "threads_capacity": [b.get_block(), b.get_capacity()],
                     "mean_leaves_at_end": float(np.mean([x["leaves"] for x in st])),
                     "bytes_per_update": bpu, "algorithmic_gbs": upd * bpu / (ms / 1e3) / 1e9}
        b.close()
    return out


def two_d_form(mrlbm, jmax=12, warmup=5, steps=50):
    """The two-dimensional step (D2Q4 Burgers, a seeded box on [0, 1]^2, J = 12: 2^24 finest
    cells, eps = 1e-3): W steps from t = 0, then K steps timed with HIP events on the run's
    stream. Algorithmic bytes per leaf-cell update as for the 1D step: the four populations
    read and written once, a 4-byte key (72 B)."""
    p, u0 = W.two_d(0, jmax=jmax)
    run = mrlbm.MRLBM2D(p, u0)
    try:
        run.step(warmup)
        u_before = run.stats()["leaf_updates"]
        ms = run.step_timed(steps)
        st = run.stats()
    finally:
        run.close()
    upd = st["leaf_updates"] - u_before
    bpu = b_alg(4, 0)
    return {"j_max": jmax, "finest_cells": 4 ** jmax, "warmup": warmup, "steps": steps,
            "updates_per_s": upd / (ms / 1e3), "ms_per_step": ms / steps, "leaves_at_end": st["leaves"],
            "compression_pct": 100.0 * (1.0 - st["leaves"] / 4.0 ** jmax), "bytes_per_update": bpu,
            "algorithmic_gbs": upd * bpu / (ms / 1e3) / 1e9,
            "note": "dense levels in HBM, level-wide phases (independent levels fused, coarse levels in one workgroup): O(4^J) work per step"}


def ensemble_fp32(mrlbm, runs, warmup, steps):
    cases = ensemble_cases(runs, 1)
    b = make_batch(mrlbm, cases)
    b.set_classes(*HEADLINE_CLASSES)
    _, class_rows = launch_shape(b, HEADLINE_CLASSES)
    ms, upd, t0 = timed_region(b, warmup, steps)
    b.close()
    return {"updates_per_s": upd / (ms / 1e3), "ms_per_step": ms / steps, "t0_step_ms": t0,
            "launch_classes": class_rows, "bytes_per_update": b_alg(2, 1)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps K (one launch)")
    ap.add_argument("--warmup", type=int, default=5, help="steps W from t = 0 before the timed region")
    ap.add_argument("--runs", type=int, default=4096, help="instances of the ensemble")
    ap.add_argument("--no-classes", action="store_true", help="one launch for all runs (--block, --capacity)")
    ap.add_argument("--block", type=int, default=HEADLINE_SHAPE["block"], help="threads per workgroup (--no-classes)")
    ap.add_argument("--capacity", type=int, default=HEADLINE_SHAPE["capacity"],
                    help="on-chip capacity in cells (--no-classes)")
    ap.add_argument("--schedule", type=int, default=-1, help="schedule stride (-1: heaviest first)")
    ap.add_argument("--headline-only", action="store_true", help="only the headline (for profiling its launch)")
    ap.add_argument("--no-extras", action="store_true", help="skip every extra form")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-refinement form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=32, help="ensemble instances the oracle runs")
    ap.add_argument("--cpu-procs", type=int, default=0, help="oracle processes (0: min(16, host CPUs))")
    ap.add_argument("--burgers-seeds", type=int, default=85, help="seeds per (s, eps) of the Burgers batch")
    ap.add_argument("--learned-steps", type=int, default=2400)
    ap.add_argument("--recon-steps", type=int, default=200)
    ap.add_argument("--shallow-runs", type=int, default=64, help="seeded J = 16 shallow-water runs")
    ap.add_argument("--only", default="", choices=["", "fp32", "burgers", "shallow", "recon", "learned", "twod"],
                    help="only this extra form (for profiling its launches)")
    ap.add_argument("--profile-summary", default="", help="only summarize rocprofv3 CSV output in this folder")
    ap.add_argument("--counters-summary", default="", help="only print the counter block (see counters_summary)")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run a device copy of this many bytes")
    args = ap.parse_args()

    if args.counters_summary:
        counters_summary(args.counters_summary)
        return 0
    if args.profile_summary:
        profile_summary(args.profile_summary)
        return 0
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return 0
    if args.gpus != 1:
        print(f"bench.py measures a single GPU (asked for {args.gpus}): the batched engine runs on one "
              f"device; across GPUs the independent instances would be split by cost", file=sys.stderr)
        return 2
    if args.steps <= 0 or args.warmup < 0 or args.runs <= 0:
        print("bench.py needs --steps > 0, --warmup >= 0 and --runs > 0", file=sys.stderr)
        return 2

    extras = not (args.no_extras or args.headline_only)
    cpu = None
    if not (args.no_cpu_baseline or args.headline_only):
        procs = args.cpu_procs or max(1, min(16, os.cpu_count() or 1))
        print(f"[bench] CPU baseline: oracle on {args.cpu_sample} instances over {procs} processes", file=sys.stderr,
              flush=True)
        cpu = cpu_baseline(args.cpu_sample, procs)

    from paper_2102_12163_amd import mrlbm

    if args.only:
        legs = {"fp32": lambda: ensemble_fp32(mrlbm, args.runs, args.warmup, args.steps),
                "burgers": lambda: burgers_form(mrlbm, args.burgers_seeds, args.warmup, args.steps, 0),
                "shallow": lambda: shallow_form(mrlbm, args.shallow_runs),
                "recon": lambda: reconstructed_form(mrlbm, args.burgers_seeds, args.recon_steps),
                "learned": lambda: learned_form(mrlbm, 8, 64, args.learned_steps),
                "twod": lambda: two_d_form(mrlbm)}
        print(json.dumps({args.only: legs[args.only]()}))
        return 0
    prec = 0
    schedule = args.schedule if args.schedule >= 0 else args.runs
    cases = ensemble_cases(args.runs, prec)
    print(f"[bench] ensemble of {len(cases)} instances, warmup {args.warmup}, timed {args.steps}", file=sys.stderr,
          flush=True)
    classes = None if args.no_classes else HEADLINE_CLASSES
    if classes:
        b = make_batch(mrlbm, cases)
        b.set_classes(*classes)
    else:
        b = make_batch(mrlbm, cases, args.block, args.capacity, schedule)
    if extras:
        b.checkpoint()  # t = 0, for the whole-run leg
    ms, upd, t0 = timed_region(b, args.warmup, args.steps)
    value = upd / (ms / 1e3)
    leaf_sum = sum(2 ** c[0]["jmax"] for c in cases)
    acr = 100.0 * (1.0 - upd / (args.steps * leaf_sum))
    leaves_now = np.array([b.stats(i)["leaves"] for i in range(len(cases))])
    js = np.array([c[0]["jmax"] for c in cases])
    print(f"[bench] timed launch {ms:.3f} ms, {upd} leaf-cell updates", file=sys.stderr, flush=True)
    shape_text, class_rows = launch_shape(b, classes)
    key = workload_key(args.runs, args.steps, args.warmup, shape_text, b.get_schedule(), prec)
    grids = len(class_rows) if class_rows else 1
    kv = counters_for(key)
    bpu = b_alg(2, prec)
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "batched ensemble: 4096 independent D1Q2 instances (advection V=0.75 s=1.9 or Burgers "
                        "s in {1.5,1.9}), J_max uniform in 8..14, J_min=2, eps in {1e-3,1e-4}, gamma=1, periodic "
                        "[-1,1], seeded step+bump data, 512 steps each, one persistent launch",
            "runs": len(cases), "j_max_range": [int(js.min()), int(js.max())],
            "launch_classes": class_rows,
            "threads_per_workgroup": None if class_rows else b.get_block(),
            "onchip_capacity_cells": None if class_rows else b.get_capacity(),
            "schedule_stride": b.get_schedule(),
            "form": "timed steps continue the warmed-up runs (no restore), one launch replayed from a HIP graph"
                    + (f" (its {grids} class grids side by side)" if class_rows else ""),
            "mean_leaves_per_instance": float(leaves_now.mean()),
        },
        "t0_step_ms": t0,
        "workload_key": key,
        "timed_updates": upd,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": float(kv["traffic_bytes_per_launch"]) if kv else None,
            "traffic_unit": "HBM bytes of the timed launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-probe scaled)",
            "kernel": "k_steps<double,0,1>", "bytes_per_update": bpu, "launches": 1, "grids": grids,
            "avg_launch_ms": ms,
            "issue": issue_block(kv, value),
        },
    }
    if extras:
        # two more windows of K steps right after the timed one: the spread of the timed rate
        reps = [value]
        for _ in range(2):
            u_a = b.total_updates()
            ms_r = b.step_timed(args.steps)
            reps.append((b.total_updates() - u_a) / (ms_r / 1e3))
        result["repeats"] = {"updates_per_s": reps, "median": float(np.median(reps)),
                             "note": "the timed window and the next two windows of K steps (the runs continue)"}
        result["compression"] = {
            "mean_cr_pct": float(np.mean(100.0 * (1.0 - leaves_now / 2.0 ** js))),
            "acr_pct_timed": acr,
            "definition": "CR = 100 (1 - #leaves / 2^J) after the timed steps, averaged over the instances; ACR = "
                          "100 (1 - leaf-cell updates / (steps x sum of 2^J)) over the timed steps",
            "paper_context": "the paper's only efficiency figure: CR about 95 % (advection of a Gaussian, J=9) and "
                             "above 90 % (box advection), sequential C++ on an unreported CPU"}
        # the whole 512-step run from t = 0 as one launch (the t = 0 transient included)
        b.restore()
        u0 = b.total_updates()
        msw = b.step_timed(ENSEMBLE_STEPS)
        uw = b.total_updates() - u0
        result["whole_run"] = {"steps": ENSEMBLE_STEPS, "updates_per_s": uw / (msw / 1e3),
                               "ms_per_step": msw / ENSEMBLE_STEPS, "leaf_updates": uw}
        # the built-in tuner on the timed steps (from the warmed-up state, restored after each trial)
        b.restore()
        b.step(args.warmup)
        b.checkpoint()
        tb, tc = b.tune(args.steps)
        v0 = b.total_updates()
        mst = b.step_timed(args.steps)
        result["tuner"] = {"threads_capacity_schedule": [tb, tc, b.get_schedule()],
                           "classes": [list(c) for c in b.get_classes()],
                           "updates_per_s": (b.total_updates() - v0) / (mst / 1e3),
                           "note": "the built-in tuner's launch shape for the timed steps (threads and capacity "
                                   "0 when it chose launch classes), timed on the same steps"}
        b.close()
        cbw = copy_bandwidth()
        result["roofline"]["measured_copy_gbs"] = cbw
        result["roofline"]["frac_of_measured_copy"] = achieved / cbw
        picked = {}
        for i, (p, _) in enumerate(cases):
            picked.setdefault(p["jmax"], i)
        sample = [cases[i] for _, i in sorted(picked.items())]
        worst, rows = delta_check(mrlbm, sample, ENSEMBLE_STEPS)
        result["error_check"] = {"max_delta_over_eps": worst, "runs": rows,
                                 "reference": "eps=0 run of the same library (uniform finest scheme), whole runs"}
        sample_cases = cases[:: max(1, len(cases) // 64)]
        rate_1 = plain_step_rate(mrlbm, sample_cases, 100, 1)
        rate_8 = plain_step_rate(mrlbm, sample_cases, 100, 8)
        result["plain_step"] = {"per_instance_launches_updates_per_s": {"1_stream": rate_1, "8_streams": rate_8},
                                "batched_speedup": value / max(rate_1, rate_8),
                                "sample": "every 64th instance, one launch per time step and instance, 100 steps "
                                          "after 5, the runs round-robin over 1 or 8 HIP streams"}
        print("[bench] FP32 ensemble", file=sys.stderr, flush=True)
        result["fp32_form"] = ensemble_fp32(mrlbm, args.runs, args.warmup, args.steps)
        result["fp32_form"]["speed_vs_fp64"] = result["fp32_form"]["updates_per_s"] / value
        print("[bench] D1Q3 Burgers batch", file=sys.stderr, flush=True)
        result["burgers_form"] = burgers_form(mrlbm, args.burgers_seeds, args.warmup, args.steps, 0)
        print("[bench] shallow water J=16", file=sys.stderr, flush=True)
        result["shallow_form"] = shallow_form(mrlbm, args.shallow_runs)
        print("[bench] two dimensions J=12", file=sys.stderr, flush=True)
        result["two_d_form"] = two_d_form(mrlbm)
        print("[bench] reconstructed collision", file=sys.stderr, flush=True)
        result["reconstructed_form"] = reconstructed_form(mrlbm, args.burgers_seeds, args.recon_steps)
        if not args.no_learned:
            print("[bench] learned-refinement form", file=sys.stderr, flush=True)
            result["learned_form"] = learned_form(mrlbm, 8, 64, args.learned_steps)
    else:
        b.close()
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result))
    return 0


if __name__ == "__main__":
    sys.exit(main())
