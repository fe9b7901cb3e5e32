"""Host-only checks of the C ABI: the library loads, exports every entry point that
include/mrlbm.h declares, and validates parameters on the host (no device needed)."""

import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2102_12163_amd import mrlbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "mrlbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mrlbm(?:2d)?_\w+)\s*\(", txt)))


def test_header_and_binding_agree():
    names = header_functions()
    assert len(names) >= 20
    assert set(names) == set(mrlbm.SIGNATURES), set(names) ^ set(mrlbm.SIGNATURES)


def test_library_exports_every_declared_symbol():
    L = mrlbm.lib()
    for name in header_functions():
        assert hasattr(L, name), name


def test_struct_layout():
    """The binding's structs against the header compiled by the host C compiler: size and the
    offset of every field."""
    import ctypes
    import shutil
    import subprocess
    import tempfile
    structs = {"mrlbm_params": (mrlbm.Params, {"lam": "lambda"}), "mrlbm_stats_t": (mrlbm.Stats, {}),
               "mrlbm2d_params": (mrlbm.Params2D, {"lam": "lambda"})}
    cc = shutil.which("gcc") or shutil.which("cc")
    assert cc, "a host C compiler is needed"
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mrlbm.h"', "int main(void) {"]
    for name, (cls, ren) in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {ren.get(f, f)}));')
    lines += ["return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        with open(src, "w") as fh:
            fh.write("\n".join(lines))
        exe = os.path.join(d, "layout")
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), "-o", exe, src], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, (cls, _) in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)


def good():
    p, _ = W.burgers(0, jmax=8)
    return p


@pytest.mark.parametrize("field,value", [
    ("abi_version", 99), ("scheme", 7), ("physics", 9), ("bc", 5), ("precision", 3), ("lam", 0.0),
    ("lam", -1.0), ("lam", float("inf")), ("s", [0.0]), ("s", [2.5]), ("s", [1.0, 1.0, 1.0]),
    ("x_max", -2.0), ("jmin", -1), ("jmin", 9), ("gamma", 0), ("gamma", 4), ("mu_bar", -1), ("eps", -1e-3),
    ("eps", float("nan")), ("flags", 2), ("flags", 0x80000000),
])
def test_validation_rejects(field, value):
    p = good()
    p[field] = value
    assert mrlbm.validate(p) == mrlbm.EINVAL


def test_validation_reconstructed_collision_flag():
    """Bit 0 of flags selects the reconstructed collision, which runs with gamma = 1."""
    p = good()
    p["collision"] = "reconstructed"
    assert mrlbm.make_params(p).flags == mrlbm.FLAG_RECONSTRUCTED_COLLISION
    assert mrlbm.validate(p) == mrlbm.OK
    p["gamma"] = 2
    p["jmin"] = 3
    assert mrlbm.validate(p) == mrlbm.EINVAL


def test_validation_coarsest_level_zero():
    """J_min = 0 (a one-cell coarsest level) is accepted under clamp and refused when periodic."""
    p = good()
    p["jmin"], p["bc"] = 0, 1
    assert mrlbm.validate(p) == mrlbm.OK
    p["bc"] = 0
    assert mrlbm.validate(p) == mrlbm.EINVAL


def test_validation_rejects_small_periodic_coarse_level():
    p = good()
    p["gamma"] = 2
    p["jmin"] = 2   # 4 cells < 2 gamma + 1
    assert mrlbm.validate(p) == mrlbm.EINVAL
    p["jmin"] = 3
    assert mrlbm.validate(p) == mrlbm.OK


def test_level_limits_match_the_header():
    """MAX_J and ONCHIP_MAX_J of the binding are the header's; J above the on-chip limit is
    accepted, the reconstructed collision there is not."""
    import re
    from pathlib import Path
    hdr = (Path(__file__).resolve().parents[1] / "include" / "mrlbm.h").read_text()
    assert int(re.search(r"#define MRLBM_MAX_J (\d+)", hdr).group(1)) == mrlbm.MAX_J
    assert int(re.search(r"#define MRLBM_ONCHIP_MAX_J (\d+)", hdr).group(1)) == mrlbm.ONCHIP_MAX_J
    p = good()
    p["jmax"] = mrlbm.MAX_J
    assert mrlbm.validate(p) == mrlbm.OK
    p["collision"] = "reconstructed"
    assert mrlbm.validate(p) == mrlbm.EINVAL
    p["jmax"] = mrlbm.ONCHIP_MAX_J
    assert mrlbm.validate(p) == mrlbm.OK


def test_validation_capacity_limit():
    p = good()
    p["jmax"] = mrlbm.MAX_J + 1
    assert mrlbm.validate(p) == mrlbm.ECAPACITY


def test_validation_physics_parameters():
    p, _ = W.shallow(0, jmax=8)
    p["phys"] = [0.0, 0.0, 1.4, 0.9]
    assert mrlbm.validate(p) == mrlbm.EINVAL
    p, _ = W.euler(0, jmax=8)
    p["phys"] = [0.0, 1.0, 1.0, 0.9]
    assert mrlbm.validate(p) == mrlbm.EINVAL


def test_validation_accepts_every_workload():
    for p, _ in (W.advection(0), W.burgers(0), W.shallow(0), W.euler(0), W.batch_instance(0),
                 W.burgers(0, scheme=W.D1Q3), W.shallow(0, scheme=W.D1Q5)):
        assert mrlbm.validate(p) == mrlbm.OK


def test_create_rejects_before_touching_the_device():
    p = good()
    p["eps"] = -1.0
    with pytest.raises(mrlbm.MRLBMError) as e:
        mrlbm.MRLBM(p, np.zeros((1, 2 ** p["jmax"])))
    assert e.value.code == mrlbm.EINVAL
    p = good()
    bad = np.zeros((1, 2 ** p["jmax"]))
    bad[0, 3] = np.nan
    with pytest.raises(mrlbm.MRLBMError) as e:
        mrlbm.MRLBM(p, bad)
    assert e.value.code == mrlbm.EINVAL


def test_binding_checks_the_initial_moment_shape():
    """The C side reads q_cons 2^J doubles from the initial-moment pointer: the binding refuses
    an array of another shape before the call (single runs and batches)."""
    p = good()
    n = 2 ** p["jmax"]
    for bad in (np.zeros((1, n - 1)), np.zeros((2, n)), np.zeros((1, 2 * n))):
        with pytest.raises(ValueError):
            mrlbm.MRLBM(p, bad)
        with pytest.raises(ValueError):
            mrlbm.Batch([p, p], [np.zeros((1, n)), bad])
    ps, _ = W.shallow(0, jmax=6)
    with pytest.raises(ValueError):
        mrlbm.MRLBM(ps, np.zeros((1, 64)))  # shallow water has two conserved moments
    with pytest.raises(ValueError):
        mrlbm.Batch([p], [])


def test_batch_rejects_mixed_schemes():
    p1 = good()
    p2, _ = W.advection(0, jmax=8)
    with pytest.raises(mrlbm.MRLBMError) as e:
        mrlbm.Batch([p1, p2], [np.zeros((1, 256)), np.zeros((1, 256))])
    assert e.value.code == mrlbm.EINVAL


def test_batch_calls_reject_null_handles():
    """Every batch call checks its handle and arguments on the host before any device work."""
    L = mrlbm.lib()
    assert L.mrlbm_batch_checkpoint(None) == mrlbm.EINVAL
    assert L.mrlbm_batch_restore(None) == mrlbm.EINVAL
    assert L.mrlbm_batch_set_launch_steps(None, 10) == mrlbm.EINVAL
    assert L.mrlbm_batch_set_schedule(None, 0) == mrlbm.EINVAL
    assert L.mrlbm_batch_tune(None, 10, None, None) == mrlbm.EINVAL
    assert L.mrlbm_batch_step(None, 1) == mrlbm.EINVAL


def test_bench_refuses_several_gpus_and_empty_regions():
    """bench.py measures one GPU: N > 1 and an empty timed region exit with status 2 and a
    message, before touching the library."""
    import subprocess
    import sys as _sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for args in (["--gpus", "2"], ["--steps", "0"]):
        r = subprocess.run([_sys.executable, os.path.join(root, "bench.py")] + args, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 2, (args, r.returncode, r.stderr)
        assert "bench.py" in r.stderr


def test_profile_summaries_match_the_kernel_sources():
    """The committed counter summary of the headline launch names the sha256 of the step-kernel
    sources and the launch (workload key) it was taken on; bench.py reports its traffic and
    issue figures only while both match, and the key is the one of the default command."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    h = bench.kernel_source_hash()
    assert len(h) == 64
    kv = bench.read_counters()
    assert kv, "profiles/ holds no counter summary of the headline launch"
    default_key = bench.workload_key(4096, 20, 5, bench.classes_text(bench.HEADLINE_CLASSES), 4096, 0)
    assert kv["workload_key"] == default_key
    got = bench.counters_for(default_key)
    assert (kv["kernel_source_sha256"] == h) == (got is not None)
    assert bench.counters_for(default_key.replace("steps=20", "steps=21")) is None
    if got is not None:
        iss = bench.issue_block(got, 1.0e9)
        assert iss["valu_per_update"] > 0 and iss["ceiling_updates_per_s"] > 0
        assert float(got["traffic_bytes_per_launch"]) > 0


def _bench_module():
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod2", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    return bench


def test_counter_block_sums_the_timed_launchs_class_dispatches(tmp_path, capsys):
    """bench.py --counters-summary on synthetic rocprofv3 output: the timed launch is the last
    `grids` step-kernel dispatches, summed; FETCH_SIZE and WRITE_SIZE are scaled by what the
    copy probe reads for 1 GiB (here half and all of it: scales 2 and 1)."""
    import csv
    import json as _json
    bench = _bench_module()

    def write(folder, counter, kernel, per_dispatch):
        os.makedirs(folder, exist_ok=True)
        with open(os.path.join(folder, "run_counter_collection.csv"), "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for did, val in per_dispatch.items():
                # two rows per dispatch (two XCD-level entries) that must be summed
                for half in (0.25, 0.75):
                    w.writerow({"Dispatch_Id": did, "Kernel_Name": kernel, "Counter_Name": counter,
                                "Counter_Value": val * half})

    ks = "void mrl::k_steps<double, 0, 1, false, false>(...)"
    # six dispatches: three launches of two class grids; the last two are the timed launch
    write(str(tmp_path / "f"), "FETCH_SIZE", ks, {1: 5.0, 2: 6.0, 3: 7.0, 4: 8.0, 5: 100.0, 6: 300.0})
    write(str(tmp_path / "w"), "WRITE_SIZE", ks, {1: 1.0, 2: 1.0, 3: 1.0, 4: 1.0, 5: 1000.0, 6: 24.0})
    kib = (1 << 30) / 1024.0
    write(str(tmp_path / "cf"), "FETCH_SIZE", "__amd_rocclr_copyBuffer", {1: kib / 2, 2: kib / 2})
    write(str(tmp_path / "cw"), "WRITE_SIZE", "__amd_rocclr_copyBuffer", {1: kib, 2: kib})
    write(str(tmp_path / "sq"), "SQ_INSTS_VALU", ks, {1: 1.0, 2: 2.0, 3: 3.0, 4: 4.0, 5: 50.0, 6: 70.0})
    line = {"timed_updates": 1000, "workload_key": "k", "roofline": {"grids": 2}}
    with open(tmp_path / "line.json", "w") as fh:
        fh.write("[bench] noise\n" + _json.dumps(line) + "\n")
    spec = ",".join([f"fetch={tmp_path / 'f'}", f"write={tmp_path / 'w'}", f"cfetch={tmp_path / 'cf'}",
                     f"cwrite={tmp_path / 'cw'}", f"sq={tmp_path / 'sq'}", f"json={tmp_path / 'line.json'}"])
    bench.counters_summary(spec)
    out = dict(l.split(":", 1) for l in capsys.readouterr().out.splitlines() if ":" in l)
    assert float(out["fetch_kib"]) == 400.0 and float(out["write_kib"]) == 1024.0
    want = (400.0 * 2.0 + 1024.0 * 1.0) * 1024.0
    assert abs(float(out["traffic_bytes_per_launch"]) - want) <= 1e-6 * want
    assert abs(float(out["traffic_bytes_per_update"]) - want / 1000) <= 1e-6 * want
    assert float(out["SQ_INSTS_VALU"]) == 120.0


def test_profile_summary_groups_overlapping_dispatches(tmp_path, capsys):
    """The kernel-trace summary counts dispatches whose intervals overlap as one launch and
    gives its span (last end minus first start)."""
    import csv
    bench = _bench_module()
    fields = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Workgroup_Size_X", "LDS_Block_Size",
              "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Scratch_Size"]
    ks = "void mrl::k_steps<double, 0, 1, false, false>(...)"
    spans = [(0, 400), (100, 500), (1000, 1200), (1100, 1300), (2000, 4000), (2100, 5000)]
    with open(tmp_path / "run_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for a, e in spans + [(6000, 6001)]:
            w.writerow({"Kernel_Name": ks if a < 6000 else "other", "Start_Timestamp": a * 1000, "End_Timestamp": e * 1000,
                        "Grid_Size_X": 256, "Workgroup_Size_X": 128, "LDS_Block_Size": 512, "VGPR_Count": 52,
                        "Accum_VGPR_Count": 0, "SGPR_Count": 112, "Scratch_Size": 0})
    bench.profile_summary(str(tmp_path))
    text = capsys.readouterr().out
    assert "step-kernel launches (3;" in text
    assert "L0: span     0.5000 ms, 2 dispatch(es)" in text
    assert "L2: span     3.0000 ms, 2 dispatch(es)" in text
