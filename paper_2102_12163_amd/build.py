"""Build step of the HIP library (hipcc, gfx950).

The kernels are compiled once per (storage type, scheme) from ``csrc/instances.hip``, the
host side from ``csrc/mrlbm.hip``, the network's kernels from ``csrc/mlp.hip`` and the
two-dimensional step from ``csrc/mrlbm2d.hip``, as separate objects compiled in parallel,
then linked into ``libmrlbm.so`` next to this file.
"""

import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmrlbm.so")

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # the detail/threshold arithmetic must not be contracted into FMAs: leaf sets are
    # compared bit for bit with the FP64 checks, which round every operation
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build_library(verbose=False, jobs=None):
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    tmp = tempfile.mkdtemp(prefix="mrlbm_build_")
    units = [("host", os.path.join(CSRC, "mrlbm.hip"), [])]
    for t in ("double", "float"):
        for s in range(5):
            lrn = "1" if t == "double" else "0"
            units.append((f"k_{t}_{s}", os.path.join(CSRC, "instances.hip"),
                          [f"-DMRL_T={t}", f"-DMRL_S={s}", f"-DMRL_LRN={lrn}"]))
    units.append(("mlp", os.path.join(CSRC, "mlp.hip"), []))
    units.append(("md2", os.path.join(CSRC, "mrlbm2d.hip"), []))
    jobs = jobs or min(len(units), os.cpu_count() or 4)
    procs, objs, failed = [], [], []
    pending = list(units)
    while pending or procs:
        while pending and len(procs) < jobs:
            name, src, defs = pending.pop(0)
            obj = os.path.join(tmp, name + ".o")
            cmd = [_hipcc()] + HIPCC_FLAGS + defs + inc + ["-c", "-o", obj, src]
            procs.append((name, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        name, obj, p = procs.pop(0)
        out, err = p.communicate()
        if p.returncode != 0:
            failed.append(f"[{name}]\n{out}{err}")
        objs.append(obj)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n".join(failed))
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", OUT + ".tmp"] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(OUT + ".tmp", OUT)
    for o in objs:
        if os.path.exists(o):
            os.remove(o)
    os.rmdir(tmp)
    if verbose:
        print("built", OUT)
    return OUT
