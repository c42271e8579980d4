"""Compile the HIP library libmjh.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmjh.so")
SOURCES = ["mjh_api.cpp", "mjh_kernels.hip", "mjh_adjoint.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -packed-fp32-ops: keep the compiler from emitting packed FP32 instructions.
# -fno-hip-fp32-correctly-rounded-divide-sqrt: FP32 division and square root within a
# few ulp (v_rcp/v_sqrt based) instead of the correctly rounded ~10-instruction
# sequences; pivots and line-search ratios sit on per-column dependency chains.
# -disable-machine-licm: the machine-level loop-invariant motion hoisted constants and
# address arithmetic out of the per-world step loop and held them in VGPRs for the
# whole launch; the step kernel then spilled 22 VGPRs (100 B/lane of scratch).  Without
# it the constants are rematerialised where used: 2 VGPR spills, +3 % world-steps/s.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fno-hip-fp32-correctly-rounded-divide-sqrt",
         "-mllvm", "-disable-machine-licm",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source to an object in parallel, then link libmjh.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        usage = ["-Rpass-analysis=kernel-resource-usage"] if src.endswith(".hip") else []
        cmd = [HIPCC, *FLAGS, *lang, *usage, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT, text=True)))
    failed = []
    usage = []
    for src, p in procs:
        out, _ = p.communicate()
        usage += [l for l in out.splitlines() if "[-Rpass-analysis=kernel-resource-usage]" in l]
        lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l
                 and "is not a recognized feature" not in l
                 and "[-Rpass-analysis=kernel-resource-usage]" not in l]
        if p.returncode != 0:
            failed.append(src)
            print("\n".join(lines), file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("HIP compile failed: " + ", ".join(failed))
    write_resource_usage(usage, os.path.join(objdir, "resource_usage.txt"))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def write_resource_usage(remarks, path):
    """One line per kernel from the compiler's resource-usage remarks: name, then
    key=value pairs (VGPRs, ScratchSize, spills, occupancy)."""
    rows, cur = [], None
    for line in remarks:
        m = re.search(r"remark:\s+(.*?):\s+(\S+)\s+\[-Rpass", line)
        if not m:
            continue
        key, val = m.group(1).strip(), m.group(2)
        if key == "Function Name":
            cur = [val]
            rows.append(cur)
        elif cur is not None:
            cur.append(key.replace(" ", "").replace("[bytes/lane]", "").replace(
                "[waves/SIMD]", "") + "=" + val)
    with open(path, "w") as f:
        for r in rows:
            f.write(" ".join(r) + "\n")


def resource_usage(path=os.path.join(HERE, "_build", "resource_usage.txt")):
    """{kernel symbol: {key: int}} from the last build, or None before a build."""
    if not os.path.exists(path):
        return None
    out = {}
    with open(path) as f:
        for line in f:
            name, *kv = line.split()
            out[name] = {k: int(v) for k, v in (x.split("=") for x in kv) if v.lstrip("-").isdigit()}
    return out


if __name__ == "__main__":
    print(build(verbose=True))
