"""Build librr.so (the HIP library) in-tree for gfx950.

Usage: python -m paper_1011_3583_amd.build   (or call build()).
"""
from __future__ import annotations

import glob
import json
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librr.so")
OBJ = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
    # Kernels take their 672-byte TileArgs by value.  The front end copies such
    # an argument into private memory and InstCombine folds the copy back into
    # kernarg loads only while the copy has fewer users than this limit (300 by
    # default); past it every wave spills the whole struct to scratch.
    "-mllvm", "-instcombine-max-copied-from-constant-users=4096",
]
# Per-kernel register / scratch report written next to the objects.
RESOURCES = "kernel_resources.json"


_REMARK = re.compile(r"remark:\s+(.*?):\s+(\S+) \[-Rpass-analysis=kernel-resource-usage\]")


def parse_resource_remarks(text: str) -> dict:
    """Collect the compiler's kernel-resource-usage remarks into
    {kernel symbol: {"VGPRs": .., "ScratchSize [bytes/lane]": .., ...}}."""
    out, cur = {}, None
    for line in text.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1).strip(), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[key] = int(val) if val.isdigit() else val
    return out


def _compile(src: str, objdir: str = OBJ, defines=()) -> tuple:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    extra = ["-Rpass-analysis=kernel-resource-usage"] if src.endswith(".hip") else []
    cmd = [HIPCC, *COMMON, *extra, *[f"-D{d}" for d in defines], "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    res = parse_resource_remarks(r.stderr)
    # keep warnings visible but terse
    msg = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l
                    and not l.lstrip().startswith(("|", "^")) and not re.match(r"\s*\d+ \|", l) and l.strip())
    if msg:
        sys.stderr.write(msg + "\n")
    return obj, res


def build(verbose: bool = False, out: str = OUT, defines=()) -> str:
    """Compile every source under csrc/ and link librr.so (``out``); ``defines``
    are extra -D macros (used to build alternative variants side by side)."""
    objdir = OBJ if out == OUT else out + ".objs"
    os.makedirs(objdir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        done = list(ex.map(lambda s: _compile(s, objdir, defines), srcs))
    objs = [o for o, _ in done]
    resources = {}
    for _, res in done:
        resources.update(res)
    with open(os.path.join(objdir, RESOURCES), "w") as f:
        json.dump(resources, f, indent=1, sort_keys=True)
    spilled = sorted(k for k, v in resources.items() if v.get("ScratchSize [bytes/lane]", 0))
    if spilled:
        sys.stderr.write("warning: kernels using scratch: " + ", ".join(spilled) + "\n")
    tmp = out + f".tmp{os.getpid()}"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of librr.so failed")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True)
