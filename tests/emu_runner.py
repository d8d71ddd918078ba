"""Drive the CPU emulator of librr's kernel bodies (tests/emu/rr_emu.cpp).

The emulator is built with g++ under AddressSanitizer/UBSan from the library's
own planner and per-thread kernel code; it is test infrastructure that lets the
CPU suite check kernel index arithmetic and bounds without a GPU.
"""
import os
import subprocess
import tempfile

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU_SRC = os.path.join(ROOT, "tests", "emu", "rr_emu.cpp")
EMU_BIN = os.path.join(ROOT, "tests", "emu", "_build", "rr_emu")
DEPS = [EMU_SRC,
        os.path.join(ROOT, "paper_1011_3583_amd", "csrc", "rr_batch.hpp"),
        os.path.join(ROOT, "paper_1011_3583_amd", "csrc", "rr_batch_plan.cpp"),
        os.path.join(ROOT, "paper_1011_3583_amd", "csrc", "rr_device.hpp"),
        os.path.join(ROOT, "paper_1011_3583_amd", "csrc", "rr_plan.hpp"),
        os.path.join(ROOT, "paper_1011_3583_amd", "csrc", "rr_plan.cpp"),
        os.path.join(ROOT, "include", "rr.h")]


def build():
    if os.path.exists(EMU_BIN) and all(os.path.getmtime(EMU_BIN) >= os.path.getmtime(d) for d in DEPS):
        return EMU_BIN
    os.makedirs(os.path.dirname(EMU_BIN), exist_ok=True)
    tmp = EMU_BIN + f".tmp{os.getpid()}"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall", "-Wno-unknown-pragmas",
           "-o", tmp, EMU_SRC, os.path.join(ROOT, "paper_1011_3583_amd", "csrc", "rr_plan.cpp"),
           os.path.join(ROOT, "paper_1011_3583_amd", "csrc", "rr_batch_plan.cpp")]
    subprocess.run(cmd, check=True)
    os.replace(tmp, EMU_BIN)
    return EMU_BIN


def run(jobs):
    """Run jobs through the emulator.  Each job is a dict:
       permute:     op, dims, perm, esize, input (uint8), src_off, dst_off, in_rb, out_rb, order,
                    max_g, ragged, xcd (None: the planner's choice), umt, diag,
                    fill (None: the planner's choice), weave
       reorder:     op, dims, base, range, order, esize, input (uint8), src_off, dst_off, umt, max_g
       gather:      op, src_count, esize, input (uint8), idx (int64) or start/stride/count, src_off, dst_off
       interlace:   op, n, count, esize, planes (list of uint8), off, in_rb, out_rb, weave
       deinterlace: op, n, count, esize, input (uint8), off, in_rb, out_rb, weave
    Returns a list of (status_line, output) with output a uint8 array or list of planes."""
    exe = build()
    with tempfile.TemporaryDirectory() as td:
        lines = []
        for i, j in enumerate(jobs):
            inf = os.path.join(td, f"in{i}")
            outf = os.path.join(td, f"out{i}")
            rb = f"{j.get('in_rb', 0)} {j.get('out_rb', 0)}"
            if j["op"] == "permute":
                j["input"].tofile(inf)
                nd = len(j["dims"])
                lines.append(" ".join(["permute", str(nd), *map(str, j["dims"]), *map(str, j["perm"]),
                                       str(j["esize"]), str(j.get("src_off", 0)), str(j.get("dst_off", 0)),
                                       rb, str(j.get("order", -1)), str(j.get("max_g", 0)),
                                       str(int(j.get("ragged", False))),
                                       str(-1 if j.get("xcd") is None else int(j["xcd"])),
                                       str(int(j.get("umt", 0))), str(-1 if j.get("diag") is None else int(j["diag"])),
                                       str(-1 if j.get("fill") is None else int(j["fill"])),
                                       str(int(j.get("weave", True))), inf, outf]))
            elif j["op"] == "stencil":
                np.ascontiguousarray(j["grid"], dtype=np.float32).tofile(inf)
                w = [repr(float(v)) for v in np.asarray(j["weights"], dtype=np.float32).reshape(-1)]
                lines.append(" ".join(map(str, ["stencil", j["grid"].shape[0], j["grid"].shape[1], j["radius"],
                                                 j.get("shape", 0), len(w), *w, inf, outf])))
            elif j["op"] == "gather":
                j["input"].tofile(inf)
                idxf = os.path.join(td, f"idx{i}")
                indexed = "idx" in j
                if indexed:
                    np.asarray(j["idx"], dtype=np.int64).tofile(idxf)
                count = len(j["idx"]) if indexed else j["count"]
                lines.append(" ".join(map(str, ["gather", j["src_count"], count, j["esize"], int(indexed),
                                                 j.get("start", 0), j.get("stride", 0), j.get("src_off", 0),
                                                 j.get("dst_off", 0), inf, idxf, outf])))
            elif j["op"] == "reorder":
                j["input"].tofile(inf)
                nd = len(j["dims"])
                lines.append(" ".join(["reorder", str(nd), *map(str, j["dims"]), *map(str, j["base"]),
                                       *map(str, j["range"]), str(len(j["order"])), *map(str, j["order"]),
                                       str(j["esize"]), str(j.get("src_off", 0)), str(j.get("dst_off", 0)),
                                       str(int(j.get("umt", 0))), str(j.get("max_g", 0)), inf, outf]))
            elif j["op"] == "interlace":
                np.concatenate(j["planes"]).tofile(inf)
                lines.append(f"interlace {j['n']} {j['count']} {j['esize']} {j.get('off', 0)} {rb} "
                             f"{int(j.get('weave', True))} {inf} {outf}")
            elif j["op"] == "batched":
                lines.append(f"batched {len(j['jobs'])} {rb} {j.get('order', -1)} {j.get('chunk', 0)} "
                             f"{j.get('max_g', 0)} {int(j.get('ragged', False))} {int(j.get('umt', 0))}")
                for k, sub in enumerate(j["jobs"]):
                    sf, of = os.path.join(td, f"b{i}_{k}"), os.path.join(td, f"bo{i}_{k}")
                    sub["input"].tofile(sf)
                    lines.append(" ".join(["job", str(len(sub["dims"])), *map(str, sub["dims"]),
                                           *map(str, sub["perm"]), str(sub["esize"]), sf, of]))
            else:
                j["input"].tofile(inf)
                lines.append(f"deinterlace {j['n']} {j['count']} {j['esize']} {j.get('off', 0)} {rb} "
                             f"{int(j.get('weave', True))} {inf} {outf}")
        man = os.path.join(td, "manifest")
        with open(man, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe, man], capture_output=True, text=True, env=env)
        if r.returncode != 0:
            raise AssertionError(f"emulator failed (rc={r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}")
        status = r.stdout.strip().splitlines()
        assert len(status) == len(jobs), r.stdout
        out = []
        for i, (j, s) in enumerate(zip(jobs, status)):
            outf = os.path.join(td, f"out{i}")
            if not s.startswith("ok"):
                out.append((s, None))
                continue
            if j["op"] == "batched":
                out.append((s, [np.fromfile(os.path.join(td, f"bo{i}_{k}"), dtype=np.uint8)
                                for k in range(len(j["jobs"]))]))
                continue
            if j["op"] == "stencil":
                out.append((s, np.fromfile(outf, dtype=np.float32).reshape(j["grid"].shape)))
                continue
            data = np.fromfile(outf, dtype=np.uint8)
            if j["op"] == "deinterlace":
                pb = j["count"] * j["esize"]
                data = [data[c * pb:(c + 1) * pb] for c in range(j["n"])]
            out.append((s, data))
        return out
