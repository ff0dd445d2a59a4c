"""Wait states between a matrix-core product and its first reader, on every
path through the compiled kernel.

A matrix-core (MFMA) instruction writes its result registers some cycles
after it issues; a vector or memory instruction that reads or rewrites those
registers sooner reads a stale value. The compiler pads such readers with
s_nop, but on gfx950 a branch placed between the product and its reader (a
loop whose record prefetch sits under a uniform branch, taken on the last
tiles) has been seen to leave the taken path one wait state where the
straight-line path got eight: the reads then took the previous contents and
the second tier's transmitted term came out wrong on the last tiles.

This module compiles kernel sources to gfx950 assembly and walks every path
from each MFMA (through conditional and unconditional branches) to the first
non-MFMA instruction touching its destination registers, counting wait
states (one per instruction, N + 1 for s_nop N). A path that passes through
another MFMA is left to the compiler's accounting (the intervening product
occupies the pipe for its own passes). Paths shorter than the floor for the
instruction's shape are reported.

Usage: python -m paper_2108_07001_amd.isa_scan [-j JOBS] [source.hip ...]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# Floors (wait states) the compiler itself places on straight-line code after
# the two product shapes used here.
FLOORS = {"32x32x16": 12, "16x16x32": 8}
DEFAULT_FLOOR = 12


def floor_of(mnemonic: str) -> int:
    for shape, n in FLOORS.items():
        if shape in mnemonic:
            return n
    return DEFAULT_FLOOR


def _regs(operands: str) -> set[int]:
    out: set[int] = set()
    for a, b in re.findall(r"v\[(\d+):(\d+)\]", operands):
        out.update(range(int(a), int(b) + 1))
    for a in re.findall(r"(?<![\w\[])v(\d+)\b", operands):
        out.add(int(a))
    return out


def parse(asm: str) -> list[dict]:
    """Kernels of an assembly listing: name, instructions, label -> index."""
    funcs: list[dict] = []
    cur = None
    for line in asm.split("\n"):
        if re.match(r"^_Z\S+:", line):
            cur = {"name": line.split(":")[0], "ins": [], "labels": {}}
            funcs.append(cur)
            continue
        if cur is None:
            continue
        if line.startswith(".Lfunc_end"):
            cur = None
            continue
        m = re.match(r"^(\.LBB\d+_\d+):", line)
        if m:
            cur["labels"][m.group(1)] = len(cur["ins"])
            continue
        t = line.split(";")[0].strip()
        if not t or t.startswith("."):
            continue
        cur["ins"].append(t)
    return funcs


def scan(func: dict, limit: int = 32) -> list[tuple[int, int, str, str]]:
    """(fewest wait states, index, MFMA, reader) for each MFMA with a reader
    reachable in fewer than `limit` wait states."""
    ins, labels = func["ins"], func["labels"]
    res = []
    for i, t in enumerate(ins):
        if not t.startswith("v_mfma"):
            continue
        dst = _regs(t.split(",")[0])
        best: list = [None]
        seen: dict[int, int] = {}
        stack = [(i + 1, 0)]
        while stack:
            k, ws = stack.pop()
            if ws >= limit or k >= len(ins) or seen.get(k, 1 << 30) <= ws:
                continue
            seen[k] = ws
            u = ins[k]
            op = u.split()[0]
            if op.startswith("v_mfma") or op == "s_endpgm":
                continue
            ops = u[len(op):]
            if op.startswith(("v_", "ds_", "global_", "buffer_", "flat_", "scratch_")) and _regs(ops) & dst:
                if best[0] is None or ws < best[0][0]:
                    best[0] = (ws, u)
                continue
            w = int(u.split()[1]) + 1 if op == "s_nop" else 1
            if op == "s_branch":
                stack.append((labels[u.split()[1]], ws + w))
                continue
            if op.startswith("s_cbranch"):
                stack.append((labels[u.split()[1]], ws + w))
            stack.append((k + 1, ws + w))
        if best[0] is not None:
            res.append((best[0][0], i, t, best[0][1]))
    return res


def short_paths(asm: str) -> list[str]:
    """Readers closer to their product than the shape's floor, one line each."""
    out = []
    for f in parse(asm):
        for ws, _, t, u in scan(f):
            if ws < floor_of(t.split()[0]):
                out.append(f"{f['name']}: {ws} wait states: {t} -> {u}")
    return out


def compile_asm(src: str, out_dir: str, hipcc: str | None = None) -> str:
    """gfx950 device assembly of one source, with the library's own flags."""
    from .build import FLAGS, HIPCC
    out = os.path.join(out_dir, os.path.basename(src)[:-4] + ".s")
    flags = [f for f in FLAGS if f not in ("-fPIC", "-Wall")]
    cmd = [hipcc or HIPCC, *flags, "--cuda-device-only", "-S", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc -S failed on {src}:\n{r.stderr[-2000:]}")
    return out


def mfma_sources() -> list[str]:
    """The library's sources that instantiate matrix-core kernels."""
    pats = ("mfma_inst_*.hip", "serve_inst_*.hip", "hd_mfma_inst.hip", "roofs.hip")
    return sorted(p for pat in pats for p in glob.glob(os.path.join(CSRC, pat)))


def check(sources: list[str] | None = None, jobs: int | None = None) -> list[str]:
    sources = sources or mfma_sources()
    jobs = jobs or min(len(sources), os.cpu_count() or 4, 16)
    with tempfile.TemporaryDirectory() as d:
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            paths = list(ex.map(lambda s: compile_asm(s, d), sources))
        found = []
        for p in paths:
            found += short_paths(open(p).read())
    return found


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("sources", nargs="*")
    a = ap.parse_args()
    bad = check(a.sources or None, a.j)
    print("\n".join(bad) if bad else "no short paths")
    sys.exit(1 if bad else 0)
