"""Static instruction counts per basic block of one function in an AMD GPU
assembly listing (``hipcc --cuda-device-only -S``), for per-phase models of a
kernel's loop: each block's vector-ALU, scalar-ALU, LDS and global/buffer
instruction counts, its branches and the compiler's loop-nesting comment.

  python -m paper_1402_2773_amd.isa_blocks decode.s decode_kernelILi1ELi4ELi0ELb0ELb1ELi0E

Blocks start at every label (``.LBB<f>_<n>:``) and at every fall-through
block the compiler names in a comment (``; %bb.<n>:``); block ``n`` below is
printed as its number alone.
"""
from __future__ import annotations

import argparse
import re
import sys


def function_lines(path: str, name_part: str):
    """Lines of the first function whose symbol contains name_part, up to its
    s_endpgm."""
    lines = open(path).read().split("\n")
    start = next(i for i, l in enumerate(lines)
                 if name_part in l and re.match(r"^[A-Za-z_][\w.$]*:", l))
    end = next(i for i in range(start, len(lines)) if lines[i].strip().startswith("s_endpgm"))
    return lines[start:end + 1]


def blocks(lines):
    out = []
    cur = dict(label="entry", note="", v=0, s=0, lds=0, mem=0, branches=[])
    out.append(cur)
    for l in lines[1:]:
        m = re.match(r"^\.LBB\d+_(\d+):(.*)", l) or re.match(r"^; %bb\.(\d+):(.*)", l)
        if m:
            cur = dict(label=m.group(1), note=m.group(2).strip(), v=0, s=0, lds=0, mem=0, branches=[])
            out.append(cur)
            continue
        t = l.strip()
        if not t or t.startswith("."):
            continue
        if t.startswith(";"):
            if "Loop Header" in t or "Depth" in t:
                cur["note"] += " " + t.lstrip("; ").strip()
            continue
        op = t.split()[0]
        if op.startswith("v_"):
            cur["v"] += 1
        elif op.startswith("s_"):
            cur["s"] += 1
            if op.startswith("s_cbranch") or op == "s_branch":
                cur["branches"].append(op.replace("s_cbranch_", "") + ">" + t.split()[-1].split("_")[-1])
        elif op.startswith("ds_"):
            cur["lds"] += 1
        elif op.startswith(("global_", "buffer_", "flat_", "scratch_")):
            cur["mem"] += 1
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("asm")
    ap.add_argument("function", help="part of the function's symbol name")
    args = ap.parse_args(argv)
    bl = blocks(function_lines(args.asm, args.function))
    print("block  valu salu  lds  mem  branches / loop nesting")
    for b in bl:
        note = re.sub(r"\s+", " ", b["note"])[:70]
        print(f"{b['label']:>5} {b['v']:5d} {b['s']:4d} {b['lds']:4d} {b['mem']:4d}  "
              f"{' '.join(b['branches'])}  {note}")
    print(f"total {sum(b['v'] for b in bl):5d} {sum(b['s'] for b in bl):4d} "
          f"{sum(b['lds'] for b in bl):4d} {sum(b['mem'] for b in bl):4d}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
