"""VALU instructions per pair evaluation of the FP64 symmetric near field, from
the gfx950 assembly the compiler emits for near.hip (the counts the
benchmark's near-field roofline uses).

The kernel's round loops are specialised on the tile (target blocks of eight
rows and eight sources per round, or four rows and sixteen sources) and on
the number NB of target blocks; a round evaluates NB pairs per lane.  Each
loop is found by the compiler's loop annotations and its VALU instructions
counted (v_* except MFMA); the one v_rcp_f64 per evaluation gives NB, the
loop's scalar step (8 or 16 sources) the tile.  A straight-line fit of VALU
against NB over NB = 4..12 gives the instructions per evaluation (the slope:
everything an evaluation costs, including its share of the accumulation and
sign selection) and per round (the intercept: source loads, the column
cursor, the second-side reduction and store, loop control), for the two
loop kinds: the leaf's own sources (one side, a zero-separation guard) and
the neighbours' sources (both sides, ds_bpermute row sums).

    python count_valu.py            # compiles near.hip with the build's flags
"""
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from paper_1204_3105_amd import build  # noqa: E402

KERNEL = "_ZN3fmm15k_near_fp64_symEPKNS_7EvalJobENS_8BatchMapE"


def assembly(src="near.hip"):
    out = os.path.join(tempfile.mkdtemp(), "near.s")
    cmd = [build.hipcc()] + build.flags(src) + ["--cuda-device-only", "-S", os.path.join(HERE, src), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return open(out).read().splitlines()


def loops(lines, fn):
    start = next(i for i, l in enumerate(lines) if l.startswith(fn + ":"))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    blocks, cur = [], None
    for l in lines[start:end]:
        m = re.match(r"^\.LBB(\d+_\d+):(.*)", l)
        if m:
            cur = {"name": m.group(1), "note": m.group(2), "ins": [], "full": []}
            blocks.append(cur)
        elif cur is not None:
            t = l.strip()
            if "Loop Header" in t:
                cur["note"] += " header"
            elif t and not t.startswith(";") and not t.startswith("."):
                cur["ins"].append(t.split()[0])
                cur["full"].append(t.split(";")[0].strip())
    groups = {}
    for b in blocks:
        m = re.search(r"Header=BB(\d+_\d+) Depth=", b["note"])
        key = b["name"] if "header" in b["note"] else (m.group(1) if m else None)
        if key:
            groups.setdefault(key, []).append(b)
    out = []
    for bl in groups.values():
        ins = [i for b in bl for i in b["ins"]]
        full = [i for b in bl for i in b["full"]]
        nb = sum(i.startswith("v_rcp_f64") for i in ins)
        if nb == 0:
            continue
        valu = sum(i.startswith("v_") and not i.startswith("v_mfma") for i in ins)
        two = any(i.startswith("ds_bpermute") for i in ins)
        step = [int(m.group(1)) for i in full for m in [re.match(r"s_add_i32 s\d+, s\d+, (8|16)$", i)] if m]
        out.append((two, step[0] if step else 0, nb, valu))
    return out


def fit(points):
    xs = [float(x) for x, _ in points]
    ys = [float(y) for _, y in points]
    n = len(xs)
    mx, my = sum(xs) / n, sum(ys) / n
    sxx = sum((x - mx) ** 2 for x in xs)
    slope = sum((x - mx) * (y - my) for x, y in zip(xs, ys)) / sxx
    return slope, my - slope * mx


def main():
    found = loops(assembly(), KERNEL)
    for tc, tile in ((8, "8 x 8"), (16, "4 x 16")):
        for two, name in ((True, "neighbours, both sides"), (False, "own leaf, one side")):
            pts = sorted((nb, v) for t, c, nb, v in found if t == two and c == tc and nb >= 4)
            if len(pts) < 2:
                continue
            slope, icpt = fit(pts)
            print("%-6s %-24s VALU per evaluation %.1f, per round %.1f  (NB, VALU: %s)" % (
                tile, name, slope, icpt, ", ".join("%d:%d" % p for p in pts)))


if __name__ == "__main__":
    main()
