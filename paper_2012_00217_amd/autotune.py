"""Launch-schedule autotuner for the apply and CG kernels (MI355X).

The apply kernel and the fused CG kernels take four launch parameters:
bytes of a row chunk, bytes per lane, tiles per XCD group and workgroups per
XCD.  Which combination is fastest depends on the sector dimension (how far the
high-bond gathers reach compared with an XCD's L2 and the last-level cache) and
on the row width of the block.  This tool times one block Jacobi-PCG call (the
kernels that dominate a solve) for a staged set of candidates at each shape and
writes the winners into ``csrc/apply_schedules.inc``, which the library compiles
in.  Run it on the GPU, then rebuild:

    python -m paper_2012_00217_amd.autotune --write
    python -m paper_2012_00217_amd.build

The environment variables MBL_APPLY_CHUNK_BYTES, MBL_APPLY_LANE_BYTES,
MBL_APPLY_XCD_GROUP and MBL_APPLY_SLOTS_PER_XCD override single fields of the
compiled-in choice at run time; the tuner uses them to try candidates.  A
schedule changes which workgroup handles which rows, so dot products may
differ in the last bits between schedules; with one schedule every result is
bitwise reproducible.
"""

import argparse
import datetime
import json
import math
import os
import sys

import torch

from . import api, workloads

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "apply_schedules.inc")
KNOBS = ("MBL_APPLY_CHUNK_BYTES", "MBL_APPLY_LANE_BYTES", "MBL_APPLY_XCD_GROUP",
         "MBL_APPLY_SLOTS_PER_XCD")
DEFAULT = (512, 64, 0, 256)

# (L, block columns, element type): the shapes the solver's workloads run the
# CG at -- single solves at L = 12, 20, 22, 24, 28 (at L >= 22 also on the 64
# wanted columns alone), the batched L = 14-18 realisations, and the FP32 CG
# of mixed-precision serving at L = 16-26.
SHAPES = [
    (12, 16, torch.float64), (14, 32, torch.float64), (16, 32, torch.float64),
    (18, 32, torch.float64), (20, 64, torch.float64), (22, 64, torch.float64),
    (24, 128, torch.float32), (24, 128, torch.float64), (28, 32, torch.float64),
    (16, 32, torch.float32), (18, 32, torch.float32), (20, 32, torch.float32),
    (22, 32, torch.float32), (24, 32, torch.float32), (26, 32, torch.float32),
    # the wanted columns alone, once the guard columns of a large solve stop
    (22, 64, torch.float32), (24, 64, torch.float32),
]


def _set(cand):
    for k, v in zip(KNOBS, cand):
        os.environ[k] = str(v)


def _clear():
    for k in KNOBS:
        os.environ.pop(k, None)


def time_pcg(H, R, m, cand, reps=3):
    """Fastest of `reps` timed m-step PCG calls under schedule `cand` (ms per step)."""
    _set(cand)
    try:
        H.pcg(R, 0.0, m)  # warm: plans, graph capture, caches
        best = math.inf
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            H.pcg(R, 0.0, m)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / m)
        return best
    finally:
        _clear()


def tune_shape(L, b, dtype, budget_ms=150.0, log=print):
    H = api.Hamiltonian(L, workloads.disorder(L, 4.0, 0))
    try:
        g = torch.Generator(device="cuda")
        g.manual_seed(0)
        R = torch.randn(H.n, b, dtype=dtype, device="cuda", generator=g)
        # steps per timing: enough for ~budget_ms, at least 10 so the graph replay runs
        t1 = time_pcg(H, R, 10, DEFAULT, reps=1)
        m = int(max(10, min(400, budget_ms / max(t1, 1e-3))))
        seen = {}

        def run(c):
            if c not in seen:
                seen[c] = time_pcg(H, R, m, c)
                log(json.dumps({"L": L, "b": b, "dtype": str(dtype)[6:], "cand": c,
                                "ms_per_step": round(seen[c], 5)}))
            return seen[c]

        base = run(DEFAULT)
        # stage 1: XCD grouping and workgroups per XCD at the default chunking
        # (fewer workgroups shrink the rows in flight per XCD, which helps the
        # L2 hit rate of the gathers on the largest sectors)
        for grp in (0, 64, 16, 4):
            for slots in (256, 128, 64):
                run((DEFAULT[0], DEFAULT[1], grp, slots))
        best = min(seen, key=seen.get)
        # stage 2: chunk and lane widths at the best grouping
        for cb, lb in ((512, 64), (256, 64), (256, 32), (256, 16), (128, 16), (128, 32)):
            run((cb, lb, best[2], best[3]))
        best = min(seen, key=seen.get)
        # stage 3: grouping again at the best chunking
        for grp in (0, 64, 16, 4):
            run((best[0], best[1], grp, best[3]))
        best = min(seen, key=seen.get)
        # keep the default unless the winner is clearly faster (timing noise)
        if seen[best] > 0.98 * base:
            best = DEFAULT
        return {"L": L, "n": H.n, "b": b, "elem": R.element_size(), "row_bytes": b * R.element_size(),
                "sched": best, "ms": seen[best], "default_ms": base, "m": m}
    finally:
        H.close()
        torch.cuda.empty_cache()


def write_table(results, path=TABLE, device_name=""):
    lines = [
        "// Generated by `python -m paper_2012_00217_amd.autotune --write` on "
        f"{device_name or 'the GPU'}, {datetime.date.today().isoformat()}.",
        "// {L, n, row bytes, element bytes, {chunk bytes, lane bytes, XCD group, WGs per XCD}}",
        "// and the measured block-PCG time per step: tuned (default).",
        "static const SchedEntry kSchedTable[] = {",
    ]
    for r in results:
        c = r["sched"]
        lines.append(f"    {{{r['L']}, {r['n']}, {r['row_bytes']}, {r['elem']}, "
                     f"{{{c[0]}, {c[1]}, {c[2]}, {c[3]}}}}},  "
                     f"// b={r['b']}: {r['ms']:.4f} ms ({r['default_ms']:.4f} ms)")
    lines.append("    {0, 0, 0, 0, {512, 64, 0, 256}},")
    lines.append("};")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def read_table(path=TABLE):
    """Entries of an existing schedule table (the results format of tune_shape)."""
    import re
    out = []
    pat = re.compile(r"\{(\d+), (\d+), (\d+), (\d+), \{(\d+), (\d+), (\d+), (\d+)\}\},\s*"
                     r"// b=(\d+): ([0-9.]+) ms \(([0-9.]+) ms\)")
    if not os.path.exists(path):
        return out
    for line in open(path):
        m = pat.search(line)
        if m and int(m.group(1)) > 0:
            v = [int(x) for x in m.groups()[:9]]
            out.append({"L": v[0], "n": v[1], "row_bytes": v[2], "elem": v[3],
                        "sched": tuple(v[4:8]), "b": v[8], "ms": float(m.group(10)),
                        "default_ms": float(m.group(11))})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--write", action="store_true", help="rewrite the schedule table")
    ap.add_argument("--out", default=TABLE, help="table path for --write (default: csrc/apply_schedules.inc)")
    ap.add_argument("--shapes", default="", help="comma list of L:b:f32|f64 (default: built-in)")
    ap.add_argument("--json", default="", help="also dump the results to this file")
    ap.add_argument("--merge", action="store_true",
                    help="with --write: keep the table's entries for shapes not tuned now")
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("autotune needs a GPU")
    shapes = SHAPES
    if a.shapes:
        shapes = []
        for t in a.shapes.split(","):
            L, b, d = t.split(":")
            shapes.append((int(L), int(b), torch.float32 if d == "f32" else torch.float64))
    _clear()
    results = []
    for L, b, dt in shapes:
        r = tune_shape(L, b, dt, log=lambda s: print(s, flush=True))
        print(json.dumps({"chosen": r}), flush=True)
        results.append(r)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(results, f, indent=1)
    if a.write and a.merge:
        key = lambda r: (r["L"], r["row_bytes"], r["elem"])
        fresh = {key(r) for r in results}
        results = [r for r in read_table(a.out) if key(r) not in fresh] + results
        results.sort(key=lambda r: (r["elem"], r["row_bytes"], r["L"]))
    if a.write:
        props = torch.cuda.get_device_properties(0)
        arch = getattr(props, "gcnArchName", "").split(":")[0]
        write_table(results, a.out, device_name=f"{props.name} ({arch or 'unknown arch'})")
        print(f"wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
