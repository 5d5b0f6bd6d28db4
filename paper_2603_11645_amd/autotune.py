"""Autotune GConn+Euler on the benchmark workloads and write the tuning cache.

    python -m paper_2603_11645_amd.autotune [--workloads C1,C2,C3,C4] [--reps 5]
                                            [--out paper_2603_11645_amd/tuned_gfx950.json]

For each workload graph, rst_autotune runs coordinate descent over the
method's knobs (hooking variant and sampling, sweep block, heavy degree,
ruling-set stride, ranking words per thread), timing every candidate (median
of `reps` HIP-event timings) and checking its output on the device; the
context's cache (one entry per architecture, method and size class) is then
written with rst_tune_save.  bench.py loads this file and applies the entry
that matches its graph.  One line per workload is printed: the time with the
default setting, with the chosen one, and the choice.
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuned_gfx950.json")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workloads", default="C1,C2,C3,C4")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args(argv)
    import numpy as np
    import torch
    import paper_2603_11645_amd as rst
    from paper_2603_11645_amd import inputs as I

    ctx = rst.Context(0)
    names = {v: k for k, v in vars(rst).items() if k.startswith("OPT_") and isinstance(v, int)}
    rows = []
    for w in args.workloads.split(","):
        g = I.config(w)
        off = torch.from_numpy(np.ascontiguousarray(g.offsets_typed())).cuda()
        cols = torch.from_numpy(np.ascontiguousarray(g.cols)).cuda()
        # every knob back to its default before each graph
        for opt, val in DEFAULTS.items():
            ctx.set_option(getattr(rst, opt), val)
        res = ctx.autotune(off, cols, g.root, "gconn", reps=args.reps)
        choice = {names.get(o, str(o)): v for o, v in res["options"].items()}
        row = {"workload": w, "n": g.n, "nnz": g.nnz, "ms_default": round(res["ms_default"], 4),
               "ms_best": round(res["ms_best"], 4), "candidates": res["candidates"],
               "rejected": res["rejected"], "choice": choice}
        rows.append(row)
        print(json.dumps(row), flush=True)
        del off, cols
        torch.cuda.empty_cache()
    ctx.tune_save(args.out)
    print("wrote", args.out, flush=True)
    return rows


# the library's defaults of the knobs rst_autotune searches for GConn+Euler
DEFAULTS = {"OPT_HOOK_MODE": 0, "OPT_HOOK_SAMPLE": -1, "OPT_SWEEP_BLOCK": 256,
            "OPT_HEAVY_DEGREE": 1024, "OPT_RANK_ELEMS_PER_THREAD": 4, "OPT_RANK_STRIDE": 0}

if __name__ == "__main__":
    main()
    sys.exit(0)
