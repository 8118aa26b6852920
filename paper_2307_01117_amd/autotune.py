"""Autotune the planner's launch shapes on this GPU and save the table.

Usage: python -m paper_2307_01117_amd.autotune [--out FILE] [--sizes 1e4,1e5,...]

For every precision and ring length it calls heat_autotune (which times each
temporal-blocking shape with HIP events) and installs the winner for that
decade, then heat_autotune_batch for the batching form's kernel classes; the
table is then written with heat_tune_save.  The binding loads
tune_mi355x.txt next to the library at start-up unless HEAT_TUNE_TABLE names
another file.
"""
from __future__ import annotations

import argparse
import json
import os

from paper_2307_01117_amd import heat

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_mi355x.txt")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--sizes", default="1e3,1e4,1e5,1e6,1e7,1e8")
    ap.add_argument("--precisions", default="fp64,fp32,fp32c",
                    help="precisions to tune; the others keep the loaded table's entries")
    ap.add_argument("--batch-sizes", default="1e3,1e4,1e5,1e6,1e7",
                    help="ring lengths for the batching form's classes ('' skips them)")
    ap.add_argument("--no-plain", action="store_true",
                    help="tune the batching form's classes only")
    args = ap.parse_args()
    heat.load()
    for name in args.precisions.split(","):
        prec = heat.PRECISIONS[name]
        for n in ([] if args.no_plain else args.sizes.split(",")):
            N = int(float(n))
            cfg, g = heat.autotune(prec, N, install=True)
            print(json.dumps({"precision": name, "N": N, "best": cfg, "GCUPs": round(g, 1)}),
                  flush=True)
        for n in [x for x in args.batch_sizes.split(",") if x]:
            N = int(float(n))
            cls, g = heat.autotune_batch(prec, N, install=True)
            print(json.dumps({"precision": name, "batch_N": N, "best": cls, "GCUPs": round(g, 1)}),
                  flush=True)
    heat.tune_save(args.out)
    print("saved", args.out)


if __name__ == "__main__":
    main()
