"""Autotune the planner's launch shapes on this GPU and save the table.

Usage: python -m paper_2307_01117_amd.autotune [--out FILE] [--sizes 1e4,1e5,...]

For every precision and ring length it calls heat_autotune (which times each
temporal-blocking shape with HIP events) and installs the winner for that
decade, then heat_autotune_resident per quarter decade (every resident shape
timed at the quarter decade's ends and middle against the round kernel just
installed; up to six shapes recorded for the planner to choose from per
call), then heat_autotune_batch for the
batching form's kernel classes; the table is then written with
heat_tune_save.  The binding loads
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
    ap.add_argument("--resident-sizes",
                    default="1e5,1.78e5,3.17e5,5.63e5,1e6,1.78e6,3.17e6,5.63e6,1e7",
                    help="one ring length per quarter decade to tune the resident kernel for "
                         "(timed at that quarter decade's ends and middle; '' skips it)")
    ap.add_argument("--no-plain", action="store_true",
                    help="tune the batching form's classes (and resident shapes) only")
    ap.add_argument("--no-verify", action="store_true",
                    help="install the batch classes without the check on a representative batch")
    args = ap.parse_args()
    heat.load()
    for name in args.precisions.split(","):
        prec = heat.PRECISIONS[name]
        for n in ([] if args.no_plain else args.sizes.split(",")):
            N = int(float(n))
            cfg, g = heat.autotune(prec, N, install=True)
            print(json.dumps({"precision": name, "N": N, "best": cfg, "GCUPs": round(g, 1)}),
                  flush=True)
        # the resident kernel against the round kernel just installed, per quarter decade
        for n in [x for x in args.resident_sizes.split(",") if x]:
            N = int(float(n))
            cfg, min_steps, gain = heat.autotune_resident(prec, N, install=True)
            print(json.dumps({"precision": name, "resident_N": N, "best": cfg,
                              "gain_1024_steps": round(gain, 3), "min_steps": min_steps}),
                  flush=True)
        sizes = [int(float(x)) for x in args.batch_sizes.split(",") if x]
        lines = []
        for N in sizes:
            cls, g = heat.autotune_batch(prec, N, install=True)
            print(json.dumps({"precision": name, "batch_N": N, "best": cls, "GCUPs": round(g, 1)}),
                  flush=True)
            lines.append((bucket(N), cls))
        if lines and not args.no_verify:
            verify_batch(prec, name, lines)
    heat.tune_save(args.out)
    print("saved", args.out)


def bucket(N: int) -> int:
    b = 0
    while b < 9 and N >= 10 ** (b + 1):
        b += 1
    return b


def verify_batch(prec: int, name: str, lines) -> None:
    """Keep the tuned batch classes of a precision only if a representative
    uneven batch (1,024 rings of the batching workload's distribution: N
    log-uniform in [1e3, 1e6], nt uniform in [100, 10,000], r in (0.1, 0.5];
    another seed than the benchmark's) runs faster with them than with the
    batching form's own rule; the synthetic same-decade batches the classes
    were timed on stand in for real batches only roughly."""
    import tempfile
    import time

    import torch

    from paper_2307_01117_amd import inputs
    specs = inputs.batch_specs(count=1024, seed=14)
    dt = torch.float64 if prec == heat.FP64 else torch.float32
    us = [torch.from_numpy(inputs.ring_initial(s)).to("cuda", dtype=dt) for s in specs]
    ws = [torch.empty_like(u) for u in us]
    rings = [(u, w, s.nt, s.r, prec) for u, w, s in zip(us, ws, specs)]

    def rate():
        heat.solve_batch_dev(rings)
        best = 0.0
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            heat.solve_batch_dev(rings)
            torch.cuda.synchronize()
            best = max(best, sum(s.N * s.nt for s in specs) / (time.perf_counter() - t0) / 1e9)
        return best

    def install(entries):
        with tempfile.NamedTemporaryFile("w", suffix=".txt", delete=False) as f:
            for b, c in entries:
                f.write(f"b {prec} {b} {c['cells_per_lane']} {c['waves_per_tile']} "
                        f"{c['steps_per_round']}\n")
        heat.tune_load(f.name)
        os.unlink(f.name)

    rule = [(b, {"cells_per_lane": 0, "waves_per_tile": 0, "steps_per_round": 0})
            for b, _ in lines]
    tuned_rate = rate()
    install(rule)
    rule_rate = rate()
    keep = tuned_rate > rule_rate
    if keep:
        install(lines)
    print(json.dumps({"precision": name, "verify_batch_GCUPs": {"tuned": round(tuned_rate, 1),
                                                                "rule": round(rule_rate, 1)},
                      "kept": "tuned" if keep else "rule"}), flush=True)


if __name__ == "__main__":
    main()
