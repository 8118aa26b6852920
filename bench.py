#!/usr/bin/env python3
"""Benchmark of the periodic 1D heat stencil on one MI355X.

A step is one pass of the whole hot path over the ring: the binary64
checksum of the initial state, ceil(nt/T) rounds of the temporal-blocked
window kernel (or nt launches of the one-step sweep with --kernel step),
and the checksum of the final state.  The state stays in HBM between steps
(each step continues from the previous one's result: same size, same work).

Default workload: a ring of 100 partitions x 1,000,000 cells (N = 1e8),
r = 1/2, 1,000 explicit-Euler steps per pass, Uniform[0,1) seed 1, binary64.
The metric is giga cell-updates per second (N * nt / time), the paper's
"cells processed per second".

The default run adds, in the same line, the rest of the metric measured on
the same GPU: ``precision`` (compensated and plain binary32 on the 1e8-cell
perturbed ring, r = 1/4, with the whole-ring error against binary64),
``batch`` (4,096 uneven rings batched in binary64 against the same rings
solved one by one, and in compensated binary32 with every ring's error
against binary64) and ``serve`` (Poisson arrivals at 200 requests/s for 15 s:
p50/p99 latency, GCUP/s against the offered load, alone-vs-mix bit equality
and the compensated requests' error against binary64).  ``value`` is the
plain binary64 ring's rate.

Prints ONE JSON line.  ``--gpus N`` with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# Published MI355X vector peaks (an FMA counts as 2 flops): FP64 78.6 TFLOP/s,
# FP32 157.3 TFLOP/s (256 CUs x 2.4 GHz x 128 resp. 256 flops per CU-cycle).
VECTOR_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "fp32c": 157.3}
# Algorithmic flops per cell update (CUP) of each form, the update formula as
# written (an fma counts as 2): binary64 c + r*((l - 2c) + q) = 5 (2c, -, +,
# *, +); plain binary32 the same five; compensated binary32 15: the Laplacian
# of the pair ((q-c) + (eq-ec)) - ((c-l) + (ec-el)) (7), t = fma(r, L, c)
# (2), c - t (1), its rounding error fma(r, L, c - t) (2), the coefficient's
# low part fma(rl, L, res) (2) and the addition into e (1); 13 when the
# coefficient is a binary32 number (no low part).
FLOPS_PER_CUP = {"fp64": 5, "fp32": 5, "fp32c": 15}
# Issue-rate view of the same kernels: VALU lane operations per second against
# the instruction ceiling (FP64 39.3e12 = 256 CUs x 64 lanes x 2.4 GHz; FP32
# twice that when two instructions issue together), and the minimal
# instructions per update of each form: binary64 fma(-2,c,l), +q, *r, +c = 4;
# binary32 in flux form (q-c) - (c-l), whose one-sided difference serves two
# cells: one difference, the difference of differences, *r, +c = 4;
# compensated 9 (the pair's flux, shared by two cells, 3; L 1; t 1; c - t 1;
# the error fma 1; the low-part fma 1; the addition into e 1), 8 without the
# low part.  Since the published flops count an FMA as two, a kernel that
# issues OPS_PER_CUP instructions for FLOPS_PER_CUP flops can reach at most
# FLOPS_PER_CUP / (2 * OPS_PER_CUP) of the flops peak: 0.625 for binary64 and
# plain binary32 (one FMA, the exact 2c, is all the bitwise contract allows),
# 0.83 / 0.81 for the compensated form.
VALU_PEAK_TOPS = {"fp64": 39.3, "fp32": 78.65, "fp32c": 78.65}
OPS_PER_CUP = {"fp64": 4, "fp32": 4, "fp32c": 9}


def cup_costs(prec_name: str, r: float):
    """(flops, VALU instructions) per cell update of a form at coefficient r:
    the compensated form drops its low-part term when r is a binary32 number
    (the kernels' rl = fl32(r - fl32(r)) is zero)."""
    import numpy as np
    flops, ops = FLOPS_PER_CUP[prec_name], OPS_PER_CUP[prec_name]
    if prec_name == "fp32c" and np.float32(float(r) - float(np.float32(r))) == 0:
        flops, ops = flops - 2, ops - 1
    return flops, ops


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="ring_1e8",
                    choices=["ring_1e6", "ring_1e7", "ring_1e8", "ring_1e8_perturbed",
                             "paper_ramp_1e6"])
    ap.add_argument("--ring", default=None, metavar="N,STEPS[,R]",
                    help="instead of a named workload: a Uniform[0,1) ring (seed 3) of N cells, "
                         "STEPS steps, coefficient R (default 1/2)")
    ap.add_argument("--precision", default=None, choices=["fp64", "fp32", "fp32c"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "tb", "step", "resident"])
    ap.add_argument("--cells-per-lane", type=int, default=0)
    ap.add_argument("--steps-per-round", type=int, default=0)
    ap.add_argument("--waves-per-group", type=int, default=0)
    ap.add_argument("--register-form", type=int, default=0, choices=[0, 1, 2, 3])
    ap.add_argument("--exchange", default="auto", choices=["auto", "none", "lds", "deep"],
                    help="waves of a workgroup: own tiles (none) or one shared tile with "
                         "LDS edge exchanges every K/4 steps (lds) or K/2 steps (deep)")
    ap.add_argument("--launch", default="rounds", choices=["rounds", "batch", "persistent"],
                    help="plain workload: heat_solve_dev (rounds, with both checksums), or the "
                         "ring alone through the batching form (one launch per round) or its "
                         "persistent flag-synchronised launch (no checksums in those two)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time the library's plain streaming copy of the state instead "
                         "(the bandwidth reference for the roofline and traffic counters)")
    ap.add_argument("--form", default="plain", choices=["plain", "batch", "serve"],
                    help="plain: one ring (the workload above); batch: 4,096 uneven rings "
                         "advanced together (N log-uniform in [1e3, 1e6], nt uniform in "
                         "[100, 10000], r in (0.1, 0.5]), compared with solving them one by one")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--rates", default="50,200,1000",
                    help="serve: Poisson arrival rates (requests/s)")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: seconds of arrivals")
    ap.add_argument("--warm-s", type=float, default=5.0,
                    help="serve: arrivals before this time are excluded from latency stats")
    ap.add_argument("--batch-mode", default="rounds", choices=["rounds", "graph", "persistent"])
    ap.add_argument("--no-plain-compare", action="store_true",
                    help="batch: skip solving the rings one by one for comparison")
    ap.add_argument("--cpu-steps", type=int, default=40,
                    help="time steps of the full ring the CPU oracle runs as its sample")
    ap.add_argument("--no-host-path", action="store_true",
                    help="skip timing the host-buffer boundary (heat_solve: PCIe both ways)")
    ap.add_argument("--no-cpu-threads", action="store_true",
                    help="skip the thread axis of the threaded CPU oracle (binary64 ring only)")
    ap.add_argument("--no-sub-records", action="store_true",
                    help="default run: skip the precision, batch and serve records")
    ap.add_argument("--cpu-thread-steps", type=int, default=5,
                    help="time steps of the full ring per thread count on the thread axis")
    return ap.parse_args()


def precision_report(heat, torch, u0, nparts, r, nt, prec, stream):
    """Error of one pass of a binary32 form against the binary64 path
    (bit-identical to the oracle) over the whole ring: max |x - y| / max |y|,
    against binary64 run from fl32(u0) widened (arithmetic only) and from u0
    itself (end to end); and the same form with the state stored as binary32
    offsets from the ring's mean (the library's host-buffer path with
    ``shift``), end to end."""
    import math

    import numpy as np
    d = torch.from_numpy(u0).to("cuda").float()
    heat.solve_dev(d, nparts, r, nt, precision=prec, stream=stream)
    got = d.double()
    del d
    out = {}
    for label, start in (("vs_fp64_from_fl32_u0", u0.astype(np.float32).astype(np.float64)),
                         ("vs_fp64_from_u0", u0)):
        ref = torch.from_numpy(start).to("cuda")
        heat.solve_dev(ref, nparts, r, nt, precision=heat.FP64, stream=stream)
        torch.cuda.synchronize()
        out[label] = float((got - ref).abs().max() / ref.abs().max())
        if label == "vs_fp64_from_u0":
            del got
            shift = math.fsum(u0) / u0.size
            res = heat.solve_batch([dict(u0=u0, nparts=nparts, r=r, nt=nt, precision=prec,
                                         shift=shift)])[0]
            sh = torch.from_numpy(res.u).to("cuda")
            out["mean_shifted_vs_fp64_from_u0"] = float((sh - ref).abs().max() / ref.abs().max())
            out["shift"] = shift
            del sh, res
        del ref
    out["steps"] = nt
    return out


def kernel_source_digest() -> str:
    """sha256 of the kernel sources and of the compiler flags they are built
    with (build.py's flag lists); HBM traffic taken from counters is only
    reported while the kernels are the ones that were counted."""
    import hashlib

    from paper_2307_01117_amd import build
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2307_01117_amd")
    for f in ("heat_device.h", "window.h", "round.h", "kernels.hip", "kernels_xchg.hip",
              "kernels_xchg2.hip", "kernels_f32.hip", "kernels_f32c.hip"):
        with open(os.path.join(pkg, "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(repr((build.HIPCC_FLAGS, sorted(build.SOURCE_FLAGS.items()))).encode())
    return h.hexdigest()


def measured_traffic(kernel, workload, precision, pl):
    """HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE and
    WRITE_SIZE, each scaled by what it reads for the library's copy kernel of
    known size), or None if not measured for this kernel and shape, or if the
    kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha256") != kernel_source_digest():
        return None
    key = f"{kernel}/{workload}/{precision}/K{pl['cells_per_lane']}/T{pl['steps_per_round']}"
    if pl.get("exchange_steps"):
        key += f"/G{pl['waves_per_group']}S{pl['exchange_steps']}"
    e = t.get("entries", {}).get(key)
    return None if e is None else e["bytes_per_launch"]


def cpu_baseline(u0, r, steps, precision, T):
    """The oracle, as it stands, on the host cores: single-threaded C."""
    import numpy as np

    import oracle
    t0 = time.perf_counter()
    if precision == "fp64":
        oracle.solve(u0, r, steps)
    elif precision == "fp32":
        oracle.solve_f32(u0.astype(np.float32), r, steps)
    else:
        oracle.solve_f32c(u0.astype(np.float32), r, steps, T)
    dt = time.perf_counter() - t0
    return {"value": round(u0.size * steps / dt / 1e9, 4), "unit": "GCUP/s", "cores": 1,
            "kind": "oracle",
            "sample": f"full ring of {u0.size} cells, {steps} steps ({dt:.1f} s, single thread)"}


def host_path(heat, u0, nparts, r, nt, reps=2):
    """The host-buffer boundary: heat_solve on a pageable binary64 array
    (device allocation, copy in, every step, copy out, free), best of `reps`
    calls after one untimed call.  A reported rate beside `value`, never it."""
    import numpy as np
    a = np.array(u0, dtype=np.float64, copy=True)
    lib = heat.load()
    best = None
    for i in range(reps + 1):
        a[:] = u0
        t0 = time.perf_counter()
        heat._check(lib.heat_solve(a.ctypes.data, a.size, int(nparts), float(r), int(nt)))
        dt = time.perf_counter() - t0
        if i > 0:
            best = dt if best is None else min(best, dt)
    return {"value": round(u0.size * nt / best / 1e9, 1), "unit": "GCUP/s",
            "ms": round(best * 1e3, 1),
            "what": "heat_solve on a pageable host array: H2D, all steps, D2H"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads(u0, r, steps, workload, max_threads=16):
    """The paper's own CPU method, timed along its thread axis: one thread per
    segment, ghost cells through single-producer single-consumer queues (the
    threaded oracle; every thread count gives the same bits), in its scalar
    build ("value") and with the segment sweep vectorised ("value_simd", the
    counterpart of the paper's SIMD Rust build; the same bits again).  Three
    samples: the paper's workload (ramp, 1e6 cells, 1,000 steps), the
    1e6-cell Uniform ring of 100 steps, and a few steps of the full ring timed
    above."""
    import numpy as np

    import oracle
    from paper_2307_01117_amd import inputs
    avail = len(os.sched_getaffinity(0))
    threads = [t for t in (1, 2, 4, 8, 16) if t <= min(avail, max_threads)]
    ramp = inputs.WORKLOADS["paper_ramp_1e6"]
    small = inputs.WORKLOADS["ring_1e6"]
    samples = [("paper_ramp_1e6", inputs.make_initial(ramp["init"], ramp["N"], ramp["seed"]),
                ramp["r"], ramp["nt"]),
               ("ring_1e6", inputs.make_initial(small["init"], small["N"], small["seed"]),
                small["r"], small["nt"]),
               (f"{workload}, {steps} steps", u0, r, steps)]
    res = {}
    for name, u, rr, nt in samples:
        rates, ref, same = {False: [], True: []}, None, True
        for simd in (False, True):
            for t in threads:
                t0 = time.perf_counter()
                out = oracle.solve_threads(u, t, rr, nt, simd=simd)
                dt = time.perf_counter() - t0
                rates[simd].append(round(u.size * nt / dt / 1e9, 4))
                if ref is None:
                    ref = out
                else:
                    same = same and bool(np.array_equal(out.view(np.uint64), ref.view(np.uint64)))
                del out
        res[name] = {"N": int(u.size), "nt": int(nt), "value": rates[False],
                     "value_simd": rates[True], "bitwise_equal_across_threads": same}
    return {"kind": "oracle_threads", "unit": "GCUP/s", "threads": threads,
            "cores_available": avail, "cpu": cpu_model(), "samples": res}


def run_plain(args, workload, prec_name, steps, warmup, cfg, host=True):
    """One ring: `warmup` untimed passes, then `steps` timed passes of the hot
    path (each one heat_solve_dev call with both checksums), HIP events on the
    passes' stream around every timed pass; returns the bench dict (without
    the CPU legs) and the initial state."""
    import torch

    from paper_2307_01117_amd import heat, inputs
    w = inputs.WORKLOADS[workload]
    prec = heat.PRECISIONS[prec_name]
    N, nparts, r, nt = w["N"], w["nparts"], w["r"], w["nt"]
    pl = heat.plan(N, nt, prec, **cfg)

    u0 = inputs.make_initial(w["init"], N, w["seed"])
    dt = torch.float64 if prec == heat.FP64 else torch.float32
    dev = torch.device("cuda", 0)
    d_u = torch.from_numpy(u0).to(dev, dtype=dt)
    d_work = torch.empty_like(d_u)
    stream = torch.cuda.current_stream(dev)

    launch = getattr(args, "launch", "rounds")

    def one_step():
        if launch != "rounds":
            # the ring alone through the batching form (no checksums)
            return heat.solve_batch_dev([(d_u, d_work, nt, r, prec)], stream=stream,
                                        persistent=launch == "persistent")
        # the whole hot path in one call: checksum of the state in (fused into
        # the first round), the rounds, checksum of the state out (fused into
        # the last round)
        return heat.solve_dev(d_u, nparts, r, nt, precision=prec, stream=stream, work=d_work,
                              sums=True, **cfg)

    for _ in range(warmup):
        one_step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        one_step()
        b.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed_ms = sum(a.elapsed_time(b) for a, b in evs)

    if launch != "rounds":
        # the batching form's geometry and launches are its own: the rate only
        del d_u, d_work
        return {"metric": "GCUP/s (giga cell-updates per second)",
                "value": round(N * nt * steps / elapsed / 1e9, 3), "unit": "GCUP/s",
                "n_gpus": 1, "steps": steps, "warmup": warmup,
                "ms_per_step": round(elapsed * 1e3 / steps, 3), "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "data": "synthetic",
                "dtype": {"fp64": "f64", "fp32": "f32", "fp32c": "f32 (compensated)"}[prec_name],
                "config": {"workload": workload, "N": N, "nt": nt, "r": r,
                           "precision": prec_name, "launch": launch},
                "roofline": None}, u0

    # the round launches alone: one pass without checksums between two HIP
    # events (no other kernel: rounds are even, so no copy-back)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    kern_ms = []
    for _ in range(max(2, min(steps, 5))):
        ev[0].record(stream)
        heat.solve_dev(d_u, nparts, r, nt, precision=prec, stream=stream, work=d_work, **cfg)
        ev[1].record(stream)
        torch.cuda.synchronize()
        kern_ms.append(ev[0].elapsed_time(ev[1]))

    ms_per_step = elapsed * 1e3 / steps
    value = N * nt * steps / elapsed / 1e9

    launches = pl["rounds"]
    # average launch duration over the timed region: the events around each
    # timed pass hold its round launches plus the final checksum reduction
    # and the copy of the two sums (about 10 us per pass), so this is an
    # upper bound on the round kernel's duration
    k_avg_ms = timed_ms / steps / launches
    k_alone_ms = sum(kern_ms) / len(kern_ms) / launches
    es = 8 if prec == heat.FP64 else 4
    alg_bytes = 2 * es * N                    # read the state once, write it once per launch
    steps_per_launch = nt / launches
    if pl["kernel"] == heat.KERNEL_STEP:
        achieved = alg_bytes / (k_avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}
        # the achievable bandwidth: the library's streaming copy of the same
        # bytes, timed here on the same stream
        heat.copy_dev(d_u, d_work, stream)
        ev[0].record(stream)
        for _ in range(20):
            heat.copy_dev(d_u, d_work, stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        copy_gbs = alg_bytes / (ev[0].elapsed_time(ev[1]) / 20 * 1e-3) / 1e9
        roof["copy_GBs"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(achieved / copy_gbs, 4)
    else:
        # Temporal blocking moves 2*es bytes per cell per T steps and is
        # limited by the vector ALU: achieved = algorithmic flops of the cell
        # updates per launch / launch time, against the published vector peak.
        # Beside it, the issue-rate view (VALU lane operations per second
        # against the instruction ceiling), which the bitwise contract caps the
        # flops fraction by (see OPS_PER_CUP).
        cups = N * steps_per_launch
        fpc, opc = cup_costs(prec_name, r)
        tflops = fpc * cups / (k_avg_ms * 1e-3) / 1e12
        peak = VECTOR_PEAK_TFLOPS[prec_name]
        ops = opc * cups / (k_avg_ms * 1e-3) / 1e12
        hbm = alg_bytes / (k_avg_ms * 1e-3) / 1e9
        roof = {"bound": "alu", "achieved": round(tflops, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(tflops / peak, 4), "traffic": None,
                "flops_per_cup": fpc,
                "valu_issue": {
                    "achieved": round(ops, 2), "peak": VALU_PEAK_TOPS[prec_name],
                    "unit": "T VALU lane-ops/s", "frac": round(ops / VALU_PEAK_TOPS[prec_name], 4),
                    "ops_per_cup": opc,
                    "flops_frac_cap": round(fpc / (2 * opc), 4)},
                "hbm_algorithmic_GBs": round(hbm, 1),
                "hbm_frac": round(hbm / HBM_PEAK_GBS, 4),
                # cell updates per second against the roofline of one step per
                # launch (every step reads and writes the state: 2*es bytes per
                # cell update at 8 TB/s); temporal blocking exceeds it T-fold
                "vs_one_step_hbm_roofline": round(cups / (k_avg_ms * 1e-3)
                                                  / (HBM_PEAK_GBS * 1e9 / (2 * es)), 2)}
    roof["kernel"] = {heat.KERNEL_STEP: "k_step",
                      heat.KERNEL_RESIDENT: "k_resident"}.get(pl["kernel"], "k_window")
    # the library's one kernel of its own among the round kernels: the
    # compensated form's binary32-coefficient sweep for 32-cell lone waves
    # (register forms 1 and 2)
    if (roof["kernel"] == "k_window" and prec_name == "fp32c" and cup_costs(prec_name, r)[1] == 8
            and pl["cells_per_lane"] == 32 and not pl["exchange_steps"]
            and pl["register_form"] in (1, 2)):
        roof["kernel"] = "k_window_c0_lone32"
    roof["traffic"] = measured_traffic(roof["kernel"], workload, prec_name, pl)
    roof["avg_launch_ms"] = round(k_avg_ms, 4)
    roof["avg_launch_ms_kernel_only"] = round(k_alone_ms, 4)
    roof["launches_per_step"] = launches

    err = None
    del d_u, d_work
    torch.cuda.empty_cache()
    if prec != heat.FP64:
        err = precision_report(heat, torch, u0, nparts, r, nt, prec, stream)
    out = {
        "metric": "GCUP/s (giga cell-updates per second)",
        "value": round(value, 3),
        "unit": "GCUP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32c": "f32 (compensated)"}[prec_name],
        "data": "synthetic",
        "config": {"workload": workload, "N": N, "nparts": nparts, "r": r, "nt": nt,
                   "init": w["init"], "seed": w["seed"], "precision": prec_name, "launch": launch,
                   "kernel": roof["kernel"], "cells_per_lane": pl["cells_per_lane"],
                   "steps_per_round": pl["steps_per_round"],
                   "waves_per_group": pl["waves_per_group"],
                   "register_form": pl["register_form"],
                   "exchange_steps": pl["exchange_steps"]},
        "roofline": roof,
    }
    if err is not None:
        out["error_vs_fp64"] = err
    if host and prec_name == "fp64" and not cfg.get("kernel"):
        out["host_path"] = host_path(heat, u0, nparts, r, nt)
    return out, u0


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_2307_01117_amd import heat, inputs

    heat.load()
    if args.form == "batch":
        return bench_batch(args)
    if args.form == "serve":
        return bench_serve(args)
    if args.ring:
        f = args.ring.split(",")
        N_, nt_ = int(float(f[0])), int(float(f[1]))
        args.workload = f"ring_{f[0]}_{f[1]}_steps"
        inputs.WORKLOADS[args.workload] = dict(N=N_, nparts=1, r=float(f[2]) if len(f) > 2 else 0.5,
                                               nt=nt_, init="uniform", seed=3)
    w = inputs.WORKLOADS[args.workload]
    prec_name = args.precision or ("fp64" if args.workload != "ring_1e8_perturbed" else "fp32c")
    prec = heat.PRECISIONS[prec_name]
    kernel = {"auto": 0, "tb": heat.KERNEL_TB, "step": heat.KERNEL_STEP,
              "resident": heat.KERNEL_RESIDENT}[args.kernel]
    exchange = {"auto": 0, "none": heat.EXCHANGE_NONE, "lds": heat.EXCHANGE_LDS,
                "deep": heat.EXCHANGE_LDS_DEEP}[args.exchange]
    cfg = dict(kernel=kernel, cells_per_lane=args.cells_per_lane,
               steps_per_round=args.steps_per_round, waves_per_group=args.waves_per_group,
               register_form=args.register_form, exchange=exchange)

    if args.copy_probe:
        N = w["N"]
        dt = torch.float64 if prec == heat.FP64 else torch.float32
        d_u = torch.from_numpy(inputs.make_initial(w["init"], N, w["seed"])).to("cuda", dtype=dt)
        d_work = torch.empty_like(d_u)
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        heat.copy_dev(d_u, d_work, stream)
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(args.steps):
            heat.copy_dev(d_u, d_work, stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / args.steps
        nbytes = d_u.numel() * d_u.element_size()
        print(json.dumps({"copy_bytes": nbytes, "avg_launch_ms": round(ms, 4),
                          "GBs": round(2 * nbytes / ms / 1e6, 1)}), flush=True)
        return

    out, u0 = run_plain(args, args.workload, prec_name, args.steps, args.warmup, cfg,
                        host=not args.no_host_path)
    torch.cuda.empty_cache()
    N, nt, r = w["N"], w["nt"], w["r"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(u0, r, args.cpu_steps, prec_name,
                                           heat.plan(N, nt, prec)["steps_per_round"])
    if not args.no_cpu_threads and prec_name == "fp64" and args.cpu_thread_steps > 0:
        out["cpu_threads"] = cpu_threads(u0, r, args.cpu_thread_steps, args.workload)
    del u0
    # The rest of the metric on the same GPU, in the same line: the precision
    # form on its workload, the batching form and a serving run, each against
    # the plain form (default run only).
    if args.workload == "ring_1e8" and prec_name == "fp64" and not kernel and \
            not args.no_sub_records:
        out["precision"] = sub_precision(args)
        torch.cuda.empty_cache()
        out["batch"] = sub_batch(args)
        torch.cuda.empty_cache()
        out["serve"] = sub_serve(args)
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def sub_precision(args):
    """The precision form on its workload (1e8-cell perturbed ring, r 1/4,
    1,000 steps): compensated binary32 (and plain binary32 for comparison)
    timed like the plain line, with the whole-ring error against binary64."""
    res = {}
    for name in ("fp32c", "fp32"):
        o, _ = run_plain(args, "ring_1e8_perturbed", name, 5, 2, {}, host=False)
        res[name] = {"value": o["value"], "unit": "GCUP/s", "ms_per_step": o["ms_per_step"],
                     "config": {k: o["config"][k] for k in
                                ("cells_per_lane", "steps_per_round", "waves_per_group",
                                 "exchange_steps")},
                     "roofline": {k: o["roofline"][k] for k in
                                  ("bound", "achieved", "peak", "unit", "frac", "avg_launch_ms",
                                   "traffic")},
                     "error_vs_fp64": o["error_vs_fp64"]}
    res["workload"] = "ring_1e8_perturbed (N 1e8, r 0.25, 1,000 steps, 1 + 1e-3*U[-1,1) seed 2)"
    res["error_metric"] = "max |x - y| / max |y| over the whole ring, y the binary64 result"
    return res


def sub_batch(args, count=4096, steps=3):
    """The batching form on its workload (4,096 rings): binary64 batched
    against the same rings solved one by one with the plain device form, and
    the compensated binary32 batch with the error of every ring against the
    binary64 batch (bit-identical to the oracle ring by ring)."""
    import numpy as np
    import torch

    from paper_2307_01117_amd import heat, inputs
    specs = inputs.batch_specs(count=count, seed=4)
    cups = sum(s.N * s.nt for s in specs)
    stream = torch.cuda.current_stream()
    u0 = [torch.from_numpy(inputs.ring_initial(s)).cuda() for s in specs]
    out = {"workload": f"batch_{count}_rings (N log-uniform [1e3, 1e6], nt uniform "
                       "[100, 10000], r in (0.1, 0.5], U[0,1) per ring)",
           "rings": count, "cell_updates": cups}
    res = {}
    for name, dt in (("fp64", torch.float64), ("fp32c", torch.float32)):
        prec = heat.PRECISIONS[name]
        us = [u.to(dt, copy=True) for u in u0]     # never an alias of the initial states
        ws = [torch.empty_like(u) for u in us]
        rings = [(u, w, s.nt, s.r, prec) for u, w, s in zip(us, ws, specs)]
        heat.solve_batch_dev(rings, stream=stream)        # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            heat.solve_batch_dev(rings, stream=stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rec = {"value": round(cups * steps / el / 1e9, 1), "unit": "GCUP/s",
               "ms_per_step": round(el * 1e3 / steps, 1)}
        if name == "fp64":
            # the same rings one by one with the plain device form
            for u, w, s in zip(us, ws, specs):
                heat.solve_dev(u, s.nparts, s.r, s.nt, precision=prec, stream=stream, work=w)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for u, w, s in zip(us, ws, specs):
                heat.solve_dev(u, s.nparts, s.r, s.nt, precision=prec, stream=stream, work=w)
            torch.cuda.synchronize()
            plain_s = time.perf_counter() - t1
            rec["plain_one_by_one"] = round(cups / plain_s / 1e9, 1)
            rec["batched_vs_plain"] = round(rec["value"] / rec["plain_one_by_one"], 3)
        # one pass from the initial states, kept for the error
        for u, a in zip(us, u0):
            u.copy_(a)
        heat.solve_batch_dev(rings, stream=stream)
        torch.cuda.synchronize()
        res[name] = (rec, us)
        del ws, rings
    ref = res["fp64"][1]
    errs = np.array([float((c.double() - f).abs().max() / f.abs().max())
                     for c, f in zip(res["fp32c"][1], ref)])
    out["fp64"] = res["fp64"][0]
    out["fp32c"] = res["fp32c"][0]
    out["fp32c"]["error_vs_fp64"] = {"rings": int(errs.size), "max": float(errs.max()),
                                     "p99": float(np.percentile(errs, 99)),
                                     "median": float(np.median(errs)),
                                     "metric": "per ring max |x - y| / max |y|"}
    out["fp32c"]["vs_fp64_batched"] = round(out["fp32c"]["value"] / out["fp64"]["value"], 3)
    return out


def sub_serve(args, rate=200.0, duration=15.0, warm_s=2.0):
    """A short serving run in the default line (200 requests/s for 15 s)."""
    return serve_rate(rate, duration, warm_s, check_every=23)


def bench_batch(args):
    """Batching form: all rings advance together; reported against the same
    rings solved one after another with the plain device form."""
    import torch

    from paper_2307_01117_amd import heat, inputs
    prec_name = args.precision or "fp64"
    prec = heat.PRECISIONS[prec_name]
    dt = torch.float64 if prec == heat.FP64 else torch.float32
    specs = inputs.batch_specs(count=args.batch_count, seed=4)
    us = [torch.from_numpy(inputs.ring_initial(s)).to("cuda", dtype=dt) for s in specs]
    ws = [torch.empty_like(u) for u in us]
    cups = sum(s.N * s.nt for s in specs)
    stream = torch.cuda.current_stream()
    rings = [(u, w, s.nt, s.r, prec) for u, w, s in zip(us, ws, specs)]
    kw = dict(graph=args.batch_mode == "graph", persistent=args.batch_mode == "persistent")

    def batch_step():
        heat.solve_batch_dev(rings, stream=stream, wait=True, **kw)

    def plain_step():
        for u, w, s in zip(us, ws, specs):
            heat.solve_dev(u, s.nparts, s.r, s.nt, precision=prec, stream=stream, work=w)
        torch.cuda.synchronize()

    for _ in range(args.warmup):
        batch_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch_step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    plain_s = None
    if not args.no_plain_compare:
        plain_step()
        t1 = time.perf_counter()
        plain_step()
        plain_s = time.perf_counter() - t1
    value = cups * args.steps / elapsed / 1e9
    print(json.dumps({
        "metric": "GCUP/s (giga cell-updates per second), batched",
        "value": round(value, 3), "unit": "GCUP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32c": "f32 (compensated)"}[prec_name],
        "data": "synthetic",
        "config": {"workload": f"batch_{args.batch_count}_rings", "rings": len(specs),
                   "cell_updates": cups, "precision": prec_name, "mode": args.batch_mode},
        "plain_one_by_one": None if plain_s is None else {
            "value": round(cups / plain_s / 1e9, 3), "unit": "GCUP/s", "seconds": round(plain_s, 3)},
        "batched_vs_plain": None if plain_s is None else round(value / (cups / plain_s / 1e9), 3),
    }), flush=True)


_SERVE_POOL = None


def serving_pool():
    """Pinned host pool the requests take their initial states from:
    u0[i] = pool[(off + i) mod P] as one contiguous slice (the pool's first
    10 million values are repeated at its end), plus a pinned sink for the
    results that are not checked."""
    global _SERVE_POOL
    if _SERVE_POOL is None:
        import torch

        from paper_2307_01117_amd import inputs
        P, nmax = 1 << 24, 10_000_000
        pool = torch.empty(P + nmax, dtype=torch.float64, pin_memory=True).numpy()
        pool[:P] = inputs.serving_pool(P)
        pool[P:] = pool[:nmax]
        sink = torch.empty(nmax, dtype=torch.float64, pin_memory=True).numpy()
        _SERVE_POOL = (pool, sink, P)
    return _SERVE_POOL


def serve_rate(rate, duration, warm_s, check_every=97):
    """Poisson arrivals of heat-solve requests (N log-uniform in [1e3, 1e7],
    nt uniform in [100, 5000], r in (0.1, 0.5], FP64 or compensated FP32 with
    probability 1/2) into one continuous-batching server for `duration`
    seconds.  Latency = completion - scheduled arrival.  Every
    `check_every`-th request keeps its own result, which is compared with the
    same request solved alone (same precision: bitwise) and, for compensated
    FP32 requests, with the request solved alone in binary64 (error)."""
    import numpy as np
    import torch

    from paper_2307_01117_amd import heat, inputs
    pool, sink, P = serving_pool()
    trace = inputs.serving_trace(rate, duration, pool_size=P)
    server = heat.Server()
    submitted = []          # (req, ticket, t_submit_rel, checked)
    rejected = 0
    t0 = time.perf_counter()
    for k, q in enumerate(trace):
        delay = t0 + q.t_arrival - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        u0 = pool[q.offset:q.offset + q.N]
        check = k % check_every == 0
        out = np.empty(q.N) if check else sink[:q.N]
        try:
            t = server.submit(u0, q.nt, q.r, q.precision, out=out)
        except heat.HeatError as e:
            if e.code != heat.HEAT_EBUSY:
                raise
            rejected += 1
            continue
        submitted.append((q, t, time.perf_counter() - t0, check))
    results = [(q, server.wait(t), ts, check) for (q, t, ts, check) in submitted]
    t_end = time.perf_counter() - t0
    stats = server.stats()
    server.close()
    lat = []
    cups = 0
    for q, res, ts, _ in results:
        cups += q.N * q.nt
        if q.t_arrival >= warm_s:
            lat.append((ts - q.t_arrival) + res.latency_s)
    lat = np.sort(np.array(lat)) if lat else np.array([float("nan")])
    # alone vs in the mix, and the compensated requests' error against binary64
    same = total = 0
    errs = []
    for q, res, _, check in results:
        if not check:
            continue
        dt = torch.float64 if q.precision == heat.FP64 else torch.float32
        src = torch.from_numpy(pool[q.offset:q.offset + q.N]).to("cuda")
        d = src.to(dt)
        heat.solve_dev(d, 1, q.r, q.nt, precision=q.precision)
        total += 1
        same += int(np.array_equal(d.double().cpu().numpy().view(np.uint64),
                                   res.u.view(np.uint64)))
        if q.precision == heat.FP32C:
            heat.solve_dev(src, 1, q.r, q.nt, precision=heat.FP64)
            got = torch.from_numpy(res.u).to("cuda")
            errs.append(float((got - src).abs().max() / src.abs().max()))
            del got
        del src, d
    offered = sum(q.N * q.nt for q in trace) / duration / 1e9
    return {
        "rate_req_s": rate, "value": round(cups / t_end / 1e9, 3), "unit": "GCUP/s",
        "duration_s": duration, "requests": len(trace), "completed": len(results),
        "rejected_busy": rejected,
        "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
        "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
        "latency_max_s": round(float(lat[-1]), 4),
        "latency_from_s": warm_s,
        "offered_GCUPs": round(offered, 1), "wall_s": round(t_end, 2),
        "ticks": stats["ticks"], "hbm_peak_GB": round(stats["hbm_peak"] / 1e9, 2),
        "alone_vs_mix_bitwise": f"{same}/{total}",
        "fp32c_error_vs_fp64": {
            "requests": len(errs),
            "max": max(errs) if errs else None,
            "p99": float(np.percentile(errs, 99)) if errs else None,
            "metric": "per checked request max |x - y| / max |y|, y the request solved "
                      "alone in binary64"},
        "config": {"workload": "poisson_serving", "N": "log-uniform [1e3, 1e7]",
                   "nt": "uniform [100, 5000]", "precision": "fp64 or fp32c (p = 1/2)",
                   "checked": f"every {check_every}th request"},
    }


def bench_serve(args):
    """Serving form: one JSON line per arrival rate (see serve_rate)."""
    for rate in [float(x) for x in args.rates.split(",")]:
        o = serve_rate(rate, args.duration, args.warm_s)
        line = {"metric": "serving: p50/p99 latency and GCUP/s", "n_gpus": 1,
                "higher_is_better": True, "data": "synthetic"}
        line.update(o)
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
