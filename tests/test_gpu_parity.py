"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

binary64 and plain binary32 results must be bit-identical to the oracle (the
kernels evaluate every cell with the same operations in the same order);
the compensated binary32 form must be bit-identical to the oracle's
compensated form with the same round length T, and within 1e-6 relative of
the binary64 oracle.  Full-size rings are compared at sampled cells through
the oracle's light-cone evaluation, which is bit-identical to the full ring.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2307_01117_amd import heat, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def same_bits(a, b):
    """Bit-for-bit equality of two arrays (np.array_equal takes -0.0 == +0.0).
    A binary32 array compared with a binary64 one is widened first, which is
    exact and keeps the sign of zero."""
    a, b = np.asarray(a), np.asarray(b)
    if a.shape != b.shape:
        return False
    if a.dtype != b.dtype and a.dtype.kind == "f" and b.dtype.kind == "f":
        a, b = a.astype(np.float64), b.astype(np.float64)
    if a.dtype.kind == "f":
        it = {4: np.uint32, 8: np.uint64}[a.dtype.itemsize]
        return bool(np.array_equal(np.ascontiguousarray(a).view(it),
                                   np.ascontiguousarray(b).view(it)))
    return bool(np.array_equal(a, b))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    heat.load()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def run_dev(u0, nt, r, precision=heat.FP64, nparts=1, **cfg):
    dt = torch.float64 if precision == heat.FP64 else torch.float32
    d = dev(u0, dt)
    heat.solve_dev(d, nparts, r, nt, precision=precision, **cfg)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def cfgs_fp64():
    return [
        dict(),
        dict(kernel=heat.KERNEL_STEP),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=8, steps_per_round=4),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=8, steps_per_round=16, waves_per_group=1),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=16, steps_per_round=32, waves_per_group=8),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=32, steps_per_round=64),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=32, steps_per_round=8, waves_per_group=2),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=32, steps_per_round=96, register_form=3),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=64, steps_per_round=128, register_form=3),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=64, steps_per_round=20, register_form=1,
             waves_per_group=1),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=16, steps_per_round=12, register_form=3,
             waves_per_group=8),
        # waves of a workgroup sharing one tile (LDS edge exchange every K/4 steps)
        dict(kernel=heat.KERNEL_TB, cells_per_lane=16, steps_per_round=12, waves_per_group=2,
             exchange=heat.EXCHANGE_LDS),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=32, steps_per_round=36, waves_per_group=4,
             register_form=1, exchange=heat.EXCHANGE_LDS),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=32, steps_per_round=20, waves_per_group=8,
             register_form=2, exchange=heat.EXCHANGE_LDS),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=64, steps_per_round=124, waves_per_group=4,
             register_form=3, exchange=heat.EXCHANGE_LDS),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=64, steps_per_round=60, waves_per_group=6,
             register_form=3, exchange=heat.EXCHANGE_LDS),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=16, steps_per_round=12, waves_per_group=3,
             register_form=2, exchange=heat.EXCHANGE_LDS),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=8, steps_per_round=8, waves_per_group=5),
        # the deep exchange (every K/2 steps, overlap K)
        dict(kernel=heat.KERNEL_TB, cells_per_lane=8, steps_per_round=60, waves_per_group=8,
             exchange=heat.EXCHANGE_LDS_DEEP),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=8, steps_per_round=12, waves_per_group=3,
             register_form=1, exchange=heat.EXCHANGE_LDS_DEEP),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=16, steps_per_round=60, waves_per_group=4,
             exchange=heat.EXCHANGE_LDS_DEEP),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=32, steps_per_round=36, waves_per_group=2,
             register_form=2, exchange=heat.EXCHANGE_LDS_DEEP),
        dict(kernel=heat.KERNEL_TB, cells_per_lane=64, steps_per_round=124, waves_per_group=4,
             register_form=3, exchange=heat.EXCHANGE_LDS_DEEP),
    ]


N_CFGS = len(cfgs_fp64())


# ------------------------------------------------------------ tiny rings

@pytest.mark.parametrize("ci", range(N_CFGS))
def test_tiny_rings_bitwise(ci):
    """Every ring length 1..70 (windows wrap the ring many times), run lengths
    around the round length, several r: bit-identical to the oracle."""
    cfg = cfgs_fp64()[ci]
    for N in list(range(1, 71)) + [127, 128, 129, 511, 513]:
        u0 = inputs.uniform_ring(N, (20, N))
        for nt, r in ((0, 0.5), (1, 0.5), (3, 0.25), (33, 0.5), (70, 0.3)):
            got = run_dev(u0, nt, r, **cfg)
            want = oracle.solve(u0, r, nt)
            assert same_bits(got, want), (cfg, N, nt, r)


def test_exact_small_integer_cases():
    """Dyadic r and integer states: the exact rational result (pinned in the
    oracle tests) is reproduced bit for bit."""
    for N in (1, 2, 3, 7, 16, 100):
        u0 = inputs.small_integer_ring(N, (21, N))
        for r in (0.0, 0.125, 0.25, 0.375, 0.5):
            for cfg in cfgs_fp64()[:3]:
                assert same_bits(run_dev(u0, 12, r, **cfg), oracle.solve(u0, r, 12))


def test_host_form_staged_copies():
    """heat_solve on host arrays past the size where the copies go through the
    pinned multi-lane staging (64 MiB): a ragged length that leaves a short
    last chunk in every lane, bit-identical to the oracle; nt = 0 returns the
    input bit for bit through both directions of the staging; a small ring
    takes the plain copy."""
    N = 10_000_019
    u0 = inputs.uniform_ring(N, 77)
    want = oracle.solve(u0, 0.375, 7)
    assert same_bits(heat.solve(u0, 3, 0.375, 7), want)
    a = u0.copy()
    assert heat.solve(a, 3, 0.375, 7, inplace=True) is a and same_bits(a, want)
    assert same_bits(heat.solve(u0, 1, 0.5, 0), u0)
    small = inputs.uniform_ring(1000, 78)
    assert same_bits(heat.solve(small, 2, 0.25, 9), oracle.solve(small, 0.25, 9))


# ------------------------------------------------------------ mid-size, ragged

@pytest.mark.parametrize("N", [1000, 4097, 100_003, 262_144 + 77])
def test_midsize_fp64_all_kernels(N):
    u0 = inputs.uniform_ring(N, (22, N))
    nt, r = 75, 0.5
    want = oracle.solve(u0, r, nt)
    for cfg in cfgs_fp64():
        got = run_dev(u0, nt, r, **cfg)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, (cfg, N, bad[:10])


@pytest.mark.parametrize("N", [999, 65_536 + 13, 300_001])
def test_midsize_fp32_bitwise(N):
    u0 = inputs.perturbed_ring(N, (23, N)).astype(np.float32)
    nt, r = 70, 0.25
    want = oracle.solve_f32(u0, r, nt)
    for cfg in (dict(), dict(kernel=heat.KERNEL_STEP), dict(cells_per_lane=8, steps_per_round=20),
                dict(cells_per_lane=16, steps_per_round=32),
                dict(cells_per_lane=64, steps_per_round=96, register_form=2),
                dict(cells_per_lane=64, steps_per_round=96, register_form=3),
                dict(cells_per_lane=32, steps_per_round=36, register_form=3),
                dict(cells_per_lane=32, steps_per_round=36, waves_per_group=4, register_form=1,
                     exchange=heat.EXCHANGE_LDS),
                dict(cells_per_lane=16, steps_per_round=16, waves_per_group=2, register_form=3,
                     exchange=heat.EXCHANGE_LDS),
                dict(cells_per_lane=8, steps_per_round=32, waves_per_group=8, register_form=3,
                     exchange=heat.EXCHANGE_LDS_DEEP),
                dict(cells_per_lane=64, steps_per_round=96, waves_per_group=4, register_form=1,
                     exchange=heat.EXCHANGE_LDS_DEEP)):
        got = run_dev(u0, nt, r, precision=heat.FP32, **cfg)
        assert same_bits(got, want), (cfg, N)


@pytest.mark.parametrize("N", [1, 5, 999, 65_536 + 13, 300_001])
def test_midsize_fp32c_bitwise(N):
    u0 = inputs.perturbed_ring(N, (24, N)).astype(np.float32)
    r = 0.25
    for nt in (7, 100):
        T = heat.plan(N, nt, heat.FP32C)["steps_per_round"]
        want = oracle.solve_f32c(u0, r, nt, T)
        for K, form, wpg, x in ((8, 1, 0, 0), (16, 2, 0, 0), (32, 3, 0, 0), (64, 3, 0, 0),
                                (64, 1, 0, 0), (32, 1, 4, heat.EXCHANGE_NONE),
                                (32, 2, 1, heat.EXCHANGE_NONE), (16, 3, 2, heat.EXCHANGE_LDS),
                                (32, 2, 4, heat.EXCHANGE_LDS), (32, 3, 8, heat.EXCHANGE_LDS),
                                (64, 3, 4, heat.EXCHANGE_LDS), (8, 1, 8, heat.EXCHANGE_LDS_DEEP),
                                (16, 3, 4, heat.EXCHANGE_LDS_DEEP),
                                (32, 1, 4, heat.EXCHANGE_LDS_DEEP)):
            got = run_dev(u0, nt, r, precision=heat.FP32C, cells_per_lane=K, register_form=form,
                          waves_per_group=wpg, exchange=x)
            assert same_bits(got, want), (K, form, wpg, x, N, nt)


@pytest.mark.parametrize("wpg", [1, 2, 4, 8])
def test_fp32c_binary32_coefficient_lone32(wpg):
    """The compensated form's binary32-coefficient kernel for 32-cell lone
    waves (the ping-pong sweep held to 3 waves per SIMD, taken for register
    forms 1 and 2): the oracle's bits over many tiles with a ragged tail, odd
    step counts (the sweep's single-step tail), an array that is not 16-byte
    aligned (the cell-by-cell path) and the fused checksums; and the same bits
    as the alternating form, which runs the general kernel family."""
    N = 200_003
    u0 = inputs.perturbed_ring(N, (27, wpg)).astype(np.float32)
    T = heat.plan(N, 10**6, heat.FP32C)["steps_per_round"]   # the form's fixed round length
    for r in (0.25, 0.375, 0.125):
        for nt in (7, 64, 129):
            want = oracle.solve_f32c(u0, r, nt, T)
            cfgs = [dict(cells_per_lane=32, waves_per_group=wpg, exchange=heat.EXCHANGE_NONE,
                         register_form=f, steps_per_round=T) for f in (1, 2, 3)]
            for cfg in cfgs:
                got = run_dev(u0, nt, r, precision=heat.FP32C, **cfg)
                assert same_bits(got, want), (cfg, r, nt)
            # unaligned: one cell into a larger buffer
            buf = torch.zeros(N + 1, dtype=torch.float32, device="cuda")
            d = buf[1:]
            d.copy_(torch.from_numpy(u0))
            s0, s1 = heat.solve_dev(d, 1, r, nt, precision=heat.FP32C, sums=True, **cfgs[0])
            assert same_bits(d.cpu().numpy(), want), ("unaligned", r, nt)
            assert abs(s0 - math.fsum(u0.astype(np.float64))) <= 1e-12 * abs(s0)
            assert abs(s1 - math.fsum(want.astype(np.float64))) <= 1e-12 * abs(s1)
            del buf, d


def test_signed_zeros_fp32_forms():
    """A state of +0 and -0 cells among small dyadic values: both binary32
    forms reach the oracle's bits, the signs of zeros included, on the
    one-step kernel and in every register form with lone and cooperating
    waves."""
    N = 70_001
    rng = np.random.default_rng([25, N])
    u0 = (rng.integers(-2, 3, N) * 2.0 ** -20).astype(np.float32)
    z = u0 == 0
    u0[z] = np.where(rng.random(int(z.sum())) < 0.5, np.float32(0.0), np.float32(-0.0))
    assert np.signbit(u0[z]).any() and (~np.signbit(u0[z])).any()
    shapes = [dict(kernel=heat.KERNEL_STEP)] + [
        dict(cells_per_lane=K, register_form=f, waves_per_group=g, exchange=x)
        for K in (8, 32, 64) for f in (1, 2, 3)
        for (g, x) in ((1, heat.EXCHANGE_NONE), (4, heat.EXCHANGE_LDS),
                       (4, heat.EXCHANGE_LDS_DEEP))
        if not (x == heat.EXCHANGE_LDS and K < 16) and not (K == 64 and f == 2)]
    for r in (0.25, 0.375):
        for nt in (1, 9, 130):
            want = oracle.solve_f32(u0, r, nt)
            T = heat.plan(N, nt, heat.FP32C)["steps_per_round"]
            want_c = oracle.solve_f32c(u0, r, nt, T)
            for cfg in shapes:
                got = run_dev(u0, nt, r, precision=heat.FP32, **cfg)
                assert same_bits(got, want), ("fp32", cfg, r, nt)
                if cfg.get("kernel") == heat.KERNEL_STEP:
                    continue
                got = run_dev(u0, nt, r, precision=heat.FP32C, **cfg)
                assert same_bits(got, want_c), ("fp32c", cfg, r, nt)


def test_golden_ramp_exact_on_gpu():
    """The stored exact solutions for the paper's ramp initial condition
    (tests/golden/ramp_exact.txt, rational arithmetic from the definition)
    through the C ABI in every kernel family: bit for bit."""
    import os
    from fractions import Fraction
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ramp_exact.txt")
    cases = []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            f = line.split()
            N, r, nt = int(f[0]), float(Fraction(f[1])), int(f[2])
            cases.append((N, r, nt, np.array([float(Fraction(x)) for x in f[3:3 + N]])))
    assert len(cases) >= 4
    for N, r, nt, want in cases:
        u0 = np.arange(N, dtype=np.float64)
        for cfg in (dict(), dict(kernel=heat.KERNEL_STEP),
                    dict(cells_per_lane=8, steps_per_round=4, register_form=1),
                    dict(cells_per_lane=32, steps_per_round=8, waves_per_group=4,
                         exchange=heat.EXCHANGE_LDS)):
            assert same_bits(run_dev(u0, nt, r, **cfg), want), (N, r, nt, cfg)


def test_device_form_from_many_threads():
    """The device form called from several host threads at once, each on its
    own stream and with checksums (per-thread checksum scratch, the shared
    stream-ordered pool): every result bit for bit the oracle's and every
    pair of sums equal to the exact sums."""
    import math
    import threading
    cases = [(50_000 + 7919 * k, 40 + 9 * k, 0.5 - 0.05 * k, heat.FP64 if k % 2 == 0 else heat.FP32C)
             for k in range(8)]
    inputs_ = [inputs.uniform_ring(N, (63, k)) for k, (N, _, _, _) in enumerate(cases)]
    out, errs = {}, []

    def work(k):
        try:
            N, nt, r, prec = cases[k]
            st = torch.cuda.Stream()
            dt = torch.float64 if prec == heat.FP64 else torch.float32
            with torch.cuda.stream(st):
                d = torch.from_numpy(inputs_[k]).to("cuda", dtype=dt)
                for _ in range(3):      # repeated calls reuse the thread's scratch
                    d.copy_(torch.from_numpy(inputs_[k]).to("cuda", dtype=dt))
                    sums = heat.solve_dev(d, 1, r, nt, precision=prec, stream=st, sums=True)
                out[k] = (d.cpu().numpy(), sums)
        except Exception as e:   # reported below, on the main thread
            errs.append((k, e))

    threads = [threading.Thread(target=work, args=(k,)) for k in range(len(cases))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errs, errs
    for k, (N, nt, r, prec) in enumerate(cases):
        got, (s0, s1) = out[k]
        if prec == heat.FP64:
            want = oracle.solve(inputs_[k], r, nt)
            start = inputs_[k]
        else:
            T = heat.plan(N, nt, heat.FP32C)["steps_per_round"]
            start = inputs_[k].astype(np.float32)
            want = oracle.solve_f32c(start, r, nt, T)
        assert same_bits(got, want), (k, N, nt, prec)
        assert abs(s0 - math.fsum(start.astype(np.float64))) <= 1e-12 * abs(s0), k
        assert abs(s1 - math.fsum(want.astype(np.float64))) <= 1e-12 * abs(s1), k


# ------------------------------------------------------------ invariances on the GPU

def test_partition_count_does_not_change_result():
    N = 50_001
    u0 = inputs.uniform_ring(N, 25)
    base = run_dev(u0, 40, 0.5, nparts=1)
    for P in (2, 10, 100, N):
        assert same_bits(run_dev(u0, 40, 0.5, nparts=P), base)


def test_shift_and_composition():
    N = 123_457
    u0 = inputs.uniform_ring(N, 26)
    base = run_dev(u0, 64, 0.37)
    for s in (1, 959, 960, 961, 65_536):
        assert same_bits(run_dev(np.roll(u0, s), 64, 0.37), np.roll(base, s))
    mid = run_dev(u0, 23, 0.37)
    assert same_bits(run_dev(mid, 41, 0.37), base)


def test_checksum_matches_exact_sum():
    for N in (1, 17, 1_000_000):
        u0 = inputs.uniform_ring(N, (27, N))
        s = heat.checksum_dev(dev(u0))
        exact = math.fsum(u0)
        assert abs(s - exact) <= 1e-13 * max(abs(exact), 1e-300)
        s32 = heat.checksum_dev(dev(u0, torch.float32), precision=heat.FP32)
        e32 = math.fsum(u0.astype(np.float32).astype(np.float64))
        assert abs(s32 - e32) <= 1e-13 * abs(e32)


def test_device_errors():
    d = dev(np.zeros(10))
    with pytest.raises(heat.HeatError) as ei:
        heat.solve_dev(d, 1, 0.75, 10)
    assert ei.value.code == heat.HEAT_EINVAL
    with pytest.raises(heat.HeatError):
        heat.solve_dev(dev(np.zeros(10), torch.float32), 1, 0.5, 10, precision=heat.FP32C,
                       kernel=heat.KERNEL_STEP)
    # host form agrees with the device form
    u0 = inputs.uniform_ring(1000, 28)
    assert same_bits(heat.solve(u0, 4, 0.5, 30), oracle.solve(u0, 0.5, 30))


# ------------------------------------------------------------ full-size workloads

def sample_cells(N, plan, rng, n=48):
    """Cells at and around tile edges, the edges between the waves of a tile
    (when they share it), the ring's wrap and random places."""
    W = plan["tile_cells"]
    s = {0, 1, N - 1, N - 2, N // 2}
    for t in (1, 2, N // W // 2, N // W - 1):
        for d in (-1, 0, 1):
            s.add((t * W + d) % N)
        S = plan["exchange_steps"]
        if S:
            K = plan["cells_per_lane"]
            H = (plan["waves_per_group"] * 64 * K - (plan["waves_per_group"] - 1) * 2 * S - W) // 2
            for w in range(1, plan["waves_per_group"]):
                edge = t * W + w * (64 * K - 2 * S) + S - H
                for d in (-1, 0, 1):
                    s.add((edge + d) % N)
    s.update(int(x) for x in rng.integers(0, N, n))
    return np.array(sorted(s), dtype=np.int64)


def test_ring_1e6_full_compare():
    """10 partitions x 100,000 cells, r = 1/2, 100 steps, Uniform[0,1) seed 0:
    the whole array, bit for bit, plus the conservation check."""
    w = inputs.WORKLOADS["ring_1e6"]
    u0 = inputs.make_initial(w["init"], w["N"], w["seed"])
    d = dev(u0)
    s0, s1 = heat.solve_dev(d, w["nparts"], w["r"], w["nt"], sums=True)
    got = d.cpu().numpy()
    want = oracle.solve(u0, w["r"], w["nt"])
    assert same_bits(got, want)
    assert abs(s1 - s0) <= 8 * 2.0 ** -53 * w["N"] * w["nt"]
    # the step kernel as well
    assert same_bits(run_dev(u0, w["nt"], w["r"], kernel=heat.KERNEL_STEP), want)


def test_sine_mode_decay_on_gpu():
    N, r, nt = 1_000_000, 0.5, 100
    u0 = inputs.sine_mode(N, 3)
    got = run_dev(u0, nt, r)
    g = math.cos(2 * math.pi * 3 / N)
    assert np.abs(got - g ** nt * u0).max() <= 1e-13


@pytest.mark.parametrize("cfg", [
    dict(kernel=heat.KERNEL_TB),
    dict(kernel=heat.KERNEL_STEP),
    dict(kernel=heat.KERNEL_TB, cells_per_lane=64, waves_per_group=4, register_form=3,
         exchange=heat.EXCHANGE_LDS),
    dict(kernel=heat.KERNEL_TB, cells_per_lane=64, waves_per_group=2, register_form=3,
         exchange=heat.EXCHANGE_NONE),
], ids=["tuned", "step", "k64-lds-exchange", "k64-lone-waves"])
def test_ring_1e8_sampled(cfg):
    """100 partitions x 1,000,000 cells, r = 1/2, 1,000 steps, Uniform[0,1)
    seed 1, in the launch configuration the benchmark times (the tuned one)
    and in explicit shapes: sampled cells bit for bit against light cones,
    and the binary64 sum conserved."""
    w = inputs.WORKLOADS["ring_1e8"]
    N = w["N"]
    u0 = inputs.make_initial(w["init"], N, w["seed"])
    d = dev(u0)
    s0, s1 = heat.solve_dev(d, w["nparts"], w["r"], w["nt"], sums=True, **cfg)
    pl = heat.plan(N, w["nt"], heat.FP64, **cfg)
    step = cfg["kernel"] == heat.KERNEL_STEP
    idx = sample_cells(N, pl, np.random.default_rng(31), n=8 if step else 24)
    got = d[torch.from_numpy(idx).cuda()].cpu().numpy()
    del d
    want = np.array([oracle.cone(u0, int(i), w["r"], w["nt"]) for i in idx])
    assert same_bits(got, want), idx[got != want][:10]
    assert abs(s0 - math.fsum(u0)) <= 1e-13 * abs(s0)
    assert abs(s1 - s0) <= 8 * 2.0 ** -53 * N * w["nt"]


def test_ring_1e8_whole_vs_threaded_oracle():
    """The headline workload (100 partitions x 1,000,000 cells, r = 1/2, 1,000
    steps, Uniform[0,1) seed 1) in the launch configuration the benchmark
    times, with its fused checksums: all 1e8 cells bit for bit against the
    oracle's threaded segmented solver (one segment per host thread, ghost
    cells through queues; bit-identical to the sequential oracle), about 20 s
    of host time on 16 cores."""
    w = inputs.WORKLOADS["ring_1e8"]
    N = w["N"]
    u0 = inputs.make_initial(w["init"], N, w["seed"])
    d = dev(u0)
    print("whole 1e8 ring: GPU pass", flush=True)
    s0, s1 = heat.solve_dev(d, w["nparts"], w["r"], w["nt"], sums=True)
    got = d.cpu().numpy()
    del d
    torch.cuda.empty_cache()
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    print(f"whole 1e8 ring: threaded oracle on {workers} threads", flush=True)
    want = oracle.solve_threads(u0, workers, w["r"], w["nt"])
    bad = np.flatnonzero(got.view(np.uint64) != want.view(np.uint64))
    assert bad.size == 0, (bad.size, bad[:10])
    assert abs(s1 - math.fsum(want)) <= 1e-13 * abs(s1)


@pytest.mark.parametrize("ci", range(N_CFGS))
def test_fused_checksums(ci):
    """The conservation checksum (fused into the first and last rounds of the
    temporal-blocked kernel, per wave): the sums of the state before and after
    equal the exact sums of the oracle's states to 1e-13."""
    cfg = cfgs_fp64()[ci]
    for N, nt in ((1, 3), (1000, 75), (100_003, 150)):
        u0 = inputs.uniform_ring(N, (29, N))
        d = dev(u0)
        s0, s1 = heat.solve_dev(d, 1, 0.5, nt, sums=True, **cfg)
        want = oracle.solve(u0, 0.5, nt)
        assert same_bits(d.cpu().numpy(), want), (cfg, N)
        assert abs(s0 - math.fsum(u0)) <= 1e-13 * max(abs(s0), 1.0), (cfg, N)
        assert abs(s1 - math.fsum(want)) <= 1e-13 * max(abs(s1), 1.0), (cfg, N)


def test_ring_1e8_perturbed_fp32_forms():
    """N = 1e8, r = 1/4, 1,000 steps, 1 + 1e-3*Uniform[-1,1) seed 2: the
    compensated form matches the oracle's compensated form bit for bit at
    sampled cells and stays within 1e-6 relative of binary64; plain binary32
    matches its oracle bit for bit."""
    w = inputs.WORKLOADS["ring_1e8_perturbed"]
    N, r, nt = w["N"], w["r"], w["nt"]
    u0 = inputs.make_initial(w["init"], N, w["seed"])
    u32 = u0.astype(np.float32)
    T = heat.plan(N, nt, heat.FP32C)["steps_per_round"]
    for prec in (heat.FP32C, heat.FP32):
        idx = sample_cells(N, heat.plan(N, nt, prec), np.random.default_rng(32), n=12)
        if prec == heat.FP32C:
            ref64 = np.array([oracle.cone(u32.astype(np.float64), int(i), r, nt) for i in idx])
        d = dev(u32, torch.float32)
        heat.solve_dev(d, w["nparts"], r, nt, precision=prec)
        got = d[torch.from_numpy(idx).cuda()].cpu().numpy()
        del d
        if prec == heat.FP32C:
            want = np.array([oracle.cone_f32c(u32, int(i), r, nt, T) for i in idx])
            assert same_bits(got, want)
            assert np.abs(got - ref64).max() / np.abs(ref64).max() <= 1e-6
        else:
            want = np.array([oracle.cone_f32(u32, int(i), r, nt) for i in idx])
            assert same_bits(got, want)


def test_autotuned_shape_is_result_neutral():
    """The autotuner's pick for a ring length runs and gives the oracle's bits."""
    N = 100_003
    cfg, g = heat.autotune(heat.FP64, N, install=False)
    assert g > 0 and cfg["kernel"] == heat.KERNEL_TB
    u0 = inputs.uniform_ring(N, 33)
    got = run_dev(u0, 150, 0.5, **cfg)
    assert same_bits(got, oracle.solve(u0, 0.5, 150))
    cfg32, _ = heat.autotune(heat.FP32C, 20_000, install=False)
    u32 = inputs.perturbed_ring(20_000, 34).astype(np.float32)
    T = heat.plan(20_000, 130, heat.FP32C)["steps_per_round"]
    assert cfg32["steps_per_round"] == heat.plan(20_000, 10**6, heat.FP32C)["steps_per_round"]
    got = run_dev(u32, 130, 0.25, precision=heat.FP32C, **cfg32)
    assert same_bits(got, oracle.solve_f32c(u32, 0.25, 130, T))


@pytest.mark.parametrize("nparts", [2, 20, 40])
def test_paper_ramp_workload(nparts):
    """The paper's benchmark run: 1,000,000 nodes, 1,000 steps, initial
    condition u(0, x_i) = x_i, the grid cut into 2..40 segments: bit-identical
    to the oracle for every segment count, conserved sum, bounded by the
    initial range (maximum principle, r <= 1/2)."""
    w = inputs.WORKLOADS["paper_ramp_1e6"]
    u0 = inputs.make_initial(w["init"], w["N"])
    d = dev(u0)
    s0, s1 = heat.solve_dev(d, nparts, w["r"], w["nt"], sums=True)
    got = d.cpu().numpy()
    if nparts == 2:
        assert same_bits(got, oracle.solve(u0, w["r"], w["nt"]))
        test_paper_ramp_workload.ref = got
    else:
        assert same_bits(got, test_paper_ramp_workload.ref)
    assert abs(s1 - s0) <= 1e-9 * abs(s0)
    delta = 4 * 2.0 ** -53 * w["nt"] * (w["N"] - 1)
    assert got.min() >= -delta and got.max() <= w["N"] - 1 + delta


def test_unaligned_device_array_takes_gather_path():
    """A device array that is not 16-byte aligned (a view one cell in) runs
    every tile through the cell-by-cell path: same bits."""
    N = 70_001
    u0 = inputs.uniform_ring(N, 35)
    base = torch.zeros(N + 1, dtype=torch.float64, device="cuda")
    base[1:] = torch.from_numpy(u0).cuda()
    view = base[1:]
    assert view.data_ptr() % 16 != 0
    want = oracle.solve(u0, 0.5, 90)
    for cfg in (dict(), dict(cells_per_lane=32, waves_per_group=4, exchange=heat.EXCHANGE_LDS)):
        view.copy_(torch.from_numpy(u0).cuda())
        heat.solve_dev(view, 1, 0.5, 90, **cfg)
        assert same_bits(view.cpu().numpy(), want), cfg
    v32 = torch.zeros(N + 1, dtype=torch.float32, device="cuda")
    u32 = u0.astype(np.float32)
    v32[1:] = torch.from_numpy(u32).cuda()
    heat.solve_dev(v32[1:], 1, 0.25, 70, precision=heat.FP32C)
    T = heat.plan(N, 70, heat.FP32C)["steps_per_round"]
    assert same_bits(v32[1:].cpu().numpy(), oracle.solve_f32c(u32, 0.25, 70, T))


@pytest.mark.parametrize("prec", [heat.FP32, heat.FP32C, heat.FP64])
def test_ring_beyond_2_pow_31_cells(prec):
    """Largest size class: 2^31 + 12,345 cells (64-bit tile and cell indices
    everywhere; 52 GB of HBM in binary64), a few steps, lone and cooperating
    waves; sampled cells against light cones of the initial state (drawn
    with torch on the device, copied out before the solve)."""
    N = (1 << 31) + 12_345
    dt = torch.float64 if prec == heat.FP64 else torch.float32
    g = torch.Generator(device="cuda").manual_seed(36)
    d = torch.rand(N, generator=g, device="cuda", dtype=dt)
    nt, r = 20, 0.25
    rng = np.random.default_rng(37)
    idx = sorted({0, 1, N - 1, N - 2, (1 << 31) - 1, 1 << 31, (1 << 31) + 1} |
                 {int(x) for x in rng.integers(0, N, 16)})
    wins = {}
    for i in idx:
        w = torch.arange(i - nt, i + nt + 1, device="cuda") % N
        wins[i] = d[w].cpu().numpy()
    d2 = d.clone()
    heat.solve_dev(d, 1, r, nt, precision=prec)
    # and with the waves of a workgroup sharing tiles
    heat.solve_dev(d2, 1, r, nt, precision=prec, cells_per_lane=32, waves_per_group=4,
                   exchange=heat.EXCHANGE_LDS)
    T = heat.plan(N, nt, prec)["steps_per_round"]
    for i in idx:
        if prec == heat.FP32:
            want = np.float32(oracle.cone_f32(wins[i], nt, r, nt))
        elif prec == heat.FP32C:
            want = np.float32(oracle.cone_f32c(wins[i], nt, r, nt, T))
        else:
            want = np.float64(oracle.cone(wins[i], nt, r, nt))
        got = np.array([d[i].item(), d2[i].item()], dtype=want.dtype)
        assert same_bits(got, np.array([want, want])), (i, prec)
    del d, d2
    torch.cuda.empty_cache()


def test_copy_probe_and_device_info():
    info = heat.device_info()
    assert info["wave_size"] == 64 and info["cus"] >= 1
    a = torch.rand(1 << 20, device="cuda", dtype=torch.float64)
    b = torch.empty_like(a)
    heat.copy_dev(a, b)
    torch.cuda.synchronize()
    assert same_bits(a.cpu().numpy(), b.cpu().numpy())
