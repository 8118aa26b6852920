"""GPU parity of the batching form (many uneven rings advanced together: one
launch per round over all running rings, or one persistent launch) through
the C ABI: every ring must come out bit-identical to the CPU oracle and to the
same ring solved alone by the plain device form."""
import math
import os
import time
from concurrent.futures import ThreadPoolExecutor

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


def oracle_for(prec, u0, r, nt):
    if prec == heat.FP64:
        return oracle.solve(u0, r, nt)
    u32 = u0.astype(np.float32)
    if prec == heat.FP32:
        return oracle.solve_f32(u32, r, nt).astype(np.float64)
    T = heat.plan(u0.size, nt, heat.FP32C)["steps_per_round"]
    return oracle.solve_f32c(u32, r, nt, T).astype(np.float64)


def mixed_problems(seed, count, nmax, ntmax, precs):
    rng = np.random.default_rng(seed)
    probs = []
    for k in range(count):
        N = int(rng.integers(1, nmax)) if k % 3 else int(rng.integers(1, 70))
        nt = int(rng.integers(0, ntmax))
        r = float(0.5 - 0.4 * rng.random())
        prec = int(precs[k % len(precs)])
        u0 = inputs.uniform_ring(N, (40, seed, k))
        probs.append(dict(u0=u0, nparts=1, r=r, nt=nt, precision=prec))
    return probs


@pytest.mark.parametrize("precs", [[heat.FP64], [heat.FP32], [heat.FP32C],
                                   [heat.FP64, heat.FP32C, heat.FP32]])
def test_host_batch_matches_oracle(precs):
    probs = mixed_problems(41 + len(precs) + precs[0], 40, 30_000, 300, precs)
    res = heat.solve_batch(probs)
    for p, q in zip(probs, res):
        assert q.status == heat.HEAT_OK
        want = oracle_for(p["precision"], p["u0"], p["r"], p["nt"])
        assert same_bits(q.u, want), (p["u0"].size, p["nt"], p["precision"])
        if p["precision"] == heat.FP64:
            s0 = math.fsum(p["u0"])
        else:
            s0 = math.fsum(p["u0"].astype(np.float32).astype(np.float64))
        assert abs(q.sum0 - s0) <= 1e-13 * max(abs(s0), 1.0)
        assert abs(q.sum_nt - math.fsum(want)) <= 1e-13 * max(abs(s0), 1.0)


def test_host_batch_staged_copies():
    """A host batch of more than 64 MiB, whose copies go through the pinned
    multi-lane staging as one byte stream: four rings of 1e6-3e6 cells (each
    spanning chunks and lanes) among 60 small ones (many per chunk), empty
    steps and every precision; bit-identical to the oracle."""
    rng = np.random.default_rng(91)
    sizes = [3_000_017, 2_500_001, 1_999_999, 1_000_003] + \
        [int(rng.integers(1, 20_000)) for _ in range(60)]
    precs = [heat.FP64, heat.FP32, heat.FP32C]
    probs = []
    for k, N in enumerate(sizes):
        nt = int(rng.integers(0, 12)) if k >= 4 else 6 + k
        probs.append(dict(u0=inputs.uniform_ring(N, (92, k)), nparts=1,
                          r=float(0.5 - 0.4 * rng.random()), nt=nt, precision=precs[k % 3]))
    assert sum(sizes) * 8 >= 64 << 20
    res = heat.solve_batch(probs)
    for p, q in zip(probs, res):
        assert q.status == heat.HEAT_OK
        want = oracle_for(p["precision"], p["u0"], p["r"], p["nt"])
        assert same_bits(q.u, want), (p["u0"].size, p["nt"], p["precision"])


@pytest.mark.parametrize("prec", [heat.FP32, heat.FP32C])
def test_host_batch_mean_shifted_storage(prec):
    """binary32 forms stored as offsets from a shift (the ring's mean, or any
    constant): bit-identical to the oracle's shifted composition, sums of the
    state reported as N*shift + sum of the offsets, and binary64 problems in
    the same batch ignore the shift."""
    rng = np.random.default_rng(46)
    probs, want = [], []
    for k in range(12):
        N = int(rng.integers(1, 40_000))
        nt = int(rng.integers(0, 400))
        r = float(0.5 - 0.4 * rng.random())
        u0 = inputs.perturbed_ring(N, (47, k)) * 3.0 + 5.0
        shift = (math.fsum(u0) / N) if k % 3 else float(rng.normal())
        p = dict(u0=u0, nparts=1, r=r, nt=nt, precision=prec, shift=shift)
        if prec == heat.FP32:
            w = oracle.solve_f32_shifted(u0, r, nt, shift)
        else:
            T = heat.plan(N, nt, heat.FP32C)["steps_per_round"]
            w = oracle.solve_f32c_shifted(u0, r, nt, T, shift)
        probs.append(p)
        want.append(w)
    u64 = inputs.uniform_ring(5000, 48)
    probs.append(dict(u0=u64, nparts=1, r=0.5, nt=77, precision=heat.FP64, shift=123.0))
    want.append(oracle.solve(u64, 0.5, 77))
    res = heat.solve_batch(probs)
    for p, w, q in zip(probs, want, res):
        assert q.status == heat.HEAT_OK
        assert same_bits(q.u, w), (p["u0"].size, p["nt"], p["precision"])
        if p["precision"] == heat.FP64:
            continue
        N, s = p["u0"].size, p["shift"]
        s0 = N * s + math.fsum(oracle.to_offsets(p["u0"], s).astype(np.float64))
        assert abs(q.sum0 - s0) <= 1e-12 * max(abs(s0), 1.0)
        assert abs(q.sum_nt - math.fsum(w)) <= 1e-9 * max(abs(s0), 1.0)
    with pytest.raises(heat.HeatError) as ei:
        heat.solve_batch([dict(u0=u64, nparts=1, r=0.5, nt=3, precision=prec, shift=math.inf)])
    assert ei.value.code == heat.HEAT_EINVAL


def test_host_batch_reports_bad_problem():
    good = dict(u0=inputs.uniform_ring(500, 1), nparts=1, r=0.4, nt=50)
    bad = dict(u0=inputs.uniform_ring(10, 2), nparts=1, r=0.7, nt=5)
    with pytest.raises(heat.HeatError) as ei:
        heat.solve_batch([good, bad, good])
    assert ei.value.code == heat.HEAT_EINVAL


def oracle_many(prec, u0s, rs, nts):
    """The oracle on many rings at once, one host thread per ring (the C
    oracle runs without the interpreter lock)."""
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda a: oracle_for(prec, *a), zip(u0s, rs, nts)))


_EQ_SPECS = inputs.batch_specs(count=96, seed=44, logn_hi=5.0, nt_hi=2000)
_EQ_ORACLE = {}


def eq_oracle(prec):
    """Oracle results of the scaled-down batching workload, per precision
    (computed once for the three batch modes)."""
    if prec not in _EQ_ORACLE:
        specs = _EQ_SPECS
        _EQ_ORACLE[prec] = oracle_many(prec, [inputs.ring_initial(s) for s in specs],
                                       [s.r for s in specs], [s.nt for s in specs])
    return _EQ_ORACLE[prec]


@pytest.mark.parametrize("mode", ["rounds", "graph", "persistent"])
def test_device_batch_equals_alone(mode):
    """Rings of the uneven batching workload (N log-uniform in [1e3, 1e5], nt
    uniform in [100, 2000], r in (0.1, 1/2]) in all three precisions, in each
    batch mode (one launch per round, the captured graph of those launches,
    the persistent flag-synchronised launch): every ring bit for bit equal to
    the oracle's result for it, and to the same ring solved alone."""
    specs = _EQ_SPECS
    kw = dict(graph=mode == "graph", persistent=mode == "persistent")
    for prec, dt in ((heat.FP64, torch.float64), (heat.FP32, torch.float32),
                     (heat.FP32C, torch.float32)):
        print(f"batch mode {mode}, precision {prec}: {len(specs)} rings", flush=True)
        us = [torch.from_numpy(inputs.ring_initial(s)).to("cuda", dtype=dt) for s in specs]
        alone = []
        for s, u in zip(specs, us):
            a = u.clone()
            heat.solve_dev(a, s.nparts, s.r, s.nt, precision=prec)
            alone.append(a)
        work = [torch.empty_like(u) for u in us]
        heat.solve_batch_dev([(u, w, s.nt, s.r, prec) for u, w, s in zip(us, work, specs)], **kw)
        torch.cuda.synchronize()
        want = eq_oracle(prec)
        for s, u, a, w in zip(specs, us, alone, want):
            got = u.cpu().numpy()
            assert same_bits(got, w), (mode, prec, s.N, s.nt)
            assert same_bits(got, a.cpu().numpy()), (mode, prec, s.N, s.nt)


@pytest.mark.parametrize("prec", [heat.FP64, heat.FP32C])
def test_device_batch_persistent_long_rings(prec):
    """The persistent flag-synchronised launch on rings of 1e6 to 3e6 cells
    (hundreds to thousands of tiles, each waiting on its neighbours' epoch
    counters every round) batched with short rings.  binary64: every ring
    whole against the oracle's threaded segmented solver.  Compensated
    binary32: every ring bit for bit equal to the ring solved alone (whose
    kernels the oracle pins elsewhere) and, against the oracle's light cones,
    the cells next to the first tile edges of the persistent kernel's
    geometry (32-cell lanes, one wave per tile, the form's 64-step rounds:
    halo 64, tiles of 64*32 - 2*64 = 1920 cells) and random cells."""
    rng = np.random.default_rng(60 + prec)
    Ns = [1_000_003, 3_000_017, 1_999_999, 777, 20_000]
    nts = [640, 301, 1000, 999, 65] if prec == heat.FP64 else [130, 64, 199, 999, 65]
    rs = [float(0.5 - 0.4 * rng.random()) for _ in Ns]
    dt = torch.float64 if prec == heat.FP64 else torch.float32
    u0s = [inputs.uniform_ring(N, (61, prec, k)) for k, N in enumerate(Ns)]
    us = [torch.from_numpy(u).to("cuda", dtype=dt) for u in u0s]
    work = [torch.empty_like(u) for u in us]
    print(f"persistent long rings, precision {prec}", flush=True)
    heat.solve_batch_dev([(u, w, nt, r, prec) for u, w, nt, r in zip(us, work, nts, rs)],
                         persistent=True)
    torch.cuda.synchronize()
    for k, (N, nt, r, u0, u) in enumerate(zip(Ns, nts, rs, u0s, us)):
        got = u.cpu().numpy()
        if prec == heat.FP64:
            want = oracle.solve_threads(u0, min(16, N), r, nt)
            assert same_bits(got, want), (N, nt)
            continue
        a = torch.from_numpy(u0).to("cuda", dtype=dt)
        heat.solve_dev(a, 1, r, nt, precision=prec)
        assert same_bits(got, a.cpu().numpy()), (N, nt)
        u32 = u0.astype(np.float32)
        W = 64 * 32 - 2 * 64
        cells = {0, N - 1} | {int(i) for i in rng.integers(0, N, 3)}
        for t in (1, 2, 3):
            cells.update({(t * W + d) % N for d in (-1, 0, 1)})
        for i in sorted(cells):
            want = np.float32(oracle.cone_f32c(u32, i, r, nt, 64))
            assert same_bits(got[i:i + 1], np.array([want])), (N, nt, i)


def test_device_batch_large_rings_sampled():
    """A slice of the full-size batching workload (N up to 1e6, nt up to
    10,000): sampled cells of the fused result against oracle light cones."""
    specs = inputs.batch_specs(count=4096, seed=4)
    pick = sorted(range(len(specs)), key=lambda j: -specs[j].N * specs[j].nt)[:12] + list(range(12))
    specs = [specs[j] for j in pick]
    u0s = [inputs.ring_initial(s) for s in specs]
    us = [torch.from_numpy(u).to("cuda") for u in u0s]
    work = [torch.empty_like(u) for u in us]
    heat.solve_batch_dev([(u, w, s.nt, s.r, heat.FP64) for u, w, s in zip(us, work, specs)])
    torch.cuda.synchronize()
    rng = np.random.default_rng(45)
    for s, u0, u in zip(specs, u0s, us):
        # the plain device form (pinned to the oracle above) on the same ring
        a = torch.from_numpy(u0).to("cuda")
        heat.solve_dev(a, s.nparts, s.r, s.nt)
        assert same_bits(u.cpu().numpy(), a.cpu().numpy()), (s.N, s.nt)
        if s.nt <= 3000:   # light cones of longer runs are too slow for the CPU oracle
            for i in {0, s.N - 1, int(rng.integers(0, s.N))}:
                assert u[i].item() == oracle.cone(u0, i, s.r, s.nt), (s.N, s.nt, i)


def test_device_batch_seeded_256_ring_subset():
    """A seeded subset of 256 rings of the full batching workload (4,096 rings,
    N log-uniform in [1e3, 1e6], nt uniform in [100, 10,000], r in (0.1, 0.5]),
    batched in binary64 in the benchmark's configuration: every ring bit for
    bit equal to the same ring solved alone, and one sampled cell of every
    ring equal to the oracle's light cone of that cell."""
    specs = inputs.batch_specs(count=4096, seed=4)
    pick = np.random.default_rng(51).choice(len(specs), size=256, replace=False)
    specs = [specs[j] for j in sorted(pick)]
    u0s = [inputs.ring_initial(s) for s in specs]
    us = [torch.from_numpy(u).cuda() for u in u0s]
    work = [torch.empty_like(u) for u in us]
    heat.solve_batch_dev([(u, w, s.nt, s.r, heat.FP64) for u, w, s in zip(us, work, specs)])
    torch.cuda.synchronize()
    rng = np.random.default_rng(52)
    for s, u0, u in zip(specs, u0s, us):
        a = torch.from_numpy(u0).cuda()
        heat.solve_dev(a, s.nparts, s.r, s.nt)
        assert same_bits(u.cpu().numpy(), a.cpu().numpy()), (s.N, s.nt)
        i = int(rng.integers(0, s.N))
        assert u[i].item() == oracle.cone(u0, i, s.r, s.nt), (s.N, s.nt, i)


def test_device_batch_full_4096_rings_vs_oracle():
    """Every ring of the full batching workload (4,096 rings, about 3e12 cell
    updates), batched in binary64 as the benchmark runs it, compared bit for
    bit with the oracle's segmented solver (its vectorised sweep, pinned
    bit-identical to the scalar one), one host thread per ring and up to 16
    rings at a time (the C oracle runs without the interpreter lock): about a
    minute of host CPU."""
    specs = inputs.batch_specs(count=4096, seed=4)
    u0s = [inputs.ring_initial(s) for s in specs]
    us = [torch.from_numpy(u).cuda() for u in u0s]
    work = [torch.empty_like(u) for u in us]
    heat.solve_batch_dev([(u, w, s.nt, s.r, heat.FP64) for u, w, s in zip(us, work, specs)])
    torch.cuda.synchronize()
    got = [u.cpu().numpy() for u in us]
    del us, work
    torch.cuda.empty_cache()

    def check(j):
        s = specs[j]
        return same_bits(got[j], oracle.solve_threads(u0s[j], 1, s.r, s.nt, simd=True))

    t0 = time.perf_counter()
    bad, done = [], 0
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(workers) as ex:
        for j, ok in zip(range(len(specs)), ex.map(check, range(len(specs)))):
            done += 1
            if not ok:
                bad.append(j)
            if done % 256 == 0:
                print(f"full batch parity: {done}/{len(specs)} rings checked, "
                      f"{len(bad)} mismatches, {time.perf_counter() - t0:.0f} s", flush=True)
    assert not bad, [(specs[j].N, specs[j].nt) for j in bad[:10]]


def test_device_batch_long_rings_all_classes():
    """Long binary64 rings (64K to 3M cells; the longest run as tiles of 4
    waves that swap edges through LDS, the others as one wave per tile) with
    short and odd step counts, in one batch with short rings: every ring bit
    for bit equal to the ring solved alone, and sampled cells (tile edges,
    edges between the waves of a tile) equal to the oracle's light cones."""
    rng = np.random.default_rng(49)
    Ns = [65_536, 100_003, 250_000, 1_000_001, 3_000_017, 777, 20_000]
    nts = [301, 77, 600, 451, 128, 999, 64]
    us, u0s = [], []
    for k, N in enumerate(Ns):
        u0 = inputs.uniform_ring(N, (50, k))
        u0s.append(u0)
        us.append(torch.from_numpy(u0).cuda())
    work = [torch.empty_like(u) for u in us]
    rs = [float(0.5 - 0.4 * rng.random()) for _ in Ns]
    heat.solve_batch_dev([(u, w, nt, r, heat.FP64) for u, w, nt, r in zip(us, work, nts, rs)])
    torch.cuda.synchronize()
    for k, (N, nt, r, u0, u) in enumerate(zip(Ns, nts, rs, u0s, us)):
        a = torch.from_numpy(u0).cuda()
        heat.solve_dev(a, 1, r, nt)
        assert same_bits(u.cpu().numpy(), a.cpu().numpy()), (N, nt)
        # tile and wave edges of both tile shapes the batch may have used
        cells = {0, N - 1, int(rng.integers(0, N))}
        for W, step in ((64 * 64 - 2 * 256, 0), (4 * 4096 - 3 * 32 - 2 * 256, 4096 - 32)):
            for t in (1, 2):
                cells.update({(t * W + d) % N for d in (-1, 0, 1)})
                if step:
                    cells.update({(t * W + step + 16 - 256 + d) % N for d in (-1, 0, 1)})
        for i in sorted(cells):
            assert u[i].item() == oracle.cone(u0, i, r, nt), (N, nt, i)


@pytest.mark.parametrize("prec", [heat.FP32, heat.FP32C])
def test_device_batch_binary32_long_rings(prec):
    """Binary32 rings long enough for the wide classes (plain: 64-cell lanes,
    the longest as tiles of 4 waves swapping edges through LDS; compensated:
    4-wave tiles at 32-cell lanes) batched with short ones that stay on one
    wave per tile: every ring bit for bit equal to the ring solved alone, and
    sampled cells (tile and wave edges of the shapes the batch may use) equal
    to the oracle's light cones."""
    rng = np.random.default_rng(55)
    Ns = [100_003, 250_000, 1_000_001, 2_000_003, 777, 20_000]
    nts = [301, 77, 130, 64, 999, 65]
    us, u0s = [], []
    for k, N in enumerate(Ns):
        u0 = inputs.uniform_ring(N, (56, k)).astype(np.float32)
        u0s.append(u0)
        us.append(torch.from_numpy(u0).cuda())
    work = [torch.empty_like(u) for u in us]
    rs = [float(0.5 - 0.4 * rng.random()) for _ in Ns]
    heat.solve_batch_dev([(u, w, nt, r, prec) for u, w, nt, r in zip(us, work, nts, rs)])
    torch.cuda.synchronize()
    T = heat.plan(1000, 1000, heat.FP32C)["steps_per_round"]
    if prec == heat.FP32C:   # (tile cells, offset of the second wave's window)
        shapes = ((64 * 32 - 2 * 64, 0, 8, 64), (4 * 2048 - 3 * 16 - 2 * 64, 2048 - 16, 8, 64))
    else:
        shapes = ((64 * 64 - 2 * 256, 0, 16, 256), (4 * 4096 - 3 * 32 - 2 * 256, 4096 - 32, 16, 256))
    for k, (N, nt, r, u0, u) in enumerate(zip(Ns, nts, rs, u0s, us)):
        a = torch.from_numpy(u0).cuda()
        heat.solve_dev(a, 1, r, nt, precision=prec)
        assert same_bits(u.cpu().numpy(), a.cpu().numpy()), (N, nt)
        cells = {0, N - 1, int(rng.integers(0, N))}
        for W, step, S, H in shapes:
            for t in (1, 2):
                cells.update({(t * W + d) % N for d in (-1, 0, 1)})
                if step:
                    cells.update({(t * W + step + S - H + d) % N for d in (-1, 0, 1)})
        got = u.cpu().numpy()
        for i in sorted(cells):
            if prec == heat.FP32C:
                want = np.float32(oracle.cone_f32c(u0, i, r, nt, T))
            else:
                want = np.float32(oracle.cone_f32(u0, i, r, nt))
            assert same_bits(got[i:i + 1], np.array([want])), (N, nt, i)


def test_device_batch_empty_and_zero_steps():
    heat.solve_batch_dev([])
    u = torch.rand(1000, device="cuda", dtype=torch.float64)
    ref = u.clone()
    heat.solve_batch_dev([(u, torch.empty_like(u), 0, 0.5, heat.FP64)])
    assert same_bits(u.cpu().numpy(), ref.cpu().numpy())
