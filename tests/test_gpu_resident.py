"""GPU parity of the resident kernel (HEAT_KERNEL_RESIDENT) with the oracle.

One launch runs all nt steps: every tile keeps its windows in registers and
swaps its H edge cells with its neighbours through memory every T steps
(Section 2's ghost-zone exchange between segments, H cells deep).  Its
results must be the oracle's bits, as for the round kernel: whole rings
compared for every precision, with ragged last tiles, a last tile shorter
than H, a single tile, odd and even exchange counts, one step, and the
paper's own workload; the fused checksums against the exact sum.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2307_01117_amd import heat, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    heat.load()


def same_bits(a, b):
    a, b = np.asarray(a), np.asarray(b)
    if a.shape != b.shape or a.dtype != b.dtype:
        return False
    it = {4: np.uint32, 8: np.uint64}[a.dtype.itemsize]
    return bool(np.array_equal(np.ascontiguousarray(a).view(it),
                               np.ascontiguousarray(b).view(it)))


def run_resident(u0, nt, r, precision, sums=False, **cfg):
    dt = torch.float64 if precision == heat.FP64 else torch.float32
    d = torch.from_numpy(np.ascontiguousarray(u0)).to(device="cuda", dtype=dt)
    s = heat.solve_dev(d, 1, r, nt, precision=precision, sums=sums,
                       kernel=heat.KERNEL_RESIDENT, **cfg)
    torch.cuda.synchronize()
    return d.cpu().numpy(), s


# (K, waves per group, exchange, register form)
SHAPES_FP64 = [(8, 1, heat.EXCHANGE_NONE, 3), (16, 4, heat.EXCHANGE_LDS, 3),
               (8, 4, heat.EXCHANGE_LDS_DEEP, 1), (16, 2, heat.EXCHANGE_LDS_DEEP, 2),
               (32, 4, heat.EXCHANGE_LDS, 3), (16, 1, heat.EXCHANGE_NONE, 1)]
SHAPES_FP32 = [(8, 1, heat.EXCHANGE_NONE, 1), (16, 4, heat.EXCHANGE_LDS, 1),
               (32, 4, heat.EXCHANGE_LDS_DEEP, 1), (32, 1, heat.EXCHANGE_NONE, 1)]


def plan_of(N, nt, prec, K, G, x, form, T=0):
    return heat.plan(N, nt, prec, kernel=heat.KERNEL_RESIDENT, cells_per_lane=K,
                     waves_per_group=G, exchange=x, register_form=form, steps_per_round=T)


@pytest.mark.parametrize("shape", SHAPES_FP64)
@pytest.mark.parametrize("N,nt,T", [(70_001, 100, 16), (5_003, 37, 12), (300, 41, 0),
                                    (123_457, 1, 0), (33_333, 64, 32)])
def test_resident_fp64_bitwise(shape, N, nt, T):
    K, G, x, form = shape
    u0 = inputs.uniform_ring(N, (31, N, K, G))
    cfg = dict(cells_per_lane=K, waves_per_group=G, exchange=x, register_form=form,
               steps_per_round=T)
    got, _ = run_resident(u0, nt, 0.4375, heat.FP64, **cfg)
    assert same_bits(got, oracle.solve(u0, 0.4375, nt)), (shape, N, nt, T)


def test_resident_last_tile_shorter_than_halo():
    """A ring two whole tiles plus 10 cells long: the last tile is shorter
    than H, so halos reach two tiles away and the waits walk that far."""
    K, G, x, form, T = 16, 4, heat.EXCHANGE_LDS, 3, 16
    W = plan_of(10**6, 100, heat.FP64, K, G, x, form, T)["tile_cells"]
    N = 2 * W + 10
    u0 = inputs.uniform_ring(N, 32)
    got, _ = run_resident(u0, 100, 0.5, heat.FP64, cells_per_lane=K, waves_per_group=G,
                          exchange=x, register_form=form, steps_per_round=T)
    assert same_bits(got, oracle.solve(u0, 0.5, 100))


@pytest.mark.parametrize("shape", SHAPES_FP32)
@pytest.mark.parametrize("N,nt", [(65_536 + 13, 100), (999, 33)])
def test_resident_fp32_bitwise(shape, N, nt):
    K, G, x, form = shape
    u0 = inputs.uniform_ring(N, (33, N, K)).astype(np.float32)
    got, _ = run_resident(u0, nt, 0.3, heat.FP32, cells_per_lane=K, waves_per_group=G,
                          exchange=x, register_form=form, steps_per_round=16)
    assert same_bits(got, oracle.solve_f32(u0, 0.3, nt)), (shape, N, nt)


@pytest.mark.parametrize("shape", SHAPES_FP32)
@pytest.mark.parametrize("r", [0.25, 0.3])
def test_resident_fp32c_bitwise(shape, r):
    """The compensated form folds u + e at every exchange: the exchange
    interval is its round length T, and the result is the oracle's with that T
    (r = 1/4 runs the kernel without the coefficient's low part)."""
    K, G, x, form = shape
    N, nt = 40_009, 150
    u0 = inputs.perturbed_ring(N, (34, K)).astype(np.float32)
    got, _ = run_resident(u0, nt, r, heat.FP32C, cells_per_lane=K, waves_per_group=G,
                          exchange=x, register_form=form)
    T = plan_of(N, nt, heat.FP32C, K, G, x, form)["steps_per_round"]
    assert T == 64
    assert same_bits(got, oracle.solve_f32c(u0, r, nt, T)), (shape, r)


@pytest.mark.parametrize("shape", [SHAPES_FP64[0], SHAPES_FP64[1], SHAPES_FP64[2]])
def test_resident_fused_checksums(shape):
    K, G, x, form = shape
    N, nt = 250_007, 120
    u0 = inputs.uniform_ring(N, (35, K, G))
    got, (s0, s1) = run_resident(u0, nt, 0.45, heat.FP64, sums=True, cells_per_lane=K,
                                 waves_per_group=G, exchange=x, register_form=form,
                                 steps_per_round=32)
    want = oracle.solve(u0, 0.45, nt)
    assert same_bits(got, want)
    assert abs(s0 - math.fsum(u0)) <= 1e-13 * abs(math.fsum(u0))
    assert abs(s1 - math.fsum(want)) <= 1e-13 * abs(math.fsum(want))


def test_resident_paper_workload():
    """The paper's run (ramp u0[i] = i, 1e6 nodes, r = 1/2, 1,000 steps) in
    its tuned resident shape, whole ring against the oracle."""
    N, nt, r = 1_000_000, 1000, 0.5
    u0 = np.arange(N, dtype=np.float64)
    got, _ = run_resident(u0, nt, r, heat.FP64, cells_per_lane=16, waves_per_group=4,
                          exchange=heat.EXCHANGE_LDS, register_form=3)
    assert same_bits(got, oracle.solve_threads(u0, 16, r, nt))


def test_resident_refuses_grids_it_cannot_hold():
    """More tiles than the device holds at once: refused before any launch,
    the input untouched."""
    N = 50_000_000
    u0 = torch.ones(N, dtype=torch.float64, device="cuda")
    with pytest.raises(heat.HeatError) as e:
        heat.solve_dev(u0, 1, 0.5, 10, precision=heat.FP64, kernel=heat.KERNEL_RESIDENT,
                       cells_per_lane=8, waves_per_group=1, exchange=heat.EXCHANGE_NONE)
    assert e.value.code == heat.HEAT_EINVAL
    assert "resident" in str(e.value)
    assert bool(torch.all(u0 == 1.0))


def test_resident_calls_in_a_row_count_on():
    """The epoch counters are not cleared between calls: each call counts on
    from the last one's highest epoch.  Calls in a row with more, fewer and
    then more tiles than before (the counter buffer grows and is cleared
    once), odd and even epoch counts, all bitwise."""
    shape = dict(cells_per_lane=8, waves_per_group=1, exchange=heat.EXCHANGE_NONE,
                 register_form=3, steps_per_round=16)
    for i, (N, nt) in enumerate([(40_000, 50), (9_000, 33), (40_000, 64), (150_000, 47),
                                 (20_000, 16), (150_000, 80)]):
        u0 = inputs.uniform_ring(N, (36, i))
        got, _ = run_resident(u0, nt, 0.375, heat.FP64, **shape)
        assert same_bits(got, oracle.solve(u0, 0.375, nt)), (i, N, nt)


def test_planner_fits_the_tuned_shapes_to_n(tmp_path):
    """The tuned shapes of a quarter decade fitted to N.  A CU holds
    ceil(tiles / CUs) workgroups and every tile waits for the slowest: for
    binary64 and binary32 the planner takes the longest exchange interval, at
    most the tuned one and at least half of it, that puts the fewest waves on
    the busiest SIMD; among the recorded shapes it takes the one whose gain
    at full load at N (linear in log N between the quarter decade's lower
    end, geometric middle and upper end) times its load efficiency at N is
    the largest, if that is at least 1.03, else the round kernel (the
    compensated form keeps its T)."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count

    def busiest(p):
        return (-(-p["tiles"] // cus) * p["waves_per_group"] + 3) // 4

    def efficiency(p):
        return p["tiles"] * p["waves_per_group"] / (4 * cus) / busiest(p)

    def fitted(N, prec, K, T0, G, x, form):
        Ts = [T0] if prec == heat.FP32C else [T for T in (T0, 96, 64, 48, 32, 24, 16)
                                              if T <= T0 and 2 * T >= T0]
        cand = {T: plan_of(N, 1000, prec, K, G, x, form, T) for T in Ts}
        T = min(cand, key=lambda T: (busiest(cand[T]), -T))
        return cand[T]

    def gain_at(g, b, N):
        lo, hi = math.ceil(10 ** (b / 4)), math.ceil(10 ** ((b + 1) / 4)) - 1
        pts = [lo, round(math.sqrt(lo * hi)), hi]
        x = np.log(N)
        xs, ys = np.log(pts), np.array(g) / 1000
        return float(np.interp(x, xs, ys))

    saved = tmp_path / "orig.txt"
    heat.tune_save(str(saved))
    try:
        f = tmp_path / "r.txt"
        # quarter decades 24 and 25: 10^6 to 10^6.25 and 10^6.25 to 10^6.5 cells
        lines = {(heat.FP64, 24): [(16, 48, 4, heat.EXCHANGE_LDS_DEEP, 3, (1200, 1100, 1000)),
                                   (8, 48, 4, heat.EXCHANGE_LDS_DEEP, 3, (1150, 1150, 1150))],
                 (heat.FP32, 25): [(16, 128, 4, heat.EXCHANGE_LDS_DEEP, 1, (1500, 1500, 1500)),
                                   (16, 96, 1, heat.EXCHANGE_NONE, 1, (1400, 1300, 1300))],
                 (heat.FP32C, 25): [(16, 64, 1, heat.EXCHANGE_NONE, 1, (1200, 1200, 1200))]}
        f.write_text("".join("r %d %d %d %d %d %d %d 100 100 100 %d %d %d\n"
                             % (p, b, K, T, G, form, x, *g)
                             for (p, b), shapes in lines.items()
                             for K, T, G, x, form, g in shapes))
        heat.tune_load(str(f))
        checked = 0
        for (prec, b), shapes in lines.items():
            for N in (1_000_000, 1_200_000, 1_330_000, 1_780_000, 2_000_000, 2_500_000,
                      3_000_000):
                if int(4 * np.log10(N)) != b:
                    continue
                score, want = 0.0, None
                for K, T, G, x, form, g in shapes:
                    p = fitted(N, prec, K, T, G, x, form)
                    sc = gain_at(g, b, N) * efficiency(p)
                    if sc > score:
                        score, want = sc, p
                got = heat.plan(N, 1000, prec)
                assert abs(score - 1.03) > 1e-6, "too close to the margin to test"
                if score >= 1.03:
                    assert got["kernel"] == heat.KERNEL_RESIDENT, (prec, N)
                    for key in ("cells_per_lane", "steps_per_round", "waves_per_group",
                                "tiles"):
                        assert got[key] == want[key], (prec, N, key)
                else:
                    assert got["kernel"] == heat.KERNEL_TB, (prec, N)
                checked += 1
        assert checked == 11
        # short runs keep the round kernel
        assert heat.plan(2_000_000, 99, heat.FP32)["kernel"] == heat.KERNEL_TB
        # the choice cached for a ring goes with the table it came from
        assert heat.plan(2_000_000, 1000, heat.FP32)["kernel"] == heat.KERNEL_RESIDENT
        f.write_text("r 1 25 0 0 0 0 0 0\n")
        heat.tune_load(str(f))
        assert heat.plan(2_000_000, 1000, heat.FP32)["kernel"] == heat.KERNEL_TB
    finally:
        heat.tune_load(str(saved))


def test_resident_wait_timeout_fails_cleanly(monkeypatch):
    """The failure path, forced from the host: with HEAT_RESIDENT_SPIN_LIMIT=0
    a tile gives up at its first poll that finds a neighbour's edges not yet
    there, sets the status word and leaves, and so does every other wave; the
    call reports HEAT_EDEVICE.  The next calls (limit restored) start from
    cleared tags and counters and a fresh status word, and are bitwise."""
    N, nt = 2_000_003, 200
    shape = dict(cells_per_lane=8, waves_per_group=1, exchange=heat.EXCHANGE_NONE,
                 register_form=3, steps_per_round=16)
    u0 = inputs.uniform_ring(N, 37)
    want = oracle.solve_threads(u0, 16, 0.5, nt)
    monkeypatch.setenv("HEAT_RESIDENT_SPIN_LIMIT", "0")
    failed = 0
    for _ in range(3):
        try:
            run_resident(u0, nt, 0.5, heat.FP64, **shape)
        except heat.HeatError as e:
            assert e.code == heat.HEAT_EDEVICE and "waited too long" in str(e)
            failed += 1
    assert failed > 0
    monkeypatch.delenv("HEAT_RESIDENT_SPIN_LIMIT")
    for _ in range(2):
        got, _ = run_resident(u0, nt, 0.5, heat.FP64, **shape)
        assert same_bits(got, want)


@pytest.mark.parametrize("prec,K,G,x,form,T,N,nt", [
    # 1,277 tiles of 3,984 cells, the last of 10 (shorter than H): more than
    # a CU holds with the whole tile copy in LDS
    (heat.FP64, 16, 4, heat.EXCHANGE_LDS_DEEP, 3, 32, 1276 * 3984 + 10, 70),
    # 1,130 tiles of 7,968 cells, 33 KB of LDS each with the whole copy
    (heat.FP32, 32, 4, heat.EXCHANGE_LDS_DEEP, 1, 64, 9_000_037, 150),
])
def test_resident_edge_lds_layout_bitwise(prec, K, G, x, form, T, N, nt):
    """Grids that fit only with the LDS copy of the tiles' two edge regions
    (the split layout): whole rings bitwise against the oracle."""
    p = plan_of(N, nt, prec, K, G, x, form, T)
    # with the whole tile span W + 2H in LDS, after the waves' exchange area
    # (160 KB per CU), they would not
    S, cell = p["exchange_steps"], 8 if prec == heat.FP64 else 4
    span = G * 64 * K - (G - 1) * 2 * S
    per_cu = (160 * 1024) // (span * cell + 2 * G * 2 * S * cell)
    assert p["tiles"] > per_cu * torch.cuda.get_device_properties(0).multi_processor_count
    u0 = inputs.uniform_ring(N, (38, K))
    if prec == heat.FP64:
        want = oracle.solve_threads(u0, 16, 0.5, nt)
    else:
        u0 = u0.astype(np.float32)
        want = oracle.solve_f32(u0, 0.5, nt)
    got, _ = run_resident(u0, nt, 0.5, prec, cells_per_lane=K, waves_per_group=G, exchange=x,
                          register_form=form, steps_per_round=T)
    assert same_bits(got, want)


def test_host_form_takes_the_resident_kernel():
    """heat_solve (a host array; the call always waits) on a mid-size ring
    takes the resident kernel as the planner picks it: bitwise against the
    oracle, and the input untouched."""
    N, nt, r = 2_000_003, 300, 0.5
    assert heat.plan(N, nt, heat.FP64)["kernel"] == heat.KERNEL_RESIDENT
    u0 = inputs.uniform_ring(N, 39)
    keep = u0.copy()
    got = heat.solve(u0, 4, r, nt)
    assert same_bits(u0, keep)
    assert same_bits(got, oracle.solve_threads(u0, 16, r, nt))
