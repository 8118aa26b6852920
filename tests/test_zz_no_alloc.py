"""GPU check of heat_solve_dev_noalloc, the device form that allocates
nothing (its scratch is a static device array of the library): its results
equal those of heat_solve_dev bit for bit, on consecutive calls that reuse
the same scratch, the second on a smaller ring; so do its checksums where
both calls run the round kernel (a call of heat_solve_dev that waits may take
the resident kernel, whose tiles group the partial sums differently: equal up
to rounding then, and both within rounding of the exact sums)."""
import math

import numpy as np
import pytest

import oracle
from paper_2307_01117_amd import heat, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def bits(t):
    a = t.cpu().numpy()
    return a.view({4: np.uint32, 8: np.uint64}[a.dtype.itemsize])


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    heat.load()


# (N, nt, r, precision): the largest binary64 ring near the scratch limit,
# then smaller rings (the second call must not see the first call's data)
CASES = [
    [(8_000_000, 300, 0.5, heat.FP64), (1_000_003, 101, 0.4, heat.FP64),
     (77_777, 130, 0.25, heat.FP32C)],
    [(16_000_000, 64, 0.25, heat.FP32), (3_001, 7, 0.5, heat.FP32), (1, 5, 0.5, heat.FP64)],
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_equals_device_form(case):
    stream = torch.cuda.current_stream()
    for k, (N, nt, r, prec) in enumerate(CASES[case]):
        print(f"noalloc case {case}.{k}: N {N} nt {nt} r {r} precision {prec}", flush=True)
        dt = torch.float64 if prec == heat.FP64 else torch.float32
        u0 = inputs.uniform_ring(N, (70, case, k))
        a = torch.from_numpy(u0).to("cuda", dtype=dt)
        b = a.clone()
        s0, s1 = heat.solve_dev(a, 1, r, nt, precision=prec, stream=stream, sums=True)
        d_sums = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        heat.solve_dev_noalloc(b, 1, r, nt, precision=prec, stream=stream, sums_out=d_sums)
        torch.cuda.synchronize()
        assert np.array_equal(bits(a), bits(b)), (case, k)
        got = d_sums.cpu().numpy()
        if heat.plan(N, nt, prec)["kernel"] == heat.KERNEL_RESIDENT:
            for x, y in zip(got, (s0, s1)):
                assert abs(x - y) <= 1e-13 * abs(y), (case, k, got, s0, s1)
        else:
            assert np.array_equal(got.view(np.uint64), np.array([s0, s1]).view(np.uint64)), \
                (case, k, got, s0, s1)
        x0 = u0 if prec == heat.FP64 else u0.astype(np.float32)
        exact0 = math.fsum(x0.astype(np.float64))
        assert abs(got[0] - exact0) <= 1e-13 * abs(exact0), (case, k, got[0], exact0)
        exact1 = math.fsum(b.cpu().numpy().astype(np.float64))
        assert abs(got[1] - exact1) <= 1e-13 * abs(exact1), (case, k, got[1], exact1)
        if N * nt <= 5e8:
            if prec == heat.FP64:
                want = oracle.solve(u0, r, nt)
            elif prec == heat.FP32:
                want = oracle.solve_f32(u0.astype(np.float32), r, nt)
            else:
                T = heat.plan(N, nt, heat.FP32C)["steps_per_round"]
                want = oracle.solve_f32c(u0.astype(np.float32), r, nt, T)
            assert np.array_equal(bits(b), want.view(bits(b).dtype)), (case, k)
    # without sums, twice in a row on the same tensor: the composition of runs
    N, nt = 50_001, 40
    u0 = inputs.uniform_ring(N, (71, case))
    c = torch.from_numpy(u0).cuda()
    heat.solve_dev_noalloc(c, 1, 0.5, nt, stream=stream)
    heat.solve_dev_noalloc(c, 1, 0.5, nt, stream=stream)
    torch.cuda.synchronize()
    assert np.array_equal(bits(c), oracle.solve(u0, 0.5, 2 * nt).view(np.uint64))


def test_noalloc_refuses_rings_beyond_scratch():
    big = torch.empty(9_000_000, dtype=torch.float64, device="cuda")
    with pytest.raises(heat.HeatError) as ei:
        heat.solve_dev_noalloc(big, 1, 0.5, 10)
    assert ei.value.code == heat.HEAT_EINVAL and "static scratch" in str(ei.value)
