"""GPU tests of the serving form (continuous batching) through the C ABI:
results bit-identical to the oracle and to the same request solved alone,
admission by HBM footprint, queue limits, cancellation and shutdown."""
import os
import threading
import time
from concurrent.futures import ThreadPoolExecutor, as_completed

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


def alone(u0, nt, r, prec):
    dt = torch.float64 if prec == heat.FP64 else torch.float32
    d = torch.from_numpy(u0).to("cuda", dtype=dt)
    heat.solve_dev(d, 1, r, nt, precision=prec)
    return d.double().cpu().numpy()


def requests(seed, count, nmax=200_000, ntmax=1500):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        N = int(10 ** rng.uniform(0, np.log10(nmax)))
        nt = int(rng.integers(0, ntmax))
        r = float(0.5 - 0.4 * rng.random())
        prec = heat.FP64 if k % 2 == 0 else heat.FP32C
        out.append((inputs.uniform_ring(N, (60, seed, k)), nt, r, prec))
    return out


def test_single_request_matches_oracle():
    u0 = inputs.uniform_ring(50_001, 61)
    with heat.Server(hbm_budget=1 << 30) as s:
        t = s.submit(u0, 300, 0.5)
        res = s.wait(t)
        assert res.status == heat.HEAT_OK
        assert same_bits(res.u, oracle.solve(u0, 0.5, 300))
        assert abs(res.sum_nt - res.sum0) < 1e-9
        st = s.stats()
        assert st["completed"] == 1 and st["hbm_in_use"] == 0


def test_mix_equals_alone():
    """Requests of different N, nt, r and precision submitted together: every
    result equals the same request solved alone with the plain form."""
    reqs = requests(62, 48)
    with heat.Server(hbm_budget=2 << 30) as s:
        tickets = [s.submit(u0, nt, r, prec) for (u0, nt, r, prec) in reqs]
        results = [s.wait(t) for t in tickets]
        assert s.stats()["ticks"] >= 1
    for (u0, nt, r, prec), res in zip(reqs, results):
        assert res.status == heat.HEAT_OK
        assert same_bits(res.u, alone(u0, nt, r, prec)), (u0.size, nt, prec)


def test_alone_on_idle_server_equals_in_mix():
    probe = requests(63, 4, nmax=300_000, ntmax=3000)
    background = requests(64, 40)
    with heat.Server(hbm_budget=2 << 30) as s:
        solo = [s.wait(s.submit(*q)).u for q in probe]
        tickets = []
        for k, q in enumerate(background):
            tickets.append(s.submit(*q))
            if k % 10 == 0:
                tickets.append(("probe", s.submit(*probe[k // 10])))
        mixed = {}
        for t in tickets:
            if isinstance(t, tuple):
                mixed[len(mixed)] = s.wait(t[1]).u
            else:
                s.wait(t)
    for k in range(4):
        assert same_bits(solo[k], mixed[k])


def test_mean_shifted_requests():
    """binary32 requests stored as offsets from a shift, mixed with unshifted
    ones: each equals the oracle's shifted composition bit for bit."""
    reqs = []
    for k in range(8):
        N = 20_000 + 997 * k
        u0 = inputs.perturbed_ring(N, (71, k))
        prec = heat.FP32 if k % 2 else heat.FP32C
        shift = 0.0 if k % 4 == 3 else float(np.mean(u0))
        reqs.append((u0, 300 + 11 * k, 0.25, prec, shift))
    with heat.Server(hbm_budget=1 << 30) as s:
        ts = [s.submit(u0, nt, r, prec, shift=sh) for (u0, nt, r, prec, sh) in reqs]
        outs = [s.wait(t) for t in ts]
    for (u0, nt, r, prec, sh), res in zip(reqs, outs):
        assert res.status == heat.HEAT_OK
        if prec == heat.FP32:
            want = oracle.solve_f32_shifted(u0, r, nt, sh)
        else:
            T = heat.plan(u0.size, nt, heat.FP32C)["steps_per_round"]
            want = oracle.solve_f32c_shifted(u0, r, nt, T, sh)
        assert same_bits(res.u, want), (u0.size, nt, prec, sh)


def test_tick_size_does_not_change_results(monkeypatch):
    """Ticks sized in steps (HEAT_SERVER_TICK_STEPS) regroup the rounds of
    the resident requests; every result stays bit-identical to the request
    solved alone."""
    reqs = requests(72, 24, nmax=150_000, ntmax=1200)
    for steps in ("64", "500"):
        monkeypatch.setenv("HEAT_SERVER_TICK_STEPS", steps)
        with heat.Server(hbm_budget=1 << 30) as s:
            outs = [s.wait(t) for t in [s.submit(*q) for q in reqs]]
        for q, res in zip(reqs, outs):
            assert res.status == heat.HEAT_OK
            assert same_bits(res.u, alone(*q)), (steps, q[0].size, q[1], q[3])


def test_budget_admission_and_enomem():
    budget = 24 << 20     # fits one 1e6-cell binary64 request (16 MB), not two
    with heat.Server(hbm_budget=budget) as s:
        big = inputs.uniform_ring(2_000_000, 65)
        with pytest.raises(heat.HeatError) as ei:
            s.submit(big, 10, 0.5)
        assert ei.value.code == heat.HEAT_ENOMEM
        reqs = [(inputs.uniform_ring(1_000_000, (66, k)), 200, 0.4, heat.FP64) for k in range(3)]
        ts = [s.submit(*q) for q in reqs]
        outs = [s.wait(t) for t in ts]
        st = s.stats()
        assert st["hbm_peak"] <= budget and st["hbm_in_use"] == 0
    for (u0, nt, r, _), res in zip(reqs, outs):
        assert same_bits(res.u, oracle.solve(u0, r, nt))


def test_queue_limit_busy():
    with heat.Server(hbm_budget=24 << 20, max_queue=1) as s:
        q = (inputs.uniform_ring(1_000_000, 67), 4000, 0.5, heat.FP64)
        accepted, busy = [], 0
        for _ in range(4):
            try:
                accepted.append(s.submit(*q))
            except heat.HeatError as e:
                assert e.code == heat.HEAT_EBUSY
                busy += 1
        assert busy >= 1 and accepted
        for t in accepted:
            assert s.wait(t).status == heat.HEAT_OK


def test_cancel_and_unknown_ticket():
    with heat.Server(hbm_budget=1 << 30) as s:
        long_req = (inputs.uniform_ring(4_000_000, 68), 200_000, 0.5, heat.FP64)
        short = (inputs.uniform_ring(10_000, 69), 100, 0.3, heat.FP64)
        t1 = s.submit(*long_req)
        t2 = s.submit(*short)
        time.sleep(0.01)
        s.cancel(t1)
        with pytest.raises(heat.HeatError) as ei:
            s.poll(t1)
        assert ei.value.code == heat.HEAT_ENOENT
        res = s.wait(t2)
        assert same_bits(res.u, oracle.solve(short[0], 0.3, 100))
        assert s.stats()["cancelled"] == 1
    with pytest.raises(heat.HeatError):
        heat.Server(hbm_budget=16)   # below the minimum arena


def test_one_ticket_from_many_threads():
    """Several threads wait on, poll and cancel the same tickets: exactly one
    call consumes each ticket, the others get HEAT_ENOENT, and the consumed
    result is the request's own."""
    u0 = inputs.uniform_ring(1_000_000, 71)
    want = alone(u0, 4000, 0.4, heat.FP64)
    with heat.Server(hbm_budget=1 << 30) as s:
        for trial in range(3):
            t = s.submit(u0, 4000, 0.4, heat.FP64)
            outcome = []

            def waiter():
                try:
                    outcome.append(("result", s.wait(t)))
                except heat.HeatError as e:
                    outcome.append(("error", e.code))

            def poller():
                while True:
                    try:
                        res = s.poll(t)
                    except heat.HeatError as e:
                        outcome.append(("error", e.code))
                        return
                    if res is not None:
                        outcome.append(("result", res))
                        return
                    time.sleep(0.0005)

            def canceller():
                time.sleep(0.002)
                try:
                    s.cancel(t)
                    outcome.append(("cancelled", None))
                except heat.HeatError as e:
                    outcome.append(("error", e.code))

            work = [waiter, waiter, poller] + ([canceller] if trial == 2 else [])
            th = [threading.Thread(target=f) for f in work]
            for x in th:
                x.start()
            for x in th:
                x.join(timeout=60)
            assert not any(x.is_alive() for x in th)
            assert len(outcome) == len(work)
            consumed = [o for o in outcome if o[0] != "error" or o[1] != heat.HEAT_ENOENT]
            assert len(consumed) == 1, outcome
            kind, val = consumed[0]
            if kind == "result":
                assert same_bits(val.u, want)
            elif kind == "error":
                assert val == heat.HEAT_ECANCELED and trial == 2
            else:
                assert trial == 2
            with pytest.raises(heat.HeatError) as ei:
                s.poll(t)
            assert ei.value.code == heat.HEAT_ENOENT


def test_submit_from_many_threads_and_destroy_with_work_outstanding():
    reqs = requests(70, 64, nmax=100_000, ntmax=800)
    s = heat.Server(hbm_budget=1 << 30)
    tickets = [None] * len(reqs)

    def worker(lo):
        for k in range(lo, len(reqs), 4):
            tickets[k] = s.submit(*reqs[k])

    th = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    got = [s.wait(t) for t in tickets[:16]]
    for q, res in zip(reqs[:16], got):
        assert same_bits(res.u, alone(*q))
    # more work outstanding: destroy must cancel it cleanly
    for q in reqs[:8]:
        s.submit(*q)
    s.close()


def test_busy_server_classes_equal_alone():
    """More requests resident at once than the server's light-load limit
    (64), so the later ones are admitted into the batching form's wide
    classes (64-cell lanes, 4-wave tiles): every result, of all three
    precisions, bit for bit equal to the request solved alone."""
    rng = np.random.default_rng(61)
    reqs = []
    for k in range(120):
        # the first 64 are long enough (tens of ms together) to be resident
        # when the others are admitted
        N = int(10 ** rng.uniform(6.0, 6.3)) if k < 64 else int(10 ** rng.uniform(4.5, 6.3))
        nt = int(rng.integers(2000, 3000)) if k < 64 else int(rng.integers(60, 900))
        r = float(0.5 - 0.4 * rng.random())
        prec = (heat.FP64, heat.FP32C, heat.FP32)[k % 3]
        reqs.append((inputs.uniform_ring(N, (62, k)), nt, r, prec))
    with heat.Server() as srv:
        tickets = [srv.submit(u0, nt, r, prec) for u0, nt, r, prec in reqs]
        results = [srv.wait(t) for t in tickets]
    for (u0, nt, r, prec), res in zip(reqs, results):
        assert same_bits(res.u, alone(u0, nt, r, prec)), (u0.size, nt, prec)


def test_serving_trace_vs_oracle():
    """The serving workload at 200 requests/s (Poisson arrivals, 10 s unless
    HEAT_SERVE_PARITY_SECONDS says otherwise) through one server: every
    request with N*nt <= 1e9 compared bit for bit with the oracle over the
    whole ring (binary64: the segmented C solver; compensated binary32: its C
    solver with the form's round length), and a seeded 2 % sample of the
    larger ones at 16 cells each through the oracle's light cone."""
    duration = float(os.environ.get("HEAT_SERVE_PARITY_SECONDS", "10"))
    P, nmax = 1 << 24, 10_000_000
    pool = np.empty(P + nmax)
    pool[:P] = inputs.serving_pool(P)
    pool[P:] = pool[:nmax]        # u0 of a request = one contiguous slice
    trace = inputs.serving_trace(200.0, duration, pool_size=P)
    rng = np.random.default_rng(53)
    whole = [q.N * q.nt <= 1e9 for q in trace]
    sampled = [not w and rng.random() < 0.02 for w in whole]
    sink = np.empty(nmax)
    server = heat.Server()
    subs = []
    t0 = time.perf_counter()
    for j, (q, w, sm) in enumerate(zip(trace, whole, sampled)):
        delay = t0 + q.t_arrival - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        out = np.empty(q.N) if (w or sm) else sink[:q.N]
        subs.append((j, q, w, sm, server.submit(pool[q.offset:q.offset + q.N], q.nt, q.r,
                                                q.precision, out=out)))
    done = [(j, q, w, sm, server.wait(t)) for j, q, w, sm, t in subs]
    server.close()
    print(f"served {len(done)} requests in {time.perf_counter() - t0:.0f} s; checking "
          f"{sum(whole)} whole and {sum(sampled)} sampled", flush=True)
    T = {j: heat.plan(q.N, q.nt, heat.FP32C)["steps_per_round"]
         for j, q, w, sm, _ in done if q.precision == heat.FP32C and (w or sm)}

    def verify(item):
        j, q, w, sm, res = item
        u0 = pool[q.offset:q.offset + q.N]
        if w:
            if q.precision == heat.FP64:
                want = oracle.solve_threads(u0, 1, q.r, q.nt, simd=True)
            else:
                want = oracle.solve_f32c(u0.astype(np.float32), q.r, q.nt, T[j])
            return j, q, same_bits(res.u, want)
        cells = np.random.default_rng([54, j]).integers(0, q.N, 16)
        for i in cells:
            if q.precision == heat.FP64:
                c = np.array([oracle.cone(u0, int(i), q.r, q.nt)])
            else:   # the cone rounds its window of u0 to binary32 itself
                c = np.array([oracle.cone_f32c(u0, int(i), q.r, q.nt, T[j])], dtype=np.float32)
            ok = same_bits(res.u[i:i + 1], c)
            if not ok:
                return j, q, False
        return j, q, True

    items = [d for d in done if d[2] or d[3]]
    bad, n = [], 0
    with ThreadPoolExecutor(max(1, min(16, len(os.sched_getaffinity(0))))) as ex:
        for f in as_completed([ex.submit(verify, it) for it in items]):
            j, q, ok = f.result()
            n += 1
            if not ok:
                bad.append((j, q.N, q.nt, q.precision))
            if n % 200 == 0 or n == len(items):
                print(f"serving parity: {n}/{len(items)} checked, {len(bad)} mismatches, "
                      f"{time.perf_counter() - t0:.0f} s", flush=True)
    assert not bad, bad[:10]
