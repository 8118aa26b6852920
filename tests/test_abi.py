"""C ABI checks that need no GPU: the library loads, exports every function
that include/heat.h declares, and its host-side logic (validation, planner)
behaves as documented.  No kernel is launched here."""
import os
import re

import pytest

from paper_2307_01117_amd import heat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "heat.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(heat_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(heat.LIB_PATH):
        from paper_2307_01117_amd import build
        build.build()
    return heat.load()


def test_header_declares_binding_exports():
    assert declared_functions() == sorted(heat.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version(lib):
    assert "gfx950" in heat.version()


@pytest.mark.parametrize("kw,msg", [
    (dict(N=0, nparts=1, r=0.5, nt=1), "N must be"),
    (dict(N=10, nparts=0, r=0.5, nt=1), "nparts"),
    (dict(N=10, nparts=11, r=0.5, nt=1), "nparts"),
    (dict(N=10, nparts=1, r=0.6, nt=1), "r must be"),
    (dict(N=10, nparts=1, r=-0.1, nt=1), "r must be"),
    (dict(N=10, nparts=1, r=float("nan"), nt=1), "r must be"),
    (dict(N=10, nparts=1, r=0.5, nt=-1), "nt must be"),
])
def test_validation_without_device(lib, kw, msg):
    import numpy as np
    u = np.zeros(max(kw["N"], 1))
    rc = lib.heat_solve(u.ctypes.data, kw["N"], kw["nparts"], kw["r"], kw["nt"])
    assert rc == heat.HEAT_EINVAL
    assert msg in heat.last_error()


def test_null_pointers(lib):
    assert lib.heat_solve(None, 10, 1, 0.5, 1) == heat.HEAT_EINVAL
    assert lib.heat_solve_dev(None, 10, 1, 0.5, 1, 0, None, None, None) == heat.HEAT_EINVAL
    assert lib.heat_checksum_dev(None, 10, 0, None, None) == heat.HEAT_EINVAL


def test_planner_geometry(lib):
    p = heat.plan(100_000_000, 1000, heat.FP64)
    assert p["kernel"] == heat.KERNEL_TB
    K, T, G, S = (p["cells_per_lane"], p["steps_per_round"], p["waves_per_group"],
                  p["exchange_steps"])
    # the tile's span: one window, or G windows overlapping by 2S (S = K/4)
    span = G * 64 * K - (G - 1) * 2 * S if S else 64 * K
    assert S in (0, K // 4)
    H = (span - p["tile_cells"]) // 2            # halo: >= T, whole 128-byte lines
    assert H >= T and H % 16 == 0 and 3 * H <= 64 * K
    assert p["tiles"] == -(-100_000_000 // p["tile_cells"])
    assert p["rounds"] == -(-1000 // T)
    # binary64 / binary32 results do not depend on T: the planner splits the
    # run into an even number of equal rounds (no copy-back of the state)
    for nt in (2, 5, 97, 1000, 4999):
        for prec in (heat.FP64, heat.FP32):
            q = heat.plan(10**6, nt, prec)
            assert q["rounds"] % 2 == 0 and q["rounds"] * q["steps_per_round"] >= nt
            assert (q["rounds"] - 1) * q["steps_per_round"] < nt
    # the compensated form keeps its fixed T: a short run is one round
    q = heat.plan(1000, 5, heat.FP32C)
    assert q["rounds"] == 1 and q["steps_per_round"] == 5
    s = heat.plan(1000, 7, heat.FP64, kernel=heat.KERNEL_STEP)
    assert s["rounds"] == 7 and s["steps_per_round"] == 1
    assert heat.plan(1000, 0, heat.FP32C)["rounds"] == 0


def test_overridden_cells_per_lane_takes_rounds_that_fit(lib):
    """A tuned round length too deep for a caller's cells_per_lane (e.g. the
    binary64 1e8-cell rounds of 320 steps with 8-cell lanes) is cut to the
    deepest that fits instead of failing; an explicit one is still checked."""
    for prec in (heat.FP64, heat.FP32, heat.FP32C):
        for N in (10**3, 10**5, 3 * 10**6, 10**8):
            for K in (8, 16, 32, 64):
                if K == 64 and prec == heat.FP32C:
                    continue
                p = heat.plan(N, 1000, prec, kernel=heat.KERNEL_TB, cells_per_lane=K)
                T = p["steps_per_round"]
                assert p["cells_per_lane"] == K and 3 * ((T + 3) // 4 * 4) <= 64 * K, (prec, N, K)
                assert p["rounds"] * T >= 1000
    with pytest.raises(heat.HeatError):
        heat.plan(10**8, 1000, heat.FP64, cells_per_lane=8, steps_per_round=320)


def test_compensated_round_length_is_fixed(lib):
    """The compensated form's round length T is part of its result; it must
    not depend on N or on the configuration of tiles."""
    Ts = {heat.plan(N, 1000, heat.FP32C)["steps_per_round"] for N in (1, 1000, 10**6, 10**8)}
    assert len(Ts) == 1
    for K in (8, 16, 32):
        assert heat.plan(10**6, 1000, heat.FP32C, cells_per_lane=K)["steps_per_round"] in Ts


@pytest.mark.parametrize("cfg", [
    dict(kernel=7), dict(cells_per_lane=12), dict(steps_per_round=6), dict(register_form=4),
    dict(cells_per_lane=64, register_form=2),
    dict(cells_per_lane=8, steps_per_round=256), dict(waves_per_group=9), dict(waves_per_group=-1),
    dict(exchange=4), dict(exchange=-1),
    dict(exchange=2, waves_per_group=1, cells_per_lane=32),
    dict(exchange=2, waves_per_group=4, cells_per_lane=8),
    dict(exchange=3, waves_per_group=1, cells_per_lane=16),
])
def test_planner_rejects_bad_config(lib, cfg):
    with pytest.raises(heat.HeatError) as ei:
        heat.plan(10**6, 100, heat.FP64, **cfg)
    assert ei.value.code == heat.HEAT_EINVAL


@pytest.mark.parametrize("K,G", [(16, 2), (32, 4), (64, 4), (64, 8)])
def test_plan_exchange_geometry(lib, K, G):
    """Waves sharing a tile: G windows of 64K cells overlapping by 2S, S = K/4,
    minus the outer halo H >= T on each side; one lone-wave tile is
    64K - 2H.  The tile count covers the ring."""
    N, nt = 10**7, 1000
    x = heat.plan(N, nt, heat.FP64, cells_per_lane=K, waves_per_group=G, steps_per_round=16,
                  exchange=heat.EXCHANGE_LDS)
    one = heat.plan(N, nt, heat.FP64, cells_per_lane=K, waves_per_group=G, steps_per_round=16,
                    exchange=heat.EXCHANGE_NONE)
    S = K // 4
    assert x["exchange_steps"] == S and one["exchange_steps"] == 0
    H = (64 * K - one["tile_cells"]) // 2
    assert H >= x["steps_per_round"] and H % 4 == 0
    assert x["tile_cells"] == G * 64 * K - (G - 1) * 2 * S - 2 * H
    for p in (x, one):
        assert (p["tiles"] - 1) * p["tile_cells"] < N <= p["tiles"] * p["tile_cells"]


def test_tuned_exchange_falls_back_for_lone_shapes(lib, tmp_path):
    """A tuned exchange entry is dropped (not refused) when an override makes
    the shape unable to use it; an explicit request is refused."""
    saved = tmp_path / "orig.txt"
    heat.tune_save(str(saved))
    try:
        f = tmp_path / "x.txt"
        f.write_text("0 6 32 64 4 3 2\n")
        heat.tune_load(str(f))
        assert heat.plan(5_000_000, 1000, heat.FP64)["exchange_steps"] == 8
        assert heat.plan(5_000_000, 1000, heat.FP64, waves_per_group=1)["exchange_steps"] == 0
        assert heat.plan(5_000_000, 1000, heat.FP64, cells_per_lane=8)["exchange_steps"] == 0
        with pytest.raises(heat.HeatError):
            heat.plan(5_000_000, 1000, heat.FP64, waves_per_group=1, exchange=heat.EXCHANGE_LDS)
        for bad in ("0 6 32 64 1 3 2\n", "0 6 8 64 4 3 2\n", "0 6 32 64 4 3 5\n"):
            f.write_text(bad)
            with pytest.raises(heat.HeatError):
                heat.tune_load(str(f))
    finally:
        heat.tune_load(str(saved))


def test_step_kernel_rejects_compensated(lib):
    with pytest.raises(heat.HeatError):
        heat.plan(1000, 10, heat.FP32C, kernel=heat.KERNEL_STEP)


def test_tuning_table_roundtrip(lib, tmp_path):
    """The planner follows a loaded tuning table; the compensated form keeps
    its fixed round length whatever the table says; bad tables are refused."""
    saved = tmp_path / "orig.txt"
    heat.tune_save(str(saved))
    try:
        f = tmp_path / "t.txt"
        f.write_text("# p b K T wpg form\n0 6 16 48 4 1\n2 6 8 128 1 2\n")
        heat.tune_load(str(f))
        p = heat.plan(5_000_000, 1000, heat.FP64)
        assert (p["cells_per_lane"], p["waves_per_group"], p["register_form"]) == (16, 4, 1)
        assert p["steps_per_round"] <= 48
        c = heat.plan(5_000_000, 1000, heat.FP32C)
        assert c["cells_per_lane"] == 8 and c["steps_per_round"] == heat.plan(10, 1000, heat.FP32C)["steps_per_round"]
        bad = tmp_path / "bad.txt"
        bad.write_text("0 6 12 48 4 1\n")
        with pytest.raises(heat.HeatError):
            heat.tune_load(str(bad))
        # a malformed line stops the load with HEAT_EINVAL; the lines before it stay
        part = tmp_path / "part.txt"
        part.write_text("0 6 32 96 2 3 1\n0 6 32 96 9 3 1\n")
        with pytest.raises(heat.HeatError) as ei:
            heat.tune_load(str(part))
        assert ei.value.code == heat.HEAT_EINVAL
        p = heat.plan(5_000_000, 1000, heat.FP64)
        assert (p["cells_per_lane"], p["waves_per_group"], p["register_form"]) == (32, 2, 3)
        # seven columns: the exchange column is read (LDS for this shape)
        x = tmp_path / "x.txt"
        x.write_text("0 6 32 96 4 3 2\n")
        heat.tune_load(str(x))
        assert heat.plan(5_000_000, 1000, heat.FP64)["exchange_steps"] == 8
    finally:
        heat.tune_load(str(saved))


def test_library_built_from_this_tree(lib):
    """The library carries the sha256 of the sources it was built from, and
    it is the digest of the sources in this tree (the binding refuses a
    library built from others)."""
    from paper_2307_01117_amd.build import source_digest
    v = heat.version()
    assert v.startswith("heat-mi355x ") and v.rsplit(" ", 1)[-1] == source_digest()


def test_batch_flags_refused_without_wait(lib):
    """The graph and persistent batch modes report kernel-side failures only
    to a call that waits, so without HEAT_BATCH_WAIT they are refused before
    any device work."""
    for flags in (heat.BATCH_PERSISTENT, heat.BATCH_GRAPH,
                  heat.BATCH_PERSISTENT | heat.BATCH_GRAPH):
        assert lib.heat_solve_batch_dev(None, 0, None, flags) == heat.HEAT_EINVAL
        assert "HEAT_BATCH_WAIT" in heat.last_error()
    assert lib.heat_solve_batch_dev(None, 0, None, 8) == heat.HEAT_EINVAL


def test_noalloc_size_limit_checked_on_host(lib):
    """The no-allocation device form refuses rings whose scratch exceeds its
    static array before any device work (the pointer is never touched)."""
    fake = 256
    for N, prec in ((8_500_000, heat.FP64), (17_000_000, heat.FP32C)):
        assert lib.heat_solve_dev_noalloc(fake, N, 1, 0.5, 10, prec, None, None) == heat.HEAT_EINVAL
        assert "static scratch" in heat.last_error()
    assert lib.heat_solve_dev_noalloc(None, 10, 1, 0.5, 10, heat.FP64, None, None) == heat.HEAT_EINVAL


def test_tune_table_batch_lines(lib, tmp_path):
    """Batch class lines ("b precision bucket K G T") load, are written back
    by heat_tune_save, and a line naming a class that is not built is
    refused.  (Bucket 9, rings of 1e9 cells and more, which no test runs.)"""
    good = tmp_path / "good.txt"
    good.write_text("b 0 9 64 4 256\nb 2 9 32 1 64\n")
    heat.tune_load(str(good))
    out = tmp_path / "out.txt"
    heat.tune_save(str(out))
    text = out.read_text()
    assert "b 0 9 64 4 256" in text and "b 2 9 32 1 64" in text
    # K = G = T = 0 restores the batching form's own rule (no line is saved)
    rule = tmp_path / "rule.txt"
    rule.write_text("b 0 9 0 0 0\nb 2 9 0 0 0\n")
    heat.tune_load(str(rule))
    heat.tune_save(str(out))
    assert "b 0 9" not in out.read_text() and "b 2 9" not in out.read_text()
    for bad in ("b 2 9 64 1 64\n", "b 0 9 32 4 64\n", "b 0 9 64 1 66\n", "b 1 9 64 1 4000\n",
                "b 0 9 0 1 0\n"):
        f = tmp_path / "bad.txt"
        f.write_text(bad)
        with pytest.raises(heat.HeatError) as ei:
            heat.tune_load(str(f))
        assert ei.value.code == heat.HEAT_EINVAL


@pytest.mark.parametrize("K,G,T", [(8, 8, 64), (16, 4, 60), (32, 2, 96), (64, 4, 248)])
def test_planner_deep_exchange_geometry(lib, K, G, T):
    """Waves sharing a tile with the deep exchange (every K/2 steps): windows
    of 64K cells overlapping by 2S = K, the tile's outer halo H >= T."""
    N = 1_000_000
    p = heat.plan(N, 1000, heat.FP64, kernel=heat.KERNEL_TB, cells_per_lane=K,
                  steps_per_round=T, waves_per_group=G, exchange=heat.EXCHANGE_LDS_DEEP)
    S = K // 2
    assert p["exchange_steps"] == S and p["waves_per_group"] == G
    H = (G * 64 * K - (G - 1) * 2 * S - p["tile_cells"]) // 2
    assert H >= p["steps_per_round"] and 3 * H <= 64 * K
    assert p["tiles"] == -(-N // p["tile_cells"])
    # the K/4 exchange on the same shape overlaps by half as much
    if K >= 16:
        q = heat.plan(N, 1000, heat.FP64, kernel=heat.KERNEL_TB, cells_per_lane=K,
                      steps_per_round=T, waves_per_group=G, exchange=heat.EXCHANGE_LDS)
        assert q["exchange_steps"] == K // 4
        assert q["tile_cells"] - p["tile_cells"] == (G - 1) * (K - K // 2)


def test_tune_table_resident_lines(lib, tmp_path):
    """Resident kernel lines ("r precision quarter_bucket K T G form exchange
    min_steps", or with the shortest winning run and the gain at full load at
    each of three points, up to six per quarter decade) load and are written
    back by heat_tune_save (a line with one run length as that length at
    every point and gains 0, not recorded); all-zero fields clear the quarter
    decade; inconsistent shapes are refused.
    (Quarter decades 9 and 39: rings of 178 to 316 cells, and of 10^9.75 and
    more.)"""
    good = tmp_path / "good.txt"
    good.write_text("r 0 39 16 64 4 3 3 400 500 0 1250 1300 0\n"
                    "r 0 39 8 32 1 3 1 300 0 600 1100 1000 1200\nr 2 9 32 64 1 1 1 256\n")
    heat.tune_load(str(good))
    out = tmp_path / "out.txt"
    heat.tune_save(str(out))
    text = out.read_text()
    assert ("r 0 39 16 64 4 3 3 400 500 0 1250 1300 0\n"
            "r 0 39 8 32 1 3 1 300 0 600 1100 1000 1200\n") in text
    assert "r 2 9 32 64 1 1 1 256 256 256 0 0 0\n" in text
    # a file's lines replace the shapes of the quarter decades it names
    one = tmp_path / "one.txt"
    one.write_text("r 0 39 32 64 4 3 3 200 200 200 1300 1300 1300\n")
    heat.tune_load(str(one))
    heat.tune_save(str(out))
    text = out.read_text()
    assert "r 0 39 32 64 4 3 3 200 200 200 1300 1300 1300\n" in text
    assert "r 0 39 16 " not in text and "r 0 39 8 " not in text
    assert "r 2 9 32 64 1 1 1 256 256 256 0 0 0\n" in text
    # a comment longer than the loader's line buffer is skipped whole
    lengthy = tmp_path / "long.txt"
    lengthy.write_text("# " + "x" * 600 + "\nr 2 9 32 64 1 1 1 128\n")
    heat.tune_load(str(lengthy))
    heat.tune_save(str(out))
    assert "r 2 9 32 64 1 1 1 128 128 128 0 0 0\n" in out.read_text()
    seven = tmp_path / "seven.txt"
    seven.write_text("".join("r 1 9 %d %d 4 1 3 100\n" % (K, T)
                             for K, T in ((16, 16), (16, 32), (16, 48), (16, 64), (32, 16),
                                          (32, 32), (32, 48))))
    with pytest.raises(heat.HeatError) as ei:
        heat.tune_load(str(seven))
    assert ei.value.code == heat.HEAT_EINVAL and "more than 6" in str(ei.value)
    clear = tmp_path / "clear.txt"
    clear.write_text("r 0 39 0 0 0 0 0 0\nr 2 9 0 0 0 0 0 0\n")
    heat.tune_load(str(clear))
    heat.tune_save(str(out))
    assert "r 0 39 " not in out.read_text() and "r 2 9 " not in out.read_text()
    for bad in ("r 0 9 16 64 2 3 1 400\n",      # lone waves with 2 per group
                "r 1 9 16 64 4 3 3 400\n",      # binary32 in the alternating form
                "r 0 9 8 64 4 3 2 400\n",       # K/4 exchange with 8 cells per lane
                "r 0 9 16 66 4 3 3 400\n",      # T not a multiple of 4
                "r 0 9 16 64 4 3 3 0\n",       # no minimum run length
                "r 0 9 16 64 4 3 3 400 400 400 1 -5 1\n",  # negative gain
                "r 0 9 16 64 4 3 3 0 0 0 1 1 1\n",         # no winning run anywhere
                "r 0 9 16 64 4 3 3 400 1200\n",            # a partial line
                "r 0 40 16 64 4 3 3 400\n"):   # no quarter decade 40
        f = tmp_path / "bad.txt"
        f.write_text(bad)
        with pytest.raises(heat.HeatError) as ei:
            heat.tune_load(str(f))
        assert ei.value.code == heat.HEAT_EINVAL
