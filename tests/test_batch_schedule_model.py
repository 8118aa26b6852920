"""Host-side model of the fused batch launch's dependency rule.

In the persistent launch a work item (round k, tile t) may start once every
tile within H cells of tile t has finished round k-1.  The kernel finds those
tiles by walking left and right from t until H cells are covered.  This test
checks, on many ring geometries (including a last tile shorter than H and
rings shorter than one window), that the walk yields exactly the tiles that
(a) hold a cell the window needs for its output after up to H steps, and
(b) own a cell whose output another tile's window reads -- and then runs a
randomised interleaving of the whole schedule to confirm that every read
sees the right round and nothing is overwritten early.
"""
import random

import pytest


def walk_deps(t, tiles, N, W, H):
    """The kernel's rule, restated: tiles within H cells of tile t."""
    last_len = N - (tiles - 1) * W
    deps = {t}
    for step in (-1, 1):
        acc, q = 0, t
        g = 0
        while g + 1 < tiles and acc < H:
            q = (q + step) % tiles
            deps.add(q)
            acc += last_len if q == tiles - 1 else W
            g += 1
    return deps


def cells_of(t, tiles, N, W):
    lo = t * W
    return range(lo, min(N, lo + W))


def needed_tiles(t, tiles, N, W, H):
    """Tiles owning a cell within H of tile t's cells (the light cone of its
    outputs after at most H steps)."""
    owner = {}
    for q in range(tiles):
        for i in cells_of(q, tiles, N, W):
            owner[i] = q
    lo = t * W
    hi = min(N, lo + W)
    need = set()
    for i in range(lo - H, hi + H):
        need.add(owner[i % N])
    return need


@pytest.mark.parametrize("seed", range(40))
def test_walk_equals_light_cone(seed):
    rng = random.Random(seed)
    K = rng.choice([8, 16, 32])
    H = rng.choice([4, 16, 32, 48, 64, 96])
    if 3 * H > 64 * K:
        H = 4
    W = 64 * K - 2 * H
    N = rng.choice([1, 2, 5, W - 1, W, W + 1, W + H // 2, 2 * W + 3, 3 * W - 1,
                    5 * W + rng.randrange(1, W), 7 * W + H // 3 + 1])
    tiles = -(-N // W)
    for t in range(tiles):
        deps = walk_deps(t, tiles, N, W, H)
        need = needed_tiles(t, tiles, N, W, H)
        assert need <= deps, (N, W, H, t)
        # symmetric: t waits for q iff q waits for t (covers write-after-read)
        for q in deps:
            assert t in walk_deps(q, tiles, N, W, H)


@pytest.mark.parametrize("seed", range(10))
def test_random_interleaving_is_race_free(seed):
    rng = random.Random(1000 + seed)
    W, H = 40, 12
    N = rng.choice([W * 5 + 3, W * 6 + 11, W * 3 + 1, 17])
    tiles = -(-N // W)
    rounds = rng.randint(2, 7)
    # buffer state: for each buffer and cell, the round index of the value it holds
    buf = [[0] * N, [None] * N]
    done = [0] * tiles               # epoch counters
    started = {}
    pending = [(k, t) for k in range(rounds) for t in range(tiles)]
    while pending:
        ready = [(k, t) for (k, t) in pending
                 if all(done[q] >= k for q in walk_deps(t, tiles, N, W, H))]
        assert ready, "schedule deadlocked"
        k, t = rng.choice(ready)
        pending.remove((k, t))
        src, dst = buf[k & 1], buf[(k + 1) & 1]
        # every cell that can reach the outputs must hold round k
        for i in range(t * W - H, min(N, t * W + W) + H):
            assert src[i % N] == k, (k, t, i)
        for i in cells_of(t, tiles, N, W):
            # nobody still needing round k-1 data from this cell may be pending
            for (k2, t2) in pending:
                if k2 == k - 1 and t in needed_tiles(t2, tiles, N, W, H):
                    raise AssertionError("overwrote data still needed")
            dst[i] = k + 1
        done[t] = k + 1
