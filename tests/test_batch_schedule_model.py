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


@pytest.mark.parametrize("seed", range(24))
def test_chunked_publication_drains_and_is_race_free(seed):
    """The persistent launch as the kernel runs it: waves claim chunks of
    consecutive items (round-major over rings sorted by their rounds, then
    tiles), and a wave publishes the tiles it computed only at the end of its
    chunk or before it moves on to another ring or round.  Waits see only
    published counters.  Under random interleavings of a few waves the
    schedule never deadlocks, every window reads the right round and no
    round k-1 value is overwritten while a reader is still to come."""
    rng = random.Random(5000 + seed)
    W, H = 40, 12
    chunk = rng.choice([1, 2, 3, 4, 8])
    nwaves = rng.randint(1, 6)
    rings = [(rng.choice([17, W * 3 + 1, W * 5 + 3, W * 6 + 11, W * 2]), rng.randint(1, 6))
             for _ in range(rng.randint(1, 4))]
    rings.sort(key=lambda g: -g[1])                     # by rounds, descending
    tiles = [-(-N // W) for N, _ in rings]
    items = [(k, p, t) for k in range(max(r for _, r in rings))
             for p in range(len(rings)) if rings[p][1] > k for t in range(tiles[p])]
    buf = [[[0] * N, [None] * N] for N, _ in rings]
    computed = set()
    published = [[0] * tiles[p] for p in range(len(rings))]
    counter = 0
    waves = [dict(todo=[], pend=[], key=None) for _ in range(nwaves)]

    def deps_ready(k, p, t):
        N = rings[p][0]
        return all(published[p][q] >= k for q in walk_deps(t, tiles[p], N, W, H))

    def publish(w):
        for (p, t, e) in w["pend"]:
            published[p][t] = e
        w["pend"], w["key"] = [], None

    def compute(k, p, t):
        N = rings[p][0]
        src, dst = buf[p][k & 1], buf[p][(k + 1) & 1]
        for i in range(t * W - H, min(N, t * W + W) + H):
            assert src[i % N] == k, (k, p, t, i)
        for i in cells_of(t, tiles[p], N, W):
            for (k2, p2, t2) in items:
                if p2 == p and k2 == k - 1 and (k2, p2, t2) not in computed and \
                        t in needed_tiles(t2, tiles[p], N, W, H):
                    raise AssertionError("overwrote data still needed")
            dst[i] = k + 1
        computed.add((k, p, t))

    while len(computed) < len(items) or any(w["pend"] for w in waves):
        moves = []
        for w in waves:
            if not w["todo"]:
                if w["pend"] or counter < len(items):
                    moves.append(w)
            else:
                k, p, t = items[w["todo"][0]]
                if w["pend"] and w["key"] != (p, k):
                    moves.append(w)                 # publish before switching
                elif deps_ready(k, p, t):
                    moves.append(w)
        assert moves, "schedule deadlocked"
        w = rng.choice(moves)
        if not w["todo"]:
            if w["pend"]:
                publish(w)                          # end of its chunk
            else:
                w["todo"] = list(range(counter, min(len(items), counter + chunk)))
                counter += chunk
            continue
        k, p, t = items[w["todo"][0]]
        if w["pend"] and w["key"] != (p, k):
            publish(w)
            continue
        compute(k, p, t)
        w["todo"].pop(0)
        w["pend"].append((p, t, k + 1))
        w["key"] = (p, k)
    for p, (N, r) in enumerate(rings):
        assert all(e == r for e in published[p])
        assert all(v == r for v in buf[p][r & 1])
