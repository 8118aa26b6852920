"""Host model of the resident kernel's tile geometry and edge exchange.

The resident kernel (csrc/resident.h) keeps every tile's windows in
registers for all steps and swaps tile edges through a tagged exchange area:
every exchange e writes the tile's first and last H owned cells into slots of
parity e & 1, each value carrying the tag of its epoch, and a tile reads its
halo from its neighbours' slots once their tags read e.  This model
re-implements its index arithmetic in NumPy -- windows of 64*K cells per wave
whose ends go stale by one cell per step (the lane rotation wraps inside the
window), the waves' S-cell edge swaps, the LDS copy of the tile's two edge
regions that edge and halo cells pass through, the slots each halo cell is read from (a walk over
the neighbouring tiles, the short last tile included), and the final store
into the ring -- and runs the tiles as independent actors in a random order
that respects only the kernel's waits.  Every interleaving must give the
oracle's bits (Section 2, Eq. (heat:discrete) on the periodic ring); a model
without the one-epoch run's final wait must not, and one with a single
parity of slots must deadlock or go wrong.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2307_01117_amd import inputs


def step_window(v, r):
    # one step of a whole window; its two end cells take the window's other
    # end as neighbour (the lane rotation), which only corrupts the edges
    left, right = np.roll(v, 1), np.roll(v, -1)
    return v + r * ((left - 2.0 * v) + right)


class Deadlock(Exception):
    pass


class Ring:
    def __init__(self, u0, K, G, XD, H, T, nt, r, final_wait=True, parities=2):
        self.N = N = len(u0)
        self.K, self.G, self.XD, self.H, self.T, self.nt, self.r = K, G, XD, H, T, nt, r
        self.S = K // XD if XD else 0
        self.WIN = 64 * K
        self.W = G * self.WIN - 2 * (G - 1) * self.S - 2 * H
        assert self.W >= H and N >= H
        self.tiles = -(-N // self.W)
        self.ring = np.array(u0, dtype=np.float64)
        self.slots = {}          # (parity, tile, side, j) -> (tag, value)
        self.flags = [0] * self.tiles
        self.final_wait = final_wait
        self.parities = parities

    def length(self, t):
        return min(self.W, self.N - t * self.W)

    def neighbours(self, t):
        """Tiles whose output lies within H of tile t (resident_wait_neighbours)."""
        out = []
        if self.tiles == 1:
            return out
        for direction in (-1, 1):
            acc, q, g = 0, t, 0
            while g + 1 < self.tiles and acc < self.H:
                q = (q + direction) % self.tiles
                out.append(q)
                acc += self.length(q)
                g += 1
        return out

    def halo_slot(self, t, i):
        """(tile, side, j) of halo cell i of tile t (edge_source): i < H is the
        cell H - i left of the tile, read from the last H cells (side 1) of the
        tile it falls in; i >= H the cell i - H right of its end, from the first
        H (side 0)."""
        H = self.H
        if i < H:
            d, q = H - i, t
            while True:
                q = (q - 1) % self.tiles
                L = self.length(q)
                if d <= L:
                    return q, 1, H - d
                d -= L
        d, q = i - H, t
        while True:
            q = (q + 1) % self.tiles
            L = self.length(q)
            if d < L:
                return q, 0, d
            d -= L

    def tile(self, t):
        """The kernel's work for tile t as a generator: it yields ('slots',
        [(key, tag), ...]) where the kernel polls its halo slots and ('flags',
        need) where it polls its neighbours' counters, and runs everything
        else (reads and writes of the shared memory) between yields."""
        N, K, G, XD, H, S, WIN, W = (self.N, self.K, self.G, self.XD, self.H, self.S,
                                     self.WIN, self.W)
        b = t * W
        wl = self.length(t)
        offs = [w * (WIN - 2 * S) if XD else 0 for w in range(G)]
        # window load from the ring (modulo N)
        v = [self.ring[(b - H + off + np.arange(WIN)) % N].copy() for off in offs]
        # the LDS copy holds two regions (resident_tile_cells): the runs that
        # meet tile coordinates [0, 2H) lie in [0, 2H + K), those that meet
        # [wl, wl + 2H) above b_lo; region B follows region A when disjoint
        cells = min(W + 2 * H, 4 * H + 3 * K + 4)
        a_end, b_lo = 2 * H + K, (wl - K) & ~3
        split = cells < W + 2 * H and b_lo >= a_end

        def at(c):
            return c - b_lo + a_end if split and c >= a_end else c

        class Lds:
            def __init__(self):
                self.m = np.full(cells, np.nan)

            def __setitem__(self, key, val):
                if isinstance(key, slice):
                    lo = at(key.start)
                    assert 0 <= lo and lo + (key.stop - key.start) <= cells
                    self.m[lo:lo + key.stop - key.start] = val
                else:
                    assert 0 <= at(key) < cells
                    self.m[at(key)] = val

            def __getitem__(self, key):
                if isinstance(key, slice):
                    lo = at(key.start)
                    assert 0 <= lo and lo + (key.stop - key.start) <= cells
                    return self.m[lo:lo + key.stop - key.start]
                assert 0 <= at(key) < cells
                return self.m[at(key)]

        tl = Lds()

        def exchange():
            if not XD:
                return
            new = [x.copy() for x in v]
            for w in range(1, G):
                new[w][:S] = v[w - 1][WIN - 2 * S:WIN - S]
                new[w - 1][WIN - S:] = v[w][S:2 * S]
            v[:] = new

        def lane_runs(pred):
            for w in range(G):
                for lane in range(64):
                    c0 = offs[w] + lane * K
                    if pred(c0):
                        yield w, lane, c0

        meets = lambda c0, a0, a1: c0 < a1 and a0 < c0 + K
        epoch, done = 0, 0
        while done < self.nt:
            steps = min(self.T, self.nt - done)
            if XD:
                s = 0
                while steps - s > S:
                    for _ in range(S):
                        v[:] = [step_window(x, self.r) for x in v]
                    exchange()
                    s += S
                for _ in range(steps - s):
                    v[:] = [step_window(x, self.r) for x in v]
            else:
                for _ in range(steps):
                    v[:] = [step_window(x, self.r) for x in v]
            done += steps
            if done >= self.nt:
                break
            epoch += 1
            exchange()
            par = epoch % self.parities
            for w, lane, c0 in lane_runs(lambda c: meets(c, 0, 2 * H) or meets(c, wl, wl + 2 * H)):
                tl[c0:c0 + K] = v[w][lane * K:lane * K + K]
            for i in range(2 * H):
                side, j = (0, i) if i < H else (1, i - H)
                p = j if side == 0 else wl - H + j
                if 0 <= p < wl:
                    self.slots[(par, t, side, j)] = (epoch, tl[H + p])
            keys = [(par,) + self.halo_slot(t, i) for i in range(2 * H)]
            yield ("slots", [(k, epoch) for k in keys])
            for i, k in enumerate(keys):
                tag, x = self.slots[k]
                assert tag == epoch
                p = i - H if i < H else wl + i - H
                tl[H + p] = x
            for w, lane, c0 in lane_runs(lambda c: meets(c, 0, H) or meets(c, wl + H, wl + 2 * H)):
                v[w][lane * K:lane * K + K] = tl[c0:c0 + K]
        if epoch == 0:
            # no exchange: a neighbour may not have loaded its window yet
            self.flags[t] = 1
            if self.final_wait:
                yield ("flags", 1)
        for w, off in enumerate(offs):
            lo = S if XD and w > 0 else H
            hi = WIN - S if XD and w + 1 < G else WIN - H
            for pos in range(lo, hi):
                pg = off + pos
                if H <= pg < H + wl:
                    self.ring[b + pg - H] = v[w][pos]

    def ready(self, t, wait):
        if wait is None:
            return True
        kind, need = wait
        if kind == "flags":
            return all(self.flags[q] >= need for q in self.neighbours(t))
        return all(self.slots.get(k, (0,))[0] == tag for k, tag in need)

    def run(self, seed):
        rng = np.random.default_rng(seed)
        gens = {t: self.tile(t) for t in range(self.tiles)}
        waiting = {t: None for t in gens}
        while gens:
            ready = [t for t in gens if self.ready(t, waiting[t])]
            if not ready:
                raise Deadlock()
            t = ready[rng.integers(len(ready))]
            try:
                waiting[t] = next(gens[t])
            except StopIteration:
                del gens[t]
        return self.ring


CASES = [
    # N, K, G, XD, H, T, nt: lone waves, both exchange depths, a short last tile
    # (shorter than H too), a single tile, odd and even exchange counts, runs
    # of T steps or fewer
    (3000, 8, 1, 0, 16, 16, 70),
    (2900, 8, 1, 0, 32, 24, 49),
    (5000, 16, 4, 4, 32, 32, 100),
    (4500, 16, 4, 2, 16, 12, 37),
    (4096 * 2 + 10, 16, 4, 4, 16, 16, 65),
    (4040 * 2 + 10, 16, 4, 4, 16, 16, 33),
    (3900, 16, 4, 4, 32, 20, 41),
    (900, 8, 2, 2, 16, 16, 50),
    (3000, 8, 1, 0, 16, 16, 12),         # no exchange: the counters' wait
    (3 * 480 + 44, 8, 1, 0, 16, 16, 40),  # last tile just short of the LDS split: one region
    (3 * 480 + 48, 8, 1, 0, 16, 16, 40),  # the shortest that splits: two
    (4040 * 2 + 10, 16, 4, 4, 16, 16, 16),
]


@pytest.mark.parametrize("case", CASES)
def test_resident_model_matches_oracle_any_order(case):
    N, K, G, XD, H, T, nt = case
    u0 = inputs.uniform_ring(N, (21, N))
    r = 0.4375
    want = oracle.solve(u0, r, nt)
    for seed in range(3):
        got = Ring(u0, K, G, XD, H, T, nt, r).run(seed)
        assert np.array_equal(got, want), (case, seed)


def test_resident_model_without_the_final_wait_fails():
    """A run of T steps or fewer makes no exchange, so nothing orders a tile's
    final store after its neighbours' window loads: a model without the
    counters' wait lets a fast tile overwrite cells a slow neighbour has still
    to load as halo."""
    N, K, G, XD, H, T, nt = 3000, 8, 1, 0, 16, 16, 12
    u0 = inputs.uniform_ring(N, 22)
    r = 0.4375
    want = oracle.solve(u0, r, nt)
    assert np.array_equal(Ring(u0, K, G, XD, H, T, nt, r).run(0), want)
    bad = 0
    for seed in range(40):
        got = Ring(u0, K, G, XD, H, T, nt, r, final_wait=False).run(seed)
        bad += not np.array_equal(got, want)
    assert bad > 0


def test_resident_model_with_one_parity_fails():
    """With one parity of slots a fast tile overwrites epoch e's edges with
    e + 1's before a slow neighbour has read them: the neighbour then polls
    for a tag that never comes back."""
    N, K, G, XD, H, T, nt = 3000, 8, 1, 0, 16, 16, 70
    u0 = inputs.uniform_ring(N, 23)
    r = 0.4375
    want = oracle.solve(u0, r, nt)
    bad = 0
    for seed in range(40):
        try:
            got = Ring(u0, K, G, XD, H, T, nt, r, parities=1).run(seed)
            bad += not np.array_equal(got, want)
        except Deadlock:
            bad += 1
    assert bad > 0
