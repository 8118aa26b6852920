"""Host model of the resident kernel's tile geometry and edge exchange.

The resident kernel (csrc/resident.h) keeps every tile's windows in
registers for all steps and swaps tile edges through two ring buffers,
ordered by per-tile epoch counters.  This model re-implements its index
arithmetic in NumPy -- windows of 64*K cells per wave whose ends go stale by
one cell per step (the lane rotation wraps inside the window), the waves'
S-cell edge swaps, the LDS copy of the tile that edge and halo cells pass
through, the publication of the first and last H owned cells into buf[e & 1],
the halo reads, and the final store into buf[0] -- and runs the tiles as
independent actors in a random order that respects only the kernel's waits.
Every interleaving must give the oracle's bits (Section 2, Eq.
(heat:discrete) on the periodic ring); a model with a wait dropped must not.
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


class Ring:
    def __init__(self, u0, K, G, XD, H, T, nt, r, final_wait=True):
        self.N = N = len(u0)
        self.K, self.G, self.XD, self.H, self.T, self.nt, self.r = K, G, XD, H, T, nt, r
        self.S = K // XD if XD else 0
        self.WIN = 64 * K
        self.W = G * self.WIN - 2 * (G - 1) * self.S - 2 * H
        assert self.W >= H and N >= H
        self.tiles = -(-N // self.W)
        self.buf = [np.array(u0, dtype=np.float64), np.full(N, np.nan)]
        self.flags = [0] * self.tiles
        self.final_wait = final_wait

    def neighbours(self, t):
        """Tiles whose output lies within H of tile t (resident_wait_neighbours)."""
        out = []
        if self.tiles == 1:
            return out
        last_len = self.N - (self.tiles - 1) * self.W
        for direction in (-1, 1):
            acc, q, g = 0, t, 0
            while g + 1 < self.tiles and acc < self.H:
                q = (q + direction) % self.tiles
                out.append(q)
                acc += last_len if q == self.tiles - 1 else self.W
                g += 1
        return out

    def tile(self, t):
        """The kernel's work for tile t as a generator: it yields ('wait', need)
        where the kernel polls its neighbours' counters, and runs everything
        else (reads and writes of the shared buffers) between yields."""
        N, K, G, XD, H, S, WIN, W = (self.N, self.K, self.G, self.XD, self.H, self.S,
                                     self.WIN, self.W)
        b = t * W
        wl = min(W, N - b)
        offs = [w * (WIN - 2 * S) if XD else 0 for w in range(G)]
        # window load from buf[0] (modulo N)
        v = [self.buf[0][(b - H + off + np.arange(WIN)) % N].copy() for off in offs]
        tl = np.full(W + 2 * H, np.nan)

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
            pub = self.buf[epoch & 1]
            for w, lane, c0 in lane_runs(lambda c: meets(c, 0, 2 * H) or meets(c, wl, wl + 2 * H)):
                tl[c0:c0 + K] = v[w][lane * K:lane * K + K]
            for i in range(2 * H):
                p = i if i < H else wl - 2 * H + i
                if 0 <= p < wl:
                    pub[b + p] = tl[H + p]
            self.flags[t] = epoch
            yield ("wait", epoch)
            for i in range(2 * H):
                p = i - H if i < H else wl + i - H
                q = b + p
                q = q + N if q < 0 else q - N if q >= N else q
                tl[H + p] = pub[q]
            for w, lane, c0 in lane_runs(lambda c: meets(c, 0, H) or meets(c, wl + H, wl + 2 * H)):
                v[w][lane * K:lane * K + K] = tl[c0:c0 + K]
        R = epoch + 1
        self.flags[t] = R
        if R & 1 and self.final_wait:
            yield ("wait", R)
        for w, off in enumerate(offs):
            lo = S if XD and w > 0 else H
            hi = WIN - S if XD and w + 1 < G else WIN - H
            for pos in range(lo, hi):
                pg = off + pos
                if H <= pg < H + wl:
                    self.buf[0][b + pg - H] = v[w][pos]

    def run(self, seed):
        rng = np.random.default_rng(seed)
        gens = {t: self.tile(t) for t in range(self.tiles)}
        waiting = {t: None for t in gens}   # need, or None = ready to run
        while gens:
            ready = [t for t in gens if waiting[t] is None or
                     all(self.flags[q] >= waiting[t] for q in self.neighbours(t))]
            assert ready, "deadlock"
            t = ready[rng.integers(len(ready))]
            try:
                _, need = next(gens[t])
                waiting[t] = need
            except StopIteration:
                del gens[t]
        return self.buf[0]


CASES = [
    # N, K, G, XD, H, T, nt: lone waves, both exchange depths, a short last tile
    # (shorter than H too), a single tile, odd and even exchange counts
    (3000, 8, 1, 0, 16, 16, 70),
    (2900, 8, 1, 0, 32, 24, 49),
    (5000, 16, 4, 4, 32, 32, 100),
    (4500, 16, 4, 2, 16, 12, 37),
    (4096 * 2 + 10, 16, 4, 4, 16, 16, 65),
    (4040 * 2 + 10, 16, 4, 4, 16, 16, 33),
    (3900, 16, 4, 4, 32, 20, 41),
    (900, 8, 2, 2, 16, 16, 50),
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
    """The final store into buf[0] after an odd number of epochs must wait
    for the neighbours' last halo reads: a model without that wait lets a
    fast tile overwrite edges a slow neighbour still has to read."""
    N, K, G, XD, H, T, nt = 3000, 8, 1, 0, 16, 16, 40     # 3 rounds: R odd
    u0 = inputs.uniform_ring(N, 22)
    r = 0.4375
    want = oracle.solve(u0, r, nt)
    bad = 0
    for seed in range(40):
        got = Ring(u0, K, G, XD, H, T, nt, r, final_wait=False).run(seed)
        bad += not np.array_equal(got, want)
    assert bad > 0
