"""The ensemble launch-shape tuner's selection logic on the host, with a
stand-in for the batch whose step time follows a cost model of the shape and
a fake clock: the tuner finds the cheapest shape, and a box that leaves the
physical range (whose later steps take the cheap skip path) makes it restore
the saved state and time the shape again rather than favour the shapes timed
after it."""
import numpy as np
import pytest

from paper_1004_1680_amd import autotune, mhd

BEST = (2048, 64, 1, 128, 1)


class Clock:
    def __init__(self):
        self.t = 0.0

    def perf_counter(self):
        return self.t


class FakeBatch:
    """steps cost cost(shape); after `blowup` steps from a set state one box
    leaves the physical range and every later step costs half"""

    def __init__(self, clock, blowup):
        self.clock = clock
        self.dims = [(32, 32, 32), (64, 64, 64)]
        self.prec = mhd.MHD_F32
        self.nbox = len(self.dims)
        self.keys = {mhd.MHD_BATCH_GRID_X: 1024, mhd.MHD_BATCH_CHUNK: 64, mhd.MHD_BATCH_REVERSE: 2,
                     mhd.MHD_BATCH_PAIR_CHUNK: 128, mhd.MHD_BATCH_MIDDLE: 0}
        self.blowup = blowup
        self.since_set = 0
        self.bad = False
        self.restores = 0

    def get_state(self, i):
        return np.full(4, float(i))

    def set_state(self, i, s):
        self.since_set = 0
        self.bad = False
        self.restores += 1

    def set_launch(self, k, v):
        self.keys[k] = v

    def shape(self):
        k = self.keys
        return (k[mhd.MHD_BATCH_GRID_X], k[mhd.MHD_BATCH_CHUNK], k[mhd.MHD_BATCH_REVERSE],
                k[mhd.MHD_BATCH_PAIR_CHUNK], k[mhd.MHD_BATCH_MIDDLE])

    def launch(self, k):
        if k == mhd.MHD_BATCH_MIDDLE:
            g, c, r, pc, m = self.shape()
            return m if r == 1 else 2
        return self.keys[k]

    def cost(self):
        g, c, r, pc, m = self.shape()
        t = 1.0 + 0.1 * (g != 2048) + 0.05 * (c != 64) + (0.3 if r == 2 else 0.05 * (pc != 128))
        if r == 1 and m == 1:
            t -= 0.1
        return t * (0.5 if self.bad else 1.0)

    def run(self, n, cfl, graph=True):
        for _ in range(n):
            self.clock.t += self.cost()
            self.since_set += 1
            if self.blowup and self.since_set >= self.blowup:
                self.bad = True

    def status(self, raise_on_nonphysical=True):
        return np.zeros(self.nbox, dtype=np.int64), np.array([int(self.bad)] + [0] * (self.nbox - 1))


@pytest.mark.parametrize("blowup", [0, 40])
def test_tuner_picks_the_cheapest_shape(monkeypatch, tmp_path, blowup):
    clock = Clock()
    monkeypatch.setattr(autotune, "time", clock)
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "cache.json"))
    B = FakeBatch(clock, blowup)
    shape = autotune.tune_batch(B, use_cache=False)
    assert (shape["grid"], shape["chunk"], shape["reverse"], shape["pair_chunk"], shape["middle"]) == BEST
    assert B.shape() == BEST
    if blowup:
        # restored during the search, before the final timings and at the end
        assert B.restores > 2 * B.nbox * 5
    else:
        # the four final timings and the end
        assert B.restores == 5 * B.nbox


def test_tuner_cache_round_trip(monkeypatch, tmp_path):
    clock = Clock()
    monkeypatch.setattr(autotune, "time", clock)
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "cache.json"))
    B = FakeBatch(clock, 0)
    first = autotune.tune_batch(B, use_cache=True)
    C = FakeBatch(clock, 0)
    t0 = clock.t
    again = autotune.tune_batch(C, use_cache=True)
    assert again == first and clock.t == t0          # from the cache: no step run
    assert C.shape() == BEST
