"""Pins of the oracle's sparse sharing-footprint generator (Sec. 4.3,
"Pseudorandom Sparse Footprints"; Sec. S5)."""
import numpy as np
import pytest

import oracle as o
from oracle import footprint_oracle as fo


def test_acceptance_table():
    T = fo.acceptance_table(1.4)
    assert T[0][0] == 1 << 32 and np.all(T[-1] == 1 << 32)
    assert np.all(np.diff(T[0].astype(np.float64)) <= 0) and T[0][1] > T[0][2] > T[0][4]   # decreasing
    assert np.all(T[1:-1] >= T[:-2])                              # relaxation widens
    assert abs(T[0][1] / 2 ** 32 - np.exp(-1 / (2 * 1.96))) < 1e-9


def test_first_draws_follow_the_discrete_normal():
    # the first accepted member of a set for the centre pixel q = (4, 4),
    # before any relaxation, is a rejection sample of exp(-r^2 / 2 s^2)
    # over the tile offsets other than (0, 0)
    sigma = 1.4
    firsts = []
    for r in range(40):
        cand = fo.candidates(r, 2, 64, sigma, seed=7)              # one member per set
        firsts.append(cand[4 * 8 + 4, :, 0])
    firsts = np.concatenate(firsts)
    dx, dy = firsts % 8 - 4, firsts // 8 - 4
    offs = [(x, y) for x in range(-4, 4) for y in range(-4, 4) if (x, y) != (0, 0)]
    w = np.array([np.exp(-(x * x + y * y) / (2 * sigma * sigma)) for x, y in offs])
    # relaxation only starts after 64 failed attempts, which is rare here
    p = w / w.sum()
    n = len(firsts)
    obs = np.array([np.sum((dx == x) & (dy == y)) for x, y in offs])
    chi2 = np.sum((obs - n * p) ** 2 / (n * p))
    assert chi2 < len(offs) + 6 * np.sqrt(2 * len(offs))


@pytest.mark.parametrize("k", [5, 9, 16])
def test_generated_sets_are_valid(k):
    lut, score = fo.generate(k=k, n_cand=16, sigma=1.4, trials=300, restarts=2, seed=3)
    assert lut.shape == (64, k - 1) and lut.dtype == np.uint8
    for q in range(64):
        row = lut[q].tolist()
        assert len(set(row)) == k - 1 and q not in row and max(row) < 64
    counts = np.bincount(lut.reshape(-1), minlength=64)
    assert score == int(np.sum(counts.astype(np.int64) ** 2))


def test_stage2_is_the_best_trial_and_stage3_a_local_minimum():
    cand = fo.candidates(0, 9, 16, 1.4, seed=5)
    choice, s2 = fo.stage2(cand, 0, 200, seed=5)
    # recount every trial independently
    key = np.uint32(5 ^ fo.KEY_STAGE2)
    best = None
    for t in range(200):
        with np.errstate(over="ignore"):
            h = o.pcg4d(np.arange(64, dtype=np.uint32), np.full(64, t, np.uint32), np.zeros(64, np.uint32),
                        np.full(64, key, np.uint32))
        ch = (h[0] % np.uint32(16)).astype(int)
        c = np.zeros(64, int)
        for q in range(64):
            for p in cand[q, ch[q]]:
                c[p] += 1
        s = int(np.sum(c * c))
        if best is None or s < best:
            best = s
    assert s2 == best
    final, s3 = fo.stage3(cand, choice)
    assert s3 <= s2
    for q in range(64):
        for j in range(16):
            alt = final.copy()
            alt[q] = j
            c = np.bincount(cand[np.arange(64), alt].reshape(-1), minlength=64)
            assert int(np.sum(c.astype(np.int64) ** 2)) >= s3


def test_sparse_footprints_use_lanes_more_evenly_than_3x3():
    # Sec. 4.3: the 3x3 square over-uses central lanes and under-uses the
    # tile's corners; the optimised sparse sets are more uniform
    members = o.footprint_members("square3x3")
    sq = np.bincount(members[members >= 0].reshape(-1), minlength=64) - 1   # minus the pixel itself
    lut, score = fo.generate(k=9, n_cand=16, sigma=1.4, trials=500, restarts=2, seed=1)
    counts = np.bincount(lut.reshape(-1), minlength=64)
    assert counts.sum() == sq.sum() == 64 * 8
    assert np.std(counts) < 0.5 * np.std(sq)


def test_sigma_sets_locality():
    # Sec. S5: larger sigma reaches farther lanes; the search still finds
    # nearly even usage (the ideal sum of squares is 64 * 8^2 = 4096)
    def stats(sigma):
        lut, score = fo.generate(k=9, n_cand=16, sigma=sigma, trials=300, restarts=2, seed=2)
        q = np.arange(64)[:, None]
        d = np.hypot(lut % 8 - q % 8, lut // 8 - q // 8)
        return d.mean(), score
    d1, s1 = stats(1.0)
    d2, s2 = stats(2.5)
    d3, s3 = stats(4.0)
    assert d1 < d2 < d3
    assert max(s1, s2, s3) < 1.02 * 4096
