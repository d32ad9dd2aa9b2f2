"""Oracle of the pseudorandom sparse sharing-footprint generator (Sec. 4.3,
"Pseudorandom Sparse Footprints"; Sec. S5). TEST INFRASTRUCTURE ONLY.

The generator is a three-stage search over the 64 pixels of the 8x8 tile
that one wavefront processes. Every pixel q gets K-1 other tile pixels to
share with (the pixel itself is always a member, so footprints have K
elements):

  stage 1  for every pixel, n_cand candidate sets of K-1 distinct other
           pixels drawn around it from a discrete normal distribution of
           standard deviation sigma, relaxed (widened) where draws keep
           failing, which happens near the tile borders;
  stage 2  `trials` random choices of one candidate set per pixel, scored
           by how unevenly the pixels are used for sharing (lower is
           better); the best choice is kept;
  stage 3  coordinate descent: sweep the pixels, give each the candidate
           set that lowers the score most, until a sweep changes nothing;
  restarts the whole search `restarts` times; the best result wins.

Readings (the paper gives the procedure in words only):
  * score: the paper ranks configurations by the standard deviation of the
    per-pixel usage counts. The total count is fixed (64 (K-1)), so the
    standard deviation orders configurations exactly as the integer
    sum of squared counts does; that integer is the score here, so every
    decision is exact.
  * usage counts exclude the pixel itself (a constant 1 per pixel).
  * normal draws: an offset (dx, dy) is proposed uniformly in [-7, 7]^2 and
    accepted with probability exp(-(dx^2 + dy^2) / (2 s^2)), i.e. the 2D
    normal of deviation s restricted to integer offsets (rejection
    sampling); a proposal outside the tile, equal to the pixel or already
    in the set is rejected.
  * relaxation: s = sigma * 1.25^L, L = min(attempt // 64, 7); at L = 7 any
    valid proposal is accepted. After 64 * 8 + 4096 attempts the set is
    completed with the lowest-numbered unused pixels (never reached in
    practice; it only bounds the loop).
  * ties: lowest trial index, lowest candidate index, lowest restart index.
  * random numbers: pcg4d (see stf_oracle.pcg4d) keyed as
        stage 1: pcg4d(q + 64 j, attempt, restart, seed ^ 0x5EED0001) -> (x, y, z, -)
                 dx = x mod 15 - 7, dy = y mod 15 - 7, accept iff z < T_L[dx^2 + dy^2]
        stage 2: pcg4d(q, trial, restart, seed ^ 0x5EED0002).x mod n_cand
    with T_L[r2] = floor(2^32 exp(-r2 / (2 (sigma 1.25^L)^2))) in FP64
    (T_7 = 2^32).
Pixels are numbered row-major in the tile: q = ly * 8 + lx, which is the
numbering of the footprint LUT the filtering kernels read.
"""
from __future__ import annotations

import numpy as np

from .stf_oracle import pcg4d

TILE = 8
KEY_STAGE1 = 0x5EED0001
KEY_STAGE2 = 0x5EED0002
ATTEMPTS_PER_LEVEL = 64
LEVELS = 8
ATTEMPT_CAP = ATTEMPTS_PER_LEVEL * LEVELS + 4096


def acceptance_table(sigma: float) -> np.ndarray:
    """T[L][r2] as uint64 (2^32 means always)."""
    T = np.zeros((LEVELS, 2 * 7 * 7 + 1), dtype=np.uint64)
    r2 = np.arange(T.shape[1], dtype=np.float64)
    for L in range(LEVELS - 1):
        s = sigma * 1.25 ** L
        T[L] = np.floor(4294967296.0 * np.exp(-r2 / (2.0 * s * s))).astype(np.uint64)
    T[LEVELS - 1] = 1 << 32
    return T


def candidates(restart: int, k: int, n_cand: int, sigma: float, seed: int) -> np.ndarray:
    """Stage 1 for one restart: [64, n_cand, k-1] tile pixel ids."""
    m = k - 1
    T = acceptance_table(sigma)
    nset = TILE * TILE * n_cand
    sid = np.arange(nset)
    q = sid % 64
    j = sid // 64
    qx, qy = q % TILE, q // TILE
    out = np.full((nset, m), -1, dtype=np.int64)
    filled = np.zeros(nset, dtype=np.int64)
    key = np.uint32((seed ^ KEY_STAGE1) & 0xFFFFFFFF)
    with np.errstate(over="ignore"):
        for a in range(ATTEMPT_CAP):
            act = filled < m
            if not act.any():
                break
            ids = sid[act]
            h = pcg4d((q[ids] + 64 * j[ids]).astype(np.uint32), np.full(ids.size, a, np.uint32),
                      np.full(ids.size, restart, np.uint32), np.full(ids.size, key, np.uint32))
            dx = (h[0] % np.uint32(15)).astype(np.int64) - 7
            dy = (h[1] % np.uint32(15)).astype(np.int64) - 7
            L = min(a // ATTEMPTS_PER_LEVEL, LEVELS - 1)
            ok = h[2].astype(np.uint64) < T[L][dx * dx + dy * dy]
            tx, ty = qx[ids] + dx, qy[ids] + dy
            ok &= (tx >= 0) & (tx < TILE) & (ty >= 0) & (ty < TILE)
            p = ty * TILE + tx
            ok &= p != q[ids]
            ok &= ~np.any(out[ids] == p[:, None], axis=1)
            acc = ids[ok]
            out[acc, filled[acc]] = p[ok]
            filled[acc] += 1
    for s_ in np.nonzero(filled < m)[0]:                 # completion (bounds the loop only)
        for p in range(64):
            if filled[s_] == m:
                break
            if p != q[s_] and p not in out[s_, : filled[s_]]:
                out[s_, filled[s_]] = p
                filled[s_] += 1
    return out.reshape(n_cand, 64, m).transpose(1, 0, 2).copy()


def usage_counts(cand: np.ndarray, choice: np.ndarray) -> np.ndarray:
    """How often each tile pixel is shared: [..., 64] for choice [..., 64]."""
    members = cand[np.arange(64), choice]                # [..., 64, k-1]
    flat = members.reshape(members.shape[:-2] + (-1,))
    lead = int(np.prod(flat.shape[:-1]))
    f2 = flat.reshape(lead, -1) + 64 * np.arange(lead)[:, None]
    counts = np.bincount(f2.reshape(-1), minlength=64 * lead).reshape(flat.shape[:-1] + (64,))
    return counts


def score_of(counts: np.ndarray) -> np.ndarray:
    return np.sum(counts.astype(np.int64) ** 2, axis=-1)


def stage2(cand: np.ndarray, restart: int, trials: int, seed: int):
    """Best of `trials` random choices: (choice [64], score)."""
    n_cand = cand.shape[1]
    key = np.uint32((seed ^ KEY_STAGE2) & 0xFFFFFFFF)
    t, q = np.meshgrid(np.arange(trials, dtype=np.uint32), np.arange(64, dtype=np.uint32), indexing="ij")
    with np.errstate(over="ignore"):
        h = pcg4d(q, t, np.full_like(q, restart), np.full_like(q, key))
    choice = (h[0] % np.uint32(n_cand)).astype(np.int64)                   # [trials, 64]
    scores = score_of(usage_counts(cand, choice))
    best = int(np.argmin(scores))                                          # first minimum
    return choice[best].copy(), int(scores[best])


def stage3(cand: np.ndarray, choice: np.ndarray):
    """Coordinate descent from `choice`: (choice, score)."""
    n_cand = cand.shape[1]
    choice = choice.copy()
    counts = usage_counts(cand, choice)
    score = int(score_of(counts))
    changed = True
    while changed:
        changed = False
        for q in range(64):
            base = counts.copy()
            np.subtract.at(base, cand[q, choice[q]], 1)
            trial = np.repeat(base[None, :], n_cand, axis=0)
            for j in range(n_cand):
                np.add.at(trial[j], cand[q, j], 1)
            s = score_of(trial)
            j = int(np.argmin(s))
            if s[j] < score:
                choice[q] = j
                counts = trial[j]
                score = int(s[j])
                changed = True
    return choice, score


def generate(k: int = 9, n_cand: int = 32, sigma: float = 1.4, trials: int = 10000, restarts: int = 30,
             seed: int = 0):
    """Sparse footprint LUT [64, k-1] (uint8 tile pixel ids, row-major) and
    its score (sum of squared usage counts)."""
    if not 2 <= k <= 64 or not 1 <= n_cand <= 64 or trials < 1 or restarts < 1 or sigma <= 0:
        raise ValueError("bad generator parameters")
    best = None
    for r in range(restarts):
        cand = candidates(r, k, n_cand, sigma, seed)
        choice, _ = stage2(cand, r, trials, seed)
        choice, score = stage3(cand, choice)
        if best is None or score < best[0]:
            best = (score, cand[np.arange(64), choice].astype(np.uint8))
    return best[1], best[0]
