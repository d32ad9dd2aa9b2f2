"""Oracle of the comparison estimators the paper evaluates against its own
(Sec. 4.1, "Evaluation of Existing Estimators"; results in Sec. 5.1).
TEST INFRASTRUCTURE ONLY.

Pixel c holds the n shared samples x_i of its footprint's on-screen members
i (itself included), each drawn from member i's filter PMF p_i = f_i, with
texel values T_i. With f_c the pixel's own filter weights and
w_i = f_c(x_i) / p_i(x_i):

  is          standard importance sampling, Eq. (6): (1/n) sum_i w_i T_i
  mis         multiple importance sampling, balance heuristic, one sample
              per technique: sum_i f_c(x_i) T_i / sum_j p_j(x_i)  (n^2 PMFs)
  pmis        pairwise MIS (Bitterli) with the pixel's own technique as the
              canonical one: for each of the n-1 pairs (c, i), the balance
              heuristic between p_i and p_c / (n-1), each pair weighted
              1 / (n-1):
                m_i(x) = p_i(x) / ((n-1) p_i(x) + p_c(x))                    (i != c)
                m_c(x) = 1/(n-1) sum_{i != c} p_c(x) / (p_c(x) + (n-1) p_i(x))
              (the weights sum to 1 at every x; with equal PMFs every sample
              gets 1/n); estimate sum_i m_i(x_i) f_c(x_i) T_i / p_i(x_i)
              (2n PMFs); with n = 1 it is one-tap STF
  regression  control variate with the filter weights (Eq. (7), following
              the cited Owen, Eq. 9.11):
                (1/n) sum_i [w_i T_i - beta (w_i - 1)],
                beta = sum_i (w_i - wbar) w_i T_i / sum_i (w_i - wbar)^2,
              per channel; beta = 0 when every w_i is equal
  wis         the paper's estimator, Eq. (14) (stf_oracle.stf_filter_reuse)
and, for each, a clamped variant that limits the result per channel to the
range of the texels used (the samples with f_c(x_i) > 0).

Readings: the printed beta is read with f(x_i) as the texel value and w_i as
f_c(x_i)/p_i(x_i) (the ratio whose sum has expectation 1), which is Owen's
regression coefficient for the response w_i T_i on the control w_i; n counts
the on-screen members, repeated members of a LUT footprint count repeatedly.
"""
from __future__ import annotations

import numpy as np

from . import stf_oracle as so

ESTIMATORS = ("wis", "is", "mis", "pmis", "regression")


def _weight_of(s: dict, pix: np.ndarray, sx: np.ndarray, sy: np.ndarray) -> np.ndarray:
    """Filter weight of tile pixel `pix` (per tile, [n, 64] ids) at texel (sx, sy)."""
    tiles = np.arange(s["wx"].shape[0])[:, None]
    n = s["wx"].shape[-1]
    i0x = s["i0x"][tiles, pix]
    i0y = s["i0y"][tiles, pix]
    dx = np.mod(sx - (i0x - s["delta"]), s["tw"])
    dy = np.mod(sy - (i0y - s["delta"]), s["th"])
    inside = (dx < n) & (dy < n)
    wx = np.take_along_axis(s["wx"][tiles, pix], np.minimum(dx, n - 1)[..., None], -1)[..., 0]
    wy = np.take_along_axis(s["wy"][tiles, pix], np.minimum(dy, n - 1)[..., None], -1)[..., 0]
    return np.where(inside, wx * wy, 0.0)


def stf_filter_estimator(textures, uv, filt, seed, frame, footprint, estimator, clamp=False, lut=None,
                         tiles=None, diagnostics=None, share_selection=False):
    """Per slot (values [n, 64, C], selections [n, 64, 2]) of the comparison
    estimator `estimator` over the footprint's shared samples.

    diagnostics: an optional list that receives, per slot, a dict with
    "magnitude" [n, 64, C] (sum of the absolute terms the estimate adds up,
    the scale of its rounding error) and "spread" [n, 64] (for the
    regression estimator, sum (w_i - wbar)^2 / sum w_i^2, the conditioning of
    beta; 1 otherwise)."""
    if estimator == "wis" and not clamp and diagnostics is None:
        return so.stf_filter_reuse(textures, uv, filt, seed, frame, footprint, lut=lut, tiles=tiles,
                                   share_selection=share_selection)
    if estimator not in ESTIMATORS:
        raise ValueError(estimator)
    if tiles is None:
        tiles = so.all_tiles(uv.shape[1], uv.shape[0])
    members = so.footprint_members(footprint, lut)
    K = members.shape[1]
    keys = so.selection_slots(textures, share_selection)
    out = []
    for slot, tex in enumerate(textures):
        s = so.stf_samples(tex, uv, tiles, keys[slot], filt, seed, frame)
        ntile = s["p"].shape[0]
        own = np.tile(np.arange(64)[None, :], (ntile, 1))
        # member tables [ntile, 64, K]
        mem = np.broadcast_to(np.maximum(members, 0)[None], (ntile, 64, K))
        present = np.broadcast_to((members >= 0)[None], (ntile, 64, K)) & \
            np.take_along_axis(np.broadcast_to(s["valid"][:, None, :], (ntile, 64, 64)), mem, -1)
        tix = np.arange(ntile)[:, None, None]
        sx = s["sx"][tix, mem]
        sy = s["sy"][tix, mem]
        T = s["T"][tix, mem]                                    # [ntile, 64, K, C]
        p_i = s["p"][tix, mem]                                  # each member's own PMF at its pick
        own_b = np.broadcast_to(own[..., None], (ntile, 64, K))
        f_c = _weight_of(s, own_b.reshape(ntile, -1), sx.reshape(ntile, -1), sy.reshape(ntile, -1)).reshape(sx.shape)
        f_c = np.where(present, f_c, 0.0)
        n = present.sum(-1)                                     # [ntile, 64]
        w = np.where(present, f_c / np.where(present, p_i, 1.0), 0.0)
        C = T.shape[-1]
        aT = np.abs(np.where(present[..., None], T, 0.0))
        spread = np.ones(n.shape)
        with np.errstate(invalid="ignore", divide="ignore"):
            if estimator == "wis":
                val = np.sum(w[..., None] * np.where(present[..., None], T, 0.0), -2) / np.sum(w, -1)[..., None]
                mag = np.sum(w[..., None] * aT, -2) / np.sum(w, -1)[..., None]
            elif estimator == "is":
                val = np.sum(w[..., None] * np.where(present[..., None], T, 0.0), -2) / n[..., None]
                mag = np.sum(w[..., None] * aT, -2) / n[..., None]
            elif estimator in ("mis", "pmis"):
                # p_j(x_i) for every pair of members: [ntile, 64, K(i), K(j)]
                pj = np.zeros(sx.shape + (K,))
                for jj in range(K):
                    pix_j = np.broadcast_to(mem[..., jj:jj + 1], sx.shape)
                    pj[..., jj] = _weight_of(s, pix_j.reshape(ntile, -1), sx.reshape(ntile, -1),
                                             sy.reshape(ntile, -1)).reshape(sx.shape)
                pj = np.where(present[..., None, :] & present[..., :, None], pj, 0.0)
                if estimator == "mis":
                    den = pj.sum(-1)                                # sum_j p_j(x_i) >= p_i(x_i) > 0
                    coef = np.where(present, f_c / np.where(present, den, 1.0), 0.0)
                else:
                    # canonical technique: the member that is the pixel itself
                    is_c = present & (mem == own_b)
                    first_c = is_c & (np.cumsum(is_c, -1) == 1)
                    pc_at = np.sum(np.where(first_c[..., None, :], pj, 0.0), -1)          # p_c(x_i)
                    nm1 = np.maximum(n - 1, 1)[..., None]
                    dm = nm1 * p_i + pc_at
                    m_i = np.where(dm > 0, p_i / np.where(dm > 0, dm, 1.0), 0.0)
                    # m_c at x_c: 1/(n-1) sum over the other members j of p_c(x_c) / (p_c(x_c) + (n-1) p_j(x_c))
                    xc_row = np.argmax(first_c, -1)                 # index of the canonical sample
                    pj_at_xc = np.take_along_axis(pj, xc_row[..., None, None], -2)[..., 0, :]  # p_j(x_c) [.., K]
                    pc_xc = np.take_along_axis(p_i, xc_row[..., None], -1)[..., 0]            # p_c(x_c)
                    others = present & ~first_c
                    m_c = np.sum(np.where(others, pc_xc[..., None] / (pc_xc[..., None] + nm1 * pj_at_xc), 0.0), -1) \
                        / nm1[..., 0]
                    m_c = np.where(n == 1, 1.0, m_c)
                    m = np.where(first_c, m_c[..., None], np.where(others, m_i, 0.0))
                    coef = np.where(present, m * f_c / np.where(present, p_i, 1.0), 0.0)
                val = np.sum(coef[..., None] * np.where(present[..., None], T, 0.0), -2)
                mag = np.sum(np.abs(coef)[..., None] * aT, -2)
            else:                                                   # regression
                nn = n[..., None]
                wbar = np.sum(w, -1, keepdims=True) / nn
                dw = np.where(present, w - wbar, 0.0)
                wT = w[..., None] * np.where(present[..., None], T, 0.0)
                den = np.sum(dw * dw, -1)[..., None]
                beta = np.where(den > 0, np.sum(dw[..., None] * wT, -2) / np.where(den > 0, den, 1.0), 0.0)
                cv = np.sum(np.where(present, w - 1.0, 0.0), -1)[..., None]
                val = (np.sum(wT, -2) - beta * cv) / nn
                mag = (np.sum(np.abs(wT), -2) + np.abs(beta) * np.sum(np.abs(np.where(present, w - 1.0, 0.0)), -1)[..., None]) / nn
                spread = den[..., 0] / np.maximum(np.sum(w * w, -1), 1e-300)
        if clamp:
            used = present & (f_c > 0)
            big = np.where(used[..., None], T, np.inf).min(-2)
            small = np.where(used[..., None], T, -np.inf).max(-2)
            val = np.minimum(np.maximum(val, big), small)
        val = np.where(s["valid"][..., None], val, 0.0)
        assert val.shape[-1] == C
        if diagnostics is not None:
            diagnostics.append({"magnitude": np.where(s["valid"][..., None], mag, 0.0), "spread": spread})
        out.append((val, np.stack([s["sx"], s["sy"]], -1)))
    return out
