"""The GPU sparse-footprint generator (Sec. 4.3, Sec. S5) against the oracle
generator: identical LUT and score (integer work, bit-exact), at small
sizes and at the paper's sizes (32 candidates, 10 000 trials, 30 restarts);
and filtering with generated, frame-cycled LUTs against the oracle."""
import numpy as np
import pytest

import oracle as o
from oracle import footprint_oracle as fo
import workloads as w

torch = pytest.importorskip("torch")
stf = pytest.importorskip("paper_2504_05562_amd")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,n_cand,sigma,trials,restarts,seed", [
    (9, 16, 1.4, 300, 3, 0), (5, 8, 0.8, 200, 2, 11), (16, 24, 2.2, 500, 4, 7), (2, 1, 1.0, 5, 1, 3),
    (64, 4, 3.0, 50, 2, 5)])
def test_generator_matches_oracle(k, n_cand, sigma, trials, restarts, seed):
    lut, score = stf.generate_footprints(k, n_cand, sigma, trials, restarts, seed)
    want, want_score = fo.generate(k, n_cand, sigma, trials, restarts, seed)
    torch.cuda.synchronize()
    assert np.array_equal(lut.cpu().numpy(), want)
    assert int(score.item()) == want_score


def test_generator_paper_sizes():
    lut, score = stf.generate_footprints(9, 32, 1.4, 10000, 30, 2)
    want, want_score = fo.generate(9, 32, 1.4, 10000, 30, 2)
    torch.cuda.synchronize()
    assert np.array_equal(lut.cpu().numpy(), want) and int(score.item()) == want_score
    assert want_score < 1.01 * 64 * 8 * 8


def test_frame_cycled_generated_footprints_filter_like_the_oracle():
    luts = stf.footprint_set(3, 9, 16, 1.4, 500, 4, seed=40)
    tex = w.small_texture(1, 64)
    uv = w.small_screen(96, 64, 64, 5.0, offset_seed=9)
    dt, duv = [torch.from_numpy(tex).cuda()], torch.from_numpy(uv).cuda()
    for frame in range(4):
        lut = luts[frame % 3]
        out = stf.filter_reuse(dt, duv, "lut", "bilinear", 2, frame, lut=lut)[0]
        (rv, _), = o.stf_filter_reuse([tex], uv, o.BILINEAR, 2, frame, "lut", lut=lut.cpu().numpy())
        want = o.tiles_to_image(rv, o.all_tiles(96, 64), 96, 64)
        got = out.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - want) <= 1e-5 * np.maximum(np.abs(want), 1.0))
