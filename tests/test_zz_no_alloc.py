"""stf_footprint_generate_static (the footprint generator on the library's
static per-GPU workspace, for callers that cannot allocate) against
stf_footprint_generate with a caller workspace, through the C ABI: two calls
in a row, the second with a smaller input, each bit-identical; parameters
beyond the static workspace are refused on the host."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
stf = pytest.importorskip("paper_2504_05562_amd")

pytestmark = pytest.mark.gpu

CASES = [(9, 32, 1.4, 10000, 30, 11),      # the paper's settings (~0.5 MB of workspace)
         (5, 16, 1.0, 700, 4, 3)]          # smaller: the second call reuses the array


def test_static_workspace_matches_caller_workspace():
    lib = stf.library()
    for k, n_cand, sigma, trials, restarts, seed in CASES:
        prm = stf.FootprintParams(k, n_cand, sigma, trials, restarts, seed, 0)
        need = lib.stf_footprint_workspace_bytes(ctypes.byref(prm))
        assert 0 < need <= stf.FOOTPRINT_STATIC_BYTES
        want_lut, want_score = stf.generate_footprints(k, n_cand, sigma, trials, restarts, seed)
        lut = torch.full((64, k - 1), 255, dtype=torch.uint8, device="cuda")
        score = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        rc = lib.stf_footprint_generate_static(ctypes.byref(prm), ctypes.c_void_p(lut.data_ptr()),
                                               ctypes.c_void_p(score.data_ptr()), None)
        assert rc == 0, lib.stf_last_error()
        torch.cuda.synchronize()
        assert torch.equal(lut, want_lut), (k, n_cand, restarts)
        assert int(score.item()) == int(want_score.item())
        rows = lut.cpu().numpy()
        for q in range(64):
            assert len(set(rows[q].tolist())) == k - 1 and q not in rows[q]


def test_static_workspace_limit_refused():
    lib = stf.library()
    prm = stf.FootprintParams(64, 64, 1.4, 10, 64, 0, 0)        # 64*64*64*63 bytes of candidates
    assert lib.stf_footprint_workspace_bytes(ctypes.byref(prm)) > stf.FOOTPRINT_STATIC_BYTES
    rc = lib.stf_footprint_generate_static(ctypes.byref(prm), ctypes.c_void_p(4096), ctypes.c_void_p(None), None)
    assert rc == -1 and b"static limit" in lib.stf_last_error()
    # the library still works afterwards
    lut, score = stf.generate_footprints_static(5, 8, 1.4, 100, 2, 1)
    torch.cuda.synchronize()
    assert np.all(lut.cpu().numpy() < 64)
