"""The Python binding refuses output, gradient and LUT buffers the kernels
would write out of bounds through, before anything is launched."""
import numpy as np
import pytest

import workloads as w

torch = pytest.importorskip("torch")
stf = pytest.importorskip("paper_2504_05562_amd")

pytestmark = pytest.mark.gpu


def _inputs():
    tex = [torch.from_numpy(w.plane_albedo(0, 64)).cuda(), torch.from_numpy(w.plane_normal(0, 64)).cuda()]
    uv = torch.from_numpy(w.small_screen(24, 16, 64, 4.0)).cuda()
    return tex, uv


def test_output_buffers_checked():
    tex, uv = _inputs()
    good = [torch.empty((16, 24, 4), device="cuda"), torch.empty((16, 24, 2), device="cuda")]
    stf.filter_reuse(tex, uv, "tile8x8", out=good)
    bad_cases = [good[:1],                                                       # one short
                 [good[0], torch.empty((16, 24, 4), device="cuda")],             # wrong channels
                 [good[0], torch.empty((16, 23, 2), device="cuda")],             # wrong width
                 [good[0], torch.empty((16, 24, 2), device="cuda", dtype=torch.float16)],
                 [good[0], torch.empty((16, 48, 2), device="cuda")[:, ::2]],     # not contiguous
                 [good[0], torch.empty((16, 24, 2))]]                            # host memory
    for out in bad_cases:
        with pytest.raises(ValueError):
            stf.filter_reuse(tex, uv, "tile8x8", out=out)
        with pytest.raises(ValueError):
            stf.filter(tex, uv, out=out)
        with pytest.raises(ValueError):
            stf.filter_reference(tex, uv, out=out)


def test_backward_buffers_checked():
    tex, uv = _inputs()
    g = [torch.zeros((16, 24, 4), device="cuda"), torch.zeros((16, 24, 2), device="cuda")]
    d = [torch.zeros((64, 64, 4), device="cuda"), torch.zeros((64, 64, 2), device="cuda")]
    stf.backward(tex, uv, g, "tile8x8", dtex=d)
    with pytest.raises(ValueError):
        stf.backward(tex, uv, g[:1], "tile8x8", dtex=d)
    with pytest.raises(ValueError):
        stf.backward(tex, uv, g, "tile8x8", dtex=d[:1])
    with pytest.raises(ValueError):
        stf.backward(tex, uv, [g[0], torch.zeros((16, 24, 4), device="cuda")], "tile8x8", dtex=d)
    with pytest.raises(ValueError):
        stf.backward(tex, uv, g, "tile8x8", dtex=[d[0], torch.zeros((32, 64, 2), device="cuda")])
    with pytest.raises(ValueError):
        stf.filter_reuse(tex, uv, "lut", lut=torch.zeros((64, 4), dtype=torch.uint8))   # host LUT
    assert np.isfinite(d[0].cpu().numpy()).all()
