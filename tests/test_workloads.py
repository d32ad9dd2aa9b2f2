"""The synthetic inputs have the stated shapes, ranges and magnifications."""
import numpy as np

import workloads as w


def test_perspective_plane_magnification_range_and_derivatives():
    uv, jx, jy, info = w.perspective_plane(480, 270, 2048, 2.0, 32.0)
    lo, hi = info["mag_min_axis"]
    assert abs(lo - 2.0) < 1e-6 and abs(hi - 32.0) < 0.5
    assert uv.dtype == np.float32 and uv.shape == (270, 480, 2)
    assert info["texel_extent"] < 2 ** 14          # keeps >= 9 sub-texel bits in FP32
    # analytic derivatives agree with finite differences of a float64 evaluation
    cam = w.PlaneCamera(480, 270, np.radians(info["pitch_deg"]), np.radians(info["fov_y_deg"]),
                        tile_len=info["tile_len"])
    uv64, ax, ay = cam.evaluate()
    cam_dx = w.PlaneCamera(480, 270, cam.pitch, cam.fov_y, tile_len=cam.tile_len, jitter=(1e-3, 0))
    cam_dy = w.PlaneCamera(480, 270, cam.pitch, cam.fov_y, tile_len=cam.tile_len, jitter=(0, 1e-3))
    fdx = (cam_dx.evaluate()[0] - uv64) / 1e-3
    fdy = (cam_dy.evaluate()[0] - uv64) / 1e-3
    assert np.allclose(fdx, ax, rtol=1e-2, atol=1e-9)
    assert np.allclose(fdy, ay, rtol=1e-2, atol=1e-9)


def test_textures_shapes_and_ranges():
    t = w.small_texture(0)
    assert t.shape == (256, 256, 4) and t.dtype == np.uint8
    uv = w.small_screen()
    assert uv.shape == (512, 512, 2)
    # uniform 8x: neighbouring pixels are 1/8 texel apart
    assert np.allclose(np.diff(uv[0, :, 0]) * 256, 1 / 8, atol=1e-5)
    assert np.array_equal(w.small_texture(0), w.small_texture(0))
