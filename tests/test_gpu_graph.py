"""The filter and adjoint calls under HIP graph capture (the benchmark times its launches
as one graph): the library launches on the caller's stream and allocates
nothing, so the calls can be captured. Every replay -- with eager work,
cleared outputs and synchronisations between the replays -- must equal the
eager result bit for bit (the forward pass is a pure function of its
inputs)."""
import numpy as np
import pytest

import workloads as w

torch = pytest.importorskip("torch")
stf = pytest.importorskip("paper_2504_05562_amd")

pytestmark = pytest.mark.gpu


def _inputs():
    uv = torch.from_numpy(w.perspective_plane(200, 120, 256, 1.5, 12.0)[0]).cuda()
    texs = [torch.from_numpy(w.plane_albedo(1, 256)).cuda(), torch.from_numpy(w.plane_normal(1, 256)).cuda()]
    return uv, texs


def _call(kind, texs, uv, outs, seed):
    if kind == "reuse":
        stf.filter_reuse(texs, uv, "tile8x8", "bicubic", seed, 0, out=outs)
    elif kind == "quad":
        stf.filter_reuse(texs, uv, "quad2x2", "bilinear", seed, 1, out=outs)
    elif kind == "quad_shared":                    # both textures 256^2: the one-size quad kernel
        stf.filter_reuse(texs, uv, "quad2x2", "bilinear", seed, 1, out=outs, share_selection=True)
    elif kind == "records_shared":                 # the one-size record kernel
        stf.filter_reuse(texs, uv, "square3x3", "bicubic", seed, 1, out=outs, share_selection=True)
    elif kind == "stf":
        stf.filter(texs, uv, "bicubic", seed, 0, out=outs)
    else:
        stf.filter_reference(texs, uv, "bicubic", out=outs)


@pytest.mark.parametrize("kind", ["reuse", "quad", "stf", "reference", "quad_shared", "records_shared"])
def test_graph_replays_equal_eager(kind):
    uv, texs = _inputs()
    H, W = uv.shape[:2]
    sets = [[torch.empty((H, W, int(t.shape[2])), device="cuda") for t in texs] for _ in range(3)]
    eager = []
    for k, outs in enumerate(sets):               # eager reference, one seed per set
        _call(kind, texs, uv, outs, seed=k)
        eager.append([o.clone() for o in outs])
    torch.cuda.synchronize()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for k, outs in enumerate(sets):
            _call(kind, texs, uv, outs, seed=k)
    other = [torch.empty_like(o) for o in sets[0]]
    for rep in range(4):
        for outs in sets:
            for o in outs:
                o.zero_()                          # a fill kernel, not a memset node
        _call(kind, texs, uv, other, seed=7 + rep)  # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, outs in enumerate(sets):
            for o, e in zip(outs, eager[k]):
                assert torch.equal(o, e), (kind, rep, k)


@pytest.mark.parametrize("fp", ["tile8x8", "self", "square3x3"])
def test_graph_replays_of_the_adjoint(fp):
    """stf_backward under capture: every replay (outputs cleared by a fill
    kernel, eager work in between) equals the eager adjoint to FP32 rounding
    (its global atomics sum in no fixed order)."""
    uv, texs = _inputs()
    H, W = uv.shape[:2]
    rng = np.random.default_rng(5)
    g = [torch.from_numpy(rng.standard_normal((H, W, int(t.shape[2]))).astype(np.float32)).cuda() for t in texs]
    dtex = [torch.zeros(t.shape[:2] + (int(t.shape[2]),), device="cuda") for t in texs]
    stf.backward(texs, uv, g, fp, "bicubic", 3, 1, dtex=dtex)
    torch.cuda.synchronize()
    eager = [d.clone() for d in dtex]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        stf.backward(texs, uv, g, fp, "bicubic", 3, 1, dtex=dtex)
    other = [torch.zeros_like(d) for d in dtex]
    for rep in range(4):
        for d in dtex:
            d.zero_()
        stf.backward(texs, uv, g, fp, "bicubic", 9 + rep, 0, dtex=other)   # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for d, e in zip(dtex, eager):
            scale = float(e.abs().max())
            assert scale > 0
            assert float((d - e).abs().max()) <= 1e-5 * scale, (fp, rep)
