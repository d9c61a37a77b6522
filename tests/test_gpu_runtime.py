"""GPU tests of the C ABI's runtime helpers: the overflow flags read by
pgs_check_flags (PGS_ERR_CAPACITY on a real overflow, recovery after
growing), and a rasterizer forward + backward recorded with
pgs_graph_begin / pgs_graph_end and replayed with pgs_graph_launch, each
replay checked against eager calls with unrelated eager work and host
synchronisation in between."""

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import say

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda")


def test_check_flags_reports_capacity_overflow_and_recovery():
    from paper_2601_17354_amd import _lib
    from paper_2601_17354_amd import binding as B
    from paper_2601_17354_amd.raster import Rasterizer
    P, cam, _ = synth.cfg1_inputs(0)
    params = torch.as_tensor(P, device=DEV)
    flags = torch.zeros(1, dtype=torch.int32, device=DEV)
    assert B.pgs_check_flags(flags) == (_lib.PGS_OK, 0)
    R = Rasterizer(P.shape[1], 0, 128, 128, cached=True, capacity=100, entries=1 << 12)
    R.flags.zero_()
    R.forward(params, cam)
    st, word = B.pgs_check_flags(R.flags)
    say(f"  flags after an undersized forward: status {st} word {word}")
    assert st == _lib.PGS_ERR_CAPACITY and word & _lib.PGS_FLAG_PAIR_OVERFLOW
    need = int(R.num_pairs.item())
    assert need > 100
    R.forward_checked(params, cam)                  # grows and reruns
    assert B.pgs_check_flags(R.flags) == (_lib.PGS_OK, 0) and R.capacity >= need


@pytest.mark.parametrize("cached", [True, False])
def test_graph_of_forward_and_backward_replays_like_eager_calls(cached):
    from paper_2601_17354_amd import binding as B
    from paper_2601_17354_amd.raster import Rasterizer
    scene = synth.spheres_planes_scene(1)
    P = synth.surface_gaussians(scene, 20000, seed=5, sh_degree=0, logit_sigma=0.5)
    cam = synth.ring_cameras(60, 320, 240)[4]
    params = torch.as_tensor(P, device=DEV)
    rng = np.random.default_rng(7)
    dl = torch.as_tensor(rng.normal(size=(3, 240, 320)).astype(np.float32), device=DEV)
    eager = Rasterizer(P.shape[1], 0, 320, 240, cached=cached)
    graphed = Rasterizer(P.shape[1], 0, 320, 240, cached=cached)
    for r in (eager, graphed):
        r.forward_checked(params, cam)
        r.reserve(1.5)
    g_eager = torch.zeros_like(params)
    g_graph = torch.zeros_like(params)

    def step(r, grads):
        r.forward(params, cam)
        grads.zero_()
        r.backward(params, cam, dl, grads)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.pgs_graph_begin(s)
        try:
            step(graphed, g_graph)
        finally:
            graph = B.pgs_graph_end(s)
    torch.cuda.current_stream().wait_stream(s)
    try:
        for k in range(4):
            graphed.image.fill_(-1.0)
            g_graph.fill_(7.0)
            B.pgs_graph_launch(graph)
            step(eager, g_eager)
            junk = torch.randn(1 << 20, device=DEV)
            junk.mul_(3.0).sum().item()                 # unrelated eager work, host sync
            torch.cuda.synchronize()
            assert B.pgs_check_flags(graphed.flags)[1] == 0
            np.testing.assert_array_equal(graphed.image.cpu().numpy(), eager.image.cpu().numpy())
            ge, gg = g_eager.cpu().numpy(), g_graph.cpu().numpy()
            # float atomics may add in another order: compare per field
            for row in range(ge.shape[0]):
                scale = np.abs(ge[row]).max()
                assert np.abs(gg[row] - ge[row]).max() <= 1e-5 * scale + 1e-12, (k, row)
            say(f"  replay {k}: image equal, gradients within atomic-order noise")
    finally:
        torch.cuda.synchronize()
        B.pgs_graph_destroy(graph)
