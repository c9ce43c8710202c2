"""The single-request path captured in a HIP graph: every replay equals the
eager result (replays interleaved with other eager work and host
synchronisations; the kernels clear their own buffers, nothing is memset)."""
import numpy as np
import pytest

import scenes
from gpu_helpers import assert_parity, log, to_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("make", [scenes.cfg1,
                                  lambda: scenes.tiny(seed=900, scan=(2, 2), patches=(160, 160), n_bins=256,
                                                      bin_ps=20.0, fwhm_ps=60.0, masked=False)])
def test_graph_replays_match_eager(make):
    import torch
    import paper_2506_03747_amd as nl
    sc = make()
    log(f"graph {sc.name}")
    depth, albedo, mask = to_gpu(sc)
    prm = nl.params_of(sc)
    rec = torch.empty((sc.n_patch_total, 8), device="cuda")
    n_act = torch.empty(1, dtype=torch.int32, device="cuda")
    out = torch.empty(nl.out_shape(prm), device="cuda")

    def step():
        nl.patches_from_depth(depth, sc.patch_grid, albedo, mask, cosines=sc.cosines, out=rec, n_active=n_act)
        nl.forward(prm, rec, n_act, out=out)

    step()
    torch.cuda.synchronize()
    eager = out.cpu().numpy().astype(np.float64)
    other = scenes.tiny(seed=901)
    od, oa, om = to_gpu(other)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        step()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            step()
    torch.cuda.synchronize()
    for k in range(4):
        out.fill_(-1.0)
        p, n = nl.patches_from_depth(od, other.patch_grid, oa, om)      # eager work between replays
        nl.forward(nl.params_of(other), p, n)
        g.replay()
        torch.cuda.synchronize()
        assert_parity(out.cpu().numpy(), eager, tol=1e-6, what=f"replay {k}")
