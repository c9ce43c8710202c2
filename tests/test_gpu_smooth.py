"""Smooth forward and its adjoint on the GPU against the FP64 oracle.

Bars: smooth histograms within relative L2 1e-5 per histogram (arrivals in
fp64, weights and Gaussian samples in fp32); record gradients field by
field -- dL/dz, dL/da, dL/dn_x, dL/dn_y, dL/dn_z, each within relative L2
1e-4 over the sampled records, and each record's value within 1e-4 of its
field's RMS plus 1e-3 of itself (the fields have different units and
magnitudes, so one norm over all of them would let the largest hide the
others); map gradients (autograd through the hand-written adjoints) within
relative L2 1e-4 (albedo) and 1e-3 (depth) over the map, at the tap
kernels' radius and at the moment kernels' radii 12, 16 and 20."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_helpers import assert_parity, log, to_gpu
from pins_smooth import smooth_scene

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    n = np.linalg.norm(b)
    return np.linalg.norm(a - b) / n if n > 0 else np.linalg.norm(a)


FIELDS = ("dz", "da", "dn_x", "dn_y", "dn_z")


def _assert_record_grads(got, ref, what):
    """got, ref: [n, 8] record gradients (fields at 2..6)."""
    for j, name in enumerate(FIELDS):
        g, r = got[:, 2 + j], ref[:, 2 + j]
        e = _rel(g, r)
        rms = float(np.sqrt(np.mean(r * r))) if r.size else 0.0
        worst = float(np.max(np.abs(g - r) / (1e-4 * rms + 1e-3 * np.abs(r) + 1e-300))) if r.size else 0.0
        log(f"{what} {name}: rel-L2 {e:.2e}, worst record {worst:.2f} of its bound")
        assert e <= 1e-4, f"{what} {name}: rel-L2 {e:.3e}"
        assert worst <= 1.0, f"{what} {name}: a record is off by {worst:.2f} of its bound"


def _gpu_records(sc):
    import paper_2506_03747_amd as nl
    depth, albedo, mask = to_gpu(sc)
    rec, n = nl.patches_from_depth(depth, sc.patch_grid, albedo, mask, cosines=sc.cosines)
    return depth, albedo, mask, rec, n


SCENES = [
    dict(seed=601),
    dict(seed=602, cosines=False),
    dict(seed=603, standoff_m=0.7),
    dict(seed=604, scan=(7, 5), patches=(40, 33)),                   # ragged tiles, several waves
    dict(seed=605, scan=(1, 1), patches=(9, 9), fwhm_ps=30.0),
    dict(seed=606, scan=(5, 6), patches=(12, 10), n_bins=97, bin_ps=30.0, fwhm_ps=45.0),  # T not a multiple of 4
]
# support radii ceil(6 sigma) = 12, 16, 20: the forward and the adjoint by
# moments (the scenes above have other radii: the general tap loops)
RADII = [
    dict(seed=608, bin_ps=16.0, fwhm_ps=70.0),
    dict(seed=609, bin_ps=8.0, fwhm_ps=50.0, scan=(4, 5)),
    dict(seed=610, bin_ps=4.0, fwhm_ps=30.0, n_bins=1024, standoff_m=0.0),
    # T = 2048: the forward's moment rows do not fit in LDS, so it takes the
    # straight-line taps at radius 20; the adjoint stages two scan points
    dict(seed=614, bin_ps=4.0, fwhm_ps=30.0, n_bins=2048, scan=(3, 2)),
    # the moment kernels without cosines, with a stand-off, and with the
    # patches split over workgroups (few scan points, 4096 patches)
    dict(seed=615, bin_ps=8.0, fwhm_ps=50.0, cosines=False),
    dict(seed=616, bin_ps=16.0, fwhm_ps=70.0, standoff_m=0.7, n_bins=768),
    dict(seed=617, bin_ps=8.0, fwhm_ps=50.0, scan=(3, 2), patches=(64, 64)),
    # T not a multiple of 4: scalar window reads and stores in the adjoint's
    # correlation pass, scalar staging in the gather
    dict(seed=618, bin_ps=8.0, fwhm_ps=50.0, n_bins=517, scan=(3, 2)),
    # T = 1024: the forward's rows at the compile-time pitch, with the patches
    # split over 4 workgroups per tile (outputs by float atomics)
    dict(seed=626, bin_ps=8.0, fwhm_ps=50.0, n_bins=1024, scan=(3, 2), patches=(64, 64)),
]


@pytest.mark.parametrize("kw", SCENES + RADII, ids=[str(k["seed"]) for k in SCENES + RADII])
def test_smooth_forward_parity(kw):
    import torch
    import paper_2506_03747_amd as nl
    sc = smooth_scene(**kw)
    log(f"smooth forward {kw}")
    _, _, _, rec, n = _gpu_records(sc)
    tau = nl.forward_smooth(nl.params_of(sc), rec, n)
    torch.cuda.synchronize()
    assert_parity(tau.cpu().numpy(), oracle.forward_smooth(sc), what=f"smooth {kw}")


def test_smooth_window_edges():
    """Arrivals before and after the window still reach in-window bins."""
    import torch
    import paper_2506_03747_amd as nl
    sc = smooth_scene(607, n_bins=180, bin_ps=20.0)
    ref = oracle.forward_smooth(sc)
    o = oracle.forward(sc, want_tau=False, want_bins=True)
    b = o["bins"][o["bins"] != np.iinfo(np.int32).min]
    assert b.max() >= 180                      # some arrivals fall past the window
    _, _, _, rec, n = _gpu_records(sc)
    tau = nl.forward_smooth(nl.params_of(sc), rec, n)
    torch.cuda.synchronize()
    assert_parity(tau.cpu().numpy(), ref, what="edges")


@pytest.mark.parametrize("kw", SCENES[:4] + RADII, ids=[str(k["seed"]) for k in SCENES[:4] + RADII])
def test_adjoint_records_parity(kw):
    import torch
    import paper_2506_03747_amd as nl
    sc = smooth_scene(**kw)
    log(f"adjoint records {kw}")
    _, _, _, rec, n = _gpu_records(sc)
    G = np.random.default_rng(kw["seed"]).standard_normal((sc.n_scan, sc.n_bins)).astype(np.float32)
    gr = nl.adjoint(nl.params_of(sc), rec, n, torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    k = int(n.item())
    R = rec[:k].cpu().numpy()
    idx = R[:, 7].view(np.int32)
    ref = oracle.adjoint_records(sc, G.astype(np.float64))[idx]
    got = gr[:k].cpu().numpy().astype(np.float64)
    _assert_record_grads(got, ref, f"adjoint {kw['seed']}")
    assert not gr[k:].cpu().numpy().any()


def test_cfg5_smooth_and_adjoint_sampled():
    """The full 128x128 scan x 128x128 patch workload: sampled histograms of
    the smooth forward and sampled record gradients of the adjoint."""
    import torch
    import paper_2506_03747_amd as nl
    sc = scenes.cfg5()
    log("cfg5 smooth + adjoint")
    _, _, _, rec, n = _gpu_records(sc)
    prm = nl.params_of(sc)
    tau = nl.forward_smooth(prm, rec, n)
    torch.cuda.synchronize()
    H = sc.n_scan
    sub = np.sort(np.random.default_rng(55).choice(H, 512, replace=False)).astype(np.int32)
    ref = oracle.forward_smooth(sc, subset=sub)
    assert_parity(tau.cpu().numpy().reshape(H, -1)[sub], ref, what="cfg5 smooth")
    G = np.random.default_rng(56).standard_normal((H, sc.n_bins)).astype(np.float32)
    gr = nl.adjoint(prm, rec, n, torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    k = int(n.item())
    pick = np.sort(np.random.default_rng(57).choice(k, 512, replace=False))
    R = rec.cpu().numpy()
    idx = R[pick, 7].view(np.int32)
    want = oracle.adjoint_records(sc, G.astype(np.float64), subset=idx.astype(np.int32))
    got = gr.cpu().numpy()[pick].astype(np.float64)
    _assert_record_grads(got, want, "cfg5 adjoint")


def test_adjoint_staging_partial_and_empty_ranges():
    """The gather's double-buffered row staging over several stages.  With
    128x128 patches (4 blocks of 4096) the adjoint splits the 19x17 = 323 scan
    points into 128 ranges of 3 (T = 1024 at radius 16 leaves room for two
    buffers of two scan points): most ranges take a stage of two points, then
    one of a single point, in the other buffer; range 107 holds two points and
    ranges 108 .. 127 none.  Sampled record gradients against the oracle."""
    import torch
    import paper_2506_03747_amd as nl
    sc = smooth_scene(624, scan=(19, 17), patches=(128, 128), n_bins=1024, bin_ps=8.0, fwhm_ps=50.0)
    log("adjoint staging: 323 scan points x 16383 records")
    _, _, _, rec, n = _gpu_records(sc)
    G = np.random.default_rng(624).standard_normal((sc.n_scan, sc.n_bins)).astype(np.float32)
    gr = nl.adjoint(nl.params_of(sc), rec, n, torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    k = int(n.item())
    pick = np.sort(np.random.default_rng(625).choice(k, 512, replace=False))
    R = rec.cpu().numpy()
    idx = R[pick, 7].view(np.int32)
    want = oracle.adjoint_records(sc, G.astype(np.float64), subset=idx.astype(np.int32))
    got = gr.cpu().numpy()[pick].astype(np.float64)
    _assert_record_grads(got, want, "adjoint staging")
    assert not gr[k:].cpu().numpy().any()


AUTOGRAD = [
    dict(seed=611, scan=(12, 10), patches=(24, 20), n_bins=320),
    dict(seed=612, scan=(8, 8), patches=(16, 16), cosines=False, standoff_m=0.5),
    dict(seed=613, scan=(6, 7), patches=(15, 18), masked=True),
    # the moment kernels (k_smooth_mom, k_adj_moments, k_adjoint_mom):
    # support radius 12 (16 ps bins, 70 ps FWHM), 16 (8 ps, 50 ps: the
    # 128x128 adjoint workload's), 20 (4 ps, 30 ps)
    dict(seed=619, scan=(8, 8), patches=(16, 16), n_bins=512, bin_ps=16.0, fwhm_ps=70.0),
    dict(seed=620, scan=(8, 8), patches=(16, 16), n_bins=1024, bin_ps=8.0, fwhm_ps=50.0),
    dict(seed=621, scan=(6, 6), patches=(14, 14), n_bins=1024, bin_ps=4.0, fwhm_ps=30.0),
    # radius 16 with T + 2 Rs = 549, not a multiple of 4
    dict(seed=622, scan=(5, 7), patches=(16, 12), n_bins=517, bin_ps=8.0, fwhm_ps=50.0),
    # radius 16 with a stand-off, without cosines
    dict(seed=623, scan=(6, 6), patches=(12, 12), n_bins=1024, bin_ps=8.0, fwhm_ps=50.0, standoff_m=0.6,
         cosines=False),
]


@pytest.mark.parametrize("kw", AUTOGRAD, ids=[str(k["seed"]) for k in AUTOGRAD])
def test_autograd_matches_oracle_gradient(kw):
    """L = 1/2 ||tau_s - y||^2 through torch.autograd with the hand-written
    backward: depth and albedo gradients against the oracle's chain rule."""
    import torch
    import paper_2506_03747_amd as nl
    sc = smooth_scene(**kw)
    log(f"autograd {kw}")
    target = smooth_scene(kw["seed"] + 50, **{k: v for k, v in kw.items() if k != "seed"})
    target.depth = (target.depth + np.float32(0.003)).astype(np.float32)
    prm = nl.params_of(sc)
    td, ta, tm = to_gpu(target)
    trec, tn = nl.patches_from_depth(td, target.patch_grid, ta, tm, cosines=target.cosines)
    y = nl.forward_smooth(nl.params_of(target), trec, tn)
    depth, albedo, mask = to_gpu(sc)
    depth.requires_grad_(True)
    albedo.requires_grad_(True)
    tau = nl.smooth_transient(depth, albedo, sc.patch_grid, prm, mask)
    loss = 0.5 * ((tau - y) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    ref = oracle.smooth_grad(sc, y.detach().cpu().numpy().astype(np.float64))
    assert abs(loss.item() - ref["loss"]) <= 1e-4 * ref["loss"]
    e_a = _rel(albedo.grad.cpu().numpy(), ref["grad_albedo"])
    e_d = _rel(depth.grad.cpu().numpy(), ref["grad_depth"])
    log(f"  rel-L2 albedo {e_a:.2e} depth {e_d:.2e}")
    assert e_a <= 1e-4
    assert e_d <= 1e-3
