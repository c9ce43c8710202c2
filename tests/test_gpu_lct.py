"""The paper's FFT (light-cone) route on the GPU against its numpy fp64
oracle, and against the direct operator on the GPU.

Bar: every histogram within relative L2 1e-5 of the oracle (fp64 transforms
on both sides, fp32 output); histograms the oracle leaves at transform noise
(norm below 1e-9 of the largest) within 1e-7 of the largest norm in absolute
terms.  Cross-check: correlation with the direct operator (cosines off, no
stand-off) above 0.9, as for the oracles."""
import numpy as np
import pytest

from gpu_helpers import gpu_forward, log, to_gpu
from oracle import lct as lct_oracle
from pins_lct import lct_scene

pytestmark = pytest.mark.gpu

CASES = [dict(N=16, M=256, bin_ps=32.0, seed=1),
         dict(N=32, M=512, seed=2),
         dict(N=32, M=512, seed=3, half=1.0, zlo=0.5, zhi=1.1),
         dict(N=24, M=256, bin_ps=32.0, seed=4, masked=False),
         dict(N=8, M=64, bin_ps=120.0, seed=5, zlo=0.2, zhi=0.9, fwhm_ps=0.0)]


def _gpu_lct(sc, no_albedo=False):
    import torch
    import paper_2506_03747_amd as nl
    depth, albedo, mask = to_gpu(sc)
    prm = nl.params_of(sc)
    tau = nl.lct_forward(prm, depth, None if no_albedo else albedo, mask)
    torch.cuda.synchronize()
    return tau.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("kw", CASES, ids=[str(k["seed"]) for k in CASES])
def test_lct_parity(kw):
    sc = lct_scene(**kw)
    log(f"lct {kw}")
    got = _gpu_lct(sc)
    ref = lct_oracle.forward(sc)
    g = got.reshape(-1, sc.n_bins)
    r = ref.reshape(-1, sc.n_bins)
    nr = np.linalg.norm(r, axis=1)
    big = nr > 1e-9 * nr.max()
    err = np.linalg.norm(g - r, axis=1)
    assert np.all(err[big] <= 1e-5 * nr[big]), float((err[big] / nr[big]).max())
    assert np.all(err[~big] <= 1e-7 * nr.max())


def test_lct_default_albedo():
    sc = lct_scene(N=16, M=256, bin_ps=32.0, seed=6)
    got = _gpu_lct(sc, no_albedo=True)
    sc.albedo = None
    ref = lct_oracle.forward(sc)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("kw", [dict(), dict(half=1.0, zlo=0.5, zhi=1.1)], ids=["1m", "2m"])
def test_lct_correlates_with_direct(kw):
    sc = lct_scene(**kw)
    got = _gpu_lct(sc)
    direct, _, _ = gpu_forward(sc)
    r = float(np.corrcoef(got.ravel(), direct.cpu().numpy().ravel().astype(np.float64))[0, 1])
    log(f"  corr {r:.4f}")
    assert r > 0.9
