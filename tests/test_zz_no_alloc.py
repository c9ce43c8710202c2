"""The no-allocation forward (GPU): nlos_forward_noalloc, called through the
C ABI, gives nlos_forward's output bit for bit (the same kernels and record
summaries; where patches are split over workgroups the partial histograms
meet in float atomics, so there to 1e-6 per histogram), on two calls in a
row that share the library's scratch, the second with a smaller input; and
it rejects a record count beyond its scratch."""
import ctypes as C

import numpy as np
import pytest

import scenes
from gpu_helpers import assert_parity, gpu_patches, log

pytestmark = pytest.mark.gpu


def _noalloc(prm, patches, n_active, out):
    import torch
    from paper_2506_03747_amd._native import check, lib
    rc = lib().nlos_forward_noalloc(C.byref(prm), C.c_void_p(patches.data_ptr()), patches.shape[0],
                                    None if n_active is None else C.c_void_p(n_active.data_ptr()),
                                    C.c_void_p(out.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    check(rc, "nlos_forward_noalloc")


@pytest.mark.parametrize("first,second", [
    (lambda: scenes.cfg2(), lambda: scenes.cfg1()),
    (lambda: scenes.tiny(seed=530, scan=(9, 7), patches=(90, 80), n_bins=300, standoff_m=0.4),
     lambda: scenes.tiny(seed=531, scan=(4, 4), patches=(20, 10), n_bins=96, laser=(2, 2), standoff_m=0.3)),
    (lambda: scenes.tiny(seed=532, scan=(2, 2), patches=(160, 160), n_bins=256, bin_ps=20.0, fwhm_ps=60.0,
                         masked=False),
     lambda: scenes.tiny(seed=533, scan=(3, 3), patches=(12, 12), n_bins=64)),
], ids=["cfg2-then-cfg1", "tiny-then-nonconfocal", "split-then-tiny"])
def test_noalloc_matches_forward(first, second):
    import torch
    import paper_2506_03747_amd as nl
    for make in (first, second):
        sc = make()
        log(f"noalloc {sc.name}")
        patches, n_act = gpu_patches(sc)
        prm = nl.params_of(sc)
        ref = nl.forward(prm, patches, n_act)
        got = torch.full_like(ref, float("nan"))
        _noalloc(prm, patches, n_act, got)
        torch.cuda.synchronize()
        if nl.get_plan(prm, patches.shape[0])["n_split"] > 1:
            assert_parity(got.cpu().numpy(), ref.cpu().numpy().astype(np.float64), tol=1e-6,
                          what=f"noalloc {sc.name}")
        else:
            assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), f"noalloc {sc.name} differs"


def test_noalloc_rejects_beyond_scratch():
    import torch
    import paper_2506_03747_amd as nl
    from paper_2506_03747_amd._native import NLOS_ENOSPC, NLOS_NOALLOC_MAX_PATCHES, lib
    sc = scenes.tiny(seed=534, scan=(2, 2), patches=(8, 8), n_bins=64)
    prm = nl.params_of(sc)
    patches, n_act = gpu_patches(sc)
    out = torch.empty(nl.out_shape(prm), dtype=torch.float32, device="cuda")
    # capacity beyond the scratch (only the count is checked: nothing is read)
    rc = lib().nlos_forward_noalloc(C.byref(prm), C.c_void_p(patches.data_ptr()), NLOS_NOALLOC_MAX_PATCHES + 1,
                                    C.c_void_p(n_act.data_ptr()), C.c_void_p(out.data_ptr()), None)
    assert rc == NLOS_ENOSPC
