"""FP64 numpy oracle of the paper's FFT ("light-cone") forward route.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the tests and the
benchmark's CPU baseline use it; the product never imports it.

Section 2 rewrites Eq. (1) with u = z^2 and v = (t c / 2)^2 as a 3-D
convolution of the resampled volume with a cone (Eq. (3)-(5)); Algorithm 1
steps 1.1-2.3 evaluate it with 3-D FFTs.  Written out here, step by step, in
the paper's order (readings of its garbled pieces are listed in the design
notes):

  V[x, y, j]    depth-to-volume (step 2.1): albedo at depth layer
                j = floor(D / dz), dz = c dt / 2 (the time-bin spacing in
                depth), 0 <= j < M; nothing where the pixel is absent.
  R_z           fold layer J = j + 1 to the fine sample u = J^2 (of M^2) with
                weight 1 / J (the 1 / sqrt(i) of R_z), then pairwise means,
                log2(M) times, back to M samples.
  PSF           on the (2N, 2N, 2M) grid of lateral offsets n = -N .. N-1
                cells at x = n / N (so that [-1, 1) spans the 2N cells and
                offset 0 is a grid point) and layers z = k / M, k = 0 .. 2M-1:
                1 at the layer k minimising |(4 slope)^2 (x^2 + y^2) - z| for
                each (x, y) (every layer attaining the minimum: the paper's
                "= 0" on a discrete grid) when k < M, else 0; slope =
                w / (M c dt); the cone's apex (zero time offset) is layer 0.
                Layers k >= M only reach times past the window; kept, they
                would wrap around the FFT's period into the first bins, so the
                2M-layer grid is the zero padding of a linear convolution.
                (Where the cone leaves the grid the minimum falls on the last
                layer, which this drops.)
  conv          F^-1[F(pad(R_z V)) . F(PSF laterally centred)], 3-D FFTs on the
                (2N, 2N, 2M) grid, kept [0, N) x [0, N) x [0, M).
  tau           back to time bins: time bin j (J = j + 1) spans the fine
                samples [j^2, (j+1)^2) of v; its value is the mean of the
                convolution over that span (coarse samples weighted by
                overlap), divided by v^(3/2) with v = (J dz)^2 -- Eq. (3),
                v^(3/2) tau = the convolution, sampled without dropping the
                coarse samples that fall between two squares; then the
                Gaussian jitter of step 2.3 (same taps as the direct operator).
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0


def rz_matrix(M: int) -> np.ndarray:
    """R_z after the pairwise means: [M coarse u-samples, M depth layers]."""
    if M < 1 or (M & (M - 1)) != 0:
        raise ValueError("M must be a power of two")
    fine = np.zeros((M * M, M))
    for J in range(1, M + 1):
        fine[J * J - 1, J - 1] = 1.0 / J            # (R_z)_{i, j} = 1 / sqrt(i) for i = j^2
    mtx = fine
    while mtx.shape[0] > M:
        mtx = 0.5 * (mtx[0::2] + mtx[1::2])         # average adjacent samples
    return mtx


def rt_matrix(M: int) -> np.ndarray:
    """Time resampling: [M time bins, M coarse v-samples], row j the overlap of
    the fine span [j^2, (j+1)^2) with each coarse sample's span [cM, (c+1)M),
    divided by the span's length 2j + 1 (a mean)."""
    R = np.zeros((M, M))
    for j in range(M):
        lo, hi = j * j, (j + 1) * (j + 1)
        for c in range(lo // M, min((hi - 1) // M, M - 1) + 1):
            ov = min(hi, (c + 1) * M) - max(lo, c * M)
            if ov > 0:
                R[j, c] = ov / (2 * j + 1)
    return R


def psf(N: int, M: int, slope: float) -> np.ndarray:
    """Boolean cone on the (2N, 2N, 2M) grid, laterally centred (index
    (N, N) of the unshifted grid moved to (0, 0))."""
    x = np.arange(-N, N, dtype=np.float64) / N
    z = np.arange(0, 2 * M, dtype=np.float64) / M
    X, Y = np.meshgrid(x, x, indexing="ij")
    res = np.abs((4.0 * slope) ** 2 * (X ** 2 + Y ** 2)[:, :, None] - z[None, None, :])
    cone = (res == res.min(axis=2, keepdims=True)).astype(np.float64)
    cone[:, :, M:] = 0.0
    return np.roll(cone, shift=(-N, -N), axis=(0, 1))


def volume(depth, albedo, mask, M: int, dz: float) -> np.ndarray:
    """V[x, y, j]: albedo (0.5 without a map) at layer floor(D / dz)."""
    D = np.asarray(depth, np.float64)
    A = np.full(D.shape, 0.5) if albedo is None else np.asarray(albedo, np.float64)
    present = np.isfinite(D) & (D > 0) & (A > 0)
    if mask is not None:
        present &= np.asarray(mask) != 0
    V = np.zeros(D.shape + (M,))
    with np.errstate(invalid="ignore"):
        j = np.floor(np.where(present, D, 0.0) / dz)
    ok = present & (j >= 0) & (j < M)
    ix, iy = np.nonzero(ok)
    V[ix, iy, j[ok].astype(np.int64)] = A[ok]
    return V


def taps(fwhm_ps: float, bin_ps: float) -> np.ndarray:
    """Normalised Gaussian jitter taps, R = ceil(2 sigma) (Section 2)."""
    if fwhm_ps == 0.0:
        return np.ones(1)
    sigma = fwhm_ps / (2.0 * math.sqrt(2.0 * math.log(2.0))) / bin_ps
    R = int(math.ceil(2.0 * sigma))
    j = np.arange(-R, R + 1)
    g = np.exp(-(j * j) / (2.0 * sigma * sigma))
    return g / g.sum()


def forward(scene, jitter: bool = True, return_parts: bool = False):
    """LCT forward of a confocal scene whose depth map is co-registered with
    its N x N relay grid (half side w, centred); T = M bins must be a power of
    two; no stand-off (time measured from the wall).  [N, N, M] fp64."""
    g, pg = scene.relay, scene.patch_grid
    N, M = int(g["nx"]), int(scene.n_bins)
    if g["ny"] != N or pg["nx"] != N or pg["ny"] != N or scene.laser is not None or scene.standoff_m != 0.0:
        raise ValueError("the FFT route needs a confocal N x N scan co-registered with the depth map, s = 0")
    w = float(g["half_x"])
    dt = scene.bin_ps * 1e-12
    dz = C_LIGHT * dt / 2.0
    slope = w / (M * C_LIGHT * dt)
    V = volume(scene.depth, scene.albedo, scene.mask, M, dz)
    Rz = rz_matrix(M)
    RV = np.einsum("cj,xyj->xyc", Rz, V)
    pad = np.zeros((2 * N, 2 * N, 2 * M))
    pad[:N, :N, :M] = RV
    conv = np.real(np.fft.ifftn(np.fft.fftn(pad) * np.fft.fftn(psf(N, M, slope))))[:N, :N, :M]
    J = np.arange(1, M + 1, dtype=np.float64)
    v = (J * dz) ** 2
    tau = np.einsum("jc,xyc->xyj", rt_matrix(M), conv) / v ** 1.5
    if jitter:
        k = taps(scene.fwhm_ps, scene.bin_ps)
        R = (len(k) - 1) // 2
        out = np.zeros_like(tau)
        for i in range(-R, R + 1):
            src = slice(max(0, -i), M - max(0, i))
            dst = slice(max(0, i), M - max(0, -i))
            out[:, :, dst] += k[i + R] * tau[:, :, src]
        tau = out
    if return_parts:
        return tau, dict(V=V, Rz=Rz, RV=RV, conv=conv, slope=slope, dz=dz)
    return tau
