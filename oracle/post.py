"""FP64 reference of the post-transfer products: Gaussian beam convolution and
the l,v mean projection.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the benchmark's CPU leg may use it; the product path never
does. Plain NumPy, written from the paper:

  beam_convolve -- "Beam Convolution": the ideal PPV cube convolved over its two
                   sky axes with a Gaussian beam given by its full width at half
                   maximum.
  lv_mean       -- the l,v projections of the paper's figures: the mean of a PPV
                   cube over one sky axis.

Readings (the paper states neither): the beam is a Gaussian sampled at pixel
offsets, sigma = FWHM / (2 sqrt(2 ln 2)), truncated at |offset| <= ceil(4 sigma)
along each axis and normalised to unit sum over that square; the sky beyond the
map is empty (zero padding). The FWHM is given in pixels; an angular beam needs
the pixel's angular size, which the caller supplies.
"""

from __future__ import annotations

import math

import numpy as np


def beam_sigma(fwhm_pix: float) -> float:
    return fwhm_pix / (2.0 * math.sqrt(2.0 * math.log(2.0)))


def beam_radius(fwhm_pix: float) -> int:
    return int(math.ceil(4.0 * beam_sigma(fwhm_pix)))


def beam_kernel(fwhm_pix: float) -> np.ndarray:
    """The 2-D beam [2R+1][2R+1], unit sum."""
    s = beam_sigma(fwhm_pix)
    r = beam_radius(fwhm_pix)
    i = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2.0 * s * s))
    return k / k.sum()


def beam_convolve(cube: np.ndarray, fwhm_pix: float) -> np.ndarray:
    """cube [n1][n2][C] -> the same shape, each channel map convolved with the
    beam by direct summation over the kernel's taps (zero outside the map)."""
    cube = np.asarray(cube, dtype=np.float64)
    n1, n2, _ = cube.shape
    k = beam_kernel(fwhm_pix)
    r = (k.shape[0] - 1) // 2
    out = np.zeros_like(cube)
    for di in range(-r, r + 1):
        for dj in range(-r, r + 1):
            w = k[di + r, dj + r]
            # out[p1, p2] += w * cube[p1 + di, p2 + dj] where both are inside the map.
            a1, b1 = max(0, -di), min(n1, n1 - di)
            a2, b2 = max(0, -dj), min(n2, n2 - dj)
            if a1 < b1 and a2 < b2:
                out[a1:b1, a2:b2] += w * cube[a1 + di:b1 + di, a2 + dj:b2 + dj]
    return out


def lv_mean(cube: np.ndarray, axis: int) -> np.ndarray:
    """cube [n1][n2][C] -> the mean over sky axis `axis` (0 or 1): [n_other][C]."""
    cube = np.asarray(cube, dtype=np.float64)
    n = cube.shape[axis]
    acc = np.zeros(cube.shape[:axis] + cube.shape[axis + 1:], dtype=np.float64)
    for i in range(n):
        acc += cube[i] if axis == 0 else cube[:, i]
    return acc / n
