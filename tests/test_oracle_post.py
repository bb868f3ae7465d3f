"""Pins of the post-transfer reference (beam convolution, l,v mean) against
properties of Gaussian convolution that its code does not contain."""

import math

import numpy as np
import pytest

from oracle import post


def test_beam_half_maximum_at_half_the_fwhm():
    # The response to one bright pixel is the beam; at an offset of FWHM/2 it is half the peak.
    for fwhm in (2.0, 4.0, 6.0):
        cube = np.zeros((41, 41, 1))
        cube[20, 20, 0] = 1.0
        out = post.beam_convolve(cube, fwhm)[:, :, 0]
        h = int(fwhm / 2)
        assert out[20 + h, 20] / out[20, 20] == pytest.approx(0.5, rel=1e-12)
        assert out[20, 20 - h] / out[20, 20] == pytest.approx(0.5, rel=1e-12)
        assert out.sum() == pytest.approx(1.0, rel=1e-13)


def test_beam_second_moments_add():
    # Convolution adds variances: a Gaussian source of width s1 comes out with
    # width sqrt(s1^2 + sigma^2) (discrete sums, far from the edges).
    n, s1, fwhm = 81, 2.5, 5.0
    i = np.arange(n) - n // 2
    src = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2 * s1 ** 2))[:, :, None]
    out = post.beam_convolve(src, fwhm)[:, :, 0]
    var = np.sum(out * i[:, None] ** 2) / out.sum()
    assert var == pytest.approx(s1 ** 2 + post.beam_sigma(fwhm) ** 2, rel=2e-3)
    assert out.sum() == pytest.approx(src.sum(), rel=1e-12)


def test_beam_keeps_a_uniform_interior_and_loses_flux_at_the_edges():
    n, fwhm = 30, 3.0
    r = post.beam_radius(fwhm)
    cube = np.full((n, n, 3), 2.0)
    out = post.beam_convolve(cube, fwhm)
    np.testing.assert_allclose(out[r:n - r, r:n - r], 2.0, rtol=1e-13)
    # A corner keeps the beam's mass inside the map: (sum over one half-axis)^2.
    s = post.beam_sigma(fwhm)
    w = np.exp(-np.arange(-r, r + 1) ** 2 / (2 * s * s))
    w /= w.sum()
    assert out[0, 0, 1] == pytest.approx(2.0 * w[r:].sum() ** 2, rel=1e-12)


def test_beam_commutes_with_transposition_and_is_linear():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((13, 17, 4))
    b = rng.standard_normal((13, 17, 4))
    fwhm = 2.5
    ca = post.beam_convolve(a, fwhm)
    np.testing.assert_allclose(post.beam_convolve(a.transpose(1, 0, 2), fwhm), ca.transpose(1, 0, 2),
                               rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(post.beam_convolve(2 * a + b, fwhm),
                               2 * ca + post.beam_convolve(b, fwhm), rtol=1e-12, atol=1e-13)


def test_lv_mean():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((9, 5, 3))
    # A map varying only along the kept axis comes back unchanged; sums are kept.
    only1 = np.broadcast_to(a[:, :1, :], a.shape)
    np.testing.assert_allclose(post.lv_mean(only1, 1), a[:, 0, :], rtol=1e-14)
    np.testing.assert_allclose(post.lv_mean(a, 0).sum(), a.sum() / 9, rtol=1e-12)
    np.testing.assert_allclose(post.lv_mean(np.full((4, 6, 2), 1.5), 0), 1.5, rtol=0)
