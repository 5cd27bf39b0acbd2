"""Pins of the stamp convolution and subtraction oracle (Sec. 2.2.4,
Eq. 8-10): FFT convolution for a spatially constant kernel, a delta
template giving the kernel in closed form, stamp extents and normalised
centres by hand, linearity in the coefficients, an antisymmetric basis
term on a symmetric template, and a difference that vanishes where the
model holds."""
import math

import numpy as np
import pytest

from oracle import subtract as sb


def _fft_conv(R, K):
    """Zero-padded linear convolution R (x) K by FFT (K indexed [v, u],
    centred), cut back to R's shape."""
    h, w = R.shape
    kh = K.shape[0]
    hw = kh // 2
    H, W = h + kh, w + kh
    F = np.fft.rfft2(R.astype(np.float64), s=(H, W)) * \
        np.fft.rfft2(K, s=(H, W))
    full = np.fft.irfft2(F, s=(H, W))
    return full[hw:hw + h, hw:hw + w]


def test_constant_kernel_equals_fft_convolution():
    rng = np.random.default_rng(1)
    I = rng.normal(100, 10, (50, 47)).astype(np.float32)
    R = rng.normal(80, 10, (50, 47)).astype(np.float32)
    sig, ords, hw = [1.0, 2.5], [2, 1], 5
    nb = len(sb.basis_terms(sig, ords))
    a = [[c] + [0.0] * (sb.n_poly(1) - 1) for c in rng.normal(0, 1, nb)]
    D = sb.subtract(I, R, sig, ords, hw, a, 1, [3.0], 0, stamp=21)
    K = np.tensordot(np.array([c[0] for c in a]), sb.basis(sig, ords, hw),
                     axes=1)
    want = (I.astype(np.float64) + 3.0) - _fft_conv(R, K)
    np.testing.assert_allclose(D, want, rtol=0, atol=1e-9 * np.abs(R).max()
                               * np.abs(K).sum())


def test_delta_template_gives_the_kernel():
    R = np.zeros((40, 40), dtype=np.float32)
    R[17, 22] = 1.0
    I = np.zeros_like(R)
    D = sb.subtract(I, R, [2.0], [0], 6, [[3.0]], 0, [0.0], 0)
    y, x = np.mgrid[0:40, 0:40]
    r2 = (x - 22.0) ** 2 + (y - 17.0) ** 2
    want = np.where((np.abs(x - 22) <= 6) & (np.abs(y - 17) <= 6),
                    -3.0 * np.exp(-r2 / 8.0), 0.0)
    np.testing.assert_allclose(D, want, rtol=1e-14, atol=1e-300)


def test_stamps_and_normalised_centres():
    assert sb.stamps(43, 21) == [(0, 21, 10.0), (21, 42, 31.0),
                                 (42, 43, 42.0)]
    assert sb.norm_coord(10.0, 43) == (20.0 - 42.0) / 42.0
    assert sb.norm_coord(42.0, 43) == 1.0 and sb.norm_coord(0.0, 1) == 0.0
    # c00 + c01 y + c10 x for degree 1, in the order p, then q
    assert sb.poly([1.0, 2.0, 3.0], 1, 0.5, -0.25) == 1.0 - 0.5 + 1.5


def test_linear_in_the_coefficients():
    rng = np.random.default_rng(2)
    I = np.zeros((44, 30), dtype=np.float32)
    R = rng.normal(10, 3, (44, 30)).astype(np.float32)
    sig, ords, hw = [1.5], [1], 4
    nb = len(sb.basis_terms(sig, ords))
    a1 = rng.normal(0, 1, (nb, sb.n_poly(2))).tolist()
    a2 = rng.normal(0, 1, (nb, sb.n_poly(2))).tolist()
    a12 = (np.array(a1) + np.array(a2)).tolist()
    d1 = sb.subtract(I, R, sig, ords, hw, a1, 2, [0.0], 0, stamp=13)
    d2 = sb.subtract(I, R, sig, ords, hw, a2, 2, [0.0], 0, stamp=13)
    d12 = sb.subtract(I, R, sig, ords, hw, a12, 2, [0.0], 0, stamp=13)
    np.testing.assert_allclose(d1 + d2, d12, rtol=0, atol=1e-9)
    # the kernel varies over the frame: stamps differ
    assert not np.allclose(d1[:13, :13] - d1[:13, :13].mean(), 0)


def test_antisymmetric_term_on_a_symmetric_template():
    y, x = np.mgrid[0:31, 0:31]
    R = np.exp(-((x - 15.0) ** 2 + (y - 15.0) ** 2) / 20.0).astype(
        np.float32)
    I = np.zeros_like(R)
    # basis of one Gaussian of order 1: (i, j) = (0,0), (0,1), (1,0); only
    # the u^1 term (index 2) is used
    D = sb.subtract(I, R, [2.0], [1], 5, [[0.0], [0.0], [1.0]], 0, [0.0], 0,
                    stamp=31)
    assert abs(D[15, 15]) <= 1e-15
    # odd in x about the centre column
    np.testing.assert_allclose(D[:, 15 - 4], -D[:, 15 + 4], atol=1e-14)


def test_difference_vanishes_where_the_model_holds():
    rng = np.random.default_rng(4)
    R = rng.normal(500, 30, (36, 36)).astype(np.float64)
    sig, ords, hw = [1.2, 3.0], [0, 2], 6
    nb = len(sb.basis_terms(sig, ords))
    c = rng.normal(0, 0.3, nb)
    K = np.tensordot(c, sb.basis(sig, ords, hw), axes=1)
    B = -12.5
    I = (_fft_conv(R, K) - B)
    D = sb.subtract(I.astype(np.float32), R.astype(np.float32), sig, ords,
                    hw, [[v] for v in c], 0, [B], 0)
    # I was rounded to binary32: the difference is that rounding
    assert np.max(np.abs(D)) <= 4 * np.finfo(np.float32).eps * np.abs(I).max()
