"""Pins of the oracle's forward operators against closed forms and symmetries.

Radon (hat model, unit bins):
  * partition of unity: every pixel's weights sum to 1 at every angle when no bin is
    truncated, so each projection conserves mass;
  * theta = 0 / pi/2 projections of an even-sized image are column / row sums split
    0.5/0.5 between the two neighbouring bins;
  * rotating the image by 90 degrees shifts the angle by pi/2; theta + pi reverses bins;
  * adjoint identity <Hu, b> = <u, H^T b>.
Blur: agrees with scipy.ndimage.correlate (zero boundary) on the 2-D kernel and with
two 1-D passes of the separable factor; delta response; adjoint identity.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import forward
from synth import bins_for


def _rng(s=0):
    return np.random.default_rng(s)


@pytest.mark.parametrize("n", [8, 9, 32])
def test_radon_mass_conservation(n):
    nb = bins_for(n)
    u = _rng(n).random((1, n, n))
    ang = _rng(1).uniform(0, math.pi, size=(1, 7))
    b = forward.radon_fwd(u, ang, nb)
    np.testing.assert_allclose(b.sum(axis=2), np.full((1, 7), u.sum()), rtol=1e-13)


def test_radon_axis_angles_closed_form():
    n = 8
    nb = bins_for(n)            # 11 bins, centres d_j = j - 5
    u = _rng(2).random((1, n, n))
    ang = np.array([[0.0, math.pi / 2]])
    b = forward.radon_fwd(u, ang, nb)
    col = u[0].sum(axis=0)      # sums over y for each x;  X = x - 3.5
    row = u[0].sum(axis=1)      # sums over x for each y;  Y = y - 3.5
    exp0 = np.zeros(nb)
    exp1 = np.zeros(nb)
    for x in range(n):
        X = x - 3.5
        for d in (X - 0.5, X + 0.5):           # the two integer bin centres around X
            exp0[int(d) + 5] += 0.5 * col[x]
            exp1[int(d) + 5] += 0.5 * row[x]
    np.testing.assert_allclose(b[0, 0], exp0, atol=1e-14)
    np.testing.assert_allclose(b[0, 1], exp1, atol=1e-13)


def test_radon_rotation_and_reversal():
    n = 10
    nb = bins_for(n)
    u = _rng(3).random((n, n))
    # u'[y', x'] = u[n-1-x', y'] is u rotated by +90 degrees about the centre.
    up = np.empty_like(u)
    for yp in range(n):
        for xp in range(n):
            up[yp, xp] = u[n - 1 - xp, yp]
    th = 0.37
    a = forward.radon_fwd(up[None], np.array([[th]]), nb)[0, 0]
    b = forward.radon_fwd(u[None], np.array([[th - math.pi / 2]]), nb)[0, 0]
    np.testing.assert_allclose(a, b, atol=1e-12)
    c = forward.radon_fwd(u[None], np.array([[th + math.pi]]), nb)[0, 0]
    d = forward.radon_fwd(u[None], np.array([[th]]), nb)[0, 0]
    np.testing.assert_allclose(c, d[::-1], atol=1e-12)


@pytest.mark.parametrize("shape,nth,nb", [((2, 8, 8), 5, 11), ((3, 6, 9), 4, 9), ((1, 7, 5), 3, 5)])
def test_radon_adjoint(shape, nth, nb):
    r = _rng(4)
    u = r.standard_normal(shape)
    ang = r.uniform(0, math.pi, size=(shape[0], nth))
    b = r.standard_normal((shape[0], nth, nb))
    lhs = (forward.radon_fwd(u, ang, nb) * b).sum()
    rhs = (u * forward.radon_adj(b, ang, shape[1], shape[2])).sum()
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)


def test_radon_disk_near_isotropic():
    n = 64
    nb = bins_for(n)
    y, x = np.mgrid[0:n, 0:n]
    r = 20.0
    u = (((x - 31.5) ** 2 + (y - 31.5) ** 2) <= r * r).astype(float)[None]
    ang = np.linspace(0, math.pi, 12, endpoint=False)[None]
    b = forward.radon_fwd(u, ang, nb)[0]
    d = np.arange(nb) - (nb - 1) / 2.0
    chord = 2 * np.sqrt(np.maximum(r * r - d * d, 0.0))
    # every angle approximates the chord-length profile of the disk
    for k in range(12):
        assert np.linalg.norm(b[k] - chord) < 0.1 * np.linalg.norm(chord)
        assert abs(b[k].sum() - u.sum()) < 1e-9


def test_blur_matches_library_correlate_and_separable():
    r = _rng(5)
    u = r.random((2, 23, 17))
    out = forward.blur(u, 9, 2.0)
    K = forward.gaussian_kernel(9, 2.0)
    i = np.arange(-4, 5)
    k1 = np.exp(-i * i / 8.0)
    k1 /= k1.sum()
    np.testing.assert_allclose(K, np.outer(k1, k1), rtol=1e-14)
    for t in range(2):
        lib = ndimage.convolve(u[t], K, mode="constant", cval=0.0)
        np.testing.assert_allclose(out[t], lib, atol=1e-14)
        sep = ndimage.convolve1d(ndimage.convolve1d(u[t], k1, axis=0, mode="constant"), k1, axis=1, mode="constant")
        np.testing.assert_allclose(out[t], sep, atol=1e-14)


def test_blur_delta_and_adjoint():
    u = np.zeros((1, 15, 15))
    u[0, 7, 6] = 1.0
    out = forward.blur(u)[0]
    K = forward.gaussian_kernel()
    np.testing.assert_allclose(out[3:12, 2:11], K, atol=1e-16)
    assert abs(out.sum() - 1.0) < 1e-14
    r = _rng(6)
    a = r.standard_normal((2, 12, 19))
    b = r.standard_normal((2, 12, 19))
    lhs = (forward.blur(a) * b).sum()
    rhs = (a * forward.blur_adj(b)).sum()
    assert abs(lhs - rhs) < 1e-12
    np.testing.assert_allclose(forward.blur(a), forward.blur_adj(a), atol=1e-14)
