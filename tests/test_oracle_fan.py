"""Pins of the oracle's fan-beam projector (flat detector, Joseph's ray-driven method).

* Linear images: Joseph's row sampling is exact for a linear function, so a ray that
  crosses every row inside the frame sums to the line integral of the function between the
  first and last row edges, ny |d| / |d_y| (a X(0) + c) for u = a X + b Y + c (closed form).
* Chord lengths: the projection of a disk (pixels weighted by their covered area) matches
  the analytic line integrals 2 sqrt(R^2 - p^2), p the ray's distance from the centre.
* Similar triangles: at theta = 0 a single pixel at (X, Y) feeds the two bins around
  u = X dsd / (dso + Y) and no other.
* Rotating a square frame by 90 degrees (numpy's rot90) and the angles by -90 degrees leaves
  the sinogram unchanged; the transpose passes the adjoint identity.
"""
import math

import numpy as np
import pytest

from oracle import forward

GEO = dict(dso=60.0, dsd=120.0, du=1.7)


@pytest.mark.parametrize("theta", [0.0, 0.35, -0.2])
def test_linear_image_line_integrals(theta):
    ny, nx, nb = 21, 40, 9
    dso, dsd, du = 200.0, 300.0, 1.0
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    X, Y = x - (nx - 1) / 2.0, y - (ny - 1) / 2.0
    a, c = 0.3, 1.5
    img = (a * X - 0.7 * Y + c)[None]
    got = forward.fan_fwd(img, np.array([[theta]]), nb, dso, dsd, du)[0, 0]
    S = (dso * math.sin(theta), -dso * math.cos(theta))
    for j in range(nb):
        uj = (j - (nb - 1) / 2.0) * du
        dx = -dsd * math.sin(theta) + uj * math.cos(theta)
        dy = dsd * math.cos(theta) + uj * math.sin(theta)
        X0 = S[0] - S[1] * dx / dy              # the ray's X on the middle row (Y = 0)
        xs = S[0] + (np.array([-(ny - 1) / 2.0, (ny - 1) / 2.0]) - S[1]) * dx / dy + (nx - 1) / 2.0
        assert xs.min() > 1 and xs.max() < nx - 2  # the ray stays inside the frame
        exp = ny * math.hypot(dx, dy) / abs(dy) * (a * X0 + c)
        assert abs(got[j] - exp) <= 1e-11 * abs(exp), j


def _disk_area(n, R, sub=16):
    """Fraction of every pixel inside the centred disk of radius R (sub x sub samples)."""
    c = (n - 1) / 2.0
    off = (np.arange(sub) + 0.5) / sub - 0.5
    y, x = np.mgrid[0:n, 0:n].astype(float)
    acc = np.zeros((n, n))
    for dy in off:
        for dx in off:
            acc += ((x + dx - c) ** 2 + (y + dy - c) ** 2) <= R * R
    return acc / (sub * sub)


@pytest.mark.parametrize("theta,du", [(0.0, 1.5), (0.7, 1.5), (0.7, 3.0), (2.0, 0.8)])
def test_disk_chords(theta, du):
    n, R = 64, 20.0
    dso, dsd = 90.0, 180.0
    nb = int(2 * 30 * dsd / dso / du) + 1
    img = _disk_area(n, R)[None]
    got = forward.fan_fwd(img, np.array([[theta]]), nb, dso, dsd, du)[0, 0]
    u = (np.arange(nb) - (nb - 1) / 2.0) * du
    p = dso * np.abs(u) / np.sqrt(dsd * dsd + u * u)
    exact = 2.0 * np.sqrt(np.maximum(R * R - p * p, 0.0))
    inner = p < 0.9 * R
    assert np.max(np.abs(got[inner] - exact[inner]) / exact[inner]) < 0.03   # pixelised disk


def test_single_pixel_similar_triangles():
    ny, nx, nb = 9, 11, 41
    y, x = 2, 8
    img = np.zeros((1, ny, nx))
    img[0, y, x] = 1.0
    got = forward.fan_fwd(img, np.array([[0.0]]), nb, **GEO)[0, 0]
    X, Y = x - (nx - 1) / 2.0, y - (ny - 1) / 2.0
    uu = X * GEO["dsd"] / (GEO["dso"] + Y)
    pos = uu / GEO["du"] + (nb - 1) / 2.0
    hit = np.nonzero(got)[0]
    assert set(hit) <= {math.floor(pos) - 1, math.floor(pos), math.floor(pos) + 1, math.floor(pos) + 2}
    assert got[math.floor(pos)] > 0 or got[math.floor(pos) + 1] > 0


def test_rot90_and_adjoint():
    r = np.random.default_rng(2)
    n, nb = 13, 31
    u = r.standard_normal((1, n, n))
    ang = np.array([[0.3, 1.1, 2.5]])
    b = forward.fan_fwd(u, ang, nb, **GEO)
    b_rot = forward.fan_fwd(np.rot90(u, axes=(1, 2)), ang - np.pi / 2, nb, **GEO)
    assert np.allclose(b, b_rot, atol=1e-12 * np.abs(b).max())
    w = r.standard_normal(b.shape)
    lhs = float((b * w).sum())
    rhs = float((u * forward.fan_adj(w, ang, n, n, **GEO)).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_angle_schedules_match_the_printed_examples():
    """The three schedules of Sec. 5 reproduce the interval starts printed there; every
    frame's n_views angles are evenly spaced over its half-open interval."""
    import json
    import os
    from synth import angle_schedule
    with open(os.path.join(os.path.dirname(__file__), "golden", "angle_schedules.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        ang = np.degrees(angle_schedule(c["kind"], c["n_t"], c["n_views"]))
        np.testing.assert_allclose(ang[:, 0], c["starts"], atol=1e-12)
        step = c["width"] / c["n_views"]
        np.testing.assert_allclose(np.diff(ang, axis=1), step, atol=1e-12)
        assert np.all(ang[:, -1] < np.array(c["starts"]) + c["width"])
    fixed = np.degrees(angle_schedule("fixed", 5, 6))
    np.testing.assert_allclose(fixed, np.tile(np.arange(6) * 30.0, (5, 1)), atol=1e-12)
