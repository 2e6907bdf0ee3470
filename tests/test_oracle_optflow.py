"""Pins of the oracle's optical-flow pieces.

App. C derivatives: exact on space-time ramps away from borders; constants give 0;
the mirrored border of a ramp gives half the slope (closed form of the half-sample
symmetric extension).
Horn-Schunck sweeps: their fixed point solves the normal equations of the p = q = 2
flow energy (eq. of_reg), checked against a sparse direct solve; a flat image (no
gradient) reduces the sweep to neighbour averaging.
Reverse flow: a uniform integer translation reverses exactly where pixels land.
"""
import numpy as np
import pytest

from oracle import optflow


@pytest.mark.parametrize("dr", [1, 2])
def test_derivs_exact_on_ramps(dr):
    n_t, ny, nx = 3, 11, 13
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    a, b, c = 0.6, -0.25, 1.5
    u = np.stack([a * x + b * y + c * t for t in range(n_t)])
    I = optflow.of_derivs(u, dr)
    inner = (slice(None), slice(dr, -dr), slice(dr, -dr))
    np.testing.assert_allclose(I[:, 0][inner], a, atol=1e-13)
    np.testing.assert_allclose(I[:, 1][inner], b, atol=1e-13)
    np.testing.assert_allclose(I[:, 2], c, atol=1e-13)        # time difference is exact everywhere
    assert np.abs(optflow.of_derivs(np.full((2, 5, 6), 3.0), dr)).max() == 0


def test_derivs_mirrored_border():
    ny, nx = 6, 7
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    u = np.stack([0.8 * x, 0.8 * x])
    I = optflow.of_derivs(u, 1)
    # at x = 0 the neighbour x-1 mirrors to x = 0: (u(1) - u(0))/2 = slope/2
    np.testing.assert_allclose(I[0, 0][:, 0], 0.4, atol=1e-14)
    np.testing.assert_allclose(I[0, 0][:, -1], 0.4, atol=1e-14)
    np.testing.assert_allclose(I[0, 0][:, 1:-1], 0.8, atol=1e-14)


def test_hs_fixed_point_is_direct_solution():
    r = np.random.default_rng(1)
    ny, nx = 7, 8
    I = r.standard_normal((3, ny, nx))
    gamma = 0.5
    s = np.zeros((2, ny, nx))
    for _ in range(4000):
        s = optflow.hs_sweep(I, s, gamma)
    direct = optflow.hs_direct(I, gamma)
    np.testing.assert_allclose(s, direct, atol=1e-10)
    # the energy at the fixed point is not above that at nearby perturbations
    e0 = optflow.hs_energy(I, direct, gamma)
    for _ in range(5):
        assert optflow.hs_energy(I, direct + 1e-3 * r.standard_normal(direct.shape), gamma) >= e0


def test_hs_flat_image_is_averaging():
    ny, nx = 5, 6
    I = np.zeros((3, ny, nx))
    s = np.random.default_rng(2).standard_normal((2, ny, nx))
    out = optflow.hs_sweep(I, s, 0.01)
    np.testing.assert_allclose(out[0], optflow.neighbour_mean(s[0]))
    # corner has 2 neighbours, edge 3, interior 4
    assert optflow.neighbour_count(ny, nx)[0, 0] == 2 and optflow.neighbour_count(ny, nx)[0, 2] == 3


def test_reverse_flow_uniform_integer_translation():
    n = 10
    v = np.zeros((2, 2, n, n))
    v[:, 0], v[:, 1] = 2.0, -1.0
    vr = optflow.reverse_flow(v)
    # pixels (x, y) with x >= 2 and y <= n-2 are hit exactly once
    hit = np.zeros((n, n), bool)
    hit[: n - 1, 2:] = True
    np.testing.assert_array_equal(vr[:, 0][:, hit], -2.0)
    np.testing.assert_array_equal(vr[:, 1][:, hit], 1.0)
    np.testing.assert_array_equal(vr[:, :, ~hit], 0.0)


def test_reverse_flow_collisions_are_averaged():
    v = np.zeros((1, 2, 1, 4))
    v[0, 0, 0] = [1.0, 0.0, 0.4, -2.0]   # pixels 0 and 1 both land on x = 1; 2 -> 2; 3 -> 1
    vr = optflow.reverse_flow(v)
    np.testing.assert_allclose(vr[0, 0, 0], [0.0, -(1.0 + 0.0 - 2.0) / 3.0, -0.4, 0.0])
