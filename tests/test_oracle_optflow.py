"""Pins of the oracle's optical-flow pieces.

App. C derivatives: exact on space-time ramps away from borders; constants give 0;
the mirrored border of a ramp gives half the slope (closed form of the half-sample
symmetric extension); an impulse gives the closed-form averaging windows of every
derivative (inside and on the mirrored border).
Horn-Schunck sweeps: their fixed point solves the normal equations of the p = q = 2
flow energy (eq. of_reg), checked against a sparse direct solve; a flat image (no
gradient) reduces the sweep to neighbour averaging.
Reverse flow: a uniform integer translation reverses exactly where pixels land.
Rescaled flow: block means exact (edge blocks over in-frame pixels), bilinear upscaling
reproduces constant and linear fields times f, f = 1 is the plain update, and a pattern
translating by 2 px/frame gets a flow of about 2 px through frames reduced by 2.
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


@pytest.mark.parametrize("dr", [1, 2])
def test_derivs_impulse_closed_form(dr):
    """App. C box averaging pinned by an impulse: frame 0 holds a unit impulse at (y0, x0)
    well inside, frame 1 is zero.  The x-derivative is a column difference of half-width dr
    averaged over 2dr+1 rows, so it is +1/((2dr+1) 2dr) on column x0-dr and -1/((2dr+1) 2dr)
    on column x0+dr over rows y0-dr..y0+dr, zero elsewhere (I_y likewise with rows and columns
    exchanged), and the time difference averaged over the (2dr+1)^2 box is -1/(2dr+1)^2 on
    the box around the impulse.  A wrong averaging window, a missing box mean on I_t or a
    wrong half-width changes one of these entries."""
    ny, nx, y0, x0 = 13, 15, 6, 7
    u = np.zeros((2, ny, nx))
    u[0, y0, x0] = 1.0
    I = optflow.of_derivs(u, dr)[0]
    box = 2 * dr + 1
    c = 1.0 / (box * 2 * dr)
    ex = np.zeros((ny, nx))
    ey = np.zeros((ny, nx))
    et = np.zeros((ny, nx))
    rows = slice(y0 - dr, y0 + dr + 1)
    cols = slice(x0 - dr, x0 + dr + 1)
    ex[rows, x0 - dr] = c
    ex[rows, x0 + dr] = -c
    ey[y0 - dr, cols] = c
    ey[y0 + dr, cols] = -c
    et[rows, cols] = -1.0 / box ** 2
    np.testing.assert_allclose(I[0], ex, atol=1e-15)
    np.testing.assert_allclose(I[1], ey, atol=1e-15)
    np.testing.assert_allclose(I[2], et, atol=1e-15)


def test_derivs_impulse_on_the_border_is_mirrored():
    """The half-sample-symmetric mirror (index -1 reads index 0): an impulse in column 0 is
    also seen by the x-difference of column 0 through its mirrored left neighbour, so both
    columns 0 and 1 carry -1/6 (dr = 1) on the rows around the impulse, and the box mean of
    the time difference counts the impulse twice at column 0 (2 of the 9 box samples of a
    pixel in column 0 read it, one through the mirror) and once at column 1."""
    ny, nx, y0 = 9, 8, 4
    u = np.zeros((2, ny, nx))
    u[0, y0, 0] = 1.0
    I = optflow.of_derivs(u, 1)[0]
    ex = np.zeros((ny, nx))
    ex[y0 - 1:y0 + 2, 0] = -1.0 / 6.0
    ex[y0 - 1:y0 + 2, 1] = -1.0 / 6.0
    np.testing.assert_allclose(I[0], ex, atol=1e-15)
    et = np.zeros((ny, nx))
    et[y0 - 1:y0 + 2, 0] = -2.0 / 9.0
    et[y0 - 1:y0 + 2, 1] = -1.0 / 9.0
    np.testing.assert_allclose(I[2], et, atol=1e-15)


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


# --------------------------------------------------------------------------- rescaled flow


def test_box_down_block_means_and_edges():
    """Exact block means, and edge blocks over their in-frame pixels only (5 -> 3 at f = 2)."""
    u = np.arange(25, dtype=float).reshape(5, 5)
    d = optflow.box_down(u, 2)
    assert d.shape == (3, 3)
    assert d[0, 0] == (0 + 1 + 5 + 6) / 4
    assert d[0, 2] == (4 + 9) / 2            # right edge: one column
    assert d[2, 0] == (20 + 21) / 2          # bottom edge: one row
    assert d[2, 2] == 24.0                   # corner: one pixel
    # a linear ramp reduces to its values at the block centres when f divides the size
    y, x = np.mgrid[0:8, 0:12]
    ramp = 0.5 * x - 0.25 * y + 3.0
    yc, xc = np.mgrid[0:2, 0:3]
    np.testing.assert_allclose(optflow.box_down(ramp, 4), 0.5 * (4 * xc + 1.5) - 0.25 * (4 * yc + 1.5) + 3.0,
                               rtol=0, atol=1e-13)


def test_flow_up_constant_and_linear():
    """Upscaling multiplies by f; bilinear sampling reproduces a field linear in the reduced
    coordinates away from the clamped border."""
    f, nys, nxs = 4, 5, 6
    c = np.full((2, nys, nxs), 0.75)
    np.testing.assert_allclose(optflow.flow_up(c, f, nys * f, nxs * f), 3.0, rtol=0, atol=1e-14)
    Y, X = np.mgrid[0:nys, 0:nxs]
    lin = np.stack([0.3 * X - 0.1 * Y, 0.05 * X + 0.2 * Y])
    up = optflow.flow_up(lin, f, nys * f, nxs * f)
    y, x = np.mgrid[0:nys * f, 0:nxs * f]
    Xs, Ys = (x + 0.5) / f - 0.5, (y + 0.5) / f - 0.5
    inside = (Xs >= 0) & (Xs <= nxs - 1) & (Ys >= 0) & (Ys <= nys - 1)
    exp = f * np.stack([0.3 * Xs - 0.1 * Ys, 0.05 * Xs + 0.2 * Ys])
    assert inside.sum() > 0.6 * inside.size
    np.testing.assert_allclose(up[:, inside], exp[:, inside], rtol=0, atol=1e-13)


def test_flow_update_scaled_reduces_to_plain_and_tracks_translation():
    r = np.random.default_rng(3)
    u = np.cumsum(np.cumsum(r.standard_normal((3, 24, 24)), axis=1), axis=2) * 0.05
    v = r.uniform(-0.3, 0.3, size=(2, 2, 24, 24))
    np.testing.assert_array_equal(optflow.flow_update_scaled(u, v, 0.2, 7, 1, 1), optflow.flow_update(u, v, 0.2, 7, 1))
    # a smooth pattern translating by 2 px/frame: on frames reduced by 2 the flow is about
    # 1 px, and the upscaled flow about 2 px in the interior
    yy, xx = np.mgrid[0:32, 0:32]
    frames = np.stack([np.sin(0.25 * (xx - 2 * t)) + np.cos(0.2 * yy) for t in range(3)])
    out = optflow.flow_update_scaled(frames, np.zeros((2, 2, 32, 32)), 0.05, 400, 1, 2)
    # (u_{t+1}(x + 2) = u_t(x): the flow is +2 px in x and 0 in y)
    assert abs(np.median(out[:, 0, 8:24, 8:24]) - 2.0) < 0.3
    assert abs(np.median(out[:, 1, 8:24, 8:24])) < 0.3
