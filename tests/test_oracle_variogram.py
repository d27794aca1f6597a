"""Pins of the oracle's empirical semivariogram (O7) and exponential fit (O8):
brute force over explicit pairs, closed forms of linear ramps, exact recovery
of a noise-free exponential model, and recovery of a known range from a
synthetic field whose axis semivariogram is exponential by construction."""
import numpy as np
import pytest

pytestmark = []


def _grid(orc, nx, ny, dx=2.0, dy=2.0):
    return orc.Grid(0.0, 0.0, dx, dy, nx, ny)


def test_variogram_brute_force_with_holes(orc):
    rng = np.random.default_rng(3)
    nx, ny, nlags = 9, 7, 6
    z = rng.normal(0.0, 5.0, (ny, nx))
    z[rng.random((ny, nx)) < 0.2] = np.nan
    gx, gy, px, py = orc.variogram(_grid(orc, nx, ny), z, nlags)
    for k in range(1, nlags + 1):
        sx = sy = 0.0
        cx = cy = 0
        for a in range(ny):
            for b in range(nx):
                for (a2, b2, horiz) in ((a, b + k, True), (a + k, b, False)):
                    if a2 >= ny or b2 >= nx:
                        continue
                    z1, z2 = z[a, b], z[a2, b2]
                    if np.isnan(z1) or np.isnan(z2):
                        continue
                    if horiz:
                        sx += (z1 - z2) ** 2
                        cx += 1
                    else:
                        sy += (z1 - z2) ** 2
                        cy += 1
        assert px[k - 1] == cx and py[k - 1] == cy
        if cx:
            assert gx[k - 1] == pytest.approx(sx / (2 * cx), rel=1e-14)
        else:
            assert np.isnan(gx[k - 1])
        if cy:
            assert gy[k - 1] == pytest.approx(sy / (2 * cy), rel=1e-14)
        else:
            assert np.isnan(gy[k - 1])


def test_variogram_linear_ramps_closed_form(orc):
    nx, ny, nlags = 40, 30, 12
    c = 0.75
    b = np.arange(nx, dtype=np.float64)
    ramp_x = np.tile(c * b - 4000.0, (ny, 1))          # varies along x only
    gx, gy, px, py = orc.variogram(_grid(orc, nx, ny), ramp_x, nlags)
    k = np.arange(1, nlags + 1)
    assert np.array_equal(px, ny * (nx - k)) and np.array_equal(py, nx * (ny - k))
    assert np.allclose(gx, 0.5 * (c * k) ** 2, rtol=1e-12, atol=0)
    assert np.all(gy == 0.0)
    ramp_y = ramp_x.T.copy()                              # now ny x nx = 40 x 30
    gx2, gy2, _, _ = orc.variogram(_grid(orc, ny, nx), ramp_y, nlags)
    assert np.all(gx2 == 0.0)
    assert np.allclose(gy2, 0.5 * (c * k) ** 2, rtol=1e-12, atol=0)


def test_fit_recovers_noise_free_exponential(orc):
    h = np.arange(1, 41) * 2.0
    for a_true, c_true in ((13.7, 7.3), (3.0, 0.02), (150.0, 2500.0)):
        g = c_true * (1.0 - np.exp(-h / a_true))
        w = np.linspace(1.0, 3.0, h.size)
        a, c, rc = orc.fit_exponential(h, g, w)
        assert rc == 0
        assert a == pytest.approx(a_true, rel=1e-7)
        assert c == pytest.approx(c_true, rel=1e-7)


def test_fit_ignores_zero_weight_and_nan_points(orc):
    h = np.arange(1, 31) * 1.5
    g = 4.0 * (1.0 - np.exp(-h / 9.0))
    w = np.ones_like(h)
    g2, w2 = g.copy(), w.copy()
    g2[3] = np.nan
    g2[7] = 1e6
    w2[7] = 0.0
    a, c, _ = orc.fit_exponential(h, g2, w2)
    assert a == pytest.approx(9.0, rel=1e-7) and c == pytest.approx(4.0, rel=1e-7)


def test_fit_reports_no_sill_for_a_linear_variogram(orc):
    h = np.arange(1, 21) * 1.0
    _, _, rc = orc.fit_exponential(h, 0.3 * h, np.ones_like(h))
    assert rc == -2


def _separable_exponential_field(n, dx, a, sigma, seed):
    """Unit-variance AR(1) along rows, then along columns: covariance
    rho^|i| rho^|j| with rho = exp(-dx / a), so along either axis the
    semivariogram is sigma^2 (1 - exp(-h / a)) exactly (in expectation)."""
    rng = np.random.default_rng(seed)
    rho = np.exp(-dx / a)
    s = np.sqrt(1.0 - rho * rho)
    e = rng.standard_normal((n, n))
    f = np.empty_like(e)
    f[:, 0] = e[:, 0]
    for j in range(1, n):
        f[:, j] = rho * f[:, j - 1] + s * e[:, j]
    g = np.empty_like(f)
    g[0, :] = f[0, :]
    for i in range(1, n):
        g[i, :] = rho * g[i - 1, :] + s * f[i, :]
    return sigma * g - 4500.0


def test_fit_recovers_range_of_synthetic_field(orc):
    dx, a_true, sigma = 2.0, 20.0, 3.0
    z = _separable_exponential_field(768, dx, a_true, sigma, seed=17)
    a, c, rc = orc.fit_grid_range(_grid(orc, 768, 768, dx, dx), z, 40)
    assert rc == 0
    assert a == pytest.approx(a_true, rel=0.15)
    assert c == pytest.approx(sigma * sigma, rel=0.2)
