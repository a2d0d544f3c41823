"""Pins of the oracle transport operators and implicit diffusion solves."""
import numpy as np
import pytest

import synth
from oracle import transport as tr


def test_advection_fourth_order_on_smooth_periodic_field():
    errs = []
    for n in (16, 32, 64):
        dx = 1.0 / n
        x = (np.arange(n) + 0.5) * dx
        # cell averages of sin(2 pi x) and the exact average of -u d/dx
        avg = (np.cos(2 * np.pi * (x - dx / 2)) - np.cos(2 * np.pi * (x + dx / 2))) / (2 * np.pi * dx)
        exact = -3.0 * (np.sin(2 * np.pi * (x + dx / 2)) - np.sin(2 * np.pi * (x - dx / 2))) / dx
        FA = tr.advection(avg[None], (3.0,), (dx,))[0]
        errs.append(np.abs(FA - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.8)


def test_advection_2d_uses_both_directions_and_conserves():
    rng = np.random.default_rng(0)
    phi = rng.standard_normal((3, 12, 10))
    out = tr.advection(phi, (2.0, -1.5), (0.1, 0.2))
    np.testing.assert_allclose(out.sum(axis=(1, 2)), 0.0, atol=1e-12)
    # a field constant in x is moved only by the y velocity
    col = np.repeat(rng.standard_normal((1, 12, 1)), 10, axis=2)
    ox = tr.advection(col, (2.0, 0.0), (0.1, 0.2))
    assert np.abs(ox).max() < 1e-12


def test_diffusion_second_order_and_closure():
    m = synth.make_mechanism(9, 21, 0)
    errs = []
    for n in (32, 64, 128):
        dx = 1.0 / n
        x = (np.arange(n) + 0.5) * dx
        T = 900.0 + 300.0 * np.sin(2 * np.pi * x)
        th = tr.theta(T)
        phi = np.cos(2 * np.pi * x)
        # exact d/dx (theta dphi/dx) at cell centres
        dth = 1.7 * (T / 300.0) ** 0.7 / 300.0 * 300.0 * 2 * np.pi * np.cos(2 * np.pi * x)
        exact = dth * (-2 * np.pi * np.sin(2 * np.pi * x)) + th * (-(2 * np.pi) ** 2 * np.cos(2 * np.pi * x))
        L = tr.laplacian_theta(phi[None], th, (dx,))[0]
        errs.append(np.abs(L - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.9)
    rng = np.random.default_rng(1)
    Y = rng.uniform(0.01, 0.2, (9, 16))
    phi = np.concatenate([Y, rng.uniform(-1e9, 1e9, (1, 16))])
    T = rng.uniform(400, 1900, 16)
    FD = tr.diffusion(m, phi, T, (0.01,))
    np.testing.assert_allclose(FD[:9].sum(axis=0), 0.0, atol=1e-9 * np.abs(FD[:9]).max())
    np.testing.assert_allclose(FD.sum(axis=1), 0.0, atol=1e-9 * np.abs(FD).max())


@pytest.mark.parametrize("shape", [(40,), (12, 18)])
def test_helmholtz_constant_coefficient_matches_fft(shape):
    rng = np.random.default_rng(2)
    dx = tuple([0.01] * len(shape))
    rhs = rng.standard_normal(shape)
    th = np.ones(shape)
    c, k0 = 3e-5, 0.3
    y = tr.helmholtz_solve(th, k0, c, rhs, dx)
    # eigenvalues of the periodic 2nd-order Laplacian: -4 sin^2(pi k / n) / dx^2
    lam = 0.0
    for d, n in enumerate(shape):
        k = np.fft.fftfreq(n) * n
        sh = [1] * len(shape)
        sh[d] = n
        lam = lam + (-4.0 * np.sin(np.pi * k / n) ** 2 / dx[len(shape) - 1 - d] ** 2).reshape(sh)
    yf = np.real(np.fft.ifftn(np.fft.fftn(rhs) / (1.0 - c * k0 * lam)))
    np.testing.assert_allclose(y, yf, rtol=0, atol=1e-13 * np.abs(yf).max())


def test_diffusion_solve_closure_and_residual():
    m = synth.make_mechanism(9, 21, 0)
    T, rhs = synth.random_helmholtz_problem((10, 14), 10, seed=3)
    rhs[:9] = np.abs(rhs[:9]) * 0.05
    c = 1e-5
    y = tr.diffusion_solve(m, c, rhs, T, (0.01, 0.01))
    # every diffused field satisfies its system; the closure keeps sum(Y)
    k0 = tr.diffusion_coefficients(m)
    th = tr.theta(T)
    for f in list(range(8)) + [9]:
        res = y[f] - c * k0[f] * tr.laplacian_theta(y[f][None], th, (0.01, 0.01))[0] - rhs[f]
        assert np.abs(res).max() < 1e-12 * max(1.0, np.abs(rhs[f]).max())
    np.testing.assert_allclose(y[:9].sum(axis=0), rhs[:9].sum(axis=0), atol=1e-14)
    # conservative: domain totals unchanged by the solve
    np.testing.assert_allclose(y.sum(axis=(1, 2)), rhs.sum(axis=(1, 2)), rtol=1e-12, atol=1e-12)
