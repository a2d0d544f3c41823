"""Pins of the oracle chemistry: thermodynamics, rates, Jacobian and the
backward-Euler reaction solve (step S5)."""
import numpy as np
import pytest

import synth
from oracle import chemistry as ch


@pytest.fixture(scope="module")
def mech9():
    return synth.make_mechanism(9, 21, 0)


def _tiny_mech(react, prod, W, hf, s0, cp, A, beta=0.0, Ea=0.0, rho0=1e-3):
    """Hand-built mechanism dict in the generator's format."""
    N = len(W)
    R = len(react)
    r = -np.ones((R, 2), dtype=np.int32)
    p = -np.ones((R, 2), dtype=np.int32)
    for j in range(R):
        r[j, :len(react[j])] = react[j]
        p[j, :len(prod[j])] = prod[j]
    return dict(N=N, R=R, bath=N - 1, W=np.array(W, float), react=r, prod=p,
                A=np.full(R, A, float), beta=np.full(R, beta, float), Ea=np.full(R, Ea, float),
                cp=np.array(cp, float), hf=np.array(hf, float), s0=np.array(s0, float),
                D0=np.full(N, 0.2), alpha0=0.2, rho0=rho0, p_atm=synth.P_ATM,
                R_u=synth.R_U, R_c=synth.R_CAL)


def test_temperature_inverts_enthalpy(mech9):
    Yb, Tb, c, Yg = synth.random_cell_batch(mech9, 500, seed=1)
    h = ch.enthalpy(mech9, Yb, Tb)
    np.testing.assert_allclose(ch.temperature(mech9, Yb, h), Tb, rtol=1e-13)


def test_mechanism_is_element_and_mass_balanced(mech9):
    nu_f, nu_r = ch._stoich(mech9)
    nu = nu_r - nu_f
    assert np.all(mech9["comp"] @ nu == 0)
    np.testing.assert_allclose(mech9["W"] @ nu, 0.0, atol=1e-12)


def test_analytic_jacobian_matches_complex_step(mech9):
    Yb, Tb, c, Yg = synth.random_cell_batch(mech9, 64, seed=2)
    dY, dT = ch.reaction_source_jacobian(mech9, Yb, Tb)
    h = 1e-40
    N = mech9["N"]
    for l in range(N):
        Yc = Yb.astype(np.complex128)
        Yc[l] += 1j * h
        col = ch.reaction_source(mech9, Yc, Tb.astype(np.complex128)).imag / h
        np.testing.assert_allclose(dY[:, l, :], col, rtol=1e-11,
                                   atol=1e-11 * np.abs(col).max())
    colT = ch.reaction_source(mech9, Yb.astype(np.complex128), Tb + 1j * h).imag / h
    np.testing.assert_allclose(dT, colT, rtol=1e-11, atol=1e-11 * np.abs(colT).max())


def test_be_jacobian_matches_complex_step_of_residual(mech9):
    Yb, Tb, c, Yg = synth.random_cell_batch(mech9, 16, seed=4)
    hh = ch.enthalpy(mech9, Yb, Tb)
    T = Tb * 1.01
    J = ch.be_jacobian(mech9, c, Yg, T)
    h = 1e-40
    N = mech9["N"]
    for l in range(N + 1):
        Yc = Yg.astype(np.complex128)
        Tc = T.astype(np.complex128)
        if l < N:
            Yc[l] += 1j * h
        else:
            Tc = Tc + 1j * h
        col = ch.be_residual(mech9, c, Yb, hh, Yc, Tc).imag / h     # (N+1, n)
        np.testing.assert_allclose(J[:, :, l], col.T, rtol=1e-10,
                                   atol=1e-10 * np.abs(col).max())


def test_thermoneutral_isomerisation_equilibrium():
    # A <=> B with equal W, hf and cp: T is constant and the equilibrium ratio
    # is Kc = exp((s_B - s_A) / R_u) (no mole change).
    s0 = [50.0 * 4.184e7, 53.0 * 4.184e7, 45.0 * 4.184e7]
    m = _tiny_mech([(0,)], [(1,)], W=[30.0, 30.0, 28.0], hf=[1e11, 1e11, 0.0], s0=s0,
                   cp=[5 * synth.R_U] * 3, A=1e6)
    Kc = np.exp((s0[1] - s0[0]) / synth.R_U)
    Y = np.array([[0.2], [0.1], [0.7]])
    T = np.array([1200.0])
    h = ch.enthalpy(m, Y, T)
    Yn, Tn, it = ch.reaction_solve(m, np.array([1e9]), Y, h, Y)
    assert it[0] > 0
    np.testing.assert_allclose(Yn[1, 0] / Yn[0, 0], Kc, rtol=1e-12)
    np.testing.assert_allclose(Tn, T, rtol=1e-13)


def test_linear_be_step_closed_form():
    # A <=> B, equal W, thermoneutral: FR_A = -kf Y_A + kr Y_B, so one BE step
    # is a 2x2 linear solve.
    s0 = [50.0 * 4.184e7, 52.0 * 4.184e7, 45.0 * 4.184e7]
    m = _tiny_mech([(0,)], [(1,)], W=[30.0, 30.0, 28.0], hf=[1e11, 1e11, 0.0], s0=s0,
                   cp=[5 * synth.R_U] * 3, A=2e5, beta=0.5, Ea=3000.0)
    T = np.array([900.0])
    kf, kr, _, _ = ch.rate_constants(m, T)
    kf, kr = kf[0, 0], kr[0, 0]
    b = np.array([[0.25], [0.05], [0.7]])
    c = 3e-6
    A = np.array([[1 + c * kf, -c * kr], [-c * kf, 1 + c * kr]])
    yab = np.linalg.solve(A, b[:2, 0])
    h = ch.enthalpy(m, b, T)
    Yn, Tn, it = ch.reaction_solve(m, np.array([c]), b, h, b)
    np.testing.assert_allclose(Yn[:2, 0], yab, rtol=1e-13)
    assert Yn[2, 0] == pytest.approx(0.7, abs=1e-15)


def test_dimerisation_equilibrium_quadratic():
    # 2A <=> B with W_B = 2 W_A, thermoneutral per mass: at equilibrium
    # [B] / [A]^2 = Kc, a quadratic in Y_A for fixed Y_A + Y_B.
    WA = 20.0
    s0 = [50.0 * 4.184e7, 70.0 * 4.184e7, 45.0 * 4.184e7]
    hf = [1e11, 2e11, 0.0]
    cp = [4 * synth.R_U, 8 * synth.R_U, 3.5 * synth.R_U]
    m = _tiny_mech([(0, 0)], [(1,)], W=[WA, 2 * WA, 28.0], hf=hf, s0=s0, cp=cp, A=1e12, rho0=2e-4)
    Y = np.array([[0.2], [0.1], [0.7]])
    T = np.array([1500.0])
    h = ch.enthalpy(m, Y, T)
    Yn, Tn, it = ch.reaction_solve(m, np.array([1e6]), Y, h, Y)
    # thermodynamic Kc at the final temperature
    Tf = Tn[0]
    g = [hf[k] + cp[k] * (Tf - 298.15) - Tf * (s0[k] + cp[k] * np.log(Tf / 298.15)) for k in range(2)]
    Kc = np.exp(-(g[1] - 2 * g[0]) / (synth.R_U * Tf)) * (synth.P_ATM / (synth.R_U * Tf)) ** (-1)
    rho = m["rho0"]
    XA, XB = rho * Yn[0, 0] / WA, rho * Yn[1, 0] / (2 * WA)
    assert XB / XA ** 2 == pytest.approx(Kc, rel=1e-9)
    # mass is conserved: Y_A + Y_B unchanged
    assert Yn[0, 0] + Yn[1, 0] == pytest.approx(0.3, abs=1e-15)


def test_reaction_solve_conserves_elements_and_converges(mech9):
    Yb, Tb, c, Yg = synth.random_cell_batch(mech9, 400, seed=7)
    h = ch.enthalpy(mech9, Yb, Tb)
    Y, T, it = ch.reaction_solve(mech9, c, Yb, h, Yg)
    assert np.all(it > 0)
    # sum of mass fractions and element totals are linear invariants of G
    np.testing.assert_allclose(Y.sum(axis=0), Yb.sum(axis=0), atol=1e-13)
    el = lambda y: mech9["comp"] @ (y / mech9["W"][:, None])
    e0 = el(Yb)
    np.testing.assert_allclose(el(Y), e0, rtol=1e-12, atol=1e-14)
    # the result satisfies the backward-Euler equations (scaled residual)
    G = ch.be_residual(mech9, c, Yb, h, Y, T)
    FR = ch.reaction_source(mech9, Y, T)
    assert np.all(np.abs(G[:-1]) <= 1e-9 * (1 + np.abs(c * FR)))
    assert np.all(Y >= -1e-10)
    # enthalpy constraint holds and T matches the closed form
    np.testing.assert_allclose(T, ch.temperature(mech9, Y, h), rtol=1e-11)


def test_reaction_solve_warm_start_is_quick(mech9):
    Yb, Tb, c, Yg = synth.random_cell_batch(mech9, 200, seed=8)
    h = ch.enthalpy(mech9, Yb, Tb)
    Y, T, it = ch.reaction_solve(mech9, c, Yb, h, Yg)
    Y2, T2, it2 = ch.reaction_solve(mech9, c, Yb, h, Y)
    assert np.all(it2 <= 3) and np.all(it2 > 0)
    np.testing.assert_allclose(Y2, Y, atol=1e-13)
