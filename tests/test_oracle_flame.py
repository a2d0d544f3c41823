"""Pins of the oracle sweeps on nonlinear problems.

* P-5: on tiny flame grids, many sweeps of every scheme reach the collocation
  solution computed independently by a dense Newton solve;
* P-6: temporal order on the paper's nonlinear test PDE: k sweeps give order
  min(k, 2M) (section 5.2: order 2 with two sweeps, 4 with four);
* P-7: conservation over a flame step (sum of mass fractions per cell, domain
  totals of elements and enthalpy).
"""
import numpy as np
import pytest

import synth
from oracle.adr import FlameProblem, relaxed_initial_state
from oracle.collocation import collocation_solve
from oracle.nagumo import Nagumo
from oracle.sdc import sdc_step


@pytest.fixture(scope="module")
def mild_flame():
    m = synth.make_mechanism(9, 21, 0, A_range=(1e2, 1e6))
    Y, T = synth.flame_1d(m, 4, dx=0.02)
    prob = FlameProblem(m, (0.02,), (100.0,))
    phi0 = relaxed_initial_state(prob, Y, T)
    return prob, phi0


@pytest.fixture(scope="module")
def mild_collocation(mild_flame):
    prob, phi0 = mild_flame
    return collocation_solve(prob, phi0, 2e-5, 5)


@pytest.mark.parametrize("scheme,nu", [("misdc", 1), ("misdcq", 1), ("cisdcq", 1), ("cisdcq", 3),
                                       ("imexq", 1)])
def test_sweeps_reach_collocation_fixed_point(mild_flame, mild_collocation, scheme, nu):
    prob, phi0 = mild_flame
    out, _ = sdc_step(prob, phi0, 2e-5, 5, 60, scheme, nu=nu)
    scale = np.abs(mild_collocation[-1]).max(axis=1, keepdims=True)
    assert (np.abs(out - mild_collocation[-1]) / scale).max() < 1e-11


def test_collocation_residual_is_small(mild_flame, mild_collocation):
    # independent check of the brute-force solve: plug it back in
    from oracle.coefficients import sdc_tables
    prob, phi0 = mild_flame
    t = sdc_tables(5)
    F = [prob.FA(x) + prob.FD(x) + prob.FR(x) for x in mild_collocation]
    for p in range(1, 5):
        rhs = phi0 + 2e-5 * sum(t["Q"][p - 1, j] * F[j] for j in range(5))
        scale = np.abs(rhs).max(axis=1, keepdims=True)
        assert (np.abs(mild_collocation[p] - rhs) / scale).max() < 1e-13


def _nagumo_solution(scheme, nu, dt, sweeps, t_end=0.4):
    prob = Nagumo(a=1.0, d=2.0, r=4.0, nx=200)
    phi = prob.initial()
    for _ in range(int(round(t_end / dt))):
        phi, _ = sdc_step(prob, phi, dt, 5, sweeps, scheme, nu=nu)
    return phi


@pytest.fixture(scope="module")
def nagumo_reference():
    return _nagumo_solution("misdcq", 1, 0.1 / 32, 8)


@pytest.mark.slow
@pytest.mark.parametrize("scheme,nu", [("misdcq", 1), ("cisdcq", 1)])
@pytest.mark.parametrize("sweeps,order", [(2, 2), (4, 4)])
def test_nagumo_temporal_order(nagumo_reference, scheme, nu, sweeps, order):
    errs = []
    dts = (0.1, 0.05, 0.025)
    for dt in dts:
        phi = _nagumo_solution(scheme, nu, dt, sweeps)
        errs.append(np.mean(np.abs(phi - nagumo_reference)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > order - 0.35, (errs, rates)


@pytest.mark.parametrize("scheme,nu", [("misdc", 1), ("cisdcq", 2)])
def test_flame_step_conservation(scheme, nu):
    m = synth.make_mechanism(9, 21, 0)
    Y, T = synth.flame_2d(m, 12, 10)
    prob = FlameProblem(m, (0.01, 0.01), (100.0, 0.0))
    phi0 = relaxed_initial_state(prob, Y, T)
    out, _ = sdc_step(prob, phi0, 5e-5, 3, 3, scheme, nu=nu)
    N = m["N"]
    np.testing.assert_allclose(out[:N].sum(axis=0), 1.0, atol=1e-13)
    el = lambda p: m["comp"] @ (p[:N] / m["W"][:, None, None]).reshape(N, -1)
    np.testing.assert_allclose(el(out).sum(axis=1), el(phi0).sum(axis=1), rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(out[N].sum(), phi0[N].sum(), rtol=1e-13)
    assert np.all(np.isfinite(out))
    assert all(np.all(it > 0) for it in prob.newton_iters)


@pytest.fixture(scope="module")
def nagumo_fine_reference():
    return _nagumo_solution("misdcq", 1, 0.1 / 64, 8)


@pytest.mark.slow
@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_nagumo_misdc_order_per_sweep(nagumo_fine_reference, sweeps):
    # node-to-node MISDC from the spread initial value: each sweep of the
    # first-order correction raises the order by one, up to 2M (sections 3.1,
    # 5.2); the third sweep is still pre-asymptotic at these step sizes
    errs = []
    for dt in (0.05, 0.025, 0.0125):
        errs.append(np.mean(np.abs(_nagumo_solution("misdc", 1, dt, sweeps) - nagumo_fine_reference)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > sweeps - 0.2, (errs, rates)
    assert rates[-1] < sweeps + 0.5, (errs, rates)


def test_field_increments_and_progress_record_the_sweep_changes():
    """The per-field increment record of sdc_step: its differences are those
    of successive sweeps' node-M states, computed here by running the step
    with 1, 2 and 3 sweeps; the overall max-abs increment is the largest
    field difference; the progress callback sees every sweep in order."""
    mech = synth.make_mechanism(9, 21, 0)
    Y, T = synth.flame_2d(mech, 12, 10)
    prob = FlameProblem(mech, (0.01, 0.01), (100.0, 0.0))
    phi = relaxed_initial_state(prob, Y, T)
    fi, inc, seen = [], [], []
    sdc_step(prob, phi, 5e-5, 3, 3, "cisdcq", increments=inc, field_increments=fi,
             progress=lambda k, v: seen.append((k, v)))
    assert [k for k, _ in seen] == [0, 1, 2] and [v for _, v in seen] == inc
    states = [phi] + [sdc_step(prob, phi, 5e-5, 3, k, "cisdcq")[0] for k in (1, 2, 3)]
    for k in range(3):
        d = np.abs(states[k + 1] - states[k]).reshape(10, -1).max(axis=1)
        a = np.abs(states[k + 1]).reshape(10, -1).max(axis=1)
        np.testing.assert_allclose(fi[k][:, 0], d, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(fi[k][:, 1], a, rtol=1e-15)
        assert inc[k] == fi[k][:, 0].max()


def _coupled_case(mech, nx=10, ny=8, seed=3):
    """A 2-D state, a right-hand side near it and a lagged state."""
    Y, T = synth.flame_2d(mech, nx, ny)
    prob = FlameProblem(mech, (0.01, 0.01), (100.0, 0.0))
    phi = relaxed_initial_state(prob, Y, T)
    rng = np.random.default_rng(seed)
    rhs = phi * (1.0 + 1e-3 * rng.standard_normal(phi.shape))
    rhs[:9] = np.abs(rhs[:9])
    lag = phi * (1.0 + 1e-3 * rng.standard_normal(phi.shape))
    lag[:9] = np.abs(lag[:9])
    return prob, phi, rhs, lag


def test_coupled_solve_without_reactions_is_the_diffusion_solve():
    """IMEXQ's coupled solve with every rate constant zero has no reaction
    source: it is the implicit diffusion step S3/S4 of the same lagged
    coefficients (a direct solve per field and the dominant-species closure),
    computed independently by solve_D."""
    mech = synth.make_mechanism(9, 21, 0)
    mech = dict(mech, A=np.zeros_like(mech["A"]))
    prob, phi, rhs, lag = _coupled_case(mech)
    c = 3e-5
    got = prob.solve_DR(c, rhs, phi, lag)
    ref = prob.solve_D(c, rhs, lag)
    scale = np.abs(ref).reshape(10, -1).max(axis=1)[:, None, None]
    assert (np.abs(got - ref) / scale).max() <= 1e-12


def test_coupled_solve_without_diffusion_is_the_reaction_solve():
    """With every diffusivity zero the coupled solve has no spatial coupling:
    it is the per-cell backward-Euler reaction step S5 at fixed h, computed
    independently by solve_R (Newton on (Y, T) with pseudo-transient
    continuation)."""
    mech = synth.make_mechanism(9, 21, 0)
    mech = dict(mech, D0=np.zeros_like(mech["D0"]), alpha0=0.0)
    prob, phi, rhs, lag = _coupled_case(mech)
    c = 3e-5
    got = prob.solve_DR(c, rhs, phi, lag)
    ref = prob.solve_R(c, rhs, phi)
    scale = np.abs(ref).reshape(10, -1).max(axis=1)[:, None, None]
    assert (np.abs(got - ref) / scale).max() <= 1e-11


def test_coupled_solve_residual_and_conservation():
    """The coupled solve's result satisfies its equation, evaluated with the
    explicit diffusion operator at the lagged temperature and the reaction
    source; the mass fractions of every cell still sum to that of the
    right-hand side (neither operator creates mass)."""
    from oracle import chemistry as ch
    from oracle import transport as tr
    mech = synth.make_mechanism(9, 21, 0)
    prob, phi, rhs, lag = _coupled_case(mech)
    c = 3e-5
    x = prob.solve_DR(c, rhs, phi, lag)
    FD = tr.diffusion(mech, x, prob.temperature(lag), prob.dx)
    FR = prob.FR(x)
    res = x - c * (FD + FR) - rhs
    # mass fractions are O(1) quantities: a species whose largest value is
    # tiny is still measured against 1e-3
    scale = np.abs(rhs).reshape(10, -1).max(axis=1)
    scale[:9] = np.maximum(scale[:9], 1e-3)
    assert (np.abs(res) / scale[:, None, None]).max() <= 1e-12
    np.testing.assert_allclose(x[:9].sum(axis=0), rhs[:9].sum(axis=0), atol=1e-12)


def test_coupled_solve_converges_on_the_stiff_flame():
    """On the workload's stiff 1-D flame (the step size and node spacing of
    the GPU parity case) the coupled Newton converges: trace species stall at
    the rounding level of the O(1) species coupled into them, far above 1e-13
    of their own magnitude, so mass fractions are tested absolutely.  The
    result satisfies its equation and conserves the mass fractions."""
    from oracle import transport as tr
    from oracle.coefficients import sdc_tables
    mech = synth.make_mechanism(9, 21, 0)
    Y, T = synth.flame_1d(mech, 64, 0.01)
    prob = FlameProblem(mech, (0.01,), (100.0,))
    phi = relaxed_initial_state(prob, Y, T)
    c = 5e-5 * sdc_tables(3)["QI"][1, 1]
    rhs = phi + c * (prob.FD(phi) + prob.FR(phi))
    x = prob.solve_DR(c, rhs, phi, phi)
    res = x - c * (tr.diffusion(mech, x, prob.temperature(phi), prob.dx) + prob.FR(x)) - rhs
    scale = np.abs(rhs).reshape(10, -1).max(axis=1)
    scale[:9] = np.maximum(scale[:9], 1e-3)
    assert (np.abs(res) / scale[:, None]).max() <= 1e-12
    np.testing.assert_allclose(x[:9].sum(axis=0), rhs[:9].sum(axis=0), atol=1e-12)
