"""Pins of the SDC drivers on the scalar linear model problem (section 4).

* every scheme's sweeps converge to the collocation end value, which for
  phi' = z phi is the diagonal Pade approximant of exp(z);
* the counted sweeps reproduce the paper's Tables 1 and 2 after rounding;
* the spectral radii of the iteration matrices follow the paper's statements
  about its Figures 3 and 4 (whose curves are not available).
"""
import json
import os

import numpy as np
import pytest

from oracle.linear import (LinearModel, sweeps_to_tolerance, cost_ratio,
                           iteration_matrix, spectral_radius)
from oracle.sdc import sdc_step
from oracle.coefficients import sdc_tables, node_to_node_weights

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def pade_end_value(z, n_nodes):
    if n_nodes == 3:
        num = 1 + z / 2 + z * z / 12
        den = 1 - z / 2 + z * z / 12
    elif n_nodes == 5:
        num = 1 + z / 2 + 3 * z ** 2 / 28 + z ** 3 / 84 + z ** 4 / 1680
        den = 1 - z / 2 + 3 * z ** 2 / 28 - z ** 3 / 84 + z ** 4 / 1680
    else:
        raise ValueError
    return num / den


SCHEMES = [("misdc", 1), ("misdcq", 1), ("cisdcq", 1), ("cisdcq", 3), ("imexq", 1)]


@pytest.mark.parametrize("n_nodes", [3, 5])
@pytest.mark.parametrize("adr", [(1.0, -2.0, -4.0), (0.5, -1.0, -1.0), (1.0, -10.0, -20.0)])
@pytest.mark.parametrize("scheme,nu", SCHEMES)
def test_sweeps_converge_to_collocation(n_nodes, adr, scheme, nu):
    a, d, r = adr
    out, n = sdc_step(LinearModel(a, d, r), np.array(1.0), 1.0, n_nodes, 800, scheme,
                      nu=nu, stop_tol=1e-16)
    exact = pade_end_value(a + d + r, n_nodes)
    assert abs(float(out) - exact) <= 2e-14 * max(1.0, abs(exact))


def test_pade_values_printed_to_20_digits():
    # closed-form values of the 5-node collocation end value
    for z, n, v in ((-1.0, 5, 0.36787945608232267549), (-10.0, 5, 0.022038567493112947658),
                    (-100.0, 5, 0.67044528938920470395), (-1.0, 3, 0.36842105263157894737)):
        assert abs(pade_end_value(z, n) - v) <= 2e-15 * v   # a few ulps of FP64 rounding


def _table_entries():
    with open(GOLDEN) as f:
        g = json.load(f)
    out = []
    for name in ("table1", "table2"):
        for row in g[name]["rows"]:
            for nu, R in zip(g[name]["nu"], row["R"]):
                out.append((name, row["d"], row["r"], nu, R))
    return out


def test_tables_1_and_2_sweep_counts():
    """R_nu from our counted sweeps, rounded to one decimal as printed.

    12 of the 18 printed values are reproduced exactly; 3 more are
    reproduced if one of the two counts moves by one sweep (the paper does not
    say whether it counts the sweep that meets the tolerance); 3 are not
    reproduced: (d, r, nu) = (-2, -4, 3), (-10, -20, 3), (-5, -5, 1).
    """
    exact, near = set(), set()
    cache = {}

    def count(d, r, scheme, nu):
        key = (d, r, scheme, nu)
        if key not in cache:
            cache[key] = sweeps_to_tolerance(1.0, d, r, scheme, nu=nu, n_nodes=5,
                                             tol=1e-14, max_sweeps=1000)
        return cache[key]

    for name, d, r, nu, R in _table_entries():
        NM = count(d, r, "misdcq", 1)
        NC = count(d, r, "cisdcq", nu)
        assert NM is not None and NC is not None
        if round(cost_ratio(NM, NC, nu, 4), 1) == R:
            exact.add((d, r, nu))
        if any(round(cost_ratio(NM + i, NC + j, nu, 4), 1) == R
               for i in (-1, 0, 1) for j in (-1, 0, 1)):
            near.add((d, r, nu))
    expected_exact = {(-2.0, -4.0, 6), (-10.0, -20.0, 1), (-10.0, -20.0, 6),
                      (-50.0, -100.0, 1), (-50.0, -100.0, 6), (-100.0, -5.0, 1),
                      (-100.0, -5.0, 6), (-5.0, -5.0, 3), (-5.0, -5.0, 6),
                      (-5.0, -100.0, 1), (-5.0, -100.0, 3), (-5.0, -100.0, 6)}
    assert expected_exact <= exact
    assert len(near) >= 15


def _gamma(a, d, r, scheme, nu=1, n_nodes=5):
    return spectral_radius(iteration_matrix(a, d, r, scheme, nu=nu, n_nodes=n_nodes))


@pytest.mark.parametrize("n_nodes", [3, 5])
def test_gamma_nonstiff_all_schemes_equal(n_nodes):
    # |r| < 1, d = r/2: advection dominates and every scheme converges alike
    g = [_gamma(1.0, -0.005, -0.01, s, nu, n_nodes) for s, nu in
         [("misdcq", 1), ("cisdcq", 1), ("cisdcq", 3), ("cisdcq", 6), ("imexq", 1)]]
    assert max(g) - min(g) < 2e-3


@pytest.mark.parametrize("n_nodes", [3, 5])
def test_gamma_imexq_vanishes_when_stiff(n_nodes):
    g = [_gamma(1.0, r / 2, r, "imexq", 1, n_nodes) for r in (-1e2, -1e4, -1e6)]
    assert g[0] > g[1] > g[2] and g[2] < 0.02
    # the split schemes lose their convergence rate instead
    assert _gamma(1.0, -5e3, -1e4, "misdcq", 1, n_nodes) > 0.95


@pytest.mark.parametrize("r", [-4.0, -20.0, -100.0])
@pytest.mark.parametrize("dmode", ["half", "fixed"])
def test_gamma_nested_iterations_order(r, dmode):
    # intermediate stiffness: CISDCQ-1 slower than MISDCQ, CISDCQ-3 and -6 faster
    d = r / 2 if dmode == "half" else -5.0
    gm = _gamma(1.0, d, r, "misdcq")
    g1, g3, g6 = (_gamma(1.0, d, r, "cisdcq", nu) for nu in (1, 3, 6))
    assert g1 > gm > g3 >= g6 - 1e-9


@pytest.mark.parametrize("dmode", ["half", "fixed"])
def test_cisdcq_stable_over_stiffness_range(dmode):
    for r in -np.logspace(-2, 4, 13):
        d = r / 2 if dmode == "half" else -5.0
        for nu in (1, 3, 6):
            assert _gamma(1.0, d, r, "cisdcq", nu) < 1.0


def test_cost_ratio_formula():
    # eq. simple_parallel_speedup equals the ratio of the two cost expressions
    M, nu, NM, NC = 4, 3, 30, 12
    for ups_ad, ups_r in [(1.0, 1.0), (2.0, 1.0), (1.0, 3.0)]:
        alpha = (ups_ad + ups_r) / max(ups_ad, ups_r)
        direct = NM * M * (ups_ad + ups_r) / (NC * (nu * (ups_ad + ups_r) + (M - 1) * max(ups_ad, ups_r)))
        assert abs(cost_ratio(NM, NC, nu, M, alpha) - direct) < 1e-13


# ---------------------------------------------------------------------------
# adaptive nested iterations (the paper's future-work item of sections 4.1-4.3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n_nodes", [3, 5])
@pytest.mark.parametrize("adr", [(1.0, -2.0, -4.0), (0.5, -1.0, -1.0), (0.2, -3.0, -0.5)])
def test_adaptive_nested_iterations_reach_the_imexq_sweep(n_nodes, adr):
    """At a fixed point of the nested iterations (the same values in passes
    l and l+1 at every node) the reaction update returns the diffusion
    output, and the diffusion update with the lagged terms at their fixed
    values is the coupled implicit update of the IMEXQ sweep (section 3.3's
    comparison scheme; the coefficients of the linear problem do not depend
    on the lagged state).  Nested iterations run until they stall must
    therefore give IMEXQ's sweeps."""
    a, d, r = adr
    for sweeps in (1, 3):
        ps = []
        out, _ = sdc_step(LinearModel(a, d, r), np.array(1.0), 1.0, n_nodes, sweeps, "cisdcq",
                          nu=400, nu_tol=1e-15, passes=ps)
        ref, _ = sdc_step(LinearModel(a, d, r), np.array(1.0), 1.0, n_nodes, sweeps, "imexq")
        assert len(ps) == sweeps and all(2 <= v < 400 for v in ps), ps
        assert abs(float(out) - float(ref)) <= 1e-13 * abs(float(ref)), (out, ref)


def test_adaptive_pass_count_follows_the_stall_rule():
    """The passes done are the first l >= 2 whose change of the node-M value
    is at most nu_tol times the first pass's change, with the changes taken
    from separate fixed-nu sweeps (a fixed-nu sweep with nu = l ends with the
    values of pass l)."""
    model, n_nodes = LinearModel(0.5, -1.0, -1.0), 5
    vals = [float(sdc_step(model, np.array(1.0), 1.0, n_nodes, 1, "cisdcq", nu=l)[0])
            for l in range(1, 9)]
    delta = [abs(vals[0] - 1.0) / abs(vals[0])]
    delta += [abs(vals[l] - vals[l - 1]) / abs(vals[l]) for l in range(1, 8)]
    ratios = np.array(delta[1:]) / delta[0]
    assert np.all(np.diff(ratios) < 0)            # the nested iteration contracts
    for tol in (1e-2, 1e-4, 1e-7):
        assert np.min(np.abs(ratios - tol)) > 1e-3 * tol
        expect = next(l + 1 for l in range(1, 8) if delta[l] <= tol * delta[0])
        ps = []
        sdc_step(model, np.array(1.0), 1.0, n_nodes, 1, "cisdcq", nu=8, nu_tol=tol, passes=ps)
        assert ps == [expect], (tol, ps, ratios)


@pytest.mark.parametrize("n_nodes", [3, 5])
def test_adaptive_limits_are_fixed_nu(n_nodes):
    """nu_tol = 0 never stops a pass that still changes the state (fixed
    nu = nu_max); an infinite nu_tol stops after the second pass (fixed
    nu = 2): bitwise the fixed-nu sweeps."""
    model = LinearModel(1.0, -2.0, -4.0)
    fixed3 = sdc_step(model, np.array(1.0), 1.0, n_nodes, 4, "cisdcq", nu=3)[0]
    fixed2 = sdc_step(model, np.array(1.0), 1.0, n_nodes, 4, "cisdcq", nu=2)[0]
    p0, pinf = [], []
    a0 = sdc_step(model, np.array(1.0), 1.0, n_nodes, 4, "cisdcq", nu=3, nu_tol=0.0, passes=p0)[0]
    ainf = sdc_step(model, np.array(1.0), 1.0, n_nodes, 4, "cisdcq", nu=3, nu_tol=np.inf,
                    passes=pinf)[0]
    assert float(a0) == float(fixed3) and p0 == [3] * 4
    assert float(ainf) == float(fixed2) and pinf == [2] * 4


def _misdc_one_stage(a, d, r, n_nodes, sweeps, dt=1.0):
    """K node-to-node MISDC sweeps on phi' = (a + d + r) phi, phi^n = 1, written
    as a single implicit Euler stage per sub-interval.

    Eliminating phi_AD between the diffusion and the reaction update of MISDC
    (eqs. update_equation_misdc_discrete_form_D/R) leaves, with delta = dt^m,
        (1 - delta d)(1 - delta r) phi^{m+1,(k+1)} = phi^{m,(k+1)}
            + delta a (phi^{m,(k+1)} - phi^{m,(k)})
            - delta (d + r - delta d r) phi^{m+1,(k)} + dt S^{m:m+1} F^{(k)}:
    a one-stage form in which a dropped or misweighted bracket of either
    stage changes the result after the first sweep.
    """
    tau = sdc_tables(n_nodes)["tau"]
    S = node_to_node_weights(n_nodes)
    M = n_nodes - 1
    z = a + d + r
    old = np.ones(M + 1)
    for _ in range(sweeps):
        new = np.empty(M + 1)
        new[0] = 1.0
        for m in range(M):
            de = dt * (tau[m + 1] - tau[m])
            rhs = (new[m] + de * a * (new[m] - old[m]) - de * (d + r - de * d * r) * old[m + 1]
                   + dt * (S[m] @ (z * old)))
            new[m + 1] = rhs / ((1.0 - de * d) * (1.0 - de * r))
        old = new
    return old[M]


@pytest.mark.parametrize("n_nodes", [3, 5])
@pytest.mark.parametrize("adr", [(1.0, -2.0, -4.0), (0.5, -7.0, -0.3), (-1.5, -0.2, -30.0)])
def test_misdc_sweeps_equal_one_stage_form(n_nodes, adr):
    a, d, r = adr
    for K in range(1, 6):
        out, _ = sdc_step(LinearModel(a, d, r), np.array(1.0), 0.7, n_nodes, K, "misdc")
        ref = _misdc_one_stage(a, d, r, n_nodes, K, dt=0.7)
        assert abs(float(out) - ref) <= 1e-14 * max(1.0, abs(ref)), (K, float(out), ref)


@pytest.mark.parametrize("n_nodes", [3, 5])
@pytest.mark.parametrize("r", [-10.0, -100.0, -1000.0])
@pytest.mark.parametrize("dmode", ["half", "fixed"])
def test_gamma_lu_weights_beat_backward_euler(n_nodes, r, dmode):
    """Section 3.1: the LU-trick implicit weights make the sweeps converge
    faster than node-to-node backward Euler, and MISDCQ needs fewer sweeps
    than MISDC on stiff problems."""
    d = r / 2 if dmode == "half" else -5.0
    g_be = _gamma(1.0, d, r, "misdc", 1, n_nodes)
    g_lu = _gamma(1.0, d, r, "misdcq", 1, n_nodes)
    assert g_be > g_lu + 5e-3, (g_be, g_lu)
    n_be = sweeps_to_tolerance(1.0, d, r, "misdc", n_nodes=n_nodes, max_sweeps=3000)
    n_lu = sweeps_to_tolerance(1.0, d, r, "misdcq", n_nodes=n_nodes, max_sweeps=3000)
    assert n_lu is not None
    assert n_be is None or n_be > n_lu
