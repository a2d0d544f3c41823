"""Pins of the SDC coefficient tables (section 3.1) against closed forms."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.coefficients import sdc_tables, node_to_node_weights


def _f(x):
    return float(x)


def test_three_node_tables_closed_form():
    # 3 Gauss-Lobatto nodes: tau = (0, 1/2, 1); Q by exact integration of the
    # quadratic Lagrange basis; Q~I from the Doolittle LU of Q~^T.
    t = sdc_tables(3)
    assert np.array_equal(t["tau"], [0.0, 0.5, 1.0])
    Q = [[Fr(5, 24), Fr(1, 3), Fr(-1, 24)], [Fr(1, 6), Fr(2, 3), Fr(1, 6)]]
    np.testing.assert_array_equal(t["Q"], [[_f(v) for v in row] for row in Q])
    np.testing.assert_array_equal(t["QI"], [[_f(Fr(1, 3)), 0.0], [_f(Fr(2, 3)), 0.25]])
    np.testing.assert_array_equal(t["QE"], [[0.0, 0.0], [0.5, 0.0]])
    be = sdc_tables(3, qi="be")["QI"]
    np.testing.assert_array_equal(be, [[0.5, 0.0], [0.5, 0.5]])
    # both readings of the explicit weights coincide for three nodes
    np.testing.assert_array_equal(sdc_tables(3, qe="literal")["QE"], t["QE"])


def test_five_node_tables_closed_form():
    t = sdc_tables(5)
    s = np.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(t["tau"], [0, 0.5 - 0.5 * s, 0.5, 0.5 + 0.5 * s, 1], rtol=0, atol=2e-16)
    # last row of Q = Gauss-Lobatto weights on [0, 1]
    np.testing.assert_allclose(t["Q"][-1], [1 / 20, 49 / 180, 16 / 45, 49 / 180, 1 / 20], rtol=0, atol=1e-16)
    # row sums of Q are the node positions (integral of 1 from 0 to tau_p)
    np.testing.assert_allclose(t["Q"].sum(axis=1), t["tau"][1:], rtol=0, atol=3e-16)
    # exactness for t^3: integral_0^tau t^3 dt = tau^4 / 4
    np.testing.assert_allclose(t["Q"] @ t["tau"] ** 3, t["tau"][1:] ** 4 / 4, rtol=0, atol=3e-16)
    QI = t["QI"]
    assert np.all(np.triu(QI, 1) == 0.0)
    # the LU-trick diagonal for 5 Lobatto nodes ends with 1/11
    assert abs(QI[3, 3] - 1.0 / 11.0) <= 2e-17
    # transpose(Q~) = L U with L unit lower and U = transpose(QI)
    U = QI.T
    L = t["Qt"].T @ np.linalg.inv(U)
    np.testing.assert_allclose(np.diag(L), 1.0, atol=1e-14)
    np.testing.assert_allclose(np.triu(L, 1), 0.0, atol=1e-14)
    # the first column of Q~I equals the first column of Q~
    np.testing.assert_allclose(QI[:, 0], t["Qt"][:, 0], rtol=0, atol=1e-16)


def test_backward_euler_and_forward_euler_tables():
    t = sdc_tables(5, qi="be")
    dtau = np.diff(t["tau"])
    for p in range(1, 5):
        np.testing.assert_allclose(t["QI"][p - 1, :p], dtau[:p], atol=1e-16)
        np.testing.assert_allclose(t["QE"][p - 1, :p - 1], dtau[1:p], atol=1e-16)
    lit = sdc_tables(5, qe="literal")["QE"]
    assert np.count_nonzero(lit) == 3
    np.testing.assert_allclose([lit[1, 0], lit[2, 1], lit[3, 2]], dtau[1:], atol=1e-16)


@pytest.mark.parametrize("n_nodes", [2, 3, 4, 5, 6])
def test_node_to_node_weights_integrate_polynomials(n_nodes):
    S = node_to_node_weights(n_nodes)
    tau = sdc_tables(n_nodes)["tau"]
    for deg in range(n_nodes):
        exact = (tau[1:] ** (deg + 1) - tau[:-1] ** (deg + 1)) / (deg + 1)
        np.testing.assert_allclose(S @ tau ** deg, exact, rtol=0, atol=5e-16)


@pytest.mark.parametrize("n_nodes", [7, 9])
def test_many_node_tables(n_nodes):
    """Pins of the 7- and 9-node tables (the library accepts up to 9 nodes).

    The interior Gauss-Lobatto nodes are the roots of P'_M, taken here from
    NumPy's Legendre series (not the recurrence and root finder of the
    oracle); the last row of Q holds the Lobatto weights, exact for
    polynomials of degree <= 2M - 1; every row of Q integrates polynomials of
    degree <= M exactly; Q~I is the transpose of the upper Doolittle factor
    of transpose(Q~).
    """
    M = n_nodes - 1
    t = sdc_tables(n_nodes)
    dP = np.polynomial.legendre.Legendre.basis(M).deriv()
    inner = np.sort(dP.roots().real)
    np.testing.assert_allclose(t["tau"], np.concatenate([[0.0], (inner + 1) / 2, [1.0]]),
                               rtol=0, atol=1e-15)
    # a Newton step on P'_M from each oracle node moves it by at most ~ulp
    x = 2 * t["tau"][1:-1] - 1
    assert np.all(np.abs(dP(x) / dP.deriv()(x)) <= 2e-15)
    # symmetry of the nodes about 1/2
    np.testing.assert_allclose(t["tau"] + t["tau"][::-1], 1.0, rtol=0, atol=4e-16)
    w = t["Q"][-1]
    for deg in range(2 * M):
        assert abs(w @ t["tau"] ** deg - 1.0 / (deg + 1)) <= 2e-15, deg
    # not exact one degree higher (Lobatto: exactly 2M - 1)
    assert abs(w @ t["tau"] ** (2 * M) - 1.0 / (2 * M + 1)) > 1e-11
    for deg in range(M + 1):
        np.testing.assert_allclose(t["Q"] @ t["tau"] ** deg, t["tau"][1:] ** (deg + 1) / (deg + 1),
                                   rtol=0, atol=2e-15)
    QI = t["QI"]
    assert np.all(np.triu(QI, 1) == 0.0)
    L = t["Qt"].T @ np.linalg.inv(QI.T)
    np.testing.assert_allclose(np.diag(L), 1.0, atol=1e-13)
    np.testing.assert_allclose(np.triu(L, 1), 0.0, atol=1e-13)
    np.testing.assert_allclose(QI[:, 0], t["Qt"][:, 0], rtol=0, atol=1e-16)
    # backward-Euler and forward-Euler tables follow the node spacing
    dtau = np.diff(t["tau"])
    be = sdc_tables(n_nodes, qi="be")
    for p in range(1, M + 1):
        np.testing.assert_allclose(be["QI"][p - 1, :p], dtau[:p], atol=1e-16)
        np.testing.assert_allclose(be["QE"][p - 1, :p - 1], dtau[1:p], atol=1e-16)


@pytest.mark.parametrize("n_nodes", [7, 8, 9])
def test_node_to_node_weights_many_nodes(n_nodes):
    S = node_to_node_weights(n_nodes)
    tau = sdc_tables(n_nodes)["tau"]
    for deg in range(n_nodes):
        exact = (tau[1:] ** (deg + 1) - tau[:-1] ** (deg + 1)) / (deg + 1)
        np.testing.assert_allclose(S @ tau ** deg, exact, rtol=0, atol=2e-15)
