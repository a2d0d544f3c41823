"""Scalar linear model problem of section 4 (oracle; test infrastructure only).

phi' = a phi + d phi + r phi (eq. linear_model_problem), with a the explicit
advection, d the implicit diffusion and r the implicit reaction coefficient.
Provides the sweep iteration matrix G computed numerically (the sweep is an
affine map of the node values, so G is its Jacobian, obtained column by column
from unit perturbations), the collocation end value, and the cost ratio R_nu
of eq. simple_parallel_speedup.
"""
import numpy as np

from .sdc import (sdc_step, scheme_tables, sweep_misdc, sweep_misdcq,
                  sweep_cisdcq, sweep_imexq, _evalF)
from .coefficients import node_to_node_weights


class LinearModel:
    def __init__(self, a, d, r):
        self.a, self.d, self.r = float(a), float(d), float(r)

    def FA(self, phi):
        return self.a * phi

    def FD(self, phi):
        return self.d * phi

    def FR(self, phi):
        return self.r * phi

    def solve_D(self, c, rhs, lag):
        return rhs / (1.0 - c * self.d)

    def solve_R(self, c, b, guess):
        return b / (1.0 - c * self.r)

    def solve_DR(self, c, rhs, guess, lag):
        return rhs / (1.0 - c * (self.d + self.r))


def sweeps_to_tolerance(a, d, r, scheme, nu=1, n_nodes=5, dt=1.0, tol=1e-14,
                        max_sweeps=400, qe="cumulative", phi0=1.0):
    """Number of sweeps until |phi^{M,(k)} - phi^{M,(k-1)}| <= tol (section 5.1)."""
    prob = LinearModel(a, d, r)
    incs = []
    _, n = sdc_step(prob, np.array(phi0), dt, n_nodes, max_sweeps, scheme, nu=nu,
                    qe=qe, increments=incs, stop_tol=tol)
    if incs[-1] > tol:
        return None
    return n


def cost_ratio(N_M, N_C, nu, M, alpha=2.0):
    """R_nu = (N_M / N_C) * alpha M / (alpha nu + M - 1)  (eq. simple_parallel_speedup)."""
    return (N_M / N_C) * alpha * M / (alpha * nu + M - 1)


def iteration_matrix(a, d, r, scheme, nu=1, n_nodes=5, dt=1.0, qe="cumulative"):
    """G with Phi^{(k+1)} - Phi^{(k)} = G (Phi^{(k)} - Phi^{(k-1)}).

    The sweep maps the node values of sweep k (nodes 1..M; the operator values
    are linear in them) affinely to those of sweep k+1, so G is the matrix of
    its linear part, recovered from the images of the unit vectors minus the
    image of zero.
    """
    prob = LinearModel(a, d, r)
    tab = scheme_tables(n_nodes, scheme, qe)
    S = node_to_node_weights(n_nodes) if scheme == "misdc" else None
    M = tab["M"]

    def sweep(vals):
        phi = [np.array(1.0)] + [np.array(v) for v in vals]
        F = [_evalF(prob, x) for x in phi]
        if scheme == "misdc":
            out, _ = sweep_misdc(prob, phi, F, dt, tab, S)
        elif scheme == "misdcq":
            out, _ = sweep_misdcq(prob, phi, F, dt, tab)
        elif scheme == "cisdcq":
            out, _ = sweep_cisdcq(prob, phi, F, dt, tab, nu)
        else:
            out, _ = sweep_imexq(prob, phi, F, dt, tab)
        return np.array([float(x) for x in out[1:]])

    base = sweep(np.zeros(M))
    G = np.zeros((M, M))
    for i in range(M):
        e = np.zeros(M)
        e[i] = 1.0
        G[:, i] = sweep(e) - base
    return G


def spectral_radius(G):
    return float(np.max(np.abs(np.linalg.eigvals(G))))
