"""The advection-diffusion-reaction flame problem (oracle; test infrastructure only).

State per cell: phi = (Y_1..Y_N, h) with constant density rho0 (with a uniform
prescribed velocity and uniform initial density the continuity equation keeps
the density uniform, so the EOS/velocity-constraint machinery of section 2 has
nothing to do).  F = FA + FD + FR as in ``transport`` and ``chemistry``; the
enthalpy row of FR is zero.  The temperature of a state is always the
closed-form T(Y, h).

The implicit diffusion solve uses coefficients from the lagged state passed by
the SDC driver (eq. lagged_diffusion_flux); explicit evaluations of FD use the
state's own temperature.  The reaction solve keeps h fixed and solves the
backward-Euler system for (Y, T) with the guess passed by the driver.
"""
import numpy as np

from . import chemistry as chem
from . import transport as tr


class FlameProblem:
    def __init__(self, mech, dx, u, newton_tol=1e-12, newton_maxit=200):
        self.mech = mech
        self.dx = tuple(float(v) for v in dx)
        self.u = tuple(float(v) for v in u)
        self.N = mech["N"]
        self.newton_tol = newton_tol
        self.newton_maxit = newton_maxit
        self.newton_iters = []        # one array of per-cell counts per solve

    # -- helpers -----------------------------------------------------------
    def temperature(self, phi):
        N = self.N
        Y = phi[:N].reshape(N, -1)
        return chem.temperature(self.mech, Y, phi[N].reshape(-1)).reshape(phi.shape[1:])

    def state_from_YT(self, Y, T):
        h = chem.enthalpy(self.mech, Y.reshape(self.N, -1), T.reshape(-1)).reshape(T.shape)
        return np.concatenate([Y, h[None]], axis=0)

    # -- SDC problem interface ----------------------------------------------
    def FA(self, phi):
        return tr.advection(phi, self.u, self.dx)

    def FD(self, phi):
        return tr.diffusion(self.mech, phi, self.temperature(phi), self.dx)

    def FR(self, phi):
        N = self.N
        out = np.zeros_like(phi)
        Y = phi[:N].reshape(N, -1)
        T = self.temperature(phi).reshape(-1)
        out[:N] = chem.reaction_source(self.mech, Y, T).reshape(phi[:N].shape)
        return out

    def solve_D(self, c, rhs, lag):
        return tr.diffusion_solve(self.mech, c, rhs, self.temperature(lag), self.dx)

    def solve_R(self, c, b, guess):
        N = self.N
        shape = b.shape[1:]
        bY = b[:N].reshape(N, -1)
        h = b[N].reshape(-1)
        cc = np.full(h.shape, float(c))
        Y, _T, it = chem.reaction_solve(self.mech, cc, bY, h, guess[:N].reshape(N, -1),
                                        tol=self.newton_tol, maxit=self.newton_maxit)
        self.newton_iters.append(it)
        out = np.empty_like(b)
        out[:N] = Y.reshape((N,) + shape)
        out[N] = b[N]                 # no reaction source in the enthalpy
        return out


RELAX_TIME = 1.0


def relaxed_initial_state(prob, Y, T, c_relax=RELAX_TIME):
    """Initial state of the flame workloads: the synthetic (Y, T) fields at
    their enthalpy, followed by one constant-enthalpy backward-Euler reaction
    solve of length ``c_relax`` (guess = the synthetic composition).  This puts
    the initial state near the fast chemical manifold, as a physical flame
    state is; without it the very first quadrature carries reaction rates of
    order 1e10 1/s from an arbitrary composition.
    """
    phi = prob.state_from_YT(Y, T)
    return prob.solve_R(c_relax, phi, phi)
