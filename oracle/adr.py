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
backward-Euler system for (Y, T) with the guess passed by the driver.  The
coupled solve of the comparison scheme IMEXQ (section 3.2.2) treats diffusion
(lagged coefficients) and reaction implicitly together.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

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


    def solve_DR(self, c, rhs, guess, lag, tol=1e-13, maxit=30):
        """IMEXQ's implicit step: phi - c (FD_lag(phi) + FR(phi)) = rhs, with
        FD_lag the diffusion operator whose coefficients come from the lagged
        state (as in solve_D, dominant species by closure) and FR the reaction
        source at phi's own temperature T(Y, h).  Newton's method on the whole
        grid from ``guess``: the Jacobian I - c (D + R) is assembled as a
        sparse matrix, D the lagged diffusion operator of every field (the
        dominant species' row is minus the sum of the other species' rows) and
        R each cell's derivative of FR with respect to (Y, h) through
        T(Y, h), and solved directly.  Converged when every mass fraction's
        update is at most tol (mass fractions are O(1) quantities, tested
        absolutely as in the per-cell reaction solve: a trace species' update
        stalls at the rounding level of the large ones coupled into it, far
        above tol times its own magnitude) and the enthalpy's update at most
        tol times its largest magnitude."""
        mech, N = self.mech, self.N
        nf = N + 1
        shape = rhs.shape[1:]
        n = int(np.prod(shape))
        th = tr.theta(self.temperature(lag))
        L = tr.laplacian_matrix(th, self.dx)
        k0 = tr.diffusion_coefficients(mech)
        i0 = mech["bath"]
        blocks = [[None] * nf for _ in range(nf)]
        for f in range(nf):
            if f != i0:
                blocks[f][f] = k0[f] * L
        for k in range(N):
            if k != i0:
                blocks[i0][k] = -k0[k] * L
        for f in range(nf):
            if blocks[f][f] is None:
                blocks[f][f] = sp.csc_matrix((n, n))
        D = sp.bmat(blocks, format="csc")
        x = np.array(guess, dtype=np.float64).reshape(nf, n).copy()
        b = rhs.reshape(nf, n)
        idx = np.arange(n)
        for _ in range(maxit):
            Y, h = x[:N], x[N]
            T = chem.temperature(mech, Y, h)
            FR = np.zeros_like(x)
            FR[:N] = chem.reaction_source(mech, Y, T)
            G = x.ravel() - c * (D @ x.ravel() + FR.ravel()) - b.ravel()
            dY, dT = chem.reaction_source_jacobian(mech, Y, T)
            cpm = np.sum(Y * (mech["cp"] / mech["W"])[:, None], axis=0)
            hhat = chem.species_enthalpy(mech, T) / mech["W"][:, None]
            rows, cols, vals = [], [], []
            for k in range(N):
                for l in range(N):
                    rows.append(k * n + idx)
                    cols.append(l * n + idx)
                    vals.append(dY[k, l] - dT[k] * hhat[l] / cpm)
                rows.append(k * n + idx)
                cols.append(N * n + idx)
                vals.append(dT[k] / cpm)
            R = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                              shape=(nf * n, nf * n))
            A = sp.identity(nf * n, format="csc") - c * (D + R)
            d = spla.spsolve(A, G).reshape(nf, n)
            if not np.all(np.isfinite(d)):
                raise FloatingPointError("coupled diffusion-reaction Newton step is not finite")
            x -= d
            scale = np.ones(nf)
            scale[N] = np.abs(x[N]).max()
            if np.all(np.abs(d).max(axis=1) <= tol * scale):
                break
        else:
            raise RuntimeError("coupled diffusion-reaction solve did not converge")
        return x.reshape(rhs.shape)


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
