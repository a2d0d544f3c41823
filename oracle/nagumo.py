"""The paper's 1-D nonlinear test PDE (oracle; test infrastructure only).

phi_t = a phi_x + d phi_xx + r phi (phi - 1)(phi - 1/2) on [0, 20] with
phi(0) = 1, phi(20) = 0 and phi0(x) = (1 + tanh(20 - 2x)) / 2
(eq. nonlinear_test_pde).  The space discretisation here is second-order
central on cell centres with ghost values from the Dirichlet data (the time
refinement study only needs a fixed semi-discrete system); the implicit
diffusion is a tridiagonal solve and the implicit reaction a per-cell scalar
Newton solve of the cubic.
"""
import numpy as np
import scipy.linalg as sla


class Nagumo:
    def __init__(self, a=1.0, d=2.0, r=4.0, nx=200, length=20.0):
        self.a, self.d, self.r = float(a), float(d), float(r)
        self.nx = nx
        self.dx = length / nx
        self.x = (np.arange(nx) + 0.5) * self.dx

    def initial(self):
        return 0.5 * (1.0 + np.tanh(20.0 - 2.0 * self.x))

    def _ghost(self, phi):
        # Dirichlet phi(0) = 1, phi(L) = 0 imposed at the faces
        return np.concatenate([[2.0 - phi[0]], phi, [-phi[-1]]])

    def FA(self, phi):
        g = self._ghost(phi)
        return self.a * (g[2:] - g[:-2]) / (2.0 * self.dx)

    def FD(self, phi):
        g = self._ghost(phi)
        return self.d * (g[2:] - 2.0 * g[1:-1] + g[:-2]) / self.dx ** 2

    def FR(self, phi):
        return self.r * phi * (phi - 1.0) * (phi - 0.5)

    def solve_D(self, c, rhs, lag):
        # (I - c d Lap) y = rhs + boundary terms of the ghost values
        n = self.nx
        k = c * self.d / self.dx ** 2
        ab = np.zeros((3, n))
        ab[0, 1:] = -k
        ab[1, :] = 1.0 + 2.0 * k
        ab[2, :-1] = -k
        ab[1, 0] += k           # ghost 2 - phi_0
        ab[1, -1] += k          # ghost -phi_{n-1}
        b = rhs.copy()
        b[0] += 2.0 * k
        return sla.solve_banded((1, 1), ab, b)

    def solve_R(self, c, b, guess):
        y = np.array(guess, dtype=np.float64, copy=True)
        for _ in range(100):
            g = y - c * self.FR(y) - b
            dg = 1.0 - c * self.r * (3.0 * y * y - 3.0 * y + 0.5)
            dy = g / dg
            y = y - dy
            if np.max(np.abs(dy)) <= 1e-15:
                break
        return y
