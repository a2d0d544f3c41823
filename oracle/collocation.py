"""Brute-force collocation solution (oracle; test infrastructure only).

The fixed point of every sweep of section 3 is the collocation solution on the
M+1 Gauss-Lobatto nodes: with Phi = (phi^1, ..., phi^M),
    phi^p = phi^n + dt * sum_{j=0}^{M} q_{p,j} F(phi^j),   phi^0 = phi^n,
i.e. Phi = 1 (x) phi^n + dt (q (x) F(phi^n) + (Q~ (x) I) F(Phi)).
Here that nonlinear system is solved as a whole by Newton's method with a
dense Jacobian obtained by complex-step differentiation of F, which is exact
to rounding for analytic F.  No sweep and no operator splitting is involved,
so the result checks the sweeps independently.
"""
import numpy as np

from .coefficients import sdc_tables


def _F(prob, phi):
    return prob.FA(phi) + prob.FD(phi) + prob.FR(phi)


def collocation_solve(prob, phi_n, dt, n_nodes, tol=1e-14, maxit=50, h=1e-30):
    tab = sdc_tables(n_nodes)
    M = tab["M"]
    q0, Qt = tab["q0"], tab["Qt"]
    shape = phi_n.shape
    n = phi_n.size
    Fn = _F(prob, phi_n)
    const = np.concatenate([(phi_n + dt * q0[p] * Fn).ravel() for p in range(M)])

    def residual(X):
        nodes = [X[p * n:(p + 1) * n].reshape(shape) for p in range(M)]
        Fs = [_F(prob, x).ravel() for x in nodes]
        out = X - const
        for p in range(M):
            acc = 0.0
            for j in range(M):
                acc = acc + Qt[p, j] * Fs[j]
            out[p * n:(p + 1) * n] = out[p * n:(p + 1) * n] - dt * acc
        return out

    X = np.concatenate([phi_n.ravel()] * M).astype(np.float64)
    scale = np.concatenate([np.full(n, 1.0)] * M)
    for _ in range(maxit):
        G = residual(X.astype(np.complex128)).real
        J = np.empty((X.size, X.size))
        for i in range(X.size):
            Xc = X.astype(np.complex128)
            step = h * max(1.0, abs(X[i]))
            Xc[i] += 1j * step
            J[:, i] = residual(Xc).imag / step
        d = np.linalg.solve(J, G)
        X = X - d
        if np.max(np.abs(d) / np.maximum(np.abs(X), scale)) <= tol:
            break
    return [phi_n] + [X[p * n:(p + 1) * n].reshape(shape) for p in range(M)]
