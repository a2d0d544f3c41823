"""Periodic finite-volume transport operators (oracle; test infrastructure only).

Grid: uniform, periodic, 1-D (n,) or 2-D (ny, nx) with x fastest.  A state is
an array (n_fields, *grid).

Advection (eq. species_equation/enthalpy_equation, the -div(U phi) term, with a
prescribed uniform velocity): FA = -u_x d(phi)/dx - u_y d(phi)/dy in flux
form, with the fourth-order face value
    phi_{i+1/2} = (7 (phi_i + phi_{i+1}) - (phi_{i-1} + phi_{i+2})) / 12.

Diffusion, second-order flux form: for a field with diffusivity kappa_f(T),
    FD_i = [K_{i+1/2} (phi_{i+1} - phi_i) - K_{i-1/2} (phi_i - phi_{i-1})] / dx^2
(plus the y terms), with the face coefficient the arithmetic mean of the two
cell values.  Species and enthalpy use kappa = D0_k (T/300)^1.7 and
alpha0 (T/300)^1.7.  The dominant species i0 carries minus the sum of the
other species' diffusion terms (the closure of section 2).

Implicit diffusion (steps S3/S4): for every diffused field, the linear system
(I - c L_f) y = r with L_f the diffusion operator whose coefficients come from
a lagged state, solved here with a sparse direct solver (SuperLU), the
paper's "direct solver"; the dominant species then follows from the closure
y_i0 = r_i0 - sum_{k != i0} (y_k - r_k).  The matrices are symmetric, so the
LU takes the minimum-degree column order of A^T + A (less fill than the
default on 2-D grids); the fields' systems are independent and are solved
concurrently.  Both only change the rounding of an exact solve.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

THETA_EXP = 1.7
T_DIFF_REF = 300.0


def theta(T):
    """Temperature factor (T/300)^1.7 of every diffusivity."""
    return (T / T_DIFF_REF) ** THETA_EXP


def _face_value(phi, axis):
    """Fourth-order value at the face i+1/2 along ``axis`` (periodic)."""
    return (7.0 * (phi + np.roll(phi, -1, axis)) - (np.roll(phi, 1, axis) + np.roll(phi, -2, axis))) / 12.0


def advection(phi, u, dx):
    """FA for every field; phi (nf, *grid), u and dx per grid axis (x first)."""
    out = np.zeros_like(phi)
    ndim = phi.ndim - 1
    for d in range(ndim):
        axis = phi.ndim - 1 - d          # x is the last axis
        if u[d] == 0.0:
            continue
        f = _face_value(phi, axis)
        out -= u[d] * (f - np.roll(f, 1, axis)) / dx[d]
    return out


def laplacian_theta(phi, th, dx):
    """div(theta grad phi) for every field (2nd order, face mean of theta)."""
    out = np.zeros_like(phi)
    ndim = th.ndim
    for d in range(ndim):
        axis_f = phi.ndim - 1 - d
        axis_t = th.ndim - 1 - d
        K = 0.5 * (th + np.roll(th, -1, axis_t))          # face i+1/2
        flux = K[None] * (np.roll(phi, -1, axis_f) - phi)
        out += (flux - np.roll(flux, 1, axis_f)) / dx[d] ** 2
    return out


def diffusion_coefficients(mech):
    """kappa0 per field: D0 of every species, then alpha0 for the enthalpy."""
    return np.concatenate([mech["D0"], [mech["alpha0"]]])


def diffusion(mech, phi, T, dx):
    """FD for all N+1 fields with coefficients from temperature T."""
    i0 = mech["bath"]
    k0 = diffusion_coefficients(mech)
    L = laplacian_theta(phi, theta(T), dx)
    out = k0.reshape((-1,) + (1,) * T.ndim) * L
    others = [k for k in range(mech["N"]) if k != i0]
    out[i0] = -out[others].sum(axis=0)
    return out


def laplacian_matrix(th, dx):
    """Sparse matrix of phi -> div(theta grad phi) on the periodic grid."""
    shape = th.shape
    n = th.size
    idx = np.arange(n).reshape(shape)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for d in range(th.ndim):
        axis = th.ndim - 1 - d
        K = 0.5 * (th + np.roll(th, -1, axis)) / dx[d] ** 2      # face i+1/2
        Km = np.roll(K, 1, axis)                                  # face i-1/2
        nb_p = np.roll(idx, -1, axis)
        nb_m = np.roll(idx, 1, axis)
        rows += [idx.ravel(), idx.ravel()]
        cols += [nb_p.ravel(), nb_m.ravel()]
        vals += [K.ravel(), Km.ravel()]
        diag -= (K + Km).ravel()
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def helmholtz_solve(th, kappa0, c, rhs, dx, L=None):
    """Solve (I - c kappa0 L_theta) y = rhs for one field by sparse LU."""
    if L is None:
        L = laplacian_matrix(th, dx)
    A = sp.identity(th.size, format="csc") - (c * kappa0) * L
    return spla.spsolve(A, rhs.ravel(), permc_spec="MMD_AT_PLUS_A").reshape(th.shape)


SOLVE_THREADS = max(1, min(16, os.cpu_count() or 1))


def diffusion_solve(mech, c, rhs, T_lag, dx):
    """Implicit diffusion step for all N+1 fields, coefficients from T_lag."""
    i0 = mech["bath"]
    k0 = diffusion_coefficients(mech)
    th = theta(T_lag)
    L = laplacian_matrix(th, dx)
    y = np.empty_like(rhs)
    fields = [f for f in range(rhs.shape[0]) if f != i0]

    def one(f):
        y[f] = helmholtz_solve(th, k0[f], c, rhs[f], dx, L)

    if len(fields) > 1 and th.size >= 4096 and SOLVE_THREADS > 1:
        with ThreadPoolExecutor(min(SOLVE_THREADS, len(fields))) as ex:
            list(ex.map(one, fields))
    else:
        for f in fields:
            one(f)
    others = [k for k in range(mech["N"]) if k != i0]
    y[i0] = rhs[i0] - np.sum(y[others] - rhs[others], axis=0)
    return y
