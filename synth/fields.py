"""Seeded initial fields and test batches (data only).

Fields are returned as mass fractions ``Y`` (species first, cells last, x
fastest) and temperature ``T`` in K.  Converting (Y, T) into the transported
enthalpy is left to each consumer, since that conversion is part of the
model's thermodynamics.
"""
import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _tanh_profile(x, L, delta, shift_lo=0.0, shift_hi=0.0):
    """Periodic hot slab: 300 K outside, 2000 K between x = L/4 and 3L/4."""
    return 300.0 + 850.0 * (np.tanh((x - (0.25 * L + shift_lo)) / delta)
                            - np.tanh((x - (0.75 * L + shift_hi)) / delta))


def _compose(mech, T):
    w = (T - 300.0) / 1700.0
    w = np.clip(w, 0.0, 1.0)
    Y = (1.0 - w)[None] * mech["Y_cold"].reshape((-1,) + (1,) * T.ndim) \
        + w[None] * mech["Y_hot"].reshape((-1,) + (1,) * T.ndim)
    return Y


def flame_1d(mech, n=64, dx=0.01):
    """Periodic 1-D flame: two tanh fronts, 300 K -> 2000 K, width
    max(L/32, 4 dx)."""
    L = n * dx
    x = (np.arange(n) + 0.5) * dx
    T = _tanh_profile(x, L, max(L / 32.0, 4.0 * dx))
    return _compose(mech, T), T


def flame_2d(mech, nx=256, ny=256, dx=0.01, dy=0.01, seed=None):
    """Periodic 2-D flame: the 1-D slab along x with fronts displaced by
    0.05 L sin(2 pi y / L_y), so the problem is genuinely two-dimensional.
    With a seed, each front gets its own displacement: amplitudes in
    [0.02, 0.08] L of the first two modes with random phases."""
    Lx = nx * dx
    Ly = ny * dy
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Yg = np.meshgrid(x, y)            # (ny, nx), x fastest
    if seed is None:
        s_lo = 0.05 * Lx * np.sin(2.0 * np.pi * Yg / Ly)
        s_hi = -s_lo
    else:
        rng = _rng(seed)
        shifts = []
        for _ in range(2):
            a = rng.uniform(0.02, 0.08, 2) * Lx
            ph = rng.uniform(0.0, 2.0 * np.pi, 2)
            shifts.append(a[0] * np.sin(2.0 * np.pi * Yg / Ly + ph[0])
                          + a[1] * np.sin(4.0 * np.pi * Yg / Ly + ph[1]))
        s_lo, s_hi = shifts
    T = _tanh_profile(X, Lx, max(Lx / 32.0, 4.0 * dx), s_lo, s_hi)
    return _compose(mech, T), T


def ensemble_flames(mech, n_flames=64, len_range=(128, 4096), dt_base=5e-6,
                    dt_spread=10.0, dx=0.01, seed=5):
    """Independent periodic 1-D flames of uneven length and step size."""
    rng = _rng(seed)
    lengths = rng.integers(len_range[0], len_range[1] + 1, size=n_flames)
    dts = dt_base * dt_spread ** rng.uniform(0.0, 1.0, size=n_flames)
    flames = [flame_1d(mech, int(n), dx) for n in lengths]
    return lengths.astype(np.int64), dts, flames


def random_cell_batch(mech, n, seed=0, c_range=(1e-7, 1e-4), T_range=(300.0, 2200.0),
                      perturb=0.05):
    """Random per-cell reaction problems.

    Returns ``Yb`` (N, n) mass fractions of the right-hand side, ``Tb`` (n) the
    temperature that fixes the cell enthalpy, ``c`` (n) the implicit weight
    (dt times the diagonal quadrature weight), and a guess ``Yg`` (N, n) that is
    a perturbed copy of ``Yb`` with the same sum.
    """
    rng = _rng(seed)
    N = mech["N"]
    w = rng.uniform(0.0, 1.0, n)
    Yb = (1.0 - w)[None] * mech["Y_cold"][:, None] + w[None] * mech["Y_hot"][:, None]
    mix = rng.dirichlet(np.ones(N - 1), size=n).T * 0.3      # (N-1, n)
    lam = rng.uniform(0.0, 0.5, n)
    Yb[:N - 1] = (1.0 - lam)[None] * Yb[:N - 1] + lam[None] * mix
    Tb = rng.uniform(T_range[0], T_range[1], n)
    c = 10.0 ** rng.uniform(np.log10(c_range[0]), np.log10(c_range[1]), n)
    g = 1.0 + perturb * rng.uniform(-1.0, 1.0, (N - 1, n))
    Yg = Yb.copy()
    Yg[:N - 1] *= g
    Yg[N - 1] = 1.0 - Yg[:N - 1].sum(axis=0)
    return Yb, Tb, c, Yg


def random_helmholtz_problem(shape, n_fields, seed=0):
    """A smooth positive temperature field and random right-hand sides."""
    rng = _rng(seed)
    grids = np.meshgrid(*[np.arange(s) / s for s in shape], indexing="ij")
    T = 1100.0 + 700.0 * np.prod([np.sin(2 * np.pi * (g + rng.uniform())) for g in grids], axis=0)
    rhs = rng.standard_normal((n_fields,) + tuple(shape))
    return T, rhs
