"""Seeded synthetic reaction mechanisms (data only).

A mechanism is a dict of plain NumPy arrays in CGS units:

* ``N`` species, the last one (index ``bath``) an inert bath gas made of the
  fourth element only; it is the dominant species of the diffusion closure.
* ``R`` reversible reactions with at most two reactants and two products,
  stored as index slots ``react``/``prod`` of shape (R, 2) holding a species
  index or -1 (a repeated index means a stoichiometric coefficient of 2).
  Every reaction is element-balanced, hence mass-balanced.
* Arrhenius parameters ``A`` (CGS, (cm^3/mol)^(n-1)/s), ``beta`` and ``Ea``
  (cal/mol).
* Constant molar heat capacities ``cp`` (erg/mol/K), formation enthalpies
  ``hf`` (erg/mol at 298.15 K) and standard entropies ``s0`` (erg/mol/K at
  298.15 K and 1 atm).
* Diffusivities ``D0`` (cm^2/s at 300 K, one per species) and the enthalpy
  diffusivity ``alpha0`` (cm^2/s at 300 K); both scale as (T/300)^1.7.
* Reference cold and hot compositions ``Y_cold``/``Y_hot`` used by the field
  generators, and a constant density ``rho0`` (g/cm^3) taken as the ideal-gas
  density of the cold composition at 1 atm and 1000 K.

The paper's flame uses a detailed dimethyl-ether mechanism whose data is not
available here; these seeded mechanisms stand in for it with the species and
reaction counts of the workloads (9/21 and 53/325).
"""
import itertools

import numpy as np

R_U = 8.31446261815324e7       # erg / (mol K)
R_CAL = 1.98720425864083       # cal / (mol K)
P_ATM = 1.01325e6              # dyn / cm^2
ERG_PER_CAL = 4.184e7
ELEMENT_MASSES = np.array([1.008, 12.011, 15.999, 14.007])  # H-, C-, O-, N-like


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _candidate_reactions(comps):
    """All element-balanced reactions among species with compositions ``comps``.

    Sides are multisets of one or two species; the two sides must share no
    species and have equal element totals.  Returns a list of (lhs, rhs) tuples
    of sorted species-index tuples, each unordered pair listed once.
    """
    n = len(comps)
    sides = [(i,) for i in range(n)] + list(itertools.combinations_with_replacement(range(n), 2))
    groups = {}
    for s in sides:
        key = tuple(int(v) for v in np.sum([comps[i] for i in s], axis=0))
        groups.setdefault(key, []).append(s)
    cands = []
    for members in groups.values():
        for a, b in itertools.combinations(members, 2):
            if set(a) & set(b):
                continue
            cands.append((a, b))
    return cands


def _draw_compositions(rng, n_reactive, lattice):
    """Draw distinct compositions: a few small base species, then sums of two."""
    hmax, cmax, omax = lattice
    comps = []
    seen = set()
    n_base = min(max(3, n_reactive // 3), 8)
    while len(comps) < n_base:
        c = (int(rng.integers(0, 3)), int(rng.integers(0, 2)), int(rng.integers(0, 2)))
        if c != (0, 0, 0) and c not in seen:
            seen.add(c)
            comps.append(c)
    tries = 0
    while len(comps) < n_reactive:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not draw compositions")
        i, j = rng.integers(0, len(comps), size=2)
        c = tuple(a + b for a, b in zip(comps[i], comps[j]))
        if rng.random() < 0.3:  # occasionally a fresh small species
            c = (int(rng.integers(0, hmax + 1)), int(rng.integers(0, cmax + 1)),
                 int(rng.integers(0, omax + 1)))
        if c == (0, 0, 0) or c in seen:
            continue
        if c[0] > hmax or c[1] > cmax or c[2] > omax:
            continue
        seen.add(c)
        comps.append(c)
    return [np.array(c + (0,), dtype=np.int64) for c in comps]


def make_mechanism(n_species=9, n_reactions=21, seed=0, rate_spread=None,
                   A_range=(1e8, 1e16), beta_range=(-1.0, 1.0),
                   Ea_range_kcal=(0.0, 50.0), hf_range_kcal=(-30.0, 30.0),
                   dh_species_kcal=1.0, s0_base_cal=30.0, ds_species_cal=5.0,
                   cp_range=(3.5, 8.0),
                   D0_range=(0.1, 0.4), alpha0=0.2):
    """Seeded synthetic mechanism.

    ``rate_spread=(lo, hi)`` rescales every pre-exponential factor so that the
    effective first-order rate constant of the forward reaction at 1500 K and
    the 1-atm reference concentration is log-uniform in [lo, hi] (1/s).
    """
    rng = _rng(seed)
    n_reactive = n_species - 1
    lattice = (4, 2, 2) if n_reactive <= 12 else (8, 3, 4)
    for _attempt in range(1000):
        comps = _draw_compositions(rng, n_reactive, lattice)
        cands = _candidate_reactions(comps)
        covered = set(i for a, b in cands for i in a + b)
        if len(cands) >= n_reactions and len(covered) == n_reactive:
            break
    else:
        raise RuntimeError("no mechanism with enough balanced reactions")
    # pick reactions: first one per species (coverage), then random fill
    chosen = []
    order = rng.permutation(len(cands))
    used = set()
    for sp in rng.permutation(n_reactive):
        if any(sp in a + b for a, b in (cands[k] for k in chosen)):
            continue
        for k in order:
            if k not in used and sp in cands[k][0] + cands[k][1]:
                chosen.append(int(k))
                used.add(int(k))
                break
    for k in order:
        if len(chosen) >= n_reactions:
            break
        if int(k) not in used:
            chosen.append(int(k))
            used.add(int(k))
    chosen = chosen[:n_reactions]
    react = -np.ones((n_reactions, 2), dtype=np.int32)
    prod = -np.ones((n_reactions, 2), dtype=np.int32)
    for r, k in enumerate(chosen):
        a, b = cands[k]
        if rng.random() < 0.5:
            a, b = b, a
        react[r, :len(a)] = a
        prod[r, :len(b)] = b

    comp = np.zeros((4, n_species), dtype=np.int64)
    for i, c in enumerate(comps):
        comp[:, i] = c
    comp[3, n_species - 1] = 2                    # bath: N2-like
    W = ELEMENT_MASSES @ comp

    A = 10.0 ** rng.uniform(np.log10(A_range[0]), np.log10(A_range[1]), n_reactions)
    beta = rng.uniform(beta_range[0], beta_range[1], n_reactions)
    Ea = 1e3 * rng.uniform(Ea_range_kcal[0], Ea_range_kcal[1], n_reactions)   # cal/mol
    if rate_spread is not None:
        T_ref = 1500.0
        c_ref = P_ATM / (R_U * T_ref)
        order_f = (react >= 0).sum(axis=1)
        target = 10.0 ** rng.uniform(np.log10(rate_spread[0]), np.log10(rate_spread[1]), n_reactions)
        base = T_ref ** beta * np.exp(-Ea / (R_CAL * T_ref)) * c_ref ** (order_f - 1)
        A = target / base

    # Formation enthalpy and entropy = per-element contribution (cancels in
    # every balanced reaction) + a per-species part, so reaction enthalpies
    # stay within a few tens of kcal/mol and entropies of association near
    # -30 cal/mol/K, as for real gases.
    cp = rng.uniform(cp_range[0], cp_range[1], n_species) * R_U
    h_elem = rng.uniform(hf_range_kcal[0], hf_range_kcal[1], 4)
    hf = (h_elem @ comp + rng.uniform(-dh_species_kcal, dh_species_kcal, n_species))
    hf = hf * 1e3 * ERG_PER_CAL
    s_elem = rng.uniform(0.0, 10.0, 4)
    s0 = (s0_base_cal + s_elem @ comp + rng.uniform(-ds_species_cal, ds_species_cal, n_species))
    s0 = s0 * ERG_PER_CAL
    cp[-1] = 3.5 * R_U
    hf[-1] = 0.0
    s0[-1] = 45.77 * ERG_PER_CAL
    D0 = rng.uniform(D0_range[0], D0_range[1], n_species)

    def dirichlet_reactive():
        w = rng.dirichlet(np.ones(n_reactive))
        y = np.zeros(n_species)
        y[:n_reactive] = 0.3 * w
        y[-1] = 0.7
        return y

    Y_cold = dirichlet_reactive()
    Y_hot = dirichlet_reactive()
    Wbar_cold = 1.0 / np.sum(Y_cold / W)
    rho0 = P_ATM * Wbar_cold / (R_U * 1000.0)

    return dict(
        N=int(n_species), R=int(n_reactions), bath=int(n_species - 1),
        comp=comp, W=W.astype(np.float64), react=react, prod=prod,
        A=A, beta=beta, Ea=Ea, cp=cp, hf=hf, s0=s0, D0=D0, alpha0=float(alpha0),
        rho0=float(rho0), p_atm=P_ATM, R_u=R_U, R_c=R_CAL,
        Y_cold=Y_cold, Y_hot=Y_hot, seed=int(seed),
    )


def mlp_init(sizes, seed=7):
    """Initial weights of a dense network with layer widths ``sizes``:
    uniform in +-sqrt(6 / fan_in) (He), zero biases, float32 values.  Data
    only: list of (W (fan_in, fan_out), b)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / a)
        W = rng.uniform(-lim, lim, (a, b)).astype(np.float32).astype(np.float64)
        params.append((W, np.zeros(b)))
    return params
