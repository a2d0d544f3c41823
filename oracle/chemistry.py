"""Chemistry of the flame problem (oracle; test infrastructure only).

Species equation source term (eq. species_equation): the production rates
omega_i of mass-action kinetics with reversible reactions.  For reaction j,
    q_j = kf_j prod_reactants [X] - kr_j prod_products [X],
    kf_j = A_j T^beta_j exp(-Ea_j / (R_c T)),   kr_j = kf_j / Kc_j,
    Kc_j = exp(-sum_k nu_kj g_k(T) / (R_u T)) (p_atm / (R_u T))^(sum_k nu_kj),
with g_k = h_k - T s_k, h_k(T) = hf_k + cp_k (T - 298.15),
s_k(T) = s0_k + cp_k ln(T / 298.15) (constant heat capacities), and
[X_k] = rho0 Y_k / W_k.  The mass-fraction source is FR_k = W_k omega_k / rho0;
the enthalpy has no reaction source because h includes the formation
enthalpies (section 2).

Enthalpy per unit mass h = sum_k Y_k hhat_k(T), hhat_k = h_k(T) / W_k, which
with constant cp gives T in closed form from (Y, h).

Reaction step S5 (eq. reaction_step_numerical_methodology): with the density
constant, the backward-Euler system for the mass fractions is
    Y - c * FR(Y, T) = bY,   sum_k Y_k hhat_k(T) = h,
solved by Newton's method on x = (Y_1..Y_N, T) with the analytic Jacobian.
Arrays are (species, cells); everything is FP64 and vectorised over cells.
"""
import numpy as np

T_REF = 298.15


def _stoich(mech):
    """Reactant and product stoichiometric matrices nu' (N, R), nu'' (N, R)."""
    N, R = mech["N"], mech["R"]
    nu_f = np.zeros((N, R))
    nu_r = np.zeros((N, R))
    for j in range(R):
        for s in mech["react"][j]:
            if s >= 0:
                nu_f[s, j] += 1.0
        for s in mech["prod"][j]:
            if s >= 0:
                nu_r[s, j] += 1.0
    return nu_f, nu_r


def species_enthalpy(mech, T):
    """Molar h_k(T) (N, n) in erg/mol."""
    return mech["hf"][:, None] + mech["cp"][:, None] * (T[None] - T_REF)


def enthalpy(mech, Y, T):
    """Mixture enthalpy per unit mass, h = sum_k Y_k h_k(T) / W_k."""
    return np.sum(Y * species_enthalpy(mech, T) / mech["W"][:, None], axis=0)


def temperature(mech, Y, h):
    """Closed-form inverse of ``enthalpy`` for constant heat capacities."""
    W = mech["W"][:, None]
    h_form = np.sum(Y * mech["hf"][:, None] / W, axis=0)
    cp_mix = np.sum(Y * mech["cp"][:, None] / W, axis=0)
    return T_REF + (h - h_form) / cp_mix


def rate_constants(mech, T):
    """kf, kr (R, n) and d ln kf/dT, d ln kr/dT."""
    nu_f, nu_r = _stoich(mech)
    nu = nu_r - nu_f                                           # net (N, R)
    Ru, Rc, patm = mech["R_u"], mech["R_c"], mech["p_atm"]
    A, beta, Ea = (mech[k][:, None] for k in ("A", "beta", "Ea"))
    lnT = np.log(T)[None]
    kf = A * np.exp(beta * lnT - Ea / (Rc * T[None]))
    hk = species_enthalpy(mech, T)                             # (N, n)
    sk = mech["s0"][:, None] + mech["cp"][:, None] * np.log(T[None] / T_REF)
    gk = hk - T[None] * sk
    dG = nu.T @ gk                                             # (R, n)
    dn = nu.sum(axis=0)[:, None]                               # (R, 1)
    lnKc = -dG / (Ru * T[None]) + dn * np.log(patm / (Ru * T[None]))
    kr = kf * np.exp(-lnKc)
    dlnkf = beta / T[None] + Ea / (Rc * T[None] ** 2)
    # van 't Hoff: d ln Kc / dT = sum_k nu_kj h_k / (R_u T^2) - dn / T
    dlnKc = (nu.T @ hk) / (Ru * T[None] ** 2) - dn / T[None]
    dlnkr = dlnkf - dlnKc
    return kf, kr, dlnkf, dlnkr


def rates_of_progress(mech, Y, T):
    """q (R, n), together with the forward/reverse products and kf, kr."""
    nu_f, nu_r = _stoich(mech)
    X = mech["rho0"] * Y / mech["W"][:, None]                  # mol/cm^3
    kf, kr, dlnkf, dlnkr = rate_constants(mech, T)
    R = mech["R"]
    n = Y.shape[1]
    dtype = np.result_type(Y, T, np.float64)     # complex inputs stay complex
    pf = np.ones((R, n), dtype=dtype)
    pr = np.ones((R, n), dtype=dtype)
    for j in range(R):
        for s in mech["react"][j]:
            if s >= 0:
                pf[j] = pf[j] * X[s]
        for s in mech["prod"][j]:
            if s >= 0:
                pr[j] = pr[j] * X[s]
    q = kf * pf - kr * pr
    return q, kf, kr, pf, pr, dlnkf, dlnkr, X


def production_rates(mech, Y, T):
    """omega (N, n) in mol/cm^3/s."""
    nu_f, nu_r = _stoich(mech)
    q = rates_of_progress(mech, Y, T)[0]
    return (nu_r - nu_f) @ q


def reaction_source(mech, Y, T):
    """FR_k = W_k omega_k / rho0 (N, n), in 1/s."""
    return mech["W"][:, None] * production_rates(mech, Y, T) / mech["rho0"]


def reaction_source_jacobian(mech, Y, T):
    """dFR/dY (N, N, n) and dFR/dT (N, n), analytic."""
    nu_f, nu_r = _stoich(mech)
    nu = nu_r - nu_f
    W = mech["W"]
    rho0 = mech["rho0"]
    q, kf, kr, pf, pr, dlnkf, dlnkr, X = rates_of_progress(mech, Y, T)
    N, R = mech["N"], mech["R"]
    n = Y.shape[1]
    dq_dX = np.zeros((R, N, n), dtype=np.result_type(Y, T, np.float64))
    for j in range(R):
        for side, k, prod in ((mech["react"][j], kf[j], 1.0), (mech["prod"][j], kr[j], -1.0)):
            slots = [s for s in side if s >= 0]
            for a, s in enumerate(slots):
                other = np.ones(n, dtype=dq_dX.dtype)
                for b, t in enumerate(slots):
                    if b != a:
                        other = other * X[t]
                dq_dX[j, s] += prod * k * other
    dq_dT = kf * dlnkf * pf - kr * dlnkr * pr                  # (R, n)
    # dFR_k/dY_l = W_k/rho0 sum_j nu_kj dq_j/dX_l * rho0/W_l
    dFR_dY = np.einsum("kj,jln->kln", nu, dq_dX) * (W[:, None, None] / W[None, :, None])
    dFR_dT = (W[:, None] / rho0) * (nu @ dq_dT)
    return dFR_dY, dFR_dT


def newton_scale(mech):
    """Constant that converts the enthalpy residual (erg/g) to kelvin."""
    return float(np.mean(mech["cp"] / mech["W"]))


def be_residual(mech, c, bY, h, Y, T):
    """G(x) = [Y - c FR(Y, T) - bY ; (sum_k Y_k hhat_k(T) - h) / scale]."""
    GY = Y - c[None] * reaction_source(mech, Y, T) - bY
    GT = (enthalpy(mech, Y, T) - h) / newton_scale(mech)
    return np.concatenate([GY, GT[None]], axis=0)


def be_jacobian(mech, c, Y, T):
    """dG/dx (n, N+1, N+1) for x = (Y, T)."""
    N = mech["N"]
    n = Y.shape[1]
    dY, dT = reaction_source_jacobian(mech, Y, T)
    J = np.zeros((n, N + 1, N + 1), dtype=np.result_type(Y, T, np.float64))
    J[:, :N, :N] = np.eye(N)[None] - c[:, None, None] * np.moveaxis(dY, 2, 0)
    J[:, :N, N] = -(c[None] * dT).T
    s = newton_scale(mech)
    J[:, N, :N] = (species_enthalpy(mech, T) / mech["W"][:, None]).T / s
    J[:, N, N] = np.sum(Y * mech["cp"][:, None] / mech["W"][:, None], axis=0) / s
    return J


def reaction_solve(mech, c, bY, h, Yguess, tol=1e-12, maxit=200, dtau0=1.0,
                   dtau_max=1e10, neg_slack=1e-6):
    """Backward-Euler reaction step S5: solve G(x) = 0 for x = (Y, T) in every
    cell, by Newton's method with the analytic Jacobian, globalised by
    pseudo-transient continuation (the paper does not say how its Newton
    solver is safeguarded; this is the reading used on both sides).

    Per cell, starting from x0 = (Yguess, T(Yguess, h)) with pseudo-step
    dtau = infinity (plain Newton):
      * solve (J(x) + I/dtau) delta = G(x) by LU with partial pivoting
        (LAPACK here); every such solve counts as one iteration;
      * the trial x - delta is rejected if it is not finite, if T <= 0, or if
        some Y_k falls below min(bY_k, 0) - neg_slack; then dtau <- dtau0 if it
        was infinite, else dtau / 4, and x is kept;
      * otherwise x <- x - delta and, if dtau is finite,
        dtau <- dtau * max(2, |G_old| / |G|), becoming infinite above dtau_max;
      * converged when a plain Newton step (dtau infinite) was accepted with
        max_k |delta_Yk| <= tol and |delta_T| <= tol * T.
    Returns (Y, T, iters); iters = -1 marks a cell that did not converge in
    ``maxit`` solves.
    """
    N = mech["N"]
    Y = np.array(Yguess, dtype=np.float64, copy=True)
    n = Y.shape[1]
    T = temperature(mech, Y, h)
    floor = np.minimum(bY, 0.0) - neg_slack
    inv_dtau = np.zeros(n)                     # 1/dtau; 0 means plain Newton
    gnorm_old = np.full(n, np.nan)
    iters = np.zeros(n, dtype=np.int64)
    active = np.ones(n, dtype=bool)
    eye = np.eye(N + 1)
    for _it in range(maxit):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        Ya, Ta = Y[:, idx], T[idx]
        G = be_residual(mech, c[idx], bY[:, idx], h[idx], Ya, Ta)
        J = be_jacobian(mech, c[idx], Ya, Ta) + inv_dtau[idx, None, None] * eye[None]
        iters[idx] += 1
        with np.errstate(all="ignore"):
            try:
                delta = np.linalg.solve(J, G.T[:, :, None])[:, :, 0].T
            except np.linalg.LinAlgError:
                delta = np.full((N + 1, idx.size), np.nan)
                for q in range(idx.size):
                    try:
                        delta[:, q] = np.linalg.solve(J[q], G[:, q])
                    except np.linalg.LinAlgError:
                        pass
            Yt = Ya - delta[:N]
            Tt = Ta - delta[N]
            ok = (np.all(np.isfinite(delta), axis=0) & (Tt > 0.0)
                  & np.all(Yt >= floor[:, idx], axis=0))
        # rejected trial: shrink the pseudo-step, keep x
        rej = idx[~ok]
        inv_dtau[rej] = np.where(inv_dtau[rej] == 0.0, 1.0 / dtau0, inv_dtau[rej] * 4.0)
        # accepted trial
        acc = idx[ok]
        was_newton = inv_dtau[acc] == 0.0
        Y[:, acc] = Yt[:, ok]
        T[acc] = Tt[ok]
        gnorm = np.sqrt(np.sum(G[:, ok] ** 2, axis=0))
        ptc = ~was_newton
        grow = np.maximum(2.0, np.where(np.isfinite(gnorm_old[acc]) & (gnorm > 0),
                                        gnorm_old[acc] / np.where(gnorm > 0, gnorm, 1.0), 2.0))
        new_inv = inv_dtau[acc] / grow
        new_inv = np.where(new_inv < 1.0 / dtau_max, 0.0, new_inv)
        inv_dtau[acc] = np.where(ptc, new_inv, 0.0)
        gnorm_old[acc] = gnorm
        d = delta[:, ok]
        conv = was_newton & (np.max(np.abs(d[:N]), axis=0) <= tol) & (np.abs(d[N]) <= tol * Tt[ok])
        active[acc[conv]] = False
    iters[active] = -1
    return Y, T, iters
