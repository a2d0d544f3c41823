"""Generic SDC step and sweep drivers (oracle; test infrastructure only).

A problem object supplies the three right-hand-side pieces and the implicit
sub-solves used by the schemes of section 3 of the paper:

    FA(phi), FD(phi), FR(phi)    advection, diffusion, reaction terms
    solve_D(c, rhs, lag)         phi - c * FD_lag(phi) = rhs, where FD_lag is the
                                 diffusion operator with its coefficients frozen
                                 at the state ``lag`` (the lagged flux of the
                                 species-update step S3, eq. lagged_diffusion_flux)
    solve_R(c, b, guess)         phi - c * FR(phi) = b (reaction step, S5)
    solve_DR(c, rhs, guess, lag) phi - c * (FD_lag + FR)(phi) = rhs (IMEXQ only)

States are NumPy arrays of any shape; the drivers only add, scale and copy
them.  Every update below is written bracket by bracket in the order the paper
prints it, with no folding of terms.

Schemes
-------
"misdc"   node-to-node MISDC, eqs. update_equation_misdc_discrete_form_D/R,
          with backward-Euler diffusion/reaction and forward-Euler advection
          over each sub-interval and the node-to-node quadrature S^{m:m+1}.
"misdcq"  MISDCQ, eqs. update_equation_misdcq_discrete_form_D/R: Q-form with
          the LU-trick implicit weights Q~I and forward-Euler weights Q~E.
"cisdcq"  CISDCQ-nu, eqs. update_equation_amisdcq_discrete_form_D and
          update_equation_amisdcq_discrete_form_R_alt, with the lag
          initialisation initial_lagged_values_A/D/R and nu nested iterations.
"imexq"   IMEXQ: explicit advection, fully coupled implicit diffusion+reaction
          with the LU-trick weights (the comparison scheme of section 3.2.2).
"""
import numpy as np

from .coefficients import sdc_tables, node_to_node_weights


class _F:
    """Operator values (FA, FD, FR) at one node."""
    __slots__ = ("A", "D", "R")

    def __init__(self, A, D, R):
        self.A, self.D, self.R = A, D, R

    def total(self):
        return self.A + self.D + self.R


def _evalF(prob, phi):
    return _F(prob.FA(phi), prob.FD(phi), prob.FR(phi))


def scheme_tables(n_nodes, scheme, qe="cumulative"):
    return sdc_tables(n_nodes, qi="be" if scheme == "misdc" else "lu", qe=qe)


def sweep_misdc(prob, phi, F, dt, tab, S):
    """One node-to-node MISDC sweep.  phi, F: lists over nodes 0..M (sweep k)."""
    M = tab["M"]
    new_phi = [phi[0]] + [None] * M
    new_F = [F[0]] + [None] * M
    for m in range(M):
        p = m + 1
        dtm = dt * tab["dtau"][m]
        quad = dt * sum(S[m, j] * F[j].total() for j in range(M + 1))
        # phi_AD^{m+1} = phi^{m,(k+1)} + dt^m [FA(phi^{m,(k+1)}) - FA(phi^{m,(k)})
        #                + FD(phi_AD^{m+1}) - FD(phi^{m+1,(k)})] + dt S^{m:m+1} F^{(k)}
        rhs = new_phi[m] + dtm * (new_F[m].A - F[m].A) - dtm * F[p].D + quad
        phi_ad = prob.solve_D(dtm, rhs, phi[p])
        # phi^{m+1} = phi_AD^{m+1} + dt^m [FR(phi^{m+1}) - FR(phi^{m+1,(k)})]
        b = phi_ad - dtm * F[p].R
        new_phi[p] = prob.solve_R(dtm, b, phi[p])
        new_F[p] = _evalF(prob, new_phi[p])
    return new_phi, new_F


def sweep_misdcq(prob, phi, F, dt, tab):
    """One MISDCQ sweep (Q-form, serial diffusion then reaction per node)."""
    M = tab["M"]
    Q, QI, QE = tab["Q"], tab["QI"], tab["QE"]
    phi0 = phi[0]
    new_phi = [phi0] + [None] * M
    new_F = [F[0]] + [None] * M
    for p in range(1, M + 1):
        m = p - 1
        # Q^{0:m+1}(F(phi^{(k)}))
        quad = sum(Q[p - 1, j] * F[j].total() for j in range(M + 1))
        rhs = phi0 + dt * quad
        for j in range(1, m + 1):
            rhs = rhs + dt * QE[p - 1, j - 1] * (new_F[j].A - F[j].A)
        for j in range(1, m + 1):
            rhs = rhs + dt * QI[p - 1, j - 1] * (new_F[j].D - F[j].D)
        c = dt * QI[p - 1, p - 1]
        rhs = rhs - c * F[p].D                       # known half of the implicit bracket
        phi_ad = prob.solve_D(c, rhs, phi[p])
        # reaction update = (MISDCQ-R) - (MISDCQ-D): the reaction brackets
        b = phi_ad
        for j in range(1, m + 1):
            b = b + dt * QI[p - 1, j - 1] * (new_F[j].R - F[j].R)
        b = b - c * F[p].R
        new_phi[p] = prob.solve_R(c, b, phi[p])
        new_F[p] = _evalF(prob, new_phi[p])
    return new_phi, new_F


def relative_change(new, old):
    """max over fields of max_i |new_f - old_f| / max_i |new_f| (fields on the
    first axis; a 0-d or 1-d state is one field).  A field with max |new_f| = 0
    counts 0 if it did not change and infinity otherwise."""
    new = np.asarray(new, dtype=np.float64)
    old = np.asarray(old, dtype=np.float64)
    if new.ndim <= 1:
        new, old = new.reshape(1, -1), old.reshape(1, -1)
    else:
        new, old = new.reshape(new.shape[0], -1), old.reshape(old.shape[0], -1)
    out = 0.0
    for f in range(new.shape[0]):
        d = float(np.max(np.abs(new[f] - old[f])))
        m = float(np.max(np.abs(new[f])))
        r = d / m if m > 0 else (0.0 if d == 0 else np.inf)
        out = max(out, r)
    return out


def sweep_cisdcq(prob, phi, F, dt, tab, nu, nu_tol=None, passes=None, changes=None):
    """One CISDCQ-nu sweep: nu nested iterations over the nodes.

    Buffers: ``prev`` holds the values of nested iteration l (l = 0 is the lag
    initialisation), ``cur`` those of iteration l+1 being computed.  The
    diffusion update at node m+1 uses iteration-(l+1) values at nodes
    j <= m-1 and iteration-l (lagged) values at nodes m and m+1; the reaction
    update is the correction form of eq. ..._R_alt.

    Adaptive nested iterations (``nu_tol``; the paper leaves the rule to
    future work in its sections 4.1-4.3): nu is then the largest number of
    passes.  delta_l = relative_change of the node-M state made by pass l
    (delta_1 against sweep k's values).  After pass l >= 2 the sweep stops
    if delta_l <= nu_tol * delta_1: the nested iteration has stalled
    relative to the sweep's own change.  The number of passes done is
    appended to ``passes``, the list of the sweep's delta_l to ``changes``.
    """
    M = tab["M"]
    Q, QI, QE = tab["Q"], tab["QI"], tab["QE"]
    phi0 = phi[0]
    # S1 / eq. initial_lagged_values_R: iteration-0 state and reaction terms
    # are those of sweep k.
    prev_phi = list(phi)
    prev_F = list(F)
    ad_F = [None] * (M + 1)         # FA, FD at phi_AD^{m,(k+1,1)} (lag init A/D)
    deltas = []
    for ell in range(nu):
        cur_phi = [phi0] + [None] * M
        cur_F = [F[0]] + [None] * M
        for p in range(1, M + 1):
            m = p - 1
            # ---- diffusion step at node m+1, iteration l+1 ----
            quad = sum(Q[p - 1, j] * F[j].total() for j in range(M + 1))
            rhs = phi0 + dt * quad
            for j in range(1, m):        # j = 1..m-1: values of iteration l+1
                rhs = rhs + dt * QE[p - 1, j - 1] * (cur_F[j].A - F[j].A)
            for j in range(1, m):
                rhs = rhs + dt * QI[p - 1, j - 1] * (cur_F[j].D - F[j].D + cur_F[j].R - F[j].R)
            if m >= 1:
                if ell == 0:
                    # eqs. initial_lagged_values_A/D: the most recent AD update at
                    # node m, i.e. phi_AD^{m,(k+1,1)} of this pass
                    lagA, lagD = ad_F[m].A, ad_F[m].D
                else:
                    lagA, lagD = prev_F[m].A, prev_F[m].D
                lagR = prev_F[m].R
                rhs = rhs + dt * QE[p - 1, m - 1] * (lagA - F[m].A)
                rhs = rhs + dt * QI[p - 1, m - 1] * (lagD - F[m].D + lagR - F[m].R)
            c = dt * QI[p - 1, p - 1]
            rhs = rhs + c * (prev_F[p].R - F[p].R) - c * F[p].D
            lag_state = phi[p] if ell == 0 else prev_phi[p]      # eq. lagged_diffusion_flux
            phi_ad = prob.solve_D(c, rhs, lag_state)
            if ell == 0:
                ad_F[p] = _F(prob.FA(phi_ad), prob.FD(phi_ad), None)
            # ---- reaction step at node m+1, iteration l+1 (eq. ..._R_alt) ----
            b = phi_ad
            if m >= 1:
                b = b + dt * QI[p - 1, m - 1] * (cur_F[m].R - prev_F[m].R)
            b = b - c * prev_F[p].R
            cur_phi[p] = prob.solve_R(c, b, prev_phi[p])
            cur_F[p] = _evalF(prob, cur_phi[p])
        done = ell + 1
        stop = False
        if nu_tol is not None:
            delta = relative_change(cur_phi[M], prev_phi[M])
            deltas.append(delta)
            stop = ell >= 1 and delta <= nu_tol * deltas[0]
        prev_phi, prev_F = cur_phi, cur_F
        if stop:
            break
    if passes is not None:
        passes.append(done)
    if changes is not None:
        changes.append(deltas)
    return prev_phi, prev_F          # S7


def sweep_imexq(prob, phi, F, dt, tab):
    """One IMEXQ sweep: explicit advection, coupled implicit diffusion+reaction."""
    M = tab["M"]
    Q, QI, QE = tab["Q"], tab["QI"], tab["QE"]
    phi0 = phi[0]
    new_phi = [phi0] + [None] * M
    new_F = [F[0]] + [None] * M
    for p in range(1, M + 1):
        m = p - 1
        quad = sum(Q[p - 1, j] * F[j].total() for j in range(M + 1))
        rhs = phi0 + dt * quad
        for j in range(1, m + 1):
            rhs = rhs + dt * QE[p - 1, j - 1] * (new_F[j].A - F[j].A)
            rhs = rhs + dt * QI[p - 1, j - 1] * (new_F[j].D - F[j].D + new_F[j].R - F[j].R)
        c = dt * QI[p - 1, p - 1]
        rhs = rhs - c * (F[p].D + F[p].R)
        new_phi[p] = prob.solve_DR(c, rhs, phi[p], phi[p])
        new_F[p] = _evalF(prob, new_phi[p])
    return new_phi, new_F


def sdc_step(prob, phi_n, dt, n_nodes, sweeps, scheme, nu=1, qe="cumulative",
             increments=None, stop_tol=None, norm=None, nu_tol=None, passes=None,
             changes=None, field_increments=None, progress=None):
    """Advance phi_n by one step of size dt.

    I1-I2: node 0 and every node of sweep 0 hold phi^n; I4: the operator values
    at phi^n serve for the first sweep's quadrature.  After each sweep the
    increment |phi^{M,(k+1)} - phi^{M,(k)}| (``norm``, default max-abs) is
    appended to ``increments``, and, for states with a leading field axis,
    the pair (max over cells of |phi^{M,(k+1)} - phi^{M,(k)}|, max over cells
    of |phi^{M,(k+1)}|) of every field to ``field_increments``; ``progress``
    (if given) is called with (sweep index, increment) after each sweep.
    With ``stop_tol`` the step stops at the first sweep whose increment is <=
    stop_tol.  CISDCQ with ``nu_tol`` adapts the number of nested iterations
    of each sweep (see sweep_cisdcq); the passes done per sweep are appended
    to ``passes`` and their changes to ``changes``.  Returns (phi^{n+1},
    sweeps done).
    """
    tab = scheme_tables(n_nodes, scheme, qe)
    S = node_to_node_weights(n_nodes) if scheme == "misdc" else None
    M = tab["M"]
    phi = [np.array(phi_n, dtype=np.float64, copy=True) for _ in range(M + 1)]
    F0 = _evalF(prob, phi[0])
    F = [F0] * (M + 1)
    norm = norm or (lambda x: float(np.max(np.abs(x))))
    done = 0
    for _k in range(sweeps):
        if scheme == "misdc":
            new_phi, new_F = sweep_misdc(prob, phi, F, dt, tab, S)
        elif scheme == "misdcq":
            new_phi, new_F = sweep_misdcq(prob, phi, F, dt, tab)
        elif scheme == "cisdcq":
            new_phi, new_F = sweep_cisdcq(prob, phi, F, dt, tab, nu, nu_tol, passes, changes)
        elif scheme == "imexq":
            new_phi, new_F = sweep_imexq(prob, phi, F, dt, tab)
        else:
            raise ValueError(scheme)
        inc = norm(new_phi[M] - phi[M])
        if increments is not None:
            increments.append(inc)
        if field_increments is not None:
            nf = new_phi[M].shape[0]
            diff = np.abs(new_phi[M] - phi[M]).reshape(nf, -1).max(axis=1)
            mag = np.abs(new_phi[M]).reshape(nf, -1).max(axis=1)
            field_increments.append(np.stack([diff, mag], axis=1))
        if progress is not None:
            progress(done, inc)
        phi, F = new_phi, new_F
        done += 1
        if stop_tol is not None and inc <= stop_tol:
            break
    return phi[M], done
