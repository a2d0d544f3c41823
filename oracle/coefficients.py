"""SDC coefficient tables (oracle; test infrastructure only).

Section 3.1 of the paper: M+1 Gauss-Lobatto nodes on [t^n, t^n + dt], the
integration matrix Q with entries q_{m+1,j} = (1/dt) * integral from t^0 to
t^{m+1} of the Lagrange polynomial L_j (eq. "weights"), its first column q and
remaining block Q~, the implicit weights Q~I = transpose of the upper factor of
the LU decomposition of transpose(Q~) (Weiser's choice), and the explicit
forward-Euler weights Q~E.

Everything is computed in 50-digit arithmetic with mpmath and rounded to FP64
once, so the FP64 tables are correctly rounded.

Index convention: rows p = 1..M are stored at row p-1.  Q has M+1 columns
(j = 0..M); Q~, Q~I and Q~E have M columns for j = 1..M stored at column j-1.
All weights are divided by dt (dimensionless).
"""
import mpmath as mp
import numpy as np

_DPS = 50


def lobatto_nodes_mp(n_nodes):
    """Gauss-Lobatto nodes on [0, 1]: the end points and the roots of P'_{M}."""
    with mp.workdps(_DPS):
        M = n_nodes - 1
        if M < 1:
            raise ValueError("need at least two nodes")
        inner = []
        if M > 1:
            # roots of P'_M on (-1, 1); P_M by the three-term recurrence
            # (coefficients, highest degree first), then its derivative
            p0, p1 = [mp.mpf(1)], [mp.mpf(1), mp.mpf(0)]
            for k in range(2, M + 1):
                a = [(2 * k - 1) * c / mp.mpf(k) for c in p1] + [mp.mpf(0)]
                b = [mp.mpf(0), mp.mpf(0)] + [(k - 1) * c / mp.mpf(k) for c in p0]
                p0, p1 = p1, [x - y for x, y in zip(a, b)]
            PM = p1 if M > 1 else p1
            deg = len(PM) - 1
            dPM = [c * (deg - i) for i, c in enumerate(PM[:-1])]
            roots = mp.polyroots(dPM, maxsteps=200, extraprec=200)
            inner = [mp.re(r) for r in roots]
        xs = [mp.mpf(-1)] + sorted(inner) + [mp.mpf(1)]
        return [(x + 1) / 2 for x in xs]


def _lagrange_integrals(tau, upper):
    """integral_0^upper L_j(t) dt for all j, by exact polynomial algebra."""
    n = len(tau)
    out = []
    for j in range(n):
        # coefficients of prod_{i != j} (t - tau_i) / (tau_j - tau_i), low order first
        coeffs = [mp.mpf(1)]
        denom = mp.mpf(1)
        for i in range(n):
            if i == j:
                continue
            new = [mp.mpf(0)] * (len(coeffs) + 1)
            for d, a in enumerate(coeffs):
                new[d + 1] += a
                new[d] -= a * tau[i]
            coeffs = new
            denom *= tau[j] - tau[i]
        integral = sum(a * upper ** (d + 1) / (d + 1) for d, a in enumerate(coeffs))
        out.append(integral / denom)
    return out


def tables_mp(n_nodes):
    """High-precision (tau, Q, QI_lu, QI_be, QE_cum, QE_lit) as mpmath matrices."""
    with mp.workdps(_DPS):
        tau = lobatto_nodes_mp(n_nodes)
        M = n_nodes - 1
        Q = mp.matrix(M, M + 1)
        for p in range(1, M + 1):
            row = _lagrange_integrals(tau, tau[p])
            for j in range(M + 1):
                Q[p - 1, j] = row[j]
        # Q~ = Q without its first column; Doolittle LU of transpose(Q~)
        Qt_T = mp.matrix(M, M)
        for a in range(M):
            for b in range(M):
                Qt_T[a, b] = Q[b, a + 1]
        L = mp.eye(M)
        U = mp.matrix(M, M)
        for i in range(M):
            for k in range(i, M):
                U[i, k] = Qt_T[i, k] - sum(L[i, s] * U[s, k] for s in range(i))
            for k in range(i + 1, M):
                L[k, i] = (Qt_T[k, i] - sum(L[k, s] * U[s, i] for s in range(i))) / U[i, i]
        QI_lu = U.T
        dtau = [tau[m + 1] - tau[m] for m in range(M)]
        QI_be = mp.matrix(M, M)
        QE_cum = mp.matrix(M, M)
        QE_lit = mp.matrix(M, M)
        for p in range(1, M + 1):
            for j in range(1, p + 1):
                QI_be[p - 1, j - 1] = dtau[j - 1]
            for j in range(1, p):
                QE_cum[p - 1, j - 1] = dtau[j]
            if p >= 2:
                QE_lit[p - 1, p - 2] = dtau[p - 1]
        return tau, Q, QI_lu, QI_be, QE_cum, QE_lit


def _to_np(A):
    if isinstance(A, list):
        return np.array([float(v) for v in A])
    return np.array([[float(A[i, j]) for j in range(A.cols)] for i in range(A.rows)])


def sdc_tables(n_nodes, qi="lu", qe="cumulative"):
    """FP64 tables for ``n_nodes`` Gauss-Lobatto nodes.

    qi: "lu" (MISDCQ / CISDCQ / IMEXQ) or "be" (cumulative backward Euler).
    qe: "cumulative" (forward Euler from every earlier node, the reading used
        throughout) or "literal" (only the (m+1, m) entry).
    Returns dict(tau, dtau, Q, q0, Qt, QI, QE).
    """
    tau, Q, QI_lu, QI_be, QE_cum, QE_lit = tables_mp(n_nodes)
    tau = _to_np(tau)
    Qn = _to_np(Q)
    QI = _to_np(QI_lu if qi == "lu" else QI_be)
    QE = _to_np(QE_cum if qe == "cumulative" else QE_lit)
    return dict(tau=tau, dtau=np.diff(tau), Q=Qn, q0=Qn[:, 0].copy(),
                Qt=Qn[:, 1:].copy(), QI=QI, QE=QE, M=n_nodes - 1)


def node_to_node_weights(n_nodes):
    """S with s_{m+1,j} = (1/dt) integral over [t^m, t^{m+1}] of L_j (rows m = 0..M-1)."""
    _, Q, *_ = tables_mp(n_nodes)
    with mp.workdps(_DPS):
        S = mp.matrix(Q.rows, Q.cols)
        for i in range(Q.rows):
            for j in range(Q.cols):
                S[i, j] = Q[i, j] - (Q[i - 1, j] if i > 0 else 0)
    return _to_np(S)
