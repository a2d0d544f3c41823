// Device code of the per-cell reaction solve (step S5, eq.
// reaction_step_numerical_methodology): thermodynamics, mass-action rates and
// their analytic Jacobian, the LU of the Newton matrix and one thread's
// Newton iteration, shared by the kernels of chem.hip and the persistent
// ensemble stage kernel (ensemble.hip).
#pragma once

#include <cfloat>
#include <cmath>

#include "misdc_impl.h"
#include "newton_hist.h"

namespace misdc {

__device__ __forceinline__ double species_h(const MechDev& m, int k, double T) {
    return m.hf[k] + m.cp[k] * (T - T_REF);
}

// T from (Y, h), closed form for constant heat capacities
template <int NS>
__device__ __forceinline__ double temperature_of(const MechDev& m, const double (&Y)[NS], double h) {
    double hform = 0.0, cpm = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        hform += Y[k] * m.hf[k] * m.invW[k];
        cpm += Y[k] * m.cp[k] * m.invW[k];
    }
    return T_REF + (h - hform) / cpm;
}

template <int NS>
__device__ __forceinline__ double pick(const double (&v)[NS], int s) {
    double r = 1.0;                 // empty slot: neutral factor
#pragma unroll
    for (int l = 0; l < NS; ++l) r = (l == s) ? v[l] : r;
    return r;
}

// Rates and (optionally) Jacobian at (Y, T).
//   FR[k]  = W_k omega_k / rho0
//   J[k][l] = d FR_k / d Y_l,  JT[k] = d FR_k / d T
// Per-species concentration, Gibbs energy and enthalpy of each lane's cell:
// in registers, or (LDS) in a [NS][64] slab per quantity indexed by lane, to
// leave registers to the Jacobian.
template <int NS, bool LDS>
struct SpeciesTerms {
    double X[LDS ? 1 : NS], gk[LDS ? 1 : NS], hk[LDS ? 1 : NS];
    double* sX;
    double* sG;
    double* sH;
    int lane;
    __device__ __forceinline__ void set(int k, double x, double g, double h) {
        if (LDS) {
            sX[k * 64 + lane] = x;
            sG[k * 64 + lane] = g;
            sH[k * 64 + lane] = h;
        } else {
            X[LDS ? 0 : k] = x;
            gk[LDS ? 0 : k] = g;
            hk[LDS ? 0 : k] = h;
        }
    }
    __device__ __forceinline__ double x(int k) const { return LDS ? sX[k * 64 + lane] : X[LDS ? 0 : k]; }
    __device__ __forceinline__ double g(int k) const { return LDS ? sG[k * 64 + lane] : gk[LDS ? 0 : k]; }
    __device__ __forceinline__ double h(int k) const { return LDS ? sH[k * 64 + lane] : hk[LDS ? 0 : k]; }
    // concentration of slot species s (wave-uniform), 1 for an empty slot
    __device__ __forceinline__ double slot_x(int s) const {
        if (LDS) return s >= 0 ? sX[s * 64 + lane] : 1.0;
        double r = 1.0;
#pragma unroll
        for (int l = 0; l < NS; ++l) r = (l == s) ? X[LDS ? 0 : l] : r;
        return r;
    }
};

//   (J[k][l] for l < NS, and d FR_k / d T in J[k][NS]: J may be the leading
//   block of the caller's Newton matrix, which is then formed in place)
template <int NS, bool JAC, bool LDS = false, int ROWS = NS, int COLS = NS + 1>
__device__ __forceinline__ void reaction_terms(const MechDev& m, const double (&Y)[NS], double T,
                                               double (&FR)[NS], double (&J)[ROWS][COLS],
                                               double* lds = nullptr, int lane = 0) {
    static_assert(!JAC || (ROWS >= NS && COLS > NS), "J holds NS rows of NS + 1 entries");
    SpeciesTerms<NS, LDS> sp;
    sp.sX = lds;
    sp.sG = lds + NS * 64;
    sp.sH = lds + 2 * NS * 64;
    sp.lane = lane;
    const double lnT = log(T);
    const double invT = 1.0 / T;
    const double lnTr = lnT - log(T_REF);
    const double RuT = m.R_u * T;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const double hkk = species_h(m, k, T);
        sp.set(k, m.rho0 * Y[k] * m.invW[k], hkk - T * (m.s0[k] + m.cp[k] * lnTr), hkk);
        FR[k] = 0.0;
        if (JAC) {
#pragma unroll
            for (int l = 0; l <= NS; ++l) J[k][l] = 0.0;
        }
    }
    const double ln_c0 = m.ln_patm_over_Ru - lnT;      // ln(p_atm / (R_u T))
    for (int j = 0; j < m.R; ++j) {
        const int r0 = m.slots[4 * j + 0], r1 = m.slots[4 * j + 1];
        const int p0 = m.slots[4 * j + 2], p1 = m.slots[4 * j + 3];
        // sum of nu g and nu h over the (at most four) slots
        double sg = 0.0, sh = 0.0;
#pragma unroll
        for (int l = 0; l < NS; ++l) {
            const double w = (double)((l == p0) + (l == p1) - (l == r0) - (l == r1));
            sg += w * sp.g(l);
            sh += w * sp.h(l);
        }
        const double dn = m.dn[j];
        const double kf = m.A[j] * exp(m.beta[j] * lnT - m.Ta[j] * invT);
        const double lnKc = -sg / RuT + dn * ln_c0;
        const double kr = kf * exp(-lnKc);
        const double xr0 = sp.slot_x(r0), xr1 = sp.slot_x(r1);
        const double xp0 = sp.slot_x(p0), xp1 = sp.slot_x(p1);
        const double pf = xr0 * xr1, pr = xp0 * xp1;
        const double q = kf * pf - kr * pr;
        double dqdT = 0.0;
        double v[NS];
        if (JAC) {
            const double dlnkf = m.beta[j] * invT + m.Ta[j] * invT * invT;
            const double dlnKc = sh / (RuT * T) - dn * invT;
            dqdT = kf * dlnkf * pf - kr * (dlnkf - dlnKc) * pr;
            const double dr0 = kf * xr1, dr1 = kf * xr0, dp0 = -kr * xp1, dp1 = -kr * xp0;
#pragma unroll
            for (int l = 0; l < NS; ++l) {
                double d = 0.0;
                d += (l == r0) ? dr0 : 0.0;
                d += (l == r1) ? dr1 : 0.0;
                d += (l == p0) ? dp0 : 0.0;
                d += (l == p1) ? dp1 : 0.0;
                v[l] = d * m.rho0 * m.invW[l];       // d q / d Y_l
            }
        }
        const double* u = m.uW + (size_t)j * m.N;  // nu_kj W_k / rho0
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const double uk = u[k];
            FR[k] += uk * q;
            if (JAC) {
                J[k][NS] += uk * dqdT;
#pragma unroll
                for (int l = 0; l < NS; ++l) J[k][l] += uk * v[l];
            }
        }
    }
}

// Solve A x = b by LU with partial pivoting on the augmented matrix [A | b]
// (n x (n+1), b in column n, replaced by x); the pivot row is the first row
// holding the largest magnitude in the column.  The exchange gathers the
// pivot row once and writes row c into the pivot's place (selects over the
// rows below c): the same data movement as swapping row c with each
// candidate in turn, with far fewer values live at once; keeping b inside
// the matrix keeps it in registers too.
template <int n>
__device__ __forceinline__ void lu_solve(double (&A)[n][n + 1]) {
#pragma unroll
    for (int c = 0; c < n; ++c) {
        int piv = c;
        double amax = fabs(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < n; ++r) {
            const double a = fabs(A[r][c]);
            const bool gt = a > amax;
            amax = gt ? a : amax;
            piv = gt ? r : piv;
        }
#pragma unroll
        for (int l = c; l <= n; ++l) {
            double pv = A[c][l];
#pragma unroll
            for (int r = c + 1; r < n; ++r) pv = (r == piv) ? A[r][l] : pv;
#pragma unroll
            for (int r = c + 1; r < n; ++r) A[r][l] = (r == piv) ? A[c][l] : A[r][l];
            A[c][l] = pv;
        }
        const double inv = 1.0 / A[c][c];
#pragma unroll
        for (int r = c + 1; r < n; ++r) {
            const double f = A[r][c] * inv;
#pragma unroll
            for (int l = c + 1; l <= n; ++l) A[r][l] -= f * A[c][l];
        }
    }
#pragma unroll
    for (int r = n - 1; r >= 0; --r) {
        double s = A[r][n];
#pragma unroll
        for (int l = r + 1; l < n; ++l) s -= A[r][l] * A[l][n];
        A[r][n] = s / A[r][r];
    }
}

// One cell-node solve by one thread.  INERT_LAST: the last species is the bath gas, which no reaction touches
// (the mechanism checks guarantee it), so its row of the Newton matrix is the
// unit row (plus the pseudo-time shift) and its column is zero but for the
// enthalpy row: its update is G_b / (1 + 1/dtau), and the remaining system in
// the reacting species and T is one row and column smaller.  The reduced
// matrix (and its pivot search) leaves registers for two wavefronts per SIMD.
template <int NS, bool INERT_LAST>
__device__ __forceinline__ int newton_cell(const MechDev& m, const NewtonArgs& a, int64_t i) {
    constexpr int NR = INERT_LAST ? NS - 1 : NS;    // species in the coupled system
    constexpr int NX = NR + 1;                      // ... and T
    int code = 0;                   // iterations, -1 when not converged
    if (i < a.n) {
    const double c = a.c ? a.c[i] * a.c_scalar : a.c_scalar;
    const double h = a.h[i];
    // b_Y (and the floor of Y) are re-read when needed rather than held in
    // registers, and Y waits in LDS while the LU runs
    __shared__ double sY[NS][64];
    __shared__ double sTerms[3 * NR * 64];          // X, g, h of the reacting species
    const int lane = threadIdx.x & 63;
    double Y[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) Y[k] = a.guess[k * a.ldg + i];
    double T = temperature_of<NS>(m, Y, h);
    const double inv_scale = 1.0 / m.newton_scale;
    double inv_dtau = 0.0;          // 0: plain Newton step
    double gnorm_old = -1.0;        // < 0: none yet
    int it = 0;
    bool conv = false;
    while (!conv && it < a.opt.maxit) {
        double FR[NR];
        double M[NX][NX + 1];        // [Newton matrix | residual G]
        double Yr[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) Yr[k] = Y[k];
        // the Jacobian of the rates in M's leading rows (column NR: d/dT)
        reaction_terms<NR, true, true>(m, Yr, T, FR, M, sTerms, lane);
        double hsum = 0.0, cpm = 0.0, hb = 0.0, Gb = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const double hk = species_h(m, k, T) * m.invW[k];
            hsum += Y[k] * hk;
            cpm += Y[k] * m.cp[k] * m.invW[k];
            if (k < NR) {
                M[k][NX] = Y[k] - c * FR[k] - a.bY[k * a.ldb + i];
#pragma unroll
                for (int l = 0; l < NR; ++l) M[k][l] = ((k == l) ? 1.0 : 0.0) - c * M[k][l];
                M[k][NR] = -c * M[k][NR];
                M[NR][k] = hk * inv_scale;
            } else {                                 // the bath: no rates
                Gb = Y[k] - c * 0.0 - a.bY[k * a.ldb + i];
                hb = hk * inv_scale;
            }
        }
        M[NR][NX] = (hsum - h) * inv_scale;
        M[NR][NR] = cpm * inv_scale;
        double gn2 = 0.0;
#pragma unroll
        for (int k = 0; k < NR; ++k) gn2 += M[k][NX] * M[k][NX];
        if (INERT_LAST) gn2 += Gb * Gb;
        gn2 += M[NR][NX] * M[NR][NX];
#pragma unroll
        for (int k = 0; k < NX; ++k) M[k][k] += inv_dtau;
        // the bath's update, eliminated from the enthalpy row
        const double db = INERT_LAST ? Gb / (1.0 + inv_dtau) : 0.0;
        if (INERT_LAST) M[NR][NX] -= hb * db;
#pragma unroll
        for (int k = 0; k < NS; ++k) sY[k][lane] = Y[k];
        lu_solve<NX>(M);             // column NX now holds delta (reacting species, T)
#pragma unroll
        for (int k = 0; k < NS; ++k) Y[k] = sY[k][lane];
        double D[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) D[k] = (k < NR) ? M[k < NR ? k : 0][NX] : db;
        const double dT = M[NR][NX];
        ++it;
        bool ok = true;
        double dmax = 0.0;
        double Yt[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            Yt[k] = Y[k] - D[k];
            const double lo = fmin(a.bY[k * a.ldb + i], 0.0) - a.opt.neg_slack;
            ok = ok && isfinite(D[k]) && (Yt[k] >= lo);
            dmax = fmax(dmax, fabs(D[k]));
        }
        const double Tt = T - dT;
        ok = ok && isfinite(dT) && (Tt > 0.0);
        if (!ok) {
            inv_dtau = (inv_dtau == 0.0) ? 1.0 / a.opt.dtau0 : inv_dtau * 4.0;
            continue;
        }
        const bool was_newton = (inv_dtau == 0.0);
        const double gnorm = sqrt(gn2);
#pragma unroll
        for (int k = 0; k < NS; ++k) Y[k] = Yt[k];
        T = Tt;
        if (!was_newton) {
            double grow = 2.0;
            if (gnorm_old >= 0.0 && gnorm > 0.0) grow = fmax(2.0, gnorm_old / gnorm);
            inv_dtau = inv_dtau / grow;
            if (inv_dtau < 1.0 / a.opt.dtau_max) inv_dtau = 0.0;
        }
        gnorm_old = gnorm;
        conv = was_newton && (dmax <= a.opt.tol) && (fabs(dT) <= a.opt.tol * fabs(Tt));
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) a.Y[k * a.ldy + i] = Y[k];
    const double Tc = temperature_of<NS>(m, Y, h);
    if (a.T) a.T[i] = Tc;
    if (a.h_out) a.h_out[i] = h;
    if (a.th_out) a.th_out[i] = pow(Tc / T_DIFF_REF, THETA_EXP);
    if (a.FR) {
        double FR[NS], J[1][NS + 1];
        reaction_terms<NS, false>(m, Y, Tc, FR, J);
#pragma unroll
        for (int k = 0; k < NS; ++k) a.FR[k * a.ldf + i] = FR[k];
    }
    code = conv ? it : -1;
    if (a.iters) a.iters[i] = code;
    }
    return code;
}

// Statistics of one wavefront's solves (all 64 lanes take part): one set of
// atomics per wavefront into one of NEWTON_BUCKETS counter sets, and the
// outcome histogram; ``wave`` numbers the wavefront.
__device__ __forceinline__ void newton_wave_stats(const NewtonArgs& a, unsigned wave, bool valid,
                                                  int code) {
    if (a.buckets) {
        // statistics of the wavefront (all 64 lanes take part), one set of
        // atomics per wavefront into one of NEWTON_BUCKETS counter sets
        int solves = valid ? 1 : 0, sum = code > 0 ? code : 0, bad = code < 0 ? 1 : 0;
        int mx = sum;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            solves += __shfl_xor(solves, off);
            sum += __shfl_xor(sum, off);
            bad += __shfl_xor(bad, off);
            const int o = __shfl_xor(mx, off);
            mx = o > mx ? o : mx;
        }
        if ((threadIdx.x & 63) == 0) {
            unsigned long long* b = a.buckets + (size_t)(wave % NEWTON_BUCKETS) *
                                                     NEWTON_BUCKET_STRIDE;
            atomicAdd(&b[0], (unsigned long long)solves);
            atomicAdd(&b[1], (unsigned long long)sum);
            if (bad) atomicAdd(&b[2], (unsigned long long)bad);
            atomicMax(&b[3], (unsigned long long)mx);
        }
        if (a.hist)
            wave_hist_add(a.hist + (size_t)(wave % NEWTON_HIST_SETS) * NEWTON_HIST_BINS, valid,
                          code);
    }
}

}  // namespace misdc
