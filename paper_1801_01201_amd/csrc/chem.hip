// Chemistry kernels: thermodynamics, mass-action rates and the per-cell
// backward-Euler reaction solve of step S5 (eq.
// reaction_step_numerical_methodology).
//
// Layout: structure of arrays, one thread per cell; field k of cell i is at
// [k * ld + i], so every load and store of a wavefront is one coalesced
// 512-byte transaction per field.  The mechanism tables are indexed with
// wave-uniform indices (reaction j, species k), so they are fetched through
// the scalar cache.  Per-thread arrays (state, residual, Jacobian) are only
// ever indexed with compile-time indices so that they stay in registers;
// runtime species indices taken from the mechanism are resolved with select
// chains over the (template) species count NS.
#include <cfloat>
#include <cmath>

#include "misdc_impl.h"
#include "newton_hist.h"

namespace misdc {

namespace {

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

// INERT_LAST: the last species is the bath gas, which no reaction touches
// (the mechanism checks guarantee it), so its row of the Newton matrix is the
// unit row (plus the pseudo-time shift) and its column is zero but for the
// enthalpy row: its update is G_b / (1 + 1/dtau), and the remaining system in
// the reacting species and T is one row and column smaller.  The reduced
// matrix (and its pivot search) leaves registers for two wavefronts per SIMD.
template <int NS, bool INERT_LAST>
__global__ void __launch_bounds__(64) newton_kernel(MechDev m, NewtonArgs a) {
    constexpr int NR = INERT_LAST ? NS - 1 : NS;    // species in the coupled system
    constexpr int NX = NR + 1;                      // ... and T
    // A wavefront iterates until its slowest cell has converged.  On a 2-D
    // grid an 8 x 8 tile of cells keeps cells at similar distances from a
    // flame front together, whichever way the front runs, so its iteration
    // counts differ less than along 64 cells of a row (256 x 256 flame: the
    // mean per-wavefront maximum falls from 2.8 to 2.3 iterations, against a
    // mean of 2.2).  The launch time follows the slowest wavefronts of its
    // one or two rounds rather than the mean, so it gains only ~1 %.  Lanes
    // outside the grid take i = n.
    int64_t i;
    if (a.tile_nx > 0) {
        const int ntx = (a.tile_nx + 7) / 8;
        const int x = (int)(blockIdx.x % ntx) * 8 + (int)(threadIdx.x & 7);
        const int y = (int)(blockIdx.x / ntx) * 8 + (int)(threadIdx.x >> 3);
        i = (x < a.tile_nx && y < a.tile_ny) ? (int64_t)y * a.tile_nx + x : a.n;
    } else {
        i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    }
    int code = 0;                   // iterations, -1 when not converged
    if (i < a.n) {
    const double c = a.c ? a.c[i] * a.c_scalar : a.c_scalar;
    const double h = a.h[i];
    // b_Y (and the floor of Y) are re-read when needed rather than held in
    // registers, and Y waits in LDS while the LU runs
    __shared__ double sY[NS][64];
    __shared__ double sTerms[3 * NR * 64];          // X, g, h of the reacting species
    const int lane = threadIdx.x;
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
    if (a.FR) {
        double FR[NS], J[1][NS + 1];
        reaction_terms<NS, false>(m, Y, Tc, FR, J);
#pragma unroll
        for (int k = 0; k < NS; ++k) a.FR[k * a.ldf + i] = FR[k];
    }
    code = conv ? it : -1;
    if (a.iters) a.iters[i] = code;
    }
    if (a.buckets) {
        // statistics of the wavefront (all 64 lanes take part), one set of
        // atomics per wavefront into one of NEWTON_BUCKETS counter sets
        int solves = (i < a.n) ? 1 : 0, sum = code > 0 ? code : 0, bad = code < 0 ? 1 : 0;
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
            unsigned long long* b = a.buckets + (size_t)((blockIdx.x * (blockDim.x / 64) +
                                                          threadIdx.x / 64) % NEWTON_BUCKETS) *
                                                     NEWTON_BUCKET_STRIDE;
            atomicAdd(&b[0], (unsigned long long)solves);
            atomicAdd(&b[1], (unsigned long long)sum);
            if (bad) atomicAdd(&b[2], (unsigned long long)bad);
            atomicMax(&b[3], (unsigned long long)mx);
        }
        if (a.hist)
            wave_hist_add(a.hist + (size_t)((blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) %
                                            NEWTON_HIST_SETS) * NEWTON_HIST_BINS,
                          i < a.n, code);
    }
}

// wave-aggregated statistics: [0] solves, [1] iterations, [2] failures, [3] max
// (grid-stride over few workgroups: the counters take one atomic per
// workgroup, and many workgroups contending for them cost more than the sum);
// with hist, the histogram of the outcomes as well
template <int NS>
__global__ void __launch_bounds__(256) newton_stats_kernel(int64_t n, const int32_t* iters,
                                                           unsigned long long* stats,
                                                           unsigned long long* hist) {
    __shared__ unsigned long long s_sum[4], s_bad[4], s_max[4];
    unsigned long long v = 0, b = 0, mx = 0;
    unsigned long long* set =
        hist ? hist + (size_t)((blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) %
                               NEWTON_HIST_SETS) * NEWTON_HIST_BINS
             : nullptr;
    // the loop bound is the same for all lanes of a wavefront
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const int32_t it = i < n ? iters[i] : 0;
        const unsigned long long vi = it > 0 ? (unsigned long long)it : 0ull;
        v += vi;
        b += (i < n && it < 0) ? 1ull : 0ull;
        mx = vi > mx ? vi : mx;
        if (set) wave_hist_add(set, i < n, it);
    }
    for (int off = 32; off > 0; off >>= 1) {
        v += __shfl_xor(v, off);
        b += __shfl_xor(b, off);
        const unsigned long long o = __shfl_xor(mx, off);
        mx = o > mx ? o : mx;
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) { s_sum[wave] = v; s_bad[wave] = b; s_max[wave] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long S = 0, B = 0, X = 0;
        const int nw = (blockDim.x + 63) / 64;
        for (int w = 0; w < nw; ++w) {
            S += s_sum[w];
            B += s_bad[w];
            X = s_max[w] > X ? s_max[w] : X;
        }
        if (blockIdx.x == 0) atomicAdd(&stats[0], (unsigned long long)n);
        atomicAdd(&stats[1], S);
        atomicAdd(&stats[2], B);
        atomicMax(&stats[3], X);
    }
}

__global__ void __launch_bounds__(256) enthalpy_kernel(MechDev m, int64_t n, const double* Yp,
                                                       const double* Tp, double* hp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double T = Tp[i];
    double h = 0.0;
    for (int k = 0; k < m.N; ++k) h += Yp[k * n + i] * species_h(m, k, T) * m.invW[k];
    hp[i] = h;
}

__global__ void __launch_bounds__(256) temperature_kernel(MechDev m, int64_t n, const double* Yp,
                                                          int64_t ldy, const double* hp,
                                                          double* Tp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double hform = 0.0, cpm = 0.0;
    for (int k = 0; k < m.N; ++k) {
        const double y = Yp[k * ldy + i];
        hform += y * m.hf[k] * m.invW[k];
        cpm += y * m.cp[k] * m.invW[k];
    }
    Tp[i] = T_REF + (hp[i] - hform) / cpm;
}

template <int NS>
__global__ void __launch_bounds__(64) source_kernel(MechDev m, int64_t n, const double* Yp,
                                                    int64_t ldy, const double* hp, double* FRp,
                                                    int64_t ldf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double Y[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) Y[k] = Yp[k * ldy + i];
    const double T = temperature_of<NS>(m, Y, hp[i]);
    double FR[NS], J[1][NS + 1];
    reaction_terms<NS, false>(m, Y, T, FR, J);
#pragma unroll
    for (int k = 0; k < NS; ++k) FRp[k * ldf + i] = FR[k];
}

inline unsigned grid_for(int64_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

int launch_enthalpy(const Mech& m, int64_t n, const double* Y, const double* T, double* h,
                    hipStream_t s) {
    if (n == 0) return MISDC_OK;
    hipLaunchKernelGGL(enthalpy_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, m.dev, n, Y,
                       T, h);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_temperature(const Mech& m, int64_t n, const double* Y, const double* h, double* T,
                       hipStream_t s) {
    if (n == 0) return MISDC_OK;
    hipLaunchKernelGGL(temperature_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, m.dev, n, Y,
                       n, h, T);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_state_temperature(const Mech& m, int64_t n, const double* state, double* T,
                             hipStream_t s) {
    if (n == 0) return MISDC_OK;
    hipLaunchKernelGGL(temperature_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, m.dev, n,
                       state, n, state + (size_t)m.dev.N * n, T);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_reaction_source(const Mech& m, int64_t n, const double* Y, const double* h,
                           double* FR, hipStream_t s) {
    if (n == 0) return MISDC_OK;
    if (m.dev.N != 9) return launch_reaction_source_wave(m, n, Y, n, h, FR, n, s);
    hipLaunchKernelGGL(source_kernel<9>, dim3(grid_for(n, 64)), dim3(64), 0, s, m.dev, n, Y, n,
                       h, FR, n);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_reaction_newton(const Mech& m, const NewtonArgs& a, hipStream_t s) {
    if (a.n == 0) return MISDC_OK;
    const int kind = a.opt.kernel;
    if (kind < MISDC_NEWTON_AUTO || kind > MISDC_NEWTON_SPECIALIZED)
        return fail(MISDC_EINVAL, "unknown reaction solve kernel %d", kind);
    // the generated kernel where it exists (automatic choice for an FP64 LU)
    const bool spec = (kind == MISDC_NEWTON_SPECIALIZED) ||
                      (kind == MISDC_NEWTON_AUTO && m.spec_fn && a.opt.lu == MISDC_LU_FP64);
    const bool thread = !spec && ((kind == MISDC_NEWTON_THREAD) ||
                                  (kind == MISDC_NEWTON_AUTO && m.dev.N == 9));
    if ((thread || spec) && a.opt.lu != MISDC_LU_FP64)
        return fail(MISDC_EINVAL, "the per-thread reaction solves compute their LU in FP64 only");
    if (spec) {
        int rc = launch_newton_spec(m, a, s);
        if (rc) return rc;
        if (a.stats && a.iters && !a.buckets) {
            const int64_t gb = grid_for(a.n, 256 * 16);
            hipLaunchKernelGGL(newton_stats_kernel<9>, dim3(gb < 32 ? gb : 32), dim3(256), 0, s,
                               a.n, a.iters, a.stats, a.hist);
            MISDC_HIP(hipGetLastError());
        }
        return MISDC_OK;
    }
    if (!thread) return launch_reaction_newton_wave(m, a, a.opt.lu, s);
    if (m.dev.N != 9)
        return fail(MISDC_EUNSUPPORTED, "per-thread reaction solve: %d species not built", m.dev.N);
    int64_t blocks = grid_for(a.n, 64);
    if (a.tile_nx > 0) {
        if (a.tile_ny <= 0 || (int64_t)a.tile_nx * a.tile_ny != a.n)
            return fail(MISDC_EINVAL, "tiled reaction solve: %d x %d cells for n = %lld", a.tile_nx,
                        a.tile_ny, (long long)a.n);
        blocks = (int64_t)((a.tile_nx + 7) / 8) * ((a.tile_ny + 7) / 8);
    }
    if (m.dev.bath == 8)
        hipLaunchKernelGGL((newton_kernel<9, true>), dim3((unsigned)blocks), dim3(64), 0, s, m.dev, a);
    else
        hipLaunchKernelGGL((newton_kernel<9, false>), dim3((unsigned)blocks), dim3(64), 0, s, m.dev, a);
    MISDC_HIP(hipGetLastError());
    if (a.stats && a.iters && !a.buckets) {
        const int64_t gb = grid_for(a.n, 256 * 16);
        hipLaunchKernelGGL(newton_stats_kernel<9>, dim3(gb < 32 ? gb : 32), dim3(256), 0, s, a.n,
                           a.iters, a.stats, a.hist);
        MISDC_HIP(hipGetLastError());
    }
    return MISDC_OK;
}

}  // namespace misdc
