// Reaction kernels with one wavefront per cell, for mechanisms of any size up
// to 63 species: the backward-Euler reaction solve of step S5 (eq.
// reaction_step_numerical_methodology) and the source F_R of eq.
// species_equation.  Used where the per-thread kernels cannot hold the
// Jacobian in registers (53 species: a 54 x 54 system per cell).
//
// Per Newton iteration of one cell:
//  * species lane k holds Y_k; the temperature row is lane N;
//  * rates: the reactions are processed in chunks of 64, one per lane; each
//    lane evaluates q_j, dq_j/dT and the derivatives of q_j with respect to
//    its (at most four) slot species and stores them in LDS;
//  * species lane k gathers F_R,k and its row of I - c J over its own
//    reaction list (fixed order: the result does not depend on scheduling);
//    the matrix is assembled in LDS;
//  * LU with partial pivoting, one matrix row per lane held in registers:
//    rows never move, the pivot of column c is the non-retired lane with
//    the largest |a_c| (lowest lane on ties); the pivot row is broadcast
//    through LDS and the back substitution broadcasts each solution entry
//    with a lane read.
// The Newton control flow (pseudo-transient continuation, acceptance and
// convergence tests) is the one of the per-thread kernel; it is uniform over
// the wavefront because the wavefront works on a single cell.
//
// With the FP32 variant the LU factors are computed in single precision on
// the matrix cores (panel of 16 columns on the vector units, trailing update
// with 16x16x4 FP32 MFMA) and the Newton correction is refined against the
// FP64 matrix (residual in FP64) until its backward error is at the FP64
// rounding level; if the residual stops contracting (cond(M) 2^-24 near 1)
// that Newton iteration uses the FP64 LU instead.
#include <cfloat>
#include <cmath>

#include "misdc_impl.h"
#include "newton_hist.h"
#include "wave.h"

namespace misdc {

namespace {

constexpr int WV = 64;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_max_step(double v) {
    return fmax(v, dpp_move<CTRL, ROW_MASK>(v));
}

// max of v over the 64 lanes (lanes of a disabled DPP row read 0, which is
// harmless for the non-negative candidates used here); uniform result
__device__ __forceinline__ double wave_max(double v) {
    v = dpp_max_step<0xB1, 0xf>(v);
    v = dpp_max_step<0x4E, 0xf>(v);
    v = dpp_max_step<0x141, 0xf>(v);
    v = dpp_max_step<0x140, 0xf>(v);
    v = dpp_max_step<0x142, 0xa>(v);
    v = dpp_max_step<0x143, 0xc>(v);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// value of v in lane src (src wave-uniform)
__device__ __forceinline__ double lane_read(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ int first_lane(unsigned long long mask) {
    return mask ? __ffsll((long long)mask) - 1 : -1;
}

typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int LDA32 = 65;

struct Lds32 {
    float* A;        // 64 x LDA32
    float* piv;      // 17: pivot row (16 panel entries) and 1/pivot
    int* pos;        // 64: pivot position of each row (64: not chosen yet)
    double* vec;     // 64: broadcast vector (FP64)
};

// LDS layout of one cell (doubles): matrix rows (stride ld), species
// buffers, the reaction chunk, the pivot row and the pivot lanes.
struct Lds {
    double* M;       // n x ld
    double* X;       // 64: concentrations
    double* gk;      // 64: Gibbs energies
    double* hk;      // 64: molar enthalpies
    double* q;       // 64: rates of progress of the chunk
    double* qT;      // 64: d q / d T
    double* D;       // 4 x 64: d q / d Y of the slot species
    double* piv;     // NXP + 2: pivot row, its right-hand side, 1/pivot
    int* plane;      // NXP: pivot lane of each column
    Lds32 s32;       // FP32 LU (LU variant only)
};

template <int NXP>
__device__ __forceinline__ Lds lds_layout(double* base, int n, int ld) {
    Lds L;
    L.M = base;
    L.X = base + (size_t)n * ld;
    L.gk = L.X + WV;
    L.hk = L.gk + WV;
    L.q = L.hk + WV;
    L.qT = L.q + WV;
    L.D = L.qT + WV;
    L.piv = L.D + 4 * WV;
    L.plane = (int*)(L.piv + NXP + 2);
    double* tail = L.piv + NXP + 2 + (NXP + 1) / 2;
    L.s32.vec = tail;
    L.s32.A = (float*)(tail + WV);
    L.s32.piv = L.s32.A + 64 * LDA32;
    L.s32.pos = (int*)(L.s32.piv + 18);
    return L;
}

template <int NXP, bool FP32>
constexpr size_t lds_doubles(int n, int ld) {
    return (size_t)n * ld + 10 * WV + NXP + 2 + (NXP + 1) / 2 +
           (FP32 ? WV + (64 * LDA32 + 18 + 64 + 1) / 2 : 0);
}

// temperature from (Y, h): closed form for constant heat capacities
__device__ __forceinline__ double wave_temperature(const MechDev& m, double y, int lane, double h) {
    const bool sp = lane < m.N;
    const double hf = wave_sum(sp ? y * m.hf[lane] * m.invW[lane] : 0.0);
    const double cpm = wave_sum(sp ? y * m.cp[lane] * m.invW[lane] : 0.0);
    return T_REF + (h - hf) / cpm;
}

// Rates of the reactions of one chunk (one per lane) at the species
// quantities in LDS; with JAC also d q/dT and the slot derivatives.
template <bool JAC>
__device__ __forceinline__ void chunk_rates(const MechDev& m, const Lds& L, int j, double T,
                                            double lnT, double invT) {
    const int lane = threadIdx.x;
    if (j >= m.R) {
        L.q[lane] = 0.0;
        return;
    }
    const int r0 = m.slots[4 * j + 0], r1 = m.slots[4 * j + 1];
    const int p0 = m.slots[4 * j + 2], p1 = m.slots[4 * j + 3];
    const double xr0 = r0 >= 0 ? L.X[r0] : 1.0, xr1 = r1 >= 0 ? L.X[r1] : 1.0;
    const double xp0 = p0 >= 0 ? L.X[p0] : 1.0, xp1 = p1 >= 0 ? L.X[p1] : 1.0;
    double sg = 0.0, sh = 0.0;
    if (p0 >= 0) { sg += L.gk[p0]; sh += L.hk[p0]; }
    if (p1 >= 0) { sg += L.gk[p1]; sh += L.hk[p1]; }
    if (r0 >= 0) { sg -= L.gk[r0]; sh -= L.hk[r0]; }
    if (r1 >= 0) { sg -= L.gk[r1]; sh -= L.hk[r1]; }
    const double RuT = m.R_u * T;
    const double dn = m.dn[j];
    const double kf = m.A[j] * exp(m.beta[j] * lnT - m.Ta[j] * invT);
    const double lnKc = -sg / RuT + dn * (m.ln_patm_over_Ru - lnT);
    const double kr = kf * exp(-lnKc);
    const double pf = xr0 * xr1, pr = xp0 * xp1;
    L.q[lane] = kf * pf - kr * pr;
    if (JAC) {
        const double dlnkf = m.beta[j] * invT + m.Ta[j] * invT * invT;
        const double dlnKc = sh / (RuT * T) - dn * invT;
        L.qT[lane] = kf * dlnkf * pf - kr * (dlnkf - dlnKc) * pr;
        L.D[0 * WV + lane] = r0 >= 0 ? kf * xr1 * m.rho0 * m.invW[r0] : 0.0;
        L.D[1 * WV + lane] = r1 >= 0 ? kf * xr0 * m.rho0 * m.invW[r1] : 0.0;
        L.D[2 * WV + lane] = p0 >= 0 ? -kr * xp1 * m.rho0 * m.invW[p0] : 0.0;
        L.D[3 * WV + lane] = p1 >= 0 ? -kr * xp0 * m.rho0 * m.invW[p1] : 0.0;
    }
}

// Species quantities of the current state into LDS (lanes < N).
__device__ __forceinline__ void species_state(const MechDev& m, const Lds& L, double y, double T,
                                              double lnT) {
    const int lane = threadIdx.x;
    if (lane < m.N) {
        const double hk = m.hf[lane] + m.cp[lane] * (T - T_REF);
        L.X[lane] = m.rho0 * y * m.invW[lane];
        L.hk[lane] = hk;
        L.gk[lane] = hk - T * (m.s0[lane] + m.cp[lane] * (lnT - log(T_REF)));
    }
}

// F_R of species lane k (and, with JAC, the rows of I - c J in LDS:
// M[k][l] -= c dFR_k/dY_l, returns dFR_k/dT in *fT).  The matrix rows must
// hold the identity part before the call.
// The entries of a chunk are taken EB at a time with all of their table
// loads issued first (no load depends on another), in list order.
template <bool JAC>
__device__ __forceinline__ double source_and_rows(const MechDev& m, const Lds& L, int ld, double T,
                                                  double c, double* fT) {
    constexpr int EB = 4;
    const int lane = threadIdx.x;
    const double lnT = log(T), invT = 1.0 / T;
    double fr = 0.0, ft = 0.0;
    const int* rc = m.rowc + (size_t)(lane < m.N ? lane : 0) * (m.nch + 1);
    for (int base = 0, ch = 0; base < m.R; base += WV, ++ch) {
        chunk_rates<JAC>(m, L, base + lane, T, lnT, invT);
        __syncthreads();
        if (lane < m.N) {
            const int e1 = rc[ch + 1];
            for (int e = rc[ch]; e < e1; e += EB) {
                int jj[EB], sl[EB][4];
                double u[EB];
#pragma unroll
                for (int q = 0; q < EB; ++q) {
                    const int ee = e + q < e1 ? e + q : e;
                    jj[q] = m.rowj[ee] - base;
                    u[q] = m.rowu[ee];
                    if (JAC)
#pragma unroll
                        for (int s = 0; s < 4; ++s) sl[q][s] = m.rowl[4 * ee + s];
                }
#pragma unroll
                for (int q = 0; q < EB; ++q) {
                    if (e + q >= e1) break;
                    fr += u[q] * L.q[jj[q]];
                    if (JAC) {
                        ft += u[q] * L.qT[jj[q]];
                        double* row = L.M + (size_t)lane * ld;
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const int l = sl[q][s];
                            if (l >= 0) row[l] -= c * u[q] * L.D[s * WV + jj[q]];
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (JAC) *fT = ft;
    return fr;
}

// ---------------------------------------------------------------------------
// FP64 LU of the lane rows (partial pivoting, rows stay in their lanes) and
// solve of one right-hand side g (lane's entry); returns the lane's entry of
// the solution.
// ---------------------------------------------------------------------------
template <int NXP>
__device__ __forceinline__ double lu_solve_lanes(double (&a)[NXP], double g, const Lds& L) {
    const int lane = threadIdx.x;
    bool done = lane >= NXP;
    double dinv = 0.0;
#pragma unroll
    for (int c = 0; c < NXP; ++c) {
        const double cand = done ? -1.0 : fabs(a[c]);
        const double mx = wave_max(cand);
        int p = first_lane(__ballot(!done && cand == mx));
        if (p < 0) p = first_lane(__ballot(!done));       // NaN column: any remaining row
        p = __builtin_amdgcn_readfirstlane(p);
        // the pivot row reaches the other lanes through scalar registers
        // (lane reads of the pivot lane), not through LDS
        const double pinv = 1.0 / lane_read(a[c], p);
        const double pg = lane_read(g, p);
        if (lane == p) {
            dinv = pinv;
            L.plane[c] = p;
            done = true;
        }
        if (!done) {
            const double f = a[c] * pinv;
            a[c] = f;
#pragma unroll
            for (int l = c + 1; l < NXP; ++l) a[l] -= f * lane_read(a[l], p);
            g -= f * pg;
        }
    }
    __syncthreads();
    double x = 0.0;
#pragma unroll
    for (int c = NXP - 1; c >= 0; --c) {
        const int p = __builtin_amdgcn_readfirstlane(L.plane[c]);
        const double xc = lane_read(g * dinv, p);
        if (lane == c) x = xc;
        g -= a[c] * xc;
    }
    return x;
}

// ---------------------------------------------------------------------------
// FP32 LU on the matrix cores.  The 64 x 64 (padded) matrix lives in LDS,
// row r at A[r * LDA32]; rows stay in place and plane[c] is the row chosen as
// pivot of column c.  Blocked right-looking factorisation with panels of 16
// columns: the panel is factorised on the vector units (row per lane,
// partial pivoting over every row not yet chosen), the 16 pivot rows'
// trailing part is transformed by the panel's unit lower triangle
// (U12 = L11^-1 A12, column per lane), and the remaining rows get the rank-16
// update A22 -= L21 U12 as 16 x 16 tiles of 16x16x4 FP32 MFMA.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_maxf(float v) {
    return (float)wave_max((double)v);
}

__device__ __forceinline__ float lane_readf(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Factorises A in place; returns this lane's pivot position and 1/pivot.
__device__ __forceinline__ void lu32_factor(const Lds32& S, int* plane, int& mypos, float& myinv) {
    const int lane = threadIdx.x;
    bool done = false;
    mypos = 64;
    myinv = 0.f;
    S.pos[lane] = 64;
    __syncthreads();
#pragma unroll
    for (int pb = 0; pb < 4; ++pb) {
        const int k0 = 16 * pb;
        float pan[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) pan[t] = S.A[lane * LDA32 + k0 + t];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            const float cand = done ? -1.f : fabsf(pan[t]);
            const float mx = wave_maxf(cand);
            int p = first_lane(__ballot(!done && cand == mx));
            if (p < 0) p = first_lane(__ballot(!done));
            p = __builtin_amdgcn_readfirstlane(p);
            // the pivot row of the panel reaches the other lanes by lane reads
            const float pinv = 1.f / lane_readf(pan[t], p);
            if (lane == p) {
                myinv = pinv;
                plane[k0 + t] = p;
                S.pos[lane] = k0 + t;
                mypos = k0 + t;
                done = true;
            }
            if (!done) {
                const float f = pan[t] * pinv;
                pan[t] = f;
#pragma unroll
                for (int u = t + 1; u < 16; ++u) pan[u] -= f * lane_readf(pan[u], p);
            }
        }
#pragma unroll
        for (int t = 0; t < 16; ++t) S.A[lane * LDA32 + k0 + t] = pan[t];
        __syncthreads();
        if (pb == 3) break;
        // U12 = L11^-1 A12 on the 16 pivot rows of the panel, column per lane
        if (lane >= k0 + 16) {
            float ut[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int pt = plane[k0 + t];
                float u = S.A[pt * LDA32 + lane];
#pragma unroll
                for (int s = 0; s < t; ++s) u -= S.A[pt * LDA32 + k0 + s] * ut[s];
                ut[t] = u;
                S.A[pt * LDA32 + lane] = u;
            }
        }
        __syncthreads();
        // A22 -= L21 U12 for the rows not chosen yet (chosen rows: zero L)
        const int li = lane % 16, lk = lane / 16;
#pragma unroll
        for (int R = 0; R < 4; ++R) {
            const int arow = 16 * R + li;
            const bool live = S.pos[arow] >= k0 + 16;
#pragma unroll
            for (int C = pb + 1; C < 4; ++C) {
                v4f acc;
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = S.A[(16 * R + 4 * lk + r) * LDA32 + 16 * C + li];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const float av = live ? -S.A[arow * LDA32 + k0 + 4 * kk + lk] : 0.f;
                    const float bv = S.A[plane[k0 + 4 * kk + lk] * LDA32 + 16 * C + li];
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) S.A[(16 * R + 4 * lk + r) * LDA32 + 16 * C + li] = acc[r];
            }
        }
        __syncthreads();
    }
}

// Solves with the FP32 factors: b is this lane's entry of the right-hand
// side (row order), the result is this lane's entry of the solution
// (column order).
__device__ __forceinline__ float lu32_solve(const Lds32& S, const int* plane, int mypos, float myinv,
                                            float b) {
    const int lane = threadIdx.x;
#pragma unroll 8
    for (int c = 0; c < 64; ++c) {
        const int p = __builtin_amdgcn_readfirstlane(plane[c]);
        const float yc = lane_readf(b, p);
        if (mypos > c) b -= S.A[lane * LDA32 + c] * yc;
    }
    float x = 0.f;
#pragma unroll 8
    for (int c = 63; c >= 0; --c) {
        const int p = __builtin_amdgcn_readfirstlane(plane[c]);
        const float xc = lane_readf(b * myinv, p);
        if (lane == c) x = xc;
        if (mypos < c) b -= S.A[lane * LDA32 + c] * xc;
    }
    return x;
}

// ---------------------------------------------------------------------------
// Newton solve, one wavefront per cell.
// ---------------------------------------------------------------------------
// FP32 refinement: at most this many FP32 solves per Newton iteration
constexpr int MAX_REFINE = 10;

template <int NXP, int LUK>
__global__ void __launch_bounds__(64) newton_wave_kernel(MechDev m, NewtonArgs a) {
    extern __shared__ double lds_base[];
    const int N = m.N, n = N + 1, ld = n + 1;
    const Lds L = lds_layout<NXP>(lds_base, n, ld);
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= a.n) return;                      // uniform over the block
    const bool sp = lane < N;
    const double c = a.c ? a.c[i] * a.c_scalar : a.c_scalar;
    const double h = a.h[i];
    double bY = 0.0, Y = 0.0, lo = 0.0;
    if (sp) {
        bY = a.bY[(size_t)lane * a.ldb + i];
        Y = a.guess[(size_t)lane * a.ldg + i];
        lo = fmin(bY, 0.0) - a.opt.neg_slack;
    }
    double T = wave_temperature(m, Y, lane, h);
    const double inv_scale = 1.0 / m.newton_scale;
    double inv_dtau = 0.0;
    double gnorm_old = -1.0;
    int it = 0, nref = 0, nfb = 0;
    bool conv = false;
    while (!conv && it < a.opt.maxit) {
        const double lnT = log(T);
        species_state(m, L, Y, T, lnT);
        // identity part of the rows (the enthalpy row is written by column:
        // lane k writes M[N][k])
        if (lane < n) {
            double* row = L.M + (size_t)lane * ld;
            for (int l = 0; l < n; ++l) row[l] = (l == lane) ? 1.0 : 0.0;
        }
        __syncthreads();
        double fT = 0.0;
        const double fr = source_and_rows<true>(m, L, ld, T, c, &fT);
        const double hkW = sp ? (m.hf[lane] + m.cp[lane] * (T - T_REF)) * m.invW[lane] : 0.0;
        const double hsum = wave_sum(sp ? Y * hkW : 0.0);
        const double cpm = wave_sum(sp ? Y * m.cp[lane] * m.invW[lane] : 0.0);
        double G = 0.0;
        if (sp) {
            G = Y - c * fr - bY;
            L.M[(size_t)lane * ld + N] = -c * fT;
            L.M[(size_t)N * ld + lane] = hkW * inv_scale;
        } else if (lane == N) {
            G = (hsum - h) * inv_scale;
            L.M[(size_t)N * ld + N] = cpm * inv_scale;
        }
        const double gn2 = wave_sum(G * G);
        if (lane < n) L.M[(size_t)lane * ld + lane] += inv_dtau;
        __syncthreads();
        double d = 0.0;
        bool fp64 = (LUK == 0);
        if (LUK == 1) {
            // FP32 factors of the (padded) matrix, then refinement of the
            // correction against the FP64 matrix
            const Lds32& S = L.s32;
            for (int l = 0; l < 64; ++l) {
                float v = (l == lane) ? 1.f : 0.f;
                if (lane < n && l < n) v = (float)L.M[(size_t)lane * ld + l];
                S.A[lane * LDA32 + l] = v;
            }
            __syncthreads();
            int mypos = 64;
            float myinv = 0.f;
            lu32_factor(S, L.plane, mypos, myinv);
            // refinement: d += M32^-1 (G - M d) with the residual in FP64,
            // until the backward error is at the FP64 rounding level
            // |G - M d| <= 4 eps (|M| |d| + |G|) (infinity norms); if the
            // residual stops shrinking by half per step first, this Newton
            // iteration takes the FP64 LU instead
            double rowsum = 0.0;
            if (lane < n)
                for (int l = 0; l < n; ++l) rowsum += fabs(L.M[(size_t)lane * ld + l]);
            const double mnorm = wave_max(rowsum);
            const double gnorm_inf = wave_max(lane < n ? fabs(G) : 0.0);
            double rhs = G, rprev = gnorm_inf;
            bool ok32 = false;
            for (int r = 0; r < MAX_REFINE; ++r) {
                const double corr = (double)lu32_solve(S, L.plane, mypos, myinv, (float)rhs);
                ++nref;
                d += (lane < n) ? corr : 0.0;
                S.vec[lane] = d;
                __syncthreads();
                double md = 0.0;
                if (lane < n) {
                    const double* row = L.M + (size_t)lane * ld;
                    for (int l = 0; l < n; ++l) md += row[l] * S.vec[l];
                }
                rhs = (lane < n) ? G - md : 0.0;
                __syncthreads();
                const double rn = wave_max(fabs(rhs));
                const double dn = wave_max(lane < n ? fabs(d) : 0.0);
                if (!isfinite(rn) || !isfinite(dn)) break;
                const double floor64 = DBL_EPSILON * (mnorm * dn + gnorm_inf);
                if (rn <= 4.0 * floor64) {
                    ok32 = true;
                    break;
                }
                if (!(rn <= 0.5 * rprev)) break;      // stalled: FP64 LU
                rprev = rn;
            }
            if (!ok32) {
                ++nfb;
                fp64 = true;
            }
        }
        if (fp64) {
            double row[NXP];
#pragma unroll
            for (int l = 0; l < NXP; ++l) {
                double v = (l == lane) ? 1.0 : 0.0;       // padding rows: identity
                if (lane < n && l < n) v = L.M[(size_t)lane * ld + l];
                row[l] = v;
            }
            d = lu_solve_lanes<NXP>(row, lane < n ? G : 0.0, L);
        }
        ++it;
        // acceptance of the trial x - delta
        const double dT = lane_read(d, N);
        const double Yt = Y - d;
        const bool bad_lane = (lane < n) && (!isfinite(d) || (sp && !(Yt >= lo)));
        const double Tt = T - dT;
        const bool ok = (__ballot(bad_lane) == 0ull) && (Tt > 0.0);
        if (!ok) {
            inv_dtau = (inv_dtau == 0.0) ? 1.0 / a.opt.dtau0 : inv_dtau * 4.0;
            continue;
        }
        const double dmax = wave_max(sp ? fabs(d) : 0.0);
        const bool was_newton = (inv_dtau == 0.0);
        const double gnorm = sqrt(gn2);
        if (sp) Y = Yt;
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
    if (sp) a.Y[(size_t)lane * a.ldy + i] = Y;
    const double Tc = wave_temperature(m, Y, lane, h);
    if (a.T && lane == 0) a.T[i] = Tc;
    if (a.FR) {
        species_state(m, L, Y, Tc, log(Tc));
        __syncthreads();
        const double fr = source_and_rows<false>(m, L, ld, Tc, 0.0, nullptr);
        if (sp) a.FR[(size_t)lane * a.ldf + i] = fr;
    }
    if (a.iters && lane == 0) a.iters[i] = conv ? it : -1;
    if (a.lu_info && lane == 0) a.lu_info[i] = (nref < 0xffff ? nref : 0xffff) | (nfb << 16);
}

// F_R at (Y, T(Y, h)), one wavefront per cell
__global__ void __launch_bounds__(64) source_wave_kernel(MechDev m, int64_t n, const double* Yp,
                                                         int64_t ldy, const double* hp, double* FRp,
                                                         int64_t ldf) {
    extern __shared__ double lds_base[];
    const int N = m.N, nn = N + 1, ld = nn + 1;
    const Lds L = lds_layout<64>(lds_base, 0, ld);
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const bool sp = lane < N;
    const double y = sp ? Yp[(size_t)lane * ldy + i] : 0.0;
    const double T = wave_temperature(m, y, lane, hp[i]);
    species_state(m, L, y, T, log(T));
    __syncthreads();
    const double fr = source_and_rows<false>(m, L, ld, T, 0.0, nullptr);
    if (sp) FRp[(size_t)lane * ldf + i] = fr;
}

inline unsigned grid_for(int64_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

// [0] solves, [1] iterations, [2] failures, [3] max iterations,
// [4] FP32 refinement solves, [5] FP64 fallbacks (with lu_info); with hist,
// the histogram of the outcomes as well
__global__ void __launch_bounds__(256) wave_stats_kernel(int64_t n, const int32_t* iters,
                                                         const int32_t* lu_info,
                                                         unsigned long long* stats,
                                                         unsigned long long* hist) {
    __shared__ unsigned long long s_sum[4], s_bad[4], s_max[4], s_ref[4], s_fb[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long v = 0, b = 0, mx = 0, rf = 0, fb = 0;
    int32_t itc = 0;
    if (i < n) {
        itc = iters[i];
        v = itc > 0 ? (unsigned long long)itc : 0ull;
        b = itc < 0 ? 1ull : 0ull;
        mx = v;
        if (lu_info) {
            rf = (unsigned long long)(lu_info[i] & 0xffff);
            fb = (unsigned long long)((unsigned)lu_info[i] >> 16);
        }
    }
    if (hist)
        wave_hist_add(hist + (size_t)((blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) %
                                      NEWTON_HIST_SETS) * NEWTON_HIST_BINS,
                      i < n, itc);
    for (int off = 32; off > 0; off >>= 1) {
        v += __shfl_xor(v, off);
        b += __shfl_xor(b, off);
        rf += __shfl_xor(rf, off);
        fb += __shfl_xor(fb, off);
        const unsigned long long o = __shfl_xor(mx, off);
        mx = o > mx ? o : mx;
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) { s_sum[wave] = v; s_bad[wave] = b; s_max[wave] = mx; s_ref[wave] = rf; s_fb[wave] = fb; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long S = 0, B = 0, X = 0, RF = 0, FB = 0;
        for (int w = 0; w < 4; ++w) {
            S += s_sum[w];
            B += s_bad[w];
            RF += s_ref[w];
            FB += s_fb[w];
            X = s_max[w] > X ? s_max[w] : X;
        }
        const int64_t lo = (int64_t)blockIdx.x * blockDim.x;
        const int64_t cnt = (n - lo) < (int64_t)blockDim.x ? (n - lo) : (int64_t)blockDim.x;
        atomicAdd(&stats[0], (unsigned long long)cnt);
        atomicAdd(&stats[1], S);
        atomicAdd(&stats[2], B);
        atomicMax(&stats[3], X);
        if (lu_info) {
            atomicAdd(&stats[4], RF);
            atomicAdd(&stats[5], FB);
        }
    }
}

}  // namespace

int launch_reaction_newton_wave(const Mech& m, const NewtonArgs& a, int lu, hipStream_t s) {
    if (a.n == 0) return MISDC_OK;
    const int N = m.dev.N, n = N + 1, ld = n + 1;
    if (N > 63) return fail(MISDC_EUNSUPPORTED, "wavefront reaction solve: at most 63 species");
    if (lu != NEWTON_LU_FP64 && lu != NEWTON_LU_FP32_MFMA)
        return fail(MISDC_EINVAL, "unknown LU variant %d", lu);
    if (a.n > 0x7fffffffll) return fail(MISDC_EINVAL, "too many cells for one launch");
    const dim3 grid((unsigned)a.n), block(64);
    if (lu == NEWTON_LU_FP32_MFMA) {
        const size_t lds = lds_doubles<64, true>(n, ld) * sizeof(double);
        hipLaunchKernelGGL((newton_wave_kernel<64, 1>), grid, block, lds, s, m.dev, a);
    } else if (n <= 16) {
        const size_t lds = lds_doubles<16, false>(n, ld) * sizeof(double);
        hipLaunchKernelGGL((newton_wave_kernel<16, 0>), grid, block, lds, s, m.dev, a);
    } else if (n <= 32) {
        const size_t lds = lds_doubles<32, false>(n, ld) * sizeof(double);
        hipLaunchKernelGGL((newton_wave_kernel<32, 0>), grid, block, lds, s, m.dev, a);
    } else if (n <= 56) {
        // (the LU runs over NXP columns: the tighter the padding, the fewer)
        const size_t lds = lds_doubles<56, false>(n, ld) * sizeof(double);
        hipLaunchKernelGGL((newton_wave_kernel<56, 0>), grid, block, lds, s, m.dev, a);
    } else {
        const size_t lds = lds_doubles<64, false>(n, ld) * sizeof(double);
        hipLaunchKernelGGL((newton_wave_kernel<64, 0>), grid, block, lds, s, m.dev, a);
    }
    MISDC_HIP(hipGetLastError());
    if (a.stats && a.iters) {
        hipLaunchKernelGGL(wave_stats_kernel, dim3(grid_for(a.n, 256)), dim3(256), 0, s, a.n,
                           a.iters, a.lu_info, a.stats, a.hist);
        MISDC_HIP(hipGetLastError());
    }
    return MISDC_OK;
}

int launch_reaction_source_wave(const Mech& m, int64_t n, const double* Y, int64_t ldy,
                                const double* h, double* FR, int64_t ldf, hipStream_t s) {
    if (n == 0) return MISDC_OK;
    if (m.dev.N > 63) return fail(MISDC_EUNSUPPORTED, "wavefront source: at most 63 species");
    if (n > 0x7fffffffll) return fail(MISDC_EINVAL, "too many cells for one launch");
    const size_t lds = lds_doubles<64, false>(0, m.dev.N + 2) * sizeof(double);
    hipLaunchKernelGGL(source_wave_kernel, dim3((unsigned)n), dim3(64), lds, s, m.dev, n, Y, ldy,
                       h, FR, ldf);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

}  // namespace misdc
