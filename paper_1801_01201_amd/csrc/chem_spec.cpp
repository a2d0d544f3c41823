// Reaction solve of step S5 (eq. reaction_step_numerical_methodology)
// specialised for one mechanism: the host writes the source of a
// one-thread-per-cell Newton kernel in which every rate constant,
// stoichiometric factor and thermodynamic coefficient is a literal and every
// species index is resolved at generation time, compiles it for the device
// with hiprtc and launches it through the module API.
//
// What specialisation buys over the generic per-thread kernel:
//  - the reactions are straight-line code, so the compiler interleaves the
//    exponentials of independent reactions instead of running one reaction's
//    dependent chain after another (one wavefront per SIMD at 65,536 cells
//    leaves no other latency hiding);
//  - the Jacobian of reaction j only touches the rows and columns of its
//    (at most four) slot species, a 4 x 5 block, where the generic kernel,
//    whose species indices are runtime values, updates all N x (N+1) entries
//    through selects;
//  - the LU of the Newton matrix pivots on the diagonal when the diagonal
//    entry is at least a tenth of the largest magnitude among the species
//    rows below it in its column (threshold pivoting; the enthalpy row is
//    eliminated last); a cell that fails the test anywhere assembles its
//    matrix again and factors it with partial pivoting.
// The arithmetic is otherwise that of the generic kernel (chem.hip): the same
// residual, pseudo-transient continuation, trial acceptance and convergence
// test, so both agree to the Newton tolerance.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "misdc_impl.h"

namespace misdc {

namespace {

// register budget of the generated kernel (at most 512 / this many VGPRs per
// lane): one cell's 9 x 10 Newton matrix, state and rates need about 260 at
// the peak, so a budget of two wavefronts per SIMD spills; one wavefront per
// SIMD is what 65,536 cells fill anyway
constexpr int NEWTON_SPEC_WAVES_PER_EU = 1;

// While a constant pool is active, the mechanism's constants go into a
// generated __constant__ table KC read at KC[kz + i], where kz is a zero the
// compiler cannot see through, produced afresh in every Newton iteration: the
// loads then stay inside the iteration (scalar loads from the constant cache)
// instead of some two hundred 64-bit literals being hoisted out of the loop
// into registers that the iteration itself needs.
struct ConstPool {
    std::vector<double> v;
    std::map<unsigned long long, int> at;
};
thread_local ConstPool* g_pool = nullptr;

// exact decimal-free literal of a double, or its slot in the active pool
std::string lit(double v) {
    char buf[64];
    if (v == 0.0) return "0.0";
    if (g_pool && v != 1.0 && v != -1.0 && v != 2.0 && v != -2.0) {
        unsigned long long bits;
        std::memcpy(&bits, &v, sizeof(bits));
        auto it = g_pool->at.find(bits);
        int idx;
        if (it == g_pool->at.end()) {
            idx = (int)g_pool->v.size();
            g_pool->v.push_back(v);
            g_pool->at[bits] = idx;
        } else {
            idx = it->second;
        }
        std::snprintf(buf, sizeof(buf), "KC[kz + %d]", idx);
        return buf;
    }
    std::snprintf(buf, sizeof(buf), "%a", v);
    return std::string("(") + buf + ")";
}

void emit(std::string& s, const char* fmt, ...) {
    char buf[4096];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    s += buf;
}

// Device-side helpers shared by every generated kernel (plain text: the
// generated program includes nothing; hiprtc supplies the HIP device API).
const char* kPrelude = R"(
typedef long long i64;
typedef unsigned long long u64;

// LU with partial pivoting of the augmented n x (n+1) matrix held in
// registers (compile-time indices only); column n becomes the solution
template <int n>
__device__ __forceinline__ void lu_pivoted(double (&A)[n][n + 1]) {
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

// LU on the diagonal pivots, refused (returns false) when a pivot is below a
// tenth of the largest magnitude among the species rows below it in its
// column, or is not finite and non-zero.  The last row (the enthalpy
// equation, whose entries h_k / cp are thousands of kelvin against the O(1)
// species diagonals) is never a candidate: it is eliminated last, and its
// own final pivot is the Schur complement of the species block.
template <int n>
__device__ __forceinline__ bool lu_threshold(double (&A)[n][n + 1]) {
    bool ok = true;
#pragma unroll
    for (int c = 0; c < n; ++c) {
        double amax = 0.0;
#pragma unroll
        for (int r = c + 1; r < n - 1; ++r) amax = fmax(amax, fabs(A[r][c]));
        ok = ok && (fabs(A[c][c]) >= 0.1 * amax) && (A[c][c] != 0.0) && isfinite(A[c][c]);
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
    return ok;
}

// outcome histogram of the wavefront's valid lanes (one atomic per distinct bin)
__device__ __forceinline__ void wave_hist(u64* set, bool valid, int code) {
    const int bin = code <= 0 ? 0 : (code < 63 ? code : 63);
    u64 rem = __ballot(valid);
    while (rem) {
        const int lead = __ffsll((long long)rem) - 1;
        const int b = __shfl(bin, lead);
        const u64 same = __ballot(valid && bin == b);
        if ((threadIdx.x & 63) == 0) atomicAdd(&set[b], (u64)__popcll(same));
        rem &= ~same;
    }
}
)";

struct MechHost {
    int N = 0, R = 0, bath = 0;
    std::vector<int> slots;              // R x 4
    std::vector<double> A, beta, Ta, dn, uW, W, invW, cp, hf, s0;
    double rho0 = 0, R_u = 0, newton_scale = 0, ln_patm_over_Ru = 0;
};

// Rates (and with jac the Jacobian) at the state (y0.., T): defines FR<k>
// for every species and, with jac, accumulates d FR_k / d Y_l into the
// expression jname(k, l) and d FR_k / d T into jname(k, -1), which the
// caller has zeroed (entries of the Newton matrix: the Jacobian is formed in
// place, so it and the matrix are never live at once).
template <class JName>
void emit_rates(std::string& s, const MechHost& m, bool jac, JName jname) {
    const int N = m.N;
    emit(s, "        const double lnT = log(T), invT = 1.0 / T, lnTr = lnT - %s;\n",
         lit(std::log(T_REF)).c_str());
    emit(s, "        const double invRuT = 1.0 / (%s * T), ln_c0 = %s - lnT;\n", lit(m.R_u).c_str(),
         lit(m.ln_patm_over_Ru).c_str());
    // with constant heat capacities a reaction's sums of nu h_k and nu g_k are
    // linear in (1, T - T_ref, T ln(T / T_ref), T) with constant coefficients
    emit(s, "        const double tm = T - %s, tl = T * lnTr;\n", lit(T_REF).c_str());
    std::vector<bool> used(N, false);
    for (int j = 0; j < m.R; ++j)
        for (int q = 0; q < 4; ++q)
            if (m.slots[4 * j + q] >= 0) used[m.slots[4 * j + q]] = true;
    for (int k = 0; k < N; ++k) {
        emit(s, "        double FR%d = 0.0;\n", k);
        if (!used[k]) continue;
        emit(s, "        const double X%d = %s * y%d;\n", k, lit(m.rho0 * m.invW[k]).c_str(), k);
    }
    for (int j = 0; j < m.R; ++j) {
        if (m.A[j] == 0.0) continue;
        const int* sl = &m.slots[4 * j];
        // net stoichiometric coefficient of species k (products - reactants)
        auto nu = [&](int k) {
            return (sl[2] == k) + (sl[3] == k) - (sl[0] == k) - (sl[1] == k);
        };
        std::vector<int> sp;                       // distinct slot species
        for (int q = 0; q < 4; ++q)
            if (sl[q] >= 0 && std::find(sp.begin(), sp.end(), sl[q]) == sp.end()) sp.push_back(sl[q]);
        emit(s, "        {   // reaction %d\n", j);
        std::string kfarg = lit(std::log(m.A[j]));
        if (m.beta[j] != 0.0) kfarg += " + " + lit(m.beta[j]) + " * lnT";
        if (m.Ta[j] != 0.0) kfarg += " - " + lit(m.Ta[j]) + " * invT";
        emit(s, "            const double kf = exp(%s);\n", kfarg.c_str());
        // sum nu h = a + cc tm, sum nu g = sum nu h - T (sum nu s0) - cc tl, with
        // h_k = hf_k + cp_k (T - T_ref) and g_k = h_k - T (s0_k + cp_k ln(T / T_ref))
        double ca = 0.0, cs = 0.0, cc = 0.0;
        for (int k : sp) {
            const int v = nu(k);
            ca += v * m.hf[k];
            cs += v * m.s0[k];
            cc += v * m.cp[k];
        }
        emit(s, "            const double sh = %s + %s * tm;\n", lit(ca).c_str(), lit(cc).c_str());
        const std::string sg = "sh - " + lit(cs) + " * T - " + lit(cc) + " * tl";
        // kr = kf / Kc, ln Kc = -sum(nu g) / (R_u T) + dn ln(p_atm / (R_u T))
        emit(s, "            const double kr = kf * exp((%s) * invRuT - %s * ln_c0);\n", sg.c_str(),
             lit(m.dn[j]).c_str());
        auto prod2 = [&](int a, int b) {
            std::string r;
            if (a >= 0) r = "X" + std::to_string(a);
            if (b >= 0) r += (r.empty() ? "" : " * ") + std::string("X") + std::to_string(b);
            return r.empty() ? std::string("1.0") : r;
        };
        emit(s, "            const double pf = %s, pr = %s;\n", prod2(sl[0], sl[1]).c_str(),
             prod2(sl[2], sl[3]).c_str());
        emit(s, "            const double q = kf * pf - kr * pr;\n");
        if (jac) {
            emit(s, "            const double dlnkf = %s * invT + %s * invT * invT;\n",
                 lit(m.beta[j]).c_str(), lit(m.Ta[j]).c_str());
            emit(s, "            const double dlnKc = sh * invRuT * invT - %s * invT;\n",
                 lit(m.dn[j]).c_str());
            emit(s, "            const double dqdT = kf * dlnkf * pf - kr * (dlnkf - dlnKc) * pr;\n");
            // d q / d X_l: each slot occurrence contributes the product of the other slot
            for (int l : sp) {
                std::string d;
                auto add = [&](const std::string& t) { d += (d.empty() ? "" : " + ") + t; };
                if (sl[0] == l) add("kf * " + (sl[1] >= 0 ? "X" + std::to_string(sl[1]) : std::string("1.0")));
                if (sl[1] == l) add("kf * " + (sl[0] >= 0 ? "X" + std::to_string(sl[0]) : std::string("1.0")));
                if (sl[2] == l) add("-kr * " + (sl[3] >= 0 ? "X" + std::to_string(sl[3]) : std::string("1.0")));
                if (sl[3] == l) add("-kr * " + (sl[2] >= 0 ? "X" + std::to_string(sl[2]) : std::string("1.0")));
                emit(s, "            const double v%d = (%s) * %s;\n", l, d.c_str(),
                     lit(m.rho0 * m.invW[l]).c_str());
            }
        }
        for (int k : sp) {
            const double u = m.uW[(size_t)j * N + k];
            if (u == 0.0) continue;
            emit(s, "            FR%d += %s * q;\n", k, lit(u).c_str());
            if (jac) {
                emit(s, "            %s += %s * dqdT;\n", jname(k, -1).c_str(), lit(u).c_str());
                for (int l : sp)
                    emit(s, "            %s += %s * v%d;\n", jname(k, l).c_str(), lit(u).c_str(), l);
            }
        }
        emit(s, "        }\n");
    }
}

std::string generate(const MechHost& m) {
    const int N = m.N, b = m.bath;
    std::vector<int> rs;                             // reacting species (all but the bath)
    for (int k = 0; k < N; ++k)
        if (k != b) rs.push_back(k);
    const int NR = (int)rs.size(), NX = NR + 1;
    std::string s = kPrelude;
    emit(s, "\nconstexpr int NS = %d, NX = %d;\n", N, NX);
    // temperature from (Y, h): constant heat capacities
    s += "__device__ __forceinline__ double temperature_of(const double (&y)[NS], double h) {\n"
         "    double hform = 0.0, cpm = 0.0;\n";
    for (int k = 0; k < N; ++k)
        emit(s, "    hform += y[%d] * %s; cpm += y[%d] * %s;\n", k, lit(m.hf[k] * m.invW[k]).c_str(),
             k, lit(m.cp[k] * m.invW[k]).c_str());
    emit(s, "    return %s + (h - hform) / cpm;\n}\n", lit(T_REF).c_str());

    // Newton matrix [M | G] at (y, T), with the bath's update db eliminated
    ConstPool pool;
    g_pool = &pool;
    std::string body;
    std::string& outer = s;
    {
    std::string& s = body;
    s += "__device__ __forceinline__ void assemble(const double (&Y)[NS], double T, double h, double c,\n"
         "        double inv_dtau, const double* bY, i64 ldb, i64 i, double (&M)[NX][NX + 1],\n"
         "        double& gn2, double& db, int kz) {\n";
    for (int k = 0; k < N; ++k) emit(s, "        const double y%d = Y[%d];\n", k, k);
    // position of each reacting species in the system; the bath has none
    std::vector<int> pos(N, -1);
    for (int i = 0; i < NR; ++i) pos[rs[i]] = i;
    s += "#pragma unroll\n"
         "        for (int r = 0; r < NX; ++r)\n"
         "#pragma unroll\n"
         "            for (int q = 0; q <= NX; ++q) M[r][q] = 0.0;\n";
    // the Jacobian goes into rows and columns of M; column NR holds d/dT
    emit_rates(s, m, true, [&](int k, int l) {
        char t[48];
        std::snprintf(t, sizeof(t), "M[%d][%d]", pos[k], l < 0 ? NR : pos[l]);
        return std::string(t);
    });
    const double inv_scale = 1.0 / m.newton_scale;
    emit(s, "        double hsum = 0.0, cpm = 0.0;\n");
    for (int k = 0; k < N; ++k) {
        emit(s, "        const double hk%d = (%s + %s * (T - %s)) * %s;\n", k, lit(m.hf[k]).c_str(),
             lit(m.cp[k]).c_str(), lit(T_REF).c_str(), lit(m.invW[k]).c_str());
        emit(s, "        hsum += y%d * hk%d; cpm += y%d * %s;\n", k, k, k, lit(m.cp[k] * m.invW[k]).c_str());
    }
    for (int i = 0; i < NR; ++i) {
        const int k = rs[i];
        emit(s, "        M[%d][NX] = y%d - c * FR%d - bY[(i64)%d * ldb + i];\n", i, k, k, k);
        emit(s, "#pragma unroll\n        for (int q = 0; q <= %d; ++q) M[%d][q] *= -c;\n", NR, i);
        emit(s, "        M[%d][%d] += 1.0 + inv_dtau;\n", i, i);
        emit(s, "        M[%d][%d] = hk%d * %s;\n", NR, i, k, lit(inv_scale).c_str());
    }
    emit(s, "        M[%d][%d] = cpm * %s + inv_dtau;\n", NR, NR, lit(inv_scale).c_str());
    emit(s, "        const double Gb = y%d - bY[(i64)%d * ldb + i];\n", b, b);
    emit(s, "        M[%d][NX] = (hsum - h) * %s;\n", NR, lit(inv_scale).c_str());
    s += "        gn2 = Gb * Gb;\n"
         "#pragma unroll\n"
         "        for (int r = 0; r < NX; ++r) gn2 += M[r][NX] * M[r][NX];\n";
    emit(s, "        db = Gb / (1.0 + inv_dtau);\n");
    emit(s, "        M[%d][NX] -= hk%d * %s * db;\n", NR, b, lit(inv_scale).c_str());
    s += "}\n";

    // rates only, at the final state
    s += "__device__ __forceinline__ void source(const double (&Y)[NS], double T, double (&F)[NS],\n"
         "                                       int kz) {\n";
    for (int k = 0; k < N; ++k) emit(s, "        const double y%d = Y[%d];\n", k, k);
    emit_rates(s, m, false, [](int, int) { return std::string(); });
    for (int k = 0; k < N; ++k) emit(s, "        F[%d] = FR%d;\n", k, k);
    s += "}\n";
    }
    g_pool = nullptr;
    outer += "__constant__ double KC[" + std::to_string(pool.v.size() ? pool.v.size() : 1) + "] = {";
    for (size_t k = 0; k < pool.v.size(); ++k) {
        char t[40];
        std::snprintf(t, sizeof(t), "%a%s", pool.v[k], k + 1 < pool.v.size() ? ", " : "");
        outer += t;
        if (k % 4 == 3) outer += "\n    ";
    }
    if (pool.v.empty()) outer += "0.0";
    outer += "};\n";
    outer += body;

    // the Newton update of every species from the solved system
    s += "__device__ __forceinline__ void update(const double (&M)[NX][NX + 1], double db,\n"
         "                                       double (&D)[NS]) {\n";
    for (int q = 0; q < NR; ++q) emit(s, "    D[%d] = M[%d][NX];\n", rs[q], q);
    emit(s, "    D[%d] = db;\n}\n", b);
    emit(s, "#define WAVES_PER_EU %d\n", NEWTON_SPEC_WAVES_PER_EU);
    emit(s, "constexpr double T_DIFF_REF = %.17g, THETA_EXP = %.17g;\n", T_DIFF_REF, THETA_EXP);
    emit(s, "constexpr int TILE_X = %d, TILE_Y = %d;\n", NEWTON_TILE_X, NEWTON_TILE_Y);
    emit(s, "constexpr int BUCKETS = %d, BUCKET_STRIDE = %d, HIST_SETS = %d, HIST_BINS = %d;\n",
         NEWTON_BUCKETS, NEWTON_BUCKET_STRIDE, NEWTON_HIST_SETS, NEWTON_HIST_BINS);
    // the kernel: the loop of the generic per-thread kernel
    s += R"(
extern "C" __global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WAVES_PER_EU)))
newton_spec(
        i64 n, const double* bY, i64 ldb, const double* hp, const double* cp, double c_scalar,
        const double* guess, i64 ldg, double* Yo, i64 ldy, double* To, double* Ho, double* Tho, double* FRo, i64 ldf,
        int* iters, u64* buckets, u64* hist, int tile_nx, int tile_ny, double tol, int maxit,
        double dtau0, double dtau_max, double neg_slack) {
    i64 i;
    if (tile_nx > 0) {
        const int ntx = (tile_nx + TILE_X - 1) / TILE_X;
        const int x = (int)(blockIdx.x % ntx) * TILE_X + (int)(threadIdx.x % TILE_X);
        const int y = (int)(blockIdx.x / ntx) * TILE_Y + (int)(threadIdx.x / TILE_X);
        i = (x < tile_nx && y < tile_ny) ? (i64)y * tile_nx + x : n;
    } else {
        i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    }
    int code = 0, retries = 0;
    if (i < n) {
        const double c = cp ? cp[i] * c_scalar : c_scalar;
        const double h = hp[i];
        double Y[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) Y[k] = guess[(i64)k * ldg + i];
        double T = temperature_of(Y, h);
        double inv_dtau = 0.0, gnorm_old = -1.0;
        int it = 0;
        retries = 0;
        bool conv = false;
        while (!conv && it < maxit) {
            double M[NX][NX + 1];
            double gn2, db;
            // diagonal pivots first; a cell whose pivots fail the threshold
            // assembles again and pivots partially
            for (int attempt = 0; attempt < 2; ++attempt) {
                int kz;
                asm volatile("s_mov_b32 %0, 0" : "=s"(kz));
                assemble(Y, T, h, c, inv_dtau, bY, ldb, i, M, gn2, db, kz);
                if (attempt == 0) {
                    if (lu_threshold<NX>(M)) break;
                } else {
                    lu_pivoted<NX>(M);
                    ++retries;
                }
            }
            double D[NS];
            update(M, db, D);
            const double dT = M[NX - 1][NX];
            ++it;
            bool ok = true;
            double dmax = 0.0, Yt[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                Yt[k] = Y[k] - D[k];
                const double lo = fmin(bY[(i64)k * ldb + i], 0.0) - neg_slack;
                ok = ok && isfinite(D[k]) && (Yt[k] >= lo);
                dmax = fmax(dmax, fabs(D[k]));
            }
            const double Tt = T - dT;
            ok = ok && isfinite(dT) && (Tt > 0.0);
            if (!ok) {
                inv_dtau = (inv_dtau == 0.0) ? 1.0 / dtau0 : inv_dtau * 4.0;
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
                if (inv_dtau < 1.0 / dtau_max) inv_dtau = 0.0;
            }
            gnorm_old = gnorm;
            conv = was_newton && (dmax <= tol) && (fabs(dT) <= tol * fabs(Tt));
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) Yo[(i64)k * ldy + i] = Y[k];
        const double Tc = temperature_of(Y, h);
        if (To) To[i] = Tc;
        if (Ho) Ho[i] = h;
        if (Tho) Tho[i] = pow(Tc / T_DIFF_REF, THETA_EXP);
        if (FRo) {
            double F[NS];
            int kz;
            asm volatile("s_mov_b32 %0, 0" : "=s"(kz));
            source(Y, Tc, F, kz);
#pragma unroll
            for (int k = 0; k < NS; ++k) FRo[(i64)k * ldf + i] = F[k];
        }
        code = conv ? it : -1;
        if (iters) iters[i] = code;
    }
    if (buckets) {
        int solves = (i < n) ? 1 : 0, sum = code > 0 ? code : 0, bad = code < 0 ? 1 : 0, mx = sum;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            solves += __shfl_xor(solves, off);
            sum += __shfl_xor(sum, off);
            bad += __shfl_xor(bad, off);
            retries += __shfl_xor(retries, off);
            const int o = __shfl_xor(mx, off);
            mx = o > mx ? o : mx;
        }
        const unsigned w = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
        if ((threadIdx.x & 63) == 0) {
            u64* bk = buckets + (size_t)(w % BUCKETS) * BUCKET_STRIDE;
            atomicAdd(&bk[0], (u64)solves);
            atomicAdd(&bk[1], (u64)sum);
            if (bad) atomicAdd(&bk[2], (u64)bad);
            atomicMax(&bk[3], (u64)mx);
            if (retries) atomicAdd(&bk[4], (u64)retries);
        }
        if (hist) wave_hist(hist + (size_t)(w % HIST_SETS) * HIST_BINS, i < n, code);
    }
}
)";
    return s;
}

struct SpecModule {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
};
std::mutex g_spec_mu;
// (device, generated source) -> loaded module; kept until the process ends
std::map<std::pair<int, std::string>, SpecModule> g_spec;

int compile(const std::string& src, std::string& msg, std::vector<char>& code) {
    hiprtcProgram prog = nullptr;
    if (hiprtcCreateProgram(&prog, src.c_str(), "newton_spec.hip", 0, nullptr, nullptr) !=
        HIPRTC_SUCCESS) {
        msg = "hiprtcCreateProgram failed";
        return -1;
    }
    // packed FP32 instructions off, as for the library's own device code
    const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                          "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        (void)hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) (void)hiprtcGetProgramLog(prog, &log[0]);
        msg = std::string("hiprtc: ") + hiprtcGetErrorString(rc) + "\n" + log.substr(0, 2000);
        (void)hiprtcDestroyProgram(&prog);
        return -1;
    }
    size_t n = 0;
    if (hiprtcGetCodeSize(prog, &n) != HIPRTC_SUCCESS || n == 0) {
        msg = "hiprtc: no code";
        (void)hiprtcDestroyProgram(&prog);
        return -1;
    }
    code.resize(n);
    const hiprtcResult gc = hiprtcGetCode(prog, code.data());
    (void)hiprtcDestroyProgram(&prog);
    if (gc != HIPRTC_SUCCESS) {
        msg = "hiprtc: code not retrieved";
        return -1;
    }
    return 0;
}

}  // namespace

int newton_spec_prepare(Mech& m, const MechTables& t) {
    m.spec_fn = nullptr;
    if (t.N > NEWTON_SPEC_MAX_SPECIES) {
        m.spec_status = "not generated: more species than the register-resident kernel holds";
        return MISDC_OK;
    }
    MechHost h;
    h.N = t.N;
    h.R = t.R;
    h.bath = t.bath;
    h.slots = t.slots;
    h.A = t.A;
    h.beta = t.beta;
    h.Ta = t.Ta;
    h.dn = t.dn;
    h.uW = t.uW;
    h.W = t.W;
    h.invW = t.invW;
    h.cp = t.cp;
    h.hf = t.hf;
    h.s0 = t.s0;
    h.rho0 = t.rho0;
    h.R_u = t.R_u;
    h.newton_scale = t.newton_scale;
    h.ln_patm_over_Ru = t.ln_patm_over_Ru;
    for (int j = 0; j < h.R; ++j)
        if (!(h.A[j] >= 0.0)) {
            m.spec_status = "not generated: negative pre-exponential factor";
            return MISDC_OK;
        }
    const std::string src = generate(h);
    std::lock_guard<std::mutex> lock(g_spec_mu);
    auto key = std::make_pair(m.device, src);
    auto it = g_spec.find(key);
    if (it == g_spec.end()) {
        std::vector<char> code;
        std::string msg;
        if (compile(src, msg, code) != 0) {
            m.spec_status = "not generated: " + msg;
            return MISDC_OK;           // the generic kernel serves
        }
        SpecModule sm;
        hipError_t e = hipModuleLoadData(&sm.mod, code.data());
        if (e == hipSuccess) e = hipModuleGetFunction(&sm.fn, sm.mod, "newton_spec");
        if (e != hipSuccess) {
            m.spec_status = std::string("not loaded: ") + hipGetErrorString(e);
            return MISDC_OK;
        }
        it = g_spec.emplace(key, sm).first;
    }
    m.spec_fn = (void*)it->second.fn;
    m.spec_status = "specialised kernel ready";
    return MISDC_OK;
}

int launch_newton_spec(const Mech& m, const NewtonArgs& a, hipStream_t s) {
    if (!m.spec_fn) return fail(MISDC_EUNSUPPORTED, "no specialised reaction solve: %s",
                                m.spec_status.c_str());
    int64_t blocks = (a.n + 63) / 64;
    if (a.tile_nx > 0) {
        if (a.tile_ny <= 0 || (int64_t)a.tile_nx * a.tile_ny != a.n)
            return fail(MISDC_EINVAL, "tiled reaction solve: %d x %d cells for n = %lld", a.tile_nx,
                        a.tile_ny, (long long)a.n);
        blocks = (int64_t)((a.tile_nx + NEWTON_TILE_X - 1) / NEWTON_TILE_X) *
                 ((a.tile_ny + NEWTON_TILE_Y - 1) / NEWTON_TILE_Y);
    }
    if (blocks > 0x7fffffffll) return fail(MISDC_EINVAL, "too many cells for one launch");
    int64_t n = a.n, ldb = a.ldb, ldg = a.ldg, ldy = a.ldy, ldf = a.ldf;
    const double* bY = a.bY;
    const double* hp = a.h;
    const double* cp = a.c;
    double c_scalar = a.c_scalar;
    const double* guess = a.guess;
    double* Yo = a.Y;
    double* To = a.T;
    double* Ho = a.h_out;
    double* Tho = a.th_out;
    double* FRo = a.FR;
    int* iters = a.iters;
    unsigned long long* buckets = a.buckets;
    unsigned long long* hist = a.buckets ? a.hist : nullptr;
    int tnx = a.tile_nx, tny = a.tile_ny;
    double tol = a.opt.tol, dtau0 = a.opt.dtau0, dtau_max = a.opt.dtau_max, slack = a.opt.neg_slack;
    int maxit = a.opt.maxit;
    void* args[] = {&n, &bY, &ldb, &hp, &cp, &c_scalar, &guess, &ldg, &Yo, &ldy, &To, &Ho, &Tho, &FRo, &ldf,
                    &iters, &buckets, &hist, &tnx, &tny, &tol, &maxit, &dtau0, &dtau_max, &slack};
    MISDC_HIP(hipModuleLaunchKernel((hipFunction_t)m.spec_fn, (unsigned)blocks, 1, 1, 64, 1, 1, 0,
                                    s, args, nullptr));
    return MISDC_OK;
}

int newton_spec_compile_check(const std::string& src, std::string& msg) {
    std::vector<char> code;
    return compile(src, msg, code);
}

// Source text of the kernel for a mechanism (tests and inspection).
std::string newton_spec_source(const MechTables& t) {
    MechHost h;
    h.N = t.N;
    h.R = t.R;
    h.bath = t.bath;
    h.slots = t.slots;
    h.A = t.A;
    h.beta = t.beta;
    h.Ta = t.Ta;
    h.dn = t.dn;
    h.uW = t.uW;
    h.W = t.W;
    h.invW = t.invW;
    h.cp = t.cp;
    h.hf = t.hf;
    h.s0 = t.s0;
    h.rho0 = t.rho0;
    h.R_u = t.R_u;
    h.newton_scale = t.newton_scale;
    h.ln_patm_over_Ru = t.ln_patm_over_Ru;
    return generate(h);
}

}  // namespace misdc
