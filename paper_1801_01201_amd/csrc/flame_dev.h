// Device code of the transport operators and the 1-D implicit diffusion
// solves, per cell or per system, shared by the kernels of transport.hip and
// the persistent ensemble stage kernel (ensemble.hip).
#pragma once

#include "misdc_impl.h"

namespace misdc {

struct GridDev {
    int dim;
    int64_t nx, ny;
    double dx, dy, ux, uy;
    int n_flames;
    const int64_t* off;     // ensemble: flame offsets (n_flames + 1)
    const double* fdx;
    const double* fu;
};

// neighbour index along x with periodic wrap inside the row (or the flame)
struct Row {
    int64_t base, len, pos;
    double dx, u;
};

__device__ __forceinline__ int64_t wrap(int64_t k, int64_t len) {
    // the neighbours of a position in [0, len) lie within one period: no
    // 64-bit remainder (a long instruction sequence) unless len < 2
    if (k >= -len && k < 2 * len) return k < 0 ? k + len : (k >= len ? k - len : k);
    k %= len;
    return k < 0 ? k + len : k;
}

__device__ __forceinline__ Row row_of(const GridDev& g, int64_t i) {
    Row r;
    if (g.n_flames > 0) {
        int lo = 0, hi = g.n_flames;           // find f with off[f] <= i < off[f+1]
        while (hi - lo > 1) {
            const int mid = (lo + hi) / 2;
            if (g.off[mid] <= i) lo = mid; else hi = mid;
        }
        r.base = g.off[lo];
        r.len = g.off[lo + 1] - g.off[lo];
        r.pos = i - r.base;
        r.dx = g.fdx[lo];
        r.u = g.fu[lo];
    } else {
        r.len = g.nx;
        r.pos = i % g.nx;
        r.base = i - r.pos;
        r.dx = g.dx;
        r.u = g.ux;
    }
    return r;
}

// The explicit operators' stencil at one cell: the four neighbours along x
// (periodic in the row or flame) and along y (2-D grids), the advection
// factors u/dx, and the face coefficients theta_face / dx^2 (mean of the two
// cells' theta) of the diffusion operator of eqs. `species_equation` and
// `enthalpy_equation`.
struct Stencil {
    int64_t xm2, xm1, xp1, xp2, ym2, ym1, yp1, yp2;
    bool two_d;
    double ax, ay, kxe, kxw, kyn, kys;
};

template <class Theta>
__device__ __forceinline__ Stencil stencil_at(const GridDev& g, int64_t i, double t0, Theta theta) {
    Stencil s;
    const Row r = row_of(g, i);
    s.xm2 = r.base + wrap(r.pos - 2, r.len);
    s.xm1 = r.base + wrap(r.pos - 1, r.len);
    s.xp1 = r.base + wrap(r.pos + 1, r.len);
    s.xp2 = r.base + wrap(r.pos + 2, r.len);
    s.ym2 = s.ym1 = s.yp1 = s.yp2 = 0;
    s.two_d = (g.dim == 2 && g.n_flames == 0);
    if (s.two_d) {
        const int64_t iy = i / g.nx, ix = i - iy * g.nx;
        s.ym2 = wrap(iy - 2, g.ny) * g.nx + ix;
        s.ym1 = wrap(iy - 1, g.ny) * g.nx + ix;
        s.yp1 = wrap(iy + 1, g.ny) * g.nx + ix;
        s.yp2 = wrap(iy + 2, g.ny) * g.nx + ix;
    }
    const double idx2 = 1.0 / (r.dx * r.dx);
    s.kxe = 0.5 * (t0 + theta(s.xp1)) * idx2;
    s.kxw = 0.5 * (t0 + theta(s.xm1)) * idx2;
    s.kyn = s.kys = 0.0;
    if (s.two_d) {
        const double idy2 = 1.0 / (g.dy * g.dy);
        s.kyn = 0.5 * (t0 + theta(s.yp1)) * idy2;
        s.kys = 0.5 * (t0 + theta(s.ym1)) * idy2;
    }
    s.ax = r.u / r.dx;
    s.ay = s.two_d ? g.uy / g.dy : 0.0;
    return s;
}

// the stencil values of one field p at cell i: c0, then x-1, x-2, x+1, x+2,
// then (TWO_D) y-1, y-2, y+1, y+2
template <bool TWO_D>
__device__ __forceinline__ void load_stencil(const Stencil& s, const double* p, int64_t i,
                                             double (&v)[9]) {
    v[0] = p[i];
    v[1] = p[s.xm1];
    v[2] = p[s.xm2];
    v[3] = p[s.xp1];
    v[4] = p[s.xp2];
    if (TWO_D) {
        v[5] = p[s.ym1];
        v[6] = p[s.ym2];
        v[7] = p[s.yp1];
        v[8] = p[s.yp2];
    }
}

// advection -div(u phi) with fourth-order face values, and div(theta grad phi)
// (the diffusion operator without kappa0), from one field's stencil values
template <bool TWO_D>
__device__ __forceinline__ void field_ops(const Stencil& s, const double (&v)[9], double& fa,
                                          double& lap) {
    const double c0 = v[0], w1 = v[1], w2 = v[2], e1 = v[3], e2 = v[4];
    // fourth-order face values at i+1/2 and i-1/2
    const double fe = (7.0 * (c0 + e1) - (w1 + e2)) / 12.0;
    const double fw = (7.0 * (w1 + c0) - (w2 + e1)) / 12.0;
    fa = -s.ax * (fe - fw);
    lap = s.kxe * (e1 - c0) - s.kxw * (c0 - w1);
    if (TWO_D) {
        const double s1 = v[5], s2 = v[6], n1 = v[7], n2 = v[8];
        const double fn = (7.0 * (c0 + n1) - (s1 + n2)) / 12.0;
        const double fs = (7.0 * (s1 + c0) - (s2 + n1)) / 12.0;
        if (s.ay != 0.0) fa -= s.ay * (fn - fs);
        lap += s.kyn * (n1 - c0) - s.kys * (c0 - s1);
    }
}

// FA and FD of every field at cell i from the stencil s, CH fields at a time:
// a chunk's stencil values are all loaded before any of its results is
// stored, so that a chunk waits for memory once rather than once per field
// (the kernel is bound by that latency: one thread per cell, one wavefront
// per SIMD).  FD of the bath species is minus the sum of the other species'.
template <int CH, bool TWO_D>
__device__ __forceinline__ void transport_fields(const Stencil& s, const MechDev& m, int64_t n,
                                                 const double* st, double* FA, double* FD,
                                                 int64_t i) {
    const int NF = m.N + 1;
    double fd_sum = 0.0;
    for (int f0 = 0; f0 < NF; f0 += CH) {
        double v[CH][9];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            // past the last field a chunk reloads that field, so every load
            // stays in bounds and none sits behind a branch
            const int f = f0 + c < NF ? f0 + c : NF - 1;
            load_stencil<TWO_D>(s, st + (size_t)f * n, i, v[c]);
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int f = f0 + c;
            if (f >= NF) continue;
            double fa, lap;
            field_ops<TWO_D>(s, v[c], fa, lap);
            if (FA) FA[(size_t)f * n + i] = fa;
            if (FD && f != m.bath) {
                const double fd = m.kappa0[f] * lap;
                FD[(size_t)f * n + i] = fd;
                if (f < m.N) fd_sum += fd;
            }
        }
    }
    if (FD) FD[(size_t)m.bath * n + i] = -fd_sum;
}

// FA and FD for every field of one cell.  FROM_T: theta = (T/300)^1.7 of the
// cell and its neighbours is computed here from T (and the cell's own value
// stored in th) instead of being read from th.  CH: fields per chunk of
// loads (see transport_fields).
template <bool FROM_T, int CH = 1>
__device__ __forceinline__ void transport_cell(const GridDev& g, const MechDev& m, int64_t n,
                                               const double* st, const double* T, double* th,
                                               double* FA, double* FD, int64_t i) {
    auto theta = [&](int64_t j) {
        return FROM_T ? pow(T[j] / T_DIFF_REF, THETA_EXP) : th[j];
    };
    const double t0 = theta(i);
    if (FROM_T) th[i] = t0;
    const Stencil s = stencil_at(g, i, t0, theta);
    if (s.two_d)
        transport_fields<CH, true>(s, m, n, st, FA, FD, i);
    else
        transport_fields<CH, false>(s, m, n, st, FA, FD, i);
}

// face coefficients of the lagged operator: Kx[i] = east face / dx^2, Ky[i] =
// north face / dy^2, both from theta = (T_lag/300)^1.7.
__device__ __forceinline__ void faces_at(const GridDev& g, int64_t i, const double* T, double* th,
                                         double* Kx, double* Ky) {
    const Row r = row_of(g, i);
    const int64_t xp1 = r.base + wrap(r.pos + 1, r.len);
    const double t0 = pow(T[i] / T_DIFF_REF, THETA_EXP);
    const double t1 = pow(T[xp1] / T_DIFF_REF, THETA_EXP);
    th[i] = t0;
    Kx[i] = 0.5 * (t0 + t1) / (r.dx * r.dx);
    if (g.dim == 2 && g.n_flames == 0) {
        const int64_t iy = i / g.nx, ix = i - iy * g.nx;
        const int64_t yp1 = wrap(iy + 1, g.ny) * g.nx + ix;
        const double t2 = pow(T[yp1] / T_DIFF_REF, THETA_EXP);
        Ky[i] = 0.5 * (t0 + t2) / (g.dy * g.dy);
    }
}

// Periodic tridiagonal solve with one wavefront per system (partition
// method).  The system of length L is cut into P = min(64, L) chunks of
// consecutive rows; the last row of every chunk is a separator.  Lane p
// eliminates the interior rows of its chunk with Thomas' algorithm for three
// right-hand sides (the load and the couplings to the separators on either
// side), so that each interior unknown is u - v G_{p-1} - w G_p in terms of
// the separator unknowns G.  Substituting into the separator rows leaves a
// periodic tridiagonal system of P unknowns (diagonally dominant, as a Schur
// complement of a diagonally dominant matrix), which lane 0 solves; every
// lane then recovers its interior rows.  The serial depth is about
// 2 L / 64 + 2 P instead of 3 L.  Scratch arrays sc, su, sv, sw hold the
// interior rows of lane p at position k P + p of the system's range.
__device__ __forceinline__ void cyclic_wave_system(const GridDev& g, const MechDev& m, int64_t n,
                                                   double c, const double* dtf, double cfac,
                                                   const double* Kx, const double* rhs, double* y,
                                                   double* sc, double* su, double* sv, double* sw,
                                                   int f, int fl) {
    __shared__ double ra[64], rb[64], rcs[64], rr[64];   // reduced system
    __shared__ double fu[64], fv[64], fw[64];            // first interior row of each chunk
    __shared__ double G[64], wc[64], wu[64];
    if (f == m.bath || f > m.N) return;     // uniform over the wavefront
    const int64_t base = g.n_flames > 0 ? g.off[fl] : 0;
    const int64_t len = g.n_flames > 0 ? g.off[fl + 1] - g.off[fl] : n;
    const double cc = (dtf ? dtf[fl] * cfac : c) * m.kappa0[f];
    const double* b = rhs + (size_t)f * n + base;
    double* x = y + (size_t)f * n + base;
    double* Sc = sc + (size_t)f * n + base;
    double* Su = su + (size_t)f * n + base;
    double* Sv = sv + (size_t)f * n + base;
    double* Sw = sw + (size_t)f * n + base;
    const double* K = Kx + base;
    const int lane = threadIdx.x & 63;
    const int P = len < 64 ? (int)len : 64;
    const int64_t s0 = len / P, rem = len % P;
    int64_t r0 = 0, mi = 0;
    double ul = 0.0, vl = -1.0, wl = 0.0;       // last interior row (none: the left separator)
    if (lane < P) {
        r0 = lane * s0 + (lane < rem ? lane : rem);
        mi = s0 + (lane < rem ? 1 : 0) - 1;
        double cprev = 0.0, uprev = 0.0, vprev = 0.0, wprev = 0.0;
        for (int64_t k = 0; k < mi; ++k) {
            const int64_t i = r0 + k;
            const double Km = K[i == 0 ? len - 1 : i - 1], K0 = K[i];
            const double a = -cc * Km, d = 1.0 + cc * (Km + K0), cu = -cc * K0;
            const double aa = (k == 0) ? 0.0 : a;
            const double den = d - aa * cprev;
            const double cn = (k == mi - 1) ? 0.0 : cu / den;
            const double u = (b[i] - aa * uprev) / den;
            const double v = ((k == 0 ? a : 0.0) - aa * vprev) / den;
            const double w = ((k == mi - 1 ? cu : 0.0) - aa * wprev) / den;
            const int64_t q = k * P + lane;
            Sc[q] = cn;
            Su[q] = u;
            Sv[q] = v;
            Sw[q] = w;
            cprev = cn;
            uprev = u;
            vprev = v;
            wprev = w;
        }
        if (mi > 0) {
            ul = uprev;
            vl = vprev;
            wl = wprev;
        }
        double un = ul, vn = vl, wn = wl;
        for (int64_t k = mi - 2; k >= 0; --k) {
            const int64_t q = k * P + lane;
            const double cn = Sc[q];
            un = Su[q] - cn * un;
            vn = Sv[q] - cn * vn;
            wn = Sw[q] - cn * wn;
            Su[q] = un;
            Sv[q] = vn;
            Sw[q] = wn;
        }
        // first interior row (none: the right separator itself)
        fu[lane] = mi > 0 ? un : 0.0;
        fv[lane] = mi > 0 ? vn : 0.0;
        fw[lane] = mi > 0 ? wn : -1.0;
    }
    __syncthreads();
    if (lane < P) {
        const int64_t i = r0 + mi;                  // separator row
        const int nx = lane + 1 == P ? 0 : lane + 1;
        const double Km = K[i == 0 ? len - 1 : i - 1], K0 = K[i];
        const double a = -cc * Km, d = 1.0 + cc * (Km + K0), cu = -cc * K0;
        ra[lane] = -a * vl;
        rb[lane] = d - a * wl - cu * fv[nx];
        rcs[lane] = -cu * fw[nx];
        rr[lane] = b[i] - a * ul - cu * fu[nx];
    }
    __syncthreads();
    if (lane == 0) {
        // periodic system of P separators: Thomas + Sherman-Morrison
        const double a0 = ra[0], cN = rcs[P - 1];
        const double gam = -rb[0];
        double dprev = rb[0] - gam;
        double cprev = rcs[0] / dprev;
        wc[0] = cprev;
        G[0] = rr[0] / dprev;
        wu[0] = gam / dprev;
        for (int i = 1; i < P; ++i) {
            double d = rb[i];
            if (i == P - 1) d -= a0 * cN / gam;
            const double ai = ra[i];
            const double den = d - ai * cprev;
            const double ru = (i == P - 1) ? cN : 0.0;
            G[i] = (rr[i] - ai * G[i - 1]) / den;
            wu[i] = (ru - ai * wu[i - 1]) / den;
            cprev = (i < P - 1) ? rcs[i] / den : 0.0;
            wc[i] = cprev;
        }
        for (int i = P - 2; i >= 0; --i) {
            G[i] -= wc[i] * G[i + 1];
            wu[i] -= wc[i] * wu[i + 1];
        }
        const double vy = G[0] + a0 / gam * G[P - 1];
        const double vu = wu[0] + a0 / gam * wu[P - 1];
        const double fct = vy / (1.0 + vu);
        for (int i = 0; i < P; ++i) G[i] -= fct * wu[i];
    }
    __syncthreads();
    if (lane < P) {
        const double gl = G[lane == 0 ? P - 1 : lane - 1], gr = G[lane];
        for (int64_t k = 0; k < mi; ++k) {
            const int64_t q = k * P + lane;
            x[r0 + k] = Su[q] - Sv[q] * gl - Sw[q] * gr;
        }
        x[r0 + mi] = gr;
    }
}

// bath closure y_i0 = r_i0 - sum_{k != i0, k < N} (y_k - r_k) of one cell, and
// with T_out the temperature of the solved state (th_out: its (T/300)^1.7)
__device__ __forceinline__ void closure_cell(const MechDev& m, int64_t n, const double* rhs,
                                             double* y, double* T_out, double* th_out, int64_t i) {
    double s = 0.0;
    for (int k = 0; k < m.N; ++k)
        if (k != m.bath) s += y[(size_t)k * n + i] - rhs[(size_t)k * n + i];
    y[(size_t)m.bath * n + i] = rhs[(size_t)m.bath * n + i] - s;
    if (T_out) {
        // temperature of the solved state, closed form for constant cp
        double hform = 0.0, cpm = 0.0;
        for (int k = 0; k < m.N; ++k) {
            const double yk = y[(size_t)k * n + i];
            hform += yk * m.hf[k] * m.invW[k];
            cpm += yk * m.cp[k] * m.invW[k];
        }
        const double Ti = T_REF + (y[(size_t)m.N * n + i] - hform) / cpm;
        T_out[i] = Ti;
        if (th_out) th_out[i] = pow(Ti / T_DIFF_REF, THETA_EXP);
    }
}

}  // namespace misdc
