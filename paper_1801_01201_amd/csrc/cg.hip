// Persistent conjugate-gradient kernels of the implicit diffusion (steps
// S3/S4, eq. lagged_diffusion_flux): every diffused field of one node solved
// at once, one launch per solve, iterating on the device until every field
// has converged.  Variants: vectors in global memory; vectors in registers
// (pipelined PCG with one fused grid barrier per iteration); and the tiled
// register variant with a block-local preconditioner.  Reductions use fixed
// orders, so results do not depend on scheduling; the grid is at most one
// workgroup per CU, so it is co-resident and the grid barrier completes.
#include <cmath>
#include <cstdlib>

#include "cg.h"
#include "wave.h"

namespace misdc {

namespace {


// ---- grid-wide barrier for the persistent CG kernels -------------------------
// bar[0]: arrival counter, bar[1]: generation.  The workgroup barrier makes
// every wave's stores complete; one agent-scope release fence per workgroup
// then publishes them to the other XCDs (L2 write-back); the last workgroup to
// arrive resets the counter and bumps the generation; the others poll the
// generation with relaxed agent-scope loads (bounded: after the limit the
// kernel records a timeout in info[2] and proceeds, so every wave always
// terminates); one acquire fence per workgroup makes the other workgroups'
// data visible before the workgroup barrier releases its waves.
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned nblocks, int32_t* info) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived =
            __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1u << 27)) {
                    __hip_atomic_store(&info[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}




// The right-hand side formed inside the tiled kernel (CGArgs lag_src): for
// cell i, the four neighbours (periodic; nx, ny >= 2), the face coefficients
// of the solve's operator from theta of lag_T (the values faces_at forms),
// and b = lag_part + (qa FA + qd FD + qr FR) of every field, FA and FD at
// lag_src from their stencils (fourth-order advection faces, the diffusion
// operator with theta of lag_src's temperature, the bath's FD minus the sum
// of the other species'); every field is written to b_w when the thread owns
// the cell, and bd returns the diffused fields' values.  Fields are taken
// CH at a time, each chunk's loads issued together.
template <int NFD>
__device__ __forceinline__ void fused_rhs(const CGArgs& a, int64_t i, bool own, int64_t& e,
                                          int64_t& w, int64_t& nn, int64_t& s, double& ke,
                                          double& kw, double& kn, double& ks, double (&bd)[NFD]) {
    constexpr int NF = NFD + 1, CH = 5;
    const int64_t nx = a.nx, ny = a.ny, n = a.n;
    const int64_t iy = i / nx, ix = i - iy * nx, row = iy * nx;
    auto wx = [&](int64_t k) { return k < 0 ? k + nx : (k >= nx ? k - nx : k); };
    auto wy = [&](int64_t k) { return k < 0 ? k + ny : (k >= ny ? k - ny : k); };
    const int64_t xm1 = row + wx(ix - 1), xm2 = row + wx(ix - 2);
    const int64_t xp1 = row + wx(ix + 1), xp2 = row + wx(ix + 2);
    const int64_t ym1 = wy(iy - 1) * nx + ix, ym2 = wy(iy - 2) * nx + ix;
    const int64_t yp1 = wy(iy + 1) * nx + ix, yp2 = wy(iy + 2) * nx + ix;
    e = xp1;
    w = xm1;
    nn = yp1;
    s = ym1;
    const double* TH = a.lag_Tsrc ? a.lag_Tsrc : a.lag_th;
    const double T0 = a.lag_T[i], Te = a.lag_T[xp1], Tw = a.lag_T[xm1], Tn = a.lag_T[yp1],
                 Ts = a.lag_T[ym1];
    const double h0 = TH[i], he = TH[xp1], hw = TH[xm1], hn = TH[yp1], hs = TH[ym1];
    // the solve's face coefficients, as faces_at forms Kx and Ky (kw = Kx of
    // the west neighbour, ks = Ky of the south neighbour)
    const double t0 = pow(T0 / T_DIFF_REF, THETA_EXP), te = pow(Te / T_DIFF_REF, THETA_EXP);
    const double tw = pow(Tw / T_DIFF_REF, THETA_EXP), tn = pow(Tn / T_DIFF_REF, THETA_EXP);
    const double ts = pow(Ts / T_DIFF_REF, THETA_EXP);
    ke = 0.5 * (t0 + te) / (a.dx * a.dx);
    kw = 0.5 * (tw + t0) / (a.dx * a.dx);
    kn = 0.5 * (t0 + tn) / (a.dy * a.dy);
    ks = 0.5 * (ts + t0) / (a.dy * a.dy);
    // the lagged operators' coefficients (theta of lag_src)
    auto th_of = [&](double x) { return a.lag_Tsrc ? pow(x / T_DIFF_REF, THETA_EXP) : x; };
    const double g0 = th_of(h0);
    const double idx2 = 1.0 / (a.dx * a.dx), idy2 = 1.0 / (a.dy * a.dy);
    const double kxe = 0.5 * (g0 + th_of(he)) * idx2, kxw = 0.5 * (g0 + th_of(hw)) * idx2;
    const double kyn = 0.5 * (g0 + th_of(hn)) * idy2, kys = 0.5 * (g0 + th_of(hs)) * idy2;
    const double ax = a.ux / a.dx, ay = a.uy / a.dy;
    double bf[NF];
    double fd_sum = 0.0, fa_bath = 0.0, part_bath = 0.0, fr_bath = 0.0;
#pragma unroll
    for (int f0 = 0; f0 < NF; f0 += CH) {
        double v[CH][9], pv[CH], rv[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int f = f0 + c < NF ? f0 + c : NF - 1;
            const double* P = a.lag_src + (size_t)f * n;
            v[c][0] = P[i];
            v[c][1] = P[xm1];
            v[c][2] = P[xm2];
            v[c][3] = P[xp1];
            v[c][4] = P[xp2];
            v[c][5] = P[ym1];
            v[c][6] = P[ym2];
            v[c][7] = P[yp1];
            v[c][8] = P[yp2];
            pv[c] = a.lag_part[(size_t)f * n + i];
            rv[c] = a.lag_fr ? a.lag_fr[(size_t)(f < a.N ? f : a.N - 1) * n + i] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int f = f0 + c;
            if (f >= NF) continue;
            const double c0 = v[c][0], w1 = v[c][1], w2 = v[c][2], e1 = v[c][3], e2 = v[c][4];
            const double s1 = v[c][5], s2 = v[c][6], n1 = v[c][7], n2 = v[c][8];
            // fourth-order face values, as the explicit operators take them
            const double fe = (7.0 * (c0 + e1) - (w1 + e2)) / 12.0;
            const double fw = (7.0 * (w1 + c0) - (w2 + e1)) / 12.0;
            double fa = -ax * (fe - fw);
            double lap = kxe * (e1 - c0) - kxw * (c0 - w1);
            const double fn = (7.0 * (c0 + n1) - (s1 + n2)) / 12.0;
            const double fs = (7.0 * (s1 + c0) - (s2 + n1)) / 12.0;
            if (ay != 0.0) fa -= ay * (fn - fs);
            lap += kyn * (n1 - c0) - kys * (c0 - s1);
            const double fr = f < a.N ? rv[c] : 0.0;
            if (f == a.bath) {
                fa_bath = fa;
                part_bath = pv[c];
                fr_bath = fr;
                bf[f] = 0.0;
                continue;
            }
            const double fd = a.kappa0[f] * lap;
            if (f < a.N) fd_sum += fd;
            bf[f] = pv[c] + (a.lag_qa * fa + a.lag_qd * fd + a.lag_qr * fr);
            if (own) a.b_w[(size_t)f * n + i] = bf[f];
        }
    }
    if (own)
        a.b_w[(size_t)a.bath * n + i] =
            part_bath + (a.lag_qa * fa_bath + a.lag_qd * -fd_sum + a.lag_qr * fr_bath);
#pragma unroll
    for (int d = 0; d < NFD; ++d) bd[d] = d >= a.bath ? bf[d + 1] : bf[d];
}

// A_f v at cell i: v_i - cf (Ke (v_E - v_i) - Kw (v_i - v_W) + Kn (...) - Ks (...))
__device__ __forceinline__ void stencil_at(const CGArgs& a, int64_t i, int64_t& e, int64_t& w,
                                           int64_t& nn, int64_t& s, double& ke, double& kw,
                                           double& kn, double& ks) {
    const int64_t iy = i / a.nx, ix = i - iy * a.nx;
    e = iy * a.nx + (ix + 1 == a.nx ? 0 : ix + 1);
    w = iy * a.nx + (ix == 0 ? a.nx - 1 : ix - 1);
    nn = (iy + 1 == a.ny ? 0 : iy + 1) * a.nx + ix;
    s = (iy == 0 ? a.ny - 1 : iy - 1) * a.nx + ix;
    ke = a.Kx[i];
    kw = a.Kx[w];
    kn = a.Ky[i];
    ks = a.Ky[s];
}

// Wave-level sum, lane 0 stores the wave's value into red[slot * nw + wave].
__device__ __forceinline__ void wave_store(double v, double* red, int slot) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[slot * (CG_THREADS / 64) + (threadIdx.x >> 6)] = v;
}

// After __syncthreads: sum the wave values of every slot in a fixed order and
// write this block's partials to global memory.
__device__ __forceinline__ void block_publish(const double* red, int nslots, double* partial) {
    for (int t = threadIdx.x; t < nslots; t += CG_THREADS) {
        double s = 0.0;
        for (int k = 0; k < CG_THREADS / 64; ++k) s += red[t * (CG_THREADS / 64) + k];
        partial[(size_t)blockIdx.x * (CG_MAX_FIELDS * 4) + t] = s;
    }
}

// Sum of the partials of every block for slots [0, nslots): each wave handles
// a subset of slots, its lanes stride over the blocks, fixed order -> every
// block obtains bitwise the same totals.
__device__ __forceinline__ void grid_totals(const double* partial, int nslots, double* tot) {
    const int nb = gridDim.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = wave; t < nslots; t += CG_THREADS / 64) {
        double s = 0.0;
        for (int b = lane; b < nb; b += 64) s += partial[(size_t)b * (CG_MAX_FIELDS * 4) + t];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) tot[t] = s;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(CG_THREADS) cg_kernel(CGArgs a) {
    // slot layout: slot = field * 4 + value
    __shared__ double red[CG_MAX_FIELDS * 4 * (CG_THREADS / 64)];
    __shared__ double tot[CG_MAX_FIELDS * 4];
    __shared__ double s_rz[CG_MAX_FIELDS], s_bb[CG_MAX_FIELDS], s_alpha[CG_MAX_FIELDS],
        s_beta[CG_MAX_FIELDS];
    __shared__ int s_active[CG_MAX_FIELDS];
    __shared__ int s_any;
    const unsigned nb = gridDim.x;
    const int64_t stride = (int64_t)gridDim.x * CG_THREADS;
    const int64_t i0 = (int64_t)blockIdx.x * CG_THREADS + threadIdx.x;
    const int nf = a.nf;

    // ---- r = b - A x0, z = D^{-1} r; partials rz, rr, bb ----
    for (int d = 0; d < nf; ++d) {
        const size_t o = (size_t)a.fmap[d] * a.n;
        const double* X = a.guess_in_x ? a.x + o : a.b + o;
        const double cf = a.cf[d];
        double rz = 0.0, rr = 0.0, bb = 0.0;
        for (int64_t i = i0; i < a.n; i += stride) {
            int64_t e, w, nn, s;
            double ke, kw, kn, ks;
            stencil_at(a, i, e, w, nn, s, ke, kw, kn, ks);
            const double xi = X[i];
            const double Ax = xi - cf * (ke * (X[e] - xi) - kw * (xi - X[w]) + kn * (X[nn] - xi) -
                                         ks * (xi - X[s]));
            const double bi = a.b[o + i];
            const double ri = bi - Ax;
            const double zi = ri / (1.0 + cf * (ke + kw + kn + ks));
            a.r[o + i] = ri;
            a.z[o + i] = zi;
            if (!a.guess_in_x) a.x[o + i] = xi;
            rz += ri * zi;
            rr += ri * ri;
            bb += bi * bi;
        }
        wave_store(rz, red, d * 4 + 0);
        wave_store(rr, red, d * 4 + 1);
        wave_store(bb, red, d * 4 + 2);
    }
    __syncthreads();
    block_publish(red, nf * 4, a.partial);
    grid_barrier(a.bar, nb, a.info);
    grid_totals(a.partial, nf * 4, tot);
    if (threadIdx.x == 0) {
        for (int d = 0; d < nf; ++d) {
            s_rz[d] = tot[d * 4 + 0];
            s_bb[d] = tot[d * 4 + 2];
            s_active[d] = tot[d * 4 + 1] > a.rtol2 * s_bb[d];
            s_beta[d] = 0.0;
        }
    }
    __syncthreads();
    int it = 0;
    for (; it < a.maxit; ++it) {
        if (threadIdx.x == 0) {
            int any = 0;
            for (int d = 0; d < nf; ++d) any |= s_active[d];
            s_any = any;
        }
        __syncthreads();
        if (!s_any) break;
        // ---- p = z + beta p ; q = A z + beta q  (so q = A p) ; partial pq ----
        for (int d = 0; d < nf; ++d) {
            double pq = 0.0;
            if (s_active[d]) {
                const size_t o = (size_t)a.fmap[d] * a.n;
                const double* Z = a.z + o;
                const double cf = a.cf[d];
                const double be = s_beta[d];
                for (int64_t i = i0; i < a.n; i += stride) {
                    int64_t e, w, nn, s;
                    double ke, kw, kn, ks;
                    stencil_at(a, i, e, w, nn, s, ke, kw, kn, ks);
                    const double zi = Z[i];
                    const double Az = zi - cf * (ke * (Z[e] - zi) - kw * (zi - Z[w]) +
                                                 kn * (Z[nn] - zi) - ks * (zi - Z[s]));
                    const double pi = (it == 0) ? zi : zi + be * a.p[o + i];
                    const double qi = (it == 0) ? Az : Az + be * a.q[o + i];
                    a.p[o + i] = pi;
                    a.q[o + i] = qi;
                    pq += pi * qi;
                }
            }
            wave_store(pq, red, d * 4 + 0);
        }
        __syncthreads();
        block_publish(red, nf * 4, a.partial);
        grid_barrier(a.bar, nb, a.info);
        grid_totals(a.partial, nf * 4, tot);
        if (threadIdx.x == 0)
            for (int d = 0; d < nf; ++d) s_alpha[d] = s_active[d] ? s_rz[d] / tot[d * 4 + 0] : 0.0;
        __syncthreads();
        // ---- x += alpha p ; r -= alpha q ; z = D^{-1} r ; partials rz, rr ----
        for (int d = 0; d < nf; ++d) {
            double rz = 0.0, rr = 0.0;
            if (s_active[d]) {
                const size_t o = (size_t)a.fmap[d] * a.n;
                const double al = s_alpha[d];
                const double cf = a.cf[d];
                for (int64_t i = i0; i < a.n; i += stride) {
                    const int64_t iy = i / a.nx, ix = i - iy * a.nx;
                    const int64_t w = iy * a.nx + (ix == 0 ? a.nx - 1 : ix - 1);
                    const int64_t s = (iy == 0 ? a.ny - 1 : iy - 1) * a.nx + ix;
                    const double ksum = a.Kx[i] + a.Kx[w] + a.Ky[i] + a.Ky[s];
                    a.x[o + i] += al * a.p[o + i];
                    const double ri = a.r[o + i] - al * a.q[o + i];
                    const double zi = ri / (1.0 + cf * ksum);
                    a.r[o + i] = ri;
                    a.z[o + i] = zi;
                    rz += ri * zi;
                    rr += ri * ri;
                }
            }
            wave_store(rz, red, d * 4 + 0);
            wave_store(rr, red, d * 4 + 1);
        }
        __syncthreads();
        block_publish(red, nf * 4, a.partial);
        grid_barrier(a.bar, nb, a.info);
        grid_totals(a.partial, nf * 4, tot);
        if (threadIdx.x == 0)
            for (int d = 0; d < nf; ++d) {
                if (!s_active[d]) continue;
                const double rz_new = tot[d * 4 + 0];
                s_beta[d] = rz_new / s_rz[d];
                s_rz[d] = rz_new;
                s_active[d] = tot[d * 4 + 1] > a.rtol2 * s_bb[d];
            }
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.info[0] = it;
        int any = 0;
        for (int d = 0; d < nf; ++d) any |= s_active[d];
        a.info[1] = any;
    }
}

// Grid barrier number k (0-based) of the current launch, with a monotonic
// arrival counter that the preceding faces_kernel zeroed: every workgroup
// publishes its stores with one agent-scope release fence and one relaxed
// increment, then waits until all workgroups have arrived k+1 times (the
// increments form one release sequence, so the acquire fence after the wait
// makes every workgroup's stores visible).  Bounded wait: after the limit the
// kernel records a timeout in info[2] and proceeds, so every wave terminates.
__device__ __forceinline__ void grid_sync(unsigned* counter, unsigned nb, unsigned k,
                                          int32_t* info) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = (k + 1u) * nb;
        unsigned spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1u << 27)) {
                __hip_atomic_store(&info[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// All-reduce of nslots values fused with grid barrier k.  red holds one value
// per (slot, wave) of this workgroup.  The partials go to buffer k % 2 (so a
// workgroup that is one barrier ahead cannot overwrite values another one is
// still reading); after the barrier every workgroup loads all partials at
// once into LDS and sums them in block order: bitwise identical totals in
// every workgroup, whatever the scheduling.
template <int BS>
__device__ __forceinline__ void grid_allreduce(const CGArgs& a, unsigned k, int nslots,
                                               const double* red, double* stage, double* tot) {
    constexpr int NW = BS / 64;
    const unsigned nb = gridDim.x;
    double* part = a.partial + (size_t)(k & 1u) * CG_MAX_BLOCKS * (CG_MAX_FIELDS * 4);
    __syncthreads();
    for (int t = threadIdx.x; t < nslots; t += BS) {
        double v = 0.0;
        for (int w = 0; w < NW; ++w) v += red[t * NW + w];
        part[(size_t)blockIdx.x * (CG_MAX_FIELDS * 4) + t] = v;
    }
    grid_sync(a.bar, nb, k, a.info);
    const int total = (int)nb * nslots;
    for (int e = threadIdx.x; e < total; e += BS) {
        const int b = e / nslots, t = e - b * nslots;
        stage[e] = part[(size_t)b * (CG_MAX_FIELDS * 4) + t];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = wave; t < nslots; t += NW) {
        double v = 0.0;
        for (unsigned b = lane; b < nb; b += 64) v += stage[b * nslots + t];
        v = wave_sum(v);
        if (lane == 0) tot[t] = v;
    }
    __syncthreads();
}

template <int BS>
__device__ __forceinline__ void wave_put(double v, double* red, int slot) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[slot * (BS / 64) + (threadIdx.x >> 6)] = v;
}

// wave_put of K slots at once (value(s): this lane's value of slot s), by
// one batched reduction whose slot-s total lands in lanes 2s and 2s+1
template <int BS, int K, class F>
__device__ __forceinline__ void wave_put_slots(F value, double* red) {
    const double v = wave_sum_slots<K>(value);
    const int lane = threadIdx.x & 63;
    if ((lane & 1) == 0 && (lane >> 1) < K) red[(lane >> 1) * (BS / 64) + (threadIdx.x >> 6)] = v;
}

// Register-resident pipelined preconditioned CG (the single-reduction
// recurrences of Ghysels & Vanroose).  Every thread owns CPT cells for the
// whole solve and keeps all vectors of the NFD fields in registers; the only
// vector exchanged through memory is m = D^{-1} w, whose stencil product is
// taken after the barrier that also reduces (r,u), (w,u) and (r,r) -- one
// grid barrier per iteration.  m is double-buffered in a.z / a.q.  Fields stop
// (their updates are masked) once |r|_2 <= rtol |b|_2.
template <int NFD, int CPT, int BS>
__global__ void __launch_bounds__(BS) cg_regs_kernel(CGArgs a) {
    constexpr int NS = 3 * NFD;               // slots: gamma, delta, rr per field
    __shared__ double stage[CG_MAX_BLOCKS * NS];
    __shared__ double red[NS * (BS / 64)];
    __shared__ double tot[NS];
    __shared__ double s_bb[NFD], s_gprev[NFD], s_aprev[NFD], s_alpha[NFD], s_beta[NFD];
    __shared__ int s_active[NFD];
    const int64_t T = (int64_t)gridDim.x * BS;
    const int64_t t0 = (int64_t)blockIdx.x * BS + threadIdx.x;
    int64_t cell[CPT], ie[CPT], iw[CPT], in_[CPT], is_[CPT];
    double ke[CPT], kw[CPT], kn[CPT], ks[CPT];
    bool own[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
        cell[k] = t0 + k * T;
        own[k] = cell[k] < a.n;
        const int64_t i = own[k] ? cell[k] : 0;
        stencil_at(a, i, ie[k], iw[k], in_[k], is_[k], ke[k], kw[k], kn[k], ks[k]);
    }
    double x[NFD][CPT], r[NFD][CPT], u[NFD][CPT], w[NFD][CPT];
    double zz[NFD][CPT], qq[NFD][CPT], ss[NFD][CPT], pp[NFD][CPT];
    unsigned kb = 0;                          // grid barriers done in this launch
    // ---- r = b - A x0, u = D^{-1} r (published), partial (b, b) ----
#pragma unroll
    for (int d = 0; d < NFD; ++d) {
        const size_t o = (size_t)a.fmap[d] * a.n;
        const double* X = a.guess_in_x ? a.x + o : a.b + o;
        const double cf = a.cf[d];
        double bb = 0.0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            x[d][k] = r[d][k] = u[d][k] = w[d][k] = 0.0;
            zz[d][k] = qq[d][k] = ss[d][k] = pp[d][k] = 0.0;
            if (!own[k]) continue;
            const int64_t i = cell[k];
            const double xi = X[i];
            const double Ax = xi - cf * (ke[k] * (X[ie[k]] - xi) - kw[k] * (xi - X[iw[k]]) +
                                         kn[k] * (X[in_[k]] - xi) - ks[k] * (xi - X[is_[k]]));
            const double bi = a.b[o + i];
            x[d][k] = xi;
            r[d][k] = bi - Ax;
            u[d][k] = r[d][k] / (1.0 + cf * (ke[k] + kw[k] + kn[k] + ks[k]));
            a.r[o + i] = u[d][k];             // exchange buffer of u
            bb += bi * bi;
        }
        wave_put<BS>(bb, red, d);
    }
    grid_allreduce<BS>(a, kb++, NFD, red, stage, tot);
    if (threadIdx.x < NFD) s_bb[threadIdx.x] = tot[threadIdx.x];
    // ---- w = A u ----
#pragma unroll
    for (int d = 0; d < NFD; ++d) {
        const size_t o = (size_t)a.fmap[d] * a.n;
        const double* U = a.r + o;
        const double cf = a.cf[d];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            if (!own[k]) continue;
            const double ui = u[d][k];
            w[d][k] = ui - cf * (ke[k] * (U[ie[k]] - ui) - kw[k] * (ui - U[iw[k]]) +
                                 kn[k] * (U[in_[k]] - ui) - ks[k] * (ui - U[is_[k]]));
        }
    }
    int it = 0;
    for (; it < a.maxit; ++it) {
        // ---- m = D^{-1} w (published), partials gamma = (r,u), delta = (w,u), rr ----
        double* Mbuf = (it & 1) ? a.q : a.z;
#pragma unroll
        for (int d = 0; d < NFD; ++d) {
            const size_t o = (size_t)a.fmap[d] * a.n;
            const double cf = a.cf[d];
            double g = 0.0, de = 0.0, rr = 0.0;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                if (!own[k]) continue;
                Mbuf[o + cell[k]] = w[d][k] / (1.0 + cf * (ke[k] + kw[k] + kn[k] + ks[k]));
                g += r[d][k] * u[d][k];
                de += w[d][k] * u[d][k];
                rr += r[d][k] * r[d][k];
            }
            wave_put<BS>(g, red, 3 * d + 0);
            wave_put<BS>(de, red, 3 * d + 1);
            wave_put<BS>(rr, red, 3 * d + 2);
        }
        grid_allreduce<BS>(a, kb++, NS, red, stage, tot);
        // recurrence coefficients, one thread per field
        if (threadIdx.x < NFD) {
            const int d = threadIdx.x;
            const double g = tot[3 * d], de = tot[3 * d + 1], rr = tot[3 * d + 2];
            const int act = rr > a.rtol2 * s_bb[d];
            double al = 0.0, be = 0.0;
            if (act) {
                if (it == 0) {
                    al = g / de;
                } else {
                    be = g / s_gprev[d];
                    al = g / (de - be * g / s_aprev[d]);
                }
                s_gprev[d] = g;
                s_aprev[d] = al;
            }
            s_active[d] = act;
            s_alpha[d] = al;
            s_beta[d] = be;
        }
        __syncthreads();
        int any = 0;
#pragma unroll
        for (int d = 0; d < NFD; ++d) any |= s_active[d];
        if (!any) break;
        // ---- n = A m ; recurrences ----
#pragma unroll
        for (int d = 0; d < NFD; ++d) {
            const size_t o = (size_t)a.fmap[d] * a.n;
            const double* Mv = Mbuf + o;
            const double cf = a.cf[d];
            const bool act = s_active[d];
            const double al = s_alpha[d], be = s_beta[d];
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                if (!own[k]) continue;
                const double mi = Mv[cell[k]];
                const double ni = mi - cf * (ke[k] * (Mv[ie[k]] - mi) - kw[k] * (mi - Mv[iw[k]]) +
                                             kn[k] * (Mv[in_[k]] - mi) - ks[k] * (mi - Mv[is_[k]]));
                const double z1 = ni + be * zz[d][k];
                const double q1 = mi + be * qq[d][k];
                const double s1 = w[d][k] + be * ss[d][k];
                const double p1 = u[d][k] + be * pp[d][k];
                zz[d][k] = act ? z1 : zz[d][k];
                qq[d][k] = act ? q1 : qq[d][k];
                ss[d][k] = act ? s1 : ss[d][k];
                pp[d][k] = act ? p1 : pp[d][k];
                x[d][k] = act ? x[d][k] + al * p1 : x[d][k];
                r[d][k] = act ? r[d][k] - al * s1 : r[d][k];
                u[d][k] = act ? u[d][k] - al * q1 : u[d][k];
                w[d][k] = act ? w[d][k] - al * z1 : w[d][k];
            }
        }
    }
#pragma unroll
    for (int d = 0; d < NFD; ++d) {
        const size_t o = (size_t)a.fmap[d] * a.n;
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (own[k]) a.x[o + cell[k]] = x[d][k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.info[0] = it;
        int any = 0;
        for (int d = 0; d < NFD; ++d) any |= s_active[d];
        a.info[1] = (it == a.maxit) ? any : 0;
    }
}

// ---------------------------------------------------------------------------
// Tiled variant: the same pipelined PCG, with every workgroup owning a
// TX x TY tile of cells and a block-local preconditioner.  The
// preconditioner applies KSW Jacobi sweeps, started from zero, to the tile's
// own operator (the 5-point stencil with the neighbours outside the tile
// dropped): z = sum_{j <= KSW} (I - D^-1 A_t)^j D^-1 v.  That is a fixed
// polynomial in the symmetric matrix D^-1/2 A_t D^-1/2 whose eigenvalues lie
// in (0, 2), so it is symmetric positive definite and CG stays valid.  It
// couples the cells within a tile through LDS, so it costs no grid barrier,
// and it replaces the diagonal preconditioner at the two places the
// pipelined recurrence applies one (u = M^-1 r, m = M^-1 w).
// ---------------------------------------------------------------------------
// Edges and halo of a tile, TILE_HALO slots per field each.  Edge slots of
// a tile: [0, TX) its top row (+y side), [TX, 2 TX) its bottom row, then TY
// slots for its right column (+x side) and TY for its left column.  Halo
// slots, in the same order: the row above, the row below, the column to the
// right and the column to the left (periodic wrap) -- each is an edge of the
// neighbouring tile on that side: the row above is the bottom edge of the
// tile above, and so on.  Slots beyond a ragged tile's width or height are
// unused.  Returns the offset of halo slot s of field d of tile (bx, by) in
// one parity half of the edge buffer (-1 when the slot is unused).
__device__ __forceinline__ int halo_source(const CGArgs& a, int nty, int bx, int by, int wt,
                                           int ht, int d, int s) {
    int tile, slot;
    if (s < TILE_X) {                                      // above: its bottom row
        if (s >= wt) return -1;
        tile = ((by + 1) % nty) * a.ntx + bx;
        slot = TILE_X + s;
    } else if (s < 2 * TILE_X) {                           // below: its top row
        s -= TILE_X;
        if (s >= wt) return -1;
        tile = ((by - 1 + nty) % nty) * a.ntx + bx;
        slot = s;
    } else if (s < 2 * TILE_X + TILE_Y) {                  // right: its left column
        s -= 2 * TILE_X;
        if (s >= ht) return -1;
        tile = by * a.ntx + (bx + 1) % a.ntx;
        slot = 2 * TILE_X + TILE_Y + s;
    } else {                                               // left: its right column
        s -= 2 * TILE_X + TILE_Y;
        if (s >= ht) return -1;
        tile = by * a.ntx + (bx - 1 + a.ntx) % a.ntx;
        slot = 2 * TILE_X + s;
    }
    return (tile * 9 + d) * TILE_HALO + slot;
}

// The exchange around this barrier orders relaxed agent-scope atomics with
// s_waitcnt and workgroup barriers only, with no release/acquire pair.  That
// another XCD then sees the data is how gfx950 executes such atomics (they
// bypass the non-coherent per-CU caches and are ordered once complete), not
// a guarantee of the HIP memory model, so any other target is refused.
#if defined(__HIP_DEVICE_COMPILE__) && !defined(__gfx950__)
#error "the fence-free grid exchange of the tiled CG is written for gfx950 only"
#endif

// Grid barrier k without cache maintenance, for data exchanged only through
// agent-scope atomic stores and loads (which the hardware keeps coherent
// across the XCDs without writing back or invalidating the L2): every wave
// waits until its stores have completed, then the workgroup arrives.
// Arrival is two-level, so that no counter takes more than 16 atomics per
// barrier: workgroup b counts into group b mod 8 (its own cache line), and
// the last arrival of a group counts the group into bar[BAR_GLOBAL], on which
// every workgroup waits (bounded as in grid_sync).  k counts these barriers
// only (from 0 in each launch; the counters are zeroed before it).
__device__ __forceinline__ void grid_sync_direct(unsigned* bar, unsigned nb, unsigned k,
                                                 int32_t* info) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned* counter = bar + BAR_GLOBAL;
        const unsigned g = blockIdx.x % BAR_GROUPS;
        const unsigned gsize = (nb - 1u - g) / BAR_GROUPS + 1u;      // workgroups of group g
        const unsigned ngroups = nb < (unsigned)BAR_GROUPS ? nb : (unsigned)BAR_GROUPS;
        const unsigned before = __hip_atomic_fetch_add(&bar[BAR_STRIDE * (1 + g)], 1u,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (before + 1u == (k + 1u) * gsize)
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = (k + 1u) * ngroups;
        unsigned spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1u << 27)) {
                __hip_atomic_store(&info[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
}

// The blocks' partial sums of one exchange, slot-major: thread (slot t =
// tid mod 32, group g = tid / 32) loads slot t of blocks g, g + G, g + 2G,
// ... (G = 16 groups of the workgroup) and adds them in that order; the
// group sums go to stage[g * 32 + t] (4 KB of LDS for every block count),
// which slot_total adds in group order.  Loads are issued together with the
// caller's halo loads, so the exchange costs one memory latency.
constexpr int TILE_GROUPS = TILE_BS / 32;
constexpr int TILE_BPG = (TILE_NB + TILE_GROUPS - 1) / TILE_GROUPS;
__device__ __forceinline__ double group_partial(const double* part, unsigned nb, int nslots) {
    const int t = threadIdx.x & 31, g = threadIdx.x >> 5;
    double pv[TILE_BPG];
#pragma unroll
    for (int j = 0; j < TILE_BPG; ++j) {
        const unsigned b = (unsigned)(g + TILE_GROUPS * j);
        pv[j] = (t < nslots && b < nb)
                    ? __hip_atomic_load(&part[b * (CG_MAX_FIELDS * 4) + (unsigned)t],
                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                    : 0.0;
    }
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < TILE_BPG; ++j) acc += pv[j];
    return acc;
}
__device__ __forceinline__ double slot_total(const double* stage, int t) {
    double v = 0.0;
#pragma unroll
    for (int g = 0; g < TILE_GROUPS; ++g) v += stage[g * 32 + t];
    return v;
}

// Exchange 0 of the tiled kernel (its prologue): the blocks' partial sums of
// NFD fields and the tile's edges of mt (u of every field) travel through
// agent-scope atomic stores and loads around the barrier without cache
// maintenance, as in the iterations; afterwards tot holds the NFD totals and
// halo the tile's halo of u.
template <int BS, int NFD, int HPT>
__device__ __forceinline__ void grid_exchange_first(const CGArgs& a, const double* red,
                                                    double* stage, double* tot, const double* mt,
                                                    const int (&elds)[HPT], const int (&hsrc)[HPT],
                                                    double* halo) {
    static_assert(BS == TILE_BS, "slot-major partials: 16 groups of 32 threads");
    constexpr int NW = BS / 64;
    const unsigned nb = gridDim.x;
    double* part = a.partial;                                // parity of exchange 0
    double* eb = a.edge;                                     // edge half of exchange 0
    __syncthreads();
    for (int t = threadIdx.x; t < NFD; t += BS) {
        double v = 0.0;
        for (int w = 0; w < NW; ++w) v += red[t * NW + w];
        __hip_atomic_store(&part[(size_t)blockIdx.x * (CG_MAX_FIELDS * 4) + t], v,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const int e = threadIdx.x + j * BS;                // (field, slot) of this tile
        if (elds[j] >= 0)
            __hip_atomic_store(&eb[(size_t)blockIdx.x * (NFD * TILE_HALO) + e], mt[elds[j]],
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    grid_sync_direct(a.bar, nb, 0u, a.info);
    double hv[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j)
        hv[j] = hsrc[j] >= 0
                    ? __hip_atomic_load(&eb[(unsigned)hsrc[j]], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT)
                    : 0.0;
    stage[threadIdx.x] = group_partial(part, nb, NFD);
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const int e = threadIdx.x + j * BS;
        if (e < NFD * TILE_HALO) halo[e] = hv[j];
    }
    __syncthreads();
    if (threadIdx.x < NFD) tot[threadIdx.x] = slot_total(stage, threadIdx.x);
    __syncthreads();
}

// grid_sync_direct in two halves, so that a workgroup can work while the
// other workgroups arrive: grid_arrive waits for this workgroup's stores and
// counts it into its group and, if it completes the group, the group into
// the barrier (at once, since the other workgroups wait on that count);
// grid_wait waits for barrier k and synchronises the workgroup.
__device__ __forceinline__ void grid_arrive(unsigned* bar, unsigned nb, unsigned k) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned g = blockIdx.x % BAR_GROUPS;
        const unsigned gsize = (nb - 1u - g) / BAR_GROUPS + 1u;      // workgroups of group g
        const unsigned before = __hip_atomic_fetch_add(&bar[BAR_STRIDE * (1 + g)], 1u,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (before + 1u == (k + 1u) * gsize)
            __hip_atomic_fetch_add(bar + BAR_GLOBAL, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}
__device__ __forceinline__ void grid_wait(unsigned* bar, unsigned nb, unsigned k, int32_t* info) {
    if (threadIdx.x == 0) {
        const unsigned ngroups = nb < (unsigned)BAR_GROUPS ? nb : (unsigned)BAR_GROUPS;
        const unsigned target = (k + 1u) * ngroups;
        unsigned spins = 0;
        while (__hip_atomic_load(bar + BAR_GLOBAL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1u << 27)) {
                __hip_atomic_store(&info[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
}

// Reduction of the partial sums (r,u), (w,u), (r,r) of every field over
// the blocks, fused with the recurrence coefficients: the wavefront that
// reduces a field's three sums computes its coefficients.  A field whose
// residual has met the tolerance stays inactive (its sums are no longer
// formed).  The partials and the tile's edges of m (copied from the tile
// ``mt`` in LDS: elds holds the LDS index of each of this thread's edge
// slots, -1 for none) travel through agent-scope atomic stores and loads, so
// the barrier needs no cache write-back or invalidation.  After it every
// thread issues all of its loads at once -- its share of the blocks'
// partials (group sums into ``stage``) and of the tile's halo of m (hsrc:
// offsets into the edge half ``eb``, -1 for none; into ``halo``) -- so the
// exchange costs one memory latency.
template <int BS, int NFD, int HPT>
__device__ __forceinline__ void grid_publish_arrive(const CGArgs& a, unsigned k,
                                                        const double* red, const double* mt,
                                                        const int (&elds)[HPT], double* eb,
                                                        const int* s_active) {
    constexpr int NW = BS / 64, NS = 3 * NFD;
    double* part = a.partial + (size_t)(k & 1u) * CG_MAX_BLOCKS * (CG_MAX_FIELDS * 4);
    __syncthreads();
    for (int t = threadIdx.x; t < NS; t += BS) {
        double v = 0.0;
        for (int w = 0; w < NW; ++w) v += red[t * NW + w];
        __hip_atomic_store(&part[(size_t)blockIdx.x * (CG_MAX_FIELDS * 4) + t], v,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const int e = threadIdx.x + j * BS;                // (field, slot) of this tile
        if (elds[j] >= 0 && s_active[e / TILE_HALO])
            __hip_atomic_store(&eb[(size_t)blockIdx.x * (NFD * TILE_HALO) + e], mt[elds[j]],
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    grid_arrive(a.bar, gridDim.x, k);
}

template <int BS, int NFD, int HPT>
__device__ __forceinline__ void grid_finish_coeffs(const CGArgs& a, unsigned k, int it,
                                                   double* stage,
                                                   double* eb, const int (&hsrc)[HPT],
                                                   double* halo, const double* s_bb,
                                                   double* s_gprev, double* s_aprev,
                                                   double* s_alpha, double* s_beta,
                                                   int* s_active) {
    static_assert(BS == TILE_BS && 3 * NFD <= 32, "slot-major partials: 32 slots per group");
    constexpr int NW = BS / 64, NS = 3 * NFD;
    const unsigned nb = gridDim.x;
    double* part = a.partial + (size_t)(k & 1u) * CG_MAX_BLOCKS * (CG_MAX_FIELDS * 4);
    grid_wait(a.bar, nb, k, a.info);
    double hv[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j)
        hv[j] = hsrc[j] >= 0
                    ? __hip_atomic_load(&eb[(unsigned)hsrc[j]], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT)
                    : 0.0;
    stage[threadIdx.x] = group_partial(part, nb, NS);
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const int e = threadIdx.x + j * BS;
        if (e < NFD * TILE_HALO) halo[e] = hv[j];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = wave; d < NFD; d += NW) {
        if (!s_active[d]) continue;
        double g = lane < TILE_GROUPS ? stage[lane * 32 + 3 * d] : 0.0;
        double de = lane < TILE_GROUPS ? stage[lane * 32 + 3 * d + 1] : 0.0;
        double rr = lane < TILE_GROUPS ? stage[lane * 32 + 3 * d + 2] : 0.0;
        g = wave_sum(g);
        de = wave_sum(de);
        rr = wave_sum(rr);
        if (lane == 0) {
            const int act = rr > a.rtol2 * s_bb[d];
            double al = 0.0, be = 0.0;
            if (act) {
                if (it == 0) {
                    al = g / de;
                } else {
                    be = g / s_gprev[d];
                    al = g / (de - be * g / s_aprev[d]);
                }
                s_gprev[d] = g;
                s_aprev[d] = al;
            }
            s_active[d] = act;
            s_alpha[d] = al;
            s_beta[d] = be;
        }
    }
    __syncthreads();
}

// z = M^-1 v for the fields marked in ``live`` (others untouched); dinv
// holds D^-1 per field and cell of the tile (LDS, rounded to single
// precision: any fixed symmetric positive definite preconditioner will do,
// and the rounded diagonal is one); zt is the sweeps' work tile, which
// nothing else reads, so only the sweeps synchronise (the workgroup
// barriers of the exchange separate one call's reads of zt from the next
// call's writes); every thread of the workgroup must call it
template <int NFD, int KSW>
__device__ __forceinline__ void tile_precond(const double (&v)[NFD], double (&z)[NFD],
                                             const float* dinv, const double (&cf)[NFD],
                                             double ke, double kw, double kn, double ks,
                                             bool he, bool hw, bool hn, bool hs, double* zt,
                                             const int* live) {
    const int t = threadIdx.x;
#pragma unroll
    for (int d = 0; d < NFD; ++d)
        if (live[d]) z[d] = dinv[d * TILE_BS + t] * v[d];
#pragma unroll
    for (int sw = 0; sw < KSW; ++sw) {
#pragma unroll
        for (int d = 0; d < NFD; ++d)
            if (live[d]) zt[d * TILE_BS + t] = z[d];
        __syncthreads();
#pragma unroll
        for (int d = 0; d < NFD; ++d) {
            if (!live[d]) continue;
            const double* Z = zt + d * TILE_BS;
            double nb = 0.0;
            if (he) nb += ke * Z[t + 1];
            if (hw) nb += kw * Z[t - 1];
            if (hn) nb += kn * Z[t + TILE_X];
            if (hs) nb += ks * Z[t - TILE_X];
            z[d] = dinv[d * TILE_BS + t] * (v[d] + cf[d] * nb);
        }
        if (sw + 1 < KSW) __syncthreads();
    }
}

template <int NFD, int KSW, bool FUSED = false>
__global__ void __launch_bounds__(TILE_BS) cg_tile_kernel(CGArgs a) {
    static_assert(NFD == 9, "the edge buffer holds 9 fields per tile");
    constexpr int BS = TILE_BS;
    constexpr int NS = 3 * NFD;
    constexpr int HPT = (NFD * TILE_HALO + BS - 1) / BS;   // halo slots per thread
    // one workgroup per CU (register bound), so LDS is plentiful: the
    // preconditioner's work tile; m of this tile (the stencil's neighbours
    // inside the tile, and the edges it publishes); D^-1 and the iterate x
    // (kept out of registers); the halo of m and the groups' sums of the
    // blocks' partials
    __shared__ double zt[NFD * BS];
    __shared__ double mt[NFD * BS];
    __shared__ float dinv[NFD * BS];
    __shared__ double xt[NFD * BS];
    __shared__ double halo[NFD * TILE_HALO];
    __shared__ double stage[TILE_BS];
    __shared__ double red[NS * (BS / 64)];
    __shared__ double tot[NS];
    __shared__ double s_bb[NFD], s_gprev[NFD], s_aprev[NFD], s_alpha[NFD], s_beta[NFD];
    __shared__ int s_last;
    __shared__ int s_active[NFD];
    if (threadIdx.x < NFD) s_active[threadIdx.x] = 1;
    __syncthreads();
    const int tx = threadIdx.x % TILE_X, ty = threadIdx.x / TILE_X;
    const int gx = (blockIdx.x % a.ntx) * TILE_X + tx, gy = (blockIdx.x / a.ntx) * TILE_Y + ty;
    const bool own = gx < a.nx && gy < a.ny;
    const int64_t cell = own ? (int64_t)gy * a.nx + gx : 0;
    int64_t ie, iw, in_, is_;
    double ke, kw, kn, ks;
    double bfz[NFD];                 // the right-hand side formed here (FUSED)
    if (FUSED)
        fused_rhs<NFD>(a, cell, own, ie, iw, in_, is_, ke, kw, kn, ks, bfz);
    else
        stencil_at(a, cell, ie, iw, in_, is_, ke, kw, kn, ks);
    // neighbours inside this tile (and inside the grid)
    const bool he = own && tx + 1 < TILE_X && gx + 1 < a.nx;
    const bool hw = own && tx > 0;
    const bool hn = own && ty + 1 < TILE_Y && gy + 1 < a.ny;
    const bool hs = own && ty > 0;
    // the halo slots this thread loads after every barrier, and the edges
    // of this tile that its cell lies on
    int hsrc[HPT];
    const int x0 = (blockIdx.x % a.ntx) * TILE_X, y0 = (blockIdx.x / a.ntx) * TILE_Y;
    const int wt = min(TILE_X, a.nx - x0), ht = min(TILE_Y, a.ny - y0);
    {
        const int nty = (a.ny + TILE_Y - 1) / TILE_Y;
        const int bx = blockIdx.x % a.ntx, by = blockIdx.x / a.ntx;
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            const int e = threadIdx.x + j * BS;
            hsrc[j] = e < NFD * TILE_HALO
                          ? halo_source(a, nty, bx, by, wt, ht, e / TILE_HALO, e % TILE_HALO)
                          : -1;
        }
    }
    // the edge slots this thread publishes: LDS index of the cell in mt
    int elds[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        const int e = threadIdx.x + j * BS;
        int sl = e % TILE_HALO, lx = -1, ly = -1;
        if (e >= NFD * TILE_HALO) {
        } else if (sl < TILE_X) {
            if (sl < wt) lx = sl, ly = ht - 1;
        } else if (sl < 2 * TILE_X) {
            if (sl - TILE_X < wt) lx = sl - TILE_X, ly = 0;
        } else if (sl < 2 * TILE_X + TILE_Y) {
            if (sl - 2 * TILE_X < ht) lx = wt - 1, ly = sl - 2 * TILE_X;
        } else {
            if (sl - 2 * TILE_X - TILE_Y < ht) lx = 0, ly = sl - 2 * TILE_X - TILE_Y;
        }
        elds[j] = lx >= 0 ? (e / TILE_HALO) * BS + ly * TILE_X + lx : -1;
    }
    double cf[NFD];
#pragma unroll
    for (int d = 0; d < NFD; ++d) {
        cf[d] = a.cf[d];
        dinv[d * BS + threadIdx.x] = own ? (float)(1.0 / (1.0 + cf[d] * (ke + kw + kn + ks))) : 0.0f;
    }
    double r[NFD], u[NFD], w[NFD], zz[NFD], qq[NFD], ss[NFD], pp[NFD];
    unsigned kb = 0;
    // ---- r = b - A x0, u = M^-1 r (published), partial (b, b) ----
    // every field's values are loaded before any is used, so the prologue
    // waits for memory once (threads outside the grid load those of cell 0,
    // which exist, and discard them)
    {
        double bv[NFD], xc[NFD], xe[NFD], xw[NFD], xn[NFD], xs[NFD];
#pragma unroll
        for (int d = 0; d < NFD; ++d) {
            const size_t o = (size_t)a.fmap[d] * a.n;
            const double* X = a.guess_in_x ? a.x + o : a.b + o;
            xc[d] = X[cell];
            xe[d] = X[ie];
            xw[d] = X[iw];
            xn[d] = X[in_];
            xs[d] = X[is_];
            bv[d] = FUSED ? bfz[d] : a.b[o + cell];
        }
#pragma unroll
        for (int d = 0; d < NFD; ++d) {
            const double xi = xc[d];
            const double Ax = xi - cf[d] * (ke * (xe[d] - xi) - kw * (xi - xw[d]) +
                                            kn * (xn[d] - xi) - ks * (xi - xs[d]));
            w[d] = zz[d] = qq[d] = ss[d] = pp[d] = 0.0;
            xt[d * BS + threadIdx.x] = own ? xi : 0.0;
            r[d] = own ? bv[d] - Ax : 0.0;
        }
        wave_put_slots<BS, NFD>([&](int d) { return own ? bv[d] * bv[d] : 0.0; }, red);
    }
#pragma unroll
    for (int d = 0; d < NFD; ++d) u[d] = 0.0;
    tile_precond<NFD, KSW>(r, u, dinv, cf, ke, kw, kn, ks, he, hw, hn, hs, zt, s_active);
    // u of the tile into mt (the preconditioner has synchronised), its edges
    // and the partials (b, b) exchanged as in the iterations (exchange 0)
#pragma unroll
    for (int d = 0; d < NFD; ++d) mt[d * BS + threadIdx.x] = u[d];
    grid_exchange_first<BS, NFD, HPT>(a, red, stage, tot, mt, elds, hsrc, halo);
    ++kb;
    if (threadIdx.x < NFD) s_bb[threadIdx.x] = tot[threadIdx.x];
    // ---- w = A u (neighbours from the tile and its halo in LDS) ----
#pragma unroll
    for (int d = 0; d < NFD; ++d) {
        const double* Ut = mt + d * BS;
        const double* H = halo + d * TILE_HALO;
        if (own) {
            const int t = threadIdx.x;
            const double ui = u[d];
            const double uE = he ? Ut[t + 1] : H[2 * TILE_X + ty];
            const double uW = hw ? Ut[t - 1] : H[2 * TILE_X + TILE_Y + ty];
            const double uN = hn ? Ut[t + TILE_X] : H[tx];
            const double uS = hs ? Ut[t - TILE_X] : H[TILE_X + tx];
            w[d] = ui - cf[d] * (ke * (uE - ui) - kw * (ui - uW) + kn * (uN - ui) -
                                 ks * (ui - uS));
        }
    }
    int it = 0;
    for (; it < a.maxit; ++it) {
        // ---- m = M^-1 w (its tile edges published), partials gamma = (r,u), delta = (w,u), rr ----
        // exchange kb (the prologue's was exchange 0) uses edge half kb & 1
        double* eb = a.edge + (size_t)(kb & 1) * (TILE_EDGE_DOUBLES / 2);
        double m[NFD];
#pragma unroll
        for (int d = 0; d < NFD; ++d) m[d] = 0.0;
        tile_precond<NFD, KSW>(w, m, dinv, cf, ke, kw, kn, ks, he, hw, hn, hs, zt, s_active);
        unsigned live = 0u;                           // converged fields: nothing to reduce
#pragma unroll
        for (int d = 0; d < NFD; ++d) {
            if (!s_active[d]) continue;
            live |= 1u << d;
            mt[d * BS + threadIdx.x] = m[d];
        }
        // the 3 NFD partial sums of the wavefront in one batched reduction
        wave_put_slots<BS, NS>(
            [&](int sl) {
                const int d = sl / 3, j = sl - 3 * d;
                if (!own || !(live & (1u << d))) return 0.0;
                return (j == 1 ? w[d] : r[d]) * (j == 2 ? r[d] : u[d]);
            },
            red);
        grid_publish_arrive<BS, NFD, HPT>(a, kb, red, mt, elds, eb, s_active);
        // n = A m of the cells whose four neighbours lie in the tile, into the
        // preconditioner's (now free) tile, while the other workgroups
        // arrive; cells on the tile's edges take theirs after the exchange
        const bool inner = own && he && hw && hn && hs;
        if (inner) {
            const int t = threadIdx.x;
#pragma unroll
            for (int d = 0; d < NFD; ++d) {
                if (!(live & (1u << d))) continue;
                const double* Mt = mt + d * BS;
                const double mi = Mt[t];
                zt[d * BS + t] = mi - cf[d] * (ke * (Mt[t + 1] - mi) - kw * (mi - Mt[t - 1]) +
                                               kn * (Mt[t + TILE_X] - mi) -
                                               ks * (mi - Mt[t - TILE_X]));
            }
        }
        grid_finish_coeffs<BS, NFD, HPT>(a, kb++, it, stage, eb, hsrc, halo, s_bb, s_gprev, s_aprev,
                                         s_alpha, s_beta, s_active);
        int any = 0;
#pragma unroll
        for (int d = 0; d < NFD; ++d) any |= s_active[d];
        if (!any) break;
        // ---- n = A m (edge cells: neighbours from the tile and its halo in LDS) ; recurrences ----
#pragma unroll
        for (int d = 0; d < NFD; ++d) {
            const double* Mt = mt + d * BS;
            const double* H = halo + d * TILE_HALO;
            const bool act = s_active[d];
            const double al = s_alpha[d], be = s_beta[d];
            if (!own || !act) continue;
            const int t = threadIdx.x;
            const double mi = Mt[t];      // m of this cell, kept in LDS across the barrier
            double ni;
            if (inner) {
                ni = zt[d * BS + t];
            } else {
                const double mE = he ? Mt[t + 1] : H[2 * TILE_X + ty];
                const double mW = hw ? Mt[t - 1] : H[2 * TILE_X + TILE_Y + ty];
                const double mN = hn ? Mt[t + TILE_X] : H[tx];
                const double mS = hs ? Mt[t - TILE_X] : H[TILE_X + tx];
                ni = mi - cf[d] * (ke * (mE - mi) - kw * (mi - mW) + kn * (mN - mi) -
                                   ks * (mi - mS));
            }
            const double z1 = ni + be * zz[d];
            const double q1 = mi + be * qq[d];
            const double s1 = w[d] + be * ss[d];
            const double p1 = u[d] + be * pp[d];
            zz[d] = act ? z1 : zz[d];
            qq[d] = act ? q1 : qq[d];
            ss[d] = act ? s1 : ss[d];
            pp[d] = act ? p1 : pp[d];
            xt[d * BS + t] = xt[d * BS + t] + al * p1;     // own && act here
            r[d] = act ? r[d] - al * s1 : r[d];
            u[d] = act ? u[d] - al * q1 : u[d];
            w[d] = act ? w[d] - al * z1 : w[d];
        }
    }
    {
    double* part = a.partial + (size_t)(kb & 1u) * CG_MAX_BLOCKS * (CG_MAX_FIELDS * 4);
    if (a.cgstats) {
        // ---- the true residual |b - A x| of the result, against 10 rtol |b|
        // per field: the recurrences' residual can drift away from it, so a
        // result whose own residual fails is counted as a failed solve.  It is
        // taken over the cells whose four neighbours lie in the same tile (no
        // further exchange of x: 82 % of the cells at 32 x 16), a lower bound
        // of the whole residual, so a flagged result has failed.  Each
        // workgroup publishes its partial sums and counts itself out; the
        // last one out adds them up, so nothing is waited for ----
        const int t = threadIdx.x;
        const bool inner = own && he && hw && hn && hs;
        double bv[NFD];                               // loaded together (cell 0 off the grid)
#pragma unroll
        for (int d = 0; d < NFD; ++d) bv[d] = a.b[(size_t)a.fmap[d] * a.n + cell];
        wave_put_slots<BS, NFD>(
            [&](int d) {
                if (!inner) return 0.0;
                const double* Xt = xt + d * BS;
                const double xi = Xt[t];
                const double Ax = xi - cf[d] * (ke * (Xt[t + 1] - xi) - kw * (xi - Xt[t - 1]) +
                                                kn * (Xt[t + TILE_X] - xi) -
                                                ks * (xi - Xt[t - TILE_X]));
                const double res = bv[d] - Ax;
                return res * res;
            },
            red);
        __syncthreads();
        for (int q = threadIdx.x; q < NFD; q += BS) {
            double v = 0.0;
            for (int w2 = 0; w2 < BS / 64; ++w2) v += red[q * (BS / 64) + w2];
            __hip_atomic_store(&part[(size_t)blockIdx.x * (CG_MAX_FIELDS * 4) + q], v,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // every workgroup counts itself out (after its last grid wait); the last
    // one adds up the residual check's partials and clears the barrier
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = __hip_atomic_fetch_add(&a.bar[BAR_EXIT], 1u, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) + 1u == gridDim.x;
    __syncthreads();
    if (s_last) {                                     // uniform over the workgroup
        if (a.cgstats) {
            stage[threadIdx.x] = group_partial(part, gridDim.x, NFD);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (a.cgstats) {
                // a solve already failed at maxit is not counted twice; NaN fails
                int bad = 0, open_fields = 0;
                for (int d = 0; d < NFD; ++d) {
                    bad |= !(slot_total(stage, d) <= 100.0 * a.rtol2 * s_bb[d]);
                    open_fields |= s_active[d];
                }
                a.cgstats[5] += (it == a.maxit && open_fields) ? 0 : bad;
            }
            {
                // every barrier word back to zero for the next launch on this
                // work space (all workgroups are past their last wait), so a
                // solve that forms its own right-hand side needs no pass to
                // clear them
                __hip_atomic_store(&a.bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&a.bar[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int g = 0; g < BAR_GROUPS; ++g)
                    __hip_atomic_store(&a.bar[BAR_STRIDE * (1 + g)], 0u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&a.bar[BAR_GLOBAL], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&a.bar[BAR_EXIT], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    }
#pragma unroll
    for (int d = 0; d < NFD; ++d)
        if (own) a.x[(size_t)a.fmap[d] * a.n + cell] = xt[d * BS + threadIdx.x];
    if (a.close && own) {
        // bath closure of this cell, then T and theta of the closed state
        // (species in order, as a separate closure pass would take them).
        // The diffused fields are the N - 1 species other than the bath and
        // h, so N = NFD here; the right-hand sides and the species tables
        // are loaded together before they are used.
        const int t = threadIdx.x;
        double bk[NFD], hf_k[NFD], cp_k[NFD], iw_k[NFD];
#pragma unroll
        for (int k = 0; k < NFD; ++k) {
            bk[k] = a.b[(size_t)k * a.n + cell];
            hf_k[k] = a.hf[k];
            cp_k[k] = a.cp[k];
            iw_k[k] = a.invW[k];
        }
        double sum = 0.0, bb = 0.0;
#pragma unroll
        for (int k = 0; k < NFD; ++k) {
            if (k == a.bath) {
                bb = bk[k];
                continue;
            }
            sum += xt[a.dmap[k] * BS + t] - bk[k];
        }
        const double yb = bb - sum;
        a.x[(size_t)a.bath * a.n + cell] = yb;
        if (a.T_out) {
            double hform = 0.0, cpm = 0.0;
#pragma unroll
            for (int k = 0; k < NFD; ++k) {
                const double yk = (k == a.bath) ? yb : xt[a.dmap[k] * BS + t];
                hform += yk * hf_k[k] * iw_k[k];
                cpm += yk * cp_k[k] * iw_k[k];
            }
            const double Ti = T_REF + (xt[a.dmap[a.N] * BS + t] - hform) / cpm;
            a.T_out[cell] = Ti;
            if (a.th_out) a.th_out[cell] = pow(Ti / T_DIFF_REF, THETA_EXP);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.info[0] = it;
        int any = 0;
        for (int d = 0; d < NFD; ++d) any |= s_active[d];
        a.info[1] = (it == a.maxit) ? any : 0;
        if (a.close && a.cgstats) {
            // a barrier timeout flagged by another workgroup after this one
            // got here is counted with the next solve
            const int to = __hip_atomic_exchange(&a.info[2], 0, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            a.cgstats[0] += it;
            a.cgstats[1] = it > a.cgstats[1] ? it : a.cgstats[1];
            a.cgstats[2] += a.info[1];
            a.cgstats[3] += 1;
            a.cgstats[4] += to;
        }
    }
}


}  // namespace

int64_t cg_tile_blocks(const Grid& g) {
    if (g.dim != 2 || g.n_flames > 0) return 0;
    return ((g.nx + TILE_X - 1) / TILE_X) * ((g.ny + TILE_Y - 1) / TILE_Y);
}

int64_t cg_regs_min_blocks(int64_t n, int cpt) {
    const int64_t per = (int64_t)cg_regs_block(cpt) * cpt;
    return (n + per - 1) / per;
}

int device_cus(int& cus) {
    int dev = 0;
    MISDC_HIP(hipGetDevice(&dev));
    MISDC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    return MISDC_OK;
}

int diffusion_work_set(DiffusionWork& w, const Mech& m, const Grid& g, int variant, int blocks) {
    const int64_t n = g.cells();
    const int NF = m.dev.N + 1;
    int cus = 0;
    int rc = device_cus(cus);
    if (rc) return rc;
    const int cap = cus < CG_MAX_BLOCKS ? cus : CG_MAX_BLOCKS;
    if (blocks < 1 || blocks > cap)
        return fail(MISDC_EINVAL, "CG blocks must be in [1, %d], got %d", cap, blocks);
    int occ = 0;
    switch (variant) {
        case 0:
            MISDC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, cg_kernel, CG_THREADS, 0));
            break;
        case 1:
        case 2:
        case 4:
            if (!(NF - 1 == 9 && g.dim == 2 && g.n_flames == 0))
                return fail(MISDC_EINVAL, "register CG variants need a 2-D grid and 9 diffused fields");
            if (blocks < cg_regs_min_blocks(n, variant))
                return fail(MISDC_EINVAL, "CG variant %d needs at least %lld blocks", variant,
                            (long long)cg_regs_min_blocks(n, variant));
            if (variant == 1)
                MISDC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, cg_regs_kernel<9, 1, 512>, 512, 0));
            else if (variant == 2)
                MISDC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, cg_regs_kernel<9, 2, 256>, 256, 0));
            else
                MISDC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, cg_regs_kernel<9, 4, 256>, 256, 0));
            break;
        case 101:
        case 102:
        case 103: {
            if (!(NF - 1 == 9 && g.dim == 2 && g.n_flames == 0))
                return fail(MISDC_EINVAL, "tiled CG variants need a 2-D grid and 9 diffused fields");
            if (!w.edge) return fail(MISDC_EINVAL, "tiled CG: no edge buffer");
            const int64_t tiles = ((g.nx + TILE_X - 1) / TILE_X) * ((g.ny + TILE_Y - 1) / TILE_Y);
            if (blocks != tiles || tiles > TILE_NB)
                return fail(MISDC_EINVAL, "tiled CG: the grid has %lld tiles of %dx%d (at most %d), "
                            "blocks must equal them", (long long)tiles, TILE_X, TILE_Y, TILE_NB);
            if (variant == 101)
                MISDC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, cg_tile_kernel<9, 1>, TILE_BS, 0));
            else if (variant == 102)
                MISDC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, cg_tile_kernel<9, 2>, TILE_BS, 0));
            else
                MISDC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, cg_tile_kernel<9, 3>, TILE_BS, 0));
            break;
        }
        default:
            return fail(MISDC_EINVAL, "unknown CG variant %d", variant);
    }
    if (occ < 1) return fail(MISDC_EDEVICE, "CG variant %d cannot be resident", variant);
    w.variant = variant;
    w.blocks = blocks;
    return MISDC_OK;
}

int launch_cg(const CGArgs& a, int variant, int blocks, hipStream_t s) {
    switch (variant) {
        case 1: hipLaunchKernelGGL((cg_regs_kernel<9, 1, 512>), dim3(blocks), dim3(512), 0, s, a); break;
        case 2: hipLaunchKernelGGL((cg_regs_kernel<9, 2, 256>), dim3(blocks), dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL((cg_regs_kernel<9, 4, 256>), dim3(blocks), dim3(256), 0, s, a); break;
        case 101:
            if (a.lag_src)
                hipLaunchKernelGGL((cg_tile_kernel<9, 1, true>), dim3(blocks), dim3(TILE_BS), 0, s, a);
            else
                hipLaunchKernelGGL((cg_tile_kernel<9, 1>), dim3(blocks), dim3(TILE_BS), 0, s, a);
            break;
        case 102: hipLaunchKernelGGL((cg_tile_kernel<9, 2>), dim3(blocks), dim3(TILE_BS), 0, s, a); break;
        case 103: hipLaunchKernelGGL((cg_tile_kernel<9, 3>), dim3(blocks), dim3(TILE_BS), 0, s, a); break;
        case 0: hipLaunchKernelGGL(cg_kernel, dim3(blocks), dim3(CG_THREADS), 0, s, a); break;
        default: return fail(MISDC_EINVAL, "unknown CG variant %d", variant);
    }
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

}  // namespace misdc
