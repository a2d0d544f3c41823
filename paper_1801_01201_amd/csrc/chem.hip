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

#include "chem_dev.h"
#include "misdc_impl.h"
#include "newton_hist.h"

namespace misdc {

namespace {

template <int NS, bool INERT_LAST>
__global__ void __launch_bounds__(64) newton_kernel(MechDev m, NewtonArgs a) {
    // A wavefront iterates until its slowest cell has converged.  On a 2-D
    // grid a compact tile of cells keeps cells at similar distances from a
    // flame front together, so its iteration counts differ less than along
    // 64 cells of a row (256 x 256 flame, 8 x 8 tiles: the mean per-wavefront
    // maximum falls from 2.8 to 2.3 iterations, against a mean of 2.2).  A
    // 16 x 4 tile keeps most of that and reads whole 128-byte lines: no line
    // is fetched by two workgroups.  Lanes outside the grid take i = n.
    int64_t i;
    if (a.tile_nx > 0) {
        const int ntx = (a.tile_nx + NEWTON_TILE_X - 1) / NEWTON_TILE_X;
        const int x = (int)(blockIdx.x % ntx) * NEWTON_TILE_X + (int)(threadIdx.x % NEWTON_TILE_X);
        const int y = (int)(blockIdx.x / ntx) * NEWTON_TILE_Y + (int)(threadIdx.x / NEWTON_TILE_X);
        i = (x < a.tile_nx && y < a.tile_ny) ? (int64_t)y * a.tile_nx + x : a.n;
    } else {
        i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    }
    const int code = newton_cell<NS, INERT_LAST>(m, a, i);
    newton_wave_stats(a, blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64, i < a.n, code);
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

// T of every cell; with copy set (state layout, ldy = n), the N+1 fields of
// the cell are copied there in the same pass
__global__ void __launch_bounds__(256) temperature_kernel(MechDev m, int64_t n, const double* Yp,
                                                          int64_t ldy, const double* hp,
                                                          double* Tp, double* copy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double hform = 0.0, cpm = 0.0;
    for (int k = 0; k < m.N; ++k) {
        const double y = Yp[k * ldy + i];
        if (copy) copy[k * n + i] = y;
        hform += y * m.hf[k] * m.invW[k];
        cpm += y * m.cp[k] * m.invW[k];
    }
    const double h = hp[i];
    if (copy) copy[(int64_t)m.N * n + i] = h;
    Tp[i] = T_REF + (h - hform) / cpm;
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
                       n, h, T, nullptr);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_state_temperature(const Mech& m, int64_t n, const double* state, double* T,
                             hipStream_t s, double* copy) {
    if (n == 0) return MISDC_OK;
    hipLaunchKernelGGL(temperature_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, m.dev, n,
                       state, n, state + (size_t)m.dev.N * n, T, copy);
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
    if (!thread) {
        // the wavefront kernels leave the copy of h to a pass of its own
        if (a.h_out) {
            const int rc = launch_copy(a.h_out, a.h, a.n, s);
            if (rc) return rc;
        }
        if (a.th_out && !a.T)
            return fail(MISDC_EINVAL, "theta of the reaction solve's result needs its T");
        const int rc = launch_reaction_newton_wave(m, a, a.opt.lu, s);
        if (rc || !a.th_out) return rc;
        return launch_theta(a.n, a.T, a.th_out, s);
    }
    if (m.dev.N != 9)
        return fail(MISDC_EUNSUPPORTED, "per-thread reaction solve: %d species not built", m.dev.N);
    int64_t blocks = grid_for(a.n, 64);
    if (a.tile_nx > 0) {
        if (a.tile_ny <= 0 || (int64_t)a.tile_nx * a.tile_ny != a.n)
            return fail(MISDC_EINVAL, "tiled reaction solve: %d x %d cells for n = %lld", a.tile_nx,
                        a.tile_ny, (long long)a.n);
        blocks = (int64_t)((a.tile_nx + NEWTON_TILE_X - 1) / NEWTON_TILE_X) *
                 ((a.tile_ny + NEWTON_TILE_Y - 1) / NEWTON_TILE_Y);
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
