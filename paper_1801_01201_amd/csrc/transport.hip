// Transport kernels: explicit advection/diffusion operators, the linear
// combinations that assemble the SDC right-hand sides, the face coefficients
// and the 1-D (cyclic tridiagonal) implicit diffusion solves of steps S3/S4,
// and the launcher of the 2-D solves, whose persistent conjugate-gradient
// kernels are in cg.hip.
//
// All field arrays are structure of arrays (field-major, cells contiguous,
// x fastest), so every kernel below reads and writes whole 512-byte
// wavefront segments.
#include <cmath>
#include <cstdlib>

#include "cg.h"
#include "flame_dev.h"
#include "misdc_impl.h"
#include "wave.h"

namespace misdc {

namespace {

inline unsigned grid_for(int64_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

// ---------------------------------------------------------------------------
// linear combinations
// ---------------------------------------------------------------------------
// acc[p] = sum over the terms t, in ascending order, of W[p][t] X[t][e] (the
// terms in smask times the cell's scale) for element e = f * ncells + cell.
// A batch of LC_BATCH terms is loaded before any of them is used, so that
// the batch waits for memory once (the kernels below are bound by that
// latency, not by bandwidth, when every term waits in turn).
constexpr int LC_BATCH = 8;

__device__ __forceinline__ void lincomb_element(const LinComb& lc, int f, int64_t cell,
                                                double (&acc)[LC_MAX_OUT]) {
    const int64_t e = (int64_t)f * lc.ncells + cell;
    const double sc = lc.smask ? lc.scale[cell] : 1.0;
#pragma unroll
    for (int p = 0; p < LC_MAX_OUT; ++p) acc[p] = 0.0;
    for (int t0 = 0; t0 < lc.nterms; t0 += LC_BATCH) {
        double v[LC_BATCH];
#pragma unroll
        for (int c = 0; c < LC_BATCH; ++c) {
            const int t = t0 + c;
            v[c] = (t < lc.nterms && f < lc.nf[t]) ? lc.X[t][e] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < LC_BATCH; ++c) {
            const int t = t0 + c;
            if (t >= lc.nterms || f >= lc.nf[t]) continue;
            double x = v[c];
            if ((lc.smask >> t) & 1u) x *= sc;
#pragma unroll
            for (int p = 0; p < LC_MAX_OUT; ++p)
                if (p < lc.nout) acc[p] += lc.W[p][t] * x;
        }
    }
}

// one field per blockIdx.y, cells over blockIdx.x (grid-stride)
__global__ void __launch_bounds__(256) lincomb_kernel(LinComb lc) {
    const int f = (int)blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < lc.ncells;
         i += (int64_t)gridDim.x * blockDim.x) {
        double acc[LC_MAX_OUT];
        lincomb_element(lc, f, i, acc);
        const int64_t e = (int64_t)f * lc.ncells + i;
#pragma unroll
        for (int p = 0; p < LC_MAX_OUT; ++p)
            if (p < lc.nout) lc.out[p][e] = acc[p];
    }
}

__global__ void __launch_bounds__(256) theta_kernel(int64_t n, const double* T, double* th) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) th[i] = pow(T[i] / T_DIFF_REF, THETA_EXP);
}

__global__ void __launch_bounds__(256) copy_kernel(double* dst, const double* src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void __launch_bounds__(256) zero_kernel(unsigned* dst, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = 0u;
}

struct ZeroMany {
    unsigned* dst[4];
    int64_t words[4];
};
// blockIdx.y picks the buffer
__global__ void __launch_bounds__(256) zero_many_kernel(ZeroMany z) {
    unsigned* d = z.dst[blockIdx.y];
    const int64_t words = z.words[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        d[i] = 0u;
}

__global__ void __launch_bounds__(256) expand_kernel(int n_flames, const int64_t* off,
                                                     const double* v, double* out) {
    const int f = blockIdx.y;
    if (f >= n_flames) return;
    const int64_t b = off[f], e = off[f + 1];
    const double x = v[f];
    for (int64_t i = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < e;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = x;
}

// ---------------------------------------------------------------------------
// explicit operators
// ---------------------------------------------------------------------------
// one thread per cell; the stencil values of ten fields (every field of a
// 9-species mechanism) are loaded before any result is stored
constexpr int TRANSPORT_CHUNK = 10;

template <bool FROM_T>
__global__ void __launch_bounds__(256) transport_kernel(GridDev g, MechDev m, int64_t n,
                                                        const double* st, const double* T,
                                                        double* th, double* FA, double* FD) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    transport_cell<FROM_T, TRANSPORT_CHUNK>(g, m, n, st, T, th, FA, FD, i);
}

// ---------------------------------------------------------------------------
// implicit diffusion
// ---------------------------------------------------------------------------

// every counter of the grid barriers (see BAR_WORDS)
__device__ __forceinline__ void zero_barrier(unsigned* bar) {
    bar[0] = 0u;
    bar[1] = 0u;
    for (int g = 0; g < BAR_GROUPS; ++g) bar[BAR_STRIDE * (1 + g)] = 0u;
    bar[BAR_GLOBAL] = 0u;
    bar[BAR_EXIT] = 0u;
}

__global__ void __launch_bounds__(256) faces_kernel(GridDev g, int64_t n, const double* T,
                                                    double* th, double* Kx, double* Ky,
                                                    unsigned* bar) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the persistent CG kernel that follows on this stream counts its grid
    // barriers from zero
    if (i == 0 && bar) zero_barrier(bar);
    if (i >= n) return;
    faces_at(g, i, T, th, Kx, Ky);
}

// The right-hand side of a diffusion solve and, in the same pass, the face
// coefficients of its lagged operator (by the blocks of field 0).
__global__ void __launch_bounds__(256) lincomb_faces_kernel(LinComb lc, GridDev g, const double* T,
                                                            double* th, double* Kx, double* Ky,
                                                            unsigned* bar) {
    const int f = (int)blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f == 0 && i0 == 0 && bar) zero_barrier(bar);
    for (int64_t i = i0; i < lc.ncells; i += (int64_t)gridDim.x * blockDim.x) {
        if (f == 0) faces_at(g, i, T, th, Kx, Ky);
        double acc[LC_MAX_OUT];
        lincomb_element(lc, f, i, acc);
        const int64_t e = (int64_t)f * lc.ncells + i;
#pragma unroll
        for (int p = 0; p < LC_MAX_OUT; ++p)
            if (p < lc.nout) lc.out[p][e] = acc[p];
    }
}

// out = part + scale (qa FA + qd FD + qr FR) of every field at one cell, FA
// and FD at src, the stencil values of all fields loaded before any
// is used (as in transport_fields); the face coefficients of the lagged
// operator at T in the same pass (see launch_lag_rhs)
template <bool TWO_D>
__device__ __forceinline__ void lag_rhs_cell(const Stencil& s, const MechDev& m, int64_t n,
                                             const LagRhs& a, double sc, int64_t i) {
    constexpr int CH = TRANSPORT_CHUNK;
    const int NF = m.N + 1;
    const double wa = sc * a.qa, wd = sc * a.qd, wr = sc * a.qr;
    double fd_sum = 0.0, fa_bath = 0.0, part_bath = 0.0, fr_bath = 0.0;
    for (int f0 = 0; f0 < NF; f0 += CH) {
        double v[CH][9], pv[CH], rv[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int f = f0 + c < NF ? f0 + c : NF - 1;
            load_stencil<TWO_D>(s, a.src + (size_t)f * n, i, v[c]);
            pv[c] = a.part[(size_t)f * n + i];
            // FR has the N species only (the enthalpy's entry stays unused)
            rv[c] = a.fr ? a.fr[(size_t)(f < m.N ? f : m.N - 1) * n + i] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int f = f0 + c;
            if (f >= NF) continue;
            double fa, lap;
            field_ops<TWO_D>(s, v[c], fa, lap);
            const double fr = f < m.N ? rv[c] : 0.0;
            if (f == m.bath) {
                fa_bath = fa;
                part_bath = pv[c];
                fr_bath = fr;
                continue;
            }
            const double fd = m.kappa0[f] * lap;
            if (f < m.N) fd_sum += fd;
            a.out[(size_t)f * n + i] = pv[c] + (wa * fa + wd * fd + wr * fr);
        }
    }
    a.out[(size_t)m.bath * n + i] = part_bath + (wa * fa_bath + wd * -fd_sum + wr * fr_bath);
}

__global__ void __launch_bounds__(256) lag_rhs_kernel(GridDev g, MechDev m, int64_t n, LagRhs a,
                                                      double* th_out, double* Kx, double* Ky,
                                                      unsigned* bar) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the persistent CG kernel that follows on this stream counts its grid
    // barriers from zero
    if (i == 0 && bar) zero_barrier(bar);
    if (i >= n) return;
    faces_at(g, i, a.T_lag, th_out, Kx, Ky);
    auto theta = [&](int64_t j) {
        return a.T_src ? pow(a.T_src[j] / T_DIFF_REF, THETA_EXP) : a.th[j];
    };
    const Stencil s = stencil_at(g, i, theta(i), theta);
    const double sc = a.scale ? a.scale[i] : 1.0;
    if (s.two_d)
        lag_rhs_cell<true>(s, m, n, a, sc, i);
    else
        lag_rhs_cell<false>(s, m, n, a, sc, i);
}

// Cyclic tridiagonal solve of (I - cf L) y = r on one periodic 1-D system per
// thread: Thomas' algorithm on the tridiagonal part plus a Sherman-Morrison
// correction for the two corner entries.  Work arrays w1, w2 (same layout as
// y) hold the modified super-diagonal and the correction vector.
__global__ void __launch_bounds__(64) cyclic_kernel(GridDev g, MechDev m, int64_t n, double c,
                                                    const double* dtf, double cfac,
                                                    const double* Kx, const double* rhs,
                                                    double* y, double* w1, double* w2) {
    const int nsys_f = g.n_flames > 0 ? g.n_flames : 1;
    const int fields = m.N + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsys_f * fields) return;
    const int f = t / nsys_f, fl = t % nsys_f;
    if (f == m.bath) return;
    const int64_t base = g.n_flames > 0 ? g.off[fl] : 0;
    const int64_t len = g.n_flames > 0 ? g.off[fl + 1] - g.off[fl] : n;
    const double cc = (dtf ? dtf[fl] * cfac : c) * m.kappa0[f];
    const double* b = rhs + (size_t)f * n + base;
    double* x = y + (size_t)f * n + base;
    double* cp = w1 + (size_t)f * n + base;
    double* u = w2 + (size_t)f * n + base;
    const double* K = Kx + base;
    // row i: -cc Kw y_{i-1} + (1 + cc (Kw + Ke)) y_i - cc Ke y_{i+1}
    auto sub = [&](int64_t i) { return -cc * K[(i - 1 + len) % len]; };   // a_i
    auto sup = [&](int64_t i) { return -cc * K[i]; };                     // c_i
    auto dia = [&](int64_t i) { return 1.0 + cc * (K[(i - 1 + len) % len] + K[i]); };
    if (len == 1) { x[0] = b[0]; return; }
    const double a0 = sub(0), cN = sup(len - 1);
    const double gam = -dia(0);
    // modified diagonal: d0 - gam, d_{n-1} - a0 cN / gam
    // forward sweep for two right-hand sides: b and the vector (gam, 0, .., cN)
    double dprev = dia(0) - gam;
    double cprev = sup(0) / dprev;
    cp[0] = cprev;
    x[0] = b[0] / dprev;
    u[0] = gam / dprev;
    for (int64_t i = 1; i < len; ++i) {
        double d = dia(i);
        if (i == len - 1) d -= a0 * cN / gam;
        const double ai = sub(i);
        const double den = d - ai * cprev;
        const double rb = b[i];
        const double ru = (i == len - 1) ? cN : 0.0;
        x[i] = (rb - ai * x[i - 1]) / den;
        u[i] = (ru - ai * u[i - 1]) / den;
        cprev = (i < len - 1) ? sup(i) / den : 0.0;
        cp[i] = cprev;
    }
    for (int64_t i = len - 2; i >= 0; --i) {
        x[i] -= cp[i] * x[i + 1];
        u[i] -= cp[i] * u[i + 1];
    }
    // v = (1, 0, ..., 0, a0 / gam)
    const double vy = x[0] + a0 / gam * x[len - 1];
    const double vu = u[0] + a0 / gam * u[len - 1];
    const double fct = vy / (1.0 + vu);
    for (int64_t i = 0; i < len; ++i) x[i] -= fct * u[i];
}

__global__ void __launch_bounds__(64) cyclic_wave_kernel(GridDev g, MechDev m, int64_t n, double c,
                                                         const double* dtf, double cfac,
                                                         const double* Kx, const double* rhs,
                                                         double* y, double* sc, double* su,
                                                         double* sv, double* sw) {
    const int nsys_f = g.n_flames > 0 ? g.n_flames : 1;
    cyclic_wave_system(g, m, n, c, dtf, cfac, Kx, rhs, y, sc, su, sv, sw, blockIdx.x / nsys_f,
                       blockIdx.x % nsys_f);
}

__global__ void __launch_bounds__(256) closure_kernel(MechDev m, int64_t n, const double* rhs,
                                                      double* y, double* T_out, double* th_out,
                                                      int32_t* info, int32_t* cgstats) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && cgstats) {
        // accumulate the statistics of the CG solve that preceded on this
        // stream: [0] iterations, [1] max, [2] failures, [3] solves, [4] timeouts
        cgstats[0] += info[0];
        cgstats[1] = info[0] > cgstats[1] ? info[0] : cgstats[1];
        cgstats[2] += info[1];
        cgstats[3] += 1;
        cgstats[4] += info[2];
        info[2] = 0;
    }
    if (i >= n) return;
    closure_cell(m, n, rhs, y, T_out, th_out, i);
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
// max |a - b| and max |a| per field: per-block partials, and the block that
// finishes last reduces them in block order (one launch; the arrival counter
// `done` is reset by that block)
__global__ void __launch_bounds__(256) diffmax_kernel(int nfields, int64_t n, const double* a,
                                                      const double* b, double* partial,
                                                      double* out, unsigned* done) {
    __shared__ double sd[4], sa[4];
    __shared__ int s_last;
    const int f = blockIdx.y;
    double md = 0.0, ma = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double va = a[(size_t)f * n + i];
        md = fmax(md, fabs(va - b[(size_t)f * n + i]));
        ma = fmax(ma, fabs(va));
    }
    for (int off = 32; off > 0; off >>= 1) {
        md = fmax(md, __shfl_xor(md, off));
        ma = fmax(ma, __shfl_xor(ma, off));
    }
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    if (lane == 0) { sd[wave] = md; sa[wave] = ma; }
    __syncthreads();
    if (threadIdx.x == 0) {
        md = 0.0;
        ma = 0.0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) {
            md = fmax(md, sd[w]);
            ma = fmax(ma, sa[w]);
        }
        partial[((size_t)f * gridDim.x + blockIdx.x) * 2 + 0] = md;
        partial[((size_t)f * gridDim.x + blockIdx.x) * 2 + 1] = ma;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned total = gridDim.x * gridDim.y;
        s_last = __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                 total - 1u;
    }
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // one wavefront per field: its lanes take the blocks' partials, then a
    // wavefront maximum (max is exact in any order)
    const int nblocks = (int)gridDim.x, nw = (int)(blockDim.x / 64);
    for (int g = wave; g < nfields; g += nw) {
        double gd = 0.0, ga = 0.0;
        for (int bk = lane; bk < nblocks; bk += 64) {
            gd = fmax(gd, partial[((size_t)g * nblocks + bk) * 2 + 0]);
            ga = fmax(ga, partial[((size_t)g * nblocks + bk) * 2 + 1]);
        }
        for (int off = 32; off > 0; off >>= 1) {
            gd = fmax(gd, __shfl_xor(gd, off));
            ga = fmax(ga, __shfl_xor(ga, off));
        }
        if (lane == 0) {
            out[2 * g] = gd;
            out[2 * g + 1] = ga;
        }
    }
    if (threadIdx.x == 0) *done = 0u;
}

GridDev grid_dev(const Grid& g) {
    GridDev d;
    d.dim = g.dim;
    d.nx = g.n_flames > 0 ? g.cells() : g.nx;
    d.ny = g.n_flames > 0 ? 1 : g.ny;
    d.dx = g.dx;
    d.dy = g.dy;
    d.ux = g.ux;
    d.uy = g.uy;
    d.n_flames = g.n_flames;
    d.off = g.d_off;
    d.fdx = g.d_dx;
    d.fu = g.d_u;
    return d;
}

}  // namespace

// blocks of 256 cells along x (at most 65535; the kernels stride over the
// rest), one field per y; x = 0 when the fields do not fit a grid's y range
int launch_theta(int64_t n, const double* T, double* th, hipStream_t s) {
    if (n == 0) return MISDC_OK;
    hipLaunchKernelGGL(theta_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, n, T, th);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

static dim3 lincomb_grid(const LinComb& lc) {
    if (lc.nfields < 1 || lc.nfields > 65535) return dim3(0, 1, 1);
    unsigned bx = grid_for(lc.ncells, 256);
    if (bx > 65535u) bx = 65535u;
    return dim3(bx, (unsigned)lc.nfields, 1);
}

int launch_copy(double* dst, const double* src, int64_t count, hipStream_t s) {
    if (count <= 0) return MISDC_OK;
    unsigned blocks = grid_for(count, 256);
    if (blocks > 8192u) blocks = 8192u;
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, s, dst, src, count);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}


int launch_zero_many(void* const* dst, const int64_t* bytes, int count, hipStream_t s) {
    if (count < 1 || count > 4) return fail(MISDC_EINVAL, "zero fill of %d buffers", count);
    ZeroMany z;
    int64_t most = 0;
    for (int k = 0; k < count; ++k) {
        if (bytes[k] < 0 || bytes[k] % 4)
            return fail(MISDC_EINVAL, "zero fill of %lld bytes: not whole words", (long long)bytes[k]);
        z.dst[k] = (unsigned*)dst[k];
        z.words[k] = bytes[k] / 4;
        most = z.words[k] > most ? z.words[k] : most;
    }
    if (most == 0) return MISDC_OK;
    unsigned blocks = grid_for(most, 256);
    if (blocks > 8192u) blocks = 8192u;
    hipLaunchKernelGGL(zero_many_kernel, dim3(blocks, (unsigned)count), dim3(256), 0, s, z);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_zero(void* dst, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return MISDC_OK;
    if (bytes % 4) return fail(MISDC_EINVAL, "zero fill of %lld bytes: not whole words", (long long)bytes);
    const int64_t words = bytes / 4;
    unsigned blocks = grid_for(words, 256);
    if (blocks > 8192u) blocks = 8192u;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, s, (unsigned*)dst, words);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_expand_flames(const Grid& g, const double* v, double* out, hipStream_t s) {
    if (g.n_flames <= 0) return fail(MISDC_EINVAL, "per-flame values need an ensemble grid");
    int64_t longest = 0;
    for (int64_t L : g.len) longest = L > longest ? L : longest;
    hipLaunchKernelGGL(expand_kernel, dim3(grid_for(longest, 256), g.n_flames), dim3(256), 0, s,
                       g.n_flames, g.d_off, v, out);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_lincomb_faces(const LinComb& lc, const Grid& g, const double* T_lag, DiffusionWork& w,
                         hipStream_t s) {
    const int64_t total = (int64_t)lc.nfields * lc.ncells;
    if (total == 0) return MISDC_OK;
    if (lc.nterms > LC_MAX_TERMS || lc.nout > LC_MAX_OUT || lc.nout < 1)
        return fail(MISDC_EINVAL, "linear combination too large (%d terms, %d outputs)", lc.nterms,
                    lc.nout);
    if (lc.smask && !lc.scale) return fail(MISDC_EINVAL, "scaled terms without a scale array");
    if (lc.ncells != g.cells()) return fail(MISDC_EINVAL, "linear combination and grid differ");
    const dim3 grid = lincomb_grid(lc);
    if (!grid.x) return fail(MISDC_EINVAL, "linear combination of %d fields", lc.nfields);
    hipLaunchKernelGGL(lincomb_faces_kernel, grid, dim3(256), 0, s, lc, grid_dev(g), T_lag,
                       w.theta, w.Kx, w.Ky, w.barrier);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_lag_rhs(const Mech& m, const Grid& g, const LagRhs& a, DiffusionWork& w, hipStream_t s) {
    const int64_t n = g.cells();
    if (n == 0) return MISDC_OK;
    if (!a.src || !(a.th || a.T_src) || !a.part || !a.out || !a.T_lag)
        return fail(MISDC_EINVAL, "split right-hand side: missing array");
    hipLaunchKernelGGL(lag_rhs_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, grid_dev(g), m.dev,
                       n, a, w.theta, w.Kx, w.Ky, w.barrier);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_lincomb(const LinComb& lc, hipStream_t s) {
    const int64_t total = (int64_t)lc.nfields * lc.ncells;
    if (total == 0) return MISDC_OK;
    if (lc.nterms > LC_MAX_TERMS || lc.nout > LC_MAX_OUT || lc.nout < 1)
        return fail(MISDC_EINVAL, "linear combination too large (%d terms, %d outputs)", lc.nterms,
                    lc.nout);
    if (lc.smask && !lc.scale) return fail(MISDC_EINVAL, "scaled terms without a scale array");
    const dim3 grid = lincomb_grid(lc);
    if (!grid.x) return fail(MISDC_EINVAL, "linear combination of %d fields", lc.nfields);
    hipLaunchKernelGGL(lincomb_kernel, grid, dim3(256), 0, s, lc);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_transport(const Mech& m, const Grid& g, const double* state, const double* T,
                     double* FA, double* FD, double* work_theta, hipStream_t s, bool theta_ready) {
    const int64_t n = g.cells();
    if (n == 0) return MISDC_OK;
    // theta from T inside the same kernel unless the caller already has it
    if (theta_ready)
        hipLaunchKernelGGL(transport_kernel<false>, dim3(grid_for(n, 256)), dim3(256), 0, s,
                           grid_dev(g), m.dev, n, state, T, work_theta, FA, FD);
    else
        hipLaunchKernelGGL(transport_kernel<true>, dim3(grid_for(n, 256)), dim3(256), 0, s,
                           grid_dev(g), m.dev, n, state, T, work_theta, FA, FD);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

namespace {

// Launch configuration of a diffusion workspace whose buffers are in place
// (the tiled variants need w.edge).
int diffusion_work_choose(DiffusionWork& w, const Mech& m, const Grid& g) {
    const int64_t n = g.cells();
    const int NF = m.dev.N + 1;
    int cus = 0;
    int rc = device_cus(cus);
    if (rc) return rc;
    // At most one block per CU: the whole grid is co-resident even while
    // other kernels occupy part of every CU, so the grid barrier always
    // completes.  The register-resident kernel is used when every cell fits
    // in CPT <= 4 registers slots per thread of such a grid.
    w.variant = -1;
    // the tiled variant (one 32x16 tile per workgroup, one local
    // preconditioner sweep) where the grid has at most 128 tiles: fewer
    // iterations than the diagonal preconditioner at a small cost each
    const int64_t tiles = cg_tile_blocks(g);
    if (NF - 1 == 9 && tiles >= 1 && tiles <= cus && tiles <= TILE_NB)
        (void)diffusion_work_set(w, m, g, 101, (int)tiles);
    if (w.variant < 0 && NF - 1 == 9 && g.dim == 2 && g.n_flames == 0) {
        // grid barriers cost less with fewer blocks, so take the fewest cells
        // per thread that keeps the grid at most half the CUs, else at most
        // all of them
        const int cpts[3] = {1, 2, 4};
        for (int pass = 0; pass < 2 && w.variant < 0; ++pass) {
            const int64_t cap = pass == 0 ? cus / 2 : cus;
            for (int c : cpts) {
                const int64_t blocks = cg_regs_min_blocks(n, c);
                if (blocks > cap) continue;
                if (diffusion_work_set(w, m, g, c, (int)blocks) == MISDC_OK) break;
            }
        }
    }
    if (w.variant < 0) {
        int64_t blocks = (n + CG_THREADS - 1) / CG_THREADS;
        if (blocks > cus) blocks = cus;
        if (blocks > CG_MAX_BLOCKS) blocks = CG_MAX_BLOCKS;
        if (blocks < 1) blocks = 1;
        rc = diffusion_work_set(w, m, g, 0, (int)blocks);
        if (rc) return rc;
    }
    w.threads = CG_THREADS;
    w.fields_cap = NF;
    return MISDC_OK;
}

// Sizes in bytes of the workspace buffers, in carving order: theta, Kx, Ky,
// x, r, z, p, q, edge, partial, totals, barrier, info.
constexpr int WORK_PARTS = 13;
void diffusion_work_sizes(const Mech& m, const Grid& g, size_t (&sz)[WORK_PARTS]) {
    const size_t cells = (size_t)g.cells() * sizeof(double);
    const int NF = m.dev.N + 1;
    const bool tiled = g.dim == 2 && g.n_flames == 0 && NF - 1 == 9;
    const size_t parts[WORK_PARTS] = {
        cells, cells, cells, cells * NF, cells * NF, cells * NF, cells * NF, cells * NF,
        tiled ? TILE_EDGE_DOUBLES * sizeof(double) : 0,
        sizeof(double) * 2 * (size_t)CG_MAX_BLOCKS * CG_MAX_FIELDS * 4,
        sizeof(double) * CG_MAX_FIELDS * 4, sizeof(unsigned) * BAR_WORDS, sizeof(int32_t) * 4};
    for (int k = 0; k < WORK_PARTS; ++k) sz[k] = parts[k];
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

void diffusion_work_assign(DiffusionWork& w, void* const (&ptr)[WORK_PARTS]) {
    w.theta = (double*)ptr[0];
    w.Kx = (double*)ptr[1];
    w.Ky = (double*)ptr[2];
    w.x = (double*)ptr[3];
    w.r = (double*)ptr[4];
    w.z = (double*)ptr[5];
    w.p = (double*)ptr[6];
    w.q = (double*)ptr[7];
    w.edge = (double*)ptr[8];
    w.partial = (double*)ptr[9];
    w.totals = (double*)ptr[10];
    w.barrier = (unsigned*)ptr[11];
    w.info = (int32_t*)ptr[12];
}

}  // namespace

int diffusion_work_alloc(DiffusionWork& w, const Mech& m, const Grid& g) {
    const int NF = m.dev.N + 1;
    if (NF - 1 > CG_MAX_FIELDS)
        return fail(MISDC_EUNSUPPORTED, "at most %d diffused fields, got %d", CG_MAX_FIELDS, NF - 1);
    size_t sz[WORK_PARTS];
    diffusion_work_sizes(m, g, sz);
    void* ptr[WORK_PARTS] = {};
    for (int k = 0; k < WORK_PARTS; ++k) {
        if (sz[k] == 0) continue;
        hipError_t e = hipMalloc(&ptr[k], sz[k]);
        if (e != hipSuccess) {
            diffusion_work_assign(w, ptr);
            return fail(MISDC_ENOMEM, "diffusion workspace: %s", hipGetErrorString(e));
        }
    }
    diffusion_work_assign(w, ptr);
    MISDC_HIP(hipMemset(w.Ky, 0, sz[2]));
    MISDC_HIP(hipMemset(w.barrier, 0, sz[11]));
    MISDC_HIP(hipMemset(w.info, 0, sz[12]));
    return diffusion_work_choose(w, m, g);
}

size_t diffusion_work_bytes(const Mech& m, const Grid& g) {
    size_t sz[WORK_PARTS];
    diffusion_work_sizes(m, g, sz);
    size_t total = 0;
    for (int k = 0; k < WORK_PARTS; ++k) total += align256(sz[k]);
    return total;
}

int diffusion_work_carve(DiffusionWork& w, const Mech& m, const Grid& g, void* block, size_t bytes,
                         hipStream_t s) {
    const int NF = m.dev.N + 1;
    if (NF - 1 > CG_MAX_FIELDS)
        return fail(MISDC_EUNSUPPORTED, "at most %d diffused fields, got %d", CG_MAX_FIELDS, NF - 1);
    if (diffusion_work_bytes(m, g) > bytes)
        return fail(MISDC_EINVAL, "diffusion workspace of %zu bytes does not fit in %zu",
                    diffusion_work_bytes(m, g), bytes);
    size_t sz[WORK_PARTS];
    diffusion_work_sizes(m, g, sz);
    void* ptr[WORK_PARTS] = {};
    char* at = (char*)block;
    for (int k = 0; k < WORK_PARTS; ++k) {
        ptr[k] = sz[k] ? at : nullptr;
        at += align256(sz[k]);
    }
    w = DiffusionWork();
    diffusion_work_assign(w, ptr);
    // what must start at zero: the y-face coefficients that a 1-D grid never
    // writes, the barrier counters and the iteration record (kernels, so the
    // calls may be captured into a graph)
    int rc = launch_zero(w.Ky, (int64_t)sz[2], s);
    if (!rc) rc = launch_zero(w.barrier, (int64_t)sz[11], s);
    if (!rc) rc = launch_zero(w.info, (int64_t)sz[12], s);
    if (rc) return rc;
    return diffusion_work_choose(w, m, g);
}

void diffusion_work_free(DiffusionWork& w) {
    double* ptrs[] = {w.theta, w.Kx, w.Ky, w.x, w.r, w.z, w.p, w.q, w.partial, w.totals, w.edge};
    for (double* p : ptrs)
        if (p) (void)hipFree(p);
    if (w.barrier) (void)hipFree(w.barrier);
    if (w.info) (void)hipFree(w.info);
    w = DiffusionWork();
}

int launch_diffusion_solve(const Mech& m, const Grid& g, DiffusionWork& w, double c,
                           const double* dt_flame, double c_factor, const double* T_lag,
                           const double* rhs, double* y, int guess_in_y, double rtol, int maxit,
                           hipStream_t s, hipEvent_t core_begin, hipEvent_t core_end,
                           double* T_out, int32_t* cgstats, double* th_out, bool faces_ready,
                           const LagRhs* fused) {
    const int64_t n = g.cells();
    if (n == 0) return MISDC_OK;
    const GridDev gd = grid_dev(g);
    // the second pass of a split right-hand side: formed by the tiled solve
    // itself where it can (each thread for its cell, in the prologue),
    // otherwise by a launch of its own before the solve
    const bool single2d = !(g.dim == 1 || g.n_flames > 0);
    const bool in_solve = fused && single2d && w.variant == 101 && guess_in_y && g.nx >= 2 &&
                          g.ny >= 2 && !fused->scale && m.dev.N == 9 && T_lag == fused->T_lag;
    if (fused && !in_solve) {
        LagRhs l = *fused;
        l.out = const_cast<double*>(rhs);
        const int rc = launch_lag_rhs(m, g, l, w, s);
        if (rc) return rc;
        faces_ready = true;
    }
    if (!faces_ready && !in_solve) {
        hipLaunchKernelGGL(faces_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, gd, n, T_lag,
                           w.theta, w.Kx, w.Ky, w.barrier);
        MISDC_HIP(hipGetLastError());
    }
    if (core_begin) MISDC_HIP(hipEventRecord(core_begin, s));
    const int NF = m.dev.N + 1;
    if (g.dim == 1 || g.n_flames > 0) {
        const int nsys = (g.n_flames > 0 ? g.n_flames : 1) * NF;
        if (w.cyclic == 1)
            hipLaunchKernelGGL(cyclic_wave_kernel, dim3(nsys), dim3(64), 0, s, gd, m.dev, n, c,
                               dt_flame, c_factor, w.Kx, rhs, y, w.r, w.z, w.p, w.q);
        else
            hipLaunchKernelGGL(cyclic_kernel, dim3(grid_for(nsys, 64)), dim3(64), 0, s, gd, m.dev,
                               n, c, dt_flame, c_factor, w.Kx, rhs, y, w.r, w.z);
        MISDC_HIP(hipGetLastError());
    } else {
        CGArgs a;
        a.n = n;
        a.nx = (int)g.nx;
        a.ny = (int)g.ny;
        a.nf = 0;
        for (int f = 0; f < NF; ++f) {
            if (f == m.dev.bath) continue;
            a.fmap[a.nf] = f;
            a.cf[a.nf] = c * m.kappa0[f];
            ++a.nf;
        }
        a.Kx = w.Kx;
        a.Ky = w.Ky;
        a.b = rhs;
        a.x = y;
        a.r = w.r;
        a.z = w.z;
        a.p = w.p;
        a.q = w.q;
        a.partial = w.partial;
        a.edge = w.edge;
        a.totals = w.totals;
        a.bar = w.barrier;
        a.info = w.info;
        const double rt = rtol > 0 ? rtol : 1e-13;
        a.rtol2 = rt * rt;
        a.maxit = maxit > 0 ? maxit : 500;
        a.guess_in_x = guess_in_y;
        a.ntx = (int)((g.nx + TILE_X - 1) / TILE_X);
        // the tiled kernels close the bath themselves
        a.close = (w.variant >= 101) ? 1 : 0;
        a.N = m.dev.N;
        a.bath = m.dev.bath;
        for (int f = 0; f <= CG_MAX_FIELDS; ++f) a.dmap[f] = -1;
        for (int d = 0; d < a.nf; ++d) a.dmap[a.fmap[d]] = d;
        a.hf = m.dev.hf;
        a.cp = m.dev.cp;
        a.invW = m.dev.invW;
        a.T_out = T_out;
        a.th_out = T_out ? th_out : nullptr;
        a.cgstats = cgstats;
        if (in_solve) {
            a.lag_src = fused->src;
            a.lag_th = fused->th;
            a.lag_Tsrc = fused->T_src;
            a.lag_part = fused->part;
            a.lag_fr = fused->fr;
            a.lag_T = fused->T_lag;
            a.lag_qa = fused->qa;
            a.lag_qd = fused->qd;
            a.lag_qr = fused->qr;
            a.b_w = const_cast<double*>(rhs);
            a.kappa0 = m.dev.kappa0;
            a.dx = g.dx;
            a.dy = g.dy;
            a.ux = g.ux;
            a.uy = g.uy;
        }
        int rc = launch_cg(a, w.variant, w.blocks, s);
        if (rc) return rc;
        if (a.close) {
            if (core_end) MISDC_HIP(hipEventRecord(core_end, s));
            return MISDC_OK;
        }
    }
    if (core_end) MISDC_HIP(hipEventRecord(core_end, s));
    const bool cg2d = !(g.dim == 1 || g.n_flames > 0);
    hipLaunchKernelGGL(closure_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, m.dev, n, rhs, y,
                       T_out, T_out ? th_out : nullptr, w.info, cg2d ? cgstats : nullptr);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_field_diff_max(int nfields, int64_t n, const double* a, const double* b,
                          double* partial, int partial_blocks, double* out, hipStream_t s) {
    if (n == 0) return MISDC_OK;
    // the arrival counter follows the partials (zero between launches)
    unsigned* done = reinterpret_cast<unsigned*>(partial + (size_t)nfields * partial_blocks * 2);
    hipLaunchKernelGGL(diffmax_kernel, dim3(partial_blocks, nfields), dim3(256), 0, s, nfields, n,
                       a, b, partial, out, done);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

}  // namespace misdc
