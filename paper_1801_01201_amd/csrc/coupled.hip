// The implicit step of the comparison scheme IMEXQ (section 3.2.2): at node
// m+1, diffusion (coefficients lagged at the sweep-k state) and reaction
// treated implicitly together,
//     x - c (FD_lag(x) + FR(x)) = rhs,
// on the whole grid at once.  Newton's method; each Newton system
//     (I - c (D + R)) delta = G,   G = x - c (FD_lag(x) + FR(x)) - rhs,
// with D the lagged diffusion operator (the dominant species' row is minus the
// sum of the other species' rows) and R each cell's derivative of FR with
// respect to (Y, h) through T(Y, h), is solved by BiCGStab, preconditioned by
// the inverse of each cell's own block I - c (R_i + D_ii) (formed and solved
// by LU with partial pivoting at each application).  The unknowns are scaled per field by the size of the
// right-hand side (mass fractions by at least 1e-3), so that the enthalpy,
// some ten orders of magnitude larger, does not swamp the Krylov norms.
// Reductions are per-block partial sums added on the host in block order, so
// results do not depend on scheduling.  The loop is driven by the host, which
// reads each scalar of the iteration: a comparison scheme, not a tuned one.
#include <cmath>
#include <vector>

#include "chem_dev.h"
#include "flame_dev.h"
#include "misdc_impl.h"

namespace misdc {

namespace {

constexpr int NS = 9, NF = NS + 1;
constexpr int RED_BLOCKS = 256;

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

__global__ void __launch_bounds__(256) cpl_faces_kernel(GridDev g, int64_t n, const double* T,
                                                        double* th, double* Kx, double* Ky) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) faces_at(g, i, T, th, Kx, Ky);
}

struct Nbr {
    int64_t xm, xp, ym, yp;
    double kxe, kxw, kyn, kys;   // face coefficients / dx^2 (0 in y on a 1-D grid)
};

__device__ __forceinline__ Nbr neighbours(const GridDev& g, int64_t i, const double* Kx,
                                          const double* Ky) {
    Nbr b;
    const Row r = row_of(g, i);
    b.xm = r.base + wrap(r.pos - 1, r.len);
    b.xp = r.base + wrap(r.pos + 1, r.len);
    b.kxe = Kx[i];
    b.kxw = Kx[b.xm];
    b.ym = b.yp = i;
    b.kyn = b.kys = 0.0;
    if (g.dim == 2 && g.n_flames == 0) {
        const int64_t iy = i / g.nx, ix = i - iy * g.nx;
        b.ym = wrap(iy - 1, g.ny) * g.nx + ix;
        b.yp = wrap(iy + 1, g.ny) * g.nx + ix;
        b.kyn = Ky[i];
        b.kys = Ky[b.ym];
    }
    return b;
}

// (D u)_f at cell i for every field f of u (unscaled, field stride n)
__device__ __forceinline__ void diffuse(const MechDev& m, const Nbr& b, int64_t n, int64_t i,
                                        const double* u, const double* su, double (&Du)[NF]) {
    double bath = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const double* p = u + (size_t)f * n;
        const double s = su ? su[f] : 1.0;
        const double c0 = p[i] * s;
        const double lap = b.kxe * (p[b.xp] * s - c0) - b.kxw * (c0 - p[b.xm] * s) +
                           b.kyn * (p[b.yp] * s - c0) - b.kys * (c0 - p[b.ym] * s);
        const double d = m.kappa0[f] * lap;
        Du[f] = (f == m.bath) ? 0.0 : d;
        if (f < NS && f != m.bath) bath += d;
    }
#pragma unroll
    for (int f = 0; f < NS; ++f) Du[f] = (f == m.bath) ? -bath : Du[f];
}

// Per cell: the residual G (scaled by 1/sigma) and the reaction Jacobian with
// respect to (Y, h) (unscaled, N x NF entries, field-major over the cells).
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) cpl_prepare_kernel(GridDev g, MechDev m, int64_t n, double c,
                                                         const double* Kx, const double* Ky,
                                                         const double* x, const double* rhs,
                                                         const double* sigma, double* G,
                                                         double* JR) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double Y[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) Y[k] = x[(size_t)k * n + i];
    const double h = x[(size_t)NS * n + i];
    const double T = temperature_of<NS>(m, Y, h);
    double FR[NS], J[NS][NS + 1];
    reaction_terms<NS, true>(m, Y, T, FR, J);
    double cpm = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) cpm += Y[k] * m.cp[k] * m.invW[k];
    // through T(Y, h): dT/dY_l = -hhat_l / cp, dT/dh = 1 / cp
    double hh[NS];
#pragma unroll
    for (int l = 0; l < NS; ++l) hh[l] = species_h(m, l, T) * m.invW[l] / cpm;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const double dT = J[k][NS];
#pragma unroll
        for (int l = 0; l < NS; ++l) JR[(size_t)(k * NF + l) * n + i] = J[k][l] - dT * hh[l];
        JR[(size_t)(k * NF + NS) * n + i] = dT / cpm;
    }
    // G = x - c (D x + FR) - rhs
    const Nbr b = neighbours(g, i, Kx, Ky);
    double Dx[NF];
    diffuse(m, b, n, i, x, nullptr, Dx);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const double fr = f < NS ? FR[f] : 0.0;
        const double gf = x[(size_t)f * n + i] - c * (Dx[f] + fr) - rhs[(size_t)f * n + i];
        G[(size_t)f * n + i] = gf / sigma[f];
    }
}

// z = (cell block)^-1 r: the cell's own block of the scaled Newton matrix,
// S^-1 (I - c (R_i + D_ii)) S, with D_ii the cell's diagonal diffusion
// entries (the bath species' row holding minus the other species'), formed
// and solved at each application.  The enthalpy row of the block is its
// diagonal entry alone (no reaction source in h), so z_h comes first and the
// species block is solved by LU with partial pivoting with z_h's column
// moved to the right-hand side.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1)))
cpl_precond_kernel(GridDev g, MechDev m, int64_t n, double c, const double* Kx, const double* Ky,
                   const double* JR, const double* sigma, const double* r, double* z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Nbr b = neighbours(g, i, Kx, Ky);
    const double ksum = b.kxe + b.kxw + b.kyn + b.kys;
    // scaled: z_h = r_h / (1 + c kappa0_h ksum) (the scales of the row and
    // the column cancel)
    const double zh = r[(size_t)NS * n + i] / (1.0 + c * m.kappa0[NS] * ksum);
    const double sh = sigma[NS];
    double sg[NS];
#pragma unroll
    for (int f = 0; f < NS; ++f) sg[f] = sigma[f];
    double A[NS][NS + 1];
#pragma unroll
    for (int f = 0; f < NS; ++f) {
#pragma unroll
        for (int l = 0; l < NS; ++l) A[f][l] = -c * JR[(size_t)(f * NF + l) * n + i];
        // right-hand side in unscaled rows: sigma_f r_f - (-c R_{f,h}) sigma_h z_h
        A[f][NS] = sg[f] * r[(size_t)f * n + i] + c * JR[(size_t)(f * NF + NS) * n + i] * sh * zh;
    }
    const int bath = m.bath;
#pragma unroll
    for (int f = 0; f < NS; ++f) {
        const double d = (f == bath) ? 0.0 : -m.kappa0[f] * ksum;   // the cell's (D)_{ff}
        A[f][f] -= c * d;
#pragma unroll
        for (int q = 0; q < NS; ++q) A[q][f] += (q == bath) ? c * d : 0.0;
    }
#pragma unroll
    for (int f = 0; f < NS; ++f) A[f][f] += 1.0;
    // the unscaled species block solves for S z
    lu_solve<NS>(A);
#pragma unroll
    for (int f = 0; f < NS; ++f) z[(size_t)f * n + i] = A[f][NS] / sg[f];
    z[(size_t)NS * n + i] = zh;
}

// out = S^-1 (I - c (D + R)) S v, per cell
__global__ void __launch_bounds__(128) cpl_matvec_kernel(GridDev g, MechDev m, int64_t n, double c,
                                                         const double* Kx, const double* Ky,
                                                         const double* JR, const double* sigma,
                                                         const double* v, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Nbr b = neighbours(g, i, Kx, Ky);
    double Du[NF];
    diffuse(m, b, n, i, v, sigma, Du);
    double u[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) u[f] = v[(size_t)f * n + i] * sigma[f];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        double ru = 0.0;
        if (f < NS)
#pragma unroll
            for (int l = 0; l < NF; ++l) ru += JR[(size_t)(f * NF + l) * n + i] * u[l];
        out[(size_t)f * n + i] = (u[f] - c * (Du[f] + ru)) / sigma[f];
    }
}

// out = a x + b y + e z over all fields (any of y, z may be null)
__global__ void __launch_bounds__(256) cpl_lin3_kernel(int64_t tot, double a, const double* x,
                                                       double b, const double* y, double e,
                                                       const double* z, double* out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < tot;
         k += (int64_t)gridDim.x * blockDim.x) {
        double v = x ? a * x[k] : 0.0;
        if (y) v += b * y[k];
        if (z) v += e * z[k];
        out[k] = v;
    }
}

// per-block partial sums of a . b over all fields (fixed order within a block)
__global__ void __launch_bounds__(256) cpl_dot_kernel(int64_t tot, const double* a, const double* b,
                                                      double* partial) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < tot;
         k += (int64_t)gridDim.x * blockDim.x)
        acc += a[k] * b[k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// per field and block: max |a| (and with b, max |b| too) into partial[(f, block, 0/1)]
__global__ void __launch_bounds__(256) cpl_fieldmax_kernel(int64_t n, const double* a, const double* b,
                                                           double* partial) {
    __shared__ double sa[256], sb[256];
    const int f = blockIdx.y;
    double ma = 0.0, mb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        ma = fmax(ma, fabs(a[(size_t)f * n + i]));
        if (b) mb = fmax(mb, fabs(b[(size_t)f * n + i]));
    }
    sa[threadIdx.x] = ma;
    sb[threadIdx.x] = mb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] = fmax(sa[threadIdx.x], sa[threadIdx.x + w]);
            sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[((size_t)f * gridDim.x + blockIdx.x) * 2] = sa[0];
        partial[((size_t)f * gridDim.x + blockIdx.x) * 2 + 1] = sb[0];
    }
}

// x_f -= sigma_f d_f
__global__ void __launch_bounds__(256) cpl_update_kernel(int64_t n, const double* sigma, const double* d,
                                                         double* x) {
    const int f = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[(size_t)f * n + i] -= sigma[f] * d[(size_t)f * n + i];
}

GridDev grid_dev_of(const Grid& g) {
    GridDev d;
    d.dim = g.dim;
    d.nx = g.nx;
    d.ny = g.ny;
    d.dx = g.dx;
    d.dy = g.dy;
    d.ux = g.ux;
    d.uy = g.uy;
    d.n_flames = 0;
    d.off = nullptr;
    d.fdx = nullptr;
    d.fu = nullptr;
    return d;
}

}  // namespace

int coupled_work_alloc(CoupledWork& w, const Mech& m, const Grid& g) {
    if (m.dev.N != NS) return fail(MISDC_EUNSUPPORTED, "IMEXQ's coupled solve is built for %d species", NS);
    if (g.n_flames > 0) return fail(MISDC_EUNSUPPORTED, "IMEXQ's coupled solve takes single grids");
    const int64_t n = g.cells();
    w.n = n;
    auto grab = [&](double** p, size_t count) -> int {
        hipError_t e = hipMalloc((void**)p, sizeof(double) * count + 256);
        if (e != hipSuccess) return fail(MISDC_ENOMEM, "IMEXQ work space: %s", hipGetErrorString(e));
        return MISDC_OK;
    };
    int rc;
    double** vecs[] = {&w.G, &w.d, &w.r, &w.rh, &w.p, &w.v, &w.y, &w.s, &w.t, &w.zz};
    for (double** p : vecs)
        if ((rc = grab(p, (size_t)NF * n))) return rc;
    if ((rc = grab(&w.JR, (size_t)NS * NF * n))) return rc;
    if ((rc = grab(&w.th, (size_t)n))) return rc;
    if ((rc = grab(&w.Kx, (size_t)n))) return rc;
    if ((rc = grab(&w.Ky, (size_t)n))) return rc;
    if ((rc = grab(&w.sigma, NF))) return rc;
    if ((rc = grab(&w.partial, (size_t)RED_BLOCKS * NF * 2))) return rc;
    MISDC_HIP(hipMemset(w.Ky, 0, sizeof(double) * (size_t)n));
    return MISDC_OK;
}

void coupled_work_free(CoupledWork& w) {
    double* ptrs[] = {w.G, w.d, w.r, w.rh, w.p, w.v, w.y, w.s, w.t, w.zz, w.JR,
                      w.th, w.Kx, w.Ky, w.sigma, w.partial};
    for (double* p : ptrs)
        if (p) (void)hipFree(p);
    w = CoupledWork();
}

int coupled_solve(const Mech& m, const Grid& g, CoupledWork& w, double c, const double* T_lag,
                  const double* rhs, double* x, double newton_tol, int newton_maxit,
                  double lin_rtol, int lin_maxit, CoupledStats& st, hipStream_t s) {
    const int64_t n = g.cells();
    const int64_t tot = (int64_t)NF * n;
    const GridDev gd = grid_dev_of(g);
    const unsigned cb = blocks_for(n, 64), mb = blocks_for(n, 128);
    unsigned vb = blocks_for(tot, 256);
    if (vb > RED_BLOCKS) vb = RED_BLOCKS;
    unsigned fb = blocks_for(n, 256);
    if (fb > RED_BLOCKS) fb = RED_BLOCKS;
    std::vector<double> part((size_t)RED_BLOCKS * NF * 2);
    auto dot = [&](const double* a, const double* b, double& out) -> int {
        hipLaunchKernelGGL(cpl_dot_kernel, dim3(vb), dim3(256), 0, s, tot, a, b, w.partial);
        MISDC_HIP(hipGetLastError());
        MISDC_HIP(hipMemcpyAsync(part.data(), w.partial, sizeof(double) * vb, hipMemcpyDeviceToHost, s));
        MISDC_HIP(hipStreamSynchronize(s));
        double acc = 0.0;
        for (unsigned k = 0; k < vb; ++k) acc += part[k];
        out = acc;
        return MISDC_OK;
    };
    auto fieldmax = [&](const double* a, const double* b, double (&ma)[NF], double (&mbv)[NF]) -> int {
        hipLaunchKernelGGL(cpl_fieldmax_kernel, dim3(fb, NF), dim3(256), 0, s, n, a, b, w.partial);
        MISDC_HIP(hipGetLastError());
        MISDC_HIP(hipMemcpyAsync(part.data(), w.partial, sizeof(double) * fb * NF * 2,
                                 hipMemcpyDeviceToHost, s));
        MISDC_HIP(hipStreamSynchronize(s));
        for (int f = 0; f < NF; ++f) {
            ma[f] = mbv[f] = 0.0;
            for (unsigned k = 0; k < fb; ++k) {
                ma[f] = fmax(ma[f], part[((size_t)f * fb + k) * 2]);
                mbv[f] = fmax(mbv[f], part[((size_t)f * fb + k) * 2 + 1]);
            }
        }
        return MISDC_OK;
    };
    auto lin3 = [&](double a, const double* xv, double b, const double* yv, double e,
                    const double* zv, double* out) -> int {
        hipLaunchKernelGGL(cpl_lin3_kernel, dim3(vb), dim3(256), 0, s, tot, a, xv, b, yv, e, zv, out);
        MISDC_HIP(hipGetLastError());
        return MISDC_OK;
    };
    auto matvec = [&](const double* v, double* out) -> int {
        hipLaunchKernelGGL(cpl_matvec_kernel, dim3(mb), dim3(128), 0, s, gd, m.dev, n, c, w.Kx, w.Ky,
                           w.JR, w.sigma, v, out);
        MISDC_HIP(hipGetLastError());
        return MISDC_OK;
    };
    auto precond = [&](const double* r, double* z) -> int {
        hipLaunchKernelGGL(cpl_precond_kernel, dim3(cb), dim3(64), 0, s, gd, m.dev, n, c, w.Kx,
                           w.Ky, w.JR, w.sigma, r, z);
        MISDC_HIP(hipGetLastError());
        return MISDC_OK;
    };
    int rc;
    // lagged face coefficients, and the field scales from the right-hand side
    hipLaunchKernelGGL(cpl_faces_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, gd, n, T_lag,
                       w.th, w.Kx, w.Ky);
    MISDC_HIP(hipGetLastError());
    double rmax[NF], unused[NF], sig[NF];
    if ((rc = fieldmax(rhs, nullptr, rmax, unused))) return rc;
    for (int f = 0; f < NF; ++f) {
        sig[f] = rmax[f];
        if (f < NS && sig[f] < 1e-3) sig[f] = 1e-3;
        if (!(sig[f] > 0) || !std::isfinite(sig[f])) sig[f] = 1.0;
    }
    MISDC_HIP(hipMemcpyAsync(w.sigma, sig, sizeof(sig), hipMemcpyHostToDevice, s));
    bool converged = false;
    for (int it = 0; it < newton_maxit && !converged; ++it) {
        hipLaunchKernelGGL(cpl_prepare_kernel, dim3(cb), dim3(64), 0, s, gd, m.dev, n, c, w.Kx, w.Ky,
                           x, rhs, w.sigma, w.G, w.JR);
        MISDC_HIP(hipGetLastError());
        ++st.newton_iters;
        // BiCGStab (right side G, zero start), right-preconditioned by the blocks
        double gg = 0.0;
        if ((rc = dot(w.G, w.G, gg))) return rc;
        const double stop = lin_rtol * lin_rtol * gg;
        if ((rc = lin3(0.0, nullptr, 0.0, nullptr, 0.0, nullptr, w.d))) return rc;
        if ((rc = lin3(1.0, w.G, 0.0, nullptr, 0.0, nullptr, w.r))) return rc;
        if ((rc = lin3(1.0, w.G, 0.0, nullptr, 0.0, nullptr, w.rh))) return rc;
        if ((rc = lin3(0.0, nullptr, 0.0, nullptr, 0.0, nullptr, w.p))) return rc;
        if ((rc = lin3(0.0, nullptr, 0.0, nullptr, 0.0, nullptr, w.v))) return rc;
        double rho = 1.0, alpha = 1.0, omega = 1.0, rr = gg;
        int k = 0;
        bool lin_ok = gg == 0.0;
        for (; k < lin_maxit && !lin_ok; ++k) {
            double rho1 = 0.0;
            if ((rc = dot(w.rh, w.r, rho1))) return rc;
            if (rho1 == 0.0 || omega == 0.0) break;
            const double beta = (rho1 / rho) * (alpha / omega);
            rho = rho1;
            // p = r + beta (p - omega v)
            if ((rc = lin3(1.0, w.r, beta, w.p, -beta * omega, w.v, w.p))) return rc;
            if ((rc = precond(w.p, w.y))) return rc;
            if ((rc = matvec(w.y, w.v))) return rc;
            double rv = 0.0;
            if ((rc = dot(w.rh, w.v, rv))) return rc;
            if (rv == 0.0) break;
            alpha = rho / rv;
            // s = r - alpha v; d += alpha y
            if ((rc = lin3(1.0, w.r, -alpha, w.v, 0.0, nullptr, w.s))) return rc;
            if ((rc = lin3(1.0, w.d, alpha, w.y, 0.0, nullptr, w.d))) return rc;
            double ss = 0.0;
            if ((rc = dot(w.s, w.s, ss))) return rc;
            if (ss <= stop) {
                lin_ok = true;
                ++k;
                break;
            }
            if ((rc = precond(w.s, w.zz))) return rc;
            if ((rc = matvec(w.zz, w.t))) return rc;
            double ts = 0.0, tt = 0.0;
            if ((rc = dot(w.t, w.s, ts))) return rc;
            if ((rc = dot(w.t, w.t, tt))) return rc;
            if (tt == 0.0) break;
            omega = ts / tt;
            // d += omega z; r = s - omega t
            if ((rc = lin3(1.0, w.d, omega, w.zz, 0.0, nullptr, w.d))) return rc;
            if ((rc = lin3(1.0, w.s, -omega, w.t, 0.0, nullptr, w.r))) return rc;
            if ((rc = dot(w.r, w.r, rr))) return rc;
            if (rr <= stop) {
                lin_ok = true;
                ++k;
                break;
            }
        }
        st.krylov_iters += k;
        if (k > st.krylov_max) st.krylov_max = k;
        if (!lin_ok) ++st.krylov_failed;
        // x -= S d; converged when every mass fraction's update is at most
        // newton_tol (O(1) quantities, tested absolutely: a trace species'
        // update stalls at the rounding level of the species coupled into
        // it) and the enthalpy's at most newton_tol times its largest
        // magnitude
        hipLaunchKernelGGL(cpl_update_kernel, dim3(fb, NF), dim3(256), 0, s, n, w.sigma, w.d, x);
        MISDC_HIP(hipGetLastError());
        double dmax[NF], xmax[NF];
        if ((rc = fieldmax(w.d, x, dmax, xmax))) return rc;
        converged = true;
        for (int f = 0; f < NF; ++f) {
            const double du = dmax[f] * sig[f];
            if (!std::isfinite(du)) return fail(MISDC_ENOTCONV, "IMEXQ: non-finite Newton update");
            const double scale = f < NS ? 1.0 : xmax[f];
            if (du > newton_tol * scale) converged = false;
        }
    }
    ++st.solves;
    if (!converged) ++st.newton_failed;
    return MISDC_OK;
}

}  // namespace misdc
