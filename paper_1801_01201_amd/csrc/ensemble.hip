// One stage of a concurrent sweep over an ensemble of 1-D flames as a single
// persistent launch (steps S3-S6 of section 3 for the nodes of one stage:
// the diffusion solve at node m+1 and the reaction solve at node m).
//
// Workgroups of one wavefront pull work items from an atomic counter until
// the queue is empty:
//   - items [0, nD): one periodic tridiagonal system (flame, field) of the
//     diffusion step, longest flames first (the partition solve of
//     cyclic_wave_system);
//   - items [nD, nD + nR): 64 consecutive cells of the flattened ensemble,
//     one thread per cell-node Newton solve (newton_cell).
// Nothing waits on anything.  The workgroup that completes a flame's last
// diffusion system does that flame's closure (dominant species, T, theta)
// and, at the first nested iteration, its lag-initialisation transport; the
// workgroup that completes a flame's last Newton cells evaluates the
// explicit operators at that flame's new state.  Completion is counted per
// flame with agent-scope atomics after an agent-scope fence, and the
// finishing workgroup fences again before it reads the other workgroups'
// results (the release/acquire pattern of the HIP memory model).
#include "chem_dev.h"
#include "flame_dev.h"
#include "misdc_impl.h"
#include "newton_hist.h"

namespace misdc {

namespace {

struct StageDev {
    GridDev g;
    MechDev m;
    int64_t n;
    // diffusion part
    int nD;
    const int* d_items;          // (field << 16) | flame, longest flames first
    int d_per_flame;             // systems per flame (every field but the bath)
    double c, cfac;              // implicit factor (c, or dtf[flame] * cfac) * kappa0
    const double* dtf;
    const double* Kx;
    const double* rhs;
    double* y;
    double *sc, *su, *sv, *sw;
    double* T_out;
    double* th_out;
    double* lagFA;               // non-null: lag transport at y after the closure
    double* lagFD;
    // reaction part
    int nR;
    NewtonArgs na;
    const double* h_src;         // enthalpy of the diffusion output ...
    double* h_dst;               // ... copied into the reaction output
    const double* rstate;        // state, T, theta work and outputs of the transport
    const double* rT;
    double* rth;
    double* rFA;
    double* rFD;
    // counters: [0] next item, then d_done[flames], then r_done[flames]
    unsigned* counters;
};

__device__ __forceinline__ int flame_of(const GridDev& g, int64_t i) {
    int lo = 0, hi = g.n_flames;
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (g.off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

template <bool INERT_LAST>
__global__ void __launch_bounds__(64) stage_kernel(StageDev a) {
    __shared__ unsigned s_item;
    __shared__ int s_fin[4];
    const int lane = threadIdx.x;
    const GridDev& g = a.g;
    const unsigned total = (unsigned)(a.nD + a.nR);
    unsigned* d_done = a.counters + 1;
    unsigned* r_done = a.counters + 1 + g.n_flames;
    for (;;) {
        if (lane == 0) s_item = atomicAdd(&a.counters[0], 1u);
        __syncthreads();
        const unsigned item = s_item;
        __syncthreads();
        if (item >= total) break;                    // uniform over the workgroup
        if ((int)item < a.nD) {
            const int code = a.d_items[item];
            const int f = code >> 16, fl = code & 0xffff;
            cyclic_wave_system(g, a.m, a.n, a.c, a.dtf, a.cfac, a.Kx, a.rhs, a.y, a.sc, a.su,
                               a.sv, a.sw, f, fl);
            __threadfence();                         // release this system's solution
            __syncthreads();
            if (lane == 0) {
                const unsigned before = atomicAdd(&d_done[fl], 1u);
                s_fin[0] = (before + 1u == (unsigned)a.d_per_flame) ? 1 : 0;
            }
            __syncthreads();
            if (s_fin[0]) {
                __threadfence();                     // acquire the other systems
                const int64_t b = g.off[fl], e = g.off[fl + 1];
                for (int64_t i = b + lane; i < e; i += 64)
                    closure_cell(a.m, a.n, a.rhs, a.y, a.T_out, a.th_out, i);
                if (a.lagFA) {
                    __syncthreads();                 // every cell's theta of the flame
                    for (int64_t i = b + lane; i < e; i += 64)
                        transport_cell<false>(g, a.m, a.n, a.y, a.T_out, a.th_out, a.lagFA,
                                              a.lagFD, i);
                }
            }
        } else {
            const int64_t c0 = (int64_t)(item - (unsigned)a.nD) * 64;
            const int64_t i = c0 + lane;
            if (i < a.n) a.h_dst[i] = a.h_src[i];
            const int code = newton_cell<9, INERT_LAST>(a.m, a.na, i);
            newton_wave_stats(a.na, item, i < a.n, code);
            __threadfence();                         // release this chunk's states
            __syncthreads();
            if (lane == 0) {
                // cells of this chunk per flame; a flame whose last cells
                // these were is finished here (at most 4 flames per chunk:
                // every flame has at least 16 cells)
                const int64_t c1 = c0 + 64 < a.n ? c0 + 64 : a.n;
                int nfin = 0;
                for (int fl = flame_of(g, c0); fl < g.n_flames && g.off[fl] < c1; ++fl) {
                    const int64_t lo = g.off[fl] > c0 ? g.off[fl] : c0;
                    const int64_t hi = g.off[fl + 1] < c1 ? g.off[fl + 1] : c1;
                    const unsigned cnt = (unsigned)(hi - lo);
                    const unsigned before = atomicAdd(&r_done[fl], cnt);
                    if (before + cnt == (unsigned)(g.off[fl + 1] - g.off[fl]) && nfin < 4)
                        s_fin[nfin++] = fl;
                }
                for (int k = nfin; k < 4; ++k) s_fin[k] = -1;
            }
            __syncthreads();
            for (int k = 0; k < 4; ++k) {
                const int fl = s_fin[k];
                if (fl < 0) break;
                __threadfence();                     // acquire the flame's states
                for (int64_t j = g.off[fl] + lane; j < g.off[fl + 1]; j += 64)
                    transport_cell<true>(g, a.m, a.n, a.rstate, a.rT, a.rth, a.rFA, a.rFD, j);
            }
        }
        __syncthreads();
    }
}

}  // namespace

int launch_ensemble_stage(const Mech& m, const Grid& g, const EnsembleStage& st, hipStream_t s) {
    if (g.n_flames <= 0) return fail(MISDC_EINVAL, "a fused stage needs an ensemble grid");
    if (m.dev.N != 9) return fail(MISDC_EUNSUPPORTED, "the fused stage is built for 9 species");
    for (int64_t L : g.len)
        if (L < 16) return fail(MISDC_EUNSUPPORTED, "the fused stage needs flames of >= 16 cells");
    if (g.n_flames > 0xffff) return fail(MISDC_EUNSUPPORTED, "too many flames for a fused stage");
    StageDev a;
    a.g.dim = 1;
    a.g.nx = g.cells();
    a.g.ny = 1;
    a.g.dx = g.dx;
    a.g.dy = 0.0;
    a.g.ux = g.ux;
    a.g.uy = 0.0;
    a.g.n_flames = g.n_flames;
    a.g.off = g.d_off;
    a.g.fdx = g.d_dx;
    a.g.fu = g.d_u;
    a.m = m.dev;
    a.n = g.cells();
    a.nD = st.has_d ? st.nD : 0;
    a.d_items = st.d_items;
    a.d_per_flame = m.dev.N;
    a.c = st.c;
    a.cfac = st.cfac;
    a.dtf = st.dtf;
    a.Kx = st.Kx;
    a.rhs = st.rhs;
    a.y = st.y;
    a.sc = st.sc;
    a.su = st.su;
    a.sv = st.sv;
    a.sw = st.sw;
    a.T_out = st.T_out;
    a.th_out = st.th_out;
    a.lagFA = st.lagFA;
    a.lagFD = st.lagFD;
    a.nR = st.has_r ? (int)((a.n + 63) / 64) : 0;
    a.na = st.na;
    a.h_src = st.h_src;
    a.h_dst = st.h_dst;
    a.rstate = st.rstate;
    a.rT = st.rT;
    a.rth = st.rth;
    a.rFA = st.rFA;
    a.rFD = st.rFD;
    a.counters = st.counters;
    if (a.nD + a.nR == 0) return MISDC_OK;
    if (st.has_d && !(st.Kx && st.rhs && st.y && st.T_out && st.d_items))
        return fail(MISDC_EINVAL, "fused stage: diffusion arrays missing");
    if (st.has_r && !(a.na.bY && a.na.h && a.na.Y && a.na.T && a.na.FR && a.na.iters &&
                      st.h_src && st.h_dst && st.rth && st.rFA && st.rFD))
        return fail(MISDC_EINVAL, "fused stage: reaction arrays missing");
    int rc = launch_zero(st.counters, sizeof(unsigned) * (1 + 2 * (size_t)g.n_flames), s);
    if (rc) return rc;
    int cus = 0;
    if ((rc = device_cus(cus))) return rc;
    int occ = 0;
    if (m.dev.bath == m.dev.N - 1)
        MISDC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, stage_kernel<true>, 64, 0));
    else
        MISDC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, stage_kernel<false>, 64, 0));
    if (occ < 1) occ = 1;
    // persistent: as many workgroups as stay resident, at most one per item
    int64_t grid = (int64_t)occ * cus * st.waves_per_slot;
    if (grid > a.nD + a.nR) grid = a.nD + a.nR;
    if (m.dev.bath == m.dev.N - 1)
        hipLaunchKernelGGL(stage_kernel<true>, dim3((unsigned)grid), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL(stage_kernel<false>, dim3((unsigned)grid), dim3(64), 0, s, a);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

}  // namespace misdc
