// Integrator and C ABI.
//
// One time step (section 3.3, initialisation I1-I4 and sweeps S1-S7) is
// issued as a DAG of stream-ordered kernels on two HIP streams: the
// diffusion task (right-hand side, implicit diffusion, explicit operators at
// the advection-diffusion state) and the reaction task (right-hand side,
// per-cell Newton solve, explicit operators at the new state).  For the
// concurrent scheme the diffusion step at node m+1 and the reaction step at
// node m of the same nested iteration are independent (the decoupling of
// section 3.2.1), so the host enqueues them stage by stage on the two streams
// with events only where the update equations create a dependency:
//   D_p^(l+1) needs R_{p-2}^(l+1) (values of iteration l+1 at nodes <= m-1)
//             and, for l >= 1, R_p^(l) (lagged reaction term and lagged
//             diffusion coefficients at node m+1; R_{p-1}^(l) precedes it on
//             the reaction stream);
//   R_p^(l+1) needs D_p^(l+1) (the advection-diffusion state);
//   the next sweep's quadrature needs every reaction task of this sweep.
// Every task writes buffers of its own (one buffer set per nested
// iteration), so there is no write-after-read hazard and the result is
// bitwise independent of the interleaving (option ``serialize`` runs the same
// DAG on one stream).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "misdc_impl.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace misdc {
static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}
}  // namespace misdc

using namespace misdc;

namespace {

struct NodeBuf {
    double* phi = nullptr;   // N+1 fields
    double* T = nullptr;     // 1 field
    double* FA = nullptr;    // N+1 fields
    double* FD = nullptr;    // N+1 fields
    double* FR = nullptr;    // N fields
};

}  // namespace

struct misdc_integ_s {
    Mech* mech = nullptr;
    Grid* grid = nullptr;
    misdc_opts opt;
    Tables tab;
    int M = 0, N = 0, NF = 0, nu = 1, levels = 2;
    int64_t n = 0;
    hipStream_t sD = nullptr, sR = nullptr;       // sR is sR2 (or sRm), or sD when serialised
    hipStream_t sR2 = nullptr;                    // reaction stream (own, or the caller's)
    hipStream_t sRm = nullptr;                    // reaction stream on part of the CUs
    hipStream_t sD_own = nullptr, sR2_own = nullptr;   // the streams the library created
    bool caller_R = false;                        // sR2 is a stream of the caller's
    int cu_split = 0, sRm_split = 0;              // quarters of the CUs given to sRm
    int stagger = 0;                              // Newton waits for the next CG's start
    std::vector<std::vector<NodeBuf>> lev;        // [levels][M+1]
    std::vector<double*> phiAD, TAD, hatA, hatD;  // [M+1]
    std::vector<double*> C, CR;                   // [M+1] sweep constants (diffusion, reaction)
    double* rD = nullptr;                         // diffusion right-hand side (N+1 fields)
    // split right-hand sides (split_rhs): every term but the lagged operators,
    // one buffer per node parity, and the event that releases each
    double* rP[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> evP;                  // [M+1]
    std::vector<LagRhs> lagw;                     // [M+1] the second pass's weights
    // split sweep constants (split_constants): the next sweep's constants
    // and D_1's right-hand side without the node-M terms, formed on the
    // reaction stream during the last solve of a sweep; the node-M terms of
    // C^1..C^M after R_M (cfin), those of D_1 in D_1's own pass (d1w) after
    // R_M's Newton solve (ev_newtonM)
    bool consts_ready = false, d1_split = false, const_on_r = false, prep_newton = false;
    LinComb cfin;
    LagRhs d1w;
    hipEvent_t ev_newtonM = nullptr;
    double* thM = nullptr;                        // theta of R_M's result (from its solve)
    // R_M's transport operators, the node-M terms of C^1..C^M and the sweep
    // increment, deferred until D_1's pass of the next sweep is issued (so
    // that they do not run beside it); ev_d1 follows that pass
    struct Deferred {
        bool pending = false, cfin = false, inc = false;
        NodeBuf out;
        double* th = nullptr;
        hipStream_t s = nullptr;
        const double* inc_new = nullptr;
        const double* inc_old = nullptr;
        double* inc_out = nullptr;
    } dfr;
    hipEvent_t ev_d1 = nullptr;
    bool skip_final_ops = false;                  // the step's last R_M skips its transport
    hipEvent_t ev_const = nullptr;                // the sweep constants are formed
    // step start: F_R at the state, formed on the reaction stream beside
    // F_A, F_D
    hipEvent_t ev_source = nullptr;
    double* bR = nullptr;                         // reaction right-hand side (N fields)
    double* thD = nullptr;                        // theta work (diffusion stream)
    double* thR = nullptr;                        // theta work (reaction stream)
    int32_t* iters = nullptr;                     // Newton iterations (cells)
    unsigned long long* nstats = nullptr;         // Newton statistics (8)
    unsigned long long* nbuckets = nullptr;       // per-thread Newton kernel's counter sets
    unsigned long long* nhist = nullptr;          // Newton outcome histograms [sweep][set][bin]
    int32_t* lu_info = nullptr;                   // FP32 LU refinement record (cells)
    int32_t* cgstats = nullptr;                   // CG: [0] sum, [1] max, [2] failed, [3] solves, [4] timeouts
    double* inc = nullptr;                        // sweep increments: 64 x NF x 2
    double* inc_partial = nullptr;
    int inc_blocks = 64;
    double* pinc = nullptr;                       // per-pass changes at node M: 16 x NF x 2
    double* pinc_host = nullptr;                  // pinned host copy of pinc
    int passes[64] = {};                          // nested iterations done per sweep
    DiffusionWork dw;
    std::vector<void*> allocs;
    std::vector<hipEvent_t> evD, evR;             // [(levels) x (M+1)]
    std::vector<hipEvent_t> evC;                  // diffusion task's solve about to start
    hipEvent_t ev_in = nullptr, ev_outD = nullptr, ev_outR = nullptr;
    int last_sweeps = 0;
    int sweep_index = 0;                          // sweep being issued within the step
    // a step opened by misdc_step_begin: its state, the dt its sweeps take and
    // the sweeps done so far
    bool open = false;
    double* open_state = nullptr;
    double open_dt = 0.0;
    int open_sweeps = 0;
    bool d1_ready = false;                        // the sweep constants' pass also formed D_1's
                                                  // right-hand side, guess and face coefficients
    double dt = 0.0;
    // kernel timing (opts.profile): event pairs recorded around launches
    struct Timed { hipEvent_t a, b; int kind; };
    std::vector<Timed> timed;                     // pending pairs (not yet summed)
    std::vector<hipEvent_t> ev_pool;
    double t_ms[2] = {0.0, 0.0};                  // [0] diffusion solve, [1] Newton
    int64_t t_cnt[2] = {0, 0};
    // per-flame step sizes of an ensemble: dtf (flames, caller's array) and
    // its per-cell expansion dtc; both null for a scalar step
    const double* dtf = nullptr;
    const double* dtc = nullptr;
    double* dt_cell = nullptr;
    double tuned_ms = 0.0;                        // step time measured by the autotuner
    // learned Newton guess (optional) and recording of reaction problems
    MlpImpl* mlp = nullptr;
    int guess_sweeps = 0;                         // leading sweeps that use it (0: all)
    int32_t* choice = nullptr;                    // cells: learned guess taken
    double* cbuf = nullptr;                       // cells: implicit factor c of the task
    double* rec_buf = nullptr;                    // caller's buffer of recorded problems
    int64_t rec_cap = 0, rec_count = 0;
    // graph of one whole step, replayed while (state, dt, dev_dt) are unchanged
    bool capturing = false;
    hipGraphExec_t gexec = nullptr;
    const double* g_state = nullptr;
    double g_dt = 0.0;
    const double* g_dtf = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    // pipelined passes (opts.pipeline): the diffusion tasks of pass l run on
    // diffusion lane l % 2 (CU-masked streams on the two halves of every
    // XCD's CUs, so two persistent diffusion solves never compete for CUs),
    // the reaction tasks of pass l on reaction lane l; each lane has its own
    // work buffers
    struct DLane {
        hipStream_t s = nullptr;
        double* rD = nullptr;
        double* th = nullptr;
        DiffusionWork* dw = nullptr;
        int32_t* cgstats = nullptr;
        hipEvent_t end = nullptr;       // the lane's last work of a sweep
    };
    struct RLane {
        hipStream_t s = nullptr;
        double* bR = nullptr;
        double* th = nullptr;
        int32_t* iters = nullptr;
        int32_t* lu_info = nullptr;
        hipEvent_t end = nullptr;
    };
    bool pipe = false;
    hipStream_t s_last = nullptr;              // stream of the last sweep's last reaction task
    // ensembles: each stage of a concurrent pass as one persistent launch
    // (misdc_tune.fused) over the diffusion systems (field << 16 | flame, the
    // longest flames first) and the cells' reaction problems
    bool fused = false;
    // MISDC_SCHEME_IMEXQ: the coupled solve's work space and the last step's
    // counters
    CoupledWork cw;
    CoupledStats cst;
    int* d_items = nullptr;
    int nD_items = 0;
    unsigned* stage_counters = nullptr;
    DLane pd_lane[2];
    std::vector<RLane> pr_lane;
    DiffusionWork pdw[2];
    std::vector<hipStream_t> lane_streams;     // created by the library for the lanes
    DLane dlane(int l) {
        if (pipe) return pd_lane[l % 2];
        DLane d;
        d.s = sD;
        d.rD = rD;
        d.th = thD;
        d.dw = &dw;
        d.cgstats = cgstats;
        return d;
    }
    RLane rlane(int l) {
        if (pipe) return pr_lane[(size_t)l];
        RLane r;
        r.s = sR;
        r.bR = bR;
        r.th = thR;
        r.iters = iters;
        r.lu_info = lu_info;
        return r;
    }

    hipEvent_t& D_ev(int l, int p) { return evD[(size_t)l * (M + 1) + p]; }
    hipEvent_t& R_ev(int l, int p) { return evR[(size_t)l * (M + 1) + p]; }
    hipEvent_t& C_ev(int l, int p) { return evC[(size_t)l * (M + 1) + p]; }
};

namespace {

bool valid_ptr(const void* p) { return p != nullptr; }

int check_mech_desc(const misdc_mech_desc* d) {
    if (!d) return fail(MISDC_EINVAL, "mechanism descriptor is NULL");
    if (d->n_species < 2 || d->n_species > 256)
        return fail(MISDC_EINVAL, "n_species must be in [2, 256], got %d", d->n_species);
    if (d->n_reactions < 0 || d->n_reactions > 100000)
        return fail(MISDC_EINVAL, "n_reactions out of range: %d", d->n_reactions);
    if (d->bath < 0 || d->bath >= d->n_species)
        return fail(MISDC_EINVAL, "bath index %d outside [0, %d)", d->bath, d->n_species);
    const void* arrs[] = {d->W, d->A, d->beta, d->Ea, d->cp, d->hf, d->s0, d->D0};
    for (const void* a : arrs)
        if (!valid_ptr(a)) return fail(MISDC_EINVAL, "mechanism array is NULL");
    if (d->n_reactions > 0 && (!d->react || !d->prod))
        return fail(MISDC_EINVAL, "reaction slot arrays are NULL");
    for (int k = 0; k < d->n_species; ++k) {
        if (!(d->W[k] > 0) || !std::isfinite(d->W[k]))
            return fail(MISDC_EINVAL, "W[%d] must be positive and finite", k);
        if (!(d->cp[k] > 0) || !std::isfinite(d->cp[k]))
            return fail(MISDC_EINVAL, "cp[%d] must be positive and finite", k);
        if (!(d->D0[k] >= 0) || !std::isfinite(d->D0[k]))
            return fail(MISDC_EINVAL, "D0[%d] must be non-negative and finite", k);
        if (!std::isfinite(d->hf[k]) || !std::isfinite(d->s0[k]))
            return fail(MISDC_EINVAL, "hf/s0[%d] not finite", k);
    }
    if (!(d->alpha0 >= 0) || !(d->rho0 > 0) || !(d->p_atm > 0) || !(d->R_u > 0) || !(d->R_c > 0))
        return fail(MISDC_EINVAL, "alpha0 >= 0 and rho0, p_atm, R_u, R_c > 0 required");
    for (int j = 0; j < d->n_reactions; ++j) {
        for (int s = 0; s < 2; ++s) {
            const int a = d->react[2 * j + s], b = d->prod[2 * j + s];
            if (a < -1 || a >= d->n_species || b < -1 || b >= d->n_species)
                return fail(MISDC_EINVAL, "reaction %d: species index out of range", j);
            if (a == d->bath || b == d->bath)
                return fail(MISDC_EINVAL, "reaction %d involves the bath species", j);
        }
        if (d->react[2 * j] < 0 && d->react[2 * j + 1] < 0)
            return fail(MISDC_EINVAL, "reaction %d has no reactant", j);
        if (d->prod[2 * j] < 0 && d->prod[2 * j + 1] < 0)
            return fail(MISDC_EINVAL, "reaction %d has no product", j);
        if (!(d->A[j] >= 0) || !std::isfinite(d->A[j]) || !std::isfinite(d->beta[j]) ||
            !std::isfinite(d->Ea[j]))
            return fail(MISDC_EINVAL, "reaction %d: invalid Arrhenius parameters", j);
        // mass balance: sum of W over reactant slots equals that over product slots
        double wr = 0, wp = 0;
        for (int s = 0; s < 2; ++s) {
            if (d->react[2 * j + s] >= 0) wr += d->W[d->react[2 * j + s]];
            if (d->prod[2 * j + s] >= 0) wp += d->W[d->prod[2 * j + s]];
        }
        if (std::fabs(wr - wp) > 1e-9 * (wr + wp))
            return fail(MISDC_EINVAL, "reaction %d is not mass balanced", j);
    }
    return MISDC_OK;
}

int check_opts(const misdc_opts* o) {
    if (!o) return fail(MISDC_EINVAL, "options are NULL");
    if (o->n_nodes < 2 || o->n_nodes > MAX_NODES)
        return fail(MISDC_EINVAL, "n_nodes must be in [2, %d]", MAX_NODES);
    if (o->n_sweeps < 1 || o->n_sweeps > 64)
        return fail(MISDC_EINVAL, "n_sweeps must be in [1, 64]");
    if (o->scheme < MISDC_SCHEME_MISDC || o->scheme > MISDC_SCHEME_IMEXQ)
        return fail(MISDC_EINVAL, "unknown scheme %d", o->scheme);
    if (o->scheme == MISDC_SCHEME_IMEXQ && o->use_graph)
        return fail(MISDC_EINVAL, "IMEXQ's coupled solve is driven by the host and cannot be "
                                  "replayed as a graph");
    if (!(o->imexq_tol == o->imexq_tol) || !(o->imexq_krylov_rtol == o->imexq_krylov_rtol))
        return fail(MISDC_EINVAL, "IMEXQ tolerance is NaN");
    if (o->nu < 1 || o->nu > 16) return fail(MISDC_EINVAL, "nu must be in [1, 16]");
    if (o->scheme != MISDC_SCHEME_CISDCQ && o->nu != 1)
        return fail(MISDC_EINVAL, "nu > 1 needs the concurrent scheme");
    if (o->qe_mode != MISDC_QE_CUMULATIVE && o->qe_mode != MISDC_QE_LITERAL)
        return fail(MISDC_EINVAL, "unknown qe_mode %d", o->qe_mode);
    if (!(o->nu_tol == o->nu_tol)) return fail(MISDC_EINVAL, "nu_tol is NaN");
    if (o->nu_tol > 0 && o->scheme != MISDC_SCHEME_CISDCQ)
        return fail(MISDC_EINVAL, "adaptive nested iterations need the concurrent scheme");
    if (o->nu_tol > 0 && o->use_graph)
        return fail(MISDC_EINVAL, "adaptive nested iterations cannot be replayed as a graph");
    if (o->pipeline != 0 && o->pipeline != 1) return fail(MISDC_EINVAL, "pipeline must be 0 or 1");
    if (o->pipeline && (o->scheme != MISDC_SCHEME_CISDCQ || o->nu < 2 || o->nu_tol > 0 ||
                        o->serialize))
        return fail(MISDC_EINVAL, "pipelined passes need CISDCQ with nu >= 2 fixed passes on "
                                  "separate streams (no nu_tol, no serialize)");
    // a captured graph does not keep the diffusion lanes' CU masks, and two
    // persistent diffusion solves sharing CUs could each wait for CUs the
    // other holds
    if (o->pipeline && o->use_graph)
        return fail(MISDC_EINVAL, "pipelined passes are not replayed as a graph (the diffusion "
                                  "lanes' CU masks do not survive capture)");
    return MISDC_OK;
}

misdc_newton_opts newton_defaults(const misdc_newton_opts* in) {
    misdc_newton_opts o;
    o.tol = 1e-12;
    o.maxit = 200;
    o.dtau0 = 1.0;
    o.dtau_max = 1e10;
    o.neg_slack = 1e-6;
    o.kernel = MISDC_NEWTON_AUTO;
    o.lu = MISDC_LU_FP64;
    if (in) {
        o.kernel = in->kernel;
        o.lu = in->lu;
        if (in->tol > 0) o.tol = in->tol;
        if (in->maxit > 0) o.maxit = in->maxit;
        if (in->dtau0 > 0) o.dtau0 = in->dtau0;
        if (in->dtau_max > 0) o.dtau_max = in->dtau_max;
        if (in->neg_slack > 0) o.neg_slack = in->neg_slack;
    }
    return o;
}

template <class T>
int dalloc(misdc_integ_s* I, T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, count * sizeof(T) + 256);
    if (e != hipSuccess) return fail(MISDC_ENOMEM, "hipMalloc of %zu bytes: %s", count * sizeof(T),
                                     hipGetErrorString(e));
    I->allocs.push_back(q);
    *p = (T*)q;
    return MISDC_OK;
}

// Linear combination builder.  Terms added with addS carry a factor of the
// step size: with a scalar step it is folded into the weight (dts * w), with
// per-cell step sizes (ensembles) the kernel multiplies by dtc[cell].
struct LC {
    LinComb lc;
    double dts = 1.0;
    const double* dtc = nullptr;
    LC(int nfields, int64_t n, double dt_scalar, const double* dt_cell) {
        std::memset(&lc, 0, sizeof(lc));
        lc.nfields = nfields;
        lc.ncells = n;
        dts = dt_cell ? 1.0 : dt_scalar;
        dtc = dt_cell;
        lc.scale = dt_cell;
    }
    int out(double* p) {
        lc.out[lc.nout] = p;
        return lc.nout++;
    }
    // add weight w (to output o) of array X with nf fields; merges duplicates
    bool sc[LC_MAX_TERMS] = {};
    // fold: an array that is an output of this same pass enters as that
    // output's weights (its old content is not read)
    bool fold = false;
    void put(int o, double w, const double* X, int nf, bool scaled) {
        if (w == 0.0 || !X) return;
        if (fold)
            for (int q = 0; q < lc.nout; ++q)
                if (lc.out[q] == X && q != o) {
                    if (scaled && dtc) {           // would scale its terms twice
                        lc.nterms = LC_MAX_TERMS + 1;
                        return;
                    }
                    for (int t = 0; t < lc.nterms; ++t) lc.W[o][t] += w * lc.W[q][t];
                    return;
                }
        for (int t = 0; t < lc.nterms; ++t)
            if (lc.X[t] == X && sc[t] == scaled) {
                lc.W[o][t] += w;
                return;
            }
        // more terms than the kernel takes: launch_lincomb reports it
        if (lc.nterms >= LC_MAX_TERMS) {
            lc.nterms = LC_MAX_TERMS + 1;
            return;
        }
        const int t = lc.nterms++;
        lc.X[t] = X;
        lc.nf[t] = nf;
        sc[t] = scaled;
        for (int q = 0; q < LC_MAX_OUT; ++q) lc.W[q][t] = 0.0;
        lc.W[o][t] = w;
        if (scaled && dtc) lc.smask |= 1u << t;
    }
    void add(int o, double w, const double* X, int nf) { put(o, w, X, nf, false); }
    void addS(int o, double w, const double* X, int nf) { put(o, dts * w, X, nf, true); }
};

int eval_ops(misdc_integ_s* I, const NodeBuf& b, double* th, hipStream_t s, bool with_R) {
    int rc = launch_transport(*I->mech, *I->grid, b.phi, b.T, b.FA, b.FD, th, s);
    if (rc) return rc;
    if (with_R) {
        rc = launch_reaction_source(*I->mech, I->n, b.phi, b.phi + (size_t)I->N * I->n, b.FR, s);
        if (rc) return rc;
    }
    return MISDC_OK;
}

hipEvent_t pool_event(misdc_integ_s* I) {
    if (!I->ev_pool.empty()) {
        hipEvent_t e = I->ev_pool.back();
        I->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Sums the durations of completed timing pairs (the streams are synchronised).
int drain_timing(misdc_integ_s* I) {
    for (auto& t : I->timed) {
        float ms = 0.f;
        MISDC_HIP(hipEventElapsedTime(&ms, t.a, t.b));
        I->t_ms[t.kind] += ms;
        I->t_cnt[t.kind] += 1;
        I->ev_pool.push_back(t.a);
        I->ev_pool.push_back(t.b);
    }
    I->timed.clear();
    return MISDC_OK;
}

// Records a start event when profiling; returns it (or null).
hipEvent_t timing_begin(misdc_integ_s* I, hipStream_t s) {
    if (!I->opt.profile || I->capturing) return nullptr;
    hipEvent_t e = pool_event(I);
    if (e && hipEventRecord(e, s) != hipSuccess) return nullptr;
    return e;
}

void timing_end(misdc_integ_s* I, hipEvent_t start, hipStream_t s, int kind) {
    if (!start) return;
    hipEvent_t e = pool_event(I);
    if (!e || hipEventRecord(e, s) != hipSuccess) return;
    I->timed.push_back({start, e, kind});
}

// ---- diffusion task at node p of nested iteration ell (writes phiAD[p]) ----
// Adds to b the outputs of the diffusion task's right-hand side pass: the
// right-hand side (rD) and the solve's initial guess (phiAD[p]); returns the
// implicit factor cf (c = dt * cf) and the lagged temperature of the operator.
void diffusion_rhs(misdc_integ_s* I, int ell, int p, LC& b, double& cf_out,
                   const double*& T_lag_out) {
    const int M = I->M, N = I->N, NF = I->NF;
    const Tables& t = I->tab;
    const int m = p - 1;
    auto& L0 = I->lev[0];
    auto& Lc = I->lev[ell + 1];       // iteration ell+1 (serial schemes: the new sweep)
    auto& Lp = I->lev[ell];           // iteration ell (lagged); ell = 0: sweep k
    const int o = b.out(I->dlane(ell).rD);
    double cf = 0.0;                  // implicit factor c = dt * cf
    const double* T_lag = nullptr;
    if (I->opt.scheme == MISDC_SCHEME_MISDC) {
        cf = t.tau[p] - t.tau[p - 1];
        // phi^{m,(k+1)} + dt^m FA(phi^{m,(k+1)}) + [constant part in C]
        // (the advection bracket at node 0 vanishes: phi^0 is fixed)
        b.add(o, 1.0, I->C[p], NF);
        b.add(o, 1.0, (m == 0) ? L0[0].phi : Lc[m].phi, NF);
        if (m >= 1) b.addS(o, cf, Lc[m].FA, NF);
        T_lag = L0[p].T;
    } else if (I->opt.scheme == MISDC_SCHEME_MISDCQ) {
        cf = t.QI[p - 1][p - 1];
        b.add(o, 1.0, I->C[p], NF);
        for (int j = 1; j <= m; ++j) {
            b.addS(o, t.QE[p - 1][j - 1], Lc[j].FA, NF);
            b.addS(o, t.QI[p - 1][j - 1], Lc[j].FD, NF);
        }
        T_lag = L0[p].T;
    } else {
        cf = t.QI[p - 1][p - 1];
        b.add(o, 1.0, I->C[p], NF);
        for (int j = 1; j <= m - 1; ++j) {
            b.addS(o, t.QE[p - 1][j - 1], Lc[j].FA, NF);
            b.addS(o, t.QI[p - 1][j - 1], Lc[j].FD, NF);
            b.addS(o, t.QI[p - 1][j - 1], Lc[j].FR, N);
        }
        if (m >= 1) {
            const double* lagA = (ell == 0) ? I->hatA[m] : Lp[m].FA;
            const double* lagD = (ell == 0) ? I->hatD[m] : Lp[m].FD;
            b.addS(o, t.QE[p - 1][m - 1], lagA, NF);
            b.addS(o, t.QI[p - 1][m - 1], lagD, NF);
            b.addS(o, t.QI[p - 1][m - 1], Lp[m].FR, N);
        }
        b.addS(o, cf, Lp[p].FR, N);
        T_lag = (ell == 0) ? L0[p].T : Lp[p].T;
    }
    // initial guess of the iterative solve, the lagged state at this node,
    // copied into the solution array by the same kernel
    const double* guess = (I->opt.scheme == MISDC_SCHEME_CISDCQ && ell > 0) ? Lp[p].phi : L0[p].phi;
    const int og = b.out(I->phiAD[p]);
    b.add(og, 1.0, guess, NF);
    cf_out = cf;
    T_lag_out = T_lag;
    (void)M;
}

// Whether the right-hand side of the diffusion task at node p is formed in
// two passes: every term but the lagged operators FA, FD at phi_AD^{p-1}
// (eqs. initial_lagged_values_A/D) by a pass on the reaction stream while the
// solve of node p-1 still runs, and those two terms (formed from phi_AD^{p-1}
// itself, so no lag transport pass) with the face coefficients after it.
// Concurrent scheme, first nested iteration, p >= 2, two-stream schedule, a
// single grid: ensembles keep the one-pass form, which their persistent
// stages (misdc_tune.fused) share, so that both give the same bits.
bool split_rhs(const misdc_integ_s* I, int ell, int p) {
    return I->opt.scheme == MISDC_SCHEME_CISDCQ && ell == 0 && p >= 2 && p <= I->M &&
           !I->pipe && !I->fused && I->grid->n_flames == 0 && I->rP[0];
}

// Removes term t of a linear combination.
void drop_term(LinComb& lc, int t) {
    for (int u = t; u + 1 < lc.nterms; ++u) {
        lc.X[u] = lc.X[u + 1];
        lc.nf[u] = lc.nf[u + 1];
        for (int q = 0; q < LC_MAX_OUT; ++q) lc.W[q][u] = lc.W[q][u + 1];
    }
    const unsigned low = lc.smask & ((1u << t) - 1u);
    const unsigned high = (t + 1 < 32) ? ((lc.smask >> (t + 1)) << t) : 0u;
    lc.smask = low | high;
    --lc.nterms;
}

// The first pass of a split right-hand side (node p) on stream s: every term
// but the lagged operators into rP[p & 1], and the initial guess.  Fills the
// remaining terms' weights (qa, qd, scaled per cell or not) into lag.
int partial_rhs(misdc_integ_s* I, int p, double dt, hipStream_t s, LagRhs& lag) {
    const int NF = I->NF;
    LC b(NF, I->n, dt, I->dtc);
    double cf = 0.0;
    const double* T_lag = nullptr;
    diffusion_rhs(I, 0, p, b, cf, T_lag);
    LinComb& lc = b.lc;
    lc.out[0] = I->rP[p & 1];
    lag = LagRhs();
    for (int t = lc.nterms - 1; t >= 0; --t) {
        const bool is_a = lc.X[t] == I->hatA[p - 1], is_d = lc.X[t] == I->hatD[p - 1];
        if (!is_a && !is_d) continue;
        if (lc.W[1][t] != 0.0) return fail(MISDC_EINVAL, "lagged operator in the guess");
        (is_a ? lag.qa : lag.qd) = lc.W[0][t];
        const bool scaled = (lc.smask >> t) & 1u;
        if (scaled) lag.scale = I->dtc;
        drop_term(lc, t);
    }
    lag.src = I->phiAD[p - 1];
    lag.part = I->rP[p & 1];
    lag.T_lag = T_lag;
    return launch_lincomb(lc, s);
}

int diffusion_task(misdc_integ_s* I, int ell, int p, double dt) {
    const int NF = I->NF;
    const int64_t n = I->n;
    const misdc_integ_s::DLane L = I->dlane(ell);
    double cf = 0.0;
    const double* T_lag = nullptr;
    LC b(NF, n, dt, I->dtc);
    diffusion_rhs(I, ell, p, b, cf, T_lag);
    int rc;
    // the second pass of a split right-hand side, formed with the solve
    // (launch_diffusion_solve)
    LagRhs second;
    bool split = false;
    if (ell == 0 && p == 1 && I->d1_split) {
        // the terms of node M (prepare_constants), once R_M's solve is done
        I->d1_split = false;
        MISDC_HIP(hipStreamWaitEvent(L.s, I->ev_newtonM, 0));
        second = I->d1w;
        split = true;
        MISDC_HIP(hipEventRecord(I->ev_d1, L.s));
    } else if (split_rhs(I, ell, p)) {
        // the first pass ran on the reaction stream (run_sweep); the lagged
        // operators of node p-1 and the face coefficients now
        MISDC_HIP(hipStreamWaitEvent(L.s, I->evP[p], 0));
        second = I->lagw[p];
        second.th = L.th;
        split = true;
    } else if (ell == 0 && p == 1 && I->d1_ready) {
        I->d1_ready = false;          // formed by the sweep constants' pass
    } else {
        // the same pass computes the face coefficients of the lagged operator
        if ((rc = launch_lincomb_faces(b.lc, *I->grid, T_lag, *L.dw, L.s))) return rc;
    }
    // the solve is next on this stream: a staggered reaction task waits for this
    if (I->stagger && I->sR != I->sD) MISDC_HIP(hipEventRecord(I->C_ev(ell + 1, p), L.s));
    // with profiling, the events bracket the solve kernel itself (CG or cyclic)
    const bool timed = I->opt.profile && !I->capturing;
    hipEvent_t t0 = timed ? pool_event(I) : nullptr;
    hipEvent_t t1 = timed ? pool_event(I) : nullptr;
    const bool lag_init = (I->opt.scheme == MISDC_SCHEME_CISDCQ && ell == 0 && p < I->M);
    rc = launch_diffusion_solve(*I->mech, *I->grid, *L.dw, dt * cf, I->dtf, cf, T_lag, L.rD,
                                I->phiAD[p], 1, I->opt.cg_rtol, I->opt.cg_maxit, L.s, t0, t1,
                                I->TAD[p], L.cgstats, lag_init ? L.th : nullptr, true,
                                split ? &second : nullptr);
    if (rc) return rc;
    if (t0 && t1) I->timed.push_back({t0, t1, 0});
    return MISDC_OK;
}

// Lag initialisation (initial_lagged_values_A/D) of the concurrent scheme's
// first nested iteration: FA, FD at phi_AD^{p,(k+1,1)} (theta of T(phi_AD)
// written by the solve's closure), read only by the diffusion task of node
// p+1, so none for the last node.  Issued after the event that releases the
// reaction task of node p, which does not read them.
int lag_transport(misdc_integ_s* I, int ell, int p) {
    if (I->opt.scheme != MISDC_SCHEME_CISDCQ || ell != 0 || p >= I->M) return MISDC_OK;
    if (split_rhs(I, ell, p + 1)) return MISDC_OK;      // formed in D_{p+1}'s second pass
    const misdc_integ_s::DLane L = I->dlane(ell);
    return launch_transport(*I->mech, *I->grid, I->phiAD[p], I->TAD[p], I->hatA[p], I->hatD[p],
                            L.th, L.s, true);
}

// ---- reaction task at node p of nested iteration ell (writes lev[ell+1][p]) ----
// Right-hand side b of the reaction task at node p of nested iteration ell
// (eqs. ..._misdc_discrete_form_R, ..._misdcq_discrete_form_R and
// ..._amisdcq_discrete_form_R_alt) into out; returns the implicit factor cf
// (c = dt * cf).
double reaction_rhs(misdc_integ_s* I, int ell, int p, LC& b, double* out) {
    const int N = I->N;
    const Tables& t = I->tab;
    const int m = p - 1;
    auto& L0 = I->lev[0];
    auto& Lc = I->lev[ell + 1];
    auto& Lp = I->lev[ell];
    const int o = b.out(out);
    double cf = 0.0;
    b.add(o, 1.0, I->phiAD[p], N);
    if (I->opt.scheme == MISDC_SCHEME_MISDC) {
        cf = t.tau[p] - t.tau[p - 1];
        b.addS(o, -cf, L0[p].FR, N);
    } else if (I->opt.scheme == MISDC_SCHEME_MISDCQ) {
        cf = t.QI[p - 1][p - 1];
        b.add(o, 1.0, I->CR[p], N);
        for (int j = 1; j <= m; ++j) b.addS(o, t.QI[p - 1][j - 1], Lc[j].FR, N);
    } else {
        cf = t.QI[p - 1][p - 1];
        if (m >= 1) {
            b.addS(o, t.QI[p - 1][m - 1], Lc[m].FR, N);
            b.addS(o, -t.QI[p - 1][m - 1], Lp[m].FR, N);
        }
        b.addS(o, -cf, Lp[p].FR, N);
    }
    return cf;
}

int reaction_task(misdc_integ_s* I, int ell, int p, double dt) {
    const int N = I->N, NF = I->NF;
    const int64_t n = I->n;
    auto& Lc = I->lev[ell + 1];
    auto& Lp = I->lev[ell];
    const misdc_integ_s::RLane L = I->rlane(ell);
    LC b(N, n, dt, I->dtc);
    const double cf = reaction_rhs(I, ell, p, b, L.bR);
    int rc = launch_lincomb(b.lc, L.s);
    if (rc) return rc;
    NodeBuf& out = Lc[p];
    const double c_scalar = I->dtc ? cf : dt * cf;
    const double* guess = Lp[p].phi;
    if (I->mlp && (I->guess_sweeps <= 0 || I->sweep_index < I->guess_sweeps)) {
        // the plain guess, replaced cell by cell by the learned one where
        // that has the smaller residual
        if ((rc = launch_copy(out.phi, Lp[p].phi, (int64_t)N * n, L.s))) return rc;
        if ((rc = mlp_guess(*I->mech, I->mlp, n, L.bR, I->phiAD[p] + (size_t)N * n, I->dtc,
                            c_scalar, out.phi, n, I->choice, L.s)))
            return rc;
        if ((rc = launch_count_flags(I->choice, n, I->nstats + 6, L.s))) return rc;
        guess = out.phi;
    }
    NewtonArgs a;
    a.n = n;
    a.bY = L.bR;
    a.ldb = n;
    a.h = I->phiAD[p] + (size_t)N * n;
    // c = dt * cf: per cell for ensembles with per-flame step sizes
    a.c = I->dtc;
    a.c_scalar = c_scalar;
    a.guess = guess;
    a.ldg = n;
    a.Y = out.phi;
    a.ldy = n;
    a.T = out.T;
    // enthalpy is not changed by the reaction step: the solve copies it
    a.h_out = out.phi + (size_t)N * n;
    a.FR = out.FR;
    a.ldf = n;
    a.iters = L.iters;
    a.lu_info = (I->opt.newton.lu == MISDC_LU_FP32_MFMA) ? L.lu_info : nullptr;
    a.stats = I->nstats;
    a.buckets = I->nbuckets;
    a.hist = I->nhist + (size_t)I->sweep_index * NEWTON_HIST_SETS * NEWTON_HIST_BINS;
    if (I->grid->dim == 2 && I->grid->n_flames == 0) {
        a.tile_nx = (int)I->grid->nx;
        a.tile_ny = (int)I->grid->ny;
    }
    a.opt = I->opt.newton;
    const bool last_prep = (p == I->M && I->prep_newton);
    if (last_prep) a.th_out = I->thM;
    // staggered: the Newton solve of node p starts once the diffusion solve
    // of node p+1 (issued just before this task) is about to start, so that
    // the persistent solve's workgroups take their CUs before the Newton
    // waves fill the device
    if (I->stagger && I->sR != I->sD && I->opt.scheme == MISDC_SCHEME_CISDCQ && p < I->M)
        MISDC_HIP(hipStreamWaitEvent(L.s, I->C_ev(ell + 1, p + 1), 0));
    hipEvent_t t0 = timing_begin(I, L.s);
    rc = launch_reaction_newton(*I->mech, a, L.s);
    if (rc) return rc;
    timing_end(I, t0, L.s, 1);
    if (last_prep) {
        // the next sweep's first diffusion pass needs this solve's outputs only
        MISDC_HIP(hipEventRecord(I->ev_newtonM, L.s));
        I->prep_newton = false;
    }
    if (I->rec_buf && I->rec_count < I->rec_cap) {
        // record (b_Y, h, c, Y) of this reaction task
        double* slot = I->rec_buf + (size_t)I->rec_count * (2 * N + 2) * n;
        if ((rc = launch_copy(slot, L.bR, (int64_t)N * n, L.s))) return rc;
        if ((rc = launch_copy(slot + (size_t)N * n, I->phiAD[p] + (size_t)N * n, n, L.s))) return rc;
        if ((rc = launch_fill_c(n, I->dtc, c_scalar, slot + (size_t)(N + 1) * n, L.s))) return rc;
        if ((rc = launch_copy(slot + (size_t)(N + 2) * n, out.phi, (int64_t)N * n, L.s))) return rc;
        ++I->rec_count;
    }
    if (p == I->M && I->skip_final_ops && ell == I->nu - 1) return MISDC_OK;
    if (last_prep) {
        // after the next sweep's first diffusion pass (flush_deferred)
        I->dfr.pending = true;
        I->dfr.out = out;
        I->dfr.th = L.th;
        I->dfr.s = L.s;
        return MISDC_OK;
    }
    rc = eval_ops(I, out, L.th, L.s, false);
    (void)NF;
    return rc;
}

// ---- IMEXQ's coupled task at node p (writes lev[1][p]) ----
// Right-hand side C^p + dt sum_{j<=m} [QE_{p,j} FA_j + QI_{p,j} (FD_j + FR_j)]
// at sweep k+1, the guess phi^{p,(k)}, the coupled solve with diffusion
// coefficients lagged at phi^{p,(k)}, then FA, FD, FR and T at the result.
// Everything runs on the diffusion stream.
int imexq_task(misdc_integ_s* I, int p, double dt) {
    const int N = I->N, NF = I->NF;
    const int64_t n = I->n;
    const Tables& t = I->tab;
    const int m = p - 1;
    auto& L0 = I->lev[0];
    auto& Lc = I->lev[1];
    LC b(NF, n, dt, I->dtc);
    const int o = b.out(I->rD);
    b.add(o, 1.0, I->C[p], NF);
    for (int j = 1; j <= m; ++j) {
        b.addS(o, t.QE[p - 1][j - 1], Lc[j].FA, NF);
        b.addS(o, t.QI[p - 1][j - 1], Lc[j].FD, NF);
        b.addS(o, t.QI[p - 1][j - 1], Lc[j].FR, N);
    }
    const int og = b.out(Lc[p].phi);
    b.add(og, 1.0, L0[p].phi, NF);
    int rc = launch_lincomb(b.lc, I->sD);
    if (rc) return rc;
    const misdc_opts& op = I->opt;
    const double tol = op.imexq_tol > 0 ? op.imexq_tol : 1e-13;
    const int maxit = op.imexq_maxit > 0 ? op.imexq_maxit : 30;
    const double krtol = op.imexq_krylov_rtol > 0 ? op.imexq_krylov_rtol : 1e-9;
    const int kmaxit = op.imexq_krylov_maxit > 0 ? op.imexq_krylov_maxit : 400;
    rc = coupled_solve(*I->mech, *I->grid, I->cw, dt * t.QI[p - 1][p - 1], L0[p].T, I->rD,
                       Lc[p].phi, tol, maxit, krtol, kmaxit, I->cst, I->sD);
    if (rc) return rc;
    NodeBuf& out = Lc[p];
    if ((rc = launch_temperature(*I->mech, n, out.phi, out.phi + (size_t)N * n, out.T, I->sD)))
        return rc;
    return eval_ops(I, out, I->thD, I->sD, true);
}

// sweep-start constants (all terms of sweep k)
// The sweep constants C^1..C^M as one linear combination of the state at
// node 0 and F at the nodes of lev[0] (the sweep just finished).
LC constants_lc(misdc_integ_s* I, double dt) {
    const int M = I->M, N = I->N, NF = I->NF;
    const int64_t n = I->n;
    const Tables& t = I->tab;
    auto& L0 = I->lev[0];
    LC b(NF, n, dt, I->dtc);
    for (int p = 1; p <= M; ++p) {
        const int o = b.out(I->C[p]);
        if (I->opt.scheme == MISDC_SCHEME_MISDC) {
            // dt S^{m:m+1} F^{(k)} - dt^m FA^{m,(k)} - dt^m FD^{p,(k)}
            const double cm = t.tau[p] - t.tau[p - 1];
            for (int j = 0; j <= M; ++j) {
                b.addS(o, t.S[p - 1][j], L0[j].FA, NF);
                b.addS(o, t.S[p - 1][j], L0[j].FD, NF);
                b.addS(o, t.S[p - 1][j], L0[j].FR, N);
            }
            if (p - 1 >= 1) b.addS(o, -cm, L0[p - 1].FA, NF);
            b.addS(o, -cm, L0[p].FD, NF);
        } else {
            b.add(o, 1.0, L0[0].phi, NF);
            for (int j = 0; j <= M; ++j) {
                b.addS(o, t.Q[p - 1][j], L0[j].FA, NF);
                b.addS(o, t.Q[p - 1][j], L0[j].FD, NF);
                b.addS(o, t.Q[p - 1][j], L0[j].FR, N);
            }
            for (int j = 1; j <= p - 1; ++j) b.addS(o, -t.QE[p - 1][j - 1], L0[j].FA, NF);
            const bool with_R = (I->opt.scheme == MISDC_SCHEME_CISDCQ ||
                                  I->opt.scheme == MISDC_SCHEME_IMEXQ);
            for (int j = 1; j <= p; ++j) {
                b.addS(o, -t.QI[p - 1][j - 1], L0[j].FD, NF);
                if (with_R) b.addS(o, -t.QI[p - 1][j - 1], L0[j].FR, N);
            }
        }
    }
    return b;
}

int sweep_constants(misdc_integ_s* I, double dt) {
    const int M = I->M, N = I->N;
    const int64_t n = I->n;
    const Tables& t = I->tab;
    auto& L0 = I->lev[0];
    LC b = constants_lc(I, dt);
    int rc;
    if (I->opt.scheme == MISDC_SCHEME_MISDCQ) {
        LC r(N, n, dt, I->dtc);
        for (int p = 1; p <= M; ++p) {
            const int o = r.out(I->CR[p]);
            for (int j = 1; j <= p; ++j) r.addS(o, -t.QI[p - 1][j - 1], L0[j].FR, N);
        }
        if ((rc = launch_lincomb(r.lc, I->dlane(0).s))) return rc;
    }
    // the first diffusion task's right-hand side (which contains C^1, folded
    // in as its weights), initial guess and face coefficients in the same
    // pass: one launch fewer between the sweeps on the critical path
    I->d1_ready = false;
    if (M + 2 <= LC_MAX_OUT && I->opt.scheme != MISDC_SCHEME_IMEXQ) {
        LC f = b;
        f.fold = true;
        double cf = 0.0;
        const double* T_lag = nullptr;
        diffusion_rhs(I, 0, 1, f, cf, T_lag);
        if (f.lc.nterms <= LC_MAX_TERMS && f.lc.nout <= LC_MAX_OUT) {
            if ((rc = launch_lincomb_faces(f.lc, *I->grid, T_lag, *I->dlane(0).dw, I->dlane(0).s)))
                return rc;
            I->d1_ready = true;
            return MISDC_OK;
        }
    }
    return launch_lincomb(b.lc, I->dlane(0).s);
}

// Whether the next sweep's constants are formed in the split form
// (prepare_constants); the same conditions as split right-hand sides, a
// fixed number of nested iterations, and C^1..C^M, D_1's right-hand side and
// its guess in one pass.
bool split_constants(const misdc_integ_s* I) {
    return split_rhs(I, 0, 2) && !(I->opt.nu_tol > 0 && I->nu >= 3) && I->M + 2 <= LC_MAX_OUT &&
           !I->dtc;
}

// Issued on the reaction stream s before R_M of the sweep's last nested
// iteration (whose results are lev[lv]): the next sweep's constants and
// D_1's right-hand side (C^1 folded in) and guess, without the terms of node
// M.  Those terms follow: C^1..C^M's in cfin (after R_M), D_1's in its own
// pass (d1w, after R_M's Newton solve).  Leaves consts_ready false where the
// terms do not fit one pass.
int prepare_constants(misdc_integ_s* I, double dt, int lv, hipStream_t s) {
    const int M = I->M, NF = I->NF;
    // the next sweep's view of the levels (undone below)
    for (int p = 1; p <= M; ++p) std::swap(I->lev[0][p], I->lev[lv][p]);
    LC b = constants_lc(I, dt);
    LC f = b;
    f.fold = true;
    double cf = 0.0;
    const double* T_lag = nullptr;
    diffusion_rhs(I, 0, 1, f, cf, T_lag);
    const NodeBuf bM = I->lev[0][M];
    for (int p = 1; p <= M; ++p) std::swap(I->lev[0][p], I->lev[lv][p]);
    LinComb& lc = f.lc;
    if (lc.nterms > LC_MAX_TERMS || lc.nout > LC_MAX_OUT || lc.smask) return MISDC_OK;
    int o1 = -1;
    for (int o = 0; o < lc.nout; ++o)
        if (lc.out[o] == I->dlane(0).rD) o1 = o;
    if (o1 < 0) return MISDC_OK;
    // the completion of C^p: C^p plus its node-M terms
    LC c(NF, I->n, 1.0, nullptr);
    for (int p = 1; p <= M; ++p) {
        const int o = c.out(I->C[p]);
        c.add(o, 1.0, I->C[p], NF);
    }
    LagRhs d1;
    const double* node_m[3] = {bM.FA, bM.FD, bM.FR};
    for (int t = lc.nterms - 1; t >= 0; --t) {
        int k = -1;
        for (int q = 0; q < 3; ++q)
            if (lc.X[t] == node_m[q]) k = q;
        if (k < 0) continue;
        for (int o = 0; o < lc.nout; ++o) {
            const double w = lc.W[o][t];
            if (w == 0.0) continue;
            if (o == o1) {
                (k == 0 ? d1.qa : k == 1 ? d1.qd : d1.qr) = w;
            } else if (o < M && lc.out[o] == I->C[o + 1]) {
                c.add(o, w, lc.X[t], lc.nf[t]);
            } else {
                return fail(MISDC_EINVAL, "node-M term in output %d of the sweep constants", o);
            }
        }
        drop_term(lc, t);
    }
    if (c.lc.nterms > LC_MAX_TERMS) return MISDC_OK;
    lc.out[o1] = I->rP[1];
    int rc = launch_lincomb(lc, s);
    if (rc) return rc;
    d1.src = bM.phi;
    d1.th = I->thM;                   // written by R_M's solve
    d1.fr = bM.FR;
    d1.part = I->rP[1];
    d1.T_lag = T_lag;
    I->d1w = d1;
    I->cfin = c.lc;
    I->dfr.cfin = true;
    I->consts_ready = true;
    I->prep_newton = true;
    return MISDC_OK;
}

// max over fields of max_i |new - old| / max_i |new| from the (difference,
// magnitude) pairs of a field_diff_max reduction; a field that is zero
// everywhere counts 0 if unchanged, infinity otherwise
double pass_change(const double* pairs, int nf) {
    double worst = 0.0;
    for (int f = 0; f < nf; ++f) {
        const double d = pairs[2 * f], a = pairs[2 * f + 1];
        const double r = a > 0 ? d / a : (d == 0 ? 0.0 : HUGE_VAL);
        worst = r > worst ? r : worst;
    }
    return worst;
}

// One stage of a concurrent pass as one persistent launch (ensembles): the
// right-hand sides of D_{s+1} and R_s are formed by their usual passes, then
// one stage kernel solves the flames' diffusion systems and the cells'
// reaction problems from one work queue; everything is on the diffusion
// stream, whose order stands for the events of the two-stream schedule.
int fused_stage(misdc_integ_s* I, int ell, int s, double dt) {
    const int M = I->M, N = I->N, NF = I->NF;
    const int64_t n = I->n;
    const int pd = s + 1, pr = s;
    EnsembleStage st;
    int rc;
    if (pd <= M) {
        double cf = 0.0;
        const double* T_lag = nullptr;
        LC b(NF, n, dt, I->dtc);
        diffusion_rhs(I, ell, pd, b, cf, T_lag);
        if (ell == 0 && pd == 1 && I->d1_ready)
            I->d1_ready = false;          // formed by the sweep constants' pass
        else if ((rc = launch_lincomb_faces(b.lc, *I->grid, T_lag, I->dw, I->sD)))
            return rc;
        const bool lag_init = (ell == 0 && pd < M);
        st.has_d = true;
        st.nD = I->nD_items;
        st.d_items = I->d_items;
        st.c = dt * cf;
        st.cfac = cf;
        st.dtf = I->dtf;
        st.Kx = I->dw.Kx;
        st.rhs = I->rD;
        st.y = I->phiAD[pd];
        st.sc = I->dw.r;
        st.su = I->dw.z;
        st.sv = I->dw.p;
        st.sw = I->dw.q;
        st.T_out = I->TAD[pd];
        st.th_out = lag_init ? I->thD : nullptr;
        if (lag_init) {
            st.lagFA = I->hatA[pd];
            st.lagFD = I->hatD[pd];
        }
    }
    if (pr >= 1) {
        NodeBuf& out = I->lev[ell + 1][pr];
        LC b(N, n, dt, I->dtc);
        const double cf = reaction_rhs(I, ell, pr, b, I->bR);
        if ((rc = launch_lincomb(b.lc, I->sD))) return rc;
        NewtonArgs& a = st.na;
        a.n = n;
        a.bY = I->bR;
        a.ldb = n;
        a.h = I->phiAD[pr] + (size_t)N * n;
        a.c = I->dtc;
        a.c_scalar = I->dtc ? cf : dt * cf;
        a.guess = I->lev[ell][pr].phi;
        a.ldg = n;
        a.Y = out.phi;
        a.ldy = n;
        a.T = out.T;
        a.FR = out.FR;
        a.ldf = n;
        a.iters = I->iters;
        a.stats = I->nstats;
        a.buckets = I->nbuckets;
        a.hist = I->nhist + (size_t)I->sweep_index * NEWTON_HIST_SETS * NEWTON_HIST_BINS;
        a.opt = I->opt.newton;
        st.has_r = true;
        st.h_src = I->phiAD[pr] + (size_t)N * n;
        st.h_dst = out.phi + (size_t)N * n;
        st.rstate = out.phi;
        st.rT = out.T;
        st.rth = I->thR;
        st.rFA = out.FA;
        st.rFD = out.FD;
    }
    st.counters = I->stage_counters;
    hipEvent_t t0 = timing_begin(I, I->sD);
    if ((rc = launch_ensemble_stage(*I->mech, *I->grid, st, I->sD))) return rc;
    timing_end(I, t0, I->sD, 1);
    return MISDC_OK;
}

// Sweep 0 of a step: every node of the "previous sweep" holds phi^n and
// F(phi^n), so node 0's buffers stand for nodes 1..M (a sweep only reads
// lev[0]); the real buffers are put back before the sweep's S7 swap, or when
// the issue ends early.
struct FirstSweepNodes {
    misdc_integ_s* I;
    std::vector<NodeBuf> saved;
    FirstSweepNodes(misdc_integ_s* integ, bool on) : I(integ) {
        if (!on) return;
        auto& L0 = I->lev[0];
        saved.assign(L0.begin() + 1, L0.end());
        for (size_t p = 1; p < L0.size(); ++p) L0[p] = L0[0];
    }
    void restore() {
        for (size_t p = 0; p < saved.size(); ++p) I->lev[0][p + 1] = saved[p];
        saved.clear();
    }
    ~FirstSweepNodes() { restore(); }
};

// Issues the work deferred from a sweep's R_M (see Deferred) on its stream,
// after the event 'after' (may be null).
int flush_deferred(misdc_integ_s* I, hipEvent_t after) {
    auto& d = I->dfr;
    if (!d.pending) return MISDC_OK;
    d.pending = false;
    if (after) MISDC_HIP(hipStreamWaitEvent(d.s, after, 0));
    int rc = eval_ops(I, d.out, d.th, d.s, false);
    if (rc) return rc;
    if (d.cfin && (rc = launch_lincomb(I->cfin, d.s))) return rc;
    d.cfin = false;
    if (d.inc) {
        d.inc = false;
        rc = launch_field_diff_max(I->NF, I->n, d.inc_new, d.inc_old, I->inc_partial,
                                   I->inc_blocks, d.inc_out, d.s);
    }
    return rc;
}

// prep_next: another sweep of this step may follow (its constants can be
// prepared during this sweep's last solve); defer_inc: the sweep increment
// may be deferred with R_M's work (not when the caller reads it between
// sweeps)
int run_sweep(misdc_integ_s* I, int k, double dt, bool prep_next, bool defer_inc) {
    const int M = I->M;
    const int nu = (I->opt.scheme == MISDC_SCHEME_CISDCQ) ? I->nu : 1;
    int done = nu;                    // nested iterations done in this sweep
    int rc;
    FirstSweepNodes first(I, k == 0);
    // the step's last R_M: its F_A, F_D are never read (the next step starts
    // from the state)
    I->skip_final_ops = !prep_next && defer_inc && !(I->opt.nu_tol > 0 && I->nu >= 3);
    // the constants read every reaction output of the previous sweep; with
    // pipelined passes they also wait for every lane's last work of it,
    // since this sweep's tasks overwrite buffers those lanes read
    const hipStream_t s0 = I->dlane(0).s;
    // constants prepared by the previous sweep (prepare_constants): they are
    // complete on the reaction stream, which every later reader follows, and
    // D_1 waits for R_M's solve only
    const bool pre = I->consts_ready;
    I->consts_ready = false;
    I->const_on_r = pre;
    I->d1_split = pre;
    if (!pre) {
        MISDC_HIP(hipStreamWaitEvent(s0, I->R_ev(0, M), 0));
        if (I->pipe && k > 0) {
            MISDC_HIP(hipStreamWaitEvent(s0, I->pd_lane[1].end, 0));
            for (auto& r : I->pr_lane) MISDC_HIP(hipStreamWaitEvent(s0, r.end, 0));
        }
        rc = sweep_constants(I, dt);
        if (rc) return rc;
        // the first pass of D_2's split right-hand side reads the constants
        if (split_rhs(I, 0, 2)) MISDC_HIP(hipEventRecord(I->ev_const, s0));
    }
    if (I->opt.scheme == MISDC_SCHEME_IMEXQ) {
        for (int p = 1; p <= M; ++p)
            if ((rc = imexq_task(I, p, dt))) return rc;
        // the sweep's end is ordered on the reaction stream
        MISDC_HIP(hipEventRecord(I->R_ev(1, M), I->sD));
        MISDC_HIP(hipStreamWaitEvent(I->sR, I->R_ev(1, M), 0));
    } else if (I->opt.scheme != MISDC_SCHEME_CISDCQ) {
        for (int p = 1; p <= M; ++p) {
            if (p > 1) MISDC_HIP(hipStreamWaitEvent(I->sD, I->R_ev(1, p - 1), 0));
            rc = diffusion_task(I, 0, p, dt);
            if (rc) return rc;
            MISDC_HIP(hipEventRecord(I->D_ev(1, p), I->sD));
            MISDC_HIP(hipStreamWaitEvent(I->sR, I->D_ev(1, p), 0));
            rc = reaction_task(I, 0, p, dt);
            if (rc) return rc;
            MISDC_HIP(hipEventRecord(I->R_ev(1, p), I->sR));
        }
    } else {
        const bool adapt = I->opt.nu_tol > 0 && nu >= 3;
        for (int ell = 0; ell < nu; ++ell) {
            // the streams of this pass's tasks (the same two for every pass
            // unless the passes are pipelined)
            const hipStream_t sd = I->dlane(ell).s, sr = I->rlane(ell).s;
            if (I->fused) {
                for (int s = 0; s <= M; ++s)
                    if ((rc = fused_stage(I, ell, s, dt))) return rc;
                continue;
            }
            for (int s = 0; s <= M; ++s) {
                const int pd = s + 1;     // diffusion node
                const int pr = s;         // reaction node
                if (pd <= M) {
                    if (pd >= 3) MISDC_HIP(hipStreamWaitEvent(sd, I->R_ev(ell + 1, pd - 2), 0));
                    if (ell >= 1) MISDC_HIP(hipStreamWaitEvent(sd, I->R_ev(ell, pd), 0));
                    rc = diffusion_task(I, ell, pd, dt);
                    if (rc) return rc;
                    MISDC_HIP(hipEventRecord(I->D_ev(ell + 1, pd), sd));
                    // the previous sweep's deferred R_M work, after D_1's pass
                    if (ell == 0 && pd == 1 && (rc = flush_deferred(I, I->ev_d1))) return rc;
                    if ((rc = lag_transport(I, ell, pd))) return rc;
                }
                if (pr >= 1) {
                    // the next sweep's constants but for node M's terms, while
                    // D_M's solve runs
                    if (pr == M && prep_next && ell == nu - 1 && split_constants(I) &&
                        (rc = prepare_constants(I, dt, ell + 1, sr)))
                        return rc;
                    MISDC_HIP(hipStreamWaitEvent(sr, I->D_ev(ell + 1, pr), 0));
                    rc = reaction_task(I, ell, pr, dt);
                    if (rc) return rc;
                    MISDC_HIP(hipEventRecord(I->R_ev(ell + 1, pr), sr));
                }
                // the first pass of D_{s+2}'s split right-hand side, which
                // reads R_s's outputs, while D_{s+1}'s solve runs
                if (split_rhs(I, ell, s + 2)) {
                    if (s == 0 && !I->const_on_r) MISDC_HIP(hipStreamWaitEvent(sr, I->ev_const, 0));
                    if ((rc = partial_rhs(I, s + 2, dt, sr, I->lagw[s + 2]))) return rc;
                    MISDC_HIP(hipEventRecord(I->evP[s + 2], sr));
                }
            }
            if (adapt && ell + 1 < nu) {
                // change of the node-M state made by pass ell+1 (pass 1
                // against sweep k), on the reaction stream after its last task
                rc = launch_field_diff_max(I->NF, I->n, I->lev[ell + 1][M].phi,
                                           I->lev[ell][M].phi, I->inc_partial, I->inc_blocks,
                                           I->pinc + (size_t)ell * I->NF * 2, I->sR);
                if (rc) return rc;
                if (ell >= 1) {
                    MISDC_HIP(hipMemcpyAsync(I->pinc_host, I->pinc,
                                             sizeof(double) * (size_t)(ell + 1) * I->NF * 2,
                                             hipMemcpyDeviceToHost, I->sR));
                    MISDC_HIP(hipStreamSynchronize(I->sR));
                    const double d1 = pass_change(I->pinc_host, I->NF);
                    const double dl = pass_change(I->pinc_host + (size_t)ell * I->NF * 2, I->NF);
                    if (dl <= I->opt.nu_tol * d1) {
                        done = ell + 1;
                        break;
                    }
                }
            }
        }
    }
    I->passes[k] = done;
    const int lv = done;
    // the stream of the sweep's last reaction task
    const hipStream_t se = I->rlane(lv - 1).s;
    I->s_last = se;
    // the next sweep's constants need the reaction outputs only, so they are
    // released before the increment below (which reads buffers that only
    // later work of this same stream overwrites)
    MISDC_HIP(hipEventRecord(I->R_ev(0, M), se));
    // sweep increment at node M (reaction stream, after the last reaction
    // task; deferred with R_M's transport when that is)
    if (I->dfr.pending && defer_inc) {
        I->dfr.inc = true;
        I->dfr.inc_new = I->lev[lv][M].phi;
        I->dfr.inc_old = I->lev[0][M].phi;
        I->dfr.inc_out = I->inc + (size_t)k * I->NF * 2;
    } else {
        rc = launch_field_diff_max(I->NF, I->n, I->lev[lv][M].phi, I->lev[0][M].phi,
                                   I->inc_partial, I->inc_blocks, I->inc + (size_t)k * I->NF * 2, se);
        if (rc) return rc;
    }
    if (I->pipe) {
        for (auto& d : I->pd_lane) MISDC_HIP(hipEventRecord(d.end, d.s));
        for (auto& r : I->pr_lane) MISDC_HIP(hipEventRecord(r.end, r.s));
    }
    // S7: the last nested iteration becomes sweep k+1 (swap buffer sets)
    first.restore();
    I->skip_final_ops = false;
    for (int p = 1; p <= M; ++p) std::swap(I->lev[0][p], I->lev[lv][p]);
    return MISDC_OK;
}

// Waits for all work of the integrator's streams.
int sync_streams(misdc_integ_s* I) {
    MISDC_HIP(hipStreamSynchronize(I->sD));
    if (I->sRm) MISDC_HIP(hipStreamSynchronize(I->sRm));
    MISDC_HIP(hipStreamSynchronize(I->sR2));
    for (hipStream_t s : I->lane_streams) MISDC_HIP(hipStreamSynchronize(s));
    return MISDC_OK;
}

// CG counters of the last step over every diffusion lane: [0] iterations,
// [1] max, [2] failed, [3] solves, [4] barrier timeouts
// (results of the tiled CG whose true residual failed its check count as
// failed solves)
int read_cgstats(misdc_integ_s* I, int32_t (&cg)[8]) {
    MISDC_HIP(hipMemcpy(cg, I->cgstats, sizeof(cg), hipMemcpyDeviceToHost));
    cg[2] += cg[5];
    if (I->pipe)
        for (auto& d : I->pd_lane) {
            int32_t l[8];
            MISDC_HIP(hipMemcpy(l, d.cgstats, sizeof(l), hipMemcpyDeviceToHost));
            cg[0] += l[0];
            cg[1] = l[1] > cg[1] ? l[1] : cg[1];
            cg[2] += l[2] + l[5];
            cg[3] += l[3];
            cg[4] += l[4];
        }
    return MISDC_OK;
}


// MISDC_ENOTCONV (with a message naming the counters) if the step whose
// counters are on the device left a Newton solve or a diffusion solve
// unconverged; the streams must be synchronised.
int convergence_status(misdc_integ_s* I) {
    unsigned long long ns[8];
    int32_t cg[8];
    MISDC_HIP(hipMemcpy(ns, I->nstats, sizeof(ns), hipMemcpyDeviceToHost));
    unsigned long long failed = ns[2];
    std::vector<unsigned long long> b((size_t)NEWTON_BUCKETS * NEWTON_BUCKET_STRIDE);
    MISDC_HIP(hipMemcpy(b.data(), I->nbuckets, sizeof(unsigned long long) * b.size(),
                        hipMemcpyDeviceToHost));
    for (int k = 0; k < NEWTON_BUCKETS; ++k) failed += b[(size_t)k * NEWTON_BUCKET_STRIDE + 2];
    if (int rc = read_cgstats(I, cg)) return rc;
    if (failed > 0 || cg[2] > 0 || cg[4] > 0)
        return fail(MISDC_ENOTCONV,
                    "unconverged solves in the last step: %llu cell-node Newton solves, "
                    "%d diffusion solves at their iteration limit, %d barrier timeouts",
                    failed, cg[2], cg[4]);
    if (I->cst.newton_failed > 0)
        return fail(MISDC_ENOTCONV, "unconverged solves in the last step: %lld coupled "
                                    "diffusion-reaction solves (IMEXQ)",
                    (long long)I->cst.newton_failed);
    return MISDC_OK;
}

// Validates the arguments of a step (also used by the autotuner).
int check_step_args(misdc_integ_s* I, const double* state, double dt, const double* dev_dt) {
    if (!I) return fail(MISDC_EINVAL, "integrator is NULL");
    if (!state) return fail(MISDC_EINVAL, "state is NULL");
    if (dev_dt) {
        if (I->grid->n_flames == 0)
            return fail(MISDC_EINVAL, "per-flame step sizes need an ensemble grid");
    } else if (!(dt > 0) || !std::isfinite(dt)) {
        return fail(MISDC_EINVAL, "dt must be positive and finite");
    }
    return MISDC_OK;
}

void drop_graph(misdc_integ_s* I) {
    if (I->gexec) (void)hipGraphExecDestroy(I->gexec);
    I->gexec = nullptr;
    I->g_state = nullptr;
    I->g_dtf = nullptr;
    I->g_dt = 0.0;
}

// Issues one step on the integrator's streams.  sD is the origin: the
// reaction stream forks from it at the start and joins it at the end, so the
// whole step can be captured from sD into one graph.  Only kernels, event
// records and event waits are issued (no memset or memcpy nodes).
// I1-I4 of a step: the reaction stream forks from sD, the counters are
// cleared (the Newton histograms of zero_sweeps sweeps), every node of sweep 0
// receives phi^n and F(phi^n).  Returns the dt that the sweeps take (1 with
// per-flame step sizes, whose terms are scaled per cell).
int issue_begin(misdc_integ_s* I, double* state, double dt, const double* dtf, int zero_sweeps,
                double& dt_sweep) {
    const int M = I->M, N = I->N, NF = I->NF;
    const int64_t n = I->n;
    int rc;
    if (I->sR != I->sD || I->pipe) {
        MISDC_HIP(hipEventRecord(I->ev_fork, I->sD));
        if (I->sR != I->sD) MISDC_HIP(hipStreamWaitEvent(I->sR, I->ev_fork, 0));
        for (hipStream_t s : I->lane_streams) MISDC_HIP(hipStreamWaitEvent(s, I->ev_fork, 0));
    }
    I->s_last = I->sR;
    I->consts_ready = I->d1_split = I->const_on_r = I->prep_newton = false;
    I->dfr = misdc_integ_s::Deferred();
    I->dtf = dtf;
    I->dtc = nullptr;
    if (dtf) {
        if ((rc = launch_expand_flames(*I->grid, dtf, I->dt_cell, I->sD))) return rc;
        I->dtc = I->dt_cell;
        dt = 1.0;      // every dt-carrying term takes dtc[cell] (or dtf[flame])
    }
    {
        void* const dst[4] = {I->nstats, I->nbuckets, I->nhist, I->cgstats};
        const int64_t bytes[4] = {
            (int64_t)(8 * sizeof(unsigned long long)),
            (int64_t)(sizeof(unsigned long long) * NEWTON_BUCKETS * NEWTON_BUCKET_STRIDE),
            (int64_t)(sizeof(unsigned long long) * zero_sweeps * NEWTON_HIST_SETS *
                      NEWTON_HIST_BINS),
            (int64_t)(8 * sizeof(int32_t))};
        // on the reaction stream when there is one: every task of the step
        // follows its F_R pass below
        if ((rc = launch_zero_many(dst, bytes, 4, I->sR))) return rc;
    }
    I->cst = CoupledStats();
    if (I->pipe)
        for (auto& d : I->pd_lane)
            if ((rc = launch_zero(d.cgstats, 8 * sizeof(int32_t), I->sD))) return rc;
    // I1, I2, I4: node 0 holds phi^n (copied in T's pass) and F(phi^n); every
    // other node of sweep 0 holds the same, which sweep 0 reads from node 0's
    // buffers (FirstSweepNodes), so nothing is copied to them
    NodeBuf& b0 = I->lev[0][0];
    if (I->sR != I->sD) {
        // F_R on the reaction stream, from the state itself (the source forms
        // T from h), while node 0's copy, T, F_A and F_D are formed
        rc = launch_reaction_source(*I->mech, n, state, state + (size_t)N * n, b0.FR, I->sR);
        if (rc) return rc;
        MISDC_HIP(hipEventRecord(I->ev_source, I->sR));
        if ((rc = launch_state_temperature(*I->mech, n, state, b0.T, I->sD, b0.phi))) return rc;
        if ((rc = eval_ops(I, b0, I->thD, I->sD, false))) return rc;
        MISDC_HIP(hipStreamWaitEvent(I->sD, I->ev_source, 0));
    } else {
        if ((rc = launch_state_temperature(*I->mech, n, state, b0.T, I->sD, b0.phi))) return rc;
        if ((rc = eval_ops(I, b0, I->thD, I->sD, true))) return rc;
    }
    (void)N;
    (void)NF;
    // node 0 is shared by every nested-iteration level
    for (int l = 1; l < I->levels; ++l) I->lev[l][0] = b0;
    // "previous sweep finished" marker for the first sweep's constants
    MISDC_HIP(hipEventRecord(I->R_ev(0, M), I->sD));
    dt_sweep = dt;
    return MISDC_OK;
}

// The end of a step: node M of the last sweep back into the state, and the
// reaction stream joins sD.
int issue_end(misdc_integ_s* I, double* state) {
    int rc = flush_deferred(I, nullptr);
    if (rc) return rc;
    const hipStream_t se = I->s_last;         // after the last reaction task
    if ((rc = launch_copy(state, I->lev[0][I->M].phi, (int64_t)I->NF * I->n, se))) return rc;
    if (se != I->sD) {
        MISDC_HIP(hipEventRecord(I->ev_join, se));
        MISDC_HIP(hipStreamWaitEvent(I->sD, I->ev_join, 0));
    }
    if (I->sR != I->sD && I->sR != se) {
        MISDC_HIP(hipEventRecord(I->ev_outR, I->sR));
        MISDC_HIP(hipStreamWaitEvent(I->sD, I->ev_outR, 0));
    }
    if (I->pipe) {
        // every lane joins the origin stream (their end events of the last sweep)
        for (auto& d : I->pd_lane) MISDC_HIP(hipStreamWaitEvent(I->sD, d.end, 0));
        for (auto& r : I->pr_lane) MISDC_HIP(hipStreamWaitEvent(I->sD, r.end, 0));
    }
    return MISDC_OK;
}

int issue_step(misdc_integ_s* I, double* state, double dt, const double* dtf) {
    double dts = dt;
    int rc = issue_begin(I, state, dt, dtf, I->opt.n_sweeps, dts);
    if (rc) return rc;
    for (int k = 0; k < I->opt.n_sweeps; ++k) {
        I->sweep_index = k;
        if ((rc = run_sweep(I, k, dts, k + 1 < I->opt.n_sweeps, true))) return rc;
    }
    return issue_end(I, state);
}

}  // namespace

extern "C" {

const char* misdc_last_error(void) { return g_err; }

const char* misdc_version(void) { return "misdc-mi355x 0.1 (gfx950)"; }

}  // extern "C"

namespace {

// Host tables of a validated mechanism descriptor (those the generated
// reaction solve is written from).
void mech_tables(const misdc_mech_desc* d, MechTables& t) {
    const int N = d->n_species, R = d->n_reactions;
    t.N = N;
    t.R = R;
    t.bath = d->bath;
    t.slots.assign(4 * (size_t)R, -1);
    t.Ta.assign(R, 0.0);
    t.dn.assign(R, 0.0);
    t.uW.assign((size_t)R * N, 0.0);
    for (int j = 0; j < R; ++j) {
        for (int s = 0; s < 2; ++s) {
            t.slots[4 * j + s] = d->react[2 * j + s];
            t.slots[4 * j + 2 + s] = d->prod[2 * j + s];
            if (d->react[2 * j + s] >= 0) {
                t.uW[(size_t)j * N + d->react[2 * j + s]] -= d->W[d->react[2 * j + s]] / d->rho0;
                t.dn[j] -= 1;
            }
            if (d->prod[2 * j + s] >= 0) {
                t.uW[(size_t)j * N + d->prod[2 * j + s]] += d->W[d->prod[2 * j + s]] / d->rho0;
                t.dn[j] += 1;
            }
        }
        t.Ta[j] = d->Ea[j] / d->R_c;
    }
    t.A.assign(d->A, d->A + R);
    t.beta.assign(d->beta, d->beta + R);
    t.W.assign(d->W, d->W + N);
    t.invW.resize(N);
    double scale = 0;
    for (int k = 0; k < N; ++k) {
        t.invW[k] = 1.0 / d->W[k];
        scale += d->cp[k] / d->W[k];
    }
    t.cp.assign(d->cp, d->cp + N);
    t.hf.assign(d->hf, d->hf + N);
    t.s0.assign(d->s0, d->s0 + N);
    t.rho0 = d->rho0;
    t.R_u = d->R_u;
    t.newton_scale = scale / N;
    t.ln_patm_over_Ru = std::log(d->p_atm / d->R_u);
}

}  // namespace

extern "C" {

int misdc_mech_generate(const misdc_mech_desc* d, int compile, char* buf, size_t* len) {
    if (!len) return fail(MISDC_EINVAL, "len is NULL");
    int rc = check_mech_desc(d);
    if (rc) return rc;
    if (d->n_species > NEWTON_SPEC_MAX_SPECIES)
        return fail(MISDC_EUNSUPPORTED, "the generated reaction solve holds at most %d species",
                    NEWTON_SPEC_MAX_SPECIES);
    MechTables t;
    mech_tables(d, t);
    const std::string src = newton_spec_source(t);
    if (compile) {
        std::string msg;
        if (newton_spec_compile_check(src, msg) != 0)
            return fail(MISDC_EDEVICE, "generated reaction solve does not compile: %s", msg.c_str());
    }
    const size_t need = src.size() + 1;
    if (buf && *len >= need) std::memcpy(buf, src.c_str(), need);
    const bool fits = buf && *len >= need;
    *len = need;
    if (buf && !fits) return fail(MISDC_EINVAL, "buffer of %zu bytes, %zu needed", *len, need);
    return MISDC_OK;
}

int misdc_mech_create(const misdc_mech_desc* d, misdc_mech_t* out) {
    if (!out) return fail(MISDC_EINVAL, "output handle pointer is NULL");
    *out = nullptr;
    int rc = check_mech_desc(d);
    if (rc) return rc;
    const int N = d->n_species, R = d->n_reactions;
    auto* h = new (std::nothrow) misdc_mech_s();
    if (!h) return fail(MISDC_ENOMEM, "host allocation failed");
    Mech& m = h->m;
    // host-side table construction
    std::vector<int> slots(4 * (size_t)R);
    std::vector<double> Ta(R), dn(R), uW((size_t)R * N, 0.0), invW(N), kappa0(N + 1);
    for (int j = 0; j < R; ++j) {
        slots[4 * j + 0] = d->react[2 * j];
        slots[4 * j + 1] = d->react[2 * j + 1];
        slots[4 * j + 2] = d->prod[2 * j];
        slots[4 * j + 3] = d->prod[2 * j + 1];
        Ta[j] = d->Ea[j] / d->R_c;
        double net = 0;
        for (int s = 0; s < 2; ++s) {
            if (d->react[2 * j + s] >= 0) {
                uW[(size_t)j * N + d->react[2 * j + s]] -= d->W[d->react[2 * j + s]] / d->rho0;
                net -= 1;
            }
            if (d->prod[2 * j + s] >= 0) {
                uW[(size_t)j * N + d->prod[2 * j + s]] += d->W[d->prod[2 * j + s]] / d->rho0;
                net += 1;
            }
        }
        dn[j] = net;
    }
    double scale = 0;
    for (int k = 0; k < N; ++k) {
        invW[k] = 1.0 / d->W[k];
        scale += d->cp[k] / d->W[k];
        kappa0[k] = d->D0[k];
    }
    kappa0[N] = d->alpha0;
    scale /= N;
    // per-species reaction lists for the wavefront-per-cell kernels
    std::vector<int> rowp(N + 1, 0), rowj;
    std::vector<double> rowu;
    for (int k = 0; k < N; ++k) {
        for (int j = 0; j < R; ++j) {
            const double u = uW[(size_t)j * N + k];
            if (u != 0.0) {
                rowj.push_back(j);
                rowu.push_back(u);
            }
        }
        rowp[k + 1] = (int)rowj.size();
    }
    const size_t nnz = rowj.size();
    const int nch = (R + 63) / 64;
    std::vector<int> rowl(4 * nnz), rowc((size_t)N * (nch + 1));
    for (size_t e = 0; e < nnz; ++e)
        for (int s = 0; s < 4; ++s) rowl[4 * e + s] = slots[4 * (size_t)rowj[e] + s];
    for (int k = 0; k < N; ++k)
        for (int c = 0; c <= nch; ++c) {
            int e = rowp[k];
            while (e < rowp[k + 1] && rowj[e] < 64 * c) ++e;
            rowc[(size_t)k * (nch + 1) + c] = e;
        }
    // one device block: doubles then ints
    const size_t nd = (size_t)R * 5 + (size_t)R * N + (size_t)N * 6 + (N + 1) + nnz;
    const size_t nints = slots.size() + rowp.size() + nnz + rowl.size() + rowc.size();
    const size_t bytes = nd * sizeof(double) + nints * sizeof(int) + 64;
    hipError_t e = hipGetDevice(&m.device);
    if (e != hipSuccess) {
        delete h;
        return fail(MISDC_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    e = hipMalloc(&m.block, bytes);
    if (e != hipSuccess) {
        delete h;
        return fail(MISDC_ENOMEM, "hipMalloc(mechanism): %s", hipGetErrorString(e));
    }
    std::vector<char> host(bytes, 0);
    double* dp = (double*)host.data();
    size_t off = 0;
    auto put = [&](const double* src, size_t cnt) {
        const size_t at = off;
        if (cnt) std::memcpy(dp + off, src, cnt * sizeof(double));
        off += cnt;
        return at;
    };
    const size_t oA = put(d->A, R), ob = put(d->beta, R), oT = put(Ta.data(), R),
                 odn = put(dn.data(), R), ouW = put(uW.data(), uW.size()),
                 oW = put(d->W, N), oiW = put(invW.data(), N), ocp = put(d->cp, N),
                 ohf = put(d->hf, N), os0 = put(d->s0, N), ok0 = put(kappa0.data(), N + 1),
                 oru = put(rowu.data(), nnz);
    off += R;   // spare
    int* ip = (int*)(dp + off);
    if (!slots.empty()) std::memcpy(ip, slots.data(), slots.size() * sizeof(int));
    std::memcpy(ip + slots.size(), rowp.data(), rowp.size() * sizeof(int));
    if (nnz) std::memcpy(ip + slots.size() + rowp.size(), rowj.data(), nnz * sizeof(int));
    if (nnz) std::memcpy(ip + slots.size() + rowp.size() + nnz, rowl.data(), rowl.size() * sizeof(int));
    std::memcpy(ip + slots.size() + rowp.size() + nnz + rowl.size(), rowc.data(),
                rowc.size() * sizeof(int));
    e = hipMemcpy(m.block, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(m.block);
        delete h;
        return fail(MISDC_EDEVICE, "hipMemcpy(mechanism): %s", hipGetErrorString(e));
    }
    const double* base = (const double*)m.block;
    MechDev& md = m.dev;
    md.N = N;
    md.R = R;
    md.bath = d->bath;
    md.rho0 = d->rho0;
    md.p_atm = d->p_atm;
    md.R_u = d->R_u;
    md.R_c = d->R_c;
    md.alpha0 = d->alpha0;
    md.newton_scale = scale;
    md.ln_patm_over_Ru = std::log(d->p_atm / d->R_u);
    md.slots = (const int*)(base + off);
    md.A = base + oA;
    md.beta = base + ob;
    md.Ta = base + oT;
    md.dn = base + odn;
    md.uW = base + ouW;
    md.W = base + oW;
    md.invW = base + oiW;
    md.cp = base + ocp;
    md.hf = base + ohf;
    md.s0 = base + os0;
    md.kappa0 = base + ok0;
    md.rowu = base + oru;
    md.rowp = md.slots + slots.size();
    md.rowj = md.rowp + rowp.size();
    md.rowl = md.rowj + nnz;
    md.rowc = md.rowl + rowl.size();
    md.nch = nch;
    m.W.assign(d->W, d->W + N);
    m.cp.assign(d->cp, d->cp + N);
    m.hf.assign(d->hf, d->hf + N);
    m.kappa0 = kappa0;
    // the reaction solve generated for this mechanism (the generic kernels
    // serve where it cannot be built)
    MechTables t;
    mech_tables(d, t);
    (void)newton_spec_prepare(m, t);
    *out = h;
    return MISDC_OK;
}

int misdc_mech_specialized(misdc_mech_t mech, int32_t* available, const char** status) {
    if (!mech || !available) return fail(MISDC_EINVAL, "NULL argument");
    *available = mech->m.spec_fn ? 1 : 0;
    if (status) *status = mech->m.spec_status.c_str();
    return MISDC_OK;
}

int misdc_mech_destroy(misdc_mech_t mech) {
    if (!mech) return MISDC_OK;
    if (mech->m.block) (void)hipFree(mech->m.block);
    delete mech;
    return MISDC_OK;
}

int misdc_mech_species(misdc_mech_t mech, int32_t* n_species) {
    if (!mech || !n_species) return fail(MISDC_EINVAL, "NULL argument");
    *n_species = mech->m.dev.N;
    return MISDC_OK;
}

int misdc_enthalpy(misdc_mech_t mech, int64_t n, const double* Y, const double* T, double* h,
                   void* stream) {
    if (!mech) return fail(MISDC_EINVAL, "mechanism is NULL");
    if (n < 0) return fail(MISDC_EINVAL, "n < 0");
    if (n > 0 && (!Y || !T || !h)) return fail(MISDC_EINVAL, "NULL array");
    return launch_enthalpy(mech->m, n, Y, T, h, (hipStream_t)stream);
}

int misdc_temperature(misdc_mech_t mech, int64_t n, const double* Y, const double* h, double* T,
                      void* stream) {
    if (!mech) return fail(MISDC_EINVAL, "mechanism is NULL");
    if (n < 0) return fail(MISDC_EINVAL, "n < 0");
    if (n > 0 && (!Y || !T || !h)) return fail(MISDC_EINVAL, "NULL array");
    return launch_temperature(mech->m, n, Y, h, T, (hipStream_t)stream);
}

int misdc_reaction_source(misdc_mech_t mech, int64_t n, const double* Y, const double* h,
                          double* FR, void* stream) {
    if (!mech) return fail(MISDC_EINVAL, "mechanism is NULL");
    if (n < 0) return fail(MISDC_EINVAL, "n < 0");
    if (n > 0 && (!Y || !FR || !h)) return fail(MISDC_EINVAL, "NULL array");
    return launch_reaction_source(mech->m, n, Y, h, FR, (hipStream_t)stream);
}

int misdc_reaction_solve_batch(misdc_mech_t mech, int64_t n, const double* bY, const double* h,
                               const double* c, double* Y, double* T_out, double* FR_out,
                               int32_t* iters_out, const misdc_newton_opts* opts, void* stream) {
    if (!mech) return fail(MISDC_EINVAL, "mechanism is NULL");
    if (n < 0) return fail(MISDC_EINVAL, "n < 0");
    if (n == 0) return MISDC_OK;
    if (!bY || !h || !c || !Y || !iters_out) return fail(MISDC_EINVAL, "NULL array");
    NewtonArgs a;
    a.n = n;
    a.bY = bY;
    a.ldb = n;
    a.h = h;
    a.c = c;
    a.c_scalar = 1.0;
    a.guess = Y;
    a.ldg = n;
    a.Y = Y;
    a.ldy = n;
    a.T = T_out;
    a.FR = FR_out;
    a.ldf = n;
    a.iters = iters_out;
    a.stats = nullptr;
    a.opt = newton_defaults(opts);
    return launch_reaction_newton(mech->m, a, (hipStream_t)stream);
}

int misdc_grid_create(int dim, const int64_t* n, const double* dx, const double* u,
                      misdc_grid_t* out) {
    if (!out) return fail(MISDC_EINVAL, "output handle pointer is NULL");
    *out = nullptr;
    if (dim != 1 && dim != 2) return fail(MISDC_EINVAL, "dim must be 1 or 2, got %d", dim);
    if (!n || !dx || !u) return fail(MISDC_EINVAL, "NULL array");
    for (int d = 0; d < dim; ++d) {
        if (n[d] < 4 || n[d] > (int64_t)1 << 30)
            return fail(MISDC_EINVAL, "n[%d] must be in [4, 2^30], got %lld", d, (long long)n[d]);
        if (!(dx[d] > 0) || !std::isfinite(dx[d]) || !std::isfinite(u[d]))
            return fail(MISDC_EINVAL, "dx[%d] must be positive and u finite", d);
    }
    auto* h = new (std::nothrow) misdc_grid_s();
    if (!h) return fail(MISDC_ENOMEM, "host allocation failed");
    Grid& g = h->g;
    g.dim = dim;
    g.nx = n[0];
    g.ny = dim == 2 ? n[1] : 1;
    g.dx = dx[0];
    g.dy = dim == 2 ? dx[1] : 0.0;
    g.ux = u[0];
    g.uy = dim == 2 ? u[1] : 0.0;
    if (g.nx * g.ny > ((int64_t)1 << 31)) {
        delete h;
        return fail(MISDC_EINVAL, "grid too large");
    }
    *out = h;
    return MISDC_OK;
}

int misdc_grid_create_ensemble(int n_flames, const int64_t* lengths, const double* dx,
                               const double* u, misdc_grid_t* out) {
    if (!out) return fail(MISDC_EINVAL, "output handle pointer is NULL");
    *out = nullptr;
    if (n_flames < 1 || n_flames > 65536) return fail(MISDC_EINVAL, "n_flames out of range");
    if (!lengths || !dx || !u) return fail(MISDC_EINVAL, "NULL array");
    auto* h = new (std::nothrow) misdc_grid_s();
    if (!h) return fail(MISDC_ENOMEM, "host allocation failed");
    Grid& g = h->g;
    g.dim = 1;
    g.n_flames = n_flames;
    g.off.assign(n_flames + 1, 0);
    for (int f = 0; f < n_flames; ++f) {
        if (lengths[f] < 4 || !(dx[f] > 0) || !std::isfinite(u[f])) {
            delete h;
            return fail(MISDC_EINVAL, "flame %d: length >= 4, dx > 0 required", f);
        }
        g.off[f + 1] = g.off[f] + lengths[f];
    }
    g.len.assign(lengths, lengths + n_flames);
    g.fdx.assign(dx, dx + n_flames);
    g.fu.assign(u, u + n_flames);
    g.nx = g.off.back();
    g.ny = 1;
    hipError_t e = hipMalloc(&g.d_off, sizeof(int64_t) * (n_flames + 1));
    if (e == hipSuccess) e = hipMalloc(&g.d_dx, sizeof(double) * n_flames);
    if (e == hipSuccess) e = hipMalloc(&g.d_u, sizeof(double) * n_flames);
    if (e == hipSuccess)
        e = hipMemcpy(g.d_off, g.off.data(), sizeof(int64_t) * (n_flames + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g.d_dx, dx, sizeof(double) * n_flames, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(g.d_u, u, sizeof(double) * n_flames, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        misdc_grid_destroy(h);
        return fail(MISDC_EDEVICE, "ensemble grid: %s", hipGetErrorString(e));
    }
    *out = h;
    return MISDC_OK;
}

int misdc_grid_destroy(misdc_grid_t grid) {
    if (!grid) return MISDC_OK;
    if (grid->g.d_off) (void)hipFree(grid->g.d_off);
    if (grid->g.d_dx) (void)hipFree(grid->g.d_dx);
    if (grid->g.d_u) (void)hipFree(grid->g.d_u);
    delete grid;
    return MISDC_OK;
}

int misdc_grid_cells(misdc_grid_t grid, int64_t* n_cells) {
    if (!grid || !n_cells) return fail(MISDC_EINVAL, "NULL argument");
    *n_cells = grid->g.cells();
    return MISDC_OK;
}

int misdc_transport_operators(misdc_mech_t mech, misdc_grid_t grid, const double* state,
                              double* FA, double* FD, void* stream) {
    if (!mech || !grid) return fail(MISDC_EINVAL, "NULL handle");
    if (!state) return fail(MISDC_EINVAL, "state is NULL");
    const int64_t n = grid->g.cells();
    hipStream_t s = (hipStream_t)stream;
    double* T = nullptr;
    double* th = nullptr;
    MISDC_HIP(hipMallocAsync((void**)&T, sizeof(double) * n, s));
    MISDC_HIP(hipMallocAsync((void**)&th, sizeof(double) * n, s));
    int rc = launch_state_temperature(mech->m, n, state, T, s);
    if (!rc) rc = launch_transport(mech->m, grid->g, state, T, FA, FD, th, s);
    (void)hipFreeAsync(T, s);
    (void)hipFreeAsync(th, s);
    return rc;
}

int misdc_diffusion_solve(misdc_mech_t mech, misdc_grid_t grid, double c, const double* T_lag,
                          const double* rhs, double* y, int guess_in_y, double rtol, int maxit,
                          int32_t* iters_out, void* stream) {
    if (!mech || !grid) return fail(MISDC_EINVAL, "NULL handle");
    if (!T_lag || !rhs || !y) return fail(MISDC_EINVAL, "NULL array");
    if (rhs == y) return fail(MISDC_EINVAL, "rhs and y must not alias");
    if (!(c >= 0) || !std::isfinite(c)) return fail(MISDC_EINVAL, "c must be >= 0 and finite");
    hipStream_t s = (hipStream_t)stream;
    DiffusionWork w;
    int rc = diffusion_work_alloc(w, mech->m, grid->g);
    if (rc) {
        diffusion_work_free(w);
        return rc;
    }
    rc = launch_diffusion_solve(mech->m, grid->g, w, c, nullptr, 0.0, T_lag, rhs, y, guess_in_y,
                                rtol, maxit, s);
    if (!rc && iters_out) {
        hipError_t e = hipMemcpyAsync(iters_out, w.info, sizeof(int32_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) rc = fail(MISDC_EDEVICE, "copy iterations: %s", hipGetErrorString(e));
    }
    // the work buffers must outlive the kernels: wait before freeing
    hipError_t e = hipStreamSynchronize(s);
    diffusion_work_free(w);
    if (!rc && e != hipSuccess) rc = fail(MISDC_EDEVICE, "synchronise: %s", hipGetErrorString(e));
    return rc;
}

}  // extern "C"

namespace {

// Device scratch of the diffusion solve that allocates nothing: the CG
// vectors, face coefficients, block partials, halo edges, barrier counters
// and iteration record of one call (each GPU the library runs on holds its
// own copy until the process ends).  Host code never uses the array's name
// as an address: each device's address comes from hipGetSymbolAddress.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)MISDC_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Address of the current device's scratch, looked up on the first call on
// that device (with it current) and kept.
int scratch_address(void** out) {
    int dev = 0;
    MISDC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(MISDC_EUNSUPPORTED, "device %d beyond the %d the scratch table holds", dev,
                    NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MISDC_EDEVICE, "address of the diffusion scratch on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MISDC_OK;
}

__global__ void copy_word_kernel(int32_t* dst, const int32_t* src) { *dst = *src; }

}  // namespace

extern "C" {

int misdc_diffusion_solve_noalloc(misdc_mech_t mech, misdc_grid_t grid, double c,
                                  const double* T_lag, const double* rhs, double* y,
                                  int guess_in_y, double rtol, int maxit, int32_t* iters_out,
                                  void* stream) {
    if (!mech || !grid) return fail(MISDC_EINVAL, "NULL handle");
    if (!T_lag || !rhs || !y) return fail(MISDC_EINVAL, "NULL array");
    if (rhs == y) return fail(MISDC_EINVAL, "rhs and y must not alias");
    if (!(c >= 0) || !std::isfinite(c)) return fail(MISDC_EINVAL, "c must be >= 0 and finite");
    const size_t need = diffusion_work_bytes(mech->m, grid->g);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(MISDC_EINVAL,
                    "the solve needs %zu bytes of scratch; the no-allocation entry point holds "
                    "%zu (%d MiB): use misdc_diffusion_solve for this grid",
                    need, NOALLOC_SCRATCH_BYTES, MISDC_NOALLOC_SCRATCH_MIB);
    void* block = nullptr;
    int rc = scratch_address(&block);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    DiffusionWork w;
    if ((rc = diffusion_work_carve(w, mech->m, grid->g, block, NOALLOC_SCRATCH_BYTES, s))) return rc;
    rc = launch_diffusion_solve(mech->m, grid->g, w, c, nullptr, 0.0, T_lag, rhs, y, guess_in_y,
                                rtol, maxit, s);
    if (rc) return rc;
    if (iters_out) {
        hipLaunchKernelGGL(copy_word_kernel, dim3(1), dim3(1), 0, s, iters_out,
                           (const int32_t*)w.info);
        MISDC_HIP(hipGetLastError());
    }
    return MISDC_OK;
}

void misdc_opts_default(misdc_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n_nodes = 5;
    o->n_sweeps = 6;
    o->nu = 1;
    o->scheme = MISDC_SCHEME_CISDCQ;
    o->qe_mode = MISDC_QE_CUMULATIVE;
    o->serialize = 0;
    o->newton = newton_defaults(nullptr);
    o->cg_rtol = 1e-13;
    o->cg_maxit = 500;
    o->profile = 0;
    o->use_graph = 0;
    o->nu_tol = 0.0;
}

int misdc_integ_destroy(misdc_integ_t I);

}  // extern "C"

namespace {

// CU mask of one half of every XCD's CUs (half 0 or 1): bit i is set when
// (i / 8) mod 4 falls in that half, as for the reaction stream's CU split
int half_mask_stream(int half, hipStream_t* out) {
    int cus = 0;
    int rc = device_cus(cus);
    if (rc) return rc;
    if (cus < 32 || cus % 32)
        return fail(MISDC_EUNSUPPORTED, "pipelined passes need a multiple of 32 CUs (device has %d)",
                    cus);
    const size_t words = (size_t)cus / 32;
    std::vector<uint32_t> mask(words, 0u), back(words, 0u);
    for (int i = 0; i < cus; ++i)
        if (((i / 8) % 4) / 2 == half) mask[(size_t)i / 32] |= 1u << (i % 32);
    hipStream_t s = nullptr;
    MISDC_HIP(hipExtStreamCreateWithCUMask(&s, (uint32_t)words, mask.data()));
    hipError_t e = hipExtStreamGetCUMask(s, (uint32_t)words, back.data());
    if (e != hipSuccess || back != mask) {
        (void)hipStreamDestroy(s);
        return fail(MISDC_EDEVICE, "CU mask of a diffusion lane not applied");
    }
    *out = s;
    return MISDC_OK;
}

// The lanes of pipelined passes: two diffusion lanes on the two CU halves
// (their persistent solves must each hold all of their workgroups at once, so
// each needs CUs the other does not take) and one reaction lane per pass.
int create_lanes(misdc_integ_s* I) {
    const int64_t n = I->n;
    const int NF = I->NF, N = I->N;
    int cus = 0;
    int rc = device_cus(cus);
    if (rc) return rc;
    I->pipe = true;
    for (int h = 0; h < 2; ++h) {
        auto& d = I->pd_lane[h];
        if ((rc = half_mask_stream(h, &d.s))) return rc;
        I->lane_streams.push_back(d.s);
        if ((rc = dalloc(I, &d.rD, (size_t)NF * n))) return rc;
        if ((rc = dalloc(I, &d.th, (size_t)n))) return rc;
        if ((rc = dalloc(I, &d.cgstats, 8))) return rc;
        if ((rc = diffusion_work_alloc(I->pdw[h], *I->mech, *I->grid))) return rc;
        if (I->pdw[h].blocks > cus / 2)
            return fail(MISDC_EUNSUPPORTED,
                        "pipelined passes: the diffusion solve takes %d workgroups, more than "
                        "the %d CUs of a lane", I->pdw[h].blocks, cus / 2);
        d.dw = &I->pdw[h];
        MISDC_HIP(hipEventCreateWithFlags(&d.end, hipEventDisableTiming));
    }
    I->pr_lane.assign((size_t)I->nu, misdc_integ_s::RLane());
    for (auto& r : I->pr_lane) {
        MISDC_HIP(hipStreamCreateWithFlags(&r.s, hipStreamNonBlocking));
        I->lane_streams.push_back(r.s);
        if ((rc = dalloc(I, &r.bR, (size_t)N * n))) return rc;
        if ((rc = dalloc(I, &r.th, (size_t)n))) return rc;
        if ((rc = dalloc(I, &r.iters, (size_t)n))) return rc;
        if ((rc = dalloc(I, &r.lu_info, (size_t)n))) return rc;
        MISDC_HIP(hipEventCreateWithFlags(&r.end, hipEventDisableTiming));
    }
    I->stagger = 0;
    return MISDC_OK;
}

}  // namespace

extern "C" {

int misdc_integ_create(misdc_mech_t mech, misdc_grid_t grid, const misdc_opts* opts,
                       misdc_integ_t* out) {
    if (!out) return fail(MISDC_EINVAL, "output handle pointer is NULL");
    *out = nullptr;
    if (!mech || !grid) return fail(MISDC_EINVAL, "NULL handle");
    int rc = check_opts(opts);
    if (rc) return rc;
    if (mech->m.dev.N > 63)
        return fail(MISDC_EUNSUPPORTED, "integrator built for at most 63 species, mechanism has %d",
                    mech->m.dev.N);
    auto* I = new (std::nothrow) misdc_integ_s();
    if (!I) return fail(MISDC_ENOMEM, "host allocation failed");
    I->mech = &mech->m;
    I->grid = &grid->g;
    I->opt = *opts;
    I->opt.newton = newton_defaults(&opts->newton);
    if (!(I->opt.cg_rtol > 0)) I->opt.cg_rtol = 1e-13;
    if (I->opt.cg_maxit <= 0) I->opt.cg_maxit = 500;
    rc = make_tables(opts->n_nodes, opts->scheme == MISDC_SCHEME_MISDC ? MISDC_QI_BE : MISDC_QI_LU,
                     opts->qe_mode, I->tab);
    if (rc) {
        delete I;
        return rc;
    }
    I->M = opts->n_nodes - 1;
    I->N = mech->m.dev.N;
    I->NF = I->N + 1;
    I->n = grid->g.cells();
    I->nu = opts->scheme == MISDC_SCHEME_CISDCQ ? opts->nu : 1;
    I->levels = I->nu + 1;
    const int M = I->M, N = I->N, NF = I->NF;
    const int64_t n = I->n;
    auto bail = [&](int code) {
        misdc_integ_destroy(I);
        return code;
    };
    I->lev.assign(I->levels, std::vector<NodeBuf>(M + 1));
    for (int l = 0; l < I->levels; ++l)
        for (int p = 0; p <= M; ++p) {
            NodeBuf& b = I->lev[l][p];
            if ((rc = dalloc(I, &b.phi, (size_t)NF * n))) return bail(rc);
            if ((rc = dalloc(I, &b.T, (size_t)n))) return bail(rc);
            if ((rc = dalloc(I, &b.FA, (size_t)NF * n))) return bail(rc);
            if ((rc = dalloc(I, &b.FD, (size_t)NF * n))) return bail(rc);
            if ((rc = dalloc(I, &b.FR, (size_t)N * n))) return bail(rc);
        }
    I->phiAD.assign(M + 1, nullptr);
    I->TAD.assign(M + 1, nullptr);
    I->hatA.assign(M + 1, nullptr);
    I->hatD.assign(M + 1, nullptr);
    I->C.assign(M + 1, nullptr);
    I->CR.assign(M + 1, nullptr);
    for (int p = 1; p <= M; ++p) {
        if ((rc = dalloc(I, &I->phiAD[p], (size_t)NF * n))) return bail(rc);
        if ((rc = dalloc(I, &I->TAD[p], (size_t)n))) return bail(rc);
        if ((rc = dalloc(I, &I->hatA[p], (size_t)NF * n))) return bail(rc);
        if ((rc = dalloc(I, &I->hatD[p], (size_t)NF * n))) return bail(rc);
        if ((rc = dalloc(I, &I->C[p], (size_t)NF * n))) return bail(rc);
        if ((rc = dalloc(I, &I->CR[p], (size_t)N * n))) return bail(rc);
    }
    if ((rc = dalloc(I, &I->rD, (size_t)NF * n))) return bail(rc);
    if (opts->scheme == MISDC_SCHEME_CISDCQ && M >= 2) {
        for (auto& r : I->rP)
            if ((rc = dalloc(I, &r, (size_t)NF * n))) return bail(rc);
        if ((rc = dalloc(I, &I->thM, (size_t)n))) return bail(rc);
    }
    I->lagw.assign(M + 1, LagRhs());
    if ((rc = dalloc(I, &I->bR, (size_t)N * n))) return bail(rc);
    if ((rc = dalloc(I, &I->thD, (size_t)n))) return bail(rc);
    if ((rc = dalloc(I, &I->thR, (size_t)n))) return bail(rc);
    if ((rc = dalloc(I, &I->iters, (size_t)n))) return bail(rc);
    if ((rc = dalloc(I, &I->nstats, 8))) return bail(rc);
    if ((rc = dalloc(I, &I->nbuckets, (size_t)NEWTON_BUCKETS * NEWTON_BUCKET_STRIDE))) return bail(rc);
    if (hipMemset(I->nbuckets, 0, sizeof(unsigned long long) * NEWTON_BUCKETS * NEWTON_BUCKET_STRIDE) !=
        hipSuccess)
        return bail(fail(MISDC_EDEVICE, "clear the Newton counters"));
    if ((rc = dalloc(I, &I->nhist, (size_t)64 * NEWTON_HIST_SETS * NEWTON_HIST_BINS))) return bail(rc);
    if (hipMemset(I->nhist, 0, sizeof(unsigned long long) * 64 * NEWTON_HIST_SETS * NEWTON_HIST_BINS) !=
        hipSuccess)
        return bail(fail(MISDC_EDEVICE, "clear the Newton histograms"));
    if ((rc = dalloc(I, &I->lu_info, (size_t)n))) return bail(rc);
    if ((rc = dalloc(I, &I->choice, (size_t)n))) return bail(rc);
    if ((rc = dalloc(I, &I->cbuf, (size_t)n))) return bail(rc);
    if ((rc = dalloc(I, &I->cgstats, 8))) return bail(rc);
    if ((rc = dalloc(I, &I->inc, (size_t)64 * NF * 2))) return bail(rc);
    if ((rc = dalloc(I, &I->pinc, (size_t)16 * NF * 2))) return bail(rc);
    if (hipHostMalloc((void**)&I->pinc_host, sizeof(double) * 16 * NF * 2, hipHostMallocDefault) !=
        hipSuccess) {
        I->pinc_host = nullptr;
        return bail(fail(MISDC_ENOMEM, "pinned host buffer"));
    }
    // partials, then the arrival counter of the reduction (zero between uses)
    if ((rc = dalloc(I, &I->inc_partial, (size_t)I->inc_blocks * NF * 2 + 8))) return bail(rc);
    if (hipMemset(I->inc_partial, 0, sizeof(double) * ((size_t)I->inc_blocks * NF * 2 + 8)) !=
        hipSuccess)
        return bail(fail(MISDC_EDEVICE, "clear the reduction partials"));
    if ((rc = diffusion_work_alloc(I->dw, mech->m, grid->g))) return bail(rc);
    if (grid->g.n_flames > 0 && (rc = dalloc(I, &I->dt_cell, (size_t)n))) return bail(rc);
    hipError_t e = hipStreamCreateWithFlags(&I->sD_own, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&I->sR2_own, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(fail(MISDC_EDEVICE, "stream: %s", hipGetErrorString(e)));
    I->sD = I->sD_own;
    I->sR2 = I->sR2_own;
    I->sR = opts->serialize ? I->sD : I->sR2;
    I->stagger = opts->serialize ? 0 : 1;
    const size_t nev = (size_t)I->levels * (M + 1);
    I->evD.assign(nev, nullptr);
    I->evR.assign(nev, nullptr);
    I->evC.assign(nev, nullptr);
    for (size_t k = 0; k < nev && e == hipSuccess; ++k) {
        e = hipEventCreateWithFlags(&I->evD[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&I->evR[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&I->evC[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_outD, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_outR, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_const, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_source, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_newtonM, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&I->ev_d1, hipEventDisableTiming);
    I->evP.assign(M + 1, nullptr);
    for (int p = 0; p <= M && e == hipSuccess; ++p)
        e = hipEventCreateWithFlags(&I->evP[p], hipEventDisableTiming);
    if (e != hipSuccess) return bail(fail(MISDC_EDEVICE, "events: %s", hipGetErrorString(e)));
    if (opts->pipeline && (rc = create_lanes(I))) return bail(rc);
    if (opts->scheme == MISDC_SCHEME_IMEXQ && (rc = coupled_work_alloc(I->cw, mech->m, grid->g)))
        return bail(rc);
    if (grid->g.n_flames > 0 && grid->g.n_flames <= 0xffff) {
        // the fused stages' work list: every diffused field of every flame,
        // the longest flames first (their systems take longest)
        const Grid& g = grid->g;
        std::vector<int> order(g.n_flames);
        for (int f = 0; f < g.n_flames; ++f) order[f] = f;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return g.len[a] > g.len[b]; });
        std::vector<int> items;
        for (int fl : order)
            for (int f = 0; f <= N; ++f)
                if (f != mech->m.dev.bath) items.push_back((f << 16) | fl);
        if ((rc = dalloc(I, &I->d_items, items.size()))) return bail(rc);
        if (hipMemcpy(I->d_items, items.data(), sizeof(int) * items.size(),
                      hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(MISDC_EDEVICE, "upload of the stage work list"));
        I->nD_items = (int)items.size();
        if ((rc = dalloc(I, &I->stage_counters, 1 + 2 * (size_t)g.n_flames))) return bail(rc);
    }
    *out = I;
    return MISDC_OK;
}

int misdc_integ_destroy(misdc_integ_t I) {
    if (!I) return MISDC_OK;
    if (I->sD) (void)hipStreamSynchronize(I->sD);
    if (I->sR2) (void)hipStreamSynchronize(I->sR2);
    if (I->sRm) (void)hipStreamSynchronize(I->sRm);
    if (I->sD_own) (void)hipStreamSynchronize(I->sD_own);
    if (I->sR2_own) (void)hipStreamSynchronize(I->sR2_own);
    for (hipStream_t s : I->lane_streams) (void)hipStreamSynchronize(s);
    if (I->gexec) (void)hipGraphExecDestroy(I->gexec);
    for (auto& d : I->pd_lane)
        if (d.end) (void)hipEventDestroy(d.end);
    for (auto& r : I->pr_lane)
        if (r.end) (void)hipEventDestroy(r.end);
    for (hipStream_t s : I->lane_streams) (void)hipStreamDestroy(s);
    for (auto& w : I->pdw) diffusion_work_free(w);
    for (hipEvent_t ev : I->evD)
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : I->evR)
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : I->evC)
        if (ev) (void)hipEventDestroy(ev);
    for (auto& t : I->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (hipEvent_t ev : I->ev_pool) (void)hipEventDestroy(ev);
    if (I->ev_in) (void)hipEventDestroy(I->ev_in);
    if (I->ev_outD) (void)hipEventDestroy(I->ev_outD);
    if (I->ev_outR) (void)hipEventDestroy(I->ev_outR);
    if (I->ev_source) (void)hipEventDestroy(I->ev_source);
    if (I->ev_fork) (void)hipEventDestroy(I->ev_fork);
    if (I->ev_join) (void)hipEventDestroy(I->ev_join);
    if (I->ev_const) (void)hipEventDestroy(I->ev_const);
    if (I->ev_newtonM) (void)hipEventDestroy(I->ev_newtonM);
    if (I->ev_d1) (void)hipEventDestroy(I->ev_d1);
    for (hipEvent_t ev : I->evP)
        if (ev) (void)hipEventDestroy(ev);
    // only the streams the library created (a caller's streams stay theirs)
    if (I->sR2_own) (void)hipStreamDestroy(I->sR2_own);
    if (I->sRm) (void)hipStreamDestroy(I->sRm);
    if (I->sD_own) (void)hipStreamDestroy(I->sD_own);
    diffusion_work_free(I->dw);
    coupled_work_free(I->cw);
    if (I->pinc_host) (void)hipHostFree(I->pinc_host);
    for (void* p : I->allocs) (void)hipFree(p);
    delete I;
    return MISDC_OK;
}

int misdc_step(misdc_integ_t I, double* state, double dt, const double* dev_dt, void* stream) {
    int rc = check_step_args(I, state, dt, dev_dt);
    if (rc) return rc;
    if (I->open) return fail(MISDC_ESTATE, "a step opened by misdc_step_begin is not ended");
    hipStream_t cs = (hipStream_t)stream;
    // order after the caller's stream
    MISDC_HIP(hipEventRecord(I->ev_in, cs));
    MISDC_HIP(hipStreamWaitEvent(I->sD, I->ev_in, 0));
    if (I->opt.use_graph && !I->rec_buf) {
        if (!I->gexec || I->g_state != state || I->g_dt != dt || I->g_dtf != dev_dt) {
            drop_graph(I);
            hipGraph_t graph = nullptr;
            MISDC_HIP(hipStreamBeginCapture(I->sD, hipStreamCaptureModeThreadLocal));
            I->capturing = true;
            rc = issue_step(I, state, dt, dev_dt);
            I->capturing = false;
            hipError_t e = hipStreamEndCapture(I->sD, &graph);
            if (rc || e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc ? rc : fail(MISDC_EDEVICE, "step capture: %s", hipGetErrorString(e));
            }
            e = hipGraphInstantiate(&I->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                I->gexec = nullptr;
                return fail(MISDC_EDEVICE, "graph instantiation: %s", hipGetErrorString(e));
            }
            I->g_state = state;
            I->g_dt = dt;
            I->g_dtf = dev_dt;
        }
        MISDC_HIP(hipGraphLaunch(I->gexec, I->sD));
    } else {
        rc = issue_step(I, state, dt, dev_dt);
        if (rc) return rc;
    }
    MISDC_HIP(hipEventRecord(I->ev_outD, I->sD));
    MISDC_HIP(hipStreamWaitEvent(cs, I->ev_outD, 0));
    I->last_sweeps = I->opt.n_sweeps;
    I->dt = dt;
    return MISDC_OK;
}

int misdc_step_begin(misdc_integ_t I, double* state, double dt, const double* dev_dt,
                     void* stream) {
    int rc = check_step_args(I, state, dt, dev_dt);
    if (rc) return rc;
    if (I->open) return fail(MISDC_ESTATE, "a step is already open");
    hipStream_t cs = (hipStream_t)stream;
    MISDC_HIP(hipEventRecord(I->ev_in, cs));
    MISDC_HIP(hipStreamWaitEvent(I->sD, I->ev_in, 0));
    double dts = dt;
    if ((rc = issue_begin(I, state, dt, dev_dt, MAX_STEP_SWEEPS, dts))) return rc;
    I->open = true;
    I->open_state = state;
    I->open_dt = dts;
    I->open_sweeps = 0;
    I->last_sweeps = 0;
    I->dt = dt;
    return MISDC_OK;
}

int misdc_sweep(misdc_integ_t I, void* stream) {
    if (!I) return fail(MISDC_EINVAL, "integrator is NULL");
    if (!I->open) return fail(MISDC_ESTATE, "no step is open (misdc_step_begin)");
    if (I->open_sweeps >= MAX_STEP_SWEEPS)
        return fail(MISDC_EINVAL, "at most %d sweeps per step", MAX_STEP_SWEEPS);
    // ordered after prior work on the caller's stream
    MISDC_HIP(hipEventRecord(I->ev_in, (hipStream_t)stream));
    MISDC_HIP(hipStreamWaitEvent(I->sD, I->ev_in, 0));
    const int k = I->open_sweeps;
    I->sweep_index = k;
    int rc = run_sweep(I, k, I->open_dt, true, false);
    if (rc) return rc;
    I->open_sweeps = k + 1;
    I->last_sweeps = k + 1;             // misdc_get_stats reports the sweeps done so far
    return MISDC_OK;
}

int misdc_step_end(misdc_integ_t I, void* stream) {
    if (!I) return fail(MISDC_EINVAL, "integrator is NULL");
    if (!I->open) return fail(MISDC_ESTATE, "no step is open (misdc_step_begin)");
    MISDC_HIP(hipEventRecord(I->ev_in, (hipStream_t)stream));
    MISDC_HIP(hipStreamWaitEvent(I->sD, I->ev_in, 0));
    int rc = issue_end(I, I->open_state);
    if (rc) return rc;
    hipStream_t cs = (hipStream_t)stream;
    MISDC_HIP(hipEventRecord(I->ev_outD, I->sD));
    MISDC_HIP(hipStreamWaitEvent(cs, I->ev_outD, 0));
    I->open = false;
    I->open_state = nullptr;
    // synchronising end: the step's solver outcome is the return value
    if ((rc = sync_streams(I))) return rc;
    return convergence_status(I);
}

int misdc_integ_set_guess(misdc_integ_t I, misdc_mlp_t mlp, int sweeps) {
    if (!I) return fail(MISDC_EINVAL, "integrator is NULL");
    if (sweeps < 0) return fail(MISDC_EINVAL, "sweeps must be >= 0");
    if (I->open) return fail(MISDC_ESTATE, "a step opened by misdc_step_begin is not ended");
    if (I->pipe && mlp)
        return fail(MISDC_EUNSUPPORTED, "the learned guess's buffers serve one reaction task at a "
                                        "time; pipelined passes run several");
    if (I->fused && mlp)
        return fail(MISDC_EUNSUPPORTED, "fused stages run the plain Newton guess");
    if (I->opt.scheme == MISDC_SCHEME_IMEXQ && mlp)
        return fail(MISDC_EUNSUPPORTED, "IMEXQ has no per-cell reaction solve to guess for");
    int rc;
    if ((rc = sync_streams(I))) return rc;
    if (mlp) {
        if (mlp_dims(mlp->p, 0) != I->N + 2 || mlp_dims(mlp->p, 3) != I->N + 1)
            return fail(MISDC_EINVAL, "network widths do not match %d species", I->N);
        // every buffer a step needs is allocated now (none during a step)
        if ((rc = mlp_reserve(mlp->p, I->n))) return rc;
    }
    I->mlp = mlp ? mlp->p : nullptr;
    I->guess_sweeps = sweeps;
    drop_graph(I);
    return MISDC_OK;
}

int misdc_integ_record(misdc_integ_t I, double* dev_buf, int64_t max_tasks) {
    if (!I) return fail(MISDC_EINVAL, "integrator is NULL");
    if (max_tasks < 0 || (max_tasks > 0 && !dev_buf)) return fail(MISDC_EINVAL, "invalid buffer");
    if (I->open) return fail(MISDC_ESTATE, "a step opened by misdc_step_begin is not ended");
    if (I->fused && max_tasks > 0)
        return fail(MISDC_EUNSUPPORTED, "fused stages do not record reaction problems");
    if (I->opt.scheme == MISDC_SCHEME_IMEXQ && max_tasks > 0)
        return fail(MISDC_EUNSUPPORTED, "IMEXQ has no per-cell reaction problems to record");
    int rc;
    if ((rc = sync_streams(I))) return rc;
    I->rec_buf = max_tasks > 0 ? dev_buf : nullptr;
    I->rec_cap = max_tasks;
    I->rec_count = 0;
    drop_graph(I);
    return MISDC_OK;
}

int misdc_integ_recorded(misdc_integ_t I, int64_t* tasks) {
    if (!I || !tasks) return fail(MISDC_EINVAL, "NULL argument");
    *tasks = I->rec_count;
    return MISDC_OK;
}

// The reaction stream can be confined to part of the CUs, so that the
// persistent diffusion solve, whose workgroups must all be resident at once,
// finds CUs free of Newton waves when it starts instead of waiting for them
// to drain.  Mask bit i is set when (i / 8) mod 4 < quarters.  The driver
// hands mask bits to the XCDs either round-robin (bit i to XCD i mod 8) or in
// runs of 32 consecutive bits; either way every XCD keeps quarters/4 of its
// CUs, so each XCD can run its share of a launch's workgroups.  The diffusion
// stream is never masked.  The mask read back from the runtime must equal the
// one requested.
int reaction_stream_split(misdc_integ_s* I, int quarters) {
    if (quarters == 0 || (I->sRm && I->sRm_split == quarters)) return MISDC_OK;
    int cus = 0;
    int rc = device_cus(cus);
    if (rc) return rc;
    if (cus < 32 || cus % 32)
        return fail(MISDC_EINVAL, "cu_split needs a multiple of 32 CUs (device has %d)", cus);
    const size_t words = (size_t)cus / 32;
    std::vector<uint32_t> mask(words, 0u), back(words, 0u);
    for (int i = 0; i < cus; ++i)
        if ((i / 8) % 4 < quarters) mask[(size_t)i / 32] |= 1u << (i % 32);
    hipStream_t s = nullptr;
    MISDC_HIP(hipExtStreamCreateWithCUMask(&s, (uint32_t)words, mask.data()));
    hipError_t e = hipExtStreamGetCUMask(s, (uint32_t)words, back.data());
    if (e != hipSuccess || back != mask) {
        (void)hipStreamDestroy(s);
        return fail(MISDC_EDEVICE, "CU mask of the reaction stream not applied (%s)",
                    e != hipSuccess ? hipGetErrorString(e) : "mask differs");
    }
    if (I->sRm) {
        (void)hipStreamSynchronize(I->sRm);
        (void)hipStreamDestroy(I->sRm);
    }
    I->sRm = s;
    I->sRm_split = quarters;
    return MISDC_OK;
}

int misdc_set_streams(misdc_integ_t I, void* diffusion_stream, void* reaction_stream) {
    if (!I) return fail(MISDC_EINVAL, "integrator is NULL");
    if (I->open) return fail(MISDC_ESTATE, "a step opened by misdc_step_begin is not ended");
    if (diffusion_stream && diffusion_stream == reaction_stream)
        return fail(MISDC_EINVAL, "the two streams must differ (one stream: set_tune serialize)");
    if (I->pipe && (diffusion_stream || reaction_stream))
        return fail(MISDC_EUNSUPPORTED, "pipelined passes run on the integrator's own lanes");
    int rc;
    if ((rc = sync_streams(I))) return rc;
    const bool serial = I->sR == I->sD;
    const bool masked = I->sRm && I->sR == I->sRm;
    I->sD = diffusion_stream ? (hipStream_t)diffusion_stream : I->sD_own;
    I->sR2 = reaction_stream ? (hipStream_t)reaction_stream : I->sR2_own;
    I->caller_R = reaction_stream != nullptr;
    if (I->caller_R && masked) {
        // a caller's reaction stream replaces the library's CU-masked one
        I->cu_split = 0;
    }
    I->sR = serial ? I->sD : ((masked && !I->caller_R) ? I->sRm : I->sR2);
    drop_graph(I);
    return MISDC_OK;
}

int misdc_get_tune(misdc_integ_t I, misdc_tune* t) {
    if (!I || !t) return fail(MISDC_EINVAL, "NULL argument");
    t->cg_variant = I->dw.variant;
    t->cg_blocks = I->dw.blocks;
    t->cyclic = I->dw.cyclic;
    t->serialize = I->sR == I->sD ? 1 : 0;
    t->cu_split = I->cu_split;
    t->stagger = I->stagger;
    t->step_ms = I->tuned_ms;
    t->fused = I->fused ? 1 : 0;
    return MISDC_OK;
}

int misdc_set_tune(misdc_integ_t I, const misdc_tune* t) {
    if (!I || !t) return fail(MISDC_EINVAL, "NULL argument");
    if (I->open) return fail(MISDC_ESTATE, "a step opened by misdc_step_begin is not ended");
    if (t->cyclic != 0 && t->cyclic != 1) return fail(MISDC_EINVAL, "cyclic must be 0 or 1");
    if (t->serialize != 0 && t->serialize != 1) return fail(MISDC_EINVAL, "serialize must be 0 or 1");
    if (t->cu_split < 0 || t->cu_split > 3) return fail(MISDC_EINVAL, "cu_split must be in [0, 3]");
    if (t->stagger != 0 && t->stagger != 1) return fail(MISDC_EINVAL, "stagger must be 0 or 1");
    if (t->cu_split && !t->serialize && I->caller_R)
        return fail(MISDC_EINVAL, "cu_split needs the library's own reaction stream "
                                  "(misdc_set_streams gave one of the caller's)");
    if (I->pipe && (t->serialize || t->cu_split || t->stagger))
        return fail(MISDC_EINVAL, "pipelined passes take their own lanes: serialize, cu_split "
                                  "and stagger must be 0");
    if (t->fused != 0 && t->fused != 1) return fail(MISDC_EINVAL, "fused must be 0 or 1");
    if (t->fused) {
        const misdc_newton_opts& no = I->opt.newton;
        if (I->grid->n_flames <= 0 || !I->d_items || I->opt.scheme != MISDC_SCHEME_CISDCQ ||
            I->N != 9 || I->pipe || I->mlp || I->rec_buf)
            return fail(MISDC_EINVAL, "fused stages need an ensemble grid, CISDCQ, 9 species, "
                                      "no pipelined passes, learned guess or recording");
        if (no.lu != MISDC_LU_FP64 ||
            (no.kernel != MISDC_NEWTON_AUTO && no.kernel != MISDC_NEWTON_THREAD))
            return fail(MISDC_EINVAL, "fused stages run the FP64 one-thread-per-cell reaction "
                                      "solve");
        if (t->serialize != 1 || t->cu_split || t->stagger)
            return fail(MISDC_EINVAL, "fused stages run on one stream: serialize 1, cu_split "
                                      "and stagger 0");
        for (int64_t L : I->grid->len)
            if (L < 16) return fail(MISDC_EINVAL, "fused stages need flames of >= 16 cells");
    }
    const Grid& g = *I->grid;
    int rc;
    if ((rc = sync_streams(I))) return rc;
    if (g.dim == 2 && g.n_flames == 0) {
        DiffusionWork probe = I->dw;
        rc = diffusion_work_set(probe, *I->mech, g, t->cg_variant, t->cg_blocks);
        if (rc) return rc;
        if (I->pipe) {
            int cus = 0;
            if ((rc = device_cus(cus))) return rc;
            if (probe.blocks > cus / 2)
                return fail(MISDC_EINVAL, "pipelined passes: at most %d diffusion workgroups",
                            cus / 2);
            for (auto& w : I->pdw) {
                w.variant = probe.variant;
                w.blocks = probe.blocks;
            }
        }
        I->dw.variant = probe.variant;
        I->dw.blocks = probe.blocks;
    }
    if (!t->serialize && t->cu_split) {
        rc = reaction_stream_split(I, t->cu_split);
        if (rc) return rc;
    }
    I->dw.cyclic = t->cyclic;
    for (auto& w : I->pdw) w.cyclic = t->cyclic;
    I->fused = t->fused != 0;
    I->cu_split = t->serialize ? 0 : t->cu_split;
    I->stagger = t->serialize ? 0 : t->stagger;
    I->sR = t->serialize ? I->sD : (I->cu_split ? I->sRm : I->sR2);
    if (!I->cu_split && I->sRm) {
        // a CU-masked stream holds a hardware queue of its own (the mask is a
        // queue property) even while idle; with few queues per process an
        // idle one can make the streams in use, or a replayed graph's, share
        // a queue and run in order, so it is released when not in use
        (void)hipStreamDestroy(I->sRm);
        I->sRm = nullptr;
        I->sRm_split = 0;
    }
    drop_graph(I);
    return MISDC_OK;
}

int misdc_autotune(misdc_integ_t I, const double* state, double dt, const double* dev_dt, int reps,
                   misdc_tune* best, void* stream) {
    int rc = check_step_args(I, state, dt, dev_dt);
    if (rc) return rc;
    if (reps < 1 || reps > 100) return fail(MISDC_EINVAL, "reps must be in [1, 100]");
    if (I->open) return fail(MISDC_ESTATE, "a step opened by misdc_step_begin is not ended");
    hipStream_t cs = (hipStream_t)stream;
    const Grid& g = *I->grid;
    int cus = 0;
    if ((rc = device_cus(cus))) return rc;
    std::vector<misdc_tune> cand;
    misdc_tune base;
    misdc_get_tune(I, &base);
    for (int k = 0; k < 6; ++k) {
        // (serialize, cu_split, stagger): two streams on all CUs, staggered
        // or not; the reaction stream on 3/4 or 1/2 of the CUs; one stream
        static const int SER[6] = {0, 0, 0, 0, 0, 1}, SPLIT[6] = {0, 0, 3, 3, 2, 0},
                         STAG[6] = {0, 1, 0, 1, 0, 0};
        misdc_tune t = base;
        t.serialize = SER[k];
        t.cu_split = SPLIT[k];
        t.stagger = STAG[k];
        t.fused = 0;
        if (g.dim == 2 && g.n_flames == 0) {
            const int cap = cus < 256 ? cus : 256;
            if (I->N == 9)
                for (int c : {1, 2, 4}) {
                    const int64_t b = cg_regs_min_blocks(I->n, c);
                    if (b <= cap) {
                        t.cg_variant = c;
                        t.cg_blocks = (int)b;
                        cand.push_back(t);
                    }
                }
            const int64_t tiles = cg_tile_blocks(g);
            if (I->N == 9 && tiles >= 1 && tiles <= cap)
                for (int v : {101, 102, 103}) {
                    t.cg_variant = v;
                    t.cg_blocks = (int)tiles;
                    cand.push_back(t);
                }
            for (int div : {4, 2, 1}) {
                t.cg_variant = 0;
                t.cg_blocks = cap / div > 0 ? cap / div : 1;
                cand.push_back(t);
            }
        } else {
            for (int cy : {0, 1}) {
                t.cyclic = cy;
                cand.push_back(t);
            }
        }
    }
    if (g.n_flames > 0 && I->d_items) {
        // each stage as one persistent launch (refused where it does not apply)
        misdc_tune t = base;
        t.serialize = 1;
        t.cu_split = 0;
        t.stagger = 0;
        t.cyclic = 1;
        t.fused = 1;
        cand.push_back(t);
    }
    const size_t bytes = sizeof(double) * (size_t)I->NF * I->n;
    double* work = nullptr;
    MISDC_HIP(hipMalloc(&work, bytes));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    const int saved_graph = I->opt.use_graph;
    I->opt.use_graph = 0;
    double best_ms = -1.0;
    misdc_tune pick = base;
    for (size_t k = 0; k < cand.size() && he == hipSuccess && !rc; ++k) {
        if (misdc_set_tune(I, &cand[k]) != MISDC_OK) continue;   // does not fit: skip
        he = hipMemcpyAsync(work, state, bytes, hipMemcpyDeviceToDevice, cs);
        if (he != hipSuccess) break;
        if ((rc = misdc_step(I, work, dt, dev_dt, stream))) break;
        if ((he = hipEventRecord(e0, cs)) != hipSuccess) break;
        for (int r = 0; r < reps && !rc; ++r) rc = misdc_step(I, work, dt, dev_dt, stream);
        if (rc) break;
        if ((he = hipEventRecord(e1, cs)) != hipSuccess) break;
        if ((he = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.f;
        if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        const double per = ms / reps;
        if (best_ms < 0 || per < best_ms) {
            best_ms = per;
            pick = cand[k];
            pick.step_ms = per;
        }
    }
    I->opt.use_graph = saved_graph;
    (void)hipStreamSynchronize(cs);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(work);
    if (rc) return rc;
    if (he != hipSuccess) return fail(MISDC_EDEVICE, "autotune: %s", hipGetErrorString(he));
    if (best_ms < 0) return fail(MISDC_EDEVICE, "autotune: no configuration ran");
    if ((rc = misdc_set_tune(I, &pick))) return rc;
    I->tuned_ms = best_ms;
    if (best) *best = pick;
    return MISDC_OK;
}

int misdc_get_stats(misdc_integ_t I, misdc_stats* st) {
    if (!I || !st) return fail(MISDC_EINVAL, "NULL argument");
    int rc;
    if ((rc = sync_streams(I))) return rc;
    std::memset(st, 0, sizeof(*st));
    unsigned long long ns[8];
    int32_t cg[8];
    MISDC_HIP(hipMemcpy(ns, I->nstats, sizeof(ns), hipMemcpyDeviceToHost));
    {
        // counters the per-thread Newton kernel keeps itself
        std::vector<unsigned long long> b((size_t)NEWTON_BUCKETS * NEWTON_BUCKET_STRIDE);
        MISDC_HIP(hipMemcpy(b.data(), I->nbuckets, sizeof(unsigned long long) * b.size(),
                            hipMemcpyDeviceToHost));
        for (int k = 0; k < NEWTON_BUCKETS; ++k) {
            const unsigned long long* s = b.data() + (size_t)k * NEWTON_BUCKET_STRIDE;
            ns[0] += s[0];
            ns[1] += s[1];
            ns[2] += s[2];
            ns[3] = s[3] > ns[3] ? s[3] : ns[3];
            st->newton_pivot_retries += (int64_t)s[4];
        }
    }
    if ((rc = read_cgstats(I, cg))) return rc;
    st->newton_solves = (int64_t)ns[0];
    st->newton_iters = (int64_t)ns[1];
    st->newton_failed = (int64_t)ns[2];
    st->newton_max = (int32_t)ns[3];
    st->newton_lu_solves = (int64_t)ns[4];
    st->newton_lu_fallbacks = (int64_t)ns[5];
    st->newton_guess_learned = (int64_t)ns[6];
    st->imexq_solves = I->cst.solves;
    st->imexq_newton_iters = I->cst.newton_iters;
    st->imexq_failed = I->cst.newton_failed;
    st->imexq_krylov_iters = I->cst.krylov_iters;
    st->imexq_krylov_max = I->cst.krylov_max;
    st->imexq_krylov_failed = I->cst.krylov_failed;
    st->newton_failed += I->cst.newton_failed;
    for (int k = 0; k < I->last_sweeps && k < 64; ++k) st->nested_passes[k] = I->passes[k];
    st->cg_iters = cg[0];
    st->cg_max = cg[1];
    st->cg_failed = cg[2] + cg[4];
    st->cg_solves = cg[3];
    const int K = I->last_sweeps;
    st->n_sweeps = K;
    if ((rc = drain_timing(I))) return rc;
    st->diffusion_kernel_ms = I->t_ms[0];
    st->diffusion_kernel_launches = I->t_cnt[0];
    st->newton_kernel_ms = I->t_ms[1];
    st->newton_kernel_launches = I->t_cnt[1];
    if (K > 0) {
        std::vector<double> inc((size_t)K * I->NF * 2);
        MISDC_HIP(hipMemcpy(inc.data(), I->inc, sizeof(double) * inc.size(), hipMemcpyDeviceToHost));
        for (int k = 0; k < K && k < 64; ++k) {
            double worst = 0.0;
            for (int f = 0; f < I->NF; ++f) {
                const double d = inc[((size_t)k * I->NF + f) * 2], a = inc[((size_t)k * I->NF + f) * 2 + 1];
                const double rel = a > 0 ? d / a : d;
                worst = rel > worst ? rel : worst;
            }
            st->sweep_increment[k] = worst;
        }
    }
    // the statistics are filled either way; unconverged solves make the status
    if (st->newton_failed > 0 || st->cg_failed > 0)
        return fail(MISDC_ENOTCONV,
                    "unconverged solves in the last step: %lld cell-node Newton solves, "
                    "%d diffusion solves at their iteration limit or barrier timeout",
                    (long long)st->newton_failed, st->cg_failed);
    return MISDC_OK;
}

int misdc_get_newton_histogram(misdc_integ_t I, int sweep, int64_t* counts) {
    if (!I || !counts) return fail(MISDC_EINVAL, "NULL argument");
    if (sweep < 0 || sweep >= I->last_sweeps)
        return fail(MISDC_EINVAL, "sweep %d outside the last step's %d sweeps", sweep,
                    I->last_sweeps);
    int rc;
    if ((rc = sync_streams(I))) return rc;
    std::vector<unsigned long long> h((size_t)NEWTON_HIST_SETS * NEWTON_HIST_BINS);
    MISDC_HIP(hipMemcpy(h.data(), I->nhist + (size_t)sweep * NEWTON_HIST_SETS * NEWTON_HIST_BINS,
                        sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost));
    for (int b = 0; b < NEWTON_HIST_BINS; ++b) {
        unsigned long long c = 0;
        for (int k = 0; k < NEWTON_HIST_SETS; ++k) c += h[(size_t)k * NEWTON_HIST_BINS + b];
        counts[b] = (int64_t)c;
    }
    return MISDC_OK;
}

int misdc_reset_profile(misdc_integ_t I) {
    if (!I) return fail(MISDC_EINVAL, "integrator is NULL");
    int rc;
    if ((rc = sync_streams(I))) return rc;
    if ((rc = drain_timing(I))) return rc;
    I->t_ms[0] = I->t_ms[1] = 0.0;
    I->t_cnt[0] = I->t_cnt[1] = 0;
    return MISDC_OK;
}

}  // extern "C"
