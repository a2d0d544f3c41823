// Internal declarations of the MI355X MISDC library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "misdc.h"

namespace misdc {

// ---- error handling -------------------------------------------------------
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

#define MISDC_HIP(call)                                                          \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess)                                                    \
            return ::misdc::fail(MISDC_EDEVICE, "%s failed: %s (%s:%d)", #call,  \
                                 hipGetErrorString(e_), __FILE__, __LINE__);     \
    } while (0)

// ---- constants -------------------------------------------------------------
constexpr double T_REF = 298.15;        // thermodynamic reference temperature
constexpr double T_DIFF_REF = 300.0;    // reference of the (T/300)^1.7 law
constexpr double THETA_EXP = 1.7;
constexpr int MAX_NODES = 9;
constexpr int MAX_STEP_SWEEPS = 64;      // sweeps of one step (statistics arrays)

// ---- device mechanism tables (passed to kernels by value) ------------------
struct MechDev {
    int N, R, bath;
    double rho0, p_atm, R_u, R_c, alpha0;
    double newton_scale;          // mean of cp_k / W_k: enthalpy residual -> K
    double ln_patm_over_Ru;       // ln(p_atm / R_u)
    const int* slots;             // R x 4: reactant 0, reactant 1, product 0, product 1 (or -1)
    const double* A;              // R
    const double* beta;           // R
    const double* Ta;             // R: Ea / R_c (K)
    const double* dn;             // R: sum of net stoichiometric coefficients
    const double* uW;             // R x N: nu_kj W_k / rho0 (dense net stoichiometry)
    const double* W;              // N
    const double* invW;           // N
    const double* cp;             // N (molar)
    const double* hf;             // N
    const double* s0;             // N
    const double* kappa0;         // N+1: D0_k, then alpha0
    // per-species reaction lists (CSR over species k, reactions ascending):
    // rowj[rowp[k] .. rowp[k+1]) are the reactions with nu_kj != 0 and
    // rowu the matching nu_kj W_k / rho0
    const int* rowp;              // N+1
    const int* rowj;              // nnz
    const double* rowu;           // nnz
    // the same lists for the chunked evaluation (reactions in chunks of 64):
    // rowl[4 e + s] = slot species s of reaction rowj[e] (so an entry needs no
    // second, dependent lookup), and rowc[k (nch + 1) + c] = the first entry
    // of species k whose reaction is in chunk c or later
    const int* rowl;              // 4 nnz
    const int* rowc;              // N (nch + 1)
    int nch;                      // chunks of 64 reactions
};

struct Mech {
    MechDev dev;
    int device = 0;
    void* block = nullptr;        // one device allocation holding every table
    std::vector<double> W, cp, hf, kappa0;   // host copies (for host-side checks)
    // reaction solve generated for this mechanism (hipFunction_t, owned by a
    // process-wide cache), or null with the reason in spec_status
    void* spec_fn = nullptr;
    std::string spec_status;
};

// host copies of the tables from which a mechanism's kernels are generated
struct MechTables {
    int N = 0, R = 0, bath = 0;
    std::vector<int> slots;                         // R x 4 (reactants, products; -1 empty)
    std::vector<double> A, beta, Ta, dn, uW, W, invW, cp, hf, s0;
    double rho0 = 0, R_u = 0, newton_scale = 0, ln_patm_over_Ru = 0;
};
// largest species count of the generated one-thread-per-cell reaction solve
constexpr int NEWTON_SPEC_MAX_SPECIES = 12;
// generates, compiles (hiprtc, once per process, device and mechanism) and
// loads the specialised reaction solve; leaves m.spec_fn null (and says why
// in m.spec_status) where it cannot, so the generic kernels serve
int newton_spec_prepare(Mech& m, const MechTables& t);
std::string newton_spec_source(const MechTables& t);
// compiles a generated source for the device without loading it (no GPU needed)
int newton_spec_compile_check(const std::string& src, std::string& msg);

// ---- grid ------------------------------------------------------------------
struct Grid {
    int dim = 1;                  // 1 or 2
    int64_t nx = 0, ny = 1;       // single grid
    double dx = 0, dy = 0, ux = 0, uy = 0;
    int n_flames = 0;             // > 0: ensemble of 1-D flames
    std::vector<int64_t> len, off;
    std::vector<double> fdx, fu;
    int64_t* d_off = nullptr;     // device copies for the ensemble (n_flames + 1)
    double* d_dx = nullptr;
    double* d_u = nullptr;
    int64_t cells() const {
        if (n_flames > 0) return off.back();
        return nx * ny;
    }
};

// ---- kernel launchers (stream-ordered, no synchronisation) -----------------
int launch_enthalpy(const Mech& m, int64_t n, const double* Y, const double* T, double* h,
                    hipStream_t s);
int launch_temperature(const Mech& m, int64_t n, const double* Y, const double* h, double* T,
                       hipStream_t s);
int launch_reaction_source(const Mech& m, int64_t n, const double* Y, const double* h,
                           double* FR, hipStream_t s);
// state: N+1 fields (Y, h) with stride n; bY: N fields stride ldb;
// c: per-cell array or nullptr with c_scalar.
struct NewtonArgs {
    int64_t n;
    const double* bY; int64_t ldb;          // N fields
    const double* h;                        // n
    const double* c; double c_scalar;      // c = c[i] * c_scalar, or c_scalar
    const double* guess; int64_t ldg;       // N fields
    double* Y; int64_t ldy;                 // N fields out
    double* T;                              // n out (closed form of (Y, h)), may be null
    double* h_out = nullptr;                // n out, may be null: a copy of h (the reaction
                                            // step leaves the enthalpy unchanged)
    double* th_out = nullptr;               // n out, may be null: (T/300)^1.7 of the result
    double* FR; int64_t ldf;                // N fields out, may be null
    int32_t* iters;                         // n out, may be null
    int32_t* lu_info = nullptr;             // n out, may be null: FP32 solves | FP64 fallbacks << 16
    unsigned long long* stats;              // [0] solves, [1] iters, [2] failed, [3] max,
                                            // [4] FP32 solves, [5] fallbacks; may be null
    // per-thread kernel only, may be null: the kernel itself adds [0..3] of
    // each wavefront into NEWTON_BUCKETS sets of counters (set b at
    // b * NEWTON_BUCKET_STRIDE), and no statistics kernel follows
    unsigned long long* buckets = nullptr;
    // may be null: histogram of the solves' outcomes in NEWTON_HIST_SETS sets
    // of NEWTON_HIST_BINS counters (bin 0: not converged; bin v: converged
    // after v linear solves, the last bin also counting more); wavefront w of
    // the launch adds to set w % NEWTON_HIST_SETS
    unsigned long long* hist = nullptr;
    // per-thread kernel only: > 0 for the cells of a 2-D grid of tile_nx x
    // tile_ny cells (x fastest, tile_nx * tile_ny = n); each 64-thread block
    // then takes one NEWTON_TILE_X x NEWTON_TILE_Y tile of cells instead of
    // 64 consecutive cells
    int tile_nx = 0, tile_ny = 0;
    misdc_newton_opts opt;
};
constexpr int NEWTON_BUCKETS = 32, NEWTON_BUCKET_STRIDE = 16;   // 128-byte apart
constexpr int NEWTON_HIST_BINS = 64, NEWTON_HIST_SETS = 8;
// the cell tile of the tiled per-thread Newton launches: a row of 16 FP64
// values is one whole 128-byte line, so no line is split between two
// workgroups (which may sit on different XCDs and their L2s)
constexpr int NEWTON_TILE_X = 16, NEWTON_TILE_Y = 4;
static_assert(NEWTON_TILE_X * NEWTON_TILE_Y == 64, "one wavefront per cell tile");
int launch_reaction_newton(const Mech& m, const NewtonArgs& a, hipStream_t s);
// the generated kernel (statistics into a.buckets / a.hist when a.buckets is set)
int launch_newton_spec(const Mech& m, const NewtonArgs& a, hipStream_t s);
// one wavefront per cell (any species count up to 63): FP64 LU, or an FP32
// LU on the matrix cores refined against the FP64 matrix
enum { NEWTON_LU_FP64 = 0, NEWTON_LU_FP32_MFMA = 1 };
int launch_reaction_newton_wave(const Mech& m, const NewtonArgs& a, int lu, hipStream_t s);
int launch_reaction_source_wave(const Mech& m, int64_t n, const double* Y, int64_t ldy,
                                const double* h, double* FR, int64_t ldf, hipStream_t s);

// out[p] = sum_t W[p][t] s_t X_t, field-wise; X_t has nf_t fields (missing
// fields are zero); s_t = scale[cell] for the terms in smask (per-cell step
// sizes of an ensemble), else 1
constexpr int LC_MAX_TERMS = 32;
constexpr int LC_MAX_OUT = 8;
struct LinComb {
    int nterms = 0, nout = 0, nfields = 0;
    int64_t ncells = 0;
    const double* X[LC_MAX_TERMS];
    int nf[LC_MAX_TERMS];
    double* out[LC_MAX_OUT];
    double W[LC_MAX_OUT][LC_MAX_TERMS];
    const double* scale;
    unsigned smask;
};
int launch_lincomb(const LinComb& lc, hipStream_t s);
// device-side copy and fill (stream-ordered kernels, safe under graph capture)
int launch_copy(double* dst, const double* src, int64_t count, hipStream_t s);
// clears up to four buffers (whole 32-bit words, bytes[k] each) in one launch
int launch_zero_many(void* const* dst, const int64_t* bytes, int count, hipStream_t s);
// th = (T/300)^1.7 of n cells
int launch_theta(int64_t n, const double* T, double* th, hipStream_t s);
int launch_zero(void* dst, int64_t bytes, hipStream_t s);
// per-cell value of a per-flame array: out[i] = v[flame of cell i]
int launch_expand_flames(const Grid& g, const double* v, double* out, hipStream_t s);

// T (cells) from a state with N+1 fields
// T of a state (N+1 fields); copy (may be null) receives the state in the same pass
int launch_state_temperature(const Mech& m, int64_t n, const double* state, double* T, hipStream_t s,
                             double* copy = nullptr);
// FA and FD (N+1 fields) at a state whose temperature is T; either output may be null
// (theta_ready: work_theta already holds (T/300)^1.7)
int launch_transport(const Mech& m, const Grid& g, const double* state, const double* T,
                     double* FA, double* FD, double* work_theta, hipStream_t s,
                     bool theta_ready = false);

struct DiffusionWork {
    double* theta = nullptr;      // cells
    double* Kx = nullptr;         // cells: east-face coefficient / dx^2
    double* Ky = nullptr;         // cells: north-face coefficient / dy^2
    double* x = nullptr;          // N+1 fields (CG vectors, 2-D only)
    double* r = nullptr;
    double* z = nullptr;
    double* p = nullptr;
    double* q = nullptr;
    double* partial = nullptr;    // blocks x fields x 4
    double* edge = nullptr;       // tiled CG: edges of m of every tile (2-D, 9 diffused fields)
    double* totals = nullptr;     // fields x 4
    unsigned* barrier = nullptr;  // 4 words
    int32_t* info = nullptr;      // [0] iterations, [1] failed, [2] barrier timeout
    int blocks = 0;
    int threads = 0;
    int fields_cap = 0;
    int variant = 0;              // 0: vectors in global memory; 1, 2, 4: cells per thread in
                                  // registers; 101..103: tiled, 1..3 local preconditioner sweeps
    int cyclic = 1;               // 1-D systems: 0 one thread per system, 1 one wavefront per system
};
int diffusion_work_alloc(DiffusionWork& w, const Mech& m, const Grid& g);
// the same workspace carved out of one device block of ``bytes`` (no
// allocation; the zeroed parts are cleared by kernels on s), and the bytes it
// needs (each part 256-byte aligned)
size_t diffusion_work_bytes(const Mech& m, const Grid& g);
int diffusion_work_carve(DiffusionWork& w, const Mech& m, const Grid& g, void* block, size_t bytes,
                         hipStream_t s);
// selects the 2-D CG variant (0 global memory, 1/2/4 cells per thread in
// registers) and its block count, after checking that it fits
int diffusion_work_set(DiffusionWork& w, const Mech& m, const Grid& g, int variant, int blocks);
int64_t cg_regs_min_blocks(int64_t n, int cpt);
// tiles of the tiled CG variants (0 if the grid is not a single 2-D grid)
int64_t cg_tile_blocks(const Grid& g);
int device_cus(int& cus);
void diffusion_work_free(DiffusionWork& w);
// Solves all N+1 fields (bath by closure); y may hold the guess (guess_in_y);
// T_out (optional) receives T(y) and th_out (optional, with T_out) its
// (T/300)^1.7; cgstats (optional, 2-D solves) accumulates the CG statistics
struct LagRhs;
int launch_diffusion_solve(const Mech& m, const Grid& g, DiffusionWork& w, double c,
                           const double* dt_flame, double c_factor,
                           const double* T_lag, const double* rhs, double* y, int guess_in_y,
                           double rtol, int maxit, hipStream_t s,
                           hipEvent_t core_begin = nullptr, hipEvent_t core_end = nullptr,
                           double* T_out = nullptr, int32_t* cgstats = nullptr,
                           double* th_out = nullptr, bool faces_ready = false,
                           const LagRhs* fused = nullptr);
// right-hand side (a linear combination over the grid's cells) together with
// the face coefficients of the lagged operator at T_lag, for a solve called
// with faces_ready
int launch_lincomb_faces(const LinComb& lc, const Grid& g, const double* T_lag, DiffusionWork& w,
                         hipStream_t s);
// The last step of a diffusion right-hand side split in two passes: out =
// part + scale (qa FA(src) + qd FD(src) + qr FR) for the N+1 fields of a
// state src whose theta is th (the lagged operators of the concurrent
// scheme's first nested iteration; or the node-M terms of the first task's
// right-hand side in the next sweep), with the face coefficients of the
// solve's lagged operator at T_lag in the same pass, for a solve called with
// faces_ready.  part holds every other term, formed earlier by
// launch_lincomb; scale (may be null) is the per-cell factor of dt-carrying
// terms.  With T_src set, theta is (T_src/300)^1.7 of the cells (th unused);
// fr (may be null) holds the N species' FR.
struct LagRhs {
    const double* src = nullptr;
    const double* th = nullptr;
    const double* T_src = nullptr;
    const double* part = nullptr;
    const double* fr = nullptr;
    double* out = nullptr;
    double qa = 0.0, qd = 0.0, qr = 0.0;
    const double* scale = nullptr;
    const double* T_lag = nullptr;
};
int launch_lag_rhs(const Mech& m, const Grid& g, const LagRhs& a, DiffusionWork& w, hipStream_t s);

// max_i |a - b| and max_i |a| per field into out[2*f], out[2*f+1] (device);
// partial holds nfields * partial_blocks * 2 doubles followed by a zeroed
// 32-bit arrival counter (left zero after each launch)
int launch_field_diff_max(int nfields, int64_t n, const double* a, const double* b,
                          double* partial, int partial_blocks, double* out, hipStream_t s);

// One stage of a concurrent sweep over an ensemble of 1-D flames as one
// persistent launch (ensemble.hip): the diffusion solve at node m+1 (its
// right-hand side, guess and face coefficients already formed) and the
// reaction solve at node m (its right-hand side formed), both drawn from one
// atomic work queue; either part may be absent.
struct EnsembleStage {
    bool has_d = false, has_r = false;
    int nD = 0;                       // (field << 16 | flame) systems, longest first
    const int* d_items = nullptr;
    double c = 0.0, cfac = 0.0;       // c, or dtf[flame] * cfac, times kappa0
    const double* dtf = nullptr;
    const double* Kx = nullptr;
    const double* rhs = nullptr;
    double* y = nullptr;
    double *sc = nullptr, *su = nullptr, *sv = nullptr, *sw = nullptr;
    double* T_out = nullptr;
    double* th_out = nullptr;
    double* lagFA = nullptr;          // non-null: lag transport at y
    double* lagFD = nullptr;
    NewtonArgs na{};
    const double* h_src = nullptr;
    double* h_dst = nullptr;
    const double* rstate = nullptr;
    const double* rT = nullptr;
    double* rth = nullptr;
    double* rFA = nullptr;
    double* rFD = nullptr;
    unsigned* counters = nullptr;     // 1 + 2 n_flames words
    int waves_per_slot = 1;
};
int launch_ensemble_stage(const Mech& m, const Grid& g, const EnsembleStage& st, hipStream_t s);

// ---- the coupled implicit diffusion-reaction solve of IMEXQ (9 species) -----
struct CoupledWork {
    int64_t n = 0;
    double *G = nullptr, *d = nullptr, *r = nullptr, *rh = nullptr, *p = nullptr, *v = nullptr,
           *y = nullptr, *s = nullptr, *t = nullptr, *zz = nullptr;   // NF fields each
    double* JR = nullptr;        // reaction Jacobian w.r.t. (Y, h): N x NF entries per cell
    double *th = nullptr, *Kx = nullptr, *Ky = nullptr;
    double* sigma = nullptr;     // field scales (NF)
    double* partial = nullptr;   // per-block reduction partials
};
struct CoupledStats {
    int64_t solves = 0, newton_iters = 0, newton_failed = 0;
    int64_t krylov_iters = 0, krylov_max = 0, krylov_failed = 0;
};
int coupled_work_alloc(CoupledWork& w, const Mech& m, const Grid& g);
void coupled_work_free(CoupledWork& w);
// x (NF fields, holding the initial guess) <- the solution of
// x - c (FD_lag(x) + FR(x)) = rhs; synchronises s while it iterates
int coupled_solve(const Mech& m, const Grid& g, CoupledWork& w, double c, const double* T_lag,
                  const double* rhs, double* x, double newton_tol, int newton_maxit,
                  double lin_rtol, int lin_maxit, CoupledStats& st, hipStream_t s);

// ---- learned Newton guess (dense network on the matrix cores) ----------------
struct MlpImpl;
int mlp_create(int n_in, int n_hidden, int n_out, int prec, MlpImpl** out);
void mlp_destroy(MlpImpl* p);
int64_t mlp_param_count(const MlpImpl* p);
int mlp_dims(const MlpImpl* p, int l);
int mlp_set_params(MlpImpl* p, const float* host);
int mlp_get_params(MlpImpl* p, float* host);
int mlp_set_norm(MlpImpl* p, const float* in_mu, const float* in_sd, const float* out_sd);
int mlp_reserve(MlpImpl* p, int64_t cells);
int mlp_forward(MlpImpl* p, int64_t B, const float* x, float* y, hipStream_t s);
int mlp_gradients(MlpImpl* p, int64_t B, const float* x, const float* t, float* grad, float* loss,
                  hipStream_t s);
int mlp_adam(MlpImpl* p, const float* grad, float lr, float b1, float b2, float eps, hipStream_t s);
int mlp_train(MlpImpl* p, int64_t n, const float* x, const float* t, int64_t batch, int epochs,
              float lr, float* loss_hist, hipStream_t s);
int mlp_features(const Mech& m, MlpImpl* p, int64_t n, const double* bY, const double* h,
                 const double* c, double c_scalar, float* x, hipStream_t s);
int mlp_targets(const Mech& m, MlpImpl* p, int64_t n, const double* bY, const double* h,
                const double* Ys, float* t, hipStream_t s);
int mlp_prepare(const Mech& m, MlpImpl* p, int64_t n, const double* bY, const double* h,
                const double* c, const double* Ys, uint64_t seed, float* x, float* t,
                hipStream_t s);
int mlp_guess(const Mech& m, MlpImpl* p, int64_t n, const double* bY, const double* h,
              const double* c, double c_scalar, double* Y, int64_t ldy, int32_t* choice,
              hipStream_t s);
// sums int32 flags into *out (stream-ordered, one atomic per block)
int launch_count_flags(const int32_t* flags, int64_t n, unsigned long long* out, hipStream_t s);
// out[i] = c_scalar * (c ? c[i] : 1)
int launch_fill_c(int64_t n, const double* c, double c_scalar, double* out, hipStream_t s);

// ---- host SDC tables -------------------------------------------------------
struct Tables {
    int M = 0;
    double tau[MAX_NODES];
    double Q[MAX_NODES][MAX_NODES + 1];
    double QI[MAX_NODES][MAX_NODES];
    double QE[MAX_NODES][MAX_NODES];
    double S[MAX_NODES][MAX_NODES + 1];
};
int make_tables(int n_nodes, int qi_kind, int qe_mode, Tables& t);

}  // namespace misdc

// handles of the C ABI
struct misdc_mech_s {
    misdc::Mech m;
};

struct misdc_grid_s {
    misdc::Grid g;
};

struct misdc_mlp_s {
    misdc::MlpImpl* p = nullptr;
};
