// Persistent conjugate-gradient kernels of the implicit diffusion (steps
// S3/S4): shared definitions of the launcher and the kernels.
#pragma once

#include "misdc_impl.h"

namespace misdc {

constexpr int CG_THREADS = 256;
// block size of the register-resident CG: 512 threads with one cell each
// (2 waves per SIMD), 256 threads when each thread owns 2 or 4 cells
constexpr int cg_regs_block(int cpt) { return cpt == 1 ? 512 : 256; }
constexpr int CG_MAX_FIELDS = 64;
constexpr int CG_MAX_BLOCKS = 256;
constexpr int TILE_X = 32, TILE_Y = 16, TILE_BS = TILE_X * TILE_Y, TILE_NB = 128;
// grid-barrier words: [0] arrivals, [1] generation; the two-level barrier
// of the tiled kernel: BAR_GROUPS group counters at word BAR_STRIDE * (1 + g)
// and its count of arrived groups at BAR_GLOBAL, each on its own 128-byte
// line; BAR_EXIT counts the workgroups that have published the partial sums
// of the result's residual (the last one adds them up and zeroes it)
constexpr int BAR_GROUPS = 8, BAR_STRIDE = 32, BAR_GLOBAL = BAR_STRIDE * (1 + BAR_GROUPS),
              BAR_EXIT = BAR_GLOBAL + BAR_STRIDE, BAR_WORDS = BAR_EXIT + BAR_STRIDE;
// cells on the four sides of a tile (its edges, and the halo around it)
constexpr int TILE_HALO = 2 * TILE_X + 2 * TILE_Y;
// edge buffer of the tiled kernels: 2 (iteration parity) x tiles x 9 fields x TILE_HALO
constexpr size_t TILE_EDGE_DOUBLES = (size_t)2 * TILE_NB * 9 * TILE_HALO;

struct CGArgs {
    int64_t n;              // cells
    int nx, ny;
    int nf;                 // diffused fields (all but the bath)
    int fmap[CG_MAX_FIELDS];// field index of diffused field d
    double cf[CG_MAX_FIELDS];// c * kappa0_f
    const double* Kx;
    const double* Ky;
    const double* b;        // rhs (N+1 fields)
    double* x;              // solution (N+1 fields, bath untouched)
    double* r;
    double* z;
    double* p;
    double* q;
    double* partial;        // blocks x nf x 4
    double* edge;           // tiled variants: TILE_EDGE_DOUBLES
    double* totals;         // nf x 4 (written by the last block of a fused reduction)
    unsigned* bar;
    int32_t* info;          // [0] iterations, [1] failed, [2] barrier timeout
    double rtol2;
    int maxit;
    int guess_in_x;
    int ntx;                // tiled variant: tiles along x
    // tiled variants: the bath closure of the solution in the same launch
    // (close = 1): y_bath = r_bath - sum over the other species of (y_k - r_k),
    // then (optional) T and theta = (T/300)^1.7 of the closed state, and the
    // solve's statistics added to cgstats
    int close;
    int N, bath;
    int dmap[CG_MAX_FIELDS + 1];   // field -> diffused index (the bath: -1)
    const double* hf;
    const double* cp;
    const double* invW;
    double* T_out;
    double* th_out;
    int32_t* cgstats;       // [0] iterations, [1] max, [2] failures, [3] solves, [4] timeouts,
                            // [5] tiled variants: results whose true residual failed the check
    // tiled variants, lag_src set: the right-hand side is formed by the
    // kernel itself, each thread for its cell: b = lag_part + (qa FA(lag_src)
    // + qd FD(lag_src) + qr FR) of every field (theta of lag_src's T in
    // lag_th, or from lag_Tsrc; FR from lag_fr, may be null) is written to
    // b_w (= b), and the face coefficients come from theta of lag_T instead
    // of Kx, Ky; the guess must be in x
    const double* lag_src = nullptr;
    const double* lag_th = nullptr;
    const double* lag_Tsrc = nullptr;
    const double* lag_part = nullptr;
    const double* lag_fr = nullptr;
    const double* lag_T = nullptr;
    double lag_qa = 0.0, lag_qd = 0.0, lag_qr = 0.0;
    double* b_w = nullptr;
    const double* kappa0 = nullptr;   // N+1
    double dx = 0.0, dy = 0.0, ux = 0.0, uy = 0.0;
};

// launches the CG kernel of a variant (0 global memory, 1/2/4 register
// resident, 101..103 tiled) with ``blocks`` workgroups
int launch_cg(const CGArgs& a, int variant, int blocks, hipStream_t s);

}  // namespace misdc
