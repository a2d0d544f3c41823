// Learned initial guess of the per-cell reaction Newton solve: a dense
// network (N+2) -> H -> H -> (N+1) with ReLU hidden layers that maps the
// normalised reaction problem (b_Y, T_b, log c) to the normalised increment
// x* - (b_Y, T_b), trained on the GPU with its own kernels (forward,
// back-propagation of the mean squared error, Adam).  A cell takes the
// learned guess only when its FP64 residual |G| is below that of the plain
// guess, and Newton then runs unchanged, so the converged state is the one
// the plain guess leads to; only the iteration count can change.
//
// Every product runs on the matrix cores: BF16 operands with FP32
// accumulation (16x16x32 MFMA), or FP32 operands (16x16x4 MFMA) in the FP32
// mode.  One tiled GEMM kernel serves all of them: C = A B with arbitrary
// strides (transposed operands for the back-propagation), 128 x 128 output
// tiles per 256-thread workgroup (each wavefront 4 x 4 MFMA tiles), K staged
// through LDS in chunks of 32 with 16-byte loads along each operand's
// contiguous axis, an epilogue for bias, ReLU and the ReLU mask
// of the back-propagation, and a split-K mode whose partial sums are reduced
// in a fixed order (weight gradients over large batches).  Reductions never
// use atomics, so training is bitwise reproducible.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "misdc_impl.h"

namespace misdc {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename T> __device__ __forceinline__ T from_float(float v);
template <> __device__ __forceinline__ float from_float<float>(float v) { return v; }
template <> __device__ __forceinline__ uint16_t from_float<uint16_t>(float v) { return f2bf(v); }
__device__ __forceinline__ float to_float(float v) { return v; }
__device__ __forceinline__ float to_float(uint16_t v) { return bf2f(v); }

struct GemmArgs {
    int M, N, K;
    const void* A; int64_t sam, sak;       // A(m, k) = A[m sam + k sak]
    const void* B; int64_t sbk, sbn;       // B(k, n) = B[k sbk + n sbn]
    const float* bias;                     // [N] or null
    int relu;
    const void* mask; int64_t smm, smn;    // keep only where mask(m, n) > 0 (or null)
    float* outF; int64_t ldf;              // may be null
    void* outT; int64_t ldt;               // operand-typed copy, may be null
    float* part;                           // if set: raw sums to part[z M N + m N + n]
    int kchunk;                            // K range of one split
};

// Tile loads: 16-byte vectors along the operand's contiguous axis when the
// tile lies inside the matrix and the rows are 16-byte aligned, else one
// element at a time with zero padding.
constexpr int BM = 128, BN = 128, BK = 32, KP = BK + 8;    // LDS rows padded by 8 elements
static_assert(BK % 32 == 0, "whole 16x16x32 BF16 products per K chunk");

template <typename T>
__device__ __forceinline__ void load_tile(T (*S)[KP], const T* X, int64_t s_row, int64_t s_k,
                                          int r0, int rows, int k0, int k1, bool vec_ok) {
    constexpr int VE = 16 / sizeof(T);                     // elements per 16-byte vector
    const int tid = threadIdx.x;
    const bool kcont = (s_k == 1);
    const bool inside = (r0 + 128 <= rows) && (k0 + BK <= k1);
    if (vec_ok && inside) {
        if (kcont) {
            // 128 rows x BK: each vector covers VE consecutive k of one row
            constexpr int PER_ROW = BK / VE;
            for (int v = tid; v < 128 * PER_ROW; v += 256) {
                const int r = v / PER_ROW, kk = (v % PER_ROW) * VE;
                const uint4 q = *(const uint4*)(X + (int64_t)(r0 + r) * s_row + k0 + kk);
                *(uint4*)&S[r][kk] = q;
            }
        } else {
            // the row index is contiguous: each vector covers VE rows of one k
            constexpr int PER_K = 128 / VE;
            for (int v = tid; v < BK * PER_K; v += 256) {
                const int kk = v / PER_K, r = (v % PER_K) * VE;
                const uint4 q = *(const uint4*)(X + (int64_t)(k0 + kk) * s_k + r0 + r);
                const T* e = (const T*)&q;
#pragma unroll
                for (int u = 0; u < VE; ++u) S[r + u][kk] = e[u];
            }
        }
    } else {
        for (int v = tid; v < 128 * BK; v += 256) {
            const int r = kcont ? v / BK : v % 128;
            const int kk = kcont ? v % BK : v / 128;
            const int gr = r0 + r, gk = k0 + kk;
            S[r][kk] = (gr < rows && gk < k1) ? X[(int64_t)gr * s_row + (int64_t)gk * s_k]
                                              : from_float<T>(0.f);
        }
    }
}

// C = A B (+ epilogue): A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn];
// 128 x 128 tiles, four wavefronts of 64 x 64 (4 x 4 MFMA tiles of 16 x 16).
template <typename T>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) T As[BM][KP];     // [m][k]
    __shared__ __attribute__((aligned(16))) T Bt[BN][KP];     // [n][k]
    const T* A = (const T*)g.A;
    const T* B = (const T*)g.B;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kz0 = blockIdx.z * g.kchunk;
    const int kz1 = min(g.K, kz0 + g.kchunk);
    constexpr int VE = 16 / sizeof(T);
    // vector loads need 16-byte aligned rows along the contiguous axis
    const bool a_vec = (g.sak == 1 ? (g.sam % VE == 0) : (g.sam == 1 && g.sak % VE == 0)) &&
                       (((uintptr_t)A & 15) == 0);
    const bool b_vec = (g.sbk == 1 ? (g.sbn % VE == 0) : (g.sbn == 1 && g.sbk % VE == 0)) &&
                       (((uintptr_t)B & 15) == 0);
    const int wr = (wave / 2) * 64, wc = (wave % 2) * 64;
    const int li = lane % 16, lk = lane / 16;
    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};
    for (int k0 = kz0; k0 < kz1; k0 += BK) {
        load_tile<T>(As, A, g.sam, g.sak, m0, g.M, k0, kz1, a_vec);
        load_tile<T>(Bt, B, g.sbn, g.sbk, n0, g.N, k0, kz1, b_vec);
        __syncthreads();
        if constexpr (sizeof(T) == 2) {
#pragma unroll
            // gfx950's 16x16x32 BF16 product: each lane holds 8 consecutive k
            // of its row (A) or column (B); A and B put the same k in the same
            // slot, so the sum over the 32 slots is the dot product over k
            for (int ks = 0; ks < BK; ks += 32) {
                v8bf a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = *(const v8bf*)&As[wr + 16 * i + li][ks + 8 * lk];
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = *(const v8bf*)&Bt[wc + 16 * j + li][ks + 8 * lk];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < BK; ks += 4) {
                float a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = (float)As[wr + 16 * i + li][ks + lk];
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = (float)Bt[wc + 16 * j + li][ks + lk];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    const T* mask = (const T*)g.mask;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wr + 16 * i + 4 * lk + r;
                const int n = n0 + wc + 16 * j + li;
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][r];
                if (g.part) {
                    g.part[(int64_t)blockIdx.z * g.M * g.N + (int64_t)m * g.N + n] = v;
                    continue;
                }
                if (g.bias) v += g.bias[n];
                if (g.relu) v = fmaxf(v, 0.f);
                if (mask && !(to_float(mask[(int64_t)m * g.smm + (int64_t)n * g.smn]) > 0.f)) v = 0.f;
                if (g.outF) g.outF[(int64_t)m * g.ldf + n] = v;
                if (g.outT) ((T*)g.outT)[(int64_t)m * g.ldt + n] = from_float<T>(v);
            }
}

// out[i] = sum_z part[z][i] in order z = 0, 1, ...
__global__ void __launch_bounds__(256) reduce_parts_kernel(const float* part, int splits,
                                                           int64_t count, float* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * count + i];
    out[i] = s;
}

// column sums of dz over the rows [z rows_per, (z+1) rows_per) into
// part[z][n]: 64 columns x 4 row groups per workgroup, the groups summed in
// a fixed order
__global__ void __launch_bounds__(256) colsum_kernel(const float* dz, int64_t rows, int N,
                                                     int64_t rows_per, float* part) {
    __shared__ float red[4][64];
    const int c = threadIdx.x % 64, rg = threadIdx.x / 64;
    const int n = blockIdx.x * 64 + c;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per;
    const int64_t r1 = min(rows, r0 + rows_per);
    float s = 0.f;
    if (n < N)
        for (int64_t r = r0 + rg; r < r1; r += 4) s += dz[r * N + n];
    red[rg][c] = s;
    __syncthreads();
    if (rg == 0 && n < N)
        part[(int64_t)blockIdx.y * N + n] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// dz = scale (y - t); per-block sums of (y - t)^2 for the loss
template <typename T>
__global__ void __launch_bounds__(256) loss_grad_kernel(const float* y, const float* t, int64_t count,
                                                        float scale, float* dzF, T* dzT,
                                                        float* loss_part) {
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float sq = 0.f;
    if (i < count) {
        const float e = y[i] - t[i];
        const float d = scale * e;
        dzF[i] = d;
        dzT[i] = from_float<T>(d);
        sq = e * e;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// out = scale * sum of part[0 .. count): strided partial sums per thread,
// then a fixed tree over the workgroup
__global__ void __launch_bounds__(256) sum_kernel(const float* part, int count, float scale,
                                                  float* out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < count; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

template <typename T>
__global__ void __launch_bounds__(256) convert_kernel(const float* src, int64_t count, T* dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = from_float<T>(src[i]);
}

__global__ void __launch_bounds__(256) adam_kernel(float* w, uint16_t* wb, const float* g, float* m,
                                                   float* v, int64_t count, float lr, float b1,
                                                   float b2, float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
}

struct NormDev {
    const float* in_mu;   // n_in
    const float* in_sd;   // n_in
    const float* out_sd;  // n_out
};

__device__ __forceinline__ double cell_temperature(const MechDev& m, const double* Y, int64_t ld,
                                                   int64_t i, double h) {
    double hform = 0.0, cpm = 0.0;
    for (int k = 0; k < m.N; ++k) {
        const double y = Y[(int64_t)k * ld + i];
        hform += y * m.hf[k] * m.invW[k];
        cpm += y * m.cp[k] * m.invW[k];
    }
    return T_REF + (h - hform) / cpm;
}

// Output row of problem i: (pa i + pb) mod n, a bijection of [0, n) when
// gcd(pa, n) = 1 (pa = 1, pb = 0: the identity).
__device__ __forceinline__ int64_t out_row(int64_t i, int64_t n, uint64_t pa, uint64_t pb) {
    return (int64_t)(((uint64_t)i * pa + pb) % (uint64_t)n);
}

// x[row(i)] = ((b_Y - mu) / sd, (T_b - mu) / sd, (ln c - mu) / sd)
__global__ void __launch_bounds__(256) features_kernel(MechDev m, NormDev nd, int64_t n,
                                                       const double* bY, const double* h,
                                                       const double* c, double c_scalar,
                                                       float* x, uint64_t pa, uint64_t pb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int N = m.N, nin = N + 2;
    const double Tb = cell_temperature(m, bY, n, i, h[i]);
    const double cc = c ? c[i] * c_scalar : c_scalar;
    float* xi = x + out_row(i, n, pa, pb) * nin;
    for (int k = 0; k < N; ++k) xi[k] = (float)((bY[(int64_t)k * n + i] - nd.in_mu[k]) / nd.in_sd[k]);
    xi[N] = (float)((Tb - nd.in_mu[N]) / nd.in_sd[N]);
    xi[N + 1] = (float)((log(cc) - nd.in_mu[N + 1]) / nd.in_sd[N + 1]);
}

// t[row(i)] = ((Y* - b_Y) / sd, (T* - T_b) / sd)
__global__ void __launch_bounds__(256) targets_kernel(MechDev m, NormDev nd, int64_t n,
                                                      const double* bY, const double* h,
                                                      const double* Ys, float* t, uint64_t pa,
                                                      uint64_t pb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int N = m.N, nout = N + 1;
    const double Tb = cell_temperature(m, bY, n, i, h[i]);
    const double Ts = cell_temperature(m, Ys, n, i, h[i]);
    float* ti = t + out_row(i, n, pa, pb) * nout;
    for (int k = 0; k < N; ++k)
        ti[k] = (float)((Ys[(int64_t)k * n + i] - bY[(int64_t)k * n + i]) / nd.out_sd[k]);
    ti[N] = (float)((Ts - Tb) / nd.out_sd[N]);
}

// ---- statistics of a training set ------------------------------------------
// Raw (unnormalised) values of problem i in columns of R (Q = 2N + 3 columns
// of n): b_Y, T_b, ln c (the features), then Y* - b_Y, T* - T_b (the targets).
__global__ void __launch_bounds__(256) raw_pairs_kernel(MechDev m, int64_t n, const double* bY,
                                                        const double* h, const double* c,
                                                        const double* Ys, double* R) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int N = m.N;
    const double Tb = cell_temperature(m, bY, n, i, h[i]);
    const double Ts = cell_temperature(m, Ys, n, i, h[i]);
    for (int k = 0; k < N; ++k) {
        const double b = bY[(int64_t)k * n + i];
        R[(int64_t)k * n + i] = b;
        R[(int64_t)(N + 2 + k) * n + i] = Ys[(int64_t)k * n + i] - b;
    }
    R[(int64_t)N * n + i] = Tb;
    R[(int64_t)(N + 1) * n + i] = log(c[i]);
    R[(int64_t)(2 * N + 2) * n + i] = Ts - Tb;
}

constexpr int STAT_BLOCKS = 128;

// Partial column sums in a fixed order: block (b, q) sums v (mean == null) or
// (v - mean[q])^2 of column q over rows b*256 + t + k*STAT_BLOCKS*256 into
// part[q * STAT_BLOCKS + b].
__global__ void __launch_bounds__(256) column_sums_kernel(int64_t n, const double* R,
                                                          const double* mean, double* part) {
    __shared__ double red[256];
    const int q = blockIdx.y;
    const double mu = mean ? mean[q] : 0.0;
    const double* col = R + (int64_t)q * n;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)STAT_BLOCKS * 256) {
        const double v = col[i];
        acc += mean ? (v - mu) * (v - mu) : v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)q * STAT_BLOCKS + blockIdx.x] = red[0];
}

// Thread q totals its column's partials in block order.  Pass 0: mean[q].
// Pass 1: the normalisation: feature q < nin gets mu = mean and sd = the
// sample standard deviation (n - 1) floored at max(1e-3 |mu|, 1e-6), so that
// a constant feature stays O(1); target q gets sd floored at 1e-30.
__global__ void column_totals_kernel(int Q, int nin, int64_t n, const double* part, double* mean,
                                     int pass, float* norm) {
    const int q = threadIdx.x;
    if (q >= Q) return;
    double tot = 0.0;
    for (int b = 0; b < STAT_BLOCKS; ++b) tot += part[(int64_t)q * STAT_BLOCKS + b];
    if (pass == 0) {
        mean[q] = tot / (double)n;
        return;
    }
    const double sd = sqrt(tot / (double)(n - 1));
    const int nout = Q - nin;
    if (q < nin) {
        const double mu = mean[q];
        norm[q] = (float)mu;
        norm[nin + q] = (float)fmax(sd, fmax(1e-3 * fabs(mu), 1e-6));
    } else {
        norm[2 * nin + (q - nin)] = (float)fmax(sd, 1e-30);
    }
    (void)nout;
}

// learned candidate Y = b_Y + y sd, raised to min(b_Y, 0) where it falls
// below: the Newton iteration rejects every trial below that floor, so a
// start beneath it could never be left
__global__ void __launch_bounds__(256) candidate_kernel(int N, NormDev nd, int64_t n,
                                                        const double* bY, const float* y,
                                                        double* Yc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int nout = N + 1;
    for (int k = 0; k < N; ++k) {
        const double b = bY[(int64_t)k * n + i];
        const double v = b + (double)y[i * nout + k] * nd.out_sd[k];
        Yc[(int64_t)k * n + i] = fmax(v, fmin(b, 0.0));
    }
}

// per cell: keep the guess with the smaller |G|_2, G = Y - c FR(Y) - b_Y
__global__ void __launch_bounds__(256) select_kernel(int N, int64_t n, const double* bY,
                                                     const double* c, double c_scalar,
                                                     double* Y, int64_t ldy, const double* FRp,
                                                     const double* Yc, const double* FRc,
                                                     int32_t* choice) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double cc = c ? c[i] * c_scalar : c_scalar;
    double gp = 0.0, gc = 0.0;
    for (int k = 0; k < N; ++k) {
        const double b = bY[(int64_t)k * n + i];
        const double ep = Y[(int64_t)k * ldy + i] - cc * FRp[(int64_t)k * n + i] - b;
        const double ec = Yc[(int64_t)k * n + i] - cc * FRc[(int64_t)k * n + i] - b;
        gp += ep * ep;
        gc += ec * ec;
    }
    const bool take = (gc < gp);         // NaN in the candidate: keep the plain guess
    if (take)
        for (int k = 0; k < N; ++k) Y[(int64_t)k * ldy + i] = Yc[(int64_t)k * n + i];
    if (choice) choice[i] = take ? 1 : 0;
}

__global__ void __launch_bounds__(256) count_kernel(const int32_t* flags, int64_t n,
                                                    unsigned long long* out) {
    __shared__ unsigned red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    red[threadIdx.x] = (i < n && flags[i] != 0) ? 1u : 0u;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) atomicAdd(out, (unsigned long long)red[0]);
}

__global__ void __launch_bounds__(256) fill_c_kernel(int64_t n, const double* c, double cs,
                                                     double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = c ? c[i] * cs : cs;
}

inline unsigned grid_for(int64_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

}  // namespace

int launch_count_flags(const int32_t* flags, int64_t n, unsigned long long* out, hipStream_t s) {
    if (n == 0) return MISDC_OK;
    hipLaunchKernelGGL(count_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, flags, n, out);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int launch_fill_c(int64_t n, const double* c, double c_scalar, double* out, hipStream_t s) {
    if (n == 0) return MISDC_OK;
    hipLaunchKernelGGL(fill_c_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, n, c, c_scalar, out);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct MlpImpl {
    int dims[4] = {0, 0, 0, 0};
    int prec = 0;                       // 0 bf16, 1 fp32
    int device = 0;
    int64_t nparam = 0;
    int64_t off[6] = {0, 0, 0, 0, 0, 0};   // W1 b1 W2 b2 W3 b3 in the packed vector
    float* w = nullptr;                 // packed FP32 parameters
    uint16_t* wb = nullptr;             // packed BF16 copy
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;              // packed gradient (internal)
    int64_t t = 0;                      // Adam steps taken
    float* norm = nullptr;              // in_mu | in_sd | out_sd
    bool has_norm = false;
    // batch work buffers
    int64_t cap = 0;
    void* xT = nullptr;                 // operand-typed input
    float* h1F = nullptr; void* h1T = nullptr;
    float* h2F = nullptr; void* h2T = nullptr;
    float* y = nullptr;
    float* dz3F = nullptr; void* dz3T = nullptr;
    float* dz2F = nullptr; void* dz2T = nullptr;
    float* dz1F = nullptr; void* dz1T = nullptr;
    float* part = nullptr;              // split-K and column-sum partials
    float* loss_part = nullptr;
    float* loss = nullptr;
    // guess work (cells)
    int64_t gcap = 0;
    float* gx = nullptr;
    float* gy = nullptr;
    double* Yc = nullptr;
    double* FRp = nullptr;
    double* FRc = nullptr;
    std::vector<void*> batch_allocs, guess_allocs;
};

namespace {

constexpr int SPLITS = 32;
constexpr int64_t PART_FLOATS = (int64_t)SPLITS * 512 * 512;

size_t op_bytes(const MlpImpl& p) { return p.prec == 0 ? 2 : 4; }

NormDev norm_dev(const MlpImpl& p) {
    NormDev d;
    d.in_mu = p.norm;
    d.in_sd = p.norm + p.dims[0];
    d.out_sd = p.norm + 2 * p.dims[0];
    return d;
}

void free_list(std::vector<void*>& v) {
    for (void* q : v) (void)hipFree(q);
    v.clear();
}

int ensure_batch(MlpImpl& p, int64_t B) {
    if (B <= p.cap) return MISDC_OK;
    MISDC_HIP(hipDeviceSynchronize());
    free_list(p.batch_allocs);
    const int64_t H = p.dims[1] > p.dims[2] ? p.dims[1] : p.dims[2];
    const size_t ob = op_bytes(p);
    auto grab = [&](void** q, size_t bytes) -> int {
        hipError_t e = hipMalloc(q, bytes + 256);
        if (e != hipSuccess) return fail(MISDC_ENOMEM, "MLP work buffer: %s", hipGetErrorString(e));
        p.batch_allocs.push_back(*q);
        return MISDC_OK;
    };
    int rc = 0;
    if ((rc = grab(&p.xT, (size_t)B * p.dims[0] * ob))) return rc;
    if ((rc = grab((void**)&p.h1F, (size_t)B * H * 4))) return rc;
    if ((rc = grab(&p.h1T, (size_t)B * H * ob))) return rc;
    if ((rc = grab((void**)&p.h2F, (size_t)B * H * 4))) return rc;
    if ((rc = grab(&p.h2T, (size_t)B * H * ob))) return rc;
    if ((rc = grab((void**)&p.y, (size_t)B * p.dims[3] * 4))) return rc;
    if ((rc = grab((void**)&p.dz3F, (size_t)B * p.dims[3] * 4))) return rc;
    if ((rc = grab(&p.dz3T, (size_t)B * p.dims[3] * ob))) return rc;
    if ((rc = grab((void**)&p.dz2F, (size_t)B * H * 4))) return rc;
    if ((rc = grab(&p.dz2T, (size_t)B * H * ob))) return rc;
    if ((rc = grab((void**)&p.dz1F, (size_t)B * H * 4))) return rc;
    if ((rc = grab(&p.dz1T, (size_t)B * H * ob))) return rc;
    if ((rc = grab((void**)&p.part, (size_t)PART_FLOATS * 4))) return rc;
    if ((rc = grab((void**)&p.loss_part, (size_t)(B / 256 + 2) * p.dims[3] * 4 + 1024))) return rc;
    if ((rc = grab((void**)&p.loss, 64))) return rc;
    p.cap = B;
    return MISDC_OK;
}

int gemm(const MlpImpl& p, GemmArgs g, int splits, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.K <= 0) return MISDC_OK;
    if (splits > 1) {
        int64_t kc = (g.K + splits - 1) / splits;
        kc = (kc + BK - 1) / BK * BK;
        g.kchunk = (int)kc;
        splits = (int)((g.K + kc - 1) / kc);
        if ((int64_t)splits * g.M * g.N > PART_FLOATS) return fail(MISDC_EINVAL, "split-K partials too large");
    } else {
        g.kchunk = g.K;
        splits = 1;
    }
    const dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, splits);
    if (p.prec == 0)
        hipLaunchKernelGGL(gemm_kernel<uint16_t>, grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL(gemm_kernel<float>, grid, dim3(256), 0, s, g);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

GemmArgs gemm_args() {
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    return g;
}

// operand-typed weight of layer l (packed offsets)
const void* weight_op(const MlpImpl& p, int l) {
    return p.prec == 0 ? (const void*)(p.wb + p.off[2 * l]) : (const void*)(p.w + p.off[2 * l]);
}

// forward pass of B rows of x (operand-typed, B x dims[0]) into p.y
int forward(MlpImpl& p, int64_t B, hipStream_t s) {
    const void* in = p.xT;
    void* outsT[2] = {p.h1T, p.h2T};
    float* outsF[2] = {p.h1F, p.h2F};
    for (int l = 0; l < 3; ++l) {
        GemmArgs g = gemm_args();
        g.M = (int)B;
        g.N = p.dims[l + 1];
        g.K = p.dims[l];
        g.A = in; g.sam = p.dims[l]; g.sak = 1;
        g.B = weight_op(p, l); g.sbk = p.dims[l + 1]; g.sbn = 1;
        g.bias = p.w + p.off[2 * l + 1];
        if (l < 2) {
            g.relu = 1;
            g.outF = outsF[l]; g.ldf = p.dims[l + 1];
            g.outT = outsT[l]; g.ldt = p.dims[l + 1];
            in = outsT[l];
        } else {
            g.outF = p.y; g.ldf = p.dims[3];
        }
        int rc = gemm(p, g, 1, s);
        if (rc) return rc;
    }
    return MISDC_OK;
}

// x (FP32, B x dims[0]) -> operand type
int load_input(MlpImpl& p, int64_t B, const float* x, hipStream_t s) {
    const int64_t cnt = B * p.dims[0];
    if (p.prec == 0)
        hipLaunchKernelGGL(convert_kernel<uint16_t>, dim3(grid_for(cnt, 256)), dim3(256), 0, s, x, cnt,
                           (uint16_t*)p.xT);
    else
        hipLaunchKernelGGL(convert_kernel<float>, dim3(grid_for(cnt, 256)), dim3(256), 0, s, x, cnt,
                           (float*)p.xT);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

// gradients of the mean squared error into grad (packed), loss into p.loss
int backward(MlpImpl& p, int64_t B, const float* t, float* grad, hipStream_t s) {
    const int64_t cnt = B * p.dims[3];
    const float scale = 2.0f / (float)cnt;
    const unsigned nb = grid_for(cnt, 256);
    if (p.prec == 0)
        hipLaunchKernelGGL(loss_grad_kernel<uint16_t>, dim3(nb), dim3(256), 0, s, p.y, t, cnt, scale,
                           p.dz3F, (uint16_t*)p.dz3T, p.loss_part);
    else
        hipLaunchKernelGGL(loss_grad_kernel<float>, dim3(nb), dim3(256), 0, s, p.y, t, cnt, scale,
                           p.dz3F, (float*)p.dz3T, p.loss_part);
    MISDC_HIP(hipGetLastError());
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, p.loss_part, (int)nb, 1.0f / (float)cnt,
                       p.loss);
    MISDC_HIP(hipGetLastError());
    const void* actT[3] = {p.xT, p.h1T, p.h2T};
    float* dzF[3] = {p.dz1F, p.dz2F, p.dz3F};
    void* dzT[3] = {p.dz1T, p.dz2T, p.dz3T};
    for (int l = 2; l >= 0; --l) {
        const int fin = p.dims[l], fout = p.dims[l + 1];
        // dW_l = act_l^T dz_l (split over the batch), reduced in order
        GemmArgs g = gemm_args();
        g.M = fin; g.N = fout; g.K = (int)B;
        g.A = actT[l]; g.sam = 1; g.sak = fin;
        g.B = dzT[l]; g.sbk = fout; g.sbn = 1;
        g.part = p.part;
        int rc = gemm(p, g, SPLITS, s);
        if (rc) return rc;
        int64_t kc = (B + SPLITS - 1) / SPLITS;
        kc = (kc + BK - 1) / BK * BK;
        const int splits = (int)((B + kc - 1) / kc);
        const int64_t wc = (int64_t)fin * fout;
        hipLaunchKernelGGL(reduce_parts_kernel, dim3(grid_for(wc, 256)), dim3(256), 0, s, p.part,
                           splits, wc, grad + p.off[2 * l]);
        MISDC_HIP(hipGetLastError());
        // db_l = column sums of dz_l (row splits of 256)
        const int64_t rows_per = 256;
        const int csplits = (int)((B + rows_per - 1) / rows_per);
        if ((int64_t)csplits * fout > PART_FLOATS) return fail(MISDC_EINVAL, "batch too large");
        hipLaunchKernelGGL(colsum_kernel, dim3((fout + 63) / 64, csplits), dim3(256), 0, s,
                           dzF[l], B, fout, rows_per, p.part);
        MISDC_HIP(hipGetLastError());
        hipLaunchKernelGGL(reduce_parts_kernel, dim3(grid_for(fout, 256)), dim3(256), 0, s, p.part,
                           csplits, (int64_t)fout, grad + p.off[2 * l + 1]);
        MISDC_HIP(hipGetLastError());
        if (l == 0) break;
        // dz_{l-1} = (dz_l W_l^T) masked by act_l > 0
        GemmArgs d = gemm_args();
        d.M = (int)B; d.N = fin; d.K = fout;
        d.A = dzT[l]; d.sam = fout; d.sak = 1;
        d.B = weight_op(p, l); d.sbk = 1; d.sbn = fout;    // W_l^T (k = out, n = in)
        d.mask = actT[l]; d.smm = fin; d.smn = 1;
        d.outF = dzF[l - 1]; d.ldf = fin;
        d.outT = dzT[l - 1]; d.ldt = fin;
        rc = gemm(p, d, 1, s);
        if (rc) return rc;
    }
    return MISDC_OK;
}

int adam(MlpImpl& p, const float* grad, float lr, float b1, float b2, float eps, hipStream_t s) {
    p.t += 1;
    const float bc1 = 1.0f - powf(b1, (float)p.t);
    const float bc2 = 1.0f - powf(b2, (float)p.t);
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(p.nparam, 256)), dim3(256), 0, s, p.w, p.wb, grad,
                       p.m, p.v, p.nparam, lr, b1, b2, eps, bc1, bc2);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

}  // namespace

// --- entry points used by the C ABI and the integrator ---------------------
int mlp_create(int n_in, int n_hidden, int n_out, int prec, MlpImpl** out) {
    *out = nullptr;
    if (n_in < 1 || n_in > 512 || n_out < 1 || n_out > 512 || n_hidden < 1 || n_hidden > 512)
        return fail(MISDC_EINVAL, "layer widths must be in [1, 512]");
    if (prec != 0 && prec != 1) return fail(MISDC_EINVAL, "precision must be 0 (bf16) or 1 (fp32)");
    auto* p = new (std::nothrow) MlpImpl();
    if (!p) return fail(MISDC_ENOMEM, "host allocation failed");
    p->dims[0] = n_in;
    p->dims[1] = n_hidden;
    p->dims[2] = n_hidden;
    p->dims[3] = n_out;
    p->prec = prec;
    int64_t o = 0;
    for (int l = 0; l < 3; ++l) {
        p->off[2 * l] = o;
        o += (int64_t)p->dims[l] * p->dims[l + 1];
        p->off[2 * l + 1] = o;
        o += p->dims[l + 1];
    }
    p->nparam = o;
    hipError_t e = hipGetDevice(&p->device);
    const size_t nb = (size_t)o * 4 + 256;
    if (e == hipSuccess) e = hipMalloc(&p->w, nb);
    if (e == hipSuccess) e = hipMalloc(&p->wb, (size_t)o * 2 + 256);
    if (e == hipSuccess) e = hipMalloc(&p->m, nb);
    if (e == hipSuccess) e = hipMalloc(&p->v, nb);
    if (e == hipSuccess) e = hipMalloc(&p->grad, nb);
    if (e == hipSuccess) e = hipMalloc(&p->norm, (size_t)(2 * n_in + n_out) * 4 + 256);
    if (e == hipSuccess) e = hipMemset(p->w, 0, nb);
    if (e == hipSuccess) e = hipMemset(p->wb, 0, (size_t)o * 2 + 256);
    if (e == hipSuccess) e = hipMemset(p->m, 0, nb);
    if (e == hipSuccess) e = hipMemset(p->v, 0, nb);
    if (e != hipSuccess) {
        mlp_destroy(p);
        return fail(MISDC_EDEVICE, "MLP allocation: %s", hipGetErrorString(e));
    }
    // identity normalisation until set
    std::vector<float> nm(2 * n_in + n_out, 1.0f);
    for (int k = 0; k < n_in; ++k) nm[k] = 0.0f;
    e = hipMemcpy(p->norm, nm.data(), nm.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        mlp_destroy(p);
        return fail(MISDC_EDEVICE, "MLP normalisation: %s", hipGetErrorString(e));
    }
    *out = p;
    return MISDC_OK;
}

void mlp_destroy(MlpImpl* p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    free_list(p->batch_allocs);
    free_list(p->guess_allocs);
    void* q[] = {p->w, p->wb, p->m, p->v, p->grad, p->norm};
    for (void* x : q)
        if (x) (void)hipFree(x);
    delete p;
}

int64_t mlp_param_count(const MlpImpl* p) { return p->nparam; }
int mlp_dims(const MlpImpl* p, int l) { return p->dims[l]; }

int mlp_set_params(MlpImpl* p, const float* host) {
    MISDC_HIP(hipDeviceSynchronize());
    MISDC_HIP(hipMemcpy(p->w, host, (size_t)p->nparam * 4, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(convert_kernel<uint16_t>, dim3(grid_for(p->nparam, 256)), dim3(256), 0, 0, p->w,
                       p->nparam, p->wb);
    MISDC_HIP(hipGetLastError());
    MISDC_HIP(hipMemset(p->m, 0, (size_t)p->nparam * 4));
    MISDC_HIP(hipMemset(p->v, 0, (size_t)p->nparam * 4));
    p->t = 0;
    MISDC_HIP(hipDeviceSynchronize());
    return MISDC_OK;
}

int mlp_get_params(MlpImpl* p, float* host) {
    MISDC_HIP(hipDeviceSynchronize());
    MISDC_HIP(hipMemcpy(host, p->w, (size_t)p->nparam * 4, hipMemcpyDeviceToHost));
    return MISDC_OK;
}

int mlp_set_norm(MlpImpl* p, const float* in_mu, const float* in_sd, const float* out_sd) {
    for (int k = 0; k < p->dims[0]; ++k)
        if (!(in_sd[k] > 0) || !std::isfinite(in_mu[k]))
            return fail(MISDC_EINVAL, "input scale %d must be positive", k);
    for (int k = 0; k < p->dims[3]; ++k)
        if (!(out_sd[k] > 0)) return fail(MISDC_EINVAL, "output scale %d must be positive", k);
    std::vector<float> nm;
    nm.insert(nm.end(), in_mu, in_mu + p->dims[0]);
    nm.insert(nm.end(), in_sd, in_sd + p->dims[0]);
    nm.insert(nm.end(), out_sd, out_sd + p->dims[3]);
    MISDC_HIP(hipDeviceSynchronize());
    MISDC_HIP(hipMemcpy(p->norm, nm.data(), nm.size() * 4, hipMemcpyHostToDevice));
    p->has_norm = true;
    return MISDC_OK;
}

int mlp_reserve(MlpImpl* p, int64_t cells) {
    int rc = ensure_batch(*p, cells);
    if (rc) return rc;
    if (cells > p->gcap) {
        MISDC_HIP(hipDeviceSynchronize());
        free_list(p->guess_allocs);
        const int N = p->dims[3] - 1;
        auto grab = [&](void** q, size_t bytes) -> int {
            hipError_t e = hipMalloc(q, bytes + 256);
            if (e != hipSuccess) return fail(MISDC_ENOMEM, "MLP guess buffer: %s", hipGetErrorString(e));
            p->guess_allocs.push_back(*q);
            return MISDC_OK;
        };
        if ((rc = grab((void**)&p->gx, (size_t)cells * p->dims[0] * 4))) return rc;
        if ((rc = grab((void**)&p->gy, (size_t)cells * p->dims[3] * 4))) return rc;
        if ((rc = grab((void**)&p->Yc, (size_t)cells * N * 8))) return rc;
        if ((rc = grab((void**)&p->FRp, (size_t)cells * N * 8))) return rc;
        if ((rc = grab((void**)&p->FRc, (size_t)cells * N * 8))) return rc;
        p->gcap = cells;
    }
    return MISDC_OK;
}

int mlp_forward(MlpImpl* p, int64_t B, const float* x, float* y, hipStream_t s) {
    if (B == 0) return MISDC_OK;
    int rc = ensure_batch(*p, B);
    if (rc) return rc;
    if ((rc = load_input(*p, B, x, s))) return rc;
    if ((rc = forward(*p, B, s))) return rc;
    MISDC_HIP(hipMemcpyAsync(y, p->y, (size_t)B * p->dims[3] * 4, hipMemcpyDeviceToDevice, s));
    return MISDC_OK;
}

int mlp_gradients(MlpImpl* p, int64_t B, const float* x, const float* t, float* grad, float* loss,
                  hipStream_t s) {
    if (B == 0) return fail(MISDC_EINVAL, "empty batch");
    int rc = ensure_batch(*p, B);
    if (rc) return rc;
    if ((rc = load_input(*p, B, x, s))) return rc;
    if ((rc = forward(*p, B, s))) return rc;
    if ((rc = backward(*p, B, t, grad, s))) return rc;
    if (loss) MISDC_HIP(hipMemcpyAsync(loss, p->loss, 4, hipMemcpyDeviceToDevice, s));
    return MISDC_OK;
}

int mlp_adam(MlpImpl* p, const float* grad, float lr, float b1, float b2, float eps, hipStream_t s) {
    return adam(*p, grad, lr, b1, b2, eps, s);
}

int mlp_train(MlpImpl* p, int64_t n, const float* x, const float* t, int64_t batch, int epochs,
              float lr, float* loss_hist, hipStream_t s) {
    if (batch < 1 || batch > n) return fail(MISDC_EINVAL, "batch must be in [1, n]");
    int rc = ensure_batch(*p, batch);
    if (rc) return rc;
    const int64_t nb = n / batch;       // whole minibatches, in order
    for (int e = 0; e < epochs; ++e) {
        for (int64_t b = 0; b < nb; ++b) {
            const float* xb = x + b * batch * p->dims[0];
            const float* tb = t + b * batch * p->dims[3];
            if ((rc = load_input(*p, batch, xb, s))) return rc;
            if ((rc = forward(*p, batch, s))) return rc;
            if ((rc = backward(*p, batch, tb, p->grad, s))) return rc;
            if ((rc = adam(*p, p->grad, lr, 0.9f, 0.999f, 1e-8f, s))) return rc;
            if (loss_hist && b == nb - 1)
                MISDC_HIP(hipMemcpyAsync(loss_hist + e, p->loss, 4, hipMemcpyDeviceToDevice, s));
        }
    }
    return MISDC_OK;
}

int mlp_features(const Mech& m, MlpImpl* p, int64_t n, const double* bY, const double* h,
                 const double* c, double c_scalar, float* x, hipStream_t s) {
    if (p->dims[0] != m.dev.N + 2 || p->dims[3] != m.dev.N + 1)
        return fail(MISDC_EINVAL, "network widths %d -> %d do not match %d species", p->dims[0],
                    p->dims[3], m.dev.N);
    if (n == 0) return MISDC_OK;
    hipLaunchKernelGGL(features_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, m.dev, norm_dev(*p),
                       n, bY, h, c, c_scalar, x, (uint64_t)1, (uint64_t)0);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

int mlp_targets(const Mech& m, MlpImpl* p, int64_t n, const double* bY, const double* h,
                const double* Ys, float* t, hipStream_t s) {
    if (p->dims[0] != m.dev.N + 2 || p->dims[3] != m.dev.N + 1)
        return fail(MISDC_EINVAL, "network widths do not match the mechanism");
    if (n == 0) return MISDC_OK;
    hipLaunchKernelGGL(targets_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, m.dev, norm_dev(*p),
                       n, bY, h, Ys, t, (uint64_t)1, (uint64_t)0);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

namespace {
uint64_t splitmix64(uint64_t& z) {
    uint64_t r = (z += 0x9E3779B97F4A7C15ull);
    r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
    r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
    return r ^ (r >> 31);
}
uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}
}  // namespace

int mlp_prepare(const Mech& m, MlpImpl* p, int64_t n, const double* bY, const double* h,
                const double* c, const double* Ys, uint64_t seed, float* x, float* t,
                hipStream_t s) {
    const int N = m.dev.N, nin = N + 2, Q = 2 * N + 3;
    if (p->dims[0] != nin || p->dims[3] != N + 1)
        return fail(MISDC_EINVAL, "network widths do not match the mechanism");
    if (n < 2) return fail(MISDC_EINVAL, "at least two training problems are needed");
    if (Q > 1024) return fail(MISDC_EUNSUPPORTED, "too many species for the statistics kernel");
    // the shuffle: row i -> (pa i + pb) mod n with pa coprime to n
    uint64_t z = seed;
    uint64_t pa = 1 + splitmix64(z) % (uint64_t)(n - 1);
    while (gcd64(pa, (uint64_t)n) != 1) pa = pa % (uint64_t)(n - 1) + 1;
    const uint64_t pb = splitmix64(z) % (uint64_t)n;
    double* R = nullptr;
    double* work = nullptr;
    MISDC_HIP(hipMallocAsync((void**)&R, sizeof(double) * (size_t)Q * n, s));
    hipError_t e = hipMallocAsync((void**)&work, sizeof(double) * ((size_t)Q * STAT_BLOCKS + Q), s);
    if (e != hipSuccess) {
        (void)hipFreeAsync(R, s);
        return fail(MISDC_ENOMEM, "training statistics: %s", hipGetErrorString(e));
    }
    double* part = work;
    double* mean = work + (size_t)Q * STAT_BLOCKS;
    hipLaunchKernelGGL(raw_pairs_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, m.dev, n, bY, h, c,
                       Ys, R);
    hipLaunchKernelGGL(column_sums_kernel, dim3(STAT_BLOCKS, Q), dim3(256), 0, s, n, R,
                       (const double*)nullptr, part);
    hipLaunchKernelGGL(column_totals_kernel, dim3(1), dim3(1024), 0, s, Q, nin, n, part, mean, 0,
                       p->norm);
    hipLaunchKernelGGL(column_sums_kernel, dim3(STAT_BLOCKS, Q), dim3(256), 0, s, n, R, mean, part);
    hipLaunchKernelGGL(column_totals_kernel, dim3(1), dim3(1024), 0, s, Q, nin, n, part, mean, 1,
                       p->norm);
    hipLaunchKernelGGL(features_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, m.dev, norm_dev(*p),
                       n, bY, h, c, 1.0, x, pa, pb);
    hipLaunchKernelGGL(targets_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, m.dev, norm_dev(*p),
                       n, bY, h, Ys, t, pa, pb);
    e = hipGetLastError();
    (void)hipFreeAsync(work, s);
    (void)hipFreeAsync(R, s);
    if (e != hipSuccess) return fail(MISDC_EDEVICE, "training set: %s", hipGetErrorString(e));
    p->has_norm = true;
    return MISDC_OK;
}

// Y (N fields, stride ldy) holds the plain guess on entry and the chosen one
// on exit.
int mlp_guess(const Mech& m, MlpImpl* p, int64_t n, const double* bY, const double* h,
              const double* c, double c_scalar, double* Y, int64_t ldy, int32_t* choice,
              hipStream_t s) {
    if (n == 0) return MISDC_OK;
    if (p->dims[0] != m.dev.N + 2 || p->dims[3] != m.dev.N + 1)
        return fail(MISDC_EINVAL, "network widths do not match the mechanism");
    const int N = m.dev.N;
    if (n > p->gcap || n > p->cap) {
        int rc0 = mlp_reserve(p, n);
        if (rc0) return rc0;
    }
    int rc = mlp_features(m, p, n, bY, h, c, c_scalar, p->gx, s);
    if (rc) return rc;
    if ((rc = load_input(*p, n, p->gx, s))) return rc;
    if ((rc = forward(*p, n, s))) return rc;
    hipLaunchKernelGGL(candidate_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, N, norm_dev(*p), n,
                       bY, p->y, p->Yc);
    MISDC_HIP(hipGetLastError());
    if (ldy != n) return fail(MISDC_EINVAL, "guess array must have stride n");
    if ((rc = launch_reaction_source(m, n, Y, h, p->FRp, s))) return rc;
    if ((rc = launch_reaction_source(m, n, p->Yc, h, p->FRc, s))) return rc;
    hipLaunchKernelGGL(select_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, N, n, bY, c, c_scalar,
                       Y, ldy, p->FRp, p->Yc, p->FRc, choice);
    MISDC_HIP(hipGetLastError());
    return MISDC_OK;
}

}  // namespace misdc

using misdc::fail;

extern "C" {

int misdc_mlp_create(int n_in, int n_hidden, int n_out, int precision, misdc_mlp_t* out) {
    if (!out) return fail(MISDC_EINVAL, "output handle pointer is NULL");
    *out = nullptr;
    auto* h = new (std::nothrow) misdc_mlp_s();
    if (!h) return fail(MISDC_ENOMEM, "host allocation failed");
    int rc = misdc::mlp_create(n_in, n_hidden, n_out, precision, &h->p);
    if (rc) {
        delete h;
        return rc;
    }
    *out = h;
    return MISDC_OK;
}

int misdc_mlp_destroy(misdc_mlp_t mlp) {
    if (!mlp) return MISDC_OK;
    misdc::mlp_destroy(mlp->p);
    delete mlp;
    return MISDC_OK;
}

int misdc_mlp_param_count(misdc_mlp_t mlp, int64_t* count) {
    if (!mlp || !count) return fail(MISDC_EINVAL, "NULL argument");
    *count = misdc::mlp_param_count(mlp->p);
    return MISDC_OK;
}

int misdc_mlp_set_params(misdc_mlp_t mlp, const float* host_params) {
    if (!mlp || !host_params) return fail(MISDC_EINVAL, "NULL argument");
    return misdc::mlp_set_params(mlp->p, host_params);
}

int misdc_mlp_get_params(misdc_mlp_t mlp, float* host_params) {
    if (!mlp || !host_params) return fail(MISDC_EINVAL, "NULL argument");
    return misdc::mlp_get_params(mlp->p, host_params);
}

int misdc_mlp_set_normalization(misdc_mlp_t mlp, const float* in_mu, const float* in_sd,
                                const float* out_sd) {
    if (!mlp || !in_mu || !in_sd || !out_sd) return fail(MISDC_EINVAL, "NULL argument");
    return misdc::mlp_set_norm(mlp->p, in_mu, in_sd, out_sd);
}

int misdc_mlp_forward(misdc_mlp_t mlp, int64_t batch, const float* dev_x, float* dev_y, void* stream) {
    if (!mlp) return fail(MISDC_EINVAL, "network is NULL");
    if (batch < 0) return fail(MISDC_EINVAL, "batch < 0");
    if (batch > 0 && (!dev_x || !dev_y)) return fail(MISDC_EINVAL, "NULL array");
    return misdc::mlp_forward(mlp->p, batch, dev_x, dev_y, (hipStream_t)stream);
}

int misdc_mlp_gradients(misdc_mlp_t mlp, int64_t batch, const float* dev_x, const float* dev_t,
                        float* dev_grad, float* dev_loss, void* stream) {
    if (!mlp) return fail(MISDC_EINVAL, "network is NULL");
    if (batch < 1) return fail(MISDC_EINVAL, "batch must be >= 1");
    if (!dev_x || !dev_t || !dev_grad) return fail(MISDC_EINVAL, "NULL array");
    return misdc::mlp_gradients(mlp->p, batch, dev_x, dev_t, dev_grad, dev_loss, (hipStream_t)stream);
}

int misdc_mlp_adam_step(misdc_mlp_t mlp, const float* dev_grad, float lr, float beta1, float beta2,
                        float eps, void* stream) {
    if (!mlp || !dev_grad) return fail(MISDC_EINVAL, "NULL argument");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(MISDC_EINVAL, "invalid Adam parameters");
    return misdc::mlp_adam(mlp->p, dev_grad, lr, beta1, beta2, eps, (hipStream_t)stream);
}

int misdc_mlp_train(misdc_mlp_t mlp, int64_t n, const float* dev_x, const float* dev_t,
                    int64_t batch, int epochs, float lr, float* dev_loss, void* stream) {
    if (!mlp) return fail(MISDC_EINVAL, "network is NULL");
    if (n < 1 || !dev_x || !dev_t) return fail(MISDC_EINVAL, "empty or NULL training set");
    if (epochs < 1 || !(lr > 0)) return fail(MISDC_EINVAL, "epochs >= 1 and lr > 0 required");
    return misdc::mlp_train(mlp->p, n, dev_x, dev_t, batch, epochs, lr, dev_loss, (hipStream_t)stream);
}

int misdc_mlp_features(misdc_mech_t mech, misdc_mlp_t mlp, int64_t n, const double* dev_bY,
                       const double* dev_h, const double* dev_c, float* dev_x, void* stream) {
    if (!mech || !mlp) return fail(MISDC_EINVAL, "NULL handle");
    if (n < 0) return fail(MISDC_EINVAL, "n < 0");
    if (n > 0 && (!dev_bY || !dev_h || !dev_c || !dev_x)) return fail(MISDC_EINVAL, "NULL array");
    return misdc::mlp_features(mech->m, mlp->p, n, dev_bY, dev_h, dev_c, 1.0, dev_x,
                               (hipStream_t)stream);
}

int misdc_mlp_targets(misdc_mech_t mech, misdc_mlp_t mlp, int64_t n, const double* dev_bY,
                      const double* dev_h, const double* dev_Y, float* dev_t, void* stream) {
    if (!mech || !mlp) return fail(MISDC_EINVAL, "NULL handle");
    if (n < 0) return fail(MISDC_EINVAL, "n < 0");
    if (n > 0 && (!dev_bY || !dev_h || !dev_Y || !dev_t)) return fail(MISDC_EINVAL, "NULL array");
    return misdc::mlp_targets(mech->m, mlp->p, n, dev_bY, dev_h, dev_Y, dev_t, (hipStream_t)stream);
}

int misdc_mlp_prepare_training(misdc_mech_t mech, misdc_mlp_t mlp, int64_t n, const double* dev_bY,
                               const double* dev_h, const double* dev_c, const double* dev_Y,
                               uint64_t seed, float* dev_x, float* dev_t, void* stream) {
    if (!mech || !mlp) return fail(MISDC_EINVAL, "NULL handle");
    if (n < 2 || n > ((int64_t)1 << 31)) return fail(MISDC_EINVAL, "n must be in [2, 2^31]");
    if (!dev_bY || !dev_h || !dev_c || !dev_Y || !dev_x || !dev_t)
        return fail(MISDC_EINVAL, "NULL array");
    return misdc::mlp_prepare(mech->m, mlp->p, n, dev_bY, dev_h, dev_c, dev_Y, seed, dev_x, dev_t,
                              (hipStream_t)stream);
}

int misdc_reaction_guess_mlp(misdc_mech_t mech, misdc_mlp_t mlp, int64_t n, const double* dev_bY,
                             const double* dev_h, const double* dev_c, double* dev_Y,
                             int32_t* dev_choice, void* stream) {
    if (!mech || !mlp) return fail(MISDC_EINVAL, "NULL handle");
    if (n < 0) return fail(MISDC_EINVAL, "n < 0");
    if (n > 0 && (!dev_bY || !dev_h || !dev_c || !dev_Y)) return fail(MISDC_EINVAL, "NULL array");
    return misdc::mlp_guess(mech->m, mlp->p, n, dev_bY, dev_h, dev_c, 1.0, dev_Y, n, dev_choice,
                            (hipStream_t)stream);
}

}  // extern "C"
