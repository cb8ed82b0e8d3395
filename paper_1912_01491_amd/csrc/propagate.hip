// RK4 integration of dv/dt = Q v + K (Eq. (10); Table 1 step 3.1).
//
// Classic fourth-order Runge-Kutta with constant K:
//   k1 = f(v), k2 = f(v + h/2 k1), k3 = f(v + h/2 k2), k4 = f(v + h k3),
//   v <- v + h/6 (k1 + 2 k2 + 2 k3 + k4),   f(x) = Q x + K.
// Every stage streams Q once, so the integrator is bound by HBM bandwidth for
// a few states and by the matrix cores for many.
//
// Dense paths (per stage):
//   * B = 1: k_gemv -- one wavefront per group of rows, lanes along the row,
//     cross-lane reduction, stage combine fused into the same kernel.
//   * B >= 2: k_gemm64 / k_gemm32 -- split-K GEMM on the matrix cores
//     (v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32) writing per-slab
//     partial sums, followed by k_stage which reduces the slabs in a fixed
//     order (deterministic, no atomics) and applies the RK4 combination.
//   * M <= 256 and B*M <= 4096: k_rk4_small -- one workgroup per system runs
//     all steps with Q and the stage vectors in LDS.
// State layout inside the library: states are padded to Bp in {16, 32, 64}
// columns and stored "pair-interleaved", X[(k>>1)*2Bp + 2b + (k&1)], so that
// the 16-byte load a lane issues holds two consecutive k of one state -- the
// B-operand of two MFMAs whose A-operand is the two consecutive Q columns the
// same lane loaded. The FP32 path interleaves by four.
#include <mutex>

#include "lb_internal.h"
#include "rowdot.h"
#include "sell.h"

#include <math.h>

#include <algorithm>
#include <cstring>
#include <stdio.h>
#include <stdlib.h>

typedef double lb_double4 __attribute__((ext_vector_type(4)));
typedef float lb_float4 __attribute__((ext_vector_type(4)));
typedef unsigned int lb_u4 __attribute__((ext_vector_type(4)));

namespace {

__host__ __device__ __forceinline__ int64_t ilv2(int64_t k, int b, int Bp) { return (k >> 1) * (2 * Bp) + 2 * b + (k & 1); }
__host__ __device__ __forceinline__ int64_t ilv4(int64_t k, int b, int Bp) { return (k >> 2) * (4 * Bp) + 4 * b + (k & 3); }

// Work decomposition of a stage GEMM launch: gx row blocks x nslab k-slabs x R
// systems, launched as a 1-D grid. Workgroups are handed to the 8 XCDs round
// robin by workgroup id, so workgroup b runs on XCD b % 8; it is given work item
// w = (b % 8) * per_xcd + b / 8, i.e. each XCD walks one contiguous range of
// the slab-major work list and keeps the few X slabs it is reading resident in
// its own L2.
struct GemmGrid {
    int gx, nslab, R;
    int64_t per_xcd;
};

__device__ __forceinline__ bool gemm_work(const GemmGrid& g, int& x, int& slab, int& r) {
    const int64_t b = blockIdx.x;
    const int64_t w = (b & 7) * g.per_xcd + (b >> 3);
    if (w >= (int64_t)g.gx * g.nslab * g.R) return false;
    x = (int)(w % g.gx);
    const int64_t cmb = w / g.gx;
    slab = (int)(cmb % g.nslab);
    r = (int)(cmb / g.nslab);
    return true;
}

// ---------------------------------------------------------------------------
// Matrix-core stage GEMM, FP64: Part[slab] = Q[:, slab] X[slab, :]
// ---------------------------------------------------------------------------
// A wave owns RT row tiles of 16 rows and CT column tiles of 16 states over one
// k-slab. Lane l loads Q[row0 + 16t + (l%16)][kc + 2(l/16) + {0,1}] (16 bytes)
// and X[kc + 2(l/16) + {0,1}][16c + (l%16)]; the MFMA k-index j = l/16 maps to
// column kc + 2j (first MFMA) and kc + 2j + 1 (second).
template <int RT, int CT, bool ALIGNED>
__global__ __launch_bounds__(256) void k_gemm64(const double* const* Qs, int64_t M, int64_t Mp, int64_t ldq,
                                                const double* Xall, int64_t xstride, double* Pall,
                                                int64_t pstride, int kslab, GemmGrid gg) {
    constexpr int Bp = 16 * CT;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    int bx, slab, r;
    if (!gemm_work(gg, bx, slab, r)) return;
    const double* Q = Qs[r];
    const double* X = Xall + r * xstride;
    double* Part = Pall + r * pstride + (int64_t)slab * Mp * Bp;
    const int64_t row0 = ((int64_t)bx * (blockDim.x >> 6) + wave) * (16 * RT);
    if (row0 >= M) return;
    const int64_t k0 = (int64_t)slab * kslab;
    const int64_t k1 = k0 + kslab < M ? k0 + kslab : M;

    const double* qrow[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        int64_t row = row0 + 16 * t + lr;
        row = row < M ? row : M - 1;
        qrow[t] = Q + row * ldq;
    }
    lb_double4 acc[RT][CT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = lb_double4{0, 0, 0, 0};

    int64_t kc = k0;
    for (; kc + 16 <= k1; kc += 16) {
        double2 qa[RT], qb[RT], xa[CT], xb[CT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const double* p = qrow[t] + kc + 2 * lk;
            if (ALIGNED) {
                qa[t] = *reinterpret_cast<const double2*>(p);
                qb[t] = *reinterpret_cast<const double2*>(p + 8);
            } else {
                qa[t] = make_double2(p[0], p[1]);
                qb[t] = make_double2(p[8], p[9]);
            }
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            xa[c] = *reinterpret_cast<const double2*>(X + ((kc >> 1) + lk) * (2 * Bp) + 2 * (16 * c + lr));
            xb[c] = *reinterpret_cast<const double2*>(X + (((kc + 8) >> 1) + lk) * (2 * Bp) + 2 * (16 * c + lr));
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[t].x, xa[c].x, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[t].y, xa[c].y, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(qb[t].x, xb[c].x, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(qb[t].y, xb[c].y, acc[t][c], 0, 0, 0);
            }
    }
    if (kc < k1) {  // ragged tail: guarded scalar loads, zero beyond M
        double qa[RT][4], xa[CT][4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int64_t k = kc + 2 * lk + (h & 1) + 8 * (h >> 1);
            const bool ok = k < k1;
#pragma unroll
            for (int t = 0; t < RT; ++t) qa[t][h] = ok ? qrow[t][k] : 0.0;
#pragma unroll
            for (int c = 0; c < CT; ++c) xa[c][h] = ok ? X[ilv2(k, 16 * c + lr, Bp)] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int h = 0; h < 4; ++h)
                    acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[t][h], xa[c][h], acc[t][c], 0, 0, 0);
    }
    // D layout of v_mfma_f64_16x16x4f64: lane l, element j -> row 4j + l/16,
    // column l%16 (the FP32 variant below uses row 4(l/16) + j)
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = row0 + 16 * t + 4 * j + lk;
                if (row < M) Part[ilv2(row, 16 * c + lr, Bp)] = acc[t][c][j];
            }
}

// ---------------------------------------------------------------------------
// Matrix-core stage GEMM, FP32 operands: Q32 and X32 in FP32, FP32 products and
// accumulation within a k-slab, FP64 partial sums across slabs.
// ---------------------------------------------------------------------------
template <int RT, int CT, bool ALIGNED>
__global__ __launch_bounds__(256) void k_gemm32(const float* const* Qs, int64_t M, int64_t Mp, int64_t ldq,
                                                const float* Xall, int64_t xstride, double* Pall,
                                                int64_t pstride, int kslab, GemmGrid gg) {
    constexpr int Bp = 16 * CT;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    int bx, slab, r;
    if (!gemm_work(gg, bx, slab, r)) return;
    const float* Q = Qs[r];
    const float* X = Xall + r * xstride;
    double* Part = Pall + r * pstride + (int64_t)slab * Mp * Bp;
    const int64_t row0 = ((int64_t)bx * (blockDim.x >> 6) + wave) * (16 * RT);
    if (row0 >= M) return;
    const int64_t k0 = (int64_t)slab * kslab;
    const int64_t k1 = k0 + kslab < M ? k0 + kslab : M;

    const float* qrow[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        int64_t row = row0 + 16 * t + lr;
        row = row < M ? row : M - 1;
        qrow[t] = Q + row * ldq;
    }
    lb_float4 acc[RT][CT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = lb_float4{0, 0, 0, 0};

    // 32 columns (128 bytes of each row) per iteration, as two 16-byte loads per
    // lane: columns kc + 4(l/16) + {0..3} and kc + 16 + 4(l/16) + {0..3}
    int64_t kc = k0;
    for (; kc + 32 <= k1; kc += 32) {
        float4 qa[RT], qb[RT], xa[CT], xb[CT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const float* p = qrow[t] + kc + 4 * lk;
            if (ALIGNED) {
                qa[t] = *reinterpret_cast<const float4*>(p);
                qb[t] = *reinterpret_cast<const float4*>(p + 16);
            } else {
                qa[t] = make_float4(p[0], p[1], p[2], p[3]);
                qb[t] = make_float4(p[16], p[17], p[18], p[19]);
            }
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            xa[c] = *reinterpret_cast<const float4*>(X + ((kc >> 2) + lk) * (4 * Bp) + 4 * (16 * c + lr));
            xb[c] = *reinterpret_cast<const float4*>(X + (((kc + 16) >> 2) + lk) * (4 * Bp) + 4 * (16 * c + lr));
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].x, xa[c].x, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].y, xa[c].y, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].z, xa[c].z, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].w, xa[c].w, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qb[t].x, xb[c].x, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qb[t].y, xb[c].y, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qb[t].z, xb[c].z, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qb[t].w, xb[c].w, acc[t][c], 0, 0, 0);
            }
    }
    for (; kc + 16 <= k1; kc += 16) {
        float4 qa[RT], xa[CT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const float* p = qrow[t] + kc + 4 * lk;
            if (ALIGNED) qa[t] = *reinterpret_cast<const float4*>(p);
            else qa[t] = make_float4(p[0], p[1], p[2], p[3]);
        }
#pragma unroll
        for (int c = 0; c < CT; ++c)
            xa[c] = *reinterpret_cast<const float4*>(X + ((kc >> 2) + lk) * (4 * Bp) + 4 * (16 * c + lr));
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].x, xa[c].x, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].y, xa[c].y, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].z, xa[c].z, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].w, xa[c].w, acc[t][c], 0, 0, 0);
            }
    }
    if (kc < k1) {
        float qa[RT][4], xa[CT][4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int64_t k = kc + 4 * lk + h;
            const bool ok = k < k1;
#pragma unroll
            for (int t = 0; t < RT; ++t) qa[t][h] = ok ? qrow[t][k] : 0.0f;
#pragma unroll
            for (int c = 0; c < CT; ++c) xa[c][h] = ok ? X[ilv4(k, 16 * c + lr, Bp)] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int h = 0; h < 4; ++h)
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t][h], xa[c][h], acc[t][c], 0, 0, 0);
    }
    // D layout of v_mfma_f32_16x16x4f32: lane l, element j -> row 4(l/16) + j
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = row0 + 16 * t + 4 * lk + j;
                if (row < M) Part[ilv2(row, 16 * c + lr, Bp)] = (double)acc[t][c][j];
            }
}

// ---------------------------------------------------------------------------
// LDS-staged variants of the two stage GEMMs (rows of Q 128-byte aligned).
// ---------------------------------------------------------------------------
// The matrix-core A operand wants lane l to hold row l%16 of a 16-row tile, so
// a direct 16-byte load per lane touches 16 rows per quarter-wave and splits
// every 128-byte line of Q between two load instructions. Here a wave instead
// reads its 16*RT rows x 128 bytes (16 FP64 / 32 FP32 columns) as 2*RT loads of
// 8 complete lines (lane L: row L/8 of the group, 16-byte piece (L%8) ^ (L/8)),
// with the nontemporal hint since Q is streamed once per stage, writes the
// pieces to a wave-private LDS buffer (slot g*64 + L), and reads the operands
// back in the matrix-core layout: row r, piece c sits in slot
// (r/8)*64 + (r%8)*8 + (c ^ (r%8)), which keeps each group of 8 lanes of a
// 16-byte LDS read on distinct banks. Two chunks of loads are kept in flight.
// The columns each MFMA consumes are the same as in the direct kernels, so the
// results are bit-identical to theirs.

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-lane byte offsets (from the wave's first row) of the lane's 16-byte piece
// in each of the 2*RT groups of 8 rows; rows past M re-read row M-1.
template <int G>
__device__ __forceinline__ void stage_offsets(uint32_t (&off)[G], int64_t row0, int64_t M, int64_t rowbytes,
                                              int lane) {
    const int wr = lane >> 3, wc = (lane & 7) ^ wr;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        int64_t row = row0 + 8 * g + wr;
        row = row < M ? row : M - 1;
        off[g] = (uint32_t)((row - row0) * rowbytes + 16 * wc);
    }
}

typedef const lb_u4 __attribute__((address_space(1)))* lb_gu4;

template <int G>
__device__ __forceinline__ void stage_load(lb_u4 (&q)[G], const char* p, const uint32_t (&off)[G]) {
#pragma unroll
    for (int g = 0; g < G; ++g) q[g] = __builtin_nontemporal_load((lb_gu4)(p + off[g]));
}

// The B operand (states) of one chunk for CT column tiles, loaded together with
// the chunk's Q so that waiting for it never waits for a later prefetch.
template <int CT>
__device__ __forceinline__ void stage_xload(lb_u4 (&xa)[CT], lb_u4 (&xb)[CT], const char* x0, const char* x1) {
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        xa[c] = *(lb_gu4)(x0 + 256 * c);
        xb[c] = *(lb_gu4)(x1 + 256 * c);
    }
}

template <int G>
__device__ __forceinline__ void stage_put(lb_u4* lds, const lb_u4 (&q)[G], int lane) {
#pragma unroll
    for (int g = 0; g < G; ++g) lds[g * 64 + lane] = q[g];
}

template <int RT, int CT>
__global__ __launch_bounds__(256) void k_gemm64s(const double* const* Qs, int64_t M, int64_t Mp, int64_t ldq,
                                                 const double* Xall, int64_t xstride, double* Pall,
                                                 int64_t pstride, int kslab, GemmGrid gg) {
    extern __shared__ lb_u4 stage_lds[];
    constexpr int Bp = 16 * CT;
    constexpr int G = 2 * RT;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    int bx, slab, r;
    if (!gemm_work(gg, bx, slab, r)) return;
    const double* Q = Qs[r];
    const double* X = Xall + r * xstride;
    double* Part = Pall + r * pstride + (int64_t)slab * Mp * Bp;
    const int64_t row0 = ((int64_t)bx * (blockDim.x >> 6) + wave) * (16 * RT);
    if (row0 >= M) return;
    const int64_t k0 = (int64_t)slab * kslab;
    const int64_t k1 = k0 + kslab < M ? k0 + kslab : M;
    lb_u4* lds = stage_lds + wave * (G * 64);
    const char* qbase = reinterpret_cast<const char*>(Q + row0 * ldq);
    uint32_t off[G];
    stage_offsets<G>(off, row0, M, ldq * 8, lane);
    const int rr = lr & 7;
    const int s0 = (lr >> 3) * 64 + rr * 8 + (lk ^ rr);

    lb_double4 acc[RT][CT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = lb_double4{0, 0, 0, 0};

    // X of chunk kc for column tile c: lane's double2 at ((kc>>1) + lk)*2Bp + 2(16c + lr); the
    // chunk's second half (columns kc+8..) starts 4*2Bp doubles later.
    const char* xlane = reinterpret_cast<const char*>(X + lk * (2 * Bp) + 2 * lr);
    auto xaddr = [&](int64_t kc) { return xlane + (kc >> 1) * (2 * Bp) * 8; };
    auto mma = [&](const lb_u4 (&xa)[CT], const lb_u4 (&xb)[CT]) {
        lb_double2v qa[RT], qb[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            qa[t] = __builtin_bit_cast(lb_double2v, lds[128 * t + s0]);
            qb[t] = __builtin_bit_cast(lb_double2v, lds[(128 * t + s0) ^ 4]);
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const lb_double2v x0 = __builtin_bit_cast(lb_double2v, xa[c]);
                const lb_double2v x1 = __builtin_bit_cast(lb_double2v, xb[c]);
                acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[t].x, x0.x, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[t].y, x0.y, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(qb[t].x, x1.x, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(qb[t].y, x1.y, acc[t][c], 0, 0, 0);
            }
    };

    // two chunks in flight: (qA, xA) holds chunk j, (qB, xB) chunk j+1
    const int64_t nch = (k1 - k0) / 16;
    lb_u4 qA[G], qB[G], xA0[CT], xA1[CT], xB0[CT], xB1[CT];
    // the scheduling barriers keep each chunk's loads where they are issued here,
    // ahead of the next chunk's, instead of next to their first use
    auto fetch = [&](lb_u4 (&q)[G], lb_u4 (&x0)[CT], lb_u4 (&x1)[CT], int64_t kc) {
        __builtin_amdgcn_sched_barrier(0);
        stage_xload<CT>(x0, x1, xaddr(kc), xaddr(kc + 8));
        stage_load<G>(q, qbase + kc * 8, off);
        __builtin_amdgcn_sched_barrier(0);
    };
    // Every pass issues both prefetches (chunk indices past the end re-read the
    // last chunk), so the same loads are in flight at every loop iteration.
    auto kcl = [&](int64_t ch) { return k0 + 16 * (ch < nch ? ch : nch - 1); };
    if (nch > 0) {
        fetch(qA, xA0, xA1, kcl(0));
        fetch(qB, xB0, xB1, kcl(1));
        int64_t j = 0;
        for (; j + 1 < nch; j += 2) {
            stage_put<G>(lds, qA, lane);
            wave_lds_fence();
            mma(xA0, xA1);
            wave_lds_fence();
            fetch(qA, xA0, xA1, kcl(j + 2));
            stage_put<G>(lds, qB, lane);
            wave_lds_fence();
            mma(xB0, xB1);
            wave_lds_fence();
            fetch(qB, xB0, xB1, kcl(j + 3));
        }
        if (j < nch) {
            stage_put<G>(lds, qA, lane);
            wave_lds_fence();
            mma(xA0, xA1);
            wave_lds_fence();
        }
    }
    const int64_t kc = k0 + 16 * nch;
    if (kc < k1) {  // ragged tail: guarded scalar loads, zero beyond M
        double qa[RT][4], xa[CT][4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int64_t k = kc + 2 * lk + (h & 1) + 8 * (h >> 1);
            const bool ok = k < k1;
#pragma unroll
            for (int t = 0; t < RT; ++t) {
                int64_t row = row0 + 16 * t + lr;
                row = row < M ? row : M - 1;
                qa[t][h] = ok ? Q[row * ldq + k] : 0.0;
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) xa[c][h] = ok ? X[ilv2(k, 16 * c + lr, Bp)] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int h = 0; h < 4; ++h)
                    acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[t][h], xa[c][h], acc[t][c], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = row0 + 16 * t + 4 * j + lk;
                if (row < M) Part[ilv2(row, 16 * c + lr, Bp)] = acc[t][c][j];
            }
}

template <int RT, int CT>
__global__ __launch_bounds__(256) void k_gemm32s(const float* const* Qs, int64_t M, int64_t Mp, int64_t ldq,
                                                 const float* Xall, int64_t xstride, double* Pall,
                                                 int64_t pstride, int kslab, GemmGrid gg) {
    extern __shared__ lb_u4 stage_lds[];
    constexpr int Bp = 16 * CT;
    constexpr int G = 2 * RT;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    int bx, slab, r;
    if (!gemm_work(gg, bx, slab, r)) return;
    const float* Q = Qs[r];
    const float* X = Xall + r * xstride;
    double* Part = Pall + r * pstride + (int64_t)slab * Mp * Bp;
    const int64_t row0 = ((int64_t)bx * (blockDim.x >> 6) + wave) * (16 * RT);
    if (row0 >= M) return;
    const int64_t k0 = (int64_t)slab * kslab;
    const int64_t k1 = k0 + kslab < M ? k0 + kslab : M;
    lb_u4* lds = stage_lds + wave * (G * 64);
    const char* qbase = reinterpret_cast<const char*>(Q + row0 * ldq);
    uint32_t off[G];
    stage_offsets<G>(off, row0, M, ldq * 4, lane);
    const int rr = lr & 7;
    const int s0 = (lr >> 3) * 64 + rr * 8 + (lk ^ rr);

    lb_float4 acc[RT][CT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[t][c] = lb_float4{0, 0, 0, 0};

    // X of chunk kc for column tile c: lane's float4 at ((kc>>2) + lk)*4Bp + 4(16c + lr); the
    // chunk's second half (columns kc+16..) starts 4*4Bp floats later.
    const char* xlane = reinterpret_cast<const char*>(X + lk * (4 * Bp) + 4 * lr);
    auto xaddr = [&](int64_t kc) { return xlane + (kc >> 2) * (4 * Bp) * 4; };
    auto mma = [&](const lb_u4 (&xa)[CT], const lb_u4 (&xb)[CT]) {
        lb_float4 qa[RT], qb[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            qa[t] = __builtin_bit_cast(lb_float4, lds[128 * t + s0]);
            qb[t] = __builtin_bit_cast(lb_float4, lds[(128 * t + s0) ^ 4]);
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const lb_float4 x0 = __builtin_bit_cast(lb_float4, xa[c]);
                const lb_float4 x1 = __builtin_bit_cast(lb_float4, xb[c]);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].x, x0.x, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].y, x0.y, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].z, x0.z, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].w, x0.w, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qb[t].x, x1.x, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qb[t].y, x1.y, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qb[t].z, x1.z, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qb[t].w, x1.w, acc[t][c], 0, 0, 0);
            }
    };

    const int64_t nch = (k1 - k0) / 32;
    lb_u4 qA[G], qB[G], xA0[CT], xA1[CT], xB0[CT], xB1[CT];
    auto fetch = [&](lb_u4 (&q)[G], lb_u4 (&x0)[CT], lb_u4 (&x1)[CT], int64_t kc) {
        __builtin_amdgcn_sched_barrier(0);
        stage_xload<CT>(x0, x1, xaddr(kc), xaddr(kc + 16));
        stage_load<G>(q, qbase + kc * 4, off);
        __builtin_amdgcn_sched_barrier(0);
    };
    // Every pass issues both prefetches (chunk indices past the end re-read the
    // last chunk), so the same loads are in flight at every loop iteration.
    auto kcl = [&](int64_t ch) { return k0 + 32 * (ch < nch ? ch : nch - 1); };
    if (nch > 0) {
        fetch(qA, xA0, xA1, kcl(0));
        fetch(qB, xB0, xB1, kcl(1));
        int64_t j = 0;
        for (; j + 1 < nch; j += 2) {
            stage_put<G>(lds, qA, lane);
            wave_lds_fence();
            mma(xA0, xA1);
            wave_lds_fence();
            fetch(qA, xA0, xA1, kcl(j + 2));
            stage_put<G>(lds, qB, lane);
            wave_lds_fence();
            mma(xB0, xB1);
            wave_lds_fence();
            fetch(qB, xB0, xB1, kcl(j + 3));
        }
        if (j < nch) {
            stage_put<G>(lds, qA, lane);
            wave_lds_fence();
            mma(xA0, xA1);
            wave_lds_fence();
        }
    }
    // remainder (< 32 columns, last slab only): direct loads as in k_gemm32
    const float* qrow[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) {
        int64_t row = row0 + 16 * t + lr;
        row = row < M ? row : M - 1;
        qrow[t] = Q + row * ldq;
    }
    int64_t kc = k0 + 32 * nch;
    if (kc + 16 <= k1) {
        float4 qa[RT], xa[CT];
#pragma unroll
        for (int t = 0; t < RT; ++t) qa[t] = *reinterpret_cast<const float4*>(qrow[t] + kc + 4 * lk);
#pragma unroll
        for (int c = 0; c < CT; ++c)
            xa[c] = *reinterpret_cast<const float4*>(X + ((kc >> 2) + lk) * (4 * Bp) + 4 * (16 * c + lr));
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].x, xa[c].x, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].y, xa[c].y, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].z, xa[c].z, acc[t][c], 0, 0, 0);
                acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t].w, xa[c].w, acc[t][c], 0, 0, 0);
            }
        kc += 16;
    }
    if (kc < k1) {
        float qa[RT][4], xa[CT][4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int64_t k = kc + 4 * lk + h;
            const bool ok = k < k1;
#pragma unroll
            for (int t = 0; t < RT; ++t) qa[t][h] = ok ? qrow[t][k] : 0.0f;
#pragma unroll
            for (int c = 0; c < CT; ++c) xa[c][h] = ok ? X[ilv4(k, 16 * c + lr, Bp)] : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < RT; ++t)
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int h = 0; h < 4; ++h)
                    acc[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[t][h], xa[c][h], acc[t][c], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = row0 + 16 * t + 4 * lk + j;
                if (row < M) Part[ilv2(row, 16 * c + lr, Bp)] = (double)acc[t][c][j];
            }
}

// ---------------------------------------------------------------------------
// Stage combine: k_i = sum_slab Part + K, then the RK4 update of that stage.
// ---------------------------------------------------------------------------
struct StageArgs {
    const double* const* Ks;
    double* V;       // + r*sstride
    double* Acc;
    double* X;
    float* X32;      // may be null
    int64_t sstride; // per-system stride of V/Acc/X (doubles)
    int64_t s32stride;
    const double* Part;
    int64_t pstride;
    int nslab;
    int64_t M, Mp;
    int Bp;
    double dt;
};

__global__ void k_stage(StageArgs a, int stage) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (row, b) in row-major
    const int r = blockIdx.y;
    if (e >= a.M * a.Bp) return;
    const int64_t row = e / a.Bp;
    const int b = (int)(e % a.Bp);
    const int64_t idx = ilv2(row, b, a.Bp);
    const double* part = a.Part + r * a.pstride + idx;
    double k = 0.0;
    for (int s = 0; s < a.nslab; ++s) k += part[(int64_t)s * a.Mp * a.Bp];
    k += a.Ks[r][row];
    double* V = a.V + r * a.sstride;
    double* Acc = a.Acc + r * a.sstride;
    double* X = a.X + r * a.sstride;
    const double h = a.dt;
    double x;
    if (stage == 1) {
        Acc[idx] = k;
        x = V[idx] + 0.5 * h * k;
    } else if (stage == 2) {
        Acc[idx] = Acc[idx] + 2.0 * k;
        x = V[idx] + 0.5 * h * k;
    } else if (stage == 3) {
        Acc[idx] = Acc[idx] + 2.0 * k;
        x = V[idx] + h * k;
    } else {
        x = V[idx] + h / 6.0 * (Acc[idx] + k);
        V[idx] = x;
    }
    X[idx] = x;
    if (a.X32) a.X32[r * a.s32stride + ilv4(row, b, a.Bp)] = (float)x;
}

// user layout (B, M) -> interleaved padded (Mp, Bp); padding rows/columns zero
__global__ void k_pack(const double* const* Vu, int64_t M, int64_t Mp, int B, int Bp, double* V, double* X,
                       float* X32, int64_t sstride, int64_t s32stride) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (e >= Mp * Bp) return;
    const int64_t row = e / Bp;
    const int b = (int)(e % Bp);
    const double v = (row < M && b < B) ? Vu[r][(int64_t)b * M + row] : 0.0;
    const int64_t idx = ilv2(row, b, Bp);
    V[r * sstride + idx] = v;
    X[r * sstride + idx] = v;
    if (X32) X32[r * s32stride + ilv4(row, b, Bp)] = (float)v;
}

__global__ void k_unpack(double* const* Vu, int64_t M, int B, int Bp, const double* V, int64_t sstride) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (e >= M * B) return;
    const int b = (int)(e / M);
    const int64_t row = e % M;
    Vu[r][e] = V[r * sstride + ilv2(row, b, Bp)];
}

// ---------------------------------------------------------------------------
// One state: GEMV with the stage combine fused in (rows are complete per wave).
// A wave owns R rows; lanes read 16 bytes each along the row, so one load
// instruction covers 1 KB of a row (full lines when rows are 128-byte aligned,
// then read with the nontemporal hint: Q is streamed once per stage). A row's
// sum does not depend on R, so R only trades waves for loads in flight.
// ---------------------------------------------------------------------------
template <int R, bool ALIGNED, bool NT>
__global__ __launch_bounds__(256) void k_gemv(const double* const* Qs, const double* const* Ks,
                                              double* const* Vs, int64_t M, int64_t ldq, double* Wall,
                                              int64_t wstride, int stage, double h) {
    // W layout per system: [Acc | Xa | Xb], each Ma = M rounded up to 32
    // doubles; stage i reads X from Xa when i is odd and Xb when even, and
    // writes the other one.
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int r = blockIdx.y;
    const int64_t row0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * R;
    if (row0 >= M) return;
    const double* Q = Qs[r];
    double* W = Wall + r * wstride;
    const int64_t Ma = (M + 31) / 32 * 32;
    double* Acc = W;
    const double* Xin = (stage & 1) ? W + Ma : W + 2 * Ma;
    double* Xout = (stage & 1) ? W + 2 * Ma : W + Ma;
    double acc[R];
    const double* qrow[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        int64_t row = row0 + t;
        qrow[t] = Q + (row < M ? row : M - 1) * ldq;
    }
    wave_rowdots<R, ALIGNED, NT>(qrow, Xin, M, lane, acc);
    if (lane < R) {
        double kv = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t)
            if (t == lane) kv = acc[t];
        const int64_t row = row0 + lane;
        if (row < M) {
            const double k = kv + Ks[r][row];
            double* V = Vs[r];
            double x;
            if (stage == 1) {
                Acc[row] = k;
                x = V[row] + 0.5 * h * k;
            } else if (stage == 2) {
                Acc[row] = Acc[row] + 2.0 * k;
                x = V[row] + 0.5 * h * k;
            } else if (stage == 3) {
                Acc[row] = Acc[row] + 2.0 * k;
                x = V[row] + h * k;
            } else {
                x = V[row] + h / 6.0 * (Acc[row] + k);
                V[row] = x;
            }
            Xout[row] = x;
        }
    }
}

__global__ void k_gemv_init(double* const* Vs, int64_t M, double* Wall, int64_t wstride) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (e >= M) return;
    Wall[r * wstride + (M + 31) / 32 * 32 + e] = Vs[r][e];  // Xa = v
}

// ---------------------------------------------------------------------------
// Small systems: one workgroup integrates one system for all steps.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rk4_small(const double* const* Qs, const double* const* Ks,
                                                   double* const* Vs, int M, int64_t ldq, int B, double h,
                                                   int64_t steps, int q_in_lds) {
    extern __shared__ double sm[];
    const int r = blockIdx.x;
    const double* Qg = Qs[r];
    const double* K = Ks[r];
    double* V = Vs[r];
    const int n = M * B;
    double* X = sm;           // B x M
    double* Acc = sm + n;     // B x M
    double* Ql = sm + 2 * n;  // M x M (optional)
    for (int e = threadIdx.x; e < n; e += blockDim.x) X[e] = V[e];
    if (q_in_lds)
        for (int e = threadIdx.x; e < M * M; e += blockDim.x) Ql[e] = Qg[(int64_t)(e / M) * ldq + e % M];
    __syncthreads();
    const double* Q = q_in_lds ? Ql : Qg;
    const int64_t lq = q_in_lds ? M : ldq;
    for (int64_t st = 0; st < steps; ++st) {
        for (int stage = 1; stage <= 4; ++stage) {
            double kv[16];
            int cnt = 0;
            for (int e = threadIdx.x; e < n; e += blockDim.x) {
                const int b = e / M, i = e % M;
                const double* q = Q + (int64_t)i * lq;
                const double* x = X + b * M;
                double s = 0.0;
                for (int j = 0; j < M; ++j) s = fma(q[j], x[j], s);
                kv[cnt++] = s + K[i];
            }
            __syncthreads();
            cnt = 0;
            for (int e = threadIdx.x; e < n; e += blockDim.x) {
                const double k = kv[cnt++];
                double x;
                if (stage == 1) {
                    Acc[e] = k;
                    x = V[e] + 0.5 * h * k;
                } else if (stage == 2) {
                    Acc[e] = Acc[e] + 2.0 * k;
                    x = V[e] + 0.5 * h * k;
                } else if (stage == 3) {
                    Acc[e] = Acc[e] + 2.0 * k;
                    x = V[e] + h * k;
                } else {
                    x = V[e] + h / 6.0 * (Acc[e] + k);
                    V[e] = x;
                }
                X[e] = x;
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// Sparse RK4 stage: one launch per stage with the stage combination fused in,
// over the slice layout of sell.h (one wavefront per 64-row slice, one block of
// 256 threads per long row).
// ---------------------------------------------------------------------------

// RK4 stage combination for one element, given k = (Q x + K)_i and the values
// of v and of the accumulator loaded beforehand.
__device__ __forceinline__ void rk4_update(int stage, double h, double k, double v, double acc, int64_t i, double* V,
                                           double* Acc, double* Xout) {
    double x;
    if (stage == 1) {
        Acc[i] = k;
        x = v + 0.5 * h * k;
    } else if (stage == 2) {
        Acc[i] = acc + 2.0 * k;
        x = v + 0.5 * h * k;
    } else if (stage == 3) {
        Acc[i] = acc + 2.0 * k;
        x = v + h * k;
    } else {
        x = v + h / 6.0 * (acc + k);
        V[i] = x;
    }
    Xout[i] = x;
}

// The stage vectors of a sparse integration.
struct SellStage {
    int B;
    const double* K;
    double* V;
    double* W;  // [accumulator | x ping | x pong], M*B each
};

// DRIVE: k = (Q0 x) + eps (Q1 x) + K, the two sums formed separately.
// SB: states per pass over a slice (1, or 4 for batches).
template <bool DRIVE, int SB>
__global__ __launch_bounds__(256) void k_sell_stage(SellMat a, SellStage st, int stage, double h, double eps) {
    const int64_t M = a.M;
    const int64_t n = M * st.B;
    double* Acc = st.W;
    const double* Xin = (stage & 1) ? st.W + n : st.W + 2 * n;
    double* Xout = (stage & 1) ? st.W + 2 * n : st.W + n;
    const int wk = sell_work(a);
    if (wk < 0) return;
    if (wk < a.nlong) {
        const int64_t row = a.longrows[wk];
        for (int b = 0; b < st.B; ++b) {
            double q0, q1;
            block_row_dots<DRIVE>(a, row, Xin + (int64_t)b * M, q0, q1);
            if (threadIdx.x == 0) {
                const int64_t i = (int64_t)b * M + row;
                double k = q0;
                if (DRIVE) k += eps * q1;
                k += st.K[row];
                rk4_update(stage, h, k, st.V[i], stage > 1 ? Acc[i] : 0.0, i, st.V, Acc, Xout);
            }
        }
        return;
    }
    // one slice per wavefront; the slice index is wave-uniform
    const int sl = __builtin_amdgcn_readfirstlane((wk - a.nlong) * 4 + (int)(threadIdx.x >> 6));
    if (sl >= a.S) return;
    const int lane = threadIdx.x & (kSlice - 1);
    const int64_t r = (int64_t)sl * kSlice + lane;
    const bool mine = r < M && !((a.lmask[sl] >> lane) & 1);
    const int64_t o0 = a.off0[sl];
    const int w0 = (int)((a.off0[sl + 1] - o0) / kSlice);
    const int* c0 = a.scol0 + o0 + lane;
    const double* v0 = a.sval0 + o0 + lane;
    int w1 = 0;
    const int* c1 = nullptr;
    const double* v1 = nullptr;
    if (DRIVE) {
        const int64_t o1 = a.off1[sl];
        w1 = (int)((a.off1[sl + 1] - o1) / kSlice);
        c1 = a.scol1 + o1 + lane;
        v1 = a.sval1 + o1 + lane;
    }
    const double kr = mine ? st.K[r] : 0.0;
    for (int b0 = 0; b0 < st.B; b0 += SB) {
        const int nb = min(SB, st.B - b0);
        double vv[SB], aa[SB], acc[SB], accd[SB];
#pragma unroll
        for (int j = 0; j < SB; ++j) {
            vv[j] = aa[j] = acc[j] = accd[j] = 0.0;
            if (j < nb && mine) {
                const int64_t i = (int64_t)(b0 + j) * M + r;
                vv[j] = st.V[i];
                if (stage > 1) aa[j] = Acc[i];
            }
        }
        const double* xb = Xin + (int64_t)b0 * M;
        sell_row<SB>(c0, v0, w0, xb, M, nb, acc);
        if (DRIVE) sell_row<SB>(c1, v1, w1, xb, M, nb, accd);
#pragma unroll
        for (int j = 0; j < SB; ++j)
            if (j < nb && mine) {
                double k = acc[j];
                if (DRIVE) k += eps * accd[j];
                rk4_update(stage, h, k + kr, vv[j], aa[j], (int64_t)(b0 + j) * M + r, st.V, Acc, Xout);
            }
    }
}

__global__ void k_copy(const double* src, double* dst, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) dst[e] = src[e];
}

__global__ void k_to_f32(const double* Q, float* Q32, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) Q32[e] = (float)Q[e];
}

// ---------------------------------------------------------------------------
// Kernel selection
// ---------------------------------------------------------------------------

typedef void (*gemm64_fn)(const double* const*, int64_t, int64_t, int64_t, const double*, int64_t, double*,
                          int64_t, int, GemmGrid);
typedef void (*gemm32_fn)(const float* const*, int64_t, int64_t, int64_t, const float*, int64_t, double*,
                          int64_t, int, GemmGrid);

template <bool AL>
gemm64_fn pick64(int RT, int CT) {
    if (CT == 1) {
        if (RT == 1) return k_gemm64<1, 1, AL>;
        if (RT == 2) return k_gemm64<2, 1, AL>;
        if (RT == 4) return k_gemm64<4, 1, AL>;
        if (RT == 8) return k_gemm64<8, 1, AL>;
    } else if (CT == 2) {
        if (RT == 1) return k_gemm64<1, 2, AL>;
        if (RT == 2) return k_gemm64<2, 2, AL>;
        if (RT == 4) return k_gemm64<4, 2, AL>;
    } else if (CT == 4) {
        if (RT == 1) return k_gemm64<1, 4, AL>;
        if (RT == 2) return k_gemm64<2, 4, AL>;
        if (RT == 4) return k_gemm64<4, 4, AL>;
    }
    return nullptr;
}

template <bool AL>
gemm32_fn pick32(int RT, int CT) {
    if (CT == 1) {
        if (RT == 1) return k_gemm32<1, 1, AL>;
        if (RT == 2) return k_gemm32<2, 1, AL>;
        if (RT == 4) return k_gemm32<4, 1, AL>;
        if (RT == 8) return k_gemm32<8, 1, AL>;
    } else if (CT == 2) {
        if (RT == 1) return k_gemm32<1, 2, AL>;
        if (RT == 2) return k_gemm32<2, 2, AL>;
        if (RT == 4) return k_gemm32<4, 2, AL>;
    } else if (CT == 4) {
        if (RT == 1) return k_gemm32<1, 4, AL>;
        if (RT == 2) return k_gemm32<2, 4, AL>;
        if (RT == 4) return k_gemm32<4, 4, AL>;
    }
    return nullptr;
}

gemm64_fn pick64s(int RT, int CT) {
    if (CT == 1) {
        if (RT == 1) return k_gemm64s<1, 1>;
        if (RT == 2) return k_gemm64s<2, 1>;
        if (RT == 4) return k_gemm64s<4, 1>;
    } else if (CT == 2) {
        if (RT == 1) return k_gemm64s<1, 2>;
        if (RT == 2) return k_gemm64s<2, 2>;
        if (RT == 4) return k_gemm64s<4, 2>;
    } else if (CT == 4) {
        if (RT == 1) return k_gemm64s<1, 4>;
        if (RT == 2) return k_gemm64s<2, 4>;
        if (RT == 4) return k_gemm64s<4, 4>;
    }
    return nullptr;
}

gemm32_fn pick32s(int RT, int CT) {
    if (CT == 1) {
        if (RT == 1) return k_gemm32s<1, 1>;
        if (RT == 2) return k_gemm32s<2, 1>;
        if (RT == 4) return k_gemm32s<4, 1>;
    } else if (CT == 2) {
        if (RT == 1) return k_gemm32s<1, 2>;
        if (RT == 2) return k_gemm32s<2, 2>;
        if (RT == 4) return k_gemm32s<4, 2>;
    } else if (CT == 4) {
        if (RT == 1) return k_gemm32s<1, 4>;
        if (RT == 2) return k_gemm32s<2, 4>;
        if (RT == 4) return k_gemm32s<4, 4>;
    }
    return nullptr;
}

int bpad(int B) { return B <= 16 ? 16 : (B <= 32 ? 32 : 64); }

}  // namespace

// Default tile from sweeps on MI355X (LDS-staged kernels): 64 rows per wave for
// 16-state blocks (32 rows, one wave per block for 32/64 states), and k-slabs
// sized so that one system alone gives about 2500 row-waves x slabs (5000 for
// 32/64 states): long slabs keep the streaming loads of a wave going, and at
// N = 200 a single system still fills the chip. Slabs are a multiple of 32
// columns (128 bytes of FP32, 256 of FP64) so that every slab starts on a line,
// and at least 256 (384 for 64 states) long. The slab length fixes the
// summation order, so it depends on (M, Bp) only and never on the precision
// or on how many systems share a launch: a system's result is bit-identical
// alone and batched.
lb_tile lb_default_tile(int64_t M, int Bp, int precision, int R) {
    lb_tile t;
    const int CT = Bp / 16;
    t.rows = CT == 1 ? 64 : 32;
    t.waves = CT == 1 ? 2 : 1;
    (void)R;
    (void)precision;
    const int64_t rowwaves = (M + t.rows - 1) / t.rows;
    const int64_t target = CT == 1 ? 2500 : 5000;
    int64_t nslab = (target + rowwaves - 1) / rowwaves;
    const int64_t minslab = CT == 4 ? 384 : 256;
    const int64_t maxslab = std::max<int64_t>(1, M / minslab);
    if (nslab > maxslab) nslab = maxslab;
    if (nslab < 1) nslab = 1;
    int64_t ks = (M + nslab - 1) / nslab;
    ks = (ks + 31) / 32 * 32;
    t.kslab = (int)ks;
    return t;
}

// Tile-cache file (LB_TUNE_CACHE): one line "M Bp precision rows kslab waves".
static void load_tune_cache(lb_ctx* c) {
    if (c->cache_loaded) return;
    c->cache_loaded = true;
    const char* path = getenv("LB_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    long long M;
    int Bp, prec, rows, ks, waves;
    while (fscanf(f, "%lld %d %d %d %d %d", &M, &Bp, &prec, &rows, &ks, &waves) == 6)
        c->tuned[std::make_tuple((int64_t)M, Bp, prec)] = lb_tile{rows, ks, waves};
    fclose(f);
}

static lb_tile choose_tile(lb_ctx* c, int64_t M, int Bp, int precision, int R) {
    load_tune_cache(c);
    auto it = c->tuned.find(std::make_tuple(M, Bp, precision));
    if (it != c->tuned.end()) return it->second;
    return lb_default_tile(M, Bp, precision, R);
}

int lb_impl_q_to_f32(lb_ctx* c, int64_t M, const double* Q, int64_t ldq, float* Q32) {
    const int64_t n = M * ldq;
    hipLaunchKernelGGL(k_to_f32, dim3(lb_blocks(n, 256)), dim3(256), 0, c->stream, Q, Q32, n);
    LB_CHECK_LAUNCH();
    return LB_OK;
}

// ---------------------------------------------------------------------------
// Propagation plan: path selection, buffer layout, kernel enqueueing.
// ---------------------------------------------------------------------------

namespace {

enum PathKind { PATH_SMALL, PATH_GEMV, PATH_MFMA };

struct Plan {
    PathKind kind;
    int R;
    int64_t M, Mp, ldq;
    int B, Bp, precision;
    lb_tile tile;
    int nslab;
    int64_t sstride, s32stride, pstride, wstride;
    size_t o_ptr, o_v, o_acc, o_x, o_x32, o_part, o_w, bytes;
    size_t shm;
    int q_in_lds;
    bool aligned;
    bool staged;  // every Q and every row of Q 128-byte aligned: LDS-staged GEMM, streaming GEMV loads
    const void** d;
    double *V, *Acc, *X, *Part, *W;
    float* X32;
};

static int plan_make(Plan& p, int R, int64_t M, int64_t ldq, int B, int precision, const lb_tile& tile,
                     bool allow_small) {
    p = Plan();
    p.R = R;
    p.M = M;
    p.ldq = ldq;
    p.B = B;
    p.precision = precision;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = lb_align(off + bytes, 256);
        return o;
    };
    p.o_ptr = take(sizeof(void*) * 5 * R);
    if (allow_small && M <= 256 && (int64_t)B * M <= 4096 && precision == LB_FP64) {
        p.kind = PATH_SMALL;
        const size_t base = sizeof(double) * 2 * (size_t)B * M;
        const size_t withq = base + sizeof(double) * (size_t)M * M;
        p.q_in_lds = withq <= 64 * 1024 ? 1 : 0;
        p.shm = p.q_in_lds ? withq : base;
    } else if (B == 1 && precision == LB_FP64) {
        p.kind = PATH_GEMV;
        p.aligned = ldq % 2 == 0;
        p.wstride = 3 * (int64_t)lb_align(M, 32);
        p.o_w = take(sizeof(double) * p.wstride * R);
    } else {
        p.kind = PATH_MFMA;
        p.Bp = bpad(B);
        p.tile = tile;
        p.Mp = (M + 15) / 16 * 16;
        p.nslab = (int)((M + tile.kslab - 1) / tile.kslab);
        p.sstride = lb_align(p.Mp * p.Bp, 64);
        p.s32stride = lb_align(p.Mp * p.Bp, 128);
        p.pstride = (int64_t)p.nslab * p.Mp * p.Bp;
        p.aligned = precision == LB_FP32 ? (ldq % 4 == 0) : (ldq % 2 == 0);
        p.o_v = take(sizeof(double) * p.sstride * R);
        p.o_acc = take(sizeof(double) * p.sstride * R);
        p.o_x = take(sizeof(double) * p.sstride * R);
        if (precision == LB_FP32) p.o_x32 = take(sizeof(float) * p.s32stride * R);
        p.o_part = take(sizeof(double) * p.pstride * R);
        const int RT = tile.rows / 16, CT = p.Bp / 16;
        if (tile.rows % 16 || tile.kslab % 16 || tile.kslab <= 0 || tile.waves < 1 || tile.waves > 4 ||
            (precision == LB_FP64 ? (p.aligned ? pick64<true>(RT, CT) : pick64<false>(RT, CT)) == nullptr
                                  : (p.aligned ? pick32<true>(RT, CT) : pick32<false>(RT, CT)) == nullptr))
            return lb_fail(LB_ERR_INVALID_ARG, "unsupported tile rows=%d kslab=%d waves=%d for Bp=%d", tile.rows,
                           tile.kslab, tile.waves, p.Bp);
    }
    p.bytes = off;
    return LB_OK;
}

// Kernel choice that depends on the operands' alignment (the LDS-staged
// forms need 128-byte rows); rejects Q that is not 16-byte aligned.
static int plan_align(Plan& p, const lb_prop_sys* sys) {
    const int R = p.R;
    const int64_t es = p.precision == LB_FP32 ? 4 : 8;
    p.staged = (p.kind == PATH_MFMA || p.kind == PATH_GEMV) && (p.ldq * es) % 128 == 0;
    for (int r = 0; r < R; ++r) {
        const void* qp = p.precision == LB_FP32 ? (const void*)sys[r].Q32 : (const void*)sys[r].Q;
        if (p.kind != PATH_SMALL && ((uintptr_t)qp) % 16) return lb_fail(LB_ERR_INVALID_ARG, "Q must be 16-byte aligned");
        if (((uintptr_t)qp) % 128) p.staged = false;
    }
    if (p.staged && p.kind == PATH_MFMA) {
        const int RT = p.tile.rows / 16, CT = p.Bp / 16;
        if (p.precision == LB_FP64 ? pick64s(RT, CT) == nullptr : pick32s(RT, CT) == nullptr) p.staged = false;
    }
    return LB_OK;
}

// Points the plan's buffers into device memory `base` (p.bytes).
static void plan_buffers(Plan& p, char* base) {
    p.d = (const void**)(base + p.o_ptr);
    if (p.kind == PATH_GEMV) p.W = (double*)(base + p.o_w);
    if (p.kind == PATH_MFMA) {
        p.V = (double*)(base + p.o_v);
        p.Acc = (double*)(base + p.o_acc);
        p.X = (double*)(base + p.o_x);
        p.X32 = p.precision == LB_FP32 ? (float*)(base + p.o_x32) : nullptr;
        p.Part = (double*)(base + p.o_part);
    }
}

// Binds the plan to device memory `base` (p.bytes) and uploads the per-system
// pointer arrays through the context's pinned staging buffer. Synchronizes.
static int plan_bind(lb_ctx* c, Plan& p, char* base, const lb_prop_sys* sys) {
    const int R = p.R;
    int rc = plan_align(p, sys);
    if (rc) return rc;
    rc = lb_host_reserve(c, sizeof(void*) * 5 * R);
    if (rc) return rc;
    LB_HIP(hipStreamSynchronize(c->stream));
    const void** h = (const void**)c->host;
    for (int r = 0; r < R; ++r) {
        h[r] = sys[r].Q;
        h[R + r] = sys[r].Q32;
        h[2 * R + r] = sys[r].K;
        h[3 * R + r] = sys[r].V;
        h[4 * R + r] = sys[r].V;
    }
    LB_HIP(hipMemcpyAsync(base + p.o_ptr, h, sizeof(void*) * 5 * R, hipMemcpyHostToDevice, c->stream));
    LB_HIP(hipStreamSynchronize(c->stream));
    plan_buffers(p, base);
    return LB_OK;
}

static StageArgs stage_args(const Plan& p, double dt) {
    StageArgs sa;
    sa.Ks = (const double* const*)(p.d + 2 * p.R);
    sa.V = p.V;
    sa.Acc = p.Acc;
    sa.X = p.X;
    sa.X32 = p.X32;
    sa.sstride = p.sstride;
    sa.s32stride = p.s32stride;
    sa.Part = p.Part;
    sa.pstride = p.pstride;
    sa.nslab = p.nslab;
    sa.M = p.M;
    sa.Mp = p.Mp;
    sa.Bp = p.Bp;
    sa.dt = dt;
    return sa;
}

// One launch of the stage GEMM (MFMA path) or the stage GEMV (stage 1).
static int plan_gemm(const Plan& p, hipStream_t s, int stage, double dt) {
    if (p.kind == PATH_GEMV) {
        // rows per wave: as many as keep at least ~8192 waves in the launch
        const int64_t rows_total = p.M * p.R;
        const int RW = rows_total >= 8 * 8192 ? 8 : rows_total >= 4 * 8192 ? 4 : rows_total >= 2 * 8192 ? 2 : 1;
        const unsigned gx = lb_blocks((p.M + RW - 1) / RW, 4);
        typedef void (*gemv_fn)(const double* const*, const double* const*, double* const*, int64_t, int64_t,
                                double*, int64_t, int, double);
        gemv_fn fn;
        if (!p.aligned) fn = RW == 8 ? k_gemv<8, false, false> : RW == 4 ? k_gemv<4, false, false>
                           : RW == 2 ? k_gemv<2, false, false> : k_gemv<1, false, false>;
        else if (p.staged) fn = RW == 8 ? k_gemv<8, true, true> : RW == 4 ? k_gemv<4, true, true>
                              : RW == 2 ? k_gemv<2, true, true> : k_gemv<1, true, true>;
        else fn = RW == 8 ? k_gemv<8, true, false> : RW == 4 ? k_gemv<4, true, false>
                : RW == 2 ? k_gemv<2, true, false> : k_gemv<1, true, false>;
        hipLaunchKernelGGL(fn, dim3(gx, p.R), dim3(256), 0, s, (const double* const*)p.d,
                           (const double* const*)(p.d + 2 * p.R), (double* const*)(p.d + 3 * p.R), p.M, p.ldq, p.W,
                           p.wstride, stage, dt);
        LB_CHECK_LAUNCH();
        return LB_OK;
    }
    const int RT = p.tile.rows / 16, CT = p.Bp / 16;
    const int64_t rowwaves = (p.M + p.tile.rows - 1) / p.tile.rows;
    GemmGrid gg;
    gg.gx = (int)((rowwaves + p.tile.waves - 1) / p.tile.waves);
    gg.nslab = p.nslab;
    gg.R = p.R;
    const int64_t total = (int64_t)gg.gx * gg.nslab * gg.R;
    gg.per_xcd = (total + 7) / 8;
    const dim3 ggrid((unsigned)(8 * gg.per_xcd));
    const dim3 gblock(64 * p.tile.waves);
    // staged kernels: 2*RT KiB of LDS per wave
    const size_t shm = p.staged ? (size_t)p.tile.waves * 2 * RT * 1024 : 0;
    if (p.precision == LB_FP64) {
        gemm64_fn fn = p.staged ? pick64s(RT, CT) : (p.aligned ? pick64<true>(RT, CT) : pick64<false>(RT, CT));
        hipLaunchKernelGGL(fn, ggrid, gblock, shm, s, (const double* const*)p.d, p.M, p.Mp, p.ldq, (const double*)p.X,
                           p.sstride, p.Part, p.pstride, p.tile.kslab, gg);
    } else {
        gemm32_fn fn = p.staged ? pick32s(RT, CT) : (p.aligned ? pick32<true>(RT, CT) : pick32<false>(RT, CT));
        hipLaunchKernelGGL(fn, ggrid, gblock, shm, s, (const float* const*)(p.d + p.R), p.M, p.Mp, p.ldq,
                           (const float*)p.X32, p.s32stride, p.Part, p.pstride, p.tile.kslab, gg);
    }
    LB_CHECK_LAUNCH();
    return LB_OK;
}

static int plan_init_state(const Plan& p, hipStream_t s) {
    if (p.kind == PATH_GEMV) {
        hipLaunchKernelGGL(k_gemv_init, dim3(lb_blocks(p.M, 256), p.R), dim3(256), 0, s,
                           (double* const*)(p.d + 3 * p.R), p.M, p.W, p.wstride);
        LB_CHECK_LAUNCH();
    } else if (p.kind == PATH_MFMA) {
        hipLaunchKernelGGL(k_pack, dim3(lb_blocks(p.Mp * p.Bp, 256), p.R), dim3(256), 0, s,
                           (const double* const*)(p.d + 3 * p.R), p.M, p.Mp, p.B, p.Bp, p.V, p.X, p.X32, p.sstride,
                           p.s32stride);
        LB_CHECK_LAUNCH();
    }
    return LB_OK;
}

// Enqueues the whole integration (kernels only: no synchronization, no copies),
// so it can be recorded into a graph.
static int plan_launch(const Plan& p, hipStream_t s, double dt, int64_t steps) {
    if (steps == 0) return LB_OK;
    if (p.kind == PATH_SMALL) {
        hipLaunchKernelGGL(k_rk4_small, dim3(p.R), dim3(256), p.shm, s, (const double* const*)p.d,
                           (const double* const*)(p.d + 2 * p.R), (double* const*)(p.d + 3 * p.R), (int)p.M, p.ldq,
                           p.B, dt, steps, p.q_in_lds);
        LB_CHECK_LAUNCH();
        return LB_OK;
    }
    int rc = plan_init_state(p, s);
    if (rc) return rc;
    if (p.kind == PATH_GEMV) {
        for (int64_t st = 0; st < steps; ++st)
            for (int stage = 1; stage <= 4; ++stage) {
                rc = plan_gemm(p, s, stage, dt);
                if (rc) return rc;
            }
        return LB_OK;
    }
    const StageArgs sa = stage_args(p, dt);
    const dim3 sgrid(lb_blocks(p.M * p.Bp, 256), p.R);
    for (int64_t st = 0; st < steps; ++st)
        for (int stage = 1; stage <= 4; ++stage) {
            rc = plan_gemm(p, s, stage, dt);
            if (rc) return rc;
            hipLaunchKernelGGL(k_stage, sgrid, dim3(256), 0, s, sa, stage);
            LB_CHECK_LAUNCH();
        }
    hipLaunchKernelGGL(k_unpack, dim3(lb_blocks(p.M * p.B, 256), p.R), dim3(256), 0, s,
                       (double* const*)(p.d + 4 * p.R), p.M, p.B, p.Bp, (const double*)p.V, p.sstride);
    LB_CHECK_LAUNCH();
    return LB_OK;
}

// Average duration (ms) of the dominant stage kernel over `iters` launches,
// measured with HIP events on the context stream. The states are packed
// first; the kernel reads them but the timing loop does not advance them.
static int plan_time(lb_ctx* c, const Plan& p, int iters, double* ms) {
    hipStream_t s = c->stream;
    int rc = plan_init_state(p, s);
    if (rc) return rc;
    rc = plan_gemm(p, s, 1, 0.0);  // warm-up launch
    if (rc) return rc;
    hipEvent_t e0, e1;
    LB_HIP(hipEventCreate(&e0));
    LB_HIP(hipEventCreate(&e1));
    LB_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < iters; ++i) {
        rc = plan_gemm(p, s, p.kind == PATH_GEMV ? 1 + (i & 1) : 1, 0.0);
        if (rc) break;
    }
    LB_HIP(hipEventRecord(e1, s));
    LB_HIP(hipEventSynchronize(e1));
    float t = 0;
    LB_HIP(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *ms = (double)t / iters;
    return LB_OK;
}

static int plan_for(lb_ctx* c, Plan& p, int R, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B, int precision,
                    const lb_tile* force_tile, bool allow_small) {
    const lb_tile tile = force_tile ? *force_tile : choose_tile(c, M, bpad(B), precision, R);
    int rc = plan_make(p, R, M, ldq, B, precision, tile, allow_small && force_tile == nullptr);
    if (rc) return rc;
    rc = lb_ws_reserve(c, p.bytes);
    if (rc) return rc;
    return plan_bind(c, p, (char*)c->ws, sys);
}

}  // namespace

// R systems of size M, B states each.
int lb_impl_propagate(lb_ctx* c, int R, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B, double dt,
                      int64_t steps, int precision, const lb_tile* force_tile) {
    if (steps == 0) return LB_OK;
    Plan p;
    int rc = plan_for(c, p, R, M, sys, ldq, B, precision, force_tile, true);
    if (rc) return rc;
    return plan_launch(p, c->stream, dt, steps);
}

int lb_impl_time_stage(lb_ctx* c, int R, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B, int precision,
                       int iters, double* ms, const lb_tile* force_tile) {
    Plan p;
    int rc = plan_for(c, p, R, M, sys, ldq, B, precision, force_tile, false);
    if (rc) return rc;
    return plan_time(c, p, iters, ms);
}

// ---------------------------------------------------------------------------
// Allocation-free propagation (one system): the plan's buffers -- packed
// states, stage accumulators, split-K partials, the pointer table -- live in a
// static device array instead of the context workspace, and the pointer table
// is written by a kernel instead of a staged host copy, so the call allocates
// nothing (no device, no pinned host memory) and never synchronizes. Each GPU
// holds its own copy of the array from module load until the process ends;
// every call on a GPU shares it (nothing in it must start at zero: the plan
// writes every element it reads), so calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)LB_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each GPU

__global__ void k_set_ptrs(const void** d, const void* q, const void* q32, const void* k, void* v) {
    if (threadIdx.x == 0) {
        d[0] = q;
        d[1] = q32;
        d[2] = k;
        d[3] = v;
        d[4] = v;
    }
}

}  // namespace

// Looks up the array's device address once per device; `device` must be current.
int lb_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return lb_fail(LB_ERR_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return LB_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return lb_fail(LB_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch[device] = ptr;
    return LB_OK;
}

int lb_impl_propagate_noalloc(lb_ctx* c, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B, double dt,
                              int64_t steps, int precision) {
    if (steps == 0) return LB_OK;
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = c->device >= 0 && c->device < kMaxDevices ? g_scratch[c->device] : nullptr;
    }
    if (!base) return lb_fail(LB_ERR_DEVICE, "the static scratch of device %d is not set up", c->device);
    Plan p;
    int rc = plan_make(p, 1, M, ldq, B, precision, choose_tile(c, M, bpad(B), precision, 1), true);
    if (rc) return rc;
    if (p.bytes > kScratchBytes)
        return lb_fail(LB_ERR_UNSUPPORTED,
                       "M=%lld with %d states needs %zu bytes of scratch; the allocation-free propagate holds %zu",
                       (long long)M, B, p.bytes, kScratchBytes);
    rc = plan_align(p, sys);
    if (rc) return rc;
    plan_buffers(p, (char*)base);
    hipLaunchKernelGGL(k_set_ptrs, dim3(1), dim3(64), 0, c->stream, p.d, (const void*)sys->Q, (const void*)sys->Q32,
                       (const void*)sys->K, (void*)sys->V);
    LB_CHECK_LAUNCH();
    return plan_launch(p, c->stream, dt, steps);
}

struct lb_graph_entry {
    Plan plan;
    void* mem = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;
};

// Captured graphs kept per context (least recently used evicted first): each
// holds its plan buffers and the raw operand pointers it was captured with.
constexpr size_t kMaxGraphs = 8;

void lb_graph_free(lb_graph_entry* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->mem) (void)hipFree(g->mem);
    delete g;
}

int lb_impl_propagate_graph(lb_ctx* c, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B, double dt,
                            int64_t steps, int precision) {
    if (steps == 0) return LB_OK;
    lb_graph_key key{M, ldq, B, precision, sys->Q, sys->Q32, sys->K, sys->V, dt, steps};
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        if (c->graphs.size() >= kMaxGraphs) {
            auto lru = c->graphs.begin();
            for (auto jt = c->graphs.begin(); jt != c->graphs.end(); ++jt)
                if (jt->second->last_use < lru->second->last_use) lru = jt;
            LB_HIP(hipStreamSynchronize(c->stream));  // its last launch may still run
            lb_graph_free(lru->second);
            c->graphs.erase(lru);
        }
        lb_graph_entry* g = new lb_graph_entry();
        const lb_tile tile = choose_tile(c, M, bpad(B), precision, 1);
        int rc = plan_make(g->plan, 1, M, ldq, B, precision, tile, true);
        if (rc) {
            delete g;
            return rc;
        }
        hipError_t e = hipMalloc(&g->mem, g->plan.bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete g;
            return lb_fail(LB_ERR_OOM, "graph buffers (%zu bytes): %s", g->plan.bytes, hipGetErrorString(e));
        }
        rc = plan_bind(c, g->plan, (char*)g->mem, sys);
        if (rc) {
            lb_graph_free(g);
            return rc;
        }
        hipStream_t cs;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) {
            lb_graph_free(g);
            return lb_fail(LB_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = plan_launch(g->plan, cs, dt, steps);
            hipError_t e2 = hipStreamEndCapture(cs, &graph);
            if (!rc && e2 != hipSuccess) rc = lb_fail(LB_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e2));
        } else {
            rc = lb_fail(LB_ERR_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
        }
        (void)hipStreamDestroy(cs);
        if (!rc) {
            e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = lb_fail(LB_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (rc) {
            lb_graph_free(g);
            return rc;
        }
        it = c->graphs.emplace(key, g).first;
    }
    it->second->last_use = ++c->graph_clock;
    LB_HIP(hipGraphLaunch(it->second->exec, c->stream));
    return LB_OK;
}

// Tries tile shapes on the context stream and keeps the fastest stage kernel.
int lb_impl_autotune(lb_ctx* c, int64_t M, const lb_prop_sys* sys, int64_t ldq, int B, int precision) {
    const int Bp = bpad(B);
    if (B == 1 && precision == LB_FP64) return LB_OK;  // GEMV path has no tile
    const int CT = Bp / 16;
    std::vector<int> rows_c = CT == 1 ? std::vector<int>{32, 64} : std::vector<int>{16, 32};
    std::vector<int> waves_c = {1, 2, 4};
    std::vector<int> target_c = {1, 1250, 2500, 5000, 10000};  // 1: one slab per row block
    lb_tile best = lb_default_tile(M, Bp, precision, 1);
    double best_ms = 1e30;
    for (int rows : rows_c)
        for (int waves : waves_c)
            for (int target : target_c) {
                lb_tile t;
                t.rows = rows;
                t.waves = waves;
                const int64_t rowwaves = (M + rows - 1) / rows;
                int64_t nslab = (target + rowwaves - 1) / rowwaves;
                const int64_t maxslab = (M + 255) / 256;
                nslab = nslab < 1 ? 1 : (nslab > maxslab ? maxslab : nslab);
                int64_t ks = (M + nslab - 1) / nslab;
                t.kslab = (int)((ks + 31) / 32 * 32);
                double ms = 0;
                int rc = lb_impl_time_stage(c, 1, M, sys, ldq, B, precision, 3, &ms, &t);
                if (rc) continue;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
    c->tuned[std::make_tuple(M, Bp, precision)] = best;
    if (const char* path = getenv("LB_TUNE_CACHE")) {
        FILE* f = fopen(path, "a");
        if (f) {
            fprintf(f, "%lld %d %d %d %d %d\n", (long long)M, Bp, precision, best.rows, best.kslab, best.waves);
            fclose(f);
        }
    }
    return LB_OK;
}

// The square-wave drive eps(t) = E + A Theta(t), Theta = +1 on [0, T/2) and
// -1 on [T/2, T), of the rocked dimer (Sec. 3). `left` gives the limit from
// the left (at a switch: the half period that ends there).
static double drive_value(double t, double E, double A, double T, bool left) {
    double r = fmod(t, T);
    if (left) {
        if (r <= 0) r += T;
        return r <= 0.5 * T ? E + A : E - A;
    }
    if (r < 0) r += T;
    return r < 0.5 * T ? E + A : E - A;
}

// Stage time t0 + (k + c) dt as one product and one sum.
static double stage_time(double t0, int64_t k, double c, double dt) {
    const double kc = (double)k + c;
    volatile double p = kc * dt;
    return t0 + p;
}

static int csr_propagate(lb_ctx* c, int64_t M, const int64_t* rowptr, const int64_t* col, const double* val,
                         const int64_t* rowptr1, const int64_t* col1, const double* val1, const double* K, double* V,
                         int B, double dt, int64_t steps, double t0, int64_t k0, double E, double A, double T) {
    hipStream_t s = c->stream;
    if (steps == 0) return LB_OK;
    const bool drive = rowptr1 != nullptr;
    const int64_t n = M * B;
    SellMat m;
    size_t o_w = 0;
    int rc = sell_build(c, M, rowptr, col, val, rowptr1, col1, val1, sizeof(double) * 3 * (size_t)n, &m, &o_w);
    if (rc) return rc;
    double* W = (double*)((char*)c->ws + o_w);
    hipLaunchKernelGGL(k_copy, dim3(lb_blocks(n, 256)), dim3(256), 0, s, (const double*)V, W + n, n);
    LB_CHECK_LAUNCH();
    const SellStage st{B, K, V, W};
    const unsigned grid = (unsigned)m.nlong8 + 8u * (unsigned)m.per_xcd;
    typedef void (*stage_fn)(SellMat, SellStage, int, double, double);
    const stage_fn fn = drive ? (B == 1 ? k_sell_stage<true, 1> : k_sell_stage<true, 4>)
                              : (B == 1 ? k_sell_stage<false, 1> : k_sell_stage<false, 4>);
    for (int64_t k = 0; k < steps; ++k)
        for (int stage = 1; stage <= 4; ++stage) {
            double eps = 0.0;
            if (drive) {
                // stages seen from inside the step: t_k and t_k + dt/2 from the right, t_k + dt from the left
                const double cst = stage == 1 ? 0.0 : (stage == 4 ? 1.0 : 0.5);
                eps = drive_value(stage_time(t0, k0 + k, cst, dt), E, A, T, stage == 4);
            }
            hipLaunchKernelGGL(fn, dim3(grid), dim3(256), 0, s, m, st, stage, dt, eps);
            LB_CHECK_LAUNCH();
        }
    return LB_OK;
}

int lb_impl_propagate_csr(lb_ctx* c, int64_t M, const int64_t* rowptr, const int64_t* col, const double* val,
                          const double* K, double* V, int B, double dt, int64_t steps) {
    return csr_propagate(c, M, rowptr, col, val, nullptr, nullptr, nullptr, K, V, B, dt, steps, 0.0, 0, 0.0, 0.0, 1.0);
}

int lb_impl_propagate_csr_drive(lb_ctx* c, int64_t M, const int64_t* rowptr0, const int64_t* col0,
                                const double* val0, const int64_t* rowptr1, const int64_t* col1, const double* val1,
                                const double* K, double* V, int B, double dt, int64_t steps, double t0, int64_t k0,
                                double E, double A, double T) {
    return csr_propagate(c, M, rowptr0, col0, val0, rowptr1, col1, val1, K, V, B, dt, steps, t0, k0, E, A, T);
}
