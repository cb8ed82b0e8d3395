// Spectrum of the real generator Q (Sec. 5, Fig. 5): with rho = 1/N + sum v_n F_n the
// Lindbladian acts on the coordinates (1, v) as [[0, 0], [K, Q]], so its spectrum is 0
// and the M = N^2 - 1 eigenvalues of Q, which Fig. 5 histograms on a grid.
//
// Two stages on a copy of Q (row-major, leading dimension M):
//  1. Householder reduction to upper Hessenberg form, one column j at a time. The
//     reflector P = 1 - tau v v^T (v_0 = 1 on rows j+1..M-1) is applied from both
//     sides in one rank-2 update, P A P = A - v w^T - (tau p) v^T with p = A v,
//     q = A^T v, s = v^T p and w = tau q - tau^2 s v: a row-dot pass (p), a column
//     pass (q, partial sums per row chunk reduced in fixed order), and the update.
//     From M = kBlockedMin the reduction is blocked instead (compact WY panels, one
//     GEMV over the matrix per column, the panel's two-sided update as GEMMs).
//  2. Francis' implicit double-shift QR iteration on the Hessenberg matrix,
//     eigenvalues only (updates stay inside the active block). A sweep chases a
//     chain of b double-shift bulges spaced kSep = 4 rows apart: at that spacing no
//     bulge's reflector reads what another bulge writes in the same step, and
//     reflections from the two sides commute, so a chain step is data-parallel over
//     all b bulges at once. Blocks above kSmallBlock rows are swept over the whole
//     device (up to kWideBulges bulges, one launch per chain step); smaller blocks,
//     and the shift problems, by one workgroup (up to kMaxBulges bulges, two barrier
//     phases per chain step). The 2b shifts of a b-bulge chain are the eigenvalues of
//     the trailing 2b x 2b block, found by the same iteration on a copy in LDS
//     (recursively, down to one bulge). A block splits off where a
//     subdiagonal entry falls below eps (|h_k-1,k-1| + |h_kk|), below eps ||H||_F after
//     ten sweeps without a split and below sqrt(n) eps ||H||_F after twenty (clusters at
//     the rounding floor); 1 x 1 and 2 x 2 blocks give their eigenvalues
//     directly. Every tenth sweep without a split takes an exceptional shift to break
//     cycles; kMaxIts sweeps without one is an error.
#include "lb_internal.h"
#include "rowdot.h"


#include <float.h>
#include <algorithm>
#include <math.h>

namespace {

constexpr int kQrThreads = 1024;
constexpr int kMaxBulges = 16;              // 32 shifts per sweep
constexpr int kSep = 4;                     // rows between neighbouring bulges
constexpr int kShiftDim = 2 * kMaxBulges;   // trailing block solved for the shifts
constexpr int kMaxIts = 120;                // sweeps without a split before giving up
constexpr int kBatch = 1;                   // row / column pieces per thread with loads in flight together
constexpr int kChunkRows = 16;              // shortest row chunk of the column pass
constexpr int kMaxChunks = 256;
constexpr int kPanel = 32;                  // reflectors per panel of the blocked reduction
constexpr int kBlockedMin = 1000;           // M from which the reduction is blocked

// ---------------------------------------------------------------------------
// Stage 1: Hessenberg reduction
// ---------------------------------------------------------------------------

__device__ __forceinline__ double block_sum256(double x, double* red) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Reflector of column j: x = A[j+1.., j]; writes beta e_1 into the column, v (v_0 = 1)
// and tau (0 when the column is already reduced).
__global__ __launch_bounds__(256) void k_hh_house(double* A, int64_t ld, int M, int j, double* v, double* sc) {
    __shared__ double red[4];
    __shared__ double bc[2];
    const int L = M - j - 1;
    double s = 0.0;
    for (int i = 1 + threadIdx.x; i < L; i += 256) {
        const double x = A[(int64_t)(j + 1 + i) * ld + j];
        s = fma(x, x, s);
    }
    const double sigma = block_sum256(s, red);
    if (threadIdx.x == 0) {
        const double alpha = A[(int64_t)(j + 1) * ld + j];
        double tau = 0.0, scale = 0.0;
        if (sigma > 0.0) {
            const double beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
            A[(int64_t)(j + 1) * ld + j] = beta;
        }
        bc[0] = tau;
        bc[1] = scale;
        sc[0] = tau;
        v[0] = 1.0;
    }
    __syncthreads();
    const double tau = bc[0], scale = bc[1];
    for (int i = 1 + threadIdx.x; i < L; i += 256) {
        double* a = A + (int64_t)(j + 1 + i) * ld + j;
        v[i] = tau != 0.0 ? *a * scale : 0.0;
        if (tau != 0.0) *a = 0.0;
    }
}

// p[r] = sum_{c > j} A[r][c] v[c - j - 1] for every row r: one wavefront per row.
__global__ __launch_bounds__(256) void k_hh_p(const double* A, int64_t ld, int M, int j, const double* v, double* p) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= M) return;
    const double* row = A + (int64_t)r * ld + j + 1;
    const int L = M - j - 1;
    double s = 0.0;
    for (int c = lane; c < L; c += 64) s = fma(row[c], v[c], s);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) p[r] = s;
}

// Partial q over one chunk of rows: qpart[chunk][c] = sum_{r in chunk} v[r - j - 1] A[r][c].
__global__ __launch_bounds__(256) void k_hh_q(const double* A, int64_t ld, int M, int j, const double* v, double* qpart,
                                              int rows_per_chunk) {
    const int c = j + 1 + blockIdx.x * 256 + threadIdx.x;
    if (c >= M) return;
    const int r0 = j + 1 + blockIdx.y * rows_per_chunk;
    const int r1 = min(M, r0 + rows_per_chunk);
    double s = 0.0;
    for (int r = r0; r < r1; ++r) s = fma(v[r - j - 1], A[(int64_t)r * ld + c], s);
    qpart[(int64_t)blockIdx.y * M + c] = s;
}

// q[c] = sum of the chunk partials: a block covers 64 columns, its four wavefronts
// every fourth chunk, combined in fixed order; the last block forms s = v^T p.
__global__ __launch_bounds__(256) void k_hh_qfin(int M, int j, int nchunks, const double* qpart, const double* v,
                                                 const double* p, double* q, double* sc) {
    __shared__ double red[4];
    __shared__ double part[4][64];
    if (blockIdx.x == gridDim.x - 1) {
        double s = 0.0;
        for (int i = threadIdx.x; i < M - j - 1; i += 256) s = fma(v[i], p[j + 1 + i], s);
        s = block_sum256(s, red);
        if (threadIdx.x == 0) sc[1] = s;
        return;
    }
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int c = j + 1 + blockIdx.x * 64 + lane;
    double s = 0.0;
    if (c < M) {
#pragma unroll 8
        for (int k = grp; k < nchunks; k += 4) s += qpart[(int64_t)k * M + c];
    }
    part[grp][lane] = s;
    __syncthreads();
    if (grp == 0 && c < M) q[c] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

// A[r][c] -= v_r w_c + tau p_r v_c over rows 0..M-1 and columns j+1..M-1
// (v_r = 0 above row j+1), w_c = tau q_c - tau^2 s v_c. A block covers 64 columns x 16 rows.
__global__ __launch_bounds__(256) void k_hh_update(double* A, int64_t ld, int M, int j, const double* v, const double* p,
                                                   const double* q, const double* sc) {
    const int c = j + 1 + blockIdx.x * 64 + (threadIdx.x & 63);
    if (c >= M) return;
    const double tau = sc[0];
    if (tau == 0.0) return;
    const double s = sc[1];
    const double vc = v[c - j - 1];
    const double wc = tau * q[c] - tau * tau * s * vc;
    const int rbase = blockIdx.y * 16 + (threadIdx.x >> 6) * 4;
    for (int i = 0; i < 4; ++i) {
        const int r = rbase + i;
        if (r >= M) break;
        const double vr = r > j ? v[r - j - 1] : 0.0;
        double* a = A + (int64_t)r * ld + c;
        *a -= fma(vr, wc, tau * p[r] * vc);
    }
}

// ---------------------------------------------------------------------------
// Stage 2: multishift QR, one workgroup
// ---------------------------------------------------------------------------

// Block-uniform control of one QR solve; thread 0 decides, the others read after a barrier.
struct QrCtl {
    int u, split, its, status, b, nested;
    int64_t sweeps, steps;
    int64_t work;                                  // row / column pieces updated (each 3 entries, 10 flops)
    double anorm;                                  // ||H||_F at the start
    double s[kMaxBulges], t[kMaxBulges];           // shift pairs: sigma1 + sigma2, sigma1 sigma2
    double tau[2][kMaxBulges], w1[2][kMaxBulges], w2[2][kMaxBulges];  // reflectors, by step parity
};

__device__ __forceinline__ double& at(double* H, int64_t ld, int r, int c) { return H[(int64_t)r * ld + c]; }

// Eigenvalues of [[a, b], [c, d]], conjugate pairs with the positive imaginary part first.
__device__ void eig2(double a, double b, double c, double d, double2* l1, double2* l2) {
    const double p = 0.5 * (a - d);
    const double disc = p * p + b * c;
    if (disc >= 0.0) {
        const double z = p + copysign(sqrt(disc), p);
        if (z == 0.0) {
            *l1 = make_double2(d, 0.0);
            *l2 = make_double2(d, 0.0);
        } else {
            *l1 = make_double2(d + z, 0.0);
            *l2 = make_double2(d - (b * c) / z, 0.0);
        }
    } else {
        const double m = 0.5 * (a + d), im = sqrt(-disc);
        *l1 = make_double2(m, im);
        *l2 = make_double2(m, -im);
    }
}

// Reflector 1 - tau w w^T with w = (1, w1, w2) mapping (x, y, z) to (beta, 0, 0).
__device__ void house3(double x, double y, double z, double* tau, double* w1, double* w2, double* beta) {
    const double sc = fabs(x) + fabs(y) + fabs(z);
    if (sc == 0.0 || (y == 0.0 && z == 0.0)) {
        *tau = 0.0;
        *w1 = *w2 = 0.0;
        *beta = x;
        return;
    }
    const double xs = x / sc, ys = y / sc, zs = z / sc;
    const double bs = -copysign(sqrt(xs * xs + ys * ys + zs * zs), xs);
    *tau = (bs - xs) / bs;
    const double d = xs - bs;
    *w1 = ys / d;
    *w2 = zs / d;
    *beta = bs * sc;
}

// First column of (H - sigma1)(H - sigma2) at the top of the block [l, ...]: the
// input of a bulge's first reflector, with s = sigma1 + sigma2 and t = sigma1 sigma2.
__device__ void intro_xyz(const double* H, int64_t ld, int l, double s, double t, double* x, double* y, double* z) {
    const double h00 = H[(int64_t)l * ld + l], h01 = H[(int64_t)l * ld + l + 1];
    const double h10 = H[(int64_t)(l + 1) * ld + l], h11 = H[(int64_t)(l + 1) * ld + l + 1];
    const double h21 = H[(int64_t)(l + 2) * ld + l + 1];
    *x = h00 * h00 + h01 * h10 - s * h00 + t;
    *y = h10 * (h00 + h11 - s);
    *z = h10 * h21;
}

// All threads of the block call this with the same arguments. H: n x n upper Hessenberg
// (entries below the subdiagonal are never read), row-major with leading dimension ld,
// in global memory or LDS; destroyed. lam receives the n eigenvalues. Returns 0, or 1
// when kMaxIts sweeps pass without a split. BMAX > 1 takes its shifts from the trailing
// block through a nested BMAX = 1 solve on sub (kShiftDim^2 doubles, LDS).
template <int BMAX>
__device__ int qr_eigs(double* H, int64_t ld, int n, double2* lam, QrCtl& C, QrCtl* inner, double* sub,
                       double2* subev) {
    const int tid = threadIdx.x;
    const double eps = DBL_EPSILON;
    // Frobenius norm of the Hessenberg part: the scale of the normwise split test
    __shared__ double part[kQrThreads / 64];
    double m = 0.0;
    for (int64_t e = tid; e < (int64_t)n * n; e += kQrThreads) {
        const int r = (int)(e / n), c = (int)(e % n);
        if (r <= c + 1) {
            const double h = H[(int64_t)r * ld + c];
            m = fma(h, h, m);
        }
    }
    for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o, 64);
    if ((tid & 63) == 0) part[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        double a = 0.0;
        for (int w = 0; w < kQrThreads / 64; ++w) a += part[w];
        C.anorm = a > 0.0 ? sqrt(a) : 1.0;
        C.u = n - 1;
        C.its = 0;
        C.status = 0;
        C.sweeps = 0;
        C.steps = 0;
        C.work = 0;
        C.split = 0;
    }
    __syncthreads();
    for (;;) {
        const int u = C.u;
        if (u < 0 || C.status) break;
        // Largest k in [1, u] whose subdiagonal entry is negligible (0 if none): below
        // eps times its two diagonal neighbours, or, once ten sweeps have passed without
        // a split (a cluster whose subdiagonal sits at the rounding floor), below eps
        // ||H||_F, and after twenty below sqrt(n) eps ||H||_F: normwise backward errors of
        // the size the Householder reduction itself leaves.
        const double floor_scale = C.its >= 20 ? sqrt((double)n) * C.anorm : (C.its >= 10 ? C.anorm : 0.0);
        for (int k = u - tid; k >= 1; k -= kQrThreads) {
            const double sd = fabs(at(H, ld, k, k - 1));
            double tst = fabs(at(H, ld, k - 1, k - 1)) + fabs(at(H, ld, k, k));
            tst = tst == 0.0 ? fmax(C.anorm, floor_scale) : fmax(tst, floor_scale);
            if (sd <= eps * tst) {
                atomicMax(&C.split, k);
                break;
            }
        }
        __syncthreads();
        const int l = C.split;
        __syncthreads();
        if (l == u || l == u - 1) {
            if (tid == 0) {
                if (l > 0) at(H, ld, l, l - 1) = 0.0;
                if (l == u) {
                    lam[u] = make_double2(at(H, ld, u, u), 0.0);
                    C.u = u - 1;
                } else {
                    eig2(at(H, ld, u - 1, u - 1), at(H, ld, u - 1, u), at(H, ld, u, u - 1), at(H, ld, u, u),
                         &lam[u - 1], &lam[u]);
                    C.u = u - 2;
                }
                C.its = 0;
                C.split = 0;
            }
            __syncthreads();
            continue;
        }
        // a sweep over the unreduced block [l, u] (at least 3 x 3)
        if (tid == 0) {
            if (l > 0) at(H, ld, l, l - 1) = 0.0;
            C.split = 0;
            C.its += 1;
            C.sweeps += 1;
            if (C.its > kMaxIts) C.status = 1;
            const int na = u - l + 1;
            int b = BMAX > 1 ? min(BMAX, max(1, na / 16)) : 1;
            const bool exceptional = (C.its % 10) == 0;
            C.nested = 0;
            if (exceptional) {
                const double w = at(H, ld, u, u) +
                                 0.75 * (fabs(at(H, ld, u, u - 1)) + fabs(at(H, ld, u - 1, u - 2)));
                for (int i = 0; i < b; ++i) {
                    C.s[i] = 2.0 * w;
                    C.t[i] = w * w;
                }
            } else if (b == 1) {
                const double a = at(H, ld, u - 1, u - 1), bb = at(H, ld, u - 1, u);
                const double c = at(H, ld, u, u - 1), d = at(H, ld, u, u);
                C.s[0] = a + d;
                C.t[0] = a * d - bb * c;
            } else {
                C.nested = 1;
            }
            C.b = b;
        }
        __syncthreads();
        if (C.status) break;
        const int b = C.b;
        if constexpr (BMAX > 1) {
            if (C.nested) {
                const int mm = 2 * b, o = u - mm + 1;
                for (int e = tid; e < mm * mm; e += kQrThreads) {
                    const int r = e / mm, c = e % mm;
                    sub[e] = r <= c + 1 ? at(H, ld, o + r, o + c) : 0.0;
                }
                __syncthreads();
                const int rc = qr_eigs<1>(sub, mm, mm, subev, *inner, nullptr, nullptr, nullptr);
                if (tid == 0) {
                    if (rc != 0) {  // keep the sweep going with the trailing 2 x 2 shift
                        const double a = at(H, ld, u - 1, u - 1), bb = at(H, ld, u - 1, u);
                        const double c = at(H, ld, u, u - 1), d = at(H, ld, u, u);
                        for (int i = 0; i < b; ++i) {
                            C.s[i] = a + d;
                            C.t[i] = a * d - bb * c;
                        }
                    } else {
                        // complex values with positive imaginary part give one pair each;
                        // the real ones are sorted and paired neighbour with neighbour
                        int np = 0;
                        double re[kShiftDim];
                        int nr = 0;
                        for (int i = 0; i < mm; ++i) {
                            const double2 z = subev[i];
                            if (z.y > 0.0) {
                                C.s[np] = 2.0 * z.x;
                                C.t[np] = z.x * z.x + z.y * z.y;
                                ++np;
                            } else if (z.y == 0.0) {
                                int q = nr++;
                                while (q > 0 && re[q - 1] > z.x) {
                                    re[q] = re[q - 1];
                                    --q;
                                }
                                re[q] = z.x;
                            }
                        }
                        for (int i = 0; i + 1 < nr && np < b; i += 2) {
                            C.s[np] = re[i] + re[i + 1];
                            C.t[np] = re[i] * re[i + 1];
                            ++np;
                        }
                        for (int i = np; i < b; ++i) {  // unpaired leftovers: repeat the last pair
                            C.s[i] = np ? C.s[np - 1] : 0.0;
                            C.t[i] = np ? C.t[np - 1] : 0.0;
                        }
                    }
                }
                __syncthreads();
            }
        }
        // The chain: bulge i sits at reflector position l + t - kSep i in step t. A step
        // is two phases: every reflector from the left (rows k..k+2, columns k..u),
        // then every reflector from the right (columns k..k+2, rows l..min(k+3, u)).
        // Rows k+1..k+3 of bulge i's right update belong to its owner thread i, which
        // then holds column k of those rows, exactly the input of the bulge's next
        // reflector (or builds the next bulge's first reflector from the leading 3 x 3
        // block), so reflectors are ready after the second phase without a third.
        // Reflectors of consecutive steps alternate between two buffers.
        const int T = kSep * (b - 1) + (u - l);
        const int ld32 = (int)ld;  // n * ld < 2^31: blocks of at most kSmallBlock rows, ld <= 46340
        if (tid == 0) {
            double x, y, z, beta;
            intro_xyz(H, ld, l, C.s[0], C.t[0], &x, &y, &z);
            house3(x, y, z, &C.tau[0][0], &C.w1[0][0], &C.w2[0][0], &beta);
        }
        __syncthreads();
        for (int t = 0; t < T; ++t) {
            const int p = t & 1;
            const int ihi = min(b - 1, t / kSep);
            int ilo = 0;
            while (ilo <= ihi && l + t - kSep * ilo > u - 1) ++ilo;
            // from the left: pieces (bulge, column), bulge by bulge, columns consecutive
            int total = 0;
            for (int i = ilo; i <= ihi; ++i) total += u - (l + t - kSep * i) + 1;
            for (int base = 0; base < total; base += kQrThreads * kBatch) {
                double a0[kBatch], a1[kBatch], a2[kBatch];
                int off[kBatch], bi[kBatch];
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    bi[q] = -1;
                    int e = base + q * kQrThreads + tid;
                    if (e >= total) continue;
                    int i = ilo;
                    while (e >= u - (l + t - kSep * i) + 1) {
                        e -= u - (l + t - kSep * i) + 1;
                        ++i;
                    }
                    if (C.tau[p][i] == 0.0) continue;
                    const int k = l + t - kSep * i;
                    bi[q] = i;
                    off[q] = k * ld32 + k + e;
                    a0[q] = H[off[q]];
                    a1[q] = H[off[q] + ld32];
                    a2[q] = k + 2 <= u ? H[off[q] + 2 * ld32] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    if (bi[q] < 0) continue;
                    const int i = bi[q];
                    const double tau = C.tau[p][i], w1 = C.w1[p][i], w2 = C.w2[p][i];
                    const double r = tau * (a0[q] + w1 * a1[q] + w2 * a2[q]);
                    H[off[q]] = a0[q] - r;
                    H[off[q] + ld32] = a1[q] - r * w1;
                    if (l + t - kSep * i + 2 <= u) H[off[q] + 2 * ld32] = a2[q] - r * w2;
                }
            }
            __syncthreads();
            // from the right: the owners' rows k+1..k+3 and the next reflectors first
            if (tid < b) {
                const int i = tid;
                const int k = l + t - kSep * i;
                double tn = 0.0, w1n = 0.0, w2n = 0.0;
                if (i >= ilo && i <= ihi) {
                    const double tau = C.tau[p][i], w1 = C.w1[p][i], w2 = C.w2[p][i];
                    const bool three = k + 2 <= u;
                    double col[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int rr = 0; rr < 3; ++rr) {
                        const int row = k + 1 + rr;
                        if (row <= u) {
                            double* h = H + row * ld32 + k;
                            double h0 = h[0], h1 = h[1], h2 = three ? h[2] : 0.0;
                            if (tau != 0.0) {
                                const double q = tau * (h0 + w1 * h1 + w2 * h2);
                                h0 -= q;
                                h1 -= q * w1;
                                h2 -= q * w2;
                                h[1] = h1;
                                if (three) h[2] = h2;
                            }
                            col[rr] = h0;
                        }
                    }
                    const int kn = k + 1;
                    double beta = 0.0;
                    if (kn <= u - 1) house3(col[0], col[1], kn + 2 <= u ? col[2] : 0.0, &tn, &w1n, &w2n, &beta);
#pragma unroll
                    for (int rr = 0; rr < 3; ++rr) {
                        const int row = k + 1 + rr;
                        if (row <= u) H[row * ld32 + k] = tn != 0.0 ? (rr == 0 ? beta : 0.0) : col[rr];
                    }
                } else if (i >= 1 && t + 1 == kSep * i) {
                    double x, y, z, beta;
                    intro_xyz(H, ld, l, C.s[i], C.t[i], &x, &y, &z);
                    house3(x, y, z, &tn, &w1n, &w2n, &beta);
                }
                C.tau[p ^ 1][i] = tn;
                C.w1[p ^ 1][i] = w1n;
                C.w2[p ^ 1][i] = w2n;
            }
            // the rest: pieces (bulge, row) for rows l..k
            total = 0;
            for (int i = ilo; i <= ihi; ++i) total += (l + t - kSep * i) - l + 1;
            for (int base = 0; base < total; base += kQrThreads * kBatch) {
                double a0[kBatch], a1[kBatch], a2[kBatch];
                int off[kBatch], bi[kBatch];
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    bi[q] = -1;
                    int e = base + q * kQrThreads + tid;
                    if (e >= total) continue;
                    int i = ilo;
                    while (e >= (l + t - kSep * i) - l + 1) {
                        e -= (l + t - kSep * i) - l + 1;
                        ++i;
                    }
                    if (C.tau[p][i] == 0.0) continue;
                    const int k = l + t - kSep * i;
                    bi[q] = i;
                    off[q] = (l + e) * ld32 + k;
                    a0[q] = H[off[q]];
                    a1[q] = H[off[q] + 1];
                    a2[q] = k + 2 <= u ? H[off[q] + 2] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    if (bi[q] < 0) continue;
                    const int i = bi[q];
                    const double tau = C.tau[p][i], w1 = C.w1[p][i], w2 = C.w2[p][i];
                    const double r = tau * (a0[q] + w1 * a1[q] + w2 * a2[q]);
                    H[off[q]] = a0[q] - r;
                    H[off[q] + 1] = a1[q] - r * w1;
                    if (l + t - kSep * i + 2 <= u) H[off[q] + 2] = a2[q] - r * w2;
                }
            }
            __syncthreads();
        }
        // a bulge crossing na rows updates sum_k (u - k + 1) pieces from the left and
        // sum_k (min(k + 3, u) - l + 1) from the right: na^2 + 3 na - 7 in all
        if (tid == 0) {
            const int64_t na = u - l + 1;
            C.steps += T;
            C.work += (int64_t)b * (na * na + 3 * na - 7);
        }
        __syncthreads();
    }
    __syncthreads();
    return C.status;
}

// ---------------------------------------------------------------------------
// Stage 2 on the whole device: sweeps over large blocks, one launch per phase
// ---------------------------------------------------------------------------

// Blocks of at most kSmallBlock rows are finished by one workgroup (qr_eigs);
// sweeps over larger blocks run each phase of each chain step as a launch over the
// whole device, the kernel boundaries ordering the phases.
constexpr int kSmallBlock = 256;
constexpr int kWideBulges = 64;                 // bulges per device-wide sweep (128 shifts)
constexpr int kWideShiftDim = 2 * kWideBulges;  // trailing block solved for their shifts

// Device-side state of the host-driven iteration. The host reads the first eight
// ints back after each decision.
struct QrGlobal {
    int u, split, its, status, action, l, b, pad;  // action: 0 = split or block done, 1 = sweep
    int64_t sweeps, steps, work;                   // counts of the one-workgroup solves
    double anorm;                                  // ||H||_F
    double s[kWideBulges], t[kWideBulges];         // shift pairs of the current sweep
    double tau[2][kWideBulges], w1[2][kWideBulges], w2[2][kWideBulges];  // reflectors by step parity
};

__global__ __launch_bounds__(1024) void k_qr_init(const double* H, int64_t ld, int n, QrGlobal* g) {
    __shared__ double part[16];
    double m = 0.0;
    for (int r = threadIdx.x >> 6; r < n; r += 16) {
        const int c0 = r > 0 ? r - 1 : 0;
        for (int c = c0 + (threadIdx.x & 63); c < n; c += 64) {
            const double h = H[(int64_t)r * ld + c];
            m = fma(h, h, m);
        }
    }
    for (int o = 32; o > 0; o >>= 1) m += __shfl_xor(m, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        for (int w = 0; w < 16; ++w) a += part[w];
        g->anorm = a > 0.0 ? sqrt(a) : 1.0;
        g->u = n - 1;
        g->split = 0;
        g->its = 0;
        g->status = 0;
        g->action = 0;
        g->l = 0;
        g->b = 0;
        g->sweeps = g->steps = g->work = 0;
    }
}

// The largest k in [1, u] with a negligible subdiagonal entry (the test of qr_eigs, n the
// order of the whole matrix).
__global__ void k_qr_scan(const double* H, int64_t ld, int n, QrGlobal* g) {
    const int k = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int u = g->u;
    if (k > u) return;
    const double sd = fabs(H[(int64_t)k * ld + k - 1]);
    double tst = fabs(H[(int64_t)(k - 1) * ld + k - 1]) + fabs(H[(int64_t)k * ld + k]);
    const int its = g->its;
    const double floor_scale = its >= 20 ? sqrt((double)n) * g->anorm : (its >= 10 ? g->anorm : 0.0);
    tst = tst == 0.0 ? fmax(g->anorm, floor_scale) : fmax(tst, floor_scale);
    if (sd <= DBL_EPSILON * tst) atomicMax(&g->split, k);
}

// One decision on the bottom block [split, u]: the eigenvalues of a 1 x 1 or 2 x 2
// block, a whole small block by qr_eigs, or the set-up of a device-wide sweep
// (shifts from the trailing block, the first bulge's reflector).
__global__ __launch_bounds__(kQrThreads) void k_qr_decide(double* H, int64_t ld, QrGlobal* g, double2* lam) {
    __shared__ QrCtl outer, inner;
    __shared__ double sub[kWideShiftDim * kWideShiftDim];
    __shared__ double2 subev[kWideShiftDim];
    __shared__ double sub2[kShiftDim * kShiftDim];
    __shared__ double2 subev2[kShiftDim];
    __shared__ int sh_b, sh_exc, sh_u, sh_l;
    const int tid = threadIdx.x;
    // read once into LDS: thread 0 rewrites these fields below
    if (tid == 0) {
        sh_u = g->u;
        sh_l = g->split;
    }
    __syncthreads();
    const int u = sh_u, l = sh_l;
    if (l >= u - 1) {
        if (tid == 0) {
            if (l > 0) H[(int64_t)l * ld + l - 1] = 0.0;
            if (l == u) {
                lam[u] = make_double2(H[(int64_t)u * ld + u], 0.0);
                g->u = u - 1;
            } else {
                eig2(H[(int64_t)(u - 1) * ld + u - 1], H[(int64_t)(u - 1) * ld + u], H[(int64_t)u * ld + u - 1],
                     H[(int64_t)u * ld + u], &lam[u - 1], &lam[u]);
                g->u = u - 2;
            }
            g->its = 0;
            g->split = 0;
            g->action = 0;
        }
        return;
    }
    const int na = u - l + 1;
    if (na <= kSmallBlock) {
        if (tid == 0 && l > 0) H[(int64_t)l * ld + l - 1] = 0.0;
        __syncthreads();
        const int rc = qr_eigs<kMaxBulges>(H + (int64_t)l * ld + l, ld, na, lam + l, outer, &inner, sub2, subev2);
        if (tid == 0) {
            if (rc) g->status = 1;
            g->sweeps += outer.sweeps;
            g->steps += outer.steps;
            g->work += outer.work;
            g->u = l - 1;
            g->its = 0;
            g->split = 0;
            g->action = 0;
        }
        return;
    }
    if (tid == 0) {
        if (l > 0) H[(int64_t)l * ld + l - 1] = 0.0;
        const int its = g->its + 1;
        g->its = its;
        if (its > kMaxIts) g->status = 1;
        sh_b = min(kWideBulges, max(1, na / 16));
        sh_exc = (its % 10) == 0;
    }
    __syncthreads();
    const int b = sh_b;
    if (sh_exc) {
        if (tid == 0) {
            const double w = H[(int64_t)u * ld + u] +
                             0.75 * (fabs(H[(int64_t)u * ld + u - 1]) + fabs(H[(int64_t)(u - 1) * ld + u - 2]));
            for (int i = 0; i < b; ++i) {
                g->s[i] = 2.0 * w;
                g->t[i] = w * w;
            }
        }
    } else {
        const int mm = 2 * b, o = u - mm + 1;
        for (int e = tid; e < mm * mm; e += kQrThreads) {
            const int r = e / mm, c = e % mm;
            sub[e] = r <= c + 1 ? H[(int64_t)(o + r) * ld + o + c] : 0.0;
        }
        __syncthreads();
        const int rc = qr_eigs<kMaxBulges>(sub, mm, mm, subev, outer, &inner, sub2, subev2);
        if (tid == 0) {
            const double a = H[(int64_t)(u - 1) * ld + u - 1], bb = H[(int64_t)(u - 1) * ld + u];
            const double c = H[(int64_t)u * ld + u - 1], d = H[(int64_t)u * ld + u];
            int np = 0;
            if (rc == 0) {
                double re[kWideShiftDim];
                int nr = 0;
                for (int i = 0; i < mm; ++i) {
                    const double2 z = subev[i];
                    if (z.y > 0.0) {
                        g->s[np] = 2.0 * z.x;
                        g->t[np] = z.x * z.x + z.y * z.y;
                        ++np;
                    } else if (z.y == 0.0) {
                        int q = nr++;
                        while (q > 0 && re[q - 1] > z.x) {
                            re[q] = re[q - 1];
                            --q;
                        }
                        re[q] = z.x;
                    }
                }
                for (int i = 0; i + 1 < nr && np < b; i += 2) {
                    g->s[np] = re[i] + re[i + 1];
                    g->t[np] = re[i] * re[i + 1];
                    ++np;
                }
            }
            for (int i = np; i < b; ++i) {  // a failed shift solve or unpaired leftovers: the trailing 2 x 2
                g->s[i] = np ? g->s[np - 1] : a + d;
                g->t[i] = np ? g->t[np - 1] : a * d - bb * c;
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        double x, y, z, beta;
        intro_xyz(H, ld, l, g->s[0], g->t[0], &x, &y, &z);
        house3(x, y, z, &g->tau[0][0], &g->w1[0][0], &g->w2[0][0], &beta);
        g->l = l;
        g->b = b;
        g->split = 0;
        g->action = 1;
    }
}

// Index (q, m), 0 <= m < q, of entry e of the triangular enumeration q(q-1)/2 + m.
__device__ __forceinline__ void tri_index(int e, int* q, int* m) {
    int r = (int)((1.0 + sqrt(1.0 + 8.0 * (double)e)) * 0.5);
    while (r * (r - 1) / 2 > e) --r;
    while (r * (r + 1) / 2 <= e) ++r;
    *q = r;
    *m = e - r * (r - 1) / 2;
}

// Reflector of bulge i (positions k..k+2, two entries where k + 2 > u) applied from the
// left to column c or from the right to row r.
__device__ __forceinline__ void refl_left(double* H, int64_t ld, int k, int u, double tau, double w1, double w2,
                                          int c) {
    double* a = H + (int64_t)k * ld + c;
    const bool three = k + 2 <= u;
    const double a0 = a[0], a1 = a[ld], a2 = three ? a[2 * ld] : 0.0;
    const double r = tau * (a0 + w1 * a1 + w2 * a2);
    a[0] = a0 - r;
    a[ld] = a1 - r * w1;
    if (three) a[2 * ld] = a2 - r * w2;
}

__device__ __forceinline__ void refl_right(double* H, int64_t ld, int k, int u, double tau, double w1, double w2,
                                           int row) {
    double* h = H + (int64_t)row * ld + k;
    const bool three = k + 2 <= u;
    const double h0 = h[0], h1 = h[1], h2 = three ? h[2] : 0.0;
    const double q = tau * (h0 + w1 * h1 + w2 * h2);
    h[0] = h0 - q;
    h[1] = h1 - q * w1;
    if (three) h[2] = h2 - q * w2;
}

// Step t of a device-wide sweep over [l, u] with b bulges (bulge i at k_i = l + t - kSep i,
// active for ilo <= i <= ihi), both sides in one launch. A left reflection of bulge i
// (rows k_i..k_i+2, columns k_i..u) and a right one of bulge j (columns k_j..k_j+2, rows
// l..k_j+3) meet only in the 3 x 3 block rows(i) x columns(j) with j <= i, where they
// commute; one thread applies both there (left first), so every entry has one writer:
//   left-only:  columns k_ilo+3..u of every active bulge (nb x tail pieces), and the gap
//               columns k_i + 4m + 3 between deeper strips (triangular),
//   right-only: rows l..k_ihi-1 of every active bulge (head x nb, bulge fastest: the strips
//               of one row are adjacent), and the gap rows k_i + 3, i > j (triangular),
//   crossings:  blocks (i, j), j < i (triangular),
//   owners:     thread i of block 0 takes block (i, i) and row k_i + 3, then builds bulge
//               i's next reflector from column k_i (or the first reflector of the bulge that
//               enters at step t + 1).
__global__ __launch_bounds__(256) void k_qr_step(double* H, int64_t ld, int l, int u, int b, int t, int ilo, int ihi,
                                                 int tail, int head, int total, QrGlobal* g) {
    const int p = t & 1;
    const int nb = ihi - ilo + 1;
    if (blockIdx.x == 0 && threadIdx.x < b) {
        const int i = threadIdx.x;
        const int k = l + t - kSep * i;
        double tn = 0.0, w1n = 0.0, w2n = 0.0;
        if (i >= ilo && i <= ihi) {
            const double tau = g->tau[p][i], w1 = g->w1[p][i], w2 = g->w2[p][i];
            const bool three = k + 2 <= u;
            const int nr = k + 3 <= u ? 4 : (three ? 3 : 2);  // rows k.. (row k+3 takes the right side only)
            double B[4][3];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    B[r][c] = (r < nr && (c < 2 || three)) ? H[(int64_t)(k + r) * ld + k + c] : 0.0;
            if (tau != 0.0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double v = tau * (B[0][c] + w1 * B[1][c] + w2 * B[2][c]);
                    B[0][c] -= v;
                    B[1][c] -= v * w1;
                    B[2][c] -= v * w2;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double v = tau * (B[r][0] + w1 * B[r][1] + w2 * B[r][2]);
                    B[r][0] -= v;
                    B[r][1] -= v * w1;
                    B[r][2] -= v * w2;
                }
            }
            const int kn = k + 1;
            double beta = 0.0;
            if (kn <= u - 1) house3(B[1][0], B[2][0], kn + 2 <= u ? B[3][0] : 0.0, &tn, &w1n, &w2n, &beta);
            if (tn != 0.0) {
                B[1][0] = beta;
                B[2][0] = 0.0;
                B[3][0] = 0.0;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (r < nr && (c < 2 || three)) H[(int64_t)(k + r) * ld + k + c] = B[r][c];
        } else if (i >= 1 && t + 1 == kSep * i) {
            double x, y, z, beta;
            intro_xyz(H, ld, l, g->s[i], g->t[i], &x, &y, &z);
            house3(x, y, z, &tn, &w1n, &w2n, &beta);
        }
        g->tau[p ^ 1][i] = tn;
        g->w1[p ^ 1][i] = w1n;
        g->w2[p ^ 1][i] = w2n;
    }
    int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= total || nb < 1) return;
    const int kilo = l + t - kSep * ilo, kihi = l + t - kSep * ihi;
    const int tri = nb * (nb - 1) / 2;
    if (e < nb * tail) {  // left-only tail columns
        const int i = ilo + e / tail, c = kilo + 3 + e % tail;
        const double tau = g->tau[p][i];
        if (tau != 0.0) refl_left(H, ld, l + t - kSep * i, u, tau, g->w1[p][i], g->w2[p][i], c);
        return;
    }
    e -= nb * tail;
    if (e < tri) {  // left-only gap columns
        int q, m;
        tri_index(e, &q, &m);
        const int i = ilo + q, k = l + t - kSep * i;
        const double tau = g->tau[p][i];
        if (tau != 0.0) refl_left(H, ld, k, u, tau, g->w1[p][i], g->w2[p][i], k + kSep * m + 3);
        return;
    }
    e -= tri;
    if (e < head * nb) {  // right-only head rows
        const int row = l + e / nb, j = ilo + e % nb;
        const double tau = g->tau[p][j];
        if (tau != 0.0) refl_right(H, ld, l + t - kSep * j, u, tau, g->w1[p][j], g->w2[p][j], row);
        return;
    }
    e -= head * nb;
    if (e < tri) {  // right-only gap rows k_i + 3 of bulge j < i
        int q, m;
        tri_index(e, &q, &m);
        const int i = ilo + q, j = ilo + m;
        const double tau = g->tau[p][j];
        if (tau != 0.0) refl_right(H, ld, l + t - kSep * j, u, tau, g->w1[p][j], g->w2[p][j], l + t - kSep * i + 3);
        return;
    }
    e -= tri;
    if (e < tri) {  // crossing block rows(i) x columns(j), j < i: left of i, then right of j
        int q, m;
        tri_index(e, &q, &m);
        const int i = ilo + q, j = ilo + m;
        const int ki = l + t - kSep * i, kj = l + t - kSep * j;
        const double ti = g->tau[p][i], tj = g->tau[p][j];
        const bool cj3 = kj + 2 <= u;
        if (ti != 0.0) {
            const double w1 = g->w1[p][i], w2 = g->w2[p][i];
            for (int c = 0; c < (cj3 ? 3 : 2); ++c) refl_left(H, ld, ki, u, ti, w1, w2, kj + c);
        }
        if (tj != 0.0) {
            const double w1 = g->w1[p][j], w2 = g->w2[p][j];
            for (int r = 0; r < 3; ++r) refl_right(H, ld, kj, u, tj, w1, w2, ki + r);
        }
    }
}

// ---------------------------------------------------------------------------
// Grid counts
// ---------------------------------------------------------------------------

__global__ void k_zero_i64(int64_t* x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0;
}

__global__ void k_hist(int64_t n, const double2* lam, double re0, double dx, double im0, double dy, int nx, int ny,
                       unsigned long long* counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 z = lam[i];
    const double tx = (z.x - re0) / dx;
    const double ty = (z.y - im0) / dy;
    if (tx >= 0.0 && tx < (double)nx && ty >= 0.0 && ty < (double)ny)
        atomicAdd(&counts[(int64_t)(int)floor(ty) * nx + (int)floor(tx)], 1ull);
}

// Workspace of the reduction, from the start of the context's workspace: v, p, q
// (M doubles each), tau and s, and the column pass's chunk partials.
// ---------------------------------------------------------------------------
// Stage 1, blocked: panels of kPanel reflectors in compact WY form, Q = 1 - V T V^T.
// Inside a panel only its columns are brought up to date (from the matrix A at the
// panel's start: col = A e_c - Y V^T e_c, then col -= V T^T V^T col), and Y = A V T
// grows by one GEMV over A per reflector, y_i = tau_i (A v_i - Y V^T v_i); after the
// panel the whole trailing matrix takes A - Y V^T from the right and
// (1 - V T^T V^T) from the left as four GEMMs, and the panel's entries below the
// subdiagonal are set to exactly zero. The matrix is read once per column instead of
// three times.
// ---------------------------------------------------------------------------

// col[r] = A[r][c] - sum_{k<i} Y[k][r] V[k][c]
__global__ __launch_bounds__(256) void k_bh_col(const double* A, int64_t lda, int M, int c, int i, const double* V,
                                                const double* Y, double* col) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= M) return;
    double s = A[(int64_t)r * lda + c];
    for (int k = 0; k < i; ++k) s -= Y[(int64_t)k * M + r] * V[(int64_t)k * M + c];
    col[r] = s;
}

// out[k] = sum_{r >= r0} V[k][r] x[r] for k < gridDim.x (a block per k, fixed order)
__global__ __launch_bounds__(256) void k_bh_dots(const double* V, int M, int r0, const double* x, double* out) {
    __shared__ double red[4];
    const double* vk = V + (int64_t)blockIdx.x * M;
    double s = 0.0;
    for (int r = r0 + threadIdx.x; r < M; r += 256) s = fma(vk[r], x[r], s);
    s = block_sum256(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// col[r] -= sum_{m<i} V[m][r] z[m], z = T^T w, for rows r > j0
__global__ __launch_bounds__(256) void k_bh_left(const double* V, int M, int i, int j0, const double* T,
                                                 const double* w, double* col) {
    __shared__ double z[kPanel];
    if (threadIdx.x < i) {
        double t = 0.0;
        for (int k = 0; k <= (int)threadIdx.x; ++k) t = fma(T[k + threadIdx.x * kPanel], w[k], t);
        z[threadIdx.x] = t;
    }
    __syncthreads();
    const int r = j0 + 1 + blockIdx.x * 256 + threadIdx.x;
    if (r >= M) return;
    double s = col[r];
    for (int m = 0; m < i; ++m) s -= V[(int64_t)m * M + r] * z[m];
    col[r] = s;
}

// Reflector i of the panel from col[c+1..M-1]: V[i] (zero above row c+1, 1 at c+1), tau, beta.
__global__ __launch_bounds__(256) void k_bh_house(const double* col, int M, int c, int i, double* V, double* taus,
                                                  double* betas) {
    __shared__ double red[4];
    __shared__ double bc[2];
    double s = 0.0;
    for (int r = c + 2 + threadIdx.x; r < M; r += 256) s = fma(col[r], col[r], s);
    const double sigma = block_sum256(s, red);
    double* vi = V + (int64_t)i * M;
    if (threadIdx.x == 0) {
        const double alpha = col[c + 1];
        double tau = 0.0, scale = 0.0, beta = alpha;
        if (sigma > 0.0) {
            beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        bc[0] = scale;
        taus[i] = tau;
        betas[i] = beta;
        vi[c + 1] = 1.0;
    }
    __syncthreads();
    const double scale = bc[0];
    for (int r = c + 2 + threadIdx.x; r < M; r += 256) vi[r] = col[r] * scale;
}

// y[r] = sum_{cc > c} A[r][cc] v[cc]: one wavefront per row, the row-dot loop of
// the one-state GEMV. The dot starts at the even column c0 <= c + 1 so that,
// with 16-byte aligned rows (ALIGNED), every lane reads 16-byte pieces; v is
// zero above c + 1, so the extra column adds nothing.
template <bool ALIGNED>
__global__ __launch_bounds__(256) void k_bh_gemv(const double* A, int64_t lda, int M, int c, const double* v,
                                                 double* y) {
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= M) return;
    const int c0 = (c + 1) & ~1;
    const double* row[1] = {A + (int64_t)r * lda + c0};
    double s[1];
    wave_rowdots<1, ALIGNED, true>(row, v + c0, M - c0, lane, s);
    if (lane == 0) y[r] = s[0];
}

// Y[i][r] = tau (y[r] - sum_{k<i} Y[k][r] u[k]); block 0 also writes column i of T:
// T[m][i] = -tau sum_{m<=k<i} T[m][k] u[k], T[i][i] = tau.
__global__ __launch_bounds__(256) void k_bh_ycol(int M, int i, const double* y, const double* u, const double* taus,
                                                 double* Y, double* T) {
    const double tau = taus[i];
    if (blockIdx.x == 0 && threadIdx.x <= (unsigned)i) {
        const int m = threadIdx.x;
        if (m == i) {
            T[i + i * kPanel] = tau;
        } else {
            double t = 0.0;
            for (int k = m; k < i; ++k) t = fma(T[m + k * kPanel], u[k], t);
            T[m + i * kPanel] = -tau * t;
        }
    }
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= M) return;
    double s = y[r];
    for (int k = 0; k < i; ++k) s -= Y[(int64_t)k * M + r] * u[k];
    Y[(int64_t)i * M + r] = tau * s;
}

// Panel columns j0..j0+ib-1: beta on the subdiagonal, exact zeros below it.
__global__ void k_bh_fix(double* A, int64_t lda, int M, int j0, const double* betas) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int c = j0 + blockIdx.y;
    if (r < c + 1 || r >= M) return;
    A[(int64_t)r * lda + c] = r == c + 1 ? betas[blockIdx.y] : 0.0;
}

__global__ void k_bh_zero(double* x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

// Workspace of the blocked reduction (from the start of the workspace): the panel's
// reflectors V, Y = A V T and the two GEMM temporaries (M x kPanel each, column-major
// with leading dimension M), the current column and the GEMV result (M each), T
// (kPanel x kPanel, column-major), small vectors (w, u, tau, beta).
struct BlockedLayout {
    size_t V, Y, W, W2, col, y, T, w, u, tau, beta, end;
    explicit BlockedLayout(int M) {
        const size_t mat = lb_align(sizeof(double) * (size_t)M * kPanel, 256);
        const size_t vec = lb_align(sizeof(double) * (size_t)M, 256);
        const size_t sm = lb_align(sizeof(double) * kPanel, 256);
        V = 0;
        Y = mat;
        W = 2 * mat;
        W2 = 3 * mat;
        col = 4 * mat;
        y = col + vec;
        T = y + vec;
        w = T + lb_align(sizeof(double) * kPanel * kPanel, 256);
        u = w + sm;
        tau = u + sm;
        beta = tau + sm;
        end = beta + sm;
    }
};

struct HessLayout {
    size_t v, p, q, sc, qp, end;
    explicit HessLayout(int M) {
        const size_t vec = lb_align(sizeof(double) * (size_t)M, 256);
        v = 0;
        p = vec;
        q = 2 * vec;
        sc = 3 * vec;
        qp = sc + 256;
        end = std::max(lb_align(qp + sizeof(double) * (size_t)kMaxChunks * M, 256), BlockedLayout(M).end);
    }
};

}  // namespace

namespace {

// The blocked reduction. The products work column-major: the row-major A is the column-major
// X = A^T with leading dimension lda, so A[:, j0:] -= Y V^T is X[j0:, :] -= V Y^T, and the
// left update of A[j0+1:, j0:] is X[j0:, j0+1:] -= (X[j0:, j0+1:] V T) V^T over rows j0+1..
// of V.
int hessenberg_blocked(lb_ctx* c, int M, double* A, int64_t lda) {
    hipStream_t s = c->stream;
    const BlockedLayout lay(M);
    // rows 16-byte aligned: the GEMV reads 16-byte pieces (V's rows start on 256 bytes)
    const bool aligned = (lda % 2) == 0 && ((uintptr_t)A % 16) == 0 && (M % 2) == 0;
    char* ws = (char*)c->ws;
    double* V = (double*)(ws + lay.V);
    double* Y = (double*)(ws + lay.Y);
    double* W = (double*)(ws + lay.W);
    double* W2 = (double*)(ws + lay.W2);
    double* col = (double*)(ws + lay.col);
    double* y = (double*)(ws + lay.y);
    double* T = (double*)(ws + lay.T);
    double* w = (double*)(ws + lay.w);
    double* u = (double*)(ws + lay.u);
    double* taus = (double*)(ws + lay.tau);
    double* betas = (double*)(ws + lay.beta);
    for (int j0 = 0; j0 + 2 < M; j0 += kPanel) {
        const int ib = std::min(kPanel, M - 2 - j0);
        hipLaunchKernelGGL(k_bh_zero, dim3(lb_blocks((int64_t)M * kPanel, 256)), dim3(256), 0, s, V,
                           (int64_t)M * kPanel);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_bh_zero, dim3(lb_blocks(kPanel * kPanel, 256)), dim3(256), 0, s, T,
                           (int64_t)kPanel * kPanel);
        LB_CHECK_LAUNCH();
        for (int i = 0; i < ib; ++i) {
            const int cc = j0 + i;
            hipLaunchKernelGGL(k_bh_col, dim3(lb_blocks(M, 256)), dim3(256), 0, s, (const double*)A, lda, M, cc, i,
                               (const double*)V, (const double*)Y, col);
            LB_CHECK_LAUNCH();
            if (i > 0) {
                hipLaunchKernelGGL(k_bh_dots, dim3(i), dim3(256), 0, s, (const double*)V, M, j0 + 1,
                                   (const double*)col, w);
                LB_CHECK_LAUNCH();
                hipLaunchKernelGGL(k_bh_left, dim3(lb_blocks(M - j0 - 1, 256)), dim3(256), 0, s, (const double*)V, M,
                                   i, j0, (const double*)T, (const double*)w, col);
                LB_CHECK_LAUNCH();
            }
            hipLaunchKernelGGL(k_bh_house, dim3(1), dim3(256), 0, s, (const double*)col, M, cc, i, V, taus, betas);
            LB_CHECK_LAUNCH();
            if (i > 0) {
                hipLaunchKernelGGL(k_bh_dots, dim3(i), dim3(256), 0, s, (const double*)V, M, cc + 1,
                                   (const double*)(V + (int64_t)i * M), u);
                LB_CHECK_LAUNCH();
            }
            if (aligned)
                hipLaunchKernelGGL(k_bh_gemv<true>, dim3(lb_blocks(M, 4)), dim3(256), 0, s, (const double*)A, lda, M,
                                   cc, (const double*)(V + (int64_t)i * M), y);
            else
                hipLaunchKernelGGL(k_bh_gemv<false>, dim3(lb_blocks(M, 4)), dim3(256), 0, s, (const double*)A, lda, M,
                                   cc, (const double*)(V + (int64_t)i * M), y);
            LB_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_bh_ycol, dim3(lb_blocks(M, 256)), dim3(256), 0, s, M, i, (const double*)y,
                               (const double*)u, (const double*)taus, Y, T);
            LB_CHECK_LAUNCH();
        }
        int rc;
        // A[:, j0:] -= Y V^T
        if ((rc = lb_impl_gemm_f64(s, false, true, M - j0, M, ib, -1.0, V + j0, M, Y, M, 1.0, A + j0, lda)))
            return rc;
        // W^T = X[j0:, j0+1:] V[j0+1:], W2^T = W^T T, X[j0:, j0+1:] -= W2^T V[j0+1:]^T
        double* Xb = A + j0 + (int64_t)(j0 + 1) * lda;
        if ((rc = lb_impl_gemm_f64(s, false, false, M - j0, ib, M - j0 - 1, 1.0, Xb, lda, V + j0 + 1, M, 0.0, W,
                                   M)) ||
            (rc = lb_impl_gemm_f64(s, false, false, M - j0, ib, ib, 1.0, W, M, T, kPanel, 0.0, W2, M)) ||
            (rc = lb_impl_gemm_f64(s, false, true, M - j0, M - j0 - 1, ib, -1.0, W2, M, V + j0 + 1, M, 1.0, Xb,
                                   lda)))
            return rc;
        hipLaunchKernelGGL(k_bh_fix, dim3(lb_blocks(M, 256), ib), dim3(256), 0, s, A, lda, M, j0,
                           (const double*)betas);
        LB_CHECK_LAUNCH();
        lb_report(c, "hessenberg", (double)(j0 + ib) / (M - 2));
    }
    return LB_OK;
}

}  // namespace

int lb_impl_hessenberg(lb_ctx* c, int M, double* A, int64_t lda) {
    hipStream_t s = c->stream;
    const HessLayout lay(M);
    if (M >= kBlockedMin) {
        int rc = lb_ws_reserve(c, lay.end);
        if (rc) return rc;
        return hessenberg_blocked(c, M, A, lda);
    }
    const size_t o_v = lay.v, o_p = lay.p, o_q = lay.q, o_sc = lay.sc, o_qp = lay.qp;
    int rc = lb_ws_reserve(c, lay.end);
    if (rc) return rc;
    char* ws = (char*)c->ws;
    double* v = (double*)(ws + o_v);
    double* p = (double*)(ws + o_p);
    double* q = (double*)(ws + o_q);
    double* sc = (double*)(ws + o_sc);
    double* qpart = (double*)(ws + o_qp);
    for (int j = 0; j + 2 < M; ++j) {
        const int L = M - j - 1;
        hipLaunchKernelGGL(k_hh_house, dim3(1), dim3(256), 0, s, A, lda, M, j, v, sc);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_hh_p, dim3(lb_blocks(M, 4)), dim3(256), 0, s, (const double*)A, lda, M, j,
                           (const double*)v, p);
        LB_CHECK_LAUNCH();
        // enough row chunks for about 2048 blocks, none shorter than kChunkRows rows
        const int cb = (int)lb_blocks(L, 256);
        int nch = std::min((int)lb_blocks(L, kChunkRows), std::max(1, 2048 / cb));
        if (nch > kMaxChunks) nch = kMaxChunks;
        const int rows_per_chunk = (L + nch - 1) / nch;
        nch = (L + rows_per_chunk - 1) / rows_per_chunk;
        hipLaunchKernelGGL(k_hh_q, dim3(cb, nch), dim3(256), 0, s, (const double*)A, lda, M, j, (const double*)v,
                           qpart, rows_per_chunk);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_hh_qfin, dim3(lb_blocks(L, 64) + 1), dim3(256), 0, s, M, j, nch, (const double*)qpart,
                           (const double*)v, (const double*)p, q, sc);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_hh_update, dim3(lb_blocks(L, 64), lb_blocks(M, 16)), dim3(256), 0, s, A, lda, M, j,
                           (const double*)v, (const double*)p, (const double*)q, (const double*)sc);
        LB_CHECK_LAUNCH();
        if ((j & 255) == 255) lb_report(c, "hessenberg", (double)(j + 1) / (M - 2));
    }
    return LB_OK;
}

int lb_impl_spectrum(lb_ctx* c, int M, const double* Q, int64_t ldq, double* lam, int64_t* sweeps, int64_t* steps,
                     int64_t* work) {
    hipStream_t s = c->stream;
    // the working copy sits past the reduction's own scratch
    // the working copy's rows padded to 16 doubles (128 bytes) while M * ld keeps
    // within 32-bit element offsets
    int64_t ld = (M + 15) / 16 * 16;
    if ((int64_t)M * ld > (int64_t)INT32_MAX) ld = M;
    const size_t o_h = HessLayout(M).end;
    const size_t o_g = o_h + lb_align(sizeof(double) * (size_t)M * ld, 256);
    int rc = lb_ws_reserve(c, o_g + sizeof(QrGlobal));
    if (rc) return rc;
    rc = lb_host_reserve(c, sizeof(QrGlobal));
    if (rc) return rc;
    double* H = (double*)((char*)c->ws + o_h);
    QrGlobal* g = (QrGlobal*)((char*)c->ws + o_g);
    LB_HIP(hipMemcpy2DAsync(H, sizeof(double) * ld, Q, sizeof(double) * ldq, sizeof(double) * M, M,
                            hipMemcpyDeviceToDevice, s));
    rc = lb_impl_hessenberg(c, M, H, ld);
    if (rc) return rc;
    hipLaunchKernelGGL(k_qr_init, dim3(1), dim3(1024), 0, s, (const double*)H, ld, M, g);
    LB_CHECK_LAUNCH();
    int64_t n_sweeps = 0, n_steps = 0, n_work = 0;
    QrGlobal* hg = (QrGlobal*)c->host;
    int u = M - 1;
    // every pass either lowers u or counts a sweep, and sweeps per split are capped
    for (int64_t pass = 0; u >= 0; ++pass) {
        if (u >= 1) {
            hipLaunchKernelGGL(k_qr_scan, dim3(lb_blocks(u, 256)), dim3(256), 0, s, (const double*)H, ld, M, g);
            LB_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_qr_decide, dim3(1), dim3(kQrThreads), 0, s, H, ld, g, (double2*)lam);
        LB_CHECK_LAUNCH();
        LB_HIP(hipMemcpyAsync(hg, g, 8 * sizeof(int) + 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LB_HIP(hipStreamSynchronize(s));
        if (hg->status) return lb_fail(LB_ERR_NO_CONVERGENCE, "QR iteration: %d sweeps without a split", kMaxIts);
        if (hg->action == 1) {
            const int l = hg->l, b = hg->b;
            if (l < 0 || b < 1 || b > kWideBulges || u - l + 1 <= kSmallBlock)
                return lb_fail(LB_ERR_DEVICE, "QR iteration: inconsistent sweep l=%d u=%d b=%d", l, u, b);
            const int T = kSep * (b - 1) + (u - l);
            const int64_t na = u - l + 1;
            ++n_sweeps;
            n_steps += T;
            n_work += (int64_t)b * (na * na + 3 * na - 7);
            for (int t = 0; t < T; ++t) {
                const int ihi = std::min(b - 1, t / kSep);
                int ilo = 0;
                while (ilo <= ihi && l + t - kSep * ilo > u - 1) ++ilo;
                const int nb = ihi - ilo + 1;
                int tail = 0, head = 0, total = 0;
                if (nb >= 1) {
                    tail = std::max(0, u - (l + t - kSep * ilo) - 2);
                    head = (l + t - kSep * ihi) - l;
                    total = nb * tail + head * nb + 3 * (nb * (nb - 1) / 2);
                }
                hipLaunchKernelGGL(k_qr_step, dim3(std::max(1u, lb_blocks(total, 256))), dim3(256), 0, s, H, ld, l, u,
                                   b, t, ilo, ihi, tail, head, total, g);
                LB_CHECK_LAUNCH();
            }
        } else if (hg->u >= u) {
            return lb_fail(LB_ERR_DEVICE, "QR iteration: no progress at u=%d", u);
        }
        u = hg->u;
        if (u >= 0) lb_report(c, "qr", (double)(M - 1 - u) / M);
    }
    lb_report(c, "qr", 1.0);
    if (sweeps) *sweeps = n_sweeps + hg->sweeps;
    if (steps) *steps = n_steps + hg->steps;
    if (work) *work = n_work + hg->work;
    return LB_OK;
}

int lb_impl_spectrum_histogram(lb_ctx* c, int64_t n, const double* lam, double re0, double re1, double im0,
                               double im1, int nx, int ny, int64_t* counts) {
    hipStream_t s = c->stream;
    const int64_t cells = (int64_t)nx * ny;
    hipLaunchKernelGGL(k_zero_i64, dim3(lb_blocks(cells, 256)), dim3(256), 0, s, counts, cells);
    LB_CHECK_LAUNCH();
    if (n == 0) return LB_OK;
    const double dx = (re1 - re0) / nx, dy = (im1 - im0) / ny;
    hipLaunchKernelGGL(k_hist, dim3(lb_blocks(n, 256)), dim3(256), 0, s, n, (const double2*)lam, re0, dx, im0, dy,
                       nx, ny, (unsigned long long*)counts);
    LB_CHECK_LAUNCH();
    return LB_OK;
}
