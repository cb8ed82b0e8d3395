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
//     device (up to kWideBulges bulges in chains of kChain, each chain chased inside an
//     LDS window by one workgroup, the rest of the block updated by matrix-core
//     products of the window's orthogonal factor); smaller blocks, and the shift
//     problems, by one workgroup (up to kMaxBulges bulges, two barrier phases per
//     chain step). The 2b shifts of a b-bulge chain are the eigenvalues of
//     the trailing 2b x 2b block, found by the same iteration on a copy in LDS
//     (recursively, down to one bulge). A block splits off where a
//     subdiagonal entry falls below eps (|h_k-1,k-1| + |h_kk|), below eps ||H||_F after
//     ten sweeps without a split and below sqrt(n) eps ||H||_F after twenty (clusters at
//     the rounding floor; ||H||_F of the whole matrix, also for its diagonal blocks);
//     1 x 1 and 2 x 2 blocks give their eigenvalues
//     directly. Every tenth sweep without a split takes an exceptional shift to break
//     cycles; kMaxIts sweeps without one is an error.
#include "lb_internal.h"
#include "rowdot.h"
#include "qr_window.h"


#include <float.h>
#include <algorithm>
#include <math.h>

namespace {

using namespace lb_qr;

constexpr int kQrThreads = 1024;
constexpr int kMaxBulges = 16;              // 32 shifts per sweep
constexpr int kShiftDim = 2 * kMaxBulges;   // trailing block solved for the shifts
static_assert(kQrThreads / 64 >= kMaxBulges, "the one-workgroup sweep gives each bulge a wave");
constexpr int kMaxIts = 120;                // sweeps without a split before giving up
// Split tolerance of the shift problems (the trailing block whose eigenvalues become the next
// sweep's shifts): shifts need not be eigenvalues to the last bit, and a relative 1e-10 is far
// below the separations that set the convergence of the sweep they drive.
constexpr double kShiftTol = 1e-10;
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

// Reflector 1 - tau w w^T with w = (1, w1, w2) mapping (x, y, z) to (beta, 0, 0). The
// entries are scaled by their 1-norm; with d = xs - bs (no cancellation: bs has the
// sign opposite to xs) one reciprocal 1 / (bs d) gives both tau = (bs - xs) / bs = -d / bs
// and 1 / d, so the reflector costs two divisions and a square root.
__device__ void house3(double x, double y, double z, double* tau, double* w1, double* w2, double* beta) {
    const double sc = fabs(x) + fabs(y) + fabs(z);
    if (sc == 0.0 || (y == 0.0 && z == 0.0)) {
        *tau = 0.0;
        *w1 = *w2 = 0.0;
        *beta = x;
        return;
    }
    const double rs = 1.0 / sc;
    const double xs = x * rs, ys = y * rs, zs = z * rs;
    const double bs = -copysign(sqrt(xs * xs + ys * ys + zs * zs), xs);
    const double d = xs - bs;
    const double r = 1.0 / (bs * d);
    const double rd = bs * r;
    *tau = -d * d * r;
    *w1 = ys * rd;
    *w2 = zs * rd;
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
// block through a nested BMAX = 1 solve on sub (kShiftDim^2 doubles, LDS). The normwise
// split tests scale with max(||H||_F, norm_floor): a diagonal block of a larger matrix
// passes that matrix's norm, so a block cut out of a cluster (a tiny norm of its own)
// deflates at the backward error the whole matrix allows. tol replaces eps in the split
// tests: DBL_EPSILON for blocks whose eigenvalues are results, kShiftTol for shift problems.
template <int BMAX>
__device__ int qr_eigs(double* H, int64_t ld, int n, double2* lam, QrCtl& C, QrCtl* inner, double* sub,
                       double2* subev, double norm_floor, double tol) {
    const int tid = threadIdx.x;
    const double eps = tol;
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
        C.anorm = fmax(a > 0.0 ? sqrt(a) : 1.0, norm_floor);
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
                const int rc = qr_eigs<1>(sub, mm, mm, subev, *inner, nullptr, nullptr, nullptr, 0.0, kShiftTol);
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
            // from the left: wave i - ilo takes bulge i, lanes along its columns k..u
            const int wv = tid >> 6, lane = tid & 63;
            if (ilo + wv <= ihi) {
                const int i = ilo + wv;
                const double tau = C.tau[p][i];
                if (tau != 0.0) {
                    const int k = l + t - kSep * i;
                    const double w1 = C.w1[p][i], w2 = C.w2[p][i];
                    const bool three = k + 2 <= u;
                    for (int c = k + lane; c <= u; c += 64) {
                        const int off = k * ld32 + c;
                        const double a0 = H[off], a1 = H[off + ld32], a2 = three ? H[off + 2 * ld32] : 0.0;
                        const double r = tau * (a0 + w1 * a1 + w2 * a2);
                        H[off] = a0 - r;
                        H[off + ld32] = a1 - r * w1;
                        if (three) H[off + 2 * ld32] = a2 - r * w2;
                    }
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
            // the rest: wave i - ilo takes bulge i's rows l..k
            if (ilo + wv <= ihi) {
                const int i = ilo + wv;
                const double tau = C.tau[p][i];
                if (tau != 0.0) {
                    const int k = l + t - kSep * i;
                    const double w1 = C.w1[p][i], w2 = C.w2[p][i];
                    const bool three = k + 2 <= u;
                    for (int row = l + lane; row <= k; row += 64) {
                        const int off = row * ld32 + k;
                        const double a0 = H[off], a1 = H[off + 1], a2 = three ? H[off + 2] : 0.0;
                        const double r = tau * (a0 + w1 * a1 + w2 * a2);
                        H[off] = a0 - r;
                        H[off + 1] = a1 - r * w1;
                        if (three) H[off + 2] = a2 - r * w2;
                    }
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
// Stage 2 on the whole device: the host-driven iteration
// ---------------------------------------------------------------------------

// Blocks of at most kSmallBlock rows are finished by one workgroup (qr_eigs);
// sweeps over larger blocks run as windowed rounds over the whole device (below).
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
    double tau[kWideBulges], w1[kWideBulges], w2[kWideBulges];  // each bulge's reflector for its next step
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

// Whether subdiagonal entry k is negligible (the test of qr_eigs, n the order of the whole
// matrix, its the sweeps since the last split).
__device__ bool qr_negligible(const double* H, int64_t ld, int k, int n, int its, double anorm) {
    const double sd = fabs(H[(int64_t)k * ld + k - 1]);
    double tst = fabs(H[(int64_t)(k - 1) * ld + k - 1]) + fabs(H[(int64_t)k * ld + k]);
    const double floor_scale = its >= 20 ? sqrt((double)n) * anorm : (its >= 10 ? anorm : 0.0);
    tst = tst == 0.0 ? fmax(anorm, floor_scale) : fmax(tst, floor_scale);
    return sd <= DBL_EPSILON * tst;
}

// The largest k in [1, u] with a negligible subdiagonal entry.
__global__ void k_qr_scan(const double* H, int64_t ld, int n, QrGlobal* g) {
    const int k = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int u = g->u;
    if (k > u) return;
    if (qr_negligible(H, ld, k, n, g->its, g->anorm)) atomicMax(&g->split, k);
}

// One decision on the bottom block [split, u]: the eigenvalues of a 1 x 1 or 2 x 2
// block, a whole small block by qr_eigs, or the set-up of a device-wide sweep
// (the shifts, eigenvalues of the trailing block).
__global__ __launch_bounds__(kQrThreads) void k_qr_decide(double* H, int64_t ld, int n, QrGlobal* g, double2* lam) {
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
            // the bottom 1 x 1 or 2 x 2 block, then the next ones for as long as the new bottom
            // splits off again: the passes a scan and this branch would make next (after a
            // deflation its = 0, and the largest negligible k in [1, v] is v or v - 1 exactly
            // when these tests pass), taken here without a round trip to the host
            int v = u, k = l;
            for (;;) {
                if (k > 0) H[(int64_t)k * ld + k - 1] = 0.0;
                if (k == v) {
                    lam[v] = make_double2(H[(int64_t)v * ld + v], 0.0);
                } else {
                    eig2(H[(int64_t)(v - 1) * ld + v - 1], H[(int64_t)(v - 1) * ld + v], H[(int64_t)v * ld + v - 1],
                         H[(int64_t)v * ld + v], &lam[v - 1], &lam[v]);
                }
                v = k - 1;
                if (v <= 0) {
                    k = 0;  // rows 0..v: a 1 x 1 block (v = 0) or nothing left (v < 0)
                    if (v < 0) break;
                } else if (qr_negligible(H, ld, v, n, 0, g->anorm)) {
                    k = v;
                } else if (v == 1 || qr_negligible(H, ld, v - 1, n, 0, g->anorm)) {
                    k = v - 1;
                } else {
                    break;
                }
            }
            g->u = v;
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
        const int rc = qr_eigs<kMaxBulges>(H + (int64_t)l * ld + l, ld, na, lam + l, outer, &inner, sub2, subev2,
                                            g->anorm, DBL_EPSILON);
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
        const int rc = qr_eigs<kMaxBulges>(sub, mm, mm, subev, outer, &inner, sub2, subev2, 0.0, kShiftTol);
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
    if (tid == 0) {  // the bulges' first reflectors are built by the chase as they enter
        g->l = l;
        g->b = b;
        g->split = 0;
        g->action = 1;
    }
}

// ---------------------------------------------------------------------------
// Stage 2, level 3: sweeps as chains of bulges chased inside windows
// ---------------------------------------------------------------------------
//
// The b bulges of a device-wide sweep travel as chains of kChain bulges, kSep rows
// apart inside a chain; chain c enters kChainGap steps after chain c - 1, far enough
// that the windows of two chains never overlap. A round advances every chain by
// kAdvance steps. One workgroup per chain loads into LDS the kWin x kWin diagonal
// window holding every row and column its bulges touch in these steps, chases the
// chain there (the reflectors and the order of the direct sweep: left sides, then
// right sides, step by step) and accumulates the window's orthogonal factor U as
// U^T, one reflector at a time from the left. The rest of the active block gets
// the round at once: the window's rows to its right, X <- U^T X, and its columns
// above it, Y <- Y U, as FP64 matrix-core products. Left and right products
// commute, so where one chain's rows cross another chain's columns both apply in
// either order; the row products of all chains run in one launch, the column
// products in the next. Per round a chain moves kChain kAdvance bulge steps for
// 4 kWin^2 flop per row of the block, instead of 3 entries read and written per
// row and bulge step.
constexpr int kWinThreads = 512;
constexpr int kWinCols = 16 * (kWinThreads / 64);   // columns (rows) of the block per product pass
constexpr int kRowPasses = 1;                       // passes of a row-product workgroup over one staged U^T
constexpr int kColPasses = 2;                       // passes of a column-product workgroup (fewer registers)

typedef double qr_gd4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ qr_gd4 mfma_f64(double a, double b, qr_gd4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One round of chain blockIdx.x: load the window, chase kAdvance steps, store the
// window, U^T (kWin x kWin, rows of length kWin, at Ut_all + c kWin^2) and the
// reflectors pending for the next step (g->tau etc., by bulge). Wave j carries bulge
// j: its left side (lanes along the window columns K.., then along the columns of U^T's
// band for rows K..K+2: at most two columns per lane) and its right side (lanes along the
// rows above the bulge); every lane of the wave applies the right side to the bulge's own
// three rows below it and builds the next reflector from column K, so the reflector stays
// in registers. Two barriers per step order the sides of neighbouring bulges where they
// cross. The bulge index, its rows and its reflector are the same in every lane of a wave
// (read from the first lane), so each step's conditions are scalar branches; every load
// of a step is issued unconditionally from inside the LDS array (the array has a tail for
// the rows and columns an idle lane would read past the window) and only the stores are
// masked.
__device__ __forceinline__ void win_refl3(double* a, int ld, bool three, double tau, double w1, double w2, double a0,
                                          double a1, double a2) {
    const double r = tau * (a0 + w1 * a1 + w2 * a2);
    a[0] = a0 - r;
    a[ld] = a1 - r * w1;
    if (three) a[2 * ld] = a2 - r * w2;
}

// x as the wave's first active lane holds it, in scalar registers from here on; callers
// pass a value that is already the same in every lane (all lanes compute it alike).
__device__ __forceinline__ double wave_first(double x) {
    const long long v = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readfirstlane((int)v), hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(kWinThreads) void k_win_chase(double* H, int64_t ld, int l, int u, int b, int t0,
                                                           QrGlobal* g, double* Ut_all) {
    __shared__ double lds[kWinLds];
    double* const Hw = lds;
    double* const Uw = lds + kWin * kWinLd;
    constexpr int kRowsPerWave = kWin / (kWinThreads / 64);
    const int c = blockIdx.x;
    const WinGeom G = win_geom(l, u, b, c, t0);
    if (!G.active) return;
    const int ws = G.ws, wc = G.we - G.ws + 1;
    const int nbc = min(kChain, b - c * kChain), i0 = c * kChain;
    const int lu = u - ws, ll = l - ws;  // the block's last and first rows in window coordinates
    const int lane = threadIdx.x & 63;
    const int j = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    {
        // wave j loads window rows j, j + 8, ...: all its loads in flight together; entries
        // more than three below the diagonal are zero (Hessenberg plus bulges)
        double v[kRowsPerWave][2];
#pragma unroll
        for (int i = 0; i < kRowsPerWave; ++i)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = j + i * (kWinThreads / 64), q = lane + 64 * h;
                v[i][h] = (r < wc && q < wc && r <= q + 3) ? H[(int64_t)(ws + r) * ld + ws + q] : 0.0;
            }
#pragma unroll
        for (int i = 0; i < kRowsPerWave; ++i)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = j + i * (kWinThreads / 64), q = lane + 64 * h;
                if (r < wc && q < wc) {
                    Hw[r * kWinLd + q] = v[i][h];
                    Uw[r * kWinLd + q] = r == q ? 1.0 : 0.0;
                }
            }
    }
    const bool mine = j < nbc;
    double tau = 0.0, w1 = 0.0, w2 = 0.0;
    if (mine) {
        tau = g->tau[i0 + j];
        w1 = g->w1[i0 + j];
        w2 = g->w2[i0 + j];
    }
    __syncthreads();
    for (int s = 0; s < kAdvance; ++s) {
        const int rel = t0 + s - c * kChainGap;  // bulge j at block row l + rel - kSep j
        // some bulge of the chain active in this step (the same answer in every wave)
        const int jhi = rel < 0 ? -1 : min(nbc - 1, rel / kSep);
        const int over = rel - (u - 1 - l);
        const int jlo = over > 0 ? (over + kSep - 1) / kSep : 0;
        if (jlo > jhi) continue;
        const int K = ll + rel - kSep * j;  // window row of bulge j's reflector
        const bool act = mine && j >= jlo && j <= jhi;
        if (act && rel == kSep * j) {
            // bulge j enters at the top of the block (then ws == l): its first reflector
            double x, y, z, beta;
            intro_xyz(Hw, kWinLd, ll, g->s[i0 + j], g->t[i0 + j], &x, &y, &z);
            house3(x, y, z, &tau, &w1, &w2, &beta);
            tau = wave_first(tau);
            w1 = wave_first(w1);
            w2 = wave_first(w2);
        }
        const bool three = K + 2 <= lu;
        // left side: rows K..K+2 of window columns K..wc-1, then of U^T's columns lo..hi
        if (act && tau != 0.0) {
            const int nh = wc - K, lo = win_ut_lo(K), n = nh + win_ut_hi(K, wc) - lo + 1;
            double* p[2];
            double a[2][3];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // window column K + t, else U^T column lo + t - nh (idle lanes: lo or hi)
                const int t = lane + 64 * h;
                const int cu = lo + min(max(t - nh, 0), n - nh - 1);
                const int off = t < nh ? K + t : kWin * kWinLd + cu;
                p[h] = lds + K * kWinLd + off;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                a[h][0] = p[h][0];
                a[h][1] = p[h][kWinLd];
                const double x2 = p[h][2 * kWinLd];
                a[h][2] = three ? x2 : 0.0;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
                if (lane + 64 * h < n) win_refl3(p[h], kWinLd, three, tau, w1, w2, a[h][0], a[h][1], a[h][2]);
        }
        __syncthreads();
        // right side: rows 0..K of columns K..K+2, then (every lane) rows K+1..K+3 and the
        // next reflector from column K
        if (act) {
            const bool hi_rows = K >= 64;
            double* pa = Hw + lane * kWinLd + K;
            double* pb = Hw + (lane + 64) * kWinLd + K;
            double a[2][3], hr[3][3];
            a[0][0] = pa[0];
            a[0][1] = pa[1];
            const double x02 = pa[2];
            a[0][2] = three ? x02 : 0.0;
            if (hi_rows) {
                a[1][0] = pb[0];
                a[1][1] = pb[1];
                const double x12 = pb[2];
                a[1][2] = three ? x12 : 0.0;
            }
            const bool full = K + 3 <= lu;  // all three rows below the bulge inside the block
#pragma unroll
            for (int rr = 0; rr < 3; ++rr)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) hr[rr][cc] = Hw[(K + 1 + rr) * kWinLd + K + cc];
            if (!full) {
#pragma unroll
                for (int rr = 0; rr < 3; ++rr)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc)
                        if (!(K + 1 + rr <= lu && (cc < 2 || three))) hr[rr][cc] = 0.0;
            }
            if (tau != 0.0) {
                if (lane <= K) win_refl3(pa, 1, three, tau, w1, w2, a[0][0], a[0][1], a[0][2]);
                if (hi_rows && lane + 64 <= K) win_refl3(pb, 1, three, tau, w1, w2, a[1][0], a[1][1], a[1][2]);
#pragma unroll
                for (int rr = 0; rr < 3; ++rr) {
                    const double q = tau * (hr[rr][0] + w1 * hr[rr][1] + w2 * hr[rr][2]);
                    hr[rr][0] -= q;
                    hr[rr][1] -= q * w1;
                    hr[rr][2] -= q * w2;
                }
            }
            const int kn = K + 1;
            double tn = 0.0, w1n = 0.0, w2n = 0.0, beta = 0.0;
            if (kn <= lu - 1) house3(hr[0][0], hr[1][0], kn + 2 <= lu ? hr[2][0] : 0.0, &tn, &w1n, &w2n, &beta);
            tau = wave_first(tn);
            w1 = wave_first(w1n);
            w2 = wave_first(w2n);
            if (tau != 0.0) {
                hr[0][0] = beta;
                hr[1][0] = 0.0;
                hr[2][0] = 0.0;
            }
            if (lane == 0) {
#pragma unroll
                for (int rr = 0; rr < 3; ++rr)
#pragma unroll
                    for (int cc = 0; cc < 3; ++cc)
                        if (full || (K + 1 + rr <= lu && (cc < 2 || three)))
                            Hw[(K + 1 + rr) * kWinLd + K + cc] = hr[rr][cc];
            }
        }
        __syncthreads();
    }
    double* Ut = Ut_all + (size_t)c * kWin * kWin;
    for (int r = j; r < wc; r += kWinThreads / 64)
        for (int q = lane; q < wc; q += 64) {
            if (r <= q + 3) H[(int64_t)(ws + r) * ld + ws + q] = Hw[r * kWinLd + q];
            Ut[r * kWin + q] = Uw[r * kWinLd + q];
        }
    if (mine && lane == 0) {
        g->tau[i0 + j] = tau;
        g->w1[i0 + j] = w1;
        g->w2[i0 + j] = w2;
    }
}

// U^T of chain c into LDS (kWin x kWin, zero outside the window's wc x wc): wave w takes rows
// w, w + 8, ..., lanes along the row, all its loads in flight before the stores.
__device__ __forceinline__ void win_stage_u(double* Us, const double* Ut_all, int c, int wc) {
    constexpr int RPW = kWin / (kWinThreads / 64);
    const double* Ut = Ut_all + (size_t)c * kWin * kWin;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double v[RPW][2];
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = w + i * (kWinThreads / 64), q = lane + 64 * h;
            v[i][h] = (r < wc && q < wc) ? Ut[r * kWin + q] : 0.0;
        }
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = w + i * (kWinThreads / 64), q = lane + 64 * h;
            if (q < kWin) Us[r * kWinLd + q] = v[i][h];
        }
}

// X <- U^T X on the window's rows right of it: the near columns we+1..nb (far = 0) or the
// far columns nb+1..u (far = 1), nb = win_row_split. A wave owns 16 columns: it loads their
// wc window rows (matrix-core B operand), multiplies, and stores them back, so the product
// is in place. D = U^T X in 16 x 16 tiles: lane l holds rows 4v + l/16 of column l % 16.
__global__ __launch_bounds__(kWinThreads) void k_win_rows(double* H, int64_t ld, int l, int u, int b, int t0,
                                                          const double* Ut_all, int far) {
    __shared__ double Us[kWin * kWinLd];
    const int c = blockIdx.y;
    const WinGeom G = win_geom(l, u, b, c, t0);
    if (!G.active) return;
    const int ws = G.ws, wc = G.we - G.ws + 1;
    const int nb = win_row_split(l, u, b, c, t0, G.we);
    const int cend = far ? u : nb;  // last column
    const int cfirst = (far ? nb + 1 : G.we + 1) + blockIdx.x * (kWinCols * kRowPasses);
    if (cfirst > cend) return;
    win_stage_u(Us, Ut_all, c, wc);
    __syncthreads();
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    for (int pass = 0; pass < kRowPasses; ++pass) {
        const int col = cfirst + pass * kWinCols + (threadIdx.x >> 6) * 16 + lr;
        if (col - lr > cend) break;  // the wave's 16 columns all past the end
        const bool cok = col <= cend;
        // the window rows in two halves (fewer registers, two workgroups per compute unit);
        // every load precedes every store, so the product stays in place
        constexpr int KH = kWin / 8;
        qr_gd4 acc[kWin / 16];
#pragma unroll
        for (int ri = 0; ri < kWin / 16; ++ri) acc[ri] = qr_gd4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            double xb[KH];
#pragma unroll
            for (int kk = 0; kk < KH; ++kk) {
                const int k = 4 * (kk + KH * half) + lk;
                xb[kk] = (cok && k < wc) ? H[(int64_t)(ws + k) * ld + col] : 0.0;
            }
#pragma unroll
            for (int kk = 0; kk < KH; ++kk)
#pragma unroll
                for (int ri = 0; ri < kWin / 16; ++ri)
                    if (win_live(ri, kk + KH * half))
                        acc[ri] = mfma_f64(Us[(16 * ri + lr) * kWinLd + 4 * (kk + KH * half) + lk], xb[kk], acc[ri]);
        }
        if (cok) {
#pragma unroll
            for (int ri = 0; ri < kWin / 16; ++ri)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = 16 * ri + 4 * v + lk;
                    if (r < wc) H[(int64_t)(ws + r) * ld + col] = acc[ri][v];
                }
        }
    }
}

// Y <- Y U on the window's columns above it: the near rows split..ws-1 (far = 0) or the far
// rows l..split-1 (far = 1). A wave owns 16 rows: it loads their wc window columns
// (matrix-core A operand), multiplies, and stores them back. D = Y U in 16 x 16 tiles:
// lane l holds rows 4v + l/16 of column l % 16.
__global__ __launch_bounds__(kWinThreads) void k_win_cols(double* H, int64_t ld, int l, int u, int b, int t0,
                                                          const double* Ut_all, int far) {
    __shared__ double Us[kWin * kWinLd];
    const int c = blockIdx.y;
    const WinGeom G = win_geom(l, u, b, c, t0);
    if (!G.active) return;
    const int ws = G.ws, wc = G.we - G.ws + 1;
    const int split = win_split(l, u, b, c, t0, ws);
    const int rfirst = far ? l : split, rend = far ? split : ws;  // rows rfirst .. rend-1
    const int rbeg = rfirst + blockIdx.x * (kWinCols * kColPasses);
    if (rbeg >= rend) return;
    win_stage_u(Us, Ut_all, c, wc);
    __syncthreads();
    const int lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    for (int pass = 0; pass < kColPasses; ++pass) {
        const int r0 = rbeg + pass * kWinCols + (threadIdx.x >> 6) * 16;
        if (r0 >= rend) break;
        const int row = r0 + lr;
        constexpr int KH = kWin / 8;
        qr_gd4 acc[kWin / 16];
#pragma unroll
        for (int ci = 0; ci < kWin / 16; ++ci) acc[ci] = qr_gd4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            double ya[KH];
#pragma unroll
            for (int kk = 0; kk < KH; ++kk) {
                const int k = 4 * (kk + KH * half) + lk;
                ya[kk] = (row < rend && k < wc) ? H[(int64_t)row * ld + ws + k] : 0.0;
            }
#pragma unroll
            for (int kk = 0; kk < KH; ++kk) {
#pragma unroll
                for (int ci = 0; ci < kWin / 16; ++ci)
                    if (win_live(ci, kk + KH * half))
                        acc[ci] = mfma_f64(ya[kk], Us[(16 * ci + lr) * kWinLd + 4 * (kk + KH * half) + lk], acc[ci]);
                __builtin_amdgcn_sched_barrier(0);  // keep each step's operand reads next to its products
            }
        }
#pragma unroll
        for (int ci = 0; ci < kWin / 16; ++ci)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = r0 + 4 * v + lk, q = 16 * ci + lr;
                if (r < rend && q < wc) H[(int64_t)r * ld + ws + q] = acc[ci][v];
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

// col[r] = A[r][c] - sum_{k<i} Y[k][r] V[k][c] (the columns of Y and V ldv apart)
__global__ __launch_bounds__(256) void k_bh_col(const double* A, int64_t lda, int M, int c, int i, const double* V,
                                                int ldv, const double* Y, double* col) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= M) return;
    double s = A[(int64_t)r * lda + c];
    for (int k = 0; k < i; ++k) s -= Y[(int64_t)k * ldv + r] * V[(int64_t)k * ldv + c];
    col[r] = s;
}

// out[k] = sum_{r >= r0} V[k][r] x[r] for k < gridDim.x (a block per k, fixed order)
__global__ __launch_bounds__(256) void k_bh_dots(const double* V, int ldv, int M, int r0, const double* x,
                                                 double* out) {
    __shared__ double red[4];
    const double* vk = V + (int64_t)blockIdx.x * ldv;
    double s = 0.0;
    for (int r = r0 + threadIdx.x; r < M; r += 256) s = fma(vk[r], x[r], s);
    s = block_sum256(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// col[r] -= sum_{m<i} V[m][r] z[m], z = T^T w, for rows r > j0
__global__ __launch_bounds__(256) void k_bh_left(const double* V, int ldv, int M, int i, int j0, const double* T,
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
    for (int m = 0; m < i; ++m) s -= V[(int64_t)m * ldv + r] * z[m];
    col[r] = s;
}

// Reflector i of the panel from col[c+1..M-1]: V[i] (zero above row c+1, 1 at c+1), tau, beta.
__global__ __launch_bounds__(256) void k_bh_house(const double* col, int M, int c, int i, double* V, int ldv,
                                                  double* taus, double* betas) {
    __shared__ double red[4];
    __shared__ double bc[2];
    double s = 0.0;
    for (int r = c + 2 + threadIdx.x; r < M; r += 256) s = fma(col[r], col[r], s);
    const double sigma = block_sum256(s, red);
    double* vi = V + (int64_t)i * ldv;
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

// y[r] = sum_{cc > c} A[r][cc] v[cc]: one wavefront per kGemvRows rows, the row-dot loop of
// the one-state GEMV. The dot starts at the even column c0 <= c + 1 so that,
// with 16-byte aligned rows (ALIGNED), every lane reads 16-byte pieces; v is
// zero above c + 1, so the extra column adds nothing.
constexpr int kGemvRows = 2;  // rows per wavefront: their streams in flight together, v read once (4 measured no faster)

template <bool ALIGNED>
__global__ __launch_bounds__(256) void k_bh_gemv(const double* A, int64_t lda, int M, int c, const double* v,
                                                 double* y) {
    const int r = kGemvRows * (blockIdx.x * 4 + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (r >= M) return;
    const int c0 = (c + 1) & ~1;
    const double* row[kGemvRows];
#pragma unroll
    for (int t = 0; t < kGemvRows; ++t) row[t] = A + (int64_t)(r + t < M ? r + t : r) * lda + c0;
    double s[kGemvRows];
    wave_rowdots<kGemvRows, ALIGNED, true>(row, v + c0, M - c0, lane, s);
    if (lane == 0) {
#pragma unroll
        for (int t = 0; t < kGemvRows; ++t)
            if (r + t < M) y[r + t] = s[t];
    }
}

// Y[i][r] = tau (y[r] - sum_{k<i} Y[k][r] u[k]); block 0 also writes column i of T:
// T[m][i] = -tau sum_{m<=k<i} T[m][k] u[k], T[i][i] = tau.
__global__ __launch_bounds__(256) void k_bh_ycol(int M, int i, const double* y, const double* u, const double* taus,
                                                 double* Y, int ldv, double* T) {
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
    for (int k = 0; k < i; ++k) s -= Y[(int64_t)k * ldv + r] * u[k];
    Y[(int64_t)i * ldv + r] = tau * s;
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
    size_t YVW, W, col, y, T, G, w, u, tau, beta, end;
    explicit BlockedLayout(int M) {
        // Y, V and W2 side by side, kPanel columns each, columns M rounded up to even apart
        const size_t blk = lb_align(sizeof(double) * (size_t)(M + 1) * 3 * kPanel, 256);
        const size_t mat = lb_align(sizeof(double) * (size_t)M * kPanel, 256);
        const size_t vec = lb_align(sizeof(double) * (size_t)M, 256);
        const size_t sm = lb_align(sizeof(double) * kPanel, 256);
        const size_t sq = lb_align(sizeof(double) * kPanel * kPanel, 256);
        YVW = 0;
        W = blk;
        col = W + mat;
        y = col + vec;
        T = y + vec;
        G = T + sq;
        w = G + sq;
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
// X = A^T with leading dimension lda. A panel's two-sided update, A - Y V^T from the right and
// then A[j0+1:, j0:] -= V W2^T from the left with W2 = W T, W[c] = sum_{r > j0} A1[r][c] V[r]
// taken on the right-updated A1, is one rank-2 kPanel update A[:, j0:] -= [Y V] [V W2]^T: W is
// formed from the panel-start A as W0 - V[j0:] G, G = Y[j0+1:]^T V[j0+1:], so the trailing
// matrix is read once for W0 and read and written once for the update.
int hessenberg_blocked(lb_ctx* c, int M, double* A, int64_t lda) {
    hipStream_t s = c->stream;
    const BlockedLayout lay(M);
    // Y, V and W2 (kPanel columns each) side by side, columns ldv apart, ldv even: every v_i starts
    // on 16 bytes, so the GEMV reads 16-byte pieces of A and v whenever A's rows do
    const int ldv = M + (M & 1);
    const bool aligned = (lda % 2) == 0 && ((uintptr_t)A % 16) == 0;
    char* ws = (char*)c->ws;
    double* Y = (double*)(ws + lay.YVW);
    double* V = Y + (size_t)kPanel * ldv;
    double* W2 = Y + (size_t)2 * kPanel * ldv;
    double* W = (double*)(ws + lay.W);
    double* G = (double*)(ws + lay.G);
    double* col = (double*)(ws + lay.col);
    double* y = (double*)(ws + lay.y);
    double* T = (double*)(ws + lay.T);
    double* w = (double*)(ws + lay.w);
    double* u = (double*)(ws + lay.u);
    double* taus = (double*)(ws + lay.tau);
    double* betas = (double*)(ws + lay.beta);
    for (int j0 = 0; j0 + 2 < M; j0 += kPanel) {
        const int ib = std::min(kPanel, M - 2 - j0);
        // Y, V, W2 start at zero: a last panel of ib < kPanel reflectors leaves its other columns zero
        hipLaunchKernelGGL(k_bh_zero, dim3(lb_blocks((int64_t)ldv * 3 * kPanel, 256)), dim3(256), 0, s, Y,
                           (int64_t)ldv * 3 * kPanel);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_bh_zero, dim3(lb_blocks(kPanel * kPanel, 256)), dim3(256), 0, s, T,
                           (int64_t)kPanel * kPanel);
        LB_CHECK_LAUNCH();
        for (int i = 0; i < ib; ++i) {
            const int cc = j0 + i;
            hipLaunchKernelGGL(k_bh_col, dim3(lb_blocks(M, 256)), dim3(256), 0, s, (const double*)A, lda, M, cc, i,
                               (const double*)V, ldv, (const double*)Y, col);
            LB_CHECK_LAUNCH();
            if (i > 0) {
                hipLaunchKernelGGL(k_bh_dots, dim3(i), dim3(256), 0, s, (const double*)V, ldv, M, j0 + 1,
                                   (const double*)col, w);
                LB_CHECK_LAUNCH();
                hipLaunchKernelGGL(k_bh_left, dim3(lb_blocks(M - j0 - 1, 256)), dim3(256), 0, s, (const double*)V, ldv,
                                   M, i, j0, (const double*)T, (const double*)w, col);
                LB_CHECK_LAUNCH();
            }
            hipLaunchKernelGGL(k_bh_house, dim3(1), dim3(256), 0, s, (const double*)col, M, cc, i, V, ldv, taus,
                               betas);
            LB_CHECK_LAUNCH();
            if (i > 0) {
                hipLaunchKernelGGL(k_bh_dots, dim3(i), dim3(256), 0, s, (const double*)V, ldv, M, cc + 1,
                                   (const double*)(V + (int64_t)i * ldv), u);
                LB_CHECK_LAUNCH();
            }
            if (aligned)
                hipLaunchKernelGGL(k_bh_gemv<true>, dim3(lb_blocks(M, 4 * kGemvRows)), dim3(256), 0, s, (const double*)A, lda, M,
                                   cc, (const double*)(V + (int64_t)i * ldv), y);
            else
                hipLaunchKernelGGL(k_bh_gemv<false>, dim3(lb_blocks(M, 4 * kGemvRows)), dim3(256), 0, s, (const double*)A, lda, M,
                                   cc, (const double*)(V + (int64_t)i * ldv), y);
            LB_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_bh_ycol, dim3(lb_blocks(M, 256)), dim3(256), 0, s, M, i, (const double*)y,
                               (const double*)u, (const double*)taus, Y, ldv, T);
            LB_CHECK_LAUNCH();
        }
        int rc;
        // W0 = X[j0:, j0+1:] V[j0+1:] on the panel-start matrix, G = Y[j0+1:]^T V[j0+1:],
        // W = W0 - V[j0:] G, W2[j0:] = W T, then X[j0:, :] -= [V W2][j0:] [Y V]^T
        double* Xb = A + j0 + (int64_t)(j0 + 1) * lda;
        if ((rc = lb_impl_gemm_f64(s, false, false, M - j0, ib, M - j0 - 1, 1.0, Xb, lda, V + j0 + 1, ldv, 0.0, W,
                                   M)) ||
            (rc = lb_impl_gemm_f64(s, true, false, ib, ib, M - j0 - 1, 1.0, Y + j0 + 1, ldv, V + j0 + 1, ldv, 0.0, G,
                                   kPanel)) ||
            (rc = lb_impl_gemm_f64(s, false, false, M - j0, ib, ib, -1.0, V + j0, ldv, G, kPanel, 1.0, W, M)) ||
            (rc = lb_impl_gemm_f64(s, false, false, M - j0, ib, ib, 1.0, W, M, T, kPanel, 0.0, W2 + j0, ldv)) ||
            (rc = lb_impl_gemm_f64(s, false, true, M - j0, M, 2 * kPanel, -1.0, V + j0, ldv, Y, ldv, 1.0, A + j0,
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

int lb_impl_spectrum(lb_ctx* c, int M, const double* Q, int64_t ldq, double* lam, lb_spectrum_info* info) {
    hipStream_t s = c->stream;
    // the working copy sits past the reduction's own scratch
    // the working copy's rows padded to 16 doubles (128 bytes) while M * ld keeps
    // within 32-bit element offsets
    int64_t ld = (M + 15) / 16 * 16;
    if ((int64_t)M * ld > (int64_t)INT32_MAX) ld = M;
    const size_t o_h = HessLayout(M).end;
    const size_t o_g = o_h + lb_align(sizeof(double) * (size_t)M * ld, 256);
    const size_t o_u = o_g + lb_align(sizeof(QrGlobal), 256);
    const size_t n_u1 = (size_t)(kWideBulges / kChain) * kWin * kWin;  // U^T of every chain of a round
    const size_t n_u = 2 * n_u1;  // two rounds: the far products of one overlap the next round's chase
    int rc = lb_ws_reserve(c, o_u + sizeof(double) * n_u);
    if (rc) return rc;
    rc = lb_host_reserve(c, sizeof(QrGlobal));
    if (rc) return rc;
    double* H = (double*)((char*)c->ws + o_h);
    QrGlobal* g = (QrGlobal*)((char*)c->ws + o_g);
    double* Ut = (double*)((char*)c->ws + o_u);
    rc = lb_aux_stream(c);
    if (rc) return rc;
    hipStream_t s2 = c->aux;
    LB_HIP(hipMemcpy2DAsync(H, sizeof(double) * ld, Q, sizeof(double) * ldq, sizeof(double) * M, M,
                            hipMemcpyDeviceToDevice, s));
    rc = lb_impl_hessenberg(c, M, H, ld);
    if (rc) return rc;
    hipLaunchKernelGGL(k_qr_init, dim3(1), dim3(1024), 0, s, (const double*)H, ld, M, g);
    LB_CHECK_LAUNCH();
    int64_t n_sweeps = 0, n_steps = 0, n_work = 0, n_rounds = 0, n_flops = 0;
    QrGlobal* hg = (QrGlobal*)c->host;
    int u = M - 1;
    // every pass either lowers u or counts a sweep, and sweeps per split are capped
    for (int64_t pass = 0; u >= 0; ++pass) {
        if (u >= 1) {
            hipLaunchKernelGGL(k_qr_scan, dim3(lb_blocks(u, 256)), dim3(256), 0, s, (const double*)H, ld, M, g);
            LB_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_qr_decide, dim3(1), dim3(kQrThreads), 0, s, H, ld, M, g, (double2*)lam);
        LB_CHECK_LAUNCH();
        LB_HIP(hipMemcpyAsync(hg, g, 8 * sizeof(int) + 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LB_HIP(hipStreamSynchronize(s));
        if (hg->status) return lb_fail(LB_ERR_NO_CONVERGENCE, "QR iteration: %d sweeps without a split", kMaxIts);
        if (hg->action == 1) {
            const int l = hg->l, b = hg->b;
            if (l < 0 || b < 1 || b > kWideBulges || u - l + 1 <= kSmallBlock)
                return lb_fail(LB_ERR_DEVICE, "QR iteration: inconsistent sweep l=%d u=%d b=%d", l, u, b);
            const int nch = (b + kChain - 1) / kChain;
            const int nbl = b - (nch - 1) * kChain;
            // chain steps until the last chain's last bulge has left the block
            const int T = (nch - 1) * kChainGap + kSep * (nbl - 1) + (u - l);
            const int64_t na = u - l + 1;
            ++n_sweeps;
            n_steps += T;
            n_work += (int64_t)b * (na * na + 3 * na - 7);
            // Round r: the chase, then on this stream the near parts of the products (what the next
            // round's chases read: win_row_split, win_split), then on the auxiliary stream the far
            // parts, which touch no window of the next round and so run during its chase. The near
            // parts of a round wait for the far parts of the one before (they share rows and
            // columns); the window factors alternate between two buffers.
            for (int t0 = 0, r = 0; t0 < T; t0 += kAdvance, ++r) {
                double* Ur = Ut + (size_t)(r & 1) * n_u1;
                int near_right = 0, far_right = 0, near_above = 0, far_above = 0;
                int below_ws = u + 1;  // first row of the chain ahead's window
                for (int ch = 0; ch < nch; ++ch) {
                    const WinGeom G = win_geom(l, u, b, ch, t0);
                    if (!G.active) continue;
                    if (G.ws < l || G.we >= below_ws || G.we - G.ws + 1 > kWin)
                        return lb_fail(LB_ERR_DEVICE, "QR iteration: window [%d, %d] of chain %d in [%d, %d]", G.ws, G.we,
                                       ch, l, u);
                    below_ws = G.ws;
                    const int split = win_split(l, u, b, ch, t0, G.ws);
                    const int nb = win_row_split(l, u, b, ch, t0, G.we);
                    near_right = std::max(near_right, nb - G.we);
                    far_right = std::max(far_right, u - nb);
                    near_above = std::max(near_above, G.ws - split);
                    far_above = std::max(far_above, split - l);
                    const int64_t wc = G.we - G.ws + 1;
                    n_flops += 2 * wc * wc * (int64_t)((u - G.we) + (G.ws - l));
                }
                ++n_rounds;
                hipLaunchKernelGGL(k_win_chase, dim3(nch), dim3(kWinThreads), 0, s, H, ld, l, u, b, t0, g, Ur);
                LB_CHECK_LAUNCH();
                LB_HIP(hipStreamWaitEvent(s, c->ev_join, 0));
                if (near_right > 0) {
                    hipLaunchKernelGGL(k_win_rows, dim3(lb_blocks(near_right, kWinCols * kRowPasses), nch), dim3(kWinThreads), 0, s,
                                       H, ld, l, u, b, t0, (const double*)Ur, 0);
                    LB_CHECK_LAUNCH();
                }
                if (near_above > 0) {
                    hipLaunchKernelGGL(k_win_cols, dim3(lb_blocks(near_above, kWinCols * kColPasses), nch), dim3(kWinThreads), 0, s,
                                       H, ld, l, u, b, t0, (const double*)Ur, 0);
                    LB_CHECK_LAUNCH();
                }
                LB_HIP(hipEventRecord(c->ev_fork, s));
                LB_HIP(hipStreamWaitEvent(s2, c->ev_fork, 0));
                if (far_right > 0) {
                    hipLaunchKernelGGL(k_win_rows, dim3(lb_blocks(far_right, kWinCols * kRowPasses), nch), dim3(kWinThreads), 0, s2,
                                       H, ld, l, u, b, t0, (const double*)Ur, 1);
                    LB_CHECK_LAUNCH();
                }
                if (far_above > 0) {
                    hipLaunchKernelGGL(k_win_cols, dim3(lb_blocks(far_above, kWinCols * kColPasses), nch), dim3(kWinThreads), 0, s2,
                                       H, ld, l, u, b, t0, (const double*)Ur, 1);
                    LB_CHECK_LAUNCH();
                }
                LB_HIP(hipEventRecord(c->ev_join, s2));
            }
            LB_HIP(hipStreamWaitEvent(s, c->ev_join, 0));
        } else if (hg->u >= u) {
            return lb_fail(LB_ERR_DEVICE, "QR iteration: no progress at u=%d", u);
        }
        u = hg->u;
        if (u >= 0) lb_report(c, "qr", (double)(M - 1 - u) / M);
    }
    lb_report(c, "qr", 1.0);
    info->sweeps = n_sweeps + hg->sweeps;
    info->chain_steps = n_steps + hg->steps;
    info->updates = n_work + hg->work;
    info->rounds = n_rounds;
    info->product_flops = n_flops;
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
