// Steady state of dv/dt = Q v + K: the v with Q v = -K, i.e. the expansion
// (Eq. (7)) of the asymptotic state rho_inf, L(rho_inf) = 0, of Sec. 3 (the
// ODE of Eq. (10) at rest). FP64 throughout.
//
// Restarted GMRES with right preconditioning, x = P^-1 y: the Krylov basis is
// kept whole in HBM (restart lengths in the thousands fit in 288 GB), and each
// iteration orthogonalises by classical Gram-Schmidt applied twice in its
// delayed form, which streams the basis with full-line loads, twice per step,
// instead of the one-vector-at-a-time dependence of modified Gram-Schmidt:
//   k_dots2      one pass over the basis for V^T [u, t], u.u and u.t, partial sums per wave;
//   k_reduce     their sums in a fixed order (deterministic, no atomics);
//   k_dcgs2_fin  the lagged column of the Hessenberg matrix (by the Arnoldi relation),
//                rotated on the device by the earlier Givens rotations and a new one;
//   k_dcgs2_next the coefficients of the next projection;
//   k_dcgs2_upd  one pass over the basis that writes q_j and the next raw vector.
// The operator is the dense row-dot GEMV (one wavefront per row group, as the
// one-state RK4 stage) or the sliced sparse product; the optional
// preconditioner is the secular approximation of the Lindbladian in the energy
// eigenbasis (secular.hip). Residual estimates are read back every kLook steps;
// at the end of a cycle the rotated triangle is copied to the host for the back
// substitution and x += V y streams the basis once more (split over chunks of
// basis vectors for small systems, for enough blocks).
#include "lb_internal.h"
#include "rowdot.h"
#include "sell.h"

#include <math.h>

#include <algorithm>
#include <vector>

namespace {

constexpr int kDotJ = 32;           // basis vectors per block of k_dots (second grid dimension)
constexpr int64_t kSmallM = 262144;  // below: one row per thread (and split x updates), for enough blocks

// y = Q x, dense, R rows per wavefront.
template <int R, bool ALIGNED, bool NT>
__global__ __launch_bounds__(256) void k_mv_dense(const double* Q, int64_t M, int64_t ldq, const double* x,
                                                  double* y) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * R;
    if (row0 >= M) return;
    double acc[R];
    const double* qrow[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
        const int64_t row = row0 + t;
        qrow[t] = Q + (row < M ? row : M - 1) * ldq;
    }
    wave_rowdots<R, ALIGNED, NT>(qrow, x, M, lane, acc);
    if (lane < R) {
        double kv = 0.0;
#pragma unroll
        for (int t = 0; t < R; ++t)
            if (t == lane) kv = acc[t];
        if (row0 + lane < M) y[row0 + lane] = kv;
    }
}

// y = Q x, slice layout: one wavefront per slice, one block per long row.
__global__ __launch_bounds__(256) void k_mv_sell(SellMat a, const double* x, double* y) {
    const int wk = sell_work(a);
    if (wk < 0) return;
    if (wk < a.nlong) {
        const int64_t row = a.longrows[wk];
        double q0, q1;
        block_row_dots<false>(a, row, x, q0, q1);
        if (threadIdx.x == 0) y[row] = q0;
        return;
    }
    const int sl = __builtin_amdgcn_readfirstlane((wk - a.nlong) * 4 + (int)(threadIdx.x >> 6));
    if (sl >= a.S) return;
    const int lane = threadIdx.x & (kSlice - 1);
    const int64_t r = (int64_t)sl * kSlice + lane;
    const bool mine = r < a.M && !((a.lmask[sl] >> lane) & 1);
    const int64_t o0 = a.off0[sl];
    const int w0 = (int)((a.off0[sl + 1] - o0) / kSlice);
    double acc[1] = {0.0};
    sell_row<1>(a.scol0 + o0 + lane, a.sval0 + o0 + lane, w0, x, a.M, 1, acc);
    if (mine) y[r] = acc[0];
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Basis kernels work on row chunks of 256 E rows per block (E rows per thread,
// 256 apart); partial sums are per wavefront, p = 4 * block + wave.

// part[j * nparts + p] = sum over the rows of wave p of V_j[i] w[i], j < k;
// block (x, y) takes row chunk x and basis vectors [y kDotJ, (y + 1) kDotJ).
template <int E>
__global__ __launch_bounds__(256) void k_dots(const double* V, int64_t ldv, int k, int64_t M, const double* w,
                                              double* part, int nparts) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * 256 * E + threadIdx.x;
    double wv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t i = base + e * 256;
        wv[e] = i < M ? w[i] : 0.0;
    }
    const int p = blockIdx.x * 4 + wave;
    int j = blockIdx.y * kDotJ;
    const int jend = min(k, j + kDotJ);
    for (; j + 1 < jend; j += 2) {
        const double* v0 = V + (int64_t)j * ldv;
        const double* v1 = v0 + ldv;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t i = base + e * 256;
            if (i < M) {
                a0 = fma(v0[i], wv[e], a0);
                a1 = fma(v1[i], wv[e], a1);
            }
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        if (lane == 0) {
            part[(int64_t)j * nparts + p] = a0;
            part[(int64_t)(j + 1) * nparts + p] = a1;
        }
    }
    if (j < jend) {
        const double* v0 = V + (int64_t)j * ldv;
        double a0 = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t i = base + e * 256;
            if (i < M) a0 = fma(v0[i], wv[e], a0);
        }
        a0 = wave_sum(a0);
        if (lane == 0) part[(int64_t)j * nparts + p] = a0;
    }
}

// out[j] = sum_p part[j * nparts + p] (SQRT: its square root), one wave per j,
// lanes over p in a fixed order.
template <bool SQRT>
__global__ __launch_bounds__(256) void k_reduce(const double* part, int nparts, int k, double* out) {
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= k) return;
    const double* pj = part + (int64_t)j * nparts;
    double s = 0.0;
    for (int p = lane; p < nparts; p += 64) s += pj[p];
    s = wave_sum(s);
    if (lane == 0) out[j] = SQRT ? sqrt(s) : s;
}

// w[i] -= sgn * sum_{j<k} h[j] V_j[i]; with NORM, part[p] = the sum of the new
// w[i]^2 over the rows of wave p.
template <int E, bool NORM>
__global__ __launch_bounds__(256) void k_update(const double* V, int64_t ldv, int k, int64_t M, const double* h,
                                                double sgn, double* w, double* part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * 256 * E + threadIdx.x;
    double s[E];
#pragma unroll
    for (int e = 0; e < E; ++e) s[e] = 0.0;
    for (int j = 0; j < k; ++j) {
        const double hj = h[j];
        const double* vj = V + (int64_t)j * ldv;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t i = base + e * 256;
            if (i < M) s[e] = fma(hj, vj[i], s[e]);
        }
    }
    double nrm = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t i = base + e * 256;
        if (i < M) {
            const double x = w[i] - sgn * s[e];
            w[i] = x;
            nrm = fma(x, x, nrm);
        }
    }
    if (NORM) {
        nrm = wave_sum(nrm);
        if (lane == 0) part[blockIdx.x * 4 + wave] = nrm;
    }
}

// Split form of k_update for small M (one row per thread): part2[y * ldp + i] =
// sum over the basis vectors j of chunk y (of jc) of h[j] V_j[i] ...
__global__ __launch_bounds__(256) void k_update_part(const double* V, int64_t ldv, int k, int jc, int64_t M,
                                                     const double* h, double* part2, int64_t ldp) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M) return;
    const int j0 = blockIdx.y * jc, j1 = min(k, j0 + jc);
    double s0 = 0.0, s1 = 0.0;
    int j = j0;
    for (; j + 1 < j1; j += 2) {
        s0 = fma(h[j], V[(int64_t)j * ldv + i], s0);
        s1 = fma(h[j + 1], V[(int64_t)(j + 1) * ldv + i], s1);
    }
    if (j < j1) s0 = fma(h[j], V[(int64_t)j * ldv + i], s0);
    part2[blockIdx.y * ldp + i] = s0 + s1;
}

// ... and w[i] -= sgn * (the chunks' sums in chunk order); NORM as k_update.
template <bool NORM>
__global__ __launch_bounds__(256) void k_update_fin(int64_t M, const double* part2, int64_t ldp, int nch, double sgn,
                                                    double* w, double* part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double nrm = 0.0;
    if (i < M) {
        double t = 0.0;
        for (int c = 0; c < nch; ++c) t += part2[c * ldp + i];
        const double x = w[i] - sgn * t;
        w[i] = x;
        nrm = x * x;
    }
    if (NORM) {
        nrm = wave_sum(nrm);
        if (lane == 0) part[blockIdx.x * 4 + wave] = nrm;
    }
}

// out = a * x + b * y (elementwise); out may alias x or y.
__global__ void k_axpby(int64_t M, double a, const double* x, double b, const double* y, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

// out = x / d[0]
__global__ void k_divide(int64_t M, const double* x, const double* d, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < M) out[i] = x[i] / d[0];
}

// The operator y = Q x of either form.
struct Op {
    bool sparse;
    const double* Q;
    int64_t ldq;
    bool aligned, nt;
    SellMat m;
};

static int op_apply(const Op& op, int64_t M, const double* x, double* y, hipStream_t s) {
    if (op.sparse) {
        const unsigned grid = (unsigned)op.m.nlong8 + 8u * (unsigned)op.m.per_xcd;
        hipLaunchKernelGGL(k_mv_sell, dim3(grid), dim3(256), 0, s, op.m, x, y);
        LB_CHECK_LAUNCH();
        return LB_OK;
    }
    const int RW = M >= 8 * 8192 ? 8 : M >= 4 * 8192 ? 4 : M >= 2 * 8192 ? 2 : 1;
    const unsigned gx = lb_blocks((M + RW - 1) / RW, 4);
    typedef void (*mv_fn)(const double*, int64_t, int64_t, const double*, double*);
    mv_fn fn;
    if (!op.aligned) fn = RW == 8 ? k_mv_dense<8, false, false> : RW == 4 ? k_mv_dense<4, false, false>
                        : RW == 2 ? k_mv_dense<2, false, false> : k_mv_dense<1, false, false>;
    else if (op.nt) fn = RW == 8 ? k_mv_dense<8, true, true> : RW == 4 ? k_mv_dense<4, true, true>
                       : RW == 2 ? k_mv_dense<2, true, true> : k_mv_dense<1, true, true>;
    else fn = RW == 8 ? k_mv_dense<8, true, false> : RW == 4 ? k_mv_dense<4, true, false>
            : RW == 2 ? k_mv_dense<2, true, false> : k_mv_dense<1, true, false>;
    hipLaunchKernelGGL(fn, dim3(gx), dim3(256), 0, s, op.Q, M, op.ldq, x, y);
    LB_CHECK_LAUNCH();
    return LB_OK;
}

// Device buffers of one solve, freed on every exit.
struct SolveBufs {
    double* V = nullptr;  // (m + 1) basis vectors, stride ldv
    double* aux = nullptr;
    ~SolveBufs() {
        if (V) (void)hipFree(V);
        if (aux) (void)hipFree(aux);
    }
};

// Applies the rotations 0..j-1 to column Hj (rows 0..j+1), then the rotation
// that zeroes Hj[j+1], also applied to g; res = |g[j+1]|. One thread: the
// rotations are a recurrence through the carried entry, so the loads of eight
// steps are issued together.
__device__ void givens_column(int j, double* __restrict__ Hj, double* __restrict__ cs, double* __restrict__ sn,
                              double* __restrict__ g, double* res) {
    double carry = Hj[0];
    int i = 0;
    for (; i + 8 <= j; i += 8) {
        double b[8], c[8], s[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            b[u] = Hj[i + 1 + u];
            c[u] = cs[i + u];
            s[u] = sn[i + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            Hj[i + u] = c[u] * carry + s[u] * b[u];
            carry = -s[u] * carry + c[u] * b[u];
        }
    }
    for (; i < j; ++i) {
        const double b = Hj[i + 1];
        Hj[i] = cs[i] * carry + sn[i] * b;
        carry = -sn[i] * carry + cs[i] * b;
    }
    const double a = carry, b = Hj[j + 1];
    const double den = hypot(a, b);
    cs[j] = den > 0 ? a / den : 1.0;
    sn[j] = den > 0 ? b / den : 0.0;
    Hj[j] = den;
    Hj[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    *res = fabs(g[j + 1]);
}

// Delayed classical Gram-Schmidt with reorthogonalisation (large systems):
// entering step j the basis V_[0,j) is orthonormal and u is the next vector
// after one projection (not yet reorthogonalised or normalised). With
// t = A u, one pass over the basis gives s = V^T u, z = V^T t, alpha = u.u and
// beta = u.t; then omega = sqrt(alpha - s.s) finishes column j-1 of H (its
// second projection s and its norm), q_j = (u - V s) / omega, and by the
// Arnoldi relation A V = V H the first projection of A q_j and the next raw
// vector follow without another product:
//   h = ([z; d] - H s) / omega,  d = (beta - s.z) / omega,
//   u' = (t - V z - q_j d) / omega,
// formed in one more pass over the basis. Two passes per step instead of four.

// part rows: 2l -> V_l.u, 2l+1 -> V_l.t (l < k), 2k -> u.u, 2k+1 -> u.t.
template <int E>
__global__ __launch_bounds__(256) void k_dots2(const double* V, int64_t ldv, int k, int64_t M, const double* u,
                                               const double* t, double* part, int nparts) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * 256 * E + threadIdx.x;
    double uv[E], tv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t i = base + e * 256;
        uv[e] = i < M ? u[i] : 0.0;
        tv[e] = i < M ? t[i] : 0.0;
    }
    const int p = blockIdx.x * 4 + wave;
    const int j0 = blockIdx.y * kDotJ, j1 = min(k, j0 + kDotJ);
    int j = j0;
    // four basis vectors per round: 4 E loads issued before the products and reductions
    for (; j + 4 <= j1; j += 4) {
        double x[4][E];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t i = base + e * 256;
                x[q][e] = i < M ? V[(int64_t)(j + q) * ldv + i] : 0.0;
            }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double a = 0.0, b = 0.0;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                a = fma(x[q][e], uv[e], a);
                b = fma(x[q][e], tv[e], b);
            }
            a = wave_sum(a);
            b = wave_sum(b);
            if (lane == 0) {
                part[(int64_t)(2 * (j + q)) * nparts + p] = a;
                part[(int64_t)(2 * (j + q) + 1) * nparts + p] = b;
            }
        }
    }
    for (; j < j1; ++j) {
        const double* vj = V + (int64_t)j * ldv;
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t i = base + e * 256;
            if (i < M) {
                const double x = vj[i];
                a = fma(x, uv[e], a);
                b = fma(x, tv[e], b);
            }
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) {
            part[(int64_t)(2 * j) * nparts + p] = a;
            part[(int64_t)(2 * j + 1) * nparts + p] = b;
        }
    }
    if (blockIdx.y == 0) {
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            a = fma(uv[e], uv[e], a);
            b = fma(uv[e], tv[e], b);
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) {
            part[(int64_t)(2 * k) * nparts + p] = a;
            part[(int64_t)(2 * k + 1) * nparts + p] = b;
        }
    }
}

// Column bookkeeping of step j >= 1, part 1 (one block): finishes column j-1
// of the unrotated Hessenberg matrix (kept row-major, Hr[l * ldr + i]), rotates
// it into H (column-major; the earlier Givens rotations applied in order, then the
// one that zeroes the subdiagonal entry, applied to g as well) and sets scal = (omega, d).
__global__ __launch_bounds__(256) void k_dcgs2_fin(int j, const double* sz, double* Hr, int64_t ldr, double* H,
                                                   int64_t ldh, double* cs, double* sn, double* g, double* res,
                                                   double* brk, double* scal) {
    __shared__ double red[2][4];
    __shared__ double sh[2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double ss = 0.0, sz2 = 0.0;
    for (int l = threadIdx.x; l < j; l += blockDim.x) {
        const double sl = sz[2 * l], zl = sz[2 * l + 1];
        ss = fma(sl, sl, ss);
        sz2 = fma(sl, zl, sz2);
    }
    ss = wave_sum(ss);
    sz2 = wave_sum(sz2);
    if (lane == 0) {
        red[0][wave] = ss;
        red[1][wave] = sz2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double a = sz[2 * j], b = sz[2 * j + 1];
        const double s2 = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        const double szt = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        const double om = sqrt(fmax(a - s2, 0.0));
        sh[0] = om;
        sh[1] = (b - szt) / om;
    }
    __syncthreads();
    const double om = sh[0];
    // column j-1: rows 0..j-1 gain the second projection s, row j is omega; copied into H
    double* Hj = H + (int64_t)(j - 1) * ldh;
    for (int l = threadIdx.x; l <= j; l += blockDim.x) {
        double* e = Hr + (int64_t)l * ldr + (j - 1);
        const double x = l < j ? *e + sz[2 * l] : om;
        *e = x;
        Hj[l] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int jj = j - 1;
        givens_column(jj, Hj, cs, sn, g, res + jj);
        brk[jj] = om;
        scal[0] = om;
        scal[1] = sh[1];
    }
}

// Part 2 (one wavefront per row l <= j): the first projection of column j,
// Hr[l][j] = ((l < j ? z_l : d) - (Hr s)_l) / omega, with (Hr s)_l summed over
// the band i >= l - 1 in a fixed order.
__global__ __launch_bounds__(256) void k_dcgs2_next(int j, const double* sz, double* Hr, int64_t ldr,
                                                    const double* scal) {
    const int lane = threadIdx.x & 63;
    const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (l > j) return;
    const double* row = Hr + (int64_t)l * ldr;
    double c = 0.0;
    for (int i = (l > 0 ? l - 1 : 0) + lane; i < j; i += 64) c = fma(row[i], sz[2 * i], c);
    c = wave_sum(c);
    if (lane == 0) Hr[(int64_t)l * ldr + j] = ((l < j ? sz[2 * l + 1] : scal[1]) - c) / scal[0];
}

// q_j = (u - V s) / omega into V_j, u <- (t - V z - q_j d) / omega.
template <int E>
__global__ __launch_bounds__(256) void k_dcgs2_upd(double* V, int64_t ldv, int j, int64_t M, const double* sz,
                                                   const double* scal, double* u, const double* t) {
    const int64_t base = (int64_t)blockIdx.x * 256 * E + threadIdx.x;
    double a[E], b[E];
#pragma unroll
    for (int e = 0; e < E; ++e) a[e] = b[e] = 0.0;
    // four basis vectors per round: their coefficients and 4 E loads issued before the products
    int l = 0;
    for (; l + 4 <= j; l += 4) {
        double sc[4], zc[4], x[4][E];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            sc[u] = sz[2 * (l + u)];
            zc[u] = sz[2 * (l + u) + 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int64_t i = base + e * 256;
                x[u][e] = i < M ? V[(int64_t)(l + u) * ldv + i] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                a[e] = fma(sc[u], x[u][e], a[e]);
                b[e] = fma(zc[u], x[u][e], b[e]);
            }
    }
    for (; l < j; ++l) {
        const double sl = sz[2 * l], zl = sz[2 * l + 1];
        const double* vl = V + (int64_t)l * ldv;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t i = base + e * 256;
            if (i < M) {
                const double x = vl[i];
                a[e] = fma(sl, x, a[e]);
                b[e] = fma(zl, x, b[e]);
            }
        }
    }
    const double om = scal[0], d = scal[1];
    double* vj = V + (int64_t)j * ldv;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int64_t i = base + e * 256;
        if (i < M) {
            const double q = (u[i] - a[e]) / om;
            vj[i] = q;
            u[i] = (t[i] - b[e] - q * d) / om;
        }
    }
}

__global__ void k_copy_first(const double* src, double* dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}

// g = (beta, 0, ..., 0) with beta = |r| on the device.
__global__ void k_init_g(int64_t n, const double* beta, double* g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g[i] = i == 0 ? beta[0] : 0.0;
}

constexpr int kLook = 8;  // iterations enqueued between convergence checks

static int gmres(lb_ctx* c, int64_t M, const Op& op, const lb_secular* pre, const double* K, double* v, double tol,
                 int64_t maxit, int64_t restart, lb_solve_info* info) {
    hipStream_t s = c->stream;
    const int64_t m = restart < maxit ? restart : maxit;
    const int64_t ldv = (M + 31) / 32 * 32;
    const int64_t ldh = m + 2;  // rows of H (column j has rows 0..j+1)
    const int64_t ldr = m + 1;  // row length of the row-major unrotated Hr (m + 2 rows)
    // small systems: one row per thread and updates split over chunks of the basis
    const bool small = M < kSmallM;
    const int E = small ? 1 : 4;
    const int nrb = (int)lb_blocks(M, 256 * E);
    const int nparts = 4 * nrb;
    SolveBufs b;
    if (hipMalloc(&b.V, sizeof(double) * (size_t)(m + 1) * ldv) != hipSuccess) {
        (void)hipGetLastError();
        b.V = nullptr;
        return lb_fail(LB_ERR_OOM, "Krylov basis of %lld vectors of %lld doubles does not fit", (long long)(m + 1),
                       (long long)M);
    }
    // split updates: at most 64 chunks of at least 16 basis vectors
    const int nch_max = small ? (int)std::min<int64_t>(64, (m + 15) / 16) : 1;
    // aux: w, x, r, z, u (ldv each) | part | hb (2 (m + 1) + 1) | nrm (1) | y (m)
    //      | H (ldh m) | cs, sn (m each) | g (m + 1) | res, brk (m each) | part2 (nch_max ldv)
    //      | delayed Gram-Schmidt: Hr (ldh (m + 1)), sz (2 (m + 1) + 2), scal (2), t (ldv); part holds
    //        (2 (m + 1) + 2) nparts
    const size_t n_part = (size_t)(2 * (m + 1) + 2) * nparts;
    const size_t n_aux = 5 * (size_t)ldv + n_part + 2 * (size_t)(m + 1) + 2 + (size_t)m + (size_t)ldh * m +
                         2 * (size_t)m + (size_t)(m + 1) + 2 * (size_t)m + (nch_max > 1 ? (size_t)nch_max * ldv : 0) +
                         (size_t)ldh * (m + 1) + 2 * (size_t)(m + 1) + 4 + (size_t)ldv;
    if (hipMalloc(&b.aux, sizeof(double) * n_aux) != hipSuccess) {
        (void)hipGetLastError();
        b.aux = nullptr;
        return lb_fail(LB_ERR_OOM, "GMRES work space of %zu doubles does not fit", n_aux);
    }
    double* w = b.aux;
    double* x = w + ldv;
    double* r = x + ldv;
    double* zb = r + ldv;
    double* ub = zb + ldv;
    double* part = ub + ldv;
    double* hb = part + n_part;  // the first step's projection coefficient
    double* nrm = hb + 2 * (m + 1) + 1;
    double* yd = nrm + 1;
    double* Hd = yd + m;
    double* csd = Hd + (size_t)ldh * m;
    double* snd = csd + m;
    double* gd = snd + m;
    double* resd = gd + (m + 1);
    double* brkd = resd + m;
    double* part2 = brkd + m;
    double* Hr = part2 + (nch_max > 1 ? (size_t)nch_max * ldv : 0);
    double* szd = Hr + (size_t)ldh * (m + 1);
    double* scal = szd + 2 * (m + 1) + 2;
    double* tb = scal + 2;
    // pinned host: the estimates of a batch (R and g of a cycle reserve more later)
    int rc = lb_host_reserve(c, sizeof(double) * 2 * kLook);
    if (rc) return rc;
    double* hh = (double*)c->host;
    const unsigned eg = lb_blocks(M, 256);
    auto norm_of = [&](double* vec, double* out) -> int {
        // ||vec|| into out[0] on the device
        if (small) hipLaunchKernelGGL(k_dots<1>, dim3(nrb, 1), dim3(256), 0, s, vec, ldv, 1, M, vec, part, nparts);
        else hipLaunchKernelGGL(k_dots<4>, dim3(nrb, 1), dim3(256), 0, s, vec, ldv, 1, M, vec, part, nparts);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_reduce<true>, dim3(1), dim3(256), 0, s, part, nparts, 1, out);
        LB_CHECK_LAUNCH();
        return LB_OK;
    };
    auto fetch = [&](const double* dev, double* host, size_t n) -> int {
        LB_HIP(hipMemcpyAsync(host, dev, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        LB_HIP(hipStreamSynchronize(s));
        return LB_OK;
    };
    // out -= sgn V_[0,k) h, with the new |out|^2 partials in part when norm
    auto update = [&](int k, const double* h, double sgn, double* out, bool norm) -> int {
        if (!small) {
            if (norm)
                hipLaunchKernelGGL((k_update<4, true>), dim3(nrb), dim3(256), 0, s, (const double*)b.V, ldv, k, M, h,
                                   sgn, out, part);
            else
                hipLaunchKernelGGL((k_update<4, false>), dim3(nrb), dim3(256), 0, s, (const double*)b.V, ldv, k, M, h,
                                   sgn, out, part);
            LB_CHECK_LAUNCH();
            return LB_OK;
        }
        const int jc = std::max(16, (k + nch_max - 1) / nch_max);
        const int used = (k + jc - 1) / jc;
        hipLaunchKernelGGL(k_update_part, dim3(nrb, used), dim3(256), 0, s, (const double*)b.V, ldv, k, jc, M, h,
                           part2, ldv);
        LB_CHECK_LAUNCH();
        if (norm)
            hipLaunchKernelGGL(k_update_fin<true>, dim3(nrb), dim3(256), 0, s, M, (const double*)part2, ldv, used, sgn,
                               out, part);
        else
            hipLaunchKernelGGL(k_update_fin<false>, dim3(nrb), dim3(256), 0, s, M, (const double*)part2, ldv, used,
                               sgn, out, part);
        LB_CHECK_LAUNCH();
        return LB_OK;
    };
    auto dots = [&](int k, const double* vec) -> int {
        const dim3 grid(nrb, (unsigned)((k + kDotJ - 1) / kDotJ));
        if (small) hipLaunchKernelGGL(k_dots<1>, grid, dim3(256), 0, s, (const double*)b.V, ldv, k, M, vec, part, nparts);
        else hipLaunchKernelGGL(k_dots<4>, grid, dim3(256), 0, s, (const double*)b.V, ldv, k, M, vec, part, nparts);
        LB_CHECK_LAUNCH();
        return LB_OK;
    };
    auto apply_op = [&](const double* in, double* out) -> int {
        int e;
        if (pre) {
            if ((e = lb_impl_secular_apply(c, pre, in, zb)) || (e = op_apply(op, M, zb, out, s))) return e;
            return LB_OK;
        }
        return op_apply(op, M, in, out, s);
    };
    // delayed Gram-Schmidt step jj: finishes column jj of H (rotated, res[jj]) and writes V_{jj+1}
    auto arnoldi_delayed = [&](int64_t jj) -> int {
        int e;
        if (jj == 0) {  // u = A v_0 projected once; its coefficient is the first entry of column 0
            if ((e = apply_op(b.V, ub))) return e;
            if ((e = dots(1, ub))) return e;
            hipLaunchKernelGGL(k_reduce<false>, dim3(1), dim3(256), 0, s, (const double*)part, nparts, 1, hb);
            LB_CHECK_LAUNCH();
            if ((e = update(1, hb, 1.0, ub, false))) return e;
            hipLaunchKernelGGL(k_copy_first, dim3(1), dim3(64), 0, s, (const double*)hb, Hr);  // Hr[0][0]
            LB_CHECK_LAUNCH();
        }
        const int j = (int)(jj + 1);
        if ((e = apply_op(ub, tb))) return e;
        const dim3 grid(nrb, (unsigned)((j + kDotJ - 1) / kDotJ));
        if (small)
            hipLaunchKernelGGL(k_dots2<1>, grid, dim3(256), 0, s, (const double*)b.V, ldv, j, M, (const double*)ub,
                               (const double*)tb, part, nparts);
        else
            hipLaunchKernelGGL(k_dots2<4>, grid, dim3(256), 0, s, (const double*)b.V, ldv, j, M, (const double*)ub,
                               (const double*)tb, part, nparts);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_reduce<false>, dim3(lb_blocks(2 * j + 2, 4)), dim3(256), 0, s, (const double*)part,
                           nparts, 2 * j + 2, szd);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_dcgs2_fin, dim3(1), dim3(256), 0, s, j, (const double*)szd, Hr, ldr, Hd, ldh, csd, snd,
                           gd, resd, brkd, scal);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_dcgs2_next, dim3(lb_blocks(j + 1, 4)), dim3(256), 0, s, j, (const double*)szd, Hr, ldr,
                           (const double*)scal);
        LB_CHECK_LAUNCH();
        if (small)
            hipLaunchKernelGGL(k_dcgs2_upd<1>, dim3(nrb), dim3(256), 0, s, b.V, ldv, j, M, (const double*)szd,
                               (const double*)scal, ub, (const double*)tb);
        else
            hipLaunchKernelGGL(k_dcgs2_upd<4>, dim3(nrb), dim3(256), 0, s, b.V, ldv, j, M, (const double*)szd,
                               (const double*)scal, ub, (const double*)tb);
        LB_CHECK_LAUNCH();
        return LB_OK;
    };
    // ||K||: the scale of the residual
    double knorm = 0.0;
    LB_HIP(hipMemcpyAsync(r, K, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
    if ((rc = norm_of(r, nrm)) || (rc = fetch(nrm, &knorm, 1))) return rc;
    LB_HIP(hipMemsetAsync(x, 0, sizeof(double) * M, s));
    info->iterations = 0;
    info->restarts = 0;
    info->residual = 0.0;
    info->converged = 0;
    if (knorm == 0.0) {  // K = 0: v = 0 is the solution
        LB_HIP(hipMemcpyAsync(v, x, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
        LB_HIP(hipStreamSynchronize(s));
        info->converged = 1;
        return LB_OK;
    }
    std::vector<double> y(m);
    int64_t total = 0;
    int64_t cycles = 0;
    for (;;) {
        // r = -K - Q x
        if ((rc = op_apply(op, M, x, w, s))) return rc;
        hipLaunchKernelGGL(k_axpby, dim3(eg), dim3(256), 0, s, M, -1.0, K, -1.0, (const double*)w, r);
        LB_CHECK_LAUNCH();
        double beta = 0.0;
        if ((rc = norm_of(r, nrm)) || (rc = fetch(nrm, &beta, 1))) return rc;
        info->residual = beta / knorm;
        if (beta <= tol * knorm) {
            info->converged = 1;
            break;
        }
        if (total >= maxit) break;
        ++cycles;
        hipLaunchKernelGGL(k_divide, dim3(eg), dim3(256), 0, s, M, (const double*)r, (const double*)nrm, b.V);
        hipLaunchKernelGGL(k_init_g, dim3(lb_blocks(m + 1, 256)), dim3(256), 0, s, m + 1, (const double*)nrm, gd);
        LB_CHECK_LAUNCH();
        // Arnoldi steps in batches of kLook between reads of the residual estimates
        const int64_t lim = std::min<int64_t>(m, maxit - total);
        int64_t j = 0, used = 0;
        while (j < lim && used == 0) {
            const int64_t nb = std::min<int64_t>(kLook, lim - j);
            for (int64_t t = 0; t < nb; ++t)
                if ((rc = arnoldi_delayed(j + t))) return rc;
            LB_HIP(hipMemcpyAsync(hh, resd + j, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
            LB_HIP(hipMemcpyAsync(hh + kLook, brkd + j, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
            LB_HIP(hipStreamSynchronize(s));
            for (int64_t t = 0; t < nb && used == 0; ++t)
                if (hh[t] <= tol * knorm || hh[kLook + t] == 0.0) used = j + t + 1;
            j += nb;
        }
        const int64_t k = used ? used : j;  // columns of the least-squares problem
        total += k;
        // y = R^-1 g (R: the leading k x k block of the rotated H), then x += P^-1 V y
        if ((rc = lb_host_reserve(c, sizeof(double) * ((size_t)k * k + k + 2 * kLook)))) return rc;
        hh = (double*)c->host;
        double* Rh = hh;
        double* gh = hh + (size_t)k * k;
        LB_HIP(hipMemcpy2DAsync(Rh, sizeof(double) * k, Hd, sizeof(double) * ldh, sizeof(double) * k, k,
                                hipMemcpyDeviceToHost, s));
        LB_HIP(hipMemcpyAsync(gh, gd, sizeof(double) * k, hipMemcpyDeviceToHost, s));
        LB_HIP(hipStreamSynchronize(s));
        for (int64_t i = k - 1; i >= 0; --i) {
            double t = gh[i];
            for (int64_t l = i + 1; l < k; ++l) t -= Rh[(size_t)l * k + i] * y[l];
            const double d = Rh[(size_t)i * k + i];
            y[i] = d != 0.0 ? t / d : 0.0;
        }
        LB_HIP(hipMemcpyAsync(yd, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
        if (pre) {
            LB_HIP(hipMemsetAsync(ub, 0, sizeof(double) * M, s));
            if ((rc = update((int)k, yd, -1.0, ub, false))) return rc;
            if ((rc = lb_impl_secular_apply(c, pre, ub, zb))) return rc;
            hipLaunchKernelGGL(k_axpby, dim3(eg), dim3(256), 0, s, M, 1.0, (const double*)x, 1.0, (const double*)zb,
                               x);
            LB_CHECK_LAUNCH();
        } else if ((rc = update((int)k, yd, -1.0, x, false))) {
            return rc;
        }
    }
    LB_HIP(hipMemcpyAsync(v, x, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
    LB_HIP(hipStreamSynchronize(s));
    info->iterations = total;
    info->restarts = cycles > 0 ? cycles - 1 : 0;
    if (!info->converged)
        return lb_fail(LB_ERR_NO_CONVERGENCE, "GMRES stopped after %lld iterations at relative residual %.3e",
                       (long long)total, info->residual);
    return LB_OK;
}

}  // namespace

int lb_impl_steady_dense(lb_ctx* c, int64_t M, const double* Q, int64_t ldq, const double* K, const lb_secular* pre,
                         double* v, double tol, int64_t maxit, int64_t restart, lb_solve_info* info) {
    Op op;
    op.sparse = false;
    op.Q = Q;
    op.ldq = ldq;
    op.aligned = ((uintptr_t)Q % 16 == 0) && ldq % 2 == 0;
    op.nt = op.aligned && ((uintptr_t)Q % 128 == 0) && ldq % 16 == 0;
    return gmres(c, M, op, pre, K, v, tol, maxit, restart, info);
}

int lb_impl_steady_csr(lb_ctx* c, int64_t M, const int64_t* rowptr, const int64_t* col, const double* val,
                       const double* K, const lb_secular* pre, double* v, double tol, int64_t maxit, int64_t restart,
                       lb_solve_info* info) {
    Op op;
    op.sparse = true;
    size_t extra = 0;
    int rc = sell_build(c, M, rowptr, col, val, nullptr, nullptr, nullptr, 0, &op.m, &extra);
    if (rc) return rc;
    return gmres(c, M, op, pre, K, v, tol, maxit, restart, info);
}
