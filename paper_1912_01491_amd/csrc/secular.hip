// Preconditioner for the steady state Q v = -K of a Lindbladian given by a
// Hamiltonian H and jump operators L_p with rates g_p: the secular (rotating-
// wave) approximation of L in the energy eigenbasis H = U diag(E) U^H, which
// it inverts exactly.
//
// In that basis (tildes), L(X) = A X + X A^H + sum_p g_p L_p X L_p^H with
// A = -iH - 1/2 sum_p g_p L_p^H L_p. Keeping of A only its diagonal and of the
// jump term only what maps a matrix unit to itself, a coherence X_ab (a != b)
// is multiplied by
//   den_ab = -i (E_a - E_b) - (gt_a + gt_b) / 2 + sum_p g_p Lt_p,aa conj(Lt_p,bb),
//   gt_a = sum_b W_ba,  W_ab = sum_p g_p |Lt_p,ab|^2,
// and the populations follow the rate equations dP/dt = (W - diag(gt)) P. On
// traceless inputs the populations are solved together with sum_a P_a = 0
// through the bordered matrix [[W - diag(gt), 1], [1^T, 0]], inverted once.
// Applied to a coherence-vector residual r: R = sum_n r_n F_n (Eq. (7) without
// the identity), Rt = U^H R U, Yt = the solution above, Y = U Yt U^H,
// z_n = Tr(F_n Y) (Eq. (6)). The dimer's strongly oscillating coherences are
// then inverted exactly, so GMRES iterates only on the coupling that the
// approximation drops.
//
// Matrices are complex (interleaved re, im), column-major. The four N x N
// basis changes per application are plain complex GEMMs (vendor BLAS); the
// rest are the kernels below.
#include "lb_internal.h"

#include <math.h>

#include <vector>

struct lb_secular {
    int N = 0;
    int64_t M = 0;
    int device = 0;
    double2* U = nullptr;    // eigenvectors of H, N x N
    double2* den = nullptr;  // coherence denominators, N x N
    double* Binv = nullptr;  // inverse bordered rate matrix, (N + 1) x (N + 1), row-major
    double2* T1 = nullptr;   // scratch, N x N each
    double2* T2 = nullptr;
    double* pv = nullptr;    // 2 (N + 1) + N: right-hand side, populations, diagonal scan
    double2* part = nullptr;  // partial products of the split-k basis changes
    int64_t part_elems = 0;
};

namespace {

__global__ void k_csr_dense_cm(int N, const int64_t* rowptr, const int64_t* col, const double2* val, double2* D) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {  // duplicate entries add up, as in the CSR's sum
        double2& d = D[r + col[e] * N];
        d = make_double2(d.x + val[e].x, d.y + val[e].y);
    }
}

// W += g |Lt|^2 elementwise; d = diag(Lt).
__global__ void k_jump_accum(int N, double g, const double2* Lt, double* W, double2* d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * N) return;
    const double2 x = Lt[i];
    W[i] += g * (x.x * x.x + x.y * x.y);
    const int a = (int)(i % N), b = (int)(i / N);
    if (a == b) d[a] = x;
}

// gt[a] = sum_b W_ba (column a of W, column-major).
__global__ __launch_bounds__(256) void k_col_sums(int N, const double* W, double* gt) {
    __shared__ double red[4];
    const int a = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < N; b += blockDim.x) s += W[b + (int64_t)a * N];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) gt[a] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_den(int N, const double* E, const double* gt, int P, const double* g, const double2* d,
                      double2* den) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * N) return;
    const int a = (int)(i % N), b = (int)(i / N);
    double re = -0.5 * (gt[a] + gt[b]), im = -(E[a] - E[b]);
    for (int p = 0; p < P; ++p) {
        const double2 x = d[(int64_t)p * N + a], y = d[(int64_t)p * N + b];
        re += g[p] * (x.x * y.x + x.y * y.y);  // x conj(y)
        im += g[p] * (x.y * y.x - x.x * y.y);
    }
    den[i] = make_double2(re, im);
}

// aug (n x 2n, row-major) = [[W - diag(gt), 1], [1^T, 0] | I].
__global__ void k_border(int N, const double* W, const double* gt, double* aug) {
    const int n = N + 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * 2 * n) return;
    const int r = (int)(i / (2 * n)), c = (int)(i % (2 * n));
    double v;
    if (c >= n) v = (c - n == r) ? 1.0 : 0.0;
    else if (r < N && c < N) v = W[r + (int64_t)c * N] - (r == c ? gt[r] : 0.0);
    else if (r == N && c == N) v = 0.0;
    else v = 1.0;
    aug[i] = v;
}

// Gauss-Jordan step k, part 1: the pivot row (largest |aug[r][k]|, r >= k) and
// its value.
__global__ __launch_bounds__(1024) void k_gj_pivot(int n, const double* aug, int k, int* piv, double* pval) {
    __shared__ double bv[1024];
    __shared__ int bi[1024];
    double best = -1.0;
    int bidx = k;
    for (int r = k + threadIdx.x; r < n; r += blockDim.x) {
        const double a = fabs(aug[(int64_t)r * 2 * n + k]);
        if (a > best) {
            best = a;
            bidx = r;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double ov = bv[threadIdx.x + o];
            const int oi = bi[threadIdx.x + o];
            if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = ov;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        piv[0] = bi[0];
        pval[0] = aug[(int64_t)bi[0] * 2 * n + k];
    }
}

// Part 2: swap rows k and piv, scale row k by 1/pivot; the thread of column k
// then keeps column k (after the swap) as the elimination factors f.
__global__ void k_gj_swap(int n, double* aug, int k, const int* piv, const double* pval, double* f) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= 2 * n) return;
    const int p = piv[0];
    const double inv = 1.0 / pval[0];
    const double a = aug[(int64_t)k * 2 * n + c], b = aug[(int64_t)p * 2 * n + c];
    aug[(int64_t)p * 2 * n + c] = a;
    aug[(int64_t)k * 2 * n + c] = b * inv;
    if (c == k)
        for (int r = 0; r < n; ++r) f[r] = aug[(int64_t)r * 2 * n + k];
}

// Part 3: eliminate column k from every other row.
__global__ void k_gj_elim(int n, double* aug, int k, const double* f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * 2 * n) return;
    const int r = (int)(i / (2 * n)), c = (int)(i % (2 * n));
    if (r == k) return;
    aug[i] -= f[r] * aug[(int64_t)k * 2 * n + c];
}

__global__ void k_take_inverse(int n, const double* aug, double* Binv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * n) return;
    const int r = (int)(i / n), c = (int)(i % n);
    Binv[i] = aug[(int64_t)r * 2 * n + n + c];
}

// Inclusive scans over the diagonal part, one block of 1024 threads (N <= 2048,
// two entries per thread, a Hillis-Steele scan of the pair sums in LDS).
// SUFFIX = false: out[x] = sum_{y <= x} Re Y_yy (prefix sums of the diagonal).
// SUFFIX = true:  out[x] = sum_{l >= x} v_D(l) / sqrt(l (l + 1)) for l = 1..N-1,
// the weight that D^l puts on every position below l.
template <bool SUFFIX>
__global__ __launch_bounds__(1024) void k_diag_scan(int N, const double2* Y, const double* v, double* out) {
    __shared__ double sh[1024];
    const int64_t P = lb_npairs(N);
    const int t = threadIdx.x;
    auto item = [&](int x) -> double {
        if (x >= N) return 0.0;
        if (!SUFFIX) return Y[x + (int64_t)x * N].x;
        const int l = N - 1 - x;  // reversed order: suffix sums as prefix sums
        return l >= 1 ? v[2 * P + l - 1] / sqrt((double)l * (l + 1)) : 0.0;
    };
    const double a = item(2 * t), b = item(2 * t + 1);
    sh[t] = a + b;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const double add = t >= o ? sh[t - o] : 0.0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const double before = t > 0 ? sh[t - 1] : 0.0;
    auto put = [&](int x, double val) {
        if (x >= N) return;
        if (!SUFFIX) out[x] = val;
        else out[N - 1 - x] = val;
    };
    put(2 * t, before + a);
    put(2 * t + 1, before + a + b);
}

// R = sum_n r_n F_n (traceless Hermitian, column-major). Threads below P write
// pair q's two entries, threads from P on write a diagonal element.
__global__ void k_v_to_herm(int N, const double* v, const double* wsuf, double2* R) {
    const int64_t P = lb_npairs(N);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double s2 = 0.70710678118654752440;
    if (t < P) {
        int cls, j, k;
        lb_decode(N, t, cls, j, k);
        const double s = v[t] * s2, a = v[P + t] * s2;
        R[j + (int64_t)k * N] = make_double2(s, -a);  // (S - i J)/sqrt(2) at (j, k)
        R[k + (int64_t)j * N] = make_double2(s, a);
        return;
    }
    const int64_t x = t - P;
    if (x >= N) return;
    // D^l has 1 at positions < l and -l at position l (scaled by 1/sqrt(l(l+1)));
    // wsuf[x + 1] = sum over l > x of the scaled coefficients
    double d = x + 1 < N ? wsuf[x + 1] : 0.0;
    if (x >= 1) d -= (double)x * v[2 * P + x - 1] / sqrt((double)x * (x + 1));
    R[x + x * N] = make_double2(d, 0.0);
}

// z_n = Re Tr(F_n Y).
__global__ void k_herm_to_v(int N, const double2* Y, const double* dpre, double* z) {
    const int64_t P = lb_npairs(N);
    const int64_t M = (int64_t)N * N - 1;
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= M) return;
    const double s2 = 0.70710678118654752440;
    int cls, j, k;
    lb_decode(N, n, cls, j, k);
    if (cls == 0) {
        z[n] = (Y[k + (int64_t)j * N].x + Y[j + (int64_t)k * N].x) * s2;
    } else if (cls == 1) {
        z[n] = (Y[k + (int64_t)j * N].y - Y[j + (int64_t)k * N].y) * s2;
    } else {
        const int l = j;  // dpre[l - 1] = sum over x < l of Re Y_xx
        z[n] = (dpre[l - 1] - (double)l * Y[l + (int64_t)l * N].x) / sqrt((double)l * (l + 1));
    }
}

__global__ void k_diag_rhs(int N, const double2* Rt, double* rhs) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < N) rhs[a] = Rt[a + (int64_t)a * N].x;
    if (a == N) rhs[N] = 0.0;
}

// y = Binv x, (n x n row-major), one wavefront per row.
__global__ __launch_bounds__(256) void k_small_gemv(int n, const double* B, const double* x, double* y) {
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    const double* row = B + (int64_t)r * n;
    double s = 0.0;
    for (int c = lane; c < n; c += 64) s = fma(row[c], x[c], s);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) y[r] = s;
}

// Yt = Rt / den off the diagonal, the populations on it.
__global__ void k_apply_den(int N, double2* T, const double2* den, const double* pop) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)N * N) return;
    const int a = (int)(i % N), b = (int)(i / N);
    if (a == b) {
        T[i] = make_double2(pop[a], 0.0);
        return;
    }
    const double2 x = T[i], d = den[i];
    const double q = d.x * d.x + d.y * d.y;
    T[i] = make_double2((x.x * d.x + x.y * d.y) / q, (x.y * d.x - x.x * d.y) / q);
}

// C = op(A) op(B), N x N complex, column-major; op = conjugate transpose when ca / cb.
int zgemm(hipStream_t s, const lb_secular* pre, bool ca, bool cb, int N, const double2* A, const double2* B,
          double2* C) {
    return lb_impl_gemm_c128(s, ca, cb, N, N, N, (const double*)A, N, (const double*)B, N, (double*)C, N,
                             (double*)pre->part, pre->part_elems);
}

void secular_free(lb_secular* p) {
    if (!p) return;
    for (void* q : {(void*)p->U, (void*)p->den, (void*)p->Binv, (void*)p->T1, (void*)p->T2, (void*)p->pv,
                    (void*)p->part})
        if (q) (void)hipFree(q);
    delete p;
}

}  // namespace

int lb_impl_secular_create(lb_ctx* c, int N, const lb_csr_c128* H, int P, const double* rates,
                           const lb_csr_c128* L, lb_secular** out) {
    hipStream_t s = c->stream;
    const int64_t NN = (int64_t)N * N;
    const int n = N + 1;
    lb_secular* pre = new lb_secular();
    pre->N = N;
    pre->M = NN - 1;
    pre->device = c->device;
    auto dmalloc = [&](void** p, size_t bytes) -> int {
        if (hipMalloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return lb_fail(LB_ERR_OOM, "preconditioner allocation of %zu bytes failed", bytes);
        }
        return LB_OK;
    };
    // set-up temporaries: dense H / L, eigenvalues, W, gt, diagonals, rates, aug, f, pivot
    double2* Hd = nullptr;
    double *E = nullptr, *W = nullptr, *gt = nullptr, *gdev = nullptr, *aug = nullptr, *f = nullptr, *pval = nullptr;
    double2* dg = nullptr;
    int* piv = nullptr;
    std::vector<void*> tmp;
    auto cleanup = [&](int rc) {
        (void)hipStreamSynchronize(s);
        for (void* q : tmp)
            if (q) (void)hipFree(q);
        if (rc) secular_free(pre);
        return rc;
    };
    int rc = LB_OK;
    if ((rc = dmalloc((void**)&pre->U, sizeof(double2) * NN)) || (rc = dmalloc((void**)&pre->den, sizeof(double2) * NN)) ||
        (rc = dmalloc((void**)&pre->Binv, sizeof(double) * (size_t)n * n)) ||
        (rc = dmalloc((void**)&pre->T1, sizeof(double2) * NN)) || (rc = dmalloc((void**)&pre->T2, sizeof(double2) * NN)) ||
        (rc = dmalloc((void**)&pre->pv, sizeof(double) * (2 * (size_t)n + N))))
        return cleanup(rc);
    {
        const int S = lb_gemm_c128_splits(N, N, N);
        if (S > 1) {
            pre->part_elems = (int64_t)S * NN;
            if ((rc = dmalloc((void**)&pre->part, sizeof(double2) * (size_t)pre->part_elems))) return cleanup(rc);
        }
    }
    const int Pm = P > 0 ? P : 1;
    if ((rc = dmalloc((void**)&Hd, sizeof(double2) * NN)) || (rc = dmalloc((void**)&E, sizeof(double) * N)) ||
        (rc = dmalloc((void**)&W, sizeof(double) * NN)) || (rc = dmalloc((void**)&gt, sizeof(double) * N)) ||
        (rc = dmalloc((void**)&gdev, sizeof(double) * Pm)) || (rc = dmalloc((void**)&dg, sizeof(double2) * Pm * N)) ||
        (rc = dmalloc((void**)&aug, sizeof(double) * (size_t)n * 2 * n)) || (rc = dmalloc((void**)&f, sizeof(double) * n)) ||
        (rc = dmalloc((void**)&pval, sizeof(double))) || (rc = dmalloc((void**)&piv, sizeof(int)))) {
        tmp = {Hd, E, W, gt, gdev, dg, aug, f, pval, piv};
        return cleanup(rc);
    }
    tmp = {Hd, E, W, gt, gdev, dg, aug, f, pval, piv};
    // energy eigenbasis of H
    if (hipMemsetAsync(Hd, 0, sizeof(double2) * NN, s) != hipSuccess) return cleanup(lb_fail(LB_ERR_DEVICE, "memset"));
    hipLaunchKernelGGL(k_csr_dense_cm, dim3(lb_blocks(N, 256)), dim3(256), 0, s, N, H->rowptr, H->col,
                       (const double2*)H->val, Hd);
    if (hipGetLastError() != hipSuccess) return cleanup(lb_fail(LB_ERR_DEVICE, "launch"));
    if ((rc = lb_impl_eigh(c, N, (double*)Hd, N, E, (double*)pre->U, N, nullptr))) return cleanup(rc);
    // jump operators in that basis: W, their diagonals
    if (hipMemsetAsync(W, 0, sizeof(double) * NN, s) != hipSuccess) return cleanup(lb_fail(LB_ERR_DEVICE, "memset"));
    for (int p = 0; p < P; ++p) {
        if (hipMemsetAsync(Hd, 0, sizeof(double2) * NN, s) != hipSuccess)
            return cleanup(lb_fail(LB_ERR_DEVICE, "memset"));
        hipLaunchKernelGGL(k_csr_dense_cm, dim3(lb_blocks(N, 256)), dim3(256), 0, s, N, L[p].rowptr, L[p].col,
                           (const double2*)L[p].val, Hd);
        if ((rc = zgemm(s, pre, false, false, N, Hd, pre->U, pre->T1)) ||
            (rc = zgemm(s, pre, true, false, N, pre->U, pre->T1, pre->T2)))
            return cleanup(rc);
        hipLaunchKernelGGL(k_jump_accum, dim3(lb_blocks(NN, 256)), dim3(256), 0, s, N, rates[p],
                           (const double2*)pre->T2, W, dg + (int64_t)p * N);
    }
    if (P > 0 && hipMemcpyAsync(gdev, rates, sizeof(double) * P, hipMemcpyHostToDevice, s) != hipSuccess)
        return cleanup(lb_fail(LB_ERR_DEVICE, "copy of the rates failed"));
    hipLaunchKernelGGL(k_col_sums, dim3(N), dim3(256), 0, s, N, (const double*)W, gt);
    hipLaunchKernelGGL(k_den, dim3(lb_blocks(NN, 256)), dim3(256), 0, s, N, (const double*)E, (const double*)gt, P,
                       (const double*)gdev, (const double2*)dg, pre->den);
    // inverse of the bordered rate matrix, Gauss-Jordan with partial pivoting
    const int64_t naug = (int64_t)n * 2 * n;
    hipLaunchKernelGGL(k_border, dim3(lb_blocks(naug, 256)), dim3(256), 0, s, N, (const double*)W, (const double*)gt,
                       aug);
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(1024), 0, s, n, (const double*)aug, k, piv, pval);
        hipLaunchKernelGGL(k_gj_swap, dim3(lb_blocks(2 * n, 256)), dim3(256), 0, s, n, aug, k, (const int*)piv,
                           (const double*)pval, f);
        hipLaunchKernelGGL(k_gj_elim, dim3(lb_blocks(naug, 256)), dim3(256), 0, s, n, aug, k, (const double*)f);
    }
    hipLaunchKernelGGL(k_take_inverse, dim3(lb_blocks((int64_t)n * n, 256)), dim3(256), 0, s, n, (const double*)aug,
                       pre->Binv);
    if (hipGetLastError() != hipSuccess) return cleanup(lb_fail(LB_ERR_DEVICE, "preconditioner set-up launch failed"));
    // a singular rate matrix shows as a zero or non-finite pivot
    double last = 0.0;
    if (hipMemcpyAsync(&last, pval, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return cleanup(lb_fail(LB_ERR_DEVICE, "preconditioner set-up failed"));
    if (!(last != 0.0) || !isfinite(last)) return cleanup(lb_fail(LB_ERR_INVALID_ARG, "rate matrix is singular"));
    *out = pre;
    return cleanup(LB_OK);
}

int lb_impl_secular_apply(lb_ctx* c, const lb_secular* pre, const double* r, double* z) {
    hipStream_t s = c->stream;
    const int N = pre->N;
    const int64_t NN = (int64_t)N * N;
    const int n = N + 1;
    const int64_t P = lb_npairs(N);
    int rc;
    double* scan = pre->pv + 2 * n;
    hipLaunchKernelGGL(k_diag_scan<true>, dim3(1), dim3(1024), 0, s, N, (const double2*)nullptr, r, scan);
    hipLaunchKernelGGL(k_v_to_herm, dim3(lb_blocks(P + N, 256)), dim3(256), 0, s, N, r, (const double*)scan, pre->T1);
    LB_CHECK_LAUNCH();
    if ((rc = zgemm(s, pre, false, false, N, pre->T1, pre->U, pre->T2)) || (rc = zgemm(s, pre, true, false, N, pre->U, pre->T2, pre->T1)))
        return rc;
    hipLaunchKernelGGL(k_diag_rhs, dim3(lb_blocks(n, 256)), dim3(256), 0, s, N, (const double2*)pre->T1, pre->pv);
    hipLaunchKernelGGL(k_small_gemv, dim3(lb_blocks(n, 4)), dim3(256), 0, s, n, (const double*)pre->Binv,
                       (const double*)pre->pv, pre->pv + n);
    hipLaunchKernelGGL(k_apply_den, dim3(lb_blocks(NN, 256)), dim3(256), 0, s, N, pre->T1, (const double2*)pre->den,
                       (const double*)(pre->pv + n));
    LB_CHECK_LAUNCH();
    if ((rc = zgemm(s, pre, false, true, N, pre->T1, pre->U, pre->T2)) || (rc = zgemm(s, pre, false, false, N, pre->U, pre->T2, pre->T1)))
        return rc;
    hipLaunchKernelGGL(k_diag_scan<false>, dim3(1), dim3(1024), 0, s, N, (const double2*)pre->T1, (const double*)nullptr,
                       scan);
    hipLaunchKernelGGL(k_herm_to_v, dim3(lb_blocks(NN - 1, 256)), dim3(256), 0, s, N, (const double2*)pre->T1,
                       (const double*)scan, z);
    LB_CHECK_LAUNCH();
    return LB_OK;
}

int64_t lb_secular_size(const lb_secular* pre) { return pre->M; }

void lb_impl_secular_destroy(lb_secular* pre) {
    if (!pre) return;
    (void)hipSetDevice(pre->device);
    (void)hipDeviceSynchronize();
    secular_free(pre);
}
