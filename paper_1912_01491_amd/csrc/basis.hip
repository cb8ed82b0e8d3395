// Gell-Mann index-class generator and nonzero structure-constant enumerator.
//
// Basis (Sec. 2, Eqs. (3)-(5)): S^(j,k) and J^(j,k) for pairs j<k and the
// diagonal D^l. Structure constants (Eq. (11)): with T_abc = Tr(F_a F_b F_c),
// f_abc = 2 Im T_abc and d_abc = 2 Re T_abc for Hermitian generators. Only
// three index classes give T != 0 (Table 1, step 2.2: O(N^3) nonzeros, each
// O(1) to evaluate):
//   1. triangles: three pair generators on the edges of a vertex triangle;
//   2. a pair generator, a generator on the same pair, and a D^l whose support
//      meets the pair;
//   3. three diagonal generators (d only).
// Each thread owns one first index m; a count pass sizes the output, a host
// exclusive scan gives per-m offsets, and a fill pass writes the triples.
#include "lb_internal.h"

namespace {

constexpr double kR = 0.70710678118654752440;  // 1/sqrt(2)

__global__ void k_basis_table(int N, int64_t M, int32_t* table) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    int c, j, k;
    lb_decode(N, i, c, j, k);
    table[3 * i + 0] = c;
    table[3 * i + 1] = j;
    table[3 * i + 2] = k;
}

// (F)_{ab} of a pair generator of class cls (0 = S, 1 = J) on pair {a, b}.
__device__ __forceinline__ cd pelem(int cls, int a, int b) {
    if (cls == 0) return cmk(kR, 0.0);
    return cmk(0.0, a < b ? -kR : kR);
}

// w_l(j) != w_l(k) for j < k (structural)
__device__ __forceinline__ bool diffnz(int l, int j, int k) { return j <= l && k >= l; }
// w_l(j) + w_l(k) != 0 for j < k (structural)
__device__ __forceinline__ bool sumnz(int l, int j, int k) { return j <= l && !(j == 0 && k == 1 && l == 1); }

struct Emitter {
    int which;       // 0: f, 1: d
    bool write;
    int64_t n;       // entries emitted so far
    int32_t* mns;
    double* val;
    int32_t m;
    __device__ __forceinline__ void put(int64_t nidx, int64_t sidx, double v) {
        if (write) {
            mns[3 * n + 0] = m;
            mns[3 * n + 1] = (int32_t)nidx;
            mns[3 * n + 2] = (int32_t)sidx;
            val[n] = v;
        }
        ++n;
    }
    // T = Tr(F_m F_n F_s); emits f = 2 Im T or d = 2 Re T if structurally nonzero
    __device__ __forceinline__ void put_t(int64_t nidx, int64_t sidx, cd T, bool f_nz, bool d_nz) {
        if (which == 0 && f_nz) put(nidx, sidx, 2.0 * T.im);
        if (which == 1 && d_nz) put(nidx, sidx, 2.0 * T.re);
    }
};

__device__ void enumerate_m(int N, int64_t m, Emitter& E) {
    const int64_t P = lb_npairs(N);
    int cls, j, k;
    lb_decode(N, m, cls, j, k);
    if (cls < 2) {
        // class 1: triangles (j, k, w)
        for (int w = 0; w < N; ++w) {
            if (w == j || w == k) continue;
            const int64_t pjw = lb_upair(N, j, w), pkw = lb_upair(N, k, w);
            for (int Y = 0; Y < 2; ++Y)
                for (int Z = 0; Z < 2; ++Z) {
                    // n on {j,w}, s on {k,w}: T = (F_m)_{kj} (F_n)_{jw} (F_s)_{wk}
                    cd T = cmul(cmul(pelem(cls, k, j), pelem(Y, j, w)), pelem(Z, w, k));
                    bool fnz = T.im != 0.0, dnz = T.re != 0.0;
                    E.put_t(Y * P + pjw, Z * P + pkw, T, fnz, dnz);
                }
            for (int Y = 0; Y < 2; ++Y)
                for (int Z = 0; Z < 2; ++Z) {
                    // n on {k,w}, s on {j,w}: T = (F_m)_{jk} (F_n)_{kw} (F_s)_{wj}
                    cd T = cmul(cmul(pelem(cls, j, k), pelem(Y, k, w)), pelem(Z, w, j));
                    bool fnz = T.im != 0.0, dnz = T.re != 0.0;
                    E.put_t(Y * P + pkw, Z * P + pjw, T, fnz, dnz);
                }
        }
        // class 2: same pair and a diagonal generator
        const int64_t pjk = lb_pair(N, j, k);
        for (int Y = 0; Y < 2; ++Y) {
            const int64_t nidx = Y * P + pjk;
            for (int l = 1; l < N; ++l) {
                // n = Y(j,k), s = D^l: T = sum_{a in {j,k}} (F_m)_{a a'} (F_n)_{a' a} w_l(a)
                cd T = cadd(cscale(cmul(pelem(cls, j, k), pelem(Y, k, j)), lb_wdiag(l, j)),
                            cscale(cmul(pelem(cls, k, j), pelem(Y, j, k)), lb_wdiag(l, k)));
                const bool same = (Y == cls);
                E.put_t(nidx, 2 * P + (l - 1), T, !same && diffnz(l, j, k), same && sumnz(l, j, k));
            }
        }
        for (int l = 1; l < N; ++l) {
            for (int Z = 0; Z < 2; ++Z) {
                // n = D^l, s = Z(j,k): T = sum_a (F_m)_{a a'} w_l(a') (F_s)_{a' a}
                cd T = cadd(cscale(cmul(pelem(cls, j, k), pelem(Z, k, j)), lb_wdiag(l, k)),
                            cscale(cmul(pelem(cls, k, j), pelem(Z, j, k)), lb_wdiag(l, j)));
                const bool same = (Z == cls);
                E.put_t(2 * P + (l - 1), Z * P + pjk, T, !same && diffnz(l, j, k), same && sumnz(l, j, k));
            }
        }
    } else {
        const int l = j;
        // class 2 with m = D^l: pairs (p, q) whose support meets rows 0..l
        for (int p = 0; p <= l && p < N - 1; ++p)
            for (int q = p + 1; q < N; ++q) {
                const int64_t ppq = lb_pair(N, p, q);
                for (int Y = 0; Y < 2; ++Y)
                    for (int Z = 0; Z < 2; ++Z) {
                        // T = sum_{a in {p,q}} w_l(a) (F_n)_{a a'} (F_s)_{a' a}
                        cd T = cadd(cscale(cmul(pelem(Y, p, q), pelem(Z, q, p)), lb_wdiag(l, p)),
                                    cscale(cmul(pelem(Y, q, p), pelem(Z, p, q)), lb_wdiag(l, q)));
                        const bool same = (Y == Z);
                        E.put_t(Y * P + ppq, Z * P + ppq, T, !same && diffnz(l, p, q), same && sumnz(l, p, q));
                    }
            }
        // class 3: three diagonal generators (d only)
        if (E.which == 1) {
            for (int l2 = 1; l2 < N; ++l2)
                for (int l3 = 1; l3 < N; ++l3) {
                    double v = 0.0;
                    bool nz = false;
                    if (l2 == l && l3 > l) { v = 2.0 / sqrt((double)l3 * (l3 + 1)); nz = true; }
                    else if (l3 == l && l2 > l) { v = 2.0 / sqrt((double)l2 * (l2 + 1)); nz = true; }
                    else if (l2 == l3 && l2 < l) { v = 2.0 / sqrt((double)l * (l + 1)); nz = true; }
                    else if (l2 == l && l3 == l && l >= 2) { v = -2.0 * (l - 1) / sqrt((double)l * (l + 1)); nz = true; }
                    if (nz) E.put(2 * P + (l2 - 1), 2 * P + (l3 - 1), v);
                }
        }
    }
}

__global__ void k_fd_count(int N, int64_t M, int which, int64_t* counts) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    Emitter E{which, false, 0, nullptr, nullptr, (int32_t)m};
    enumerate_m(N, m, E);
    counts[m] = E.n;
}

__global__ void k_fd_fill(int N, int64_t M, int which, const int64_t* offsets, int32_t* mns, double* val) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const int64_t off = offsets[m];
    Emitter E{which, true, 0, mns + 3 * off, val + off, (int32_t)m};
    enumerate_m(N, m, E);
}

}  // namespace

int lb_impl_basis_table(lb_ctx* c, int N, int32_t* table) {
    const int64_t M = (int64_t)N * N - 1;
    hipLaunchKernelGGL(k_basis_table, dim3(lb_blocks(M, 256)), dim3(256), 0, c->stream, N, M, table);
    LB_CHECK_LAUNCH();
    return LB_OK;
}

// Count pass. Uses the workspace as [counts (M) | offsets (M+1)]; when
// want_offsets is set the exclusive scan of the counts is left in the
// offsets part for lb_impl_fd_fill. Synchronizes the stream.
int lb_impl_fd_count(lb_ctx* c, int N, int which, int64_t* count, int64_t* offsets_dev) {
    const int64_t M = (int64_t)N * N - 1;
    (void)offsets_dev;
    int rc = lb_ws_reserve(c, sizeof(int64_t) * (2 * M + 1));
    if (rc) return rc;
    int64_t* counts = (int64_t*)c->ws;
    int64_t* offsets = counts + M;
    hipLaunchKernelGGL(k_fd_count, dim3(lb_blocks(M, 128)), dim3(128), 0, c->stream, N, M, which, counts);
    LB_CHECK_LAUNCH();
    rc = lb_host_reserve(c, sizeof(int64_t) * (M + 1));
    if (rc) return rc;
    int64_t* h = (int64_t*)c->host;
    LB_HIP(hipMemcpyAsync(h, counts, sizeof(int64_t) * M, hipMemcpyDeviceToHost, c->stream));
    LB_HIP(hipStreamSynchronize(c->stream));
    int64_t run = 0;
    for (int64_t m = 0; m < M; ++m) {
        const int64_t v = h[m];
        h[m] = run;
        run += v;
    }
    h[M] = run;
    *count = run;
    LB_HIP(hipMemcpyAsync(offsets, h, sizeof(int64_t) * (M + 1), hipMemcpyHostToDevice, c->stream));
    LB_HIP(hipStreamSynchronize(c->stream));
    return LB_OK;
}

int lb_impl_fd_fill(lb_ctx* c, int N, int which, const int64_t* offsets_dev, int32_t* mns, double* val) {
    const int64_t M = (int64_t)N * N - 1;
    hipLaunchKernelGGL(k_fd_fill, dim3(lb_blocks(M, 128)), dim3(128), 0, c->stream, N, M, which,
                       offsets_dev, mns, val);
    LB_CHECK_LAUNCH();
    return LB_OK;
}
