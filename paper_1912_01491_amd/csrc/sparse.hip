// Sparse data preparation: Q in CSR form and K for a Hamiltonian H and jump
// operators L_p with rates g_p, i.e. a Kossakowski matrix given through its
// spectral form gamma = sum_p g_p l_p l_p^+ (Sec. 2) with sparse l_p, as in the
// dimer model of Sec. 3 (P = 1).
//
// With L(X) = -i[H, X] + sum_p g_p (L_p X L_p^+ - 1/2 {L_p^+ L_p, X}) and its
// adjoint L^+(Y) = i[H, Y] + sum_p g_p (L_p^+ Y L_p - 1/2 {L_p^+ L_p, Y}),
//     Q_sn = Tr(F_s L(F_n)) = Tr(L^+(F_s) F_n),  K_s = Tr(L^+(F_s)) / N,
// so row s of Q is the expansion of the sparse matrix L^+(F_s) over the basis:
// off-diagonal entries give the S/J columns, the diagonal gives the D columns
// through prefix sums (w_m(x) = 1/sqrt(m(m+1)) for x < m, -m/sqrt(m(m+1)) at
// x = m). Rows of the diagonal generators are built column-wise instead:
// Q[D^m][n] = sum_x w_m(x) (L(F_n))_xx, and column n contributes to every
// row m >= the first position where diag(L(F_n)) is nonzero.
//
// The identity part c = Tr(L_p)/N of each jump operator is moved into the
// Hamiltonian (H += (i g_p/2)(conj(c) L0 - c L0^+), L0 = L_p - c 1), because
// the generator basis has no identity element.
//
// Pipeline (count phase and fill phase run the same kernels; the fill phase
// additionally writes columns and values):
//   densify H, L_p -> trace shift -> G = sum_p g_p L0^+ L0, A = i H - G/2
//   column lists of A and L0_p, row lists of L0_p (ELL, width = max degree)
//   pair rows:   one thread per row, L^+(F_s) in registers, merged and expanded
//   diag lists:  diag(L(F_n)) per column n (count, scan, fill), then their
//                exclusive prefix sums
//   D rows:      one wavefront per row over the columns that carry a diagonal
// Rows are written with sorted column indices (S block, J block, D block);
// entries whose value is exactly zero are not stored.
#include "lb_internal.h"

#include <string.h>

#include <algorithm>

namespace {

constexpr double kR = 0.70710678118654752440;
constexpr int kMaxRowEntries = 64;  // entries of L^+(F_s) held per pair row

struct Ell {
    const int* idx;  // N x W
    const double* val;  // N x W complex
    const int* cnt;  // N
    int W;
};

__device__ __forceinline__ cd ell_val(const Ell& e, int i, int t) { return cload(e.val, (int64_t)i * e.W + t); }
__device__ __forceinline__ int ell_idx(const Ell& e, int i, int t) { return e.idx[(int64_t)i * e.W + t]; }

// ---------------------------------------------------------------------------
// Dense set-up kernels
// ---------------------------------------------------------------------------

__global__ void k_densify(int N, const int64_t* rowptr, const int64_t* col, const double* val, double* D) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    for (int c = 0; c < N; ++c) cstore(D, (int64_t)r * N + c, cmk(0, 0));
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        const int64_t c = col[e];
        if (c < 0 || c >= N) continue;
        cstore(D, (int64_t)r * N + c, cadd(cload(D, (int64_t)r * N + c), cload(val, e)));
    }
}

// single block: c_p = Tr(L_p)/N for all p
__global__ void k_traces(int N, int P, const double* Ld, double* c) {
    __shared__ double sr[256], si[256];
    for (int p = 0; p < P; ++p) {
        double r = 0, i = 0;
        for (int x = threadIdx.x; x < N; x += blockDim.x) {
            const cd v = cload(Ld + 2 * (int64_t)p * N * N, (int64_t)x * N + x);
            r += v.re;
            i += v.im;
        }
        sr[threadIdx.x] = r;
        si[threadIdx.x] = i;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                sr[threadIdx.x] += sr[threadIdx.x + s];
                si[threadIdx.x] += si[threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            c[2 * p] = sr[0] / N;
            c[2 * p + 1] = si[0] / N;
        }
        __syncthreads();
    }
}

// L0_p = L_p - c_p 1 (in place)
__global__ void k_shift_l(int N, int P, double* Ld, const double* c) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)P * N) return;
    const int p = (int)(t / N), x = (int)(t % N);
    double* L = Ld + 2 * (int64_t)p * N * N;
    cstore(L, (int64_t)x * N + x, csub(cload(L, (int64_t)x * N + x), cmk(c[2 * p], c[2 * p + 1])));
}

// H += sum_p (i g_p / 2)(conj(c_p) L0 - c_p L0^+);  G = sum_p g_p L0^+ L0;  A = i H - G/2
__global__ void k_heff_g_a(int N, int P, const double* rates, const double* c, const double* Ld, double* Hd,
                           double* G, double* A) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)N * N) return;
    const int a = (int)(t / N), b = (int)(t % N);
    cd h = cload(Hd, t);
    cd g = cmk(0, 0);
    for (int p = 0; p < P; ++p) {
        const double* L = Ld + 2 * (int64_t)p * N * N;
        const cd cp = cmk(c[2 * p], c[2 * p + 1]);
        const double gp = rates[p];
        const cd l_ab = cload(L, (int64_t)a * N + b);
        const cd ldag_ab = cconj(cload(L, (int64_t)b * N + a));
        const cd d = csub(cmul(cconj(cp), l_ab), cmul(cp, ldag_ab));
        h = cadd(h, cscale(cmk(-d.im, d.re), 0.5 * gp));  // (i g/2) d
        cd s = cmk(0, 0);
        for (int x = 0; x < N; ++x) {
            const cd lxa = cload(L, (int64_t)x * N + a);
            if (lxa.re == 0.0 && lxa.im == 0.0) continue;
            s = cadd(s, cmul(cconj(lxa), cload(L, (int64_t)x * N + b)));
        }
        g = cadd(g, cscale(s, gp));
    }
    cstore(Hd, t, h);
    cstore(G, t, g);
    // A = i h - g/2
    cstore(A, t, cmk(-h.im - 0.5 * g.re, h.re - 0.5 * g.im));
}

// ELL lists of the nonzeros of a dense N x N complex matrix, by column (bycol=1) or row.
__global__ void k_ell_count(int N, const double* D, int bycol, int* cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int n = 0;
    for (int j = 0; j < N; ++j) {
        const cd v = bycol ? cload(D, (int64_t)j * N + i) : cload(D, (int64_t)i * N + j);
        if (v.re != 0.0 || v.im != 0.0) ++n;
    }
    cnt[i] = n;
}

__global__ void k_ell_fill(int N, const double* D, int bycol, int W, int* idx, double* val) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int n = 0;
    for (int j = 0; j < N; ++j) {
        const cd v = bycol ? cload(D, (int64_t)j * N + i) : cload(D, (int64_t)i * N + j);
        if (v.re != 0.0 || v.im != 0.0) {
            idx[(int64_t)i * W + n] = j;
            cstore(val, (int64_t)i * W + n, v);
            ++n;
        }
    }
}

// diag(L(1))_x = 2 Re Z_xx + sum_p g_p sum_b |L0_p,xb|^2, with Z = A^+ (Re Z_xx = Re A_xx)
__global__ void k_l1diag(int N, int P, const double* rates, const double* A, const double* Ld, double* out) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= N) return;
    double s = 2.0 * cload(A, (int64_t)x * N + x).re;
    for (int p = 0; p < P; ++p) {
        const double* L = Ld + 2 * (int64_t)p * N * N;
        double q = 0;
        for (int b = 0; b < N; ++b) {
            const cd v = cload(L, (int64_t)x * N + b);
            q += v.re * v.re + v.im * v.im;
        }
        s += rates[p] * q;
    }
    out[x] = s;
}

// ---------------------------------------------------------------------------
// Pair rows: Y = L^+(F_s), F_s = al E_uv + be E_vu (u < v)
// ---------------------------------------------------------------------------

struct PairArgs {
    int N, P;
    int64_t Pp;  // number of pairs
    Ell Acol;    // columns of A = iH - G/2
    const Ell* Lrow;  // rows of L0_p (P entries, device array)
    const double* rates;
    // outputs
    int64_t* cnt;          // count phase: entries per row
    const int64_t* rowptr; // fill phase
    int64_t* col;
    double* val;
    double* K;
    int* overflow;
};

struct Ent {
    int a, c;
    cd v;
};

__device__ __forceinline__ void push(Ent* E, int& n, int a, int c, cd v, int* overflow) {
    if (n >= kMaxRowEntries) {
        *overflow = 1;
        return;
    }
    E[n].a = a;
    E[n].c = c;
    E[n].v = v;
    ++n;
}

__global__ void k_pair_rows(PairArgs g, int fill) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= 2 * g.Pp) return;
    const int N = g.N;
    const int cls = s >= g.Pp ? 1 : 0;
    const int64_t ps = s - cls * g.Pp;
    int cc, u, v;
    lb_decode(N, ps, cc, u, v);
    const cd al = cls == 0 ? cmk(kR, 0) : cmk(0, -kR);  // (F_s)_uv
    const cd be = cls == 0 ? cmk(kR, 0) : cmk(0, kR);   // (F_s)_vu
    Ent E[kMaxRowEntries];
    int n = 0;
    // i H F_s - G F_s / 2 = A F_s: (a, v) += al A_au, (a, u) += be A_av
    for (int t = 0; t < g.Acol.cnt[u]; ++t) push(E, n, ell_idx(g.Acol, u, t), v, cmul(al, ell_val(g.Acol, u, t)), g.overflow);
    for (int t = 0; t < g.Acol.cnt[v]; ++t) push(E, n, ell_idx(g.Acol, v, t), u, cmul(be, ell_val(g.Acol, v, t)), g.overflow);
    // -i F_s H - F_s G / 2 = F_s A^+: (u, c) += al conj(A_cv), (v, c) += be conj(A_cu)
    for (int t = 0; t < g.Acol.cnt[v]; ++t) push(E, n, u, ell_idx(g.Acol, v, t), cmul(al, cconj(ell_val(g.Acol, v, t))), g.overflow);
    for (int t = 0; t < g.Acol.cnt[u]; ++t) push(E, n, v, ell_idx(g.Acol, u, t), cmul(be, cconj(ell_val(g.Acol, u, t))), g.overflow);
    // g_p L0^+ F_s L0: (a, c) += g al conj(L0_ua) L0_vc + g be conj(L0_va) L0_uc
    for (int p = 0; p < g.P; ++p) {
        const Ell Lr = g.Lrow[p];
        const double gp = g.rates[p];
        if (gp == 0.0) continue;
        for (int t1 = 0; t1 < Lr.cnt[u]; ++t1)
            for (int t2 = 0; t2 < Lr.cnt[v]; ++t2) {
                const int a = ell_idx(Lr, u, t1), c = ell_idx(Lr, v, t2);
                push(E, n, a, c, cscale(cmul(al, cmul(cconj(ell_val(Lr, u, t1)), ell_val(Lr, v, t2))), gp), g.overflow);
            }
        for (int t1 = 0; t1 < Lr.cnt[v]; ++t1)
            for (int t2 = 0; t2 < Lr.cnt[u]; ++t2) {
                const int a = ell_idx(Lr, v, t1), c = ell_idx(Lr, u, t2);
                push(E, n, a, c, cscale(cmul(be, cmul(cconj(ell_val(Lr, v, t1)), ell_val(Lr, u, t2))), gp), g.overflow);
            }
    }
    // order: off-diagonal entries by (pair, a) with diagonal entries last by position;
    // key = pair position * 2 + (a > c) for off-diagonal, large + x for diagonal
    const int64_t Pp = g.Pp;
    auto key = [&](const Ent& e) -> int64_t {
        if (e.a == e.c) return 2 * Pp + e.a;
        return 2 * lb_upair(N, e.a, e.c) + (e.a > e.c ? 1 : 0);
    };
    for (int i = 1; i < n; ++i) {  // insertion sort (n is small)
        Ent x = E[i];
        const int64_t kx = key(x);
        int j = i - 1;
        while (j >= 0 && key(E[j]) > kx) {
            E[j + 1] = E[j];
            --j;
        }
        E[j + 1] = x;
    }
    // merge equal keys
    int m = 0;
    for (int i = 0; i < n; ++i) {
        if (m > 0 && key(E[m - 1]) == key(E[i])) E[m - 1].v = cadd(E[m - 1].v, E[i].v);
        else E[m++] = E[i];
    }
    // diagonal range and trace
    int first_diag = -1;
    cd tr = cmk(0, 0);
    for (int i = 0; i < m; ++i) {
        if (E[i].a == E[i].c) {
            if (first_diag < 0) first_diag = i;
            tr = cadd(tr, E[i].v);
        }
    }
    // D columns m from max(1, xmin) to xmax, or to N-1 when Tr(Y) != 0: beyond the
    // last diagonal position the value is Tr(Y)/sqrt(m(m+1)) = N K_s/sqrt(m(m+1)).
    int nd = 0, xmin = N, xhi = -1;
    if (first_diag >= 0) {
        xmin = E[first_diag].a;
        double asum = 0;
        for (int i = first_diag; i < m; ++i) asum += fabs(E[i].v.re) + fabs(E[i].v.im);
        const bool traced = fabs(tr.re) > 1e-13 * asum;
        xhi = traced ? N - 1 : E[m - 1].a;
        const int lo = xmin > 1 ? xmin : 1;
        nd = xhi >= lo ? xhi - lo + 1 : 0;
    }
    // Entries are emitted in column order (S block, J block, D block); values
    // that are exactly zero (e.g. the S part of i[H, S_pq] for real H) are not
    // stored. Count and fill run the same arithmetic, so they agree on which
    // entries are kept.
    int64_t o = fill ? g.rowptr[s] : 0;
    if (fill) g.K[s] = tr.re / N;
    for (int part = 0; part < 2; ++part) {
        for (int i = 0; i < m; ++i) {
            if (E[i].a == E[i].c) break;
            const int64_t pp = lb_upair(N, E[i].a, E[i].c);
            cd ypq = cmk(0, 0), yqp = cmk(0, 0);  // (p,q) with p < q
            if (E[i].a < E[i].c) ypq = E[i].v;
            else yqp = E[i].v;
            if (i + 1 < m && E[i + 1].a != E[i + 1].c && lb_upair(N, E[i + 1].a, E[i + 1].c) == pp) {
                ++i;
                if (E[i].a < E[i].c) ypq = cadd(ypq, E[i].v);
                else yqp = cadd(yqp, E[i].v);
            }
            // Tr(Y S_pq) = r (Y_pq + Y_qp); Tr(Y J_pq) = i r (Y_pq - Y_qp)
            const double q = part == 0 ? kR * (ypq.re + yqp.re) : -kR * (ypq.im - yqp.im);
            if (q == 0.0) continue;
            if (fill) {
                g.col[o] = part * Pp + pp;
                g.val[o] = q;
            }
            ++o;
        }
    }
    if (nd > 0) {
        cd pre = cmk(0, 0);
        int di = first_diag;
        for (int x = 0; x < N; ++x) {
            cd yx = cmk(0, 0);
            if (di < m && E[di].a == x) {
                yx = E[di].v;
                ++di;
            }
            if (x >= 1 && x >= xmin && x <= xhi) {
                const double q = (pre.re - (double)x * yx.re) / sqrt((double)x * (x + 1));
                if (q != 0.0) {
                    if (fill) {
                        g.col[o] = 2 * Pp + x - 1;
                        g.val[o] = q;
                    }
                    ++o;
                }
            }
            pre = cadd(pre, yx);
        }
    }
    if (!fill) g.cnt[s] = o;
}

// ---------------------------------------------------------------------------
// Diagonal of L(F_n) for every column n (carrying lists for the D rows)
// ---------------------------------------------------------------------------

struct DiagArgs {
    int N, P;
    int64_t Pp, M;
    const double* A;   // dense N x N, Z = A^+
    const Ell* Lcol;   // columns of L0_p
    const Ell* Lrow;   // rows of L0_p
    const double* rates;
    int64_t* cnt;
    const int64_t* off;
    int* pos;
    double* val;   // complex
};

__device__ __forceinline__ cd zel(const double* A, int N, int i, int j) { return cconj(cload(A, (int64_t)j * N + i)); }

// small sorted accumulator
struct DAcc {
    int x[kMaxRowEntries];
    cd v[kMaxRowEntries];
    int n;
    __device__ void add(int p, cd val, int* ovf) {
        for (int i = 0; i < n; ++i)
            if (x[i] == p) {
                v[i] = cadd(v[i], val);
                return;
            }
        if (n >= kMaxRowEntries) {
            *ovf = 1;
            return;
        }
        int i = n++;
        while (i > 0 && x[i - 1] > p) {
            x[i] = x[i - 1];
            v[i] = v[i - 1];
            --i;
        }
        x[i] = p;
        v[i] = val;
    }
};

__global__ void k_diag_pairs(DiagArgs g, int fill, int* ovf) {
    const int64_t nidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (nidx >= 2 * g.Pp) return;
    const int N = g.N;
    const int cls = nidx >= g.Pp ? 1 : 0;
    int cc, x, y;
    lb_decode(N, nidx - cls * g.Pp, cc, x, y);
    const cd al = cls == 0 ? cmk(kR, 0) : cmk(0, -kR);  // (F_n)_xy
    const cd be = cls == 0 ? cmk(kR, 0) : cmk(0, kR);   // (F_n)_yx
    DAcc acc;
    acc.n = 0;
    // (Z F_n + F_n Z^+)_aa: a = y: Z_yx al + be conj(Z_yx); a = x: Z_xy be + al conj(Z_xy)
    const cd zyx = zel(g.A, N, y, x), zxy = zel(g.A, N, x, y);
    const cd dy = cadd(cmul(zyx, al), cmul(be, cconj(zyx)));
    const cd dx = cadd(cmul(zxy, be), cmul(al, cconj(zxy)));
    if (dx.re != 0.0 || dx.im != 0.0) acc.add(x, dx, ovf);
    if (dy.re != 0.0 || dy.im != 0.0) acc.add(y, dy, ovf);
    // g_p (L0 F_n L0^+)_aa = g_p (L0_ax al conj(L0_ay) + L0_ay be conj(L0_ax))
    for (int p = 0; p < g.P; ++p) {
        const Ell Lc = g.Lcol[p];
        const double gp = g.rates[p];
        if (gp == 0.0) continue;
        for (int t1 = 0; t1 < Lc.cnt[x]; ++t1) {
            const int a = ell_idx(Lc, x, t1);
            for (int t2 = 0; t2 < Lc.cnt[y]; ++t2) {
                if (ell_idx(Lc, y, t2) != a) continue;
                const cd lax = ell_val(Lc, x, t1), lay = ell_val(Lc, y, t2);
                const cd d = cadd(cmul(lax, cmul(al, cconj(lay))), cmul(lay, cmul(be, cconj(lax))));
                acc.add(a, cscale(d, gp), ovf);
            }
        }
    }
    if (!fill) {
        g.cnt[nidx] = acc.n;
        return;
    }
    const int64_t o = g.off[nidx];
    for (int i = 0; i < acc.n; ++i) {
        g.pos[o + i] = acc.x[i];
        cstore(g.val, o + i, acc.v[i]);
    }
}

// D columns n = D^m': diag_a = w_m'(a) 2 Re Z_aa + sum_p g_p sum_{y <= m'} w_m'(y) |L0_p,ay|^2
__global__ void k_diag_dcols(DiagArgs g, int fill) {
    const int mm = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const int N = g.N;
    if (mm >= N) return;
    const int64_t nidx = 2 * g.Pp + mm - 1;
    int64_t o = fill ? g.off[nidx] : 0;
    int64_t n = 0;
    for (int a = 0; a < N; ++a) {
        bool nz = a <= mm;
        cd d = cmk(lb_wdiag(mm, a) * 2.0 * cload(g.A, (int64_t)a * N + a).re, 0.0);
        for (int p = 0; p < g.P; ++p) {
            const Ell Lr = g.Lrow[p];
            double s = 0;
            for (int t = 0; t < Lr.cnt[a]; ++t) {
                const int yy = ell_idx(Lr, a, t);
                if (yy > mm) continue;
                const cd l = ell_val(Lr, a, t);
                s += lb_wdiag(mm, yy) * (l.re * l.re + l.im * l.im);
                nz = true;
            }
            d.re += g.rates[p] * s;
        }
        if (!nz) continue;
        if (fill) {
            g.pos[o + n] = a;
            cstore(g.val, o + n, d);
        }
        ++n;
    }
    if (!fill) g.cnt[nidx] = n;
}

// D rows: Q[D^m][n] = sum_x w_m(x) diag_n(x) = (pre_n(m) - m diag_n(m)) / sqrt(m(m+1)),
// pre_n(m) = sum_{x<m} diag_n(x), over carrying columns n with key(n) <= m.
struct DRowArgs {
    int N;
    int64_t Pp, M;
    int64_t ncarry;
    const int64_t* carry;   // carrying column indices, increasing
    const int64_t* off;     // per column offsets into pos/val (M+1)
    const int* pos;
    const double* val;
    const double* pref;     // exclusive prefix of Re val within each column's list
    const double* l1diag;
    int64_t* cnt;
    const int64_t* rowptr;
    int64_t* col;
    double* qv;
    double* K;
};

// Exclusive prefix sums of the diagonal lists, one thread per carrying column.
__global__ void k_diag_prefix(int64_t ncarry, const int64_t* carry, const int64_t* off, const double* val,
                              double* pref) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncarry) return;
    const int64_t c = carry[t];
    double run = 0;
    for (int64_t e = off[c]; e < off[c + 1]; ++e) {
        pref[e] = run;
        run += val[2 * e];
    }
}

// One wavefront per D row: lanes take 64 carrying columns at a time; a column
// contributes when its list reaches row m (key <= m <= last position: the list
// sums to Tr L(F_n) = 0, so rows beyond its last position vanish) and the value
// is not exactly zero. A ballot keeps the columns in increasing order.
__global__ __launch_bounds__(256) void k_drows_sparse(DRowArgs g, int fill) {
    const int lane = threadIdx.x & 63;
    const int m = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) + 1;
    const int N = g.N;
    if (m >= N) return;
    const int64_t row = 2 * g.Pp + m - 1;
    const double nrm = 1.0 / sqrt((double)m * (m + 1));
    int64_t o = fill ? g.rowptr[row] : 0;
    for (int64_t t0 = 0; t0 < g.ncarry; t0 += 64) {
        const int64_t t = t0 + lane;
        int64_t c = 0;
        double q = 0.0;
        bool keep = false;
        if (t < g.ncarry) {
            c = g.carry[t];
            int64_t lo = g.off[c], hi = g.off[c + 1] - 1;
            const int key = g.pos[lo] > 1 ? g.pos[lo] : 1;
            if (key <= m && g.pos[hi] >= m) {
                while (lo < hi) {  // first entry at position >= m
                    const int64_t mid = (lo + hi) >> 1;
                    if (g.pos[mid] < m) lo = mid + 1;
                    else hi = mid;
                }
                const double at = g.pos[lo] == m ? g.val[2 * lo] : 0.0;
                q = (g.pref[lo] - (double)m * at) * nrm;
                keep = q != 0.0;
            }
        }
        const unsigned long long mask = __ballot(keep);
        if (keep && fill) {
            const int64_t r = o + __popcll(mask & ((1ull << lane) - 1ull));
            g.col[r] = c;
            g.qv[r] = q;
        }
        o += __popcll(mask);
    }
    if (lane != 0) return;
    if (!fill) {
        g.cnt[row] = o;
        return;
    }
    double k = 0;
    for (int x = 0; x <= m; ++x) k += lb_wdiag(m, x) * g.l1diag[x];
    g.K[row] = k / N;
}

__global__ void k_mark_carry(int64_t M, const int64_t* cnt, int64_t* flag) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < M) flag[c] = cnt[c] > 0 ? 1 : 0;
}

}  // namespace

// Exclusive scan of n int64 on the host through the pinned buffer; writes n+1 offsets.
static int host_scan(lb_ctx* c, int64_t* dev, int64_t n, int64_t* total) {
    int rc = lb_host_reserve(c, sizeof(int64_t) * (n + 1));
    if (rc) return rc;
    int64_t* h = (int64_t*)c->host;
    LB_HIP(hipMemcpyAsync(h, dev, sizeof(int64_t) * n, hipMemcpyDeviceToHost, c->stream));
    LB_HIP(hipStreamSynchronize(c->stream));
    int64_t run = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t v = h[i];
        h[i] = run;
        run += v;
    }
    h[n] = run;
    *total = run;
    LB_HIP(hipMemcpyAsync(dev, h, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, c->stream));
    LB_HIP(hipStreamSynchronize(c->stream));
    return LB_OK;
}

static int max_of(lb_ctx* c, const int* dev, int n, int* out) {
    int rc = lb_host_reserve(c, sizeof(int) * n);
    if (rc) return rc;
    int* h = (int*)c->host;
    LB_HIP(hipMemcpyAsync(h, dev, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
    LB_HIP(hipStreamSynchronize(c->stream));
    int m = 0;
    for (int i = 0; i < n; ++i) m = std::max(m, h[i]);
    *out = m;
    return LB_OK;
}

// Returns LB_OK, a negative status, or 1 when the workspace must grow to *want
// bytes first (growing reallocates it, so the caller restarts from the top).
static int sparse_body(lb_ctx* c, int N, const lb_csr_c128* H, int P, const double* rates, const lb_csr_c128* L,
                       int64_t* nnz, int64_t* rowptr, int64_t* col, double* val, double* K, size_t* want) {
    const bool fill = rowptr != nullptr;
    hipStream_t s = c->stream;
    const int64_t M = (int64_t)N * N - 1;
    const int64_t Pp = lb_npairs(N);
    const int64_t NN = (int64_t)N * N;
    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = lb_align(off + bytes, 256);
        return o;
    };
    const size_t o_h = take(sizeof(double) * 2 * NN);
    const size_t o_l = take(sizeof(double) * 2 * NN * (P > 0 ? P : 1));
    const size_t o_g = take(sizeof(double) * 2 * NN);
    const size_t o_a = take(sizeof(double) * 2 * NN);
    const size_t o_c = take(sizeof(double) * 2 * (P + 1));
    const size_t o_rates = take(sizeof(double) * (P + 1));
    const size_t o_l1 = take(sizeof(double) * N);
    const size_t o_cnt = take(sizeof(int) * N * (1 + 2 * (P > 0 ? P : 1)));
    const size_t o_ells = take(sizeof(Ell) * 2 * (P > 0 ? P : 1));
    const size_t o_rowcnt = take(sizeof(int64_t) * (M + 1));
    const size_t o_dcnt = take(sizeof(int64_t) * (M + 1));
    const size_t o_carry = take(sizeof(int64_t) * (M + 1));
    const size_t o_ovf = take(sizeof(int) * 2);
    const size_t fixed = off;
    int rc = lb_ws_reserve(c, fixed);
    if (rc) return rc;
    char* ws = (char*)c->ws;
    double* Hd = (double*)(ws + o_h);
    double* Ld = (double*)(ws + o_l);
    double* G = (double*)(ws + o_g);
    double* A = (double*)(ws + o_a);
    double* cvec = (double*)(ws + o_c);
    double* drates = (double*)(ws + o_rates);
    double* l1 = (double*)(ws + o_l1);
    int* cnts = (int*)(ws + o_cnt);
    int64_t* rowcnt = (int64_t*)(ws + o_rowcnt);
    int64_t* dcnt = (int64_t*)(ws + o_dcnt);
    int64_t* carryflag = (int64_t*)(ws + o_carry);
    int* ovf = (int*)(ws + o_ovf);

    // rates to the device
    rc = lb_host_reserve(c, sizeof(double) * (P + 1));
    if (rc) return rc;
    LB_HIP(hipStreamSynchronize(s));
    for (int p = 0; p < P; ++p) ((double*)c->host)[p] = rates[p];
    if (P > 0) LB_HIP(hipMemcpyAsync(drates, c->host, sizeof(double) * P, hipMemcpyHostToDevice, s));
    LB_HIP(hipMemsetAsync(ovf, 0, sizeof(int) * 2, s));

    // dense set-up
    hipLaunchKernelGGL(k_densify, dim3(lb_blocks(N, 64)), dim3(64), 0, s, N, H->rowptr, H->col, H->val, Hd);
    LB_CHECK_LAUNCH();
    for (int p = 0; p < P; ++p) {
        hipLaunchKernelGGL(k_densify, dim3(lb_blocks(N, 64)), dim3(64), 0, s, N, L[p].rowptr, L[p].col, L[p].val,
                           Ld + 2 * NN * p);
        LB_CHECK_LAUNCH();
    }
    if (P > 0) {
        hipLaunchKernelGGL(k_traces, dim3(1), dim3(256), 0, s, N, P, (const double*)Ld, cvec);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_shift_l, dim3(lb_blocks((int64_t)P * N, 256)), dim3(256), 0, s, N, P, Ld,
                           (const double*)cvec);
        LB_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_heff_g_a, dim3(lb_blocks(NN, 256)), dim3(256), 0, s, N, P, (const double*)drates,
                       (const double*)cvec, (const double*)Ld, Hd, G, A);
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_l1diag, dim3(lb_blocks(N, 64)), dim3(64), 0, s, N, P, (const double*)drates,
                       (const double*)A, (const double*)Ld, l1);
    LB_CHECK_LAUNCH();

    // ELL widths: A by column, L0_p by row and by column
    int* cntA = cnts;
    hipLaunchKernelGGL(k_ell_count, dim3(lb_blocks(N, 64)), dim3(64), 0, s, N, (const double*)A, 1, cntA);
    LB_CHECK_LAUNCH();
    for (int p = 0; p < P; ++p) {
        hipLaunchKernelGGL(k_ell_count, dim3(lb_blocks(N, 64)), dim3(64), 0, s, N, (const double*)(Ld + 2 * NN * p), 0,
                           cnts + N * (1 + 2 * p));
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_ell_count, dim3(lb_blocks(N, 64)), dim3(64), 0, s, N, (const double*)(Ld + 2 * NN * p), 1,
                           cnts + N * (2 + 2 * p));
        LB_CHECK_LAUNCH();
    }
    int WA = 0;
    std::vector<int> WLr(P), WLc(P);
    rc = max_of(c, cntA, N, &WA);
    if (rc) return rc;
    for (int p = 0; p < P; ++p) {
        rc = max_of(c, cnts + N * (1 + 2 * p), N, &WLr[p]);
        if (rc) return rc;
        rc = max_of(c, cnts + N * (2 + 2 * p), N, &WLc[p]);
        if (rc) return rc;
    }
    int bound = 4 * WA;
    for (int p = 0; p < P; ++p) bound += 2 * WLr[p] * WLr[p];
    if (bound > kMaxRowEntries)
        return lb_fail(LB_ERR_UNSUPPORTED,
                       "sparse path needs bounded degrees: up to %d entries per row of L^+(F_s) (limit %d); use "
                       "lindblad_prepare for dense operators",
                       bound, kMaxRowEntries);
    // ELL storage after the fixed part
    size_t o2 = fixed;
    auto take2 = [&](size_t bytes) {
        size_t o = o2;
        o2 = lb_align(o2 + bytes, 256);
        return o;
    };
    const size_t o_Ai = take2(sizeof(int) * (size_t)N * std::max(WA, 1));
    const size_t o_Av = take2(sizeof(double) * 2 * (size_t)N * std::max(WA, 1));
    std::vector<size_t> o_Lri(P), o_Lrv(P), o_Lci(P), o_Lcv(P);
    for (int p = 0; p < P; ++p) {
        o_Lri[p] = take2(sizeof(int) * (size_t)N * std::max(WLr[p], 1));
        o_Lrv[p] = take2(sizeof(double) * 2 * (size_t)N * std::max(WLr[p], 1));
        o_Lci[p] = take2(sizeof(int) * (size_t)N * std::max(WLc[p], 1));
        o_Lcv[p] = take2(sizeof(double) * 2 * (size_t)N * std::max(WLc[p], 1));
    }
    const size_t before_lists = o2;
    if (o2 > c->ws_bytes) {
        *want = o2 + (o2 >> 2);
        return 1;
    }
    hipLaunchKernelGGL(k_ell_fill, dim3(lb_blocks(N, 64)), dim3(64), 0, s, N, (const double*)A, 1, std::max(WA, 1),
                       (int*)(ws + o_Ai), (double*)(ws + o_Av));
    LB_CHECK_LAUNCH();
    std::vector<Ell> hl(2 * std::max(P, 1));
    for (int p = 0; p < P; ++p) {
        hipLaunchKernelGGL(k_ell_fill, dim3(lb_blocks(N, 64)), dim3(64), 0, s, N, (const double*)(Ld + 2 * NN * p), 0,
                           std::max(WLr[p], 1), (int*)(ws + o_Lri[p]), (double*)(ws + o_Lrv[p]));
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_ell_fill, dim3(lb_blocks(N, 64)), dim3(64), 0, s, N, (const double*)(Ld + 2 * NN * p), 1,
                           std::max(WLc[p], 1), (int*)(ws + o_Lci[p]), (double*)(ws + o_Lcv[p]));
        LB_CHECK_LAUNCH();
        hl[p] = Ell{(const int*)(ws + o_Lri[p]), (const double*)(ws + o_Lrv[p]), cnts + N * (1 + 2 * p),
                    std::max(WLr[p], 1)};
        hl[P + p] = Ell{(const int*)(ws + o_Lci[p]), (const double*)(ws + o_Lcv[p]), cnts + N * (2 + 2 * p),
                        std::max(WLc[p], 1)};
    }
    Ell* dells = (Ell*)(ws + o_ells);
    if (P > 0) {
        rc = lb_host_reserve(c, sizeof(Ell) * 2 * P);
        if (rc) return rc;
        LB_HIP(hipStreamSynchronize(s));
        memcpy(c->host, hl.data(), sizeof(Ell) * 2 * P);
        LB_HIP(hipMemcpyAsync(dells, c->host, sizeof(Ell) * 2 * P, hipMemcpyHostToDevice, s));
        LB_HIP(hipStreamSynchronize(s));
    }
    const Ell Acol{(const int*)(ws + o_Ai), (const double*)(ws + o_Av), cntA, std::max(WA, 1)};

    // carrying lists: diag(L(F_n)) for every column n
    DiagArgs da;
    da.N = N;
    da.P = P;
    da.Pp = Pp;
    da.M = M;
    da.A = A;
    da.Lcol = dells + P;
    da.Lrow = dells;
    da.rates = drates;
    da.cnt = dcnt;
    da.off = dcnt;
    da.pos = nullptr;
    da.val = nullptr;
    hipLaunchKernelGGL(k_diag_pairs, dim3(lb_blocks(2 * Pp, 128)), dim3(128), 0, s, da, 0, ovf + 1);
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_diag_dcols, dim3(lb_blocks(N - 1, 64)), dim3(64), 0, s, da, 0);
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_mark_carry, dim3(lb_blocks(M, 256)), dim3(256), 0, s, M, (const int64_t*)dcnt, carryflag);
    LB_CHECK_LAUNCH();
    int64_t dtotal = 0;
    rc = host_scan(c, dcnt, M, &dtotal);
    if (rc) return rc;
    // compacted carrying-column list (host: the flags are read back and compacted)
    rc = lb_host_reserve(c, sizeof(int64_t) * (M + 1));
    if (rc) return rc;
    LB_HIP(hipMemcpyAsync(c->host, carryflag, sizeof(int64_t) * M, hipMemcpyDeviceToHost, s));
    LB_HIP(hipStreamSynchronize(s));
    int64_t ncarry = 0;
    {
        int64_t* h = (int64_t*)c->host;
        for (int64_t i = 0; i < M; ++i)
            if (h[i]) h[ncarry++] = i;
    }
    size_t o3 = before_lists;
    auto take3 = [&](size_t bytes) {
        size_t o = o3;
        o3 = lb_align(o3 + bytes, 256);
        return o;
    };
    const size_t o_pos = take3(sizeof(int) * (size_t)std::max<int64_t>(dtotal, 1));
    const size_t o_dval = take3(sizeof(double) * 2 * (size_t)std::max<int64_t>(dtotal, 1));
    const size_t o_clist = take3(sizeof(int64_t) * (size_t)std::max<int64_t>(ncarry, 1));
    const size_t o_pref = take3(sizeof(double) * (size_t)std::max<int64_t>(dtotal, 1));
    if (o3 > c->ws_bytes) {
        *want = o3 + (o3 >> 3);
        return 1;
    }
    LB_HIP(hipMemcpyAsync(ws + o_clist, c->host, sizeof(int64_t) * std::max<int64_t>(ncarry, 1),
                          hipMemcpyHostToDevice, s));
    da.pos = (int*)(ws + o_pos);
    da.val = (double*)(ws + o_dval);
    hipLaunchKernelGGL(k_diag_pairs, dim3(lb_blocks(2 * Pp, 128)), dim3(128), 0, s, da, 1, ovf + 1);
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_diag_dcols, dim3(lb_blocks(N - 1, 64)), dim3(64), 0, s, da, 1);
    LB_CHECK_LAUNCH();
    if (ncarry > 0) {
        hipLaunchKernelGGL(k_diag_prefix, dim3(lb_blocks(ncarry, 64)), dim3(64), 0, s, ncarry,
                           (const int64_t*)(ws + o_clist), (const int64_t*)dcnt, (const double*)da.val,
                           (double*)(ws + o_pref));
        LB_CHECK_LAUNCH();
    }

    // row counts
    PairArgs pa;
    pa.N = N;
    pa.P = P;
    pa.Pp = Pp;
    pa.Acol = Acol;
    pa.Lrow = dells;
    pa.rates = drates;
    pa.cnt = rowcnt;
    pa.rowptr = rowptr;
    pa.col = col;
    pa.val = val;
    pa.K = K;
    pa.overflow = ovf;
    DRowArgs dr;
    dr.N = N;
    dr.Pp = Pp;
    dr.M = M;
    dr.ncarry = ncarry;
    dr.carry = (const int64_t*)(ws + o_clist);
    dr.off = dcnt;
    dr.pos = da.pos;
    dr.val = da.val;
    dr.pref = (const double*)(ws + o_pref);
    dr.l1diag = l1;
    dr.cnt = rowcnt;
    dr.rowptr = rowptr;
    dr.col = col;
    dr.qv = val;
    dr.K = K;
    if (Pp > 0) {
        hipLaunchKernelGGL(k_pair_rows, dim3(lb_blocks(2 * Pp, 64)), dim3(64), 0, s, pa, 0);
        LB_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_drows_sparse, dim3(lb_blocks((int64_t)(N - 1) * 64, 256)), dim3(256), 0, s, dr, 0);
    LB_CHECK_LAUNCH();
    int hovf[2] = {0, 0};
    LB_HIP(hipMemcpyAsync(hovf, ovf, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
    LB_HIP(hipStreamSynchronize(s));
    if (hovf[0] || hovf[1]) return lb_fail(LB_ERR_UNSUPPORTED, "sparse row buffer overflow (degrees too large)");
    int64_t total = 0;
    if (!fill) {
        rc = host_scan(c, rowcnt, M, &total);
        if (rc) return rc;
        *nnz = total;
        return LB_OK;
    }
    // fill: rowptr from the counts
    rc = lb_host_reserve(c, sizeof(int64_t) * (M + 1));
    if (rc) return rc;
    {
        int64_t* h = (int64_t*)c->host;
        LB_HIP(hipMemcpyAsync(h, rowcnt, sizeof(int64_t) * M, hipMemcpyDeviceToHost, s));
        LB_HIP(hipStreamSynchronize(s));
        int64_t run = 0;
        for (int64_t i = 0; i < M; ++i) {
            const int64_t v = h[i];
            h[i] = run;
            run += v;
        }
        h[M] = run;
        total = run;
        if (total != *nnz)
            return lb_fail(LB_ERR_INVALID_ARG, "nnz=%lld does not match the count phase (%lld)", (long long)*nnz,
                           (long long)total);
        LB_HIP(hipMemcpyAsync(rowptr, h, sizeof(int64_t) * (M + 1), hipMemcpyHostToDevice, s));
        LB_HIP(hipStreamSynchronize(s));
    }
    if (Pp > 0) {
        hipLaunchKernelGGL(k_pair_rows, dim3(lb_blocks(2 * Pp, 64)), dim3(64), 0, s, pa, 1);
        LB_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_drows_sparse, dim3(lb_blocks((int64_t)(N - 1) * 64, 256)), dim3(256), 0, s, dr, 1);
    LB_CHECK_LAUNCH();
    return LB_OK;
}

int lb_impl_sparse(lb_ctx* c, int N, const lb_csr_c128* H, int P, const double* rates, const lb_csr_c128* L,
                   int64_t* nnz, int64_t* rowptr, int64_t* col, double* val, double* K) {
    size_t want = 0;
    for (int attempt = 0; attempt < 4; ++attempt) {
        if (want) {
            int rc = lb_ws_reserve(c, want);
            if (rc) return rc;
        }
        int rc = sparse_body(c, N, H, P, rates, L, nnz, rowptr, col, val, K, &want);
        if (rc != 1) return rc;
    }
    return lb_fail(LB_ERR_OOM, "sparse workspace sizing did not converge");
}
