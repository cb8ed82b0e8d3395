// Dense data preparation: Q = Q_H + Q_D and K from a Hamiltonian H and a dense
// Kossakowski matrix gamma (Sec. 2, Eqs. (13)-(15); Table 1 steps 2.1-2.5).
//
// Formulation used here (equivalent to contracting h and gamma with the
// nonzero f, d and z = f + i d of Eqs. (11)-(12)): with the Lindbladian
// written as
//     L(X) = sum_jk gamma_jk F_j X F_k + Z X + X Z^+,
//     Z = -i H - G/2,  G = sum_jk gamma_jk F_k F_j,
// each element is Q_sn = Tr(F_s L(F_n)) and K_s = Tr(F_s L(1))/N. The first
// term is evaluated through the realigned Kossakowski matrix
//     C(a,b,c,d) = sum_jk (F_j)_{ab} gamma_jk (F_k)_{cd},
// so that Tr(F_s F_j F_n F_k) gamma_jk summed over j,k is
//     sum_{abcd} (F_s)_{da} (F_n)_{bc} C(a,b,c,d).
// Because a pair generator has two nonzeros and a diagonal generator N, an
// element with s and n on two disjoint pairs needs exactly four C values,
// i.e. two 2x2 blocks of gamma (the structure constants' nonzero pattern is
// folded into this index arithmetic). Elements touching the diagonal use
// projections of gamma's D-rows onto diagonal positions (table Pt) and
// prefix sums over the diagonal, so the whole assembly is O(M^2) work.
//
// Kernels, in launch order:
//   k_pt       Pt[a][k] = sum_l w_l(a) gamma[D^l][k]              (N x M)
//   k_cdd      Cdd[a][c] = C(a,a,c,c)                              (N x N)
//   k_gtheta   G, Theta = sum_jk gamma_jk F_j F_k, Z, Lambda = L(1) (N x N)
//   k_expand   K_s = Tr(F_s Lambda)/N
//   k_fourset  Q[pair][pair] for disjoint pairs (the bulk: ~M^2 elements),
//              mirror half into a transposed scratch
//   k_mirror   transposes the mirror half into Q
//   k_pp_shared Q[pair][pair] for pairs sharing a vertex
//   k_drows    Q[D][pair]          (prefix sums over the diagonal)
//   k_dcols    Q[pair][D]
//   k_dd1/2    Q[D][D]
// gamma is read assuming exact Hermiticity: an entry may be read from
// either triangle, whichever keeps the wavefront's loads contiguous.
#include "lb_internal.h"

namespace {

constexpr double kR = 0.70710678118654752440;  // 1/sqrt(2)

struct GV {
    const double* g;    // gamma, M x M complex
    const double* Pt;   // N x M complex
    const double* Cdd;  // N x N complex
    int64_t M, P;
    int N;
};

__device__ __forceinline__ cd gam(const GV& v, int64_t r, int64_t c) { return cload(v.g, r * v.M + c); }

// 1/2 [SS - i s2 SA - i s1 AS - s1 s2 AA] for a 2x2 block of gamma between the
// pair of (a,b) (rows S/A) and the pair of (c,d) (cols S/A), s1 = sigma(a,b),
// s2 = sigma(c,d): the value of C(a,b,c,d) for a != b, c != d.
__device__ __forceinline__ cd blk_c(cd SS, cd SA, cd AS, cd AA, double s1, double s2) {
    cd r = cadd(cadd(SS, cmis(SA, s2)), cadd(cmis(AS, s1), cscale(AA, -s1 * s2)));
    return cscale(r, 0.5);
}

__device__ __forceinline__ double sgn(int a, int b) { return a < b ? 1.0 : -1.0; }

// C(a,b,c,d) in general position (reads gamma literally, row {a,b}).
__device__ cd chat(const GV& v, int a, int b, int c, int d) {
    const int N = v.N;
    const int64_t P = v.P;
    if (a != b) {
        const int64_t p1 = lb_upair(N, a, b);
        const double s1 = sgn(a, b);
        if (c != d) {
            const int64_t p2 = lb_upair(N, c, d);
            const double s2 = sgn(c, d);
            return blk_c(gam(v, p1, p2), gam(v, p1, P + p2), gam(v, P + p1, p2), gam(v, P + p1, P + p2), s1, s2);
        }
        // sum_j (F_j)_{ab} conj(Pt[c][j])
        cd x = cconj(cload(v.Pt, (int64_t)c * v.M + p1));
        cd y = cconj(cload(v.Pt, (int64_t)c * v.M + P + p1));
        return cscale(cadd(x, cmis(y, s1)), kR);
    }
    if (c != d) {
        const int64_t p2 = lb_upair(N, c, d);
        const double s2 = sgn(c, d);
        cd x = cload(v.Pt, (int64_t)a * v.M + p2);
        cd y = cload(v.Pt, (int64_t)a * v.M + P + p2);
        return cscale(cadd(x, cmis(y, s2)), kR);
    }
    return cload(v.Cdd, (int64_t)a * N + c);
}

// Accumulator for the four outputs (S|J row) x (S|J column) of a pair-pair
// element: a term e(d,a)_X e(b,c)_Y * val contributes (times 1/2)
//   SS: Re val, SJ: s_bc Im val, JS: s_da Im val, JJ: -s_da s_bc Re val.
struct Acc4 {
    double ss = 0, sa = 0, as = 0, aa = 0;
    __device__ __forceinline__ void add(double sda, double sbc, cd v) {
        ss += v.re;
        sa += sbc * v.im;
        as += sda * v.im;
        aa -= sda * sbc * v.re;
    }
};

// Accumulator for one pair column/row against a diagonal weight vector:
// a term e(b,c)_Y * val with Y = S (factor 1/sqrt2) or J (-i s 1/sqrt2).
__device__ __forceinline__ cd ecoef(int Y, double s, cd v) { return Y == 0 ? cscale(v, kR) : cscale(cmis(v, s), kR); }

// ---------------------------------------------------------------------------
// Pre-pass kernels
// ---------------------------------------------------------------------------

// Pt[a][k] = sum_l w_l(a) gamma[D^l][k]: w_l(a) = 1/sqrt(l(l+1)) for l > a,
// -a/sqrt(a(a+1)) for l = a, 0 otherwise -> a suffix sum over l per column k.
__global__ void k_pt(GV v, double* Pt) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= v.M) return;
    const int N = v.N;
    const int64_t D0 = 2 * v.P - 1;  // row of D^l is D0 + l
    cd S = cmk(0, 0);
    for (int a = N - 1; a >= 0; --a) {
        cd val = S;
        if (a >= 1) {
            const cd ga = gam(v, D0 + a, k);
            const double nrm = 1.0 / sqrt((double)a * (a + 1));
            val = cadd(val, cscale(ga, -(double)a * nrm));
            S = cadd(S, cscale(ga, nrm));
        }
        cstore(Pt, (int64_t)a * v.M + k, val);
    }
}

// Cdd[a][c] = sum_l' Pt[a][D^l'] w_l'(c)
__global__ void k_cdd(GV v, double* Cdd) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = v.N;
    if (t >= (int64_t)N * N) return;
    const int a = (int)(t / N), c = (int)(t % N);
    const int64_t D0 = 2 * v.P - 1;
    cd s = cmk(0, 0);
    for (int l = (c > 1 ? c : 1); l < N; ++l) s = cadd(s, cscale(cload(v.Pt, (int64_t)a * v.M + D0 + l), lb_wdiag(l, c)));
    cstore(Cdd, t, s);
}

// G_ac = sum_b C(b,c,a,b), Theta_ac = sum_b C(a,b,b,c);
// Z = -iH - G/2 and Lambda = Theta - G = L(1).
__global__ void k_gtheta(GV v, const double* H, double* Z, double* Lam) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = v.N;
    if (t >= (int64_t)N * N) return;
    const int a = (int)(t / N), c = (int)(t % N);
    cd G = cmk(0, 0), Th = cmk(0, 0);
    for (int b = 0; b < N; ++b) {
        G = cadd(G, chat(v, b, c, a, b));
        Th = cadd(Th, chat(v, a, b, b, c));
    }
    const cd h = cload(H, t);
    // -i h = (h.im, -h.re)
    cstore(Z, t, cmk(h.im - 0.5 * G.re, -h.re - 0.5 * G.im));
    cstore(Lam, t, csub(Th, G));
}

// ---------------------------------------------------------------------------
// Pair x pair block
// ---------------------------------------------------------------------------
// An element with row pair {u,v} (u < v) and column pair {x,y} (x < y) on four
// distinct vertices needs two 2x2 blocks of gamma: B1 between the pairs {u,x}
// and {v,y}, B2 between {u,y} and {v,x}. Grouping the elements by their vertex
// set {a < b < c < d}: its three pairings {ab|cd}, {ac|bd}, {ad|bc} give three
// blocks G1, G2, G3 of gamma (one of each Hermitian pair), and the six elements
// whose row and column pairs partition the set each use two of them. k_fourset
// gives every set to one lane (lanes along d: each block read and the three
// "direct" elements, whose column pair holds d, are contiguous in memory) and
// writes the three "mirror" elements (row pair holds d) transposed into a
// scratch matrix T; k_mirror moves them to their place with a tiled
// transpose. Every disjoint element is written once, gamma's blocks are read
// once each. Elements whose pairs share a vertex are O(N^3) and come from
// k_pp_shared.

// A 2x2 block of gamma between a row pair and a column pair: entries (S,S),
// (S,J), (J,S), (J,J).
struct Blk {
    cd ss, sa, as, aa;
};

__device__ __forceinline__ Blk blk_load(const GV& v, int64_t pr, int64_t pc) {
    return Blk{gam(v, pr, pc), gam(v, pr, v.P + pc), gam(v, v.P + pr, pc), gam(v, v.P + pr, v.P + pc)};
}

// The block between the column pair and the row pair (gamma is Hermitian).
__device__ __forceinline__ Blk blk_t(const Blk& b) { return Blk{cconj(b.ss), cconj(b.as), cconj(b.sa), cconj(b.aa)}; }

// Four outputs (S|J row) x (S|J column) of the disjoint element ({u,v}, {x,y})
// from B1 (pairs {u,x} x {v,y}) and B2 (pairs {u,y} x {v,x}).
__device__ __forceinline__ Acc4 pp_disjoint(int u, int vv, int x, int y, const Blk& B1, const Blk& B2) {
    // C(u,x,y,v) from B1; C(v,y,x,u) from B1^H; C(u,y,x,v) from B2; C(v,x,y,u) from B2^H
    const cd c_uxyv = blk_c(B1.ss, B1.sa, B1.as, B1.aa, sgn(u, x), sgn(y, vv));
    const cd c_vyxu = blk_c(cconj(B1.ss), cconj(B1.as), cconj(B1.sa), cconj(B1.aa), sgn(vv, y), sgn(x, u));
    const cd c_uyxv = blk_c(B2.ss, B2.sa, B2.as, B2.aa, sgn(u, y), sgn(x, vv));
    const cd c_vxyu = blk_c(cconj(B2.ss), cconj(B2.as), cconj(B2.sa), cconj(B2.aa), sgn(vv, x), sgn(y, u));
    // (d,a) = (u,v): s_da = +1; (v,u): -1. (b,c) = (x,y): +1; (y,x): -1. Term C(a,b,c,d).
    Acc4 acc;
    acc.add(+1, +1, c_vxyu);
    acc.add(+1, -1, c_vyxu);
    acc.add(-1, +1, c_uxyv);
    acc.add(-1, -1, c_uyxv);
    return acc;
}

__device__ __forceinline__ void pp_store(double* Q, int64_t ldq, int64_t P, int64_t rs, int64_t cn, const Acc4& acc) {
    __builtin_nontemporal_store(0.5 * acc.ss, Q + rs * ldq + cn);
    __builtin_nontemporal_store(0.5 * acc.sa, Q + rs * ldq + P + cn);
    __builtin_nontemporal_store(0.5 * acc.as, Q + (P + rs) * ldq + cn);
    __builtin_nontemporal_store(0.5 * acc.aa, Q + (P + rs) * ldq + P + cn);
}

// The element at Q[(rs, cn)] stored at T's transposed position: T[j][i] = Q[i][j].
__device__ __forceinline__ void pp_store_t(double* T, int64_t ldt, int64_t P, int64_t rs, int64_t cn, const Acc4& acc) {
    __builtin_nontemporal_store(0.5 * acc.ss, T + cn * ldt + rs);
    __builtin_nontemporal_store(0.5 * acc.sa, T + (P + cn) * ldt + rs);
    __builtin_nontemporal_store(0.5 * acc.as, T + cn * ldt + P + rs);
    __builtin_nontemporal_store(0.5 * acc.aa, T + (P + cn) * ldt + P + rs);
}

// Block (blockIdx.x = pair index of {a,b}, blockIdx.y = chunk of kFourChunk
// column pairs); lane q runs over the pairs {c,d} with b < c < d, which are the
// pair indices from p(b+1, b+2) to P-1.
constexpr int kFourChunk = 4096;

__global__ __launch_bounds__(256) void k_fourset(GV v, const int2* pairs, double* Q, int64_t ldq, double* T,
                                                 int64_t ldt) {
    const int64_t pab = blockIdx.x;
    const int a = pairs[pab].x, b = pairs[pab].y;
    const int N = v.N;
    if (b > N - 3) return;
    const int64_t P = v.P;
    const int64_t qb = lb_pair(N, b + 1, b + 2) + (int64_t)blockIdx.y * kFourChunk;
    const int64_t qe = qb + kFourChunk < P ? qb + kFourChunk : P;
    for (int64_t q = qb + threadIdx.x; q < qe; q += blockDim.x) {
        const int c = pairs[q].x, d = pairs[q].y;
        const int64_t pac = lb_pair(N, a, c), pbd = lb_pair(N, b, d);
        const int64_t pbc = lb_pair(N, b, c), pad = lb_pair(N, a, d);
        const Blk G1 = blk_load(v, pab, q);    // {a,b} x {c,d}
        const Blk G2 = blk_load(v, pac, pbd);  // {a,c} x {b,d}
        const Blk G3 = blk_load(v, pbc, pad);  // {b,c} x {a,d}
        const Blk G2t = blk_t(G2), G3t = blk_t(G3);
        pp_store(Q, ldq, P, pab, q, pp_disjoint(a, b, c, d, G2, G3t));
        pp_store(Q, ldq, P, pac, pbd, pp_disjoint(a, c, b, d, G1, G3t));
        pp_store(Q, ldq, P, pbc, pad, pp_disjoint(b, c, a, d, G1, G2t));
        pp_store_t(T, ldt, P, q, pab, pp_disjoint(c, d, a, b, G2, G3));
        pp_store_t(T, ldt, P, pbd, pac, pp_disjoint(b, d, a, c, G1, G3));
        pp_store_t(T, ldt, P, pad, pbc, pp_disjoint(a, d, b, c, G1, G2));
    }
}

// Q[i][j] = T[j][i] for i, j < 2P whose pairs are disjoint with the larger
// vertex in the row pair (the mirror elements). 64 x 64 tiles through LDS,
// 16-byte loads along T's rows and 16-byte stores along Q's rows; the tile's
// row and column pairs are read once into LDS. Tiles whose rows' largest
// vertex never exceeds its columns' smallest are skipped (ymax/ymin: per run
// of 64 indices).
constexpr int kMirrorTile = 64;

__global__ __launch_bounds__(256) void k_mirror(const double* T, int64_t ldt, const int2* pairs, const int* ymin,
                                                const int* ymax, int64_t P, double* Q, int64_t ldq) {
    __shared__ double tile[kMirrorTile][kMirrorTile + 1];
    __shared__ int2 rp[kMirrorTile], cp[kMirrorTile];
    const int64_t ti = blockIdx.x, tj = blockIdx.y;  // row tile of Q, column tile of Q
    if (ymax[ti] <= ymin[tj]) return;
    const int64_t n2 = 2 * P;
    const int64_t i0 = ti * kMirrorTile, j0 = tj * kMirrorTile;
    const int t = threadIdx.x;
    if (t < kMirrorTile) {
        const int64_t i = i0 + t;
        rp[t] = i < n2 ? pairs[i < P ? i : i - P] : make_int2(-1, -1);
    } else if (t < 2 * kMirrorTile) {
        const int64_t j = j0 + t - kMirrorTile;
        cp[t - kMirrorTile] = j < n2 ? pairs[j < P ? j : j - P] : make_int2(-2, 1 << 30);  // never below a row pair
    }
    __syncthreads();
    // mirror element: disjoint pairs, larger vertex in the row pair; the padding
    // pairs (row: upper vertex -1, column: upper vertex 2^30) never qualify, so
    // nothing past row or column 2P - 1 of T or Q is touched
    auto mirror = [](int2 R, int2 C) { return R.x != C.x && R.x != C.y && R.y != C.x && R.y != C.y && R.y > C.y; };
    const int c2 = 2 * (t & 31), r0 = t >> 5;  // column pair within a row, first row
    // T rows j0.. (Q columns), two consecutive i per thread; only mirror elements
    // are loaded, so lines of T outside the mirror region are not fetched
    for (int r = r0; r < kMirrorTile; r += 8) {
        const int64_t j = j0 + r, i = i0 + c2;
        const int2 C = cp[r];
        const bool m0 = mirror(rp[c2], C), m1 = mirror(rp[c2 + 1], C);
        const double* src = T + j * ldt + i;
        double2 x = make_double2(0.0, 0.0);
        if (m0 && m1 && (((uintptr_t)src) & 15) == 0) {
            x = *reinterpret_cast<const double2*>(src);
        } else {
            if (m0) x.x = src[0];
            if (m1) x.y = src[1];
        }
        tile[r][c2] = x.x;
        tile[r][c2 + 1] = x.y;
    }
    __syncthreads();
    for (int r = r0; r < kMirrorTile; r += 8) {
        const int64_t i = i0 + r, j = j0 + c2;
        if (i >= n2 || j >= n2) continue;
        const int2 R = rp[r];
        const bool m0 = mirror(R, cp[c2]);
        const bool m1 = mirror(R, cp[c2 + 1]);
        double* q = Q + i * ldq + j;
        if (m0 && m1 && (((uintptr_t)q) & 15) == 0) {
            *reinterpret_cast<double2*>(q) = make_double2(tile[c2][r], tile[c2 + 1][r]);
        } else {
            if (m0) q[0] = tile[c2][r];
            if (m1) q[1] = tile[c2 + 1][r];
        }
    }
}

// Elements whose row pair {u,v} and column pair {x,y} share a vertex
// (including the diagonal element u = x, v = y): the general form.
__device__ __forceinline__ Acc4 pp_shared(const GV& v, const double* Zm, int u, int vv, int x, int y) {
    const int N = v.N;
    Acc4 acc;
    const int sv[2][2] = {{u, vv}, {vv, u}};  // (d, a)
    const int nv[2][2] = {{x, y}, {y, x}};    // (b, c)
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int d = sv[i][0], a = sv[i][1], b = nv[j][0], c = nv[j][1];
            acc.add(sgn(d, a), sgn(b, c), chat(v, a, b, c, d));
        }
    // Tr(F_s Z F_n): shared vertex d, a = s\d, b = n\d: e(d,a) Z_ab e(b,d)
    // Tr(F_s F_n Z^+): shared vertex a, d = s\a, b = n\a: e(d,a) conj(Z_db) e(a,b)
    const int sv2[2] = {u, vv}, nv2[2] = {x, y};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            if (sv2[i] != nv2[j]) continue;
            const int wv = sv2[i], so = sv2[1 - i], no = nv2[1 - j];
            acc.add(sgn(wv, so), sgn(no, wv), cload(Zm, (int64_t)so * N + no));
            acc.add(sgn(so, wv), sgn(wv, no), cconj(cload(Zm, (int64_t)so * N + no)));
        }
    return acc;
}

__device__ __forceinline__ void pp_store_plain(double* Q, int64_t ldq, int64_t P, int64_t rs, int64_t cn,
                                               const Acc4& acc) {
    Q[rs * ldq + cn] = 0.5 * acc.ss;
    Q[rs * ldq + P + cn] = 0.5 * acc.sa;
    Q[(P + rs) * ldq + cn] = 0.5 * acc.as;
    Q[(P + rs) * ldq + P + cn] = 0.5 * acc.aa;
}

// Elements of pairs sharing a vertex, grouped by vertex set {a<b<c}: its
// pairs ab, ac, bc give the six off-diagonal elements, which read the same
// three gamma blocks and Pt entries. One wavefront per pair {a,b}, lanes
// along c; lane 0 also writes the pair's diagonal element. All six values
// are formed before any store, so repeated reads need not be issued twice.
__global__ __launch_bounds__(256) void k_pp_shared(GV v, const double* Zm, const int2* pairs, double* Q,
                                                   int64_t ldq) {
    const int N = v.N;
    const int64_t P = v.P;
    const int64_t pab = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (pab >= P) return;
    const int a = pairs[pab].x, b = pairs[pab].y;
    if (lane == 0) pp_store_plain(Q, ldq, P, pab, pab, pp_shared(v, Zm, a, b, a, b));
    for (int c = b + 1 + lane; c < N; c += 64) {
        const int64_t pac = lb_pair(N, a, c), pbc = lb_pair(N, b, c);
        const Acc4 e1 = pp_shared(v, Zm, a, b, a, c), e2 = pp_shared(v, Zm, a, b, b, c);
        const Acc4 e3 = pp_shared(v, Zm, a, c, a, b), e4 = pp_shared(v, Zm, a, c, b, c);
        const Acc4 e5 = pp_shared(v, Zm, b, c, a, b), e6 = pp_shared(v, Zm, b, c, a, c);
        pp_store_plain(Q, ldq, P, pab, pac, e1);
        pp_store_plain(Q, ldq, P, pab, pbc, e2);
        pp_store_plain(Q, ldq, P, pac, pab, e3);
        pp_store_plain(Q, ldq, P, pac, pbc, e4);
        pp_store_plain(Q, ldq, P, pbc, pab, e5);
        pp_store_plain(Q, ldq, P, pbc, pac, e6);
    }
}

// ---------------------------------------------------------------------------
// Rows of the diagonal generators: Q[D^m][n] = sum_a w_m(a) (L(F_n))_aa
// ---------------------------------------------------------------------------

// One thread per pair (x, y) -> columns S(x,y) and J(x,y). The diagonal of
// L(F_n) is accumulated along a with a running prefix sum, which gives all
// N-1 rows D^m (w_m(a) = 1/sqrt(m(m+1)) for a < m, -m/sqrt(m(m+1)) at a = m).
__global__ void k_drows(GV v, const double* Zm, const int2* pairs, double* Q, int64_t ldq) {
    const int64_t pn = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t P = v.P;
    if (pn >= P) return;
    const int N = v.N;
    const int x = pairs[pn].x, y = pairs[pn].y;
    const cd zxy = cload(Zm, (int64_t)x * N + y), zyx = cload(Zm, (int64_t)y * N + x);
    cd preS = cmk(0, 0), preA = cmk(0, 0);
    for (int a = 0; a < N; ++a) {
        cd c1, c2;  // C(a,x,y,a), C(a,y,x,a)
        if (a != x && a != y) {
            const int64_t p_ax = lb_upair(N, a, x), p_ay = lb_upair(N, a, y);
            const cd ss = gam(v, p_ax, p_ay), sa = gam(v, p_ax, P + p_ay);
            const cd as = gam(v, P + p_ax, p_ay), aa = gam(v, P + p_ax, P + p_ay);
            c1 = blk_c(ss, sa, as, aa, sgn(a, x), sgn(y, a));
            c2 = blk_c(cconj(ss), cconj(as), cconj(sa), cconj(aa), sgn(a, y), sgn(x, a));
        } else {
            c1 = chat(v, a, x, y, a);
            c2 = chat(v, a, y, x, a);
        }
        // sum_{(b,c)} (F_n)_{bc} C(a,b,c,a): (x,y) has sigma +1, (y,x) has -1
        cd gS = cadd(ecoef(0, 1, c1), ecoef(0, -1, c2));
        cd gA = cadd(ecoef(1, 1, c1), ecoef(1, -1, c2));
        // (Z F_n)_aa + (F_n Z^+)_aa
        if (a == x) {
            gS = cadd(gS, cadd(ecoef(0, -1, zxy), ecoef(0, 1, cconj(zxy))));
            gA = cadd(gA, cadd(ecoef(1, -1, zxy), ecoef(1, 1, cconj(zxy))));
        } else if (a == y) {
            gS = cadd(gS, cadd(ecoef(0, 1, zyx), ecoef(0, -1, cconj(zyx))));
            gA = cadd(gA, cadd(ecoef(1, 1, zyx), ecoef(1, -1, cconj(zyx))));
        }
        if (a >= 1) {
            const double nrm = 1.0 / sqrt((double)a * (a + 1));
            const double* row = Q + (2 * P + a - 1) * ldq;
            const double qS = (preS.re - (double)a * gS.re) * nrm;
            const double qA = (preA.re - (double)a * gA.re) * nrm;
            __builtin_nontemporal_store(qS, const_cast<double*>(row) + pn);
            __builtin_nontemporal_store(qA, const_cast<double*>(row) + P + pn);
        }
        preS = cadd(preS, gS);
        preA = cadd(preA, gA);
    }
}

// ---------------------------------------------------------------------------
// Columns of the diagonal generators: Q[s][D^m] = sum_a w_m(a) (L^+(F_s))_aa
// with L^+(Y) = sum_jk gamma_jk F_k Y F_j + Z^+ Y + Y Z.
// ---------------------------------------------------------------------------

__global__ void k_dcols(GV v, const double* Zm, const int2* pairs, double* Q, int64_t ldq) {
    const int64_t ps = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t P = v.P;
    if (ps >= P) return;
    const int N = v.N;
    const int u = pairs[ps].x, w = pairs[ps].y;
    const cd zuw = cload(Zm, (int64_t)u * N + w), zwu = cload(Zm, (int64_t)w * N + u);
    double* rowS = Q + ps * ldq + 2 * P;
    double* rowA = Q + (P + ps) * ldq + 2 * P;
    cd preS = cmk(0, 0), preA = cmk(0, 0);
    for (int a = 0; a < N; ++a) {
        cd c1, c2;  // C(u,a,a,w) [(b,c) = (w,u)], C(w,a,a,u) [(b,c) = (u,w)]
        if (a != u && a != w) {
            const int64_t p_ua = lb_upair(N, u, a), p_wa = lb_upair(N, w, a);
            const cd ss = gam(v, p_ua, p_wa), sa = gam(v, p_ua, P + p_wa);
            const cd as = gam(v, P + p_ua, p_wa), aa = gam(v, P + p_ua, P + p_wa);
            c1 = blk_c(ss, sa, as, aa, sgn(u, a), sgn(a, w));
            c2 = blk_c(cconj(ss), cconj(as), cconj(sa), cconj(aa), sgn(w, a), sgn(a, u));
        } else {
            c1 = chat(v, u, a, a, w);
            c2 = chat(v, w, a, a, u);
        }
        // sum_{(b,c)} (F_s)_{bc} C(c,a,a,b): (b,c) = (u,w) sigma +1 -> C(w,a,a,u); (w,u) -1 -> C(u,a,a,w)
        cd hS = cadd(ecoef(0, 1, c2), ecoef(0, -1, c1));
        cd hA = cadd(ecoef(1, 1, c2), ecoef(1, -1, c1));
        // (F_s Z)_aa + (Z^+ F_s)_aa
        if (a == u) {
            hS = cadd(hS, cadd(ecoef(0, 1, zwu), ecoef(0, -1, cconj(zwu))));
            hA = cadd(hA, cadd(ecoef(1, 1, zwu), ecoef(1, -1, cconj(zwu))));
        } else if (a == w) {
            hS = cadd(hS, cadd(ecoef(0, -1, zuw), ecoef(0, 1, cconj(zuw))));
            hA = cadd(hA, cadd(ecoef(1, -1, zuw), ecoef(1, 1, cconj(zuw))));
        }
        if (a >= 1) {
            const double nrm = 1.0 / sqrt((double)a * (a + 1));
            rowS[a - 1] = (preS.re - (double)a * hS.re) * nrm;
            rowA[a - 1] = (preA.re - (double)a * hA.re) * nrm;
        }
        preS = cadd(preS, hS);
        preA = cadd(preA, hA);
    }
}

// ---------------------------------------------------------------------------
// Diagonal x diagonal block: (L(D^m'))_aa = sum_b C(a,b,b,a) w_m'(b) + 2 Re Z_aa w_m'(a)
// ---------------------------------------------------------------------------

__global__ void k_dd1(GV v, const double* Zm, double* T) {
    const int N = v.N;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)N * (N - 1)) return;
    const int a = (int)(t / (N - 1)), m2 = (int)(t % (N - 1)) + 1;
    cd s = cmk(0, 0);
    for (int b = 0; b <= m2; ++b) {
        cd r = chat(v, a, b, b, a);
        if (b == a) r.re += 2.0 * cload(Zm, (int64_t)a * N + a).re;
        s = cadd(s, cscale(r, lb_wdiag(m2, b)));
    }
    cstore(T, t, s);
}

__global__ void k_dd2(GV v, const double* T, double* Q, int64_t ldq) {
    const int N = v.N;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)(N - 1) * (N - 1)) return;
    const int m = (int)(t / (N - 1)) + 1, m2 = (int)(t % (N - 1)) + 1;
    double s = 0;
    for (int a = 0; a <= m; ++a) s += lb_wdiag(m, a) * cload(T, (int64_t)a * (N - 1) + (m2 - 1)).re;
    Q[(2 * v.P + m - 1) * ldq + 2 * v.P + m2 - 1] = s;
}

__global__ void k_zero_pad(double* Q, int64_t M, int64_t ldq) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = ldq - M;
    if (t >= M * w) return;
    Q[(t / w) * ldq + M + t % w] = 0.0;
}

// ---------------------------------------------------------------------------
// Expansion / reconstruction (Eqs. (6), (7))
// ---------------------------------------------------------------------------

// a[b][s] = scale * Re Tr(F_s A_b)
__global__ void k_expand(int N, int B, const double* A, double* out, double scale) {
    const int64_t M = (int64_t)N * N - 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * B) return;
    const int b = (int)(t / M);
    const int64_t s = t % M;
    const double* Ab = A + 2 * (int64_t)b * N * N;
    int cls, j, k;
    lb_decode(N, s, cls, j, k);
    double r;
    if (cls < 2) {
        // (F_s)_{jk} A_kj + (F_s)_{kj} A_jk
        const cd akj = cload(Ab, (int64_t)k * N + j), ajk = cload(Ab, (int64_t)j * N + k);
        r = cls == 0 ? kR * (akj.re + ajk.re) : kR * (akj.im - ajk.im);
    } else {
        r = 0;
        for (int x = 0; x <= j; ++x) r += lb_wdiag(j, x) * Ab[2 * ((int64_t)x * N + x)];
    }
    out[t] = scale * r;
}

// V[b][s] = <psi_b| F_s |psi_b>
__global__ void k_expand_pure(int N, int B, const double* psi, double* V) {
    const int64_t M = (int64_t)N * N - 1;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M * B) return;
    const int b = (int)(t / M);
    const int64_t s = t % M;
    const double* p = psi + 2 * (int64_t)b * N;
    int cls, j, k;
    lb_decode(N, s, cls, j, k);
    double r;
    if (cls < 2) {
        // z = conj(psi_j) psi_k; S: sqrt2 Re z, J: sqrt2 Im z
        const cd pj = cload(p, j), pk = cload(p, k);
        const cd z = cmul(cconj(pj), pk);
        r = (cls == 0 ? z.re : z.im) * (2.0 * kR);
    } else {
        r = 0;
        for (int x = 0; x <= j; ++x) {
            const cd px = cload(p, x);
            r += lb_wdiag(j, x) * (px.re * px.re + px.im * px.im);
        }
    }
    V[t] = r;
}

// rho_b = 1/N + sum_s V[b][s] F_s
__global__ void k_reconstruct(int N, int B, const double* V, double* rho) {
    const int64_t M = (int64_t)N * N - 1;
    const int64_t NN = (int64_t)N * N;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NN * B) return;
    const int b = (int)(t / NN);
    const int a = (int)((t % NN) / N), c = (int)(t % N);
    const double* v = V + (int64_t)b * M;
    const int64_t P = lb_npairs(N);
    cd r;
    if (a != c) {
        const int64_t p = lb_upair(N, a, c);
        const double vs = v[p], va = v[P + p];
        // S: 1/sqrt2; J: -i sigma(a,c)/sqrt2
        r = cmk(kR * vs, -sgn(a, c) * kR * va);
    } else {
        double s = 1.0 / N;
        for (int l = (a > 1 ? a : 1); l < N; ++l) s += v[2 * P + l - 1] * lb_wdiag(l, a);
        r = cmk(s, 0);
    }
    cstore(rho + 2 * (int64_t)b * NN, t % NN, r);
}

// per-block max |A_ij - conj(A_ji)| and max |A_ij| over an n x n complex matrix
__global__ void k_herm(int64_t n, const double* A, double* out) {
    __shared__ double sd[256], sa[256];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double dv = 0, av = 0;
    if (t < n * n) {
        const int64_t i = t / n, j = t % n;
        const cd x = cload(A, i * n + j), y = cload(A, j * n + i);
        dv = fmax(fabs(x.re - y.re), fabs(x.im + y.im));
        av = fmax(fabs(x.re), fabs(x.im));
    }
    sd[threadIdx.x] = dv;
    sa[threadIdx.x] = av;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + s]);
            sa[threadIdx.x] = fmax(sa[threadIdx.x], sa[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = sd[0];
        out[2 * blockIdx.x + 1] = sa[0];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

int lb_impl_expand(lb_ctx* c, int N, int B, const double* A, double* a, double scale) {
    const int64_t M = (int64_t)N * N - 1;
    hipLaunchKernelGGL(k_expand, dim3(lb_blocks(M * B, 256)), dim3(256), 0, c->stream, N, B, A, a, scale);
    LB_CHECK_LAUNCH();
    return LB_OK;
}

int lb_impl_expand_pure(lb_ctx* c, int N, int B, const double* psi, double* V) {
    const int64_t M = (int64_t)N * N - 1;
    hipLaunchKernelGGL(k_expand_pure, dim3(lb_blocks(M * B, 256)), dim3(256), 0, c->stream, N, B, psi, V);
    LB_CHECK_LAUNCH();
    return LB_OK;
}

int lb_impl_reconstruct(lb_ctx* c, int N, int B, const double* V, double* rho) {
    const int64_t NN = (int64_t)N * N;
    hipLaunchKernelGGL(k_reconstruct, dim3(lb_blocks(NN * B, 256)), dim3(256), 0, c->stream, N, B, V, rho);
    LB_CHECK_LAUNCH();
    return LB_OK;
}

int lb_impl_hermitian_check(lb_ctx* c, int64_t n, const double* A, double* maxdev, double* maxabs) {
    const unsigned nb = lb_blocks(n * n, 256);
    int rc = lb_ws_reserve(c, sizeof(double) * 2 * nb);
    if (rc) return rc;
    double* part = (double*)c->ws;
    hipLaunchKernelGGL(k_herm, dim3(nb), dim3(256), 0, c->stream, n, A, part);
    LB_CHECK_LAUNCH();
    rc = lb_host_reserve(c, sizeof(double) * 2 * nb);
    if (rc) return rc;
    double* h = (double*)c->host;
    LB_HIP(hipMemcpyAsync(h, part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost, c->stream));
    LB_HIP(hipStreamSynchronize(c->stream));
    double d = 0, a = 0;
    for (unsigned i = 0; i < nb; ++i) {
        d = d > h[2 * i] ? d : h[2 * i];
        a = a > h[2 * i + 1] ? a : h[2 * i + 1];
    }
    *maxdev = d;
    *maxabs = a;
    return LB_OK;
}

int lb_impl_prepare_dense(lb_ctx* c, int N, const double* H, const double* gamma, double* Q, int64_t ldq,
                          double* K) {
    const int64_t M = (int64_t)N * N - 1;
    const int64_t P = lb_npairs(N);
    // pair list, and per run of 64 pair-block indices (0..2P-1) the smallest and
    // largest upper vertex, for the mirror transpose's tile skipping
    const int64_t n2 = 2 * P;
    const int64_t nt = (n2 + kMirrorTile - 1) / kMirrorTile;
    const int64_t ldt = (n2 + 31) / 32 * 32;
    if (nt > 65535) return lb_fail(LB_ERR_UNSUPPORTED, "N=%d too large for the mirror grid", N);
    // workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = lb_align(off + bytes, 256);
        return o;
    };
    const size_t o_pt = take(sizeof(double) * 2 * (size_t)N * M);
    const size_t o_cdd = take(sizeof(double) * 2 * (size_t)N * N);
    const size_t o_z = take(sizeof(double) * 2 * (size_t)N * N);
    const size_t o_lam = take(sizeof(double) * 2 * (size_t)N * N);
    const size_t o_t = take(sizeof(double) * 2 * (size_t)N * N);
    const size_t o_pairs = take(sizeof(int2) * (size_t)P + sizeof(int) * 2 * (size_t)nt + 8);  // pairs, ymin, ymax
    const size_t o_mt = take(sizeof(double) * (size_t)n2 * ldt);
    int rc = lb_ws_reserve(c, off);
    if (rc) return rc;
    const size_t hb = sizeof(int2) * P + sizeof(int) * 2 * nt;
    rc = lb_host_reserve(c, hb);
    if (rc) return rc;
    char* ws = (char*)c->ws;
    int2* h = (int2*)c->host;
    // the pinned staging buffer may still be read by an earlier copy on this stream
    LB_HIP(hipStreamSynchronize(c->stream));
    int64_t hp = 0;
    for (int a = 0; a + 1 < N; ++a)
        for (int b = a + 1; b < N; ++b) h[hp++] = make_int2(a, b);
    int* hy = (int*)(h + P);
    for (int64_t t = 0; t < nt; ++t) {
        int lo = N, hi = -1;
        for (int64_t i = kMirrorTile * t; i < kMirrorTile * (t + 1) && i < n2; ++i) {
            const int y = h[i < P ? i : i - P].y;
            lo = y < lo ? y : lo;
            hi = y > hi ? y : hi;
        }
        hy[t] = lo;
        hy[nt + t] = hi;
    }
    LB_HIP(hipMemcpyAsync(ws + o_pairs, h, hb, hipMemcpyHostToDevice, c->stream));

    GV v;
    v.g = gamma;
    v.Pt = (const double*)(ws + o_pt);
    v.Cdd = (const double*)(ws + o_cdd);
    v.M = M;
    v.P = P;
    v.N = N;
    double* Zm = (double*)(ws + o_z);
    double* Lam = (double*)(ws + o_lam);
    double* T = (double*)(ws + o_t);
    const int2* pd = (const int2*)(ws + o_pairs);
    const int* ymin = (const int*)(ws + o_pairs + sizeof(int2) * P);
    const int* ymax = ymin + nt;
    double* MT = (double*)(ws + o_mt);
    hipStream_t s = c->stream;

    hipLaunchKernelGGL(k_pt, dim3(lb_blocks(M, 256)), dim3(256), 0, s, v, (double*)(ws + o_pt));
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_cdd, dim3(lb_blocks((int64_t)N * N, 256)), dim3(256), 0, s, v, (double*)(ws + o_cdd));
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_gtheta, dim3(lb_blocks((int64_t)N * N, 64)), dim3(64), 0, s, v, H, Zm, Lam);
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_expand, dim3(lb_blocks(M, 256)), dim3(256), 0, s, N, 1, (const double*)Lam, K, 1.0 / N);
    LB_CHECK_LAUNCH();
    if (P > 0) {
        if (N >= 4) {
            hipLaunchKernelGGL(k_fourset, dim3((unsigned)P, (unsigned)((P + kFourChunk - 1) / kFourChunk)), dim3(256),
                               0, s, v, pd, Q, ldq, MT, ldt);
            LB_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_mirror, dim3((unsigned)nt, (unsigned)nt), dim3(256), 0, s, (const double*)MT, ldt, pd,
                               ymin, ymax, P, Q, ldq);
            LB_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_pp_shared, dim3(lb_blocks(P * 64, 256)), dim3(256), 0, s, v, (const double*)Zm, pd, Q,
                           ldq);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_drows, dim3(lb_blocks(P, 64)), dim3(64), 0, s, v, (const double*)Zm, pd, Q, ldq);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_dcols, dim3(lb_blocks(P, 64)), dim3(64), 0, s, v, (const double*)Zm, pd, Q, ldq);
        LB_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_dd1, dim3(lb_blocks((int64_t)N * (N - 1), 64)), dim3(64), 0, s, v, (const double*)Zm, T);
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_dd2, dim3(lb_blocks((int64_t)(N - 1) * (N - 1), 64)), dim3(64), 0, s, v,
                       (const double*)T, Q, ldq);
    LB_CHECK_LAUNCH();
    if (ldq > M) {
        hipLaunchKernelGGL(k_zero_pad, dim3(lb_blocks(M * (ldq - M), 256)), dim3(256), 0, s, Q, M, ldq);
        LB_CHECK_LAUNCH();
    }
    return LB_OK;
}
