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
//   k_gth_a/c  partial sums over chunks of b of G and Theta from the 2x2
//              gamma blocks of pairs sharing a vertex (coalesced along a or c)
//   k_gth_fin  G, Theta, Z = -iH - G/2, Lambda = L(1)               (N x N)
//   k_expand   K_s = Tr(F_s Lambda)/N
//   then, concurrently on two streams:
//   k_quad     Q[pair][pair] for disjoint pairs (the bulk: ~M^2 elements) and
//              the shared-vertex elements inside the segments it owns; one
//              workgroup per pair (a, c) reads gamma at exactly the positions
//              of Q it writes, so gamma is read once and Q written once
//   k_segpp    shared-vertex elements in a row pair's own-vertex segments
//   k_drows    Q[D][pair]          (prefix sums over the diagonal)
//   k_dcols    Q[pair][D]
//   k_dd1/2    Q[D][D]
//   k_zero_pad the padding columns of Q
// gamma is read assuming exact Hermiticity: an entry may be read from
// either triangle, whichever keeps the wavefront's loads contiguous.
#include <algorithm>
#include <vector>

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

// ---------------------------------------------------------------------------
// Pair x pair elements
// ---------------------------------------------------------------------------
// An element with row pair {u,v} (u < v) and column pair {x,y} (x < y) on four
// distinct vertices needs two 2x2 blocks of gamma: B1 between the pairs {u,x}
// and {v,y}, B2 between {u,y} and {v,x}.

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
// from B1 (pairs {u,x} x {v,y}) and B2 (pairs {u,y} x {v,x}). The vertex order
// is fixed at each call site, so the signs are template arguments:
// S1 = sigma(u,x), S2 = sigma(y,v), T1 = sigma(u,y), T2 = sigma(x,v).
template <int S1, int S2, int T1, int T2>
__device__ __forceinline__ Acc4 pp_disjoint(const Blk& B1, const Blk& B2) {
    // C(u,x,y,v) from B1; C(v,y,x,u) from B1^H; C(u,y,x,v) from B2; C(v,x,y,u) from B2^H
    const cd c_uxyv = blk_c(B1.ss, B1.sa, B1.as, B1.aa, S1, S2);
    const cd c_vyxu = blk_c(cconj(B1.ss), cconj(B1.as), cconj(B1.sa), cconj(B1.aa), -S2, -S1);
    const cd c_uyxv = blk_c(B2.ss, B2.sa, B2.as, B2.aa, T1, T2);
    const cd c_vxyu = blk_c(cconj(B2.ss), cconj(B2.as), cconj(B2.sa), cconj(B2.aa), -T2, -T1);
    // (d,a) = (u,v): s_da = +1; (v,u): -1. (b,c) = (x,y): +1; (y,x): -1. Term C(a,b,c,d).
    Acc4 acc;
    acc.add(+1, +1, c_vxyu);
    acc.add(+1, -1, c_vyxu);
    acc.add(-1, +1, c_uxyv);
    acc.add(-1, -1, c_uyxv);
    return acc;
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

// ---------------------------------------------------------------------------
// G and Theta from the blocks of pairs that share a vertex
// ---------------------------------------------------------------------------
// G_ac = sum_b C(b,c,a,b) and Theta_ca = sum_b C(c,b,b,a). For b outside {a,c}
// both terms come from one 2x2 block of gamma, beta = gamma[{b,c}][{a,b}] (rows:
// pair {b,c}; columns: pair {a,b}), read in whichever orientation keeps a
// wavefront's loads contiguous:
//   b < a            beta itself: row {b,c} fixed per c, columns p(b,a) along a
//   a < b < c        beta = (gamma[{a,b}][{b,c}])^H: row p(a,b), columns p(b,c) along c
//   b > max(a,c)     beta itself (strided: columns p(a,b) of different segments)
// k_gth_a (lanes along a) takes the first and last ranges, k_gth_c (lanes along
// c) the middle one; both split b into chunks of kGthChunk and write one partial
// sum per chunk; k_gth_fin adds the chunks in order of b, then the b = a and
// b = c terms. Partial layout: Gp[k][a][c] (G_ac), Tp[k][x][y] (Theta_xy).
constexpr int kGthChunk = 16;

__device__ __forceinline__ void gth_add(cd& g, cd& th, const Blk& B, int a, int b, int c) {
    g = cadd(g, blk_c(B.ss, B.sa, B.as, B.aa, sgn(b, c), sgn(a, b)));
    th = cadd(th, blk_c(B.ss, B.sa, B.as, B.aa, sgn(c, b), sgn(b, a)));
}

__global__ void k_gth_a(GV v, double* Gp, double* Tp) {
    const int N = v.N;
    const int64_t NN = (int64_t)N * N;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NN) return;
    const int a = (int)(t % N), c = (int)(t / N);
    const int b0 = (int)blockIdx.y * kGthChunk, b1 = min(N, b0 + kGthChunk);
    const int hi = a > c ? a : c;
    cd g = cmk(0, 0), th = cmk(0, 0);
    for (int b = b0; b < b1; ++b) {
        if (b == a || b == c || (b > a && b < hi)) continue;
        gth_add(g, th, blk_load(v, lb_upair(N, b, c), lb_upair(N, a, b)), a, b, c);
    }
    const int64_t k = blockIdx.y;
    cstore(Gp, k * NN + (int64_t)a * N + c, g);
    cstore(Tp, k * NN + (int64_t)c * N + a, th);
}

__global__ void k_gth_c(GV v, double* Gp, double* Tp) {
    const int N = v.N;
    const int64_t NN = (int64_t)N * N;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NN) return;
    const int c = (int)(t % N), a = (int)(t / N);
    const int k0 = (int)blockIdx.y * kGthChunk;
    const int b0 = max(k0, a + 1), b1 = min(min(N, k0 + kGthChunk), c);
    cd g = cmk(0, 0), th = cmk(0, 0);
    for (int b = b0; b < b1; ++b)
        gth_add(g, th, blk_t(blk_load(v, lb_pair(N, a, b), lb_pair(N, b, c))), a, b, c);
    const int64_t k = blockIdx.y;
    cstore(Gp, k * NN + (int64_t)a * N + c, g);
    cstore(Tp, k * NN + (int64_t)c * N + a, th);
}

// Z = -iH - G/2 and Lambda = Theta - G = L(1).
__global__ void k_gth_fin(GV v, const double* H, const double* GpA, const double* TpA, const double* GpC,
                          const double* TpC, int nch, double* Z, double* Lam) {
    const int N = v.N;
    const int64_t NN = (int64_t)N * N;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NN) return;
    const int a = (int)(t / N), c = (int)(t % N);
    cd G = cmk(0, 0), Th = cmk(0, 0);
    for (int k = 0; k < nch; ++k) {
        G = cadd(G, cadd(cload(GpA, k * NN + t), cload(GpC, k * NN + t)));
        Th = cadd(Th, cadd(cload(TpA, k * NN + t), cload(TpC, k * NN + t)));
    }
    if (a == c) {
        G = cadd(G, chat(v, a, a, a, a));
        Th = cadd(Th, chat(v, a, a, a, a));
    } else {
        G = cadd(G, chat(v, a, c, a, a));   // b = a
        G = cadd(G, chat(v, c, c, a, c));   // b = c
        Th = cadd(Th, chat(v, a, a, a, c));  // b = a
        Th = cadd(Th, chat(v, a, c, c, c));  // b = c
    }
    const cd h = cload(H, t);
    cstore(Z, t, cmk(h.im - 0.5 * G.re, -h.re - 0.5 * G.im));
    cstore(Lam, t, csub(Th, G));
}

// ---------------------------------------------------------------------------
// Pair x pair elements by whole row segments
// ---------------------------------------------------------------------------
// Segment w of pair row {x<y} is the run of columns p(w, z), z > w (in both the
// S and the J column blocks). Workgroup (a, c), a < c, computes and writes these
// segments whole:
//   R  rows {w,c}, a < w < c, segment a: R[w][w'] = Q[{w,c}][{a,w'}] for w' in
//      (a, c) (w' = w is a shared-vertex element), then w' = c (shared vertex)
//      and w' > c;
//   S  row {a,c}, segments x, a < x < c: S[x][z] = Q[{a,c}][{x,z}] for z in
//      (x, c), then z = c (shared vertex) and z > c;
//   T  rows {a,x}, a < x < c, segment c: Q[{a,x}][{c,d}], d > c.
// A vertex set {a < x < z < c} gives R[z][x], R[x][z] and S[x][z], each from
// the gamma blocks at the same three positions (read transposed: gamma is
// Hermitian); a set {a < x < c < d} gives the d-th entries of T, of S's
// segment x and of R's row {x,c}, from the blocks at those positions. Every
// disjoint block of gamma is read once in each orientation, and every segment
// is produced by one workgroup, so Q's lines are written whole except where a
// segment starts or ends inside a line (the rest of that line belongs to the
// neighbouring segment, written by another workgroup). The shared-vertex
// elements outside these segments (segments x and y of row {x,y}) come from
// k_segpp.
//
// The square R is processed in 16 x 16 tiles (x block X, z block Z, X <= Z);
// block boundaries are placed so that a block's columns in segment a start a
// 128-byte line of Q. The transposed tile R[z][x] goes through LDS, and so does
// row {a,c}, whose segments are not aligned with the tiles: per x row a window
// of two lines collects the tile's values and each complete line is written
// at once. The sets {a < x < c < d} of an x block follow its tiles (lanes along
// d), so that the S and R segments end right after their tiles.
constexpr int kQuadPad = 17;

// Pair position in 32-bit arithmetic (the dense path holds M^2 complex values,
// so N stays far below the 46341 where P would leave int).
__device__ __forceinline__ int qpair(int N, int j, int k) { return j * N - ((j * (j + 1)) >> 1) + k - j - 1; }

// Block loads and output stores with the J offsets of gamma and Q precomputed.
struct QuadPtr {
    const double* g;  // gamma
    double* Q;
    int64_t M;        // gamma row length (complex entries)
    int64_t gjr;      // doubles from a gamma S row to the J row of the same pair
    int64_t ldq;
    int64_t qjr;      // doubles from a Q S row to the J row of the same pair
    int P;
};

__device__ __forceinline__ Blk quad_blk(const QuadPtr& w, int pr, int pc) {
    const double* p = w.g + 2 * ((int64_t)pr * w.M + pc);
    const int oc = 2 * w.P;
    return Blk{cload(p, 0), cload(p + oc, 0), cload(p + w.gjr, 0), cload(p + w.gjr + oc, 0)};
}

__device__ __forceinline__ void quad_put(const QuadPtr& w, int rs, int cn, const Acc4& acc) {
    double* q = w.Q + (int64_t)rs * w.ldq + cn;
    q[0] = 0.5 * acc.ss;
    q[w.P] = 0.5 * acc.sa;
    q[w.qjr] = 0.5 * acc.as;
    q[w.qjr + w.P] = 0.5 * acc.aa;
}

__device__ __forceinline__ void quad_stage_put(double (*hb)[16][kQuadPad], int tx, int tz, const Blk& B) {
    hb[0][tx][tz] = B.ss.re; hb[1][tx][tz] = B.ss.im;
    hb[2][tx][tz] = B.sa.re; hb[3][tx][tz] = B.sa.im;
    hb[4][tx][tz] = B.as.re; hb[5][tx][tz] = B.as.im;
    hb[6][tx][tz] = B.aa.re; hb[7][tx][tz] = B.aa.im;
}

__device__ __forceinline__ Blk quad_stage_get(double (*hb)[16][kQuadPad], int zl, int xl) {
    return Blk{cmk(hb[0][zl][xl], hb[1][zl][xl]), cmk(hb[2][zl][xl], hb[3][zl][xl]),
               cmk(hb[4][zl][xl], hb[5][zl][xl]), cmk(hb[6][zl][xl], hb[7][zl][xl])};
}

// One workgroup per pair (a, c) of the work order (entries with a < 0 pad the
// order to whole groups). Latency is hidden by occupancy rather than by
// register prefetch: one LDS buffer per tile, two barriers per tile.
__global__ __launch_bounds__(256) void k_quad(GV v, const double* Zm, const int2* order, double* Q, int64_t ldq) {
    __shared__ double h[8][16][kQuadPad];  // gamma blocks at positions R[z][x], staged [z][x]
    __shared__ double e[4][16][kQuadPad];  // outputs R[z][x], staged [z][x]
    __shared__ double sb[4][16][33];       // line windows of the S row, one per x of the block
    const int a = order[blockIdx.x].x, c = order[blockIdx.x].y;
    if (a < 0) return;
    const int L = c - a - 1;
    if (L <= 0) return;
    const int N = v.N;
    QuadPtr w;
    w.g = v.g;
    w.Q = Q;
    w.M = v.M;
    w.gjr = 2 * v.P * v.M;
    w.ldq = ldq;
    w.qjr = v.P * ldq;
    w.P = (int)v.P;
    const int base = qpair(N, a, a + 1);  // column of segment a's first entry
    const int r0 = base & 15;
    const int J = (L + r0 + 15) >> 4;
    const int pac = qpair(N, a, c);
    const int t = threadIdx.x;
    const int tx = t >> 4, tz = t & 15;
    for (int jx = 0; jx < J; ++jx) {
        const int ox = 16 * jx - r0 + tx;   // x offset of this thread's sets
        const int ox2 = 16 * jx - r0 + tz;  // x offset of its staging role
        // S[x][z] sits at column scol0 + oz of row {a,c}. Each x row of the block
        // has a window of 32 slots in LDS, slot k = column sline + k with sline a
        // multiple of 16: a tile's 16 values land in slots sphi .. sphi + 15, slots
        // 0..15 (one whole 128-byte line) are written out after the tile and slots
        // 16..31 carried to the next tile.
        const int scol0 = qpair(N, a + 1 + ox, a + 2 + ox) - ox - 1;
        const int ct = scol0 + 16 * jx - r0;
        const int sphi = ((ct % 16) + 16) % 16;
        int sline = ct - sphi;
        for (int jz = jx; jz < J; ++jz) {
            const int oz = 16 * jz - r0 + tz, oz2 = 16 * jz - r0 + tx;
            const bool own = ox >= 0 && oz < L && ox < oz;
            const bool stg = ox2 >= 0 && oz2 < L && ox2 < oz2;
            Blk h2, h3;
            const int x = a + 1 + ox, z = a + 1 + oz;
            const int pxc = ox >= 0 && ox < L ? qpair(N, x, c) : 0;
            if (own) {
                h2 = quad_blk(w, pxc, base + oz);
                h3 = quad_blk(w, pac, qpair(N, x, z));
            }
            if (stg) quad_stage_put(h, tx, tz, quad_blk(w, qpair(N, a + 1 + oz2, c), base + ox2));
            __syncthreads();
            if (own) {
                const Blk G1 = blk_t(quad_stage_get(h, tz, tx)), G2 = blk_t(h2), G3 = blk_t(h3);
                const Acc4 e4 = pp_disjoint<-1, 1, -1, 1>(G2, G3);  // R[z][x]: ({z,c}, {a,x})
                e[0][tz][tx] = e4.ss; e[1][tz][tx] = e4.sa; e[2][tz][tx] = e4.as; e[3][tz][tx] = e4.aa;
                quad_put(w, pxc, base + oz, pp_disjoint<-1, 1, 1, 1>(G1, G3));  // R[x][z]: ({x,c}, {a,z})
                const Acc4 sv = pp_disjoint<1, 1, 1, 1>(G1, G2);  // S[x][z]: ({a,c}, {x,z})
                const int k = sphi + tz;
                sb[0][tx][k] = sv.ss; sb[1][tx][k] = sv.sa; sb[2][tx][k] = sv.as; sb[3][tx][k] = sv.aa;
            } else if (ox >= 0 && ox == oz && oz < L) {
                quad_put(w, pxc, base + ox, pp_shared(v, Zm, x, c, a, x));  // R[x][x]: ({x,c}, {a,x})
            }
            __syncthreads();
            if (stg) {
                const Acc4 r{e[0][tx][tz], e[1][tx][tz], e[2][tx][tz], e[3][tx][tz]};
                quad_put(w, qpair(N, a + 1 + oz2, c), base + ox2, r);  // R[z][x]
            }
            {
                const int oz3 = sline - scol0 + tz;
                if (ox >= 0 && ox < oz3 && oz3 < L)
                    quad_put(w, pac, sline + tz, Acc4{sb[0][tx][tz], sb[1][tx][tz], sb[2][tx][tz], sb[3][tx][tz]});
#pragma unroll
                for (int q = 0; q < 4; ++q) sb[q][tx][tz] = sb[q][tx][16 + tz];
                sline += 16;
            }
        }
        {  // the carried part of each S line
            const int oz3 = sline - scol0 + tz;
            if (ox >= 0 && ox < oz3 && oz3 < L)
                quad_put(w, pac, sline + tz, Acc4{sb[0][tx][tz], sb[1][tx][tz], sb[2][tx][tz], sb[3][tx][tz]});
        }
        // sets {a < x < c < d} of this x block and the shared-vertex entries at
        // d = c, items (x, d) flattened over the workgroup, lanes along d
        const int lo = max(0, 16 * jx - r0), hi = min(L, 16 * jx - r0 + 16);
        const int nd = N - c;
        const int nitems = (hi - lo) * nd;
        for (int i = t; i < nitems; i += 256) {
            const int xi = i / nd;
            const int x = a + 1 + lo + xi, d = c + (i - xi * nd);
            const int pxc = qpair(N, x, c);
            if (d == c) {
                quad_put(w, pac, pxc, pp_shared(v, Zm, a, c, x, c));  // ({a,c}, {x,c})
                quad_put(w, pxc, pac, pp_shared(v, Zm, x, c, a, c));  // ({x,c}, {a,c})
                continue;
            }
            const int pax = qpair(N, a, x), pcd = qpair(N, c, d), pxd = qpair(N, x, d), pad = qpair(N, a, d);
            const Blk G1 = quad_blk(w, pax, pcd);  // {a,x} x {c,d}
            const Blk G2 = quad_blk(w, pac, pxd);  // {a,c} x {x,d}
            const Blk G3 = quad_blk(w, pxc, pad);  // {x,c} x {a,d}
            const Blk G2t = blk_t(G2), G3t = blk_t(G3);
            quad_put(w, pax, pcd, pp_disjoint<1, -1, 1, -1>(G2, G3t));  // ({a,x}, {c,d})
            quad_put(w, pac, pxd, pp_disjoint<1, -1, 1, 1>(G1, G3t));   // ({a,c}, {x,d})
            quad_put(w, pxc, pad, pp_disjoint<-1, -1, 1, 1>(G1, G2t));  // ({x,c}, {a,d})
        }
    }
}

// C(a,b,c,d) where the pairs {u,vv} (= s) and {x,y} (= n) share a vertex and
// sn = gamma[s][n]: block terms from sn or its transpose, diagonal terms (the
// projections Pt) as in chat.
__device__ __forceinline__ cd chat_pre(const GV& v, int a, int b, int c, int d, int u, int vv, const Blk& sn) {
    if (a != b && c != d) {
        const bool rows_s = (a == u && b == vv) || (a == vv && b == u);
        const Blk B = rows_s ? sn : blk_t(sn);
        return blk_c(B.ss, B.sa, B.as, B.aa, sgn(a, b), sgn(c, d));
    }
    return chat(v, a, b, c, d);
}

// pp_shared with the gamma block of (row pair, column pair) already loaded.
__device__ __forceinline__ Acc4 pp_shared_pre(const GV& v, const double* Zm, int u, int vv, int x, int y,
                                              const Blk& sn) {
    const int N = v.N;
    Acc4 acc;
    const int sv[2][2] = {{u, vv}, {vv, u}};  // (d, a)
    const int nv[2][2] = {{x, y}, {y, x}};    // (b, c)
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int d = sv[i][0], a = sv[i][1], b = nv[j][0], c = nv[j][1];
            acc.add(sgn(d, a), sgn(b, c), chat_pre(v, a, b, c, d, u, vv, sn));
        }
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

// Segments x and y of pair row {x,y}: the elements whose column pair shares a
// vertex with the row pair (and the diagonal element). One wavefront per row
// pair, lanes along the column pair's second vertex.
__global__ __launch_bounds__(256) void k_segpp(GV v, const double* Zm, const int2* pairs, double* Q, int64_t ldq) {
    const int N = v.N;
    const int64_t P = v.P;
    const int64_t ps = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (ps >= P) return;
    const int x = pairs[ps].x, y = pairs[ps].y;
    for (int z = x + 1 + lane; z < N; z += 64) {
        const int64_t pn = lb_pair(N, x, z);
        pp_store_plain(Q, ldq, P, ps, pn, pp_shared_pre(v, Zm, x, y, x, z, blk_load(v, ps, pn)));
    }
    for (int z = y + 1 + lane; z < N; z += 64) {
        const int64_t pn = lb_pair(N, y, z);
        pp_store_plain(Q, ldq, P, ps, pn, pp_shared_pre(v, Zm, x, y, y, z, blk_load(v, ps, pn)));
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

// Launch order of k_quad's workgroups (a, c): consecutive c of one a are
// grouped (kQuadGroup at a time) and dispatched together on one XCD (block i
// runs on XCD i mod 8), so that the segment boundaries they share are written
// at about the same time; groups go to the XCDs largest first, each to the
// least loaded one. Unused slots hold (-1, -1).
constexpr int kQuadGroup = 8;

static int64_t quad_order(int N, std::vector<int2>& out) {
    struct Group {
        int a, c0, c1;
        double w;
    };
    std::vector<Group> groups;
    for (int a = 0; a + 2 < N; ++a)
        for (int c0 = a + 2; c0 < N; c0 += kQuadGroup) {
            const int c1 = std::min(N, c0 + kQuadGroup);
            double w = 0;
            for (int cc = c0; cc < c1; ++cc) {
                const double L = cc - a - 1;
                w += L * (N - cc - 1) + 0.5 * L * (L + 1) + 1.0;
            }
            groups.push_back(Group{a, c0, c1, w});
        }
    std::stable_sort(groups.begin(), groups.end(), [](const Group& x, const Group& y) { return x.w > y.w; });
    std::vector<std::vector<int2>> lists(8);
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (const Group& g : groups) {
        int best = 0;
        for (int k = 1; k < 8; ++k)
            if (load[k] < load[best]) best = k;
        load[best] += g.w;
        for (int cc = g.c0; cc < g.c1; ++cc) lists[best].push_back(make_int2(g.a, cc));
    }
    size_t per = 0;
    for (auto& l : lists) per = std::max(per, l.size());
    out.assign(8 * per, make_int2(-1, -1));
    for (int k = 0; k < 8; ++k)
        for (size_t j = 0; j < lists[k].size(); ++j) out[8 * j + k] = lists[k][j];
    return (int64_t)out.size();
}

int lb_aux_stream(lb_ctx* c) {
    if (c->aux) return LB_OK;
    LB_HIP(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    LB_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    LB_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    return LB_OK;
}

int lb_impl_prepare_dense(lb_ctx* c, int N, const double* H, const double* gamma, double* Q, int64_t ldq,
                          double* K) {
    const int64_t M = (int64_t)N * N - 1;
    const int64_t P = lb_npairs(N);
    std::vector<int2> order;
    const int64_t norder = N >= 3 ? quad_order(N, order) : 0;
    const int nch = (N + kGthChunk - 1) / kGthChunk;
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
    const size_t o_gp = take(sizeof(double) * 2 * 4 * (size_t)nch * N * N);  // GpA, TpA, GpC, TpC
    const size_t o_pairs = take(sizeof(int2) * ((size_t)P + (size_t)norder) + 8);  // pairs, then the quad order
    int rc = lb_ws_reserve(c, off);
    if (rc) return rc;
    rc = lb_aux_stream(c);
    if (rc) return rc;
    const size_t hb = sizeof(int2) * ((size_t)P + (size_t)norder);
    rc = lb_host_reserve(c, hb);
    if (rc) return rc;
    char* ws = (char*)c->ws;
    int2* h = (int2*)c->host;
    // the pinned staging buffer may still be read by an earlier copy on this stream
    LB_HIP(hipStreamSynchronize(c->stream));
    int64_t hp = 0;
    for (int a = 0; a + 1 < N; ++a)
        for (int b = a + 1; b < N; ++b) h[hp++] = make_int2(a, b);
    for (int64_t i = 0; i < norder; ++i) h[P + i] = order[i];
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
    const int2* od = pd + P;
    const size_t part = (size_t)2 * nch * N * N;  // doubles per partial array
    double* GpA = (double*)(ws + o_gp);
    double* TpA = GpA + part;
    double* GpC = TpA + part;
    double* TpC = GpC + part;
    hipStream_t s = c->stream;

    hipLaunchKernelGGL(k_pt, dim3(lb_blocks(M, 256)), dim3(256), 0, s, v, (double*)(ws + o_pt));
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_cdd, dim3(lb_blocks((int64_t)N * N, 256)), dim3(256), 0, s, v, (double*)(ws + o_cdd));
    LB_CHECK_LAUNCH();
    const dim3 ggrid(lb_blocks((int64_t)N * N, 256), (unsigned)nch);
    hipLaunchKernelGGL(k_gth_a, ggrid, dim3(256), 0, s, v, GpA, TpA);
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_gth_c, ggrid, dim3(256), 0, s, v, GpC, TpC);
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_gth_fin, dim3(lb_blocks((int64_t)N * N, 256)), dim3(256), 0, s, v, H, (const double*)GpA,
                       (const double*)TpA, (const double*)GpC, (const double*)TpC, nch, Zm, Lam);
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_expand, dim3(lb_blocks(M, 256)), dim3(256), 0, s, N, 1, (const double*)Lam, K, 1.0 / N);
    LB_CHECK_LAUNCH();
    // the segments of pair rows on this stream; the shared-vertex segments, the
    // rows and columns of the diagonal generators and the padding on the
    // auxiliary stream, concurrently (they write other elements of Q)
    LB_HIP(hipEventRecord(c->ev_fork, s));
    LB_HIP(hipStreamWaitEvent(c->aux, c->ev_fork, 0));
    hipStream_t s2 = c->aux;
    if (norder > 0) {
        hipLaunchKernelGGL(k_quad, dim3((unsigned)norder), dim3(256), 0, s, v, (const double*)Zm, od, Q, ldq);
        LB_CHECK_LAUNCH();
    }
    if (P > 0) {
        hipLaunchKernelGGL(k_segpp, dim3(lb_blocks(P * 64, 256)), dim3(256), 0, s2, v, (const double*)Zm, pd, Q, ldq);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_drows, dim3(lb_blocks(P, 64)), dim3(64), 0, s2, v, (const double*)Zm, pd, Q, ldq);
        LB_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_dcols, dim3(lb_blocks(P, 64)), dim3(64), 0, s2, v, (const double*)Zm, pd, Q, ldq);
        LB_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_dd1, dim3(lb_blocks((int64_t)N * (N - 1), 64)), dim3(64), 0, s2, v, (const double*)Zm, T);
    LB_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_dd2, dim3(lb_blocks((int64_t)(N - 1) * (N - 1), 64)), dim3(64), 0, s2, v,
                       (const double*)T, Q, ldq);
    LB_CHECK_LAUNCH();
    if (ldq > M) {
        hipLaunchKernelGGL(k_zero_pad, dim3(lb_blocks(M * (ldq - M), 256)), dim3(256), 0, s2, Q, M, ldq);
        LB_CHECK_LAUNCH();
    }
    LB_HIP(hipEventRecord(c->ev_join, s2));
    LB_HIP(hipStreamWaitEvent(s, c->ev_join, 0));
    return LB_OK;
}
