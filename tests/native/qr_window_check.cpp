// Host-only check of the geometry of the windowed multishift QR sweep
// (paper_1912_01491_amd/csrc/qr_window.h), over many active-block sizes and bulge counts:
//  - each chain's window lies in the block, spans at most kWin rows, and the windows of
//    two chains of a round never overlap;
//  - every reflector position of a round (rows K..K+3 a step touches) lies in its chain's
//    window;
//  - the far parts of a round's products (run during the next round's chase) never meet a
//    window of the next round, and the near parts cover the columns and rows those
//    windows read;
//  - where one chain's rows cross another chain's window columns, neither product is split
//    with the other one falling between its parts (order: near rows, near columns, far
//    rows, far columns);
//  - the zero pattern of a window's orthogonal factor, propagated through the round's
//    reflector positions, stays inside the band the products skip outside of, and the
//    rows a reflector mixes are zero outside the columns the chase updates;
//  - every LDS load a chase step issues (unmasked, idle lanes included) lies inside the
//    chase's LDS array.
#include <algorithm>
#include <cstdio>
#include <vector>

// the library provides these qualifiers through the HIP runtime header; here plain C++
#define __host__
#define __device__
#include "qr_window.h"

using namespace lb_qr;

static long fails = 0, checks = 0;
#define CHECK(cond, ...)                           \
    do {                                           \
        ++checks;                                  \
        if (!(cond) && fails++ < 20) {             \
            std::printf(__VA_ARGS__);              \
            std::printf("\n");                     \
        }                                          \
    } while (0)

struct Rect {
    int r0, r1, c0, c1;  // inclusive bounds
    bool empty() const { return r0 > r1 || c0 > c1; }
};

static bool meet(const Rect& a, const Rect& b) {
    return !a.empty() && !b.empty() && !(a.r1 < b.r0 || b.r1 < a.r0 || a.c1 < b.c0 || b.c1 < a.c0);
}

static bool overlap(int a0, int a1, int b0, int b1) { return std::max(a0, b0) <= std::min(a1, b1); }

static void check_sweep(int l, int u, int b) {
    const int nch = (b + kChain - 1) / kChain;
    const int nbl = b - (nch - 1) * kChain;
    const int T = (nch - 1) * kChainGap + kSep * (nbl - 1) + (u - l);
    for (int t0 = 0; t0 < T; t0 += kAdvance) {
        std::vector<WinGeom> G(nch), Gn(nch);
        for (int c = 0; c < nch; ++c) {
            G[c] = win_geom(l, u, b, c, t0);
            Gn[c] = win_geom(l, u, b, c, t0 + kAdvance);
        }
        for (int c = 0; c < nch; ++c) {
            if (!G[c].active) continue;
            CHECK(G[c].ws >= l && G[c].we <= u && G[c].we - G[c].ws + 1 <= kWin && G[c].ws <= G[c].we,
                  "window [%d, %d] of chain %d outside [%d, %d] or too long (t0 %d)", G[c].ws, G[c].we, c, l, u, t0);
            for (int a = 0; a < c; ++a)
                if (G[a].active) CHECK(G[c].we < G[a].ws, "windows of chains %d and %d overlap (t0 %d)", c, a, t0);
        }
        // reflector positions of the round
        for (int c = 0; c < nch; ++c) {
            const int nbc = std::min(kChain, b - c * kChain);
            for (int s = 0; s < kAdvance; ++s) {
                const int rel = t0 + s - c * kChainGap;
                for (int j = 0; j < nbc; ++j) {
                    const int k = l + rel - kSep * j;
                    if (k < l || k > u - 1) continue;
                    CHECK(G[c].active && k >= G[c].ws && std::min(k + 3, u) <= G[c].we,
                          "bulge %d of chain %d at %d outside window [%d, %d] (t0 %d, l %d, u %d, b %d)", j, c, k,
                          G[c].ws, G[c].we, t0, l, u, b);
                }
            }
        }
        // near and far parts of the products
        std::vector<int> nb(nch), sp(nch);
        std::vector<Rect> far;
        for (int c = 0; c < nch; ++c) {
            if (!G[c].active) continue;
            nb[c] = win_row_split(l, u, b, c, t0, G[c].we);
            sp[c] = win_split(l, u, b, c, t0, G[c].ws);
            CHECK(nb[c] >= std::min(u, G[c].we + kAdvance) && nb[c] <= u, "row split %d of chain %d", nb[c], c);
            CHECK(sp[c] >= l && sp[c] <= G[c].ws, "column split %d of chain %d", sp[c], c);
            if (Gn[c].active) CHECK(Gn[c].we <= nb[c], "next window of chain %d ends past its near columns", c);
            far.push_back({G[c].ws, G[c].we, nb[c] + 1, u});
            far.push_back({l, sp[c] - 1, G[c].ws, G[c].we});
        }
        for (int c = 0; c < nch; ++c) {
            if (!Gn[c].active) continue;
            const Rect w = {Gn[c].ws, Gn[c].we, Gn[c].ws, Gn[c].we};
            for (const Rect& f : far)
                CHECK(!meet(f, w), "far part [%d..%d]x[%d..%d] meets the next window [%d, %d] of chain %d (t0 %d)",
                      f.r0, f.r1, f.c0, f.c1, w.r0, w.r1, c, t0);
        }
        // crossing blocks: rows of chain a's window, columns of chain c's window, c ahead of a
        for (int a = 0; a < nch; ++a)
            for (int c = 0; c < a; ++c) {
                if (!G[a].active || !G[c].active) continue;
                const bool lnear = overlap(G[c].ws, G[c].we, G[a].we + 1, nb[a]);
                const bool lfar = overlap(G[c].ws, G[c].we, nb[a] + 1, u);
                const bool rnear = overlap(G[a].ws, G[a].we, sp[c], G[c].ws - 1);
                const bool rfar = overlap(G[a].ws, G[a].we, l, sp[c] - 1);
                CHECK(!(lnear && lfar && rnear), "left product of chain %d split around chain %d's near columns", a, c);
                CHECK(!(rnear && rfar && lfar), "right product of chain %d split around chain %d's far rows", c, a);
            }
    }
}

// The zero pattern of U^T through a round: a reflector at window row K mixes rows K..K+2
// (K..K+1 at the block's last row), each becoming the union of their patterns.
static void check_band(int l, int u, int b) {
    const int nch = (b + kChain - 1) / kChain;
    const int nbl = b - (nch - 1) * kChain;
    const int T = (nch - 1) * kChainGap + kSep * (nbl - 1) + (u - l);
    std::vector<unsigned char> P(kWin * kWin);
    for (int t0 = 0; t0 < T; t0 += kAdvance)
        for (int c = 0; c < nch; ++c) {
            const WinGeom G = win_geom(l, u, b, c, t0);
            if (!G.active) continue;
            const int ws = G.ws, wc = G.we - G.ws + 1, nbc = std::min(kChain, b - c * kChain);
            std::fill(P.begin(), P.end(), 0);
            for (int r = 0; r < wc; ++r) P[r * kWin + r] = 1;
            for (int s = 0; s < kAdvance; ++s) {
                const int rel = t0 + s - c * kChainGap;
                for (int j = 0; j < nbc; ++j) {
                    const int k = l + rel - kSep * j;
                    if (k < l || k > u - 1) continue;
                    const int K = k - ws, n = k + 2 <= u ? 3 : 2;
                    const int lo = win_ut_lo(K), hi = win_ut_hi(K, wc);
                    CHECK((wc - K) + (hi - lo + 1) <= 128, "left side of %d columns at K %d", (wc - K) + (hi - lo + 1), K);
                    // the chase's unmasked LDS loads of this step (window at 0, U^T at kWin kWinLd):
                    // left side rows K..K+2 of window columns K..wc-1 and of U^T columns lo..hi;
                    // right side rows 0..63 (and 64..127 once K >= 64) of columns K..K+2, and
                    // rows K+1..K+3 of those columns
                    const int last_left = std::max((K + 2) * kWinLd + wc - 1, kWin * kWinLd + (K + 2) * kWinLd + hi);
                    const int last_right = std::max((K >= 64 ? 127 : 63) * kWinLd + K + 2, (K + 3) * kWinLd + K + 2);
                    CHECK(K >= 0 && K <= wc - 2 && std::max(last_left, last_right) < kWinLds,
                          "chase LDS read at %d of %d (K %d, wc %d)", std::max(last_left, last_right), kWinLds, K, wc);
                    for (int q = 0; q < wc; ++q)
                        if (q < lo || q > hi)
                            for (int m = 0; m < n; ++m)
                                CHECK(!P[(K + m) * kWin + q],
                                      "factor row %d nonzero in column %d outside [%d, %d] (chain %d, t0 %d, s %d)",
                                      K + m, q, lo, hi, c, t0, s);
                    for (int q = 0; q < wc; ++q) {
                        unsigned char v = 0;
                        for (int m = 0; m < n; ++m) v |= P[(K + m) * kWin + q];
                        for (int m = 0; m < n; ++m) P[(K + m) * kWin + q] = v;
                    }
                }
            }
            for (int r = 0; r < wc; ++r)
                for (int q = 0; q < wc; ++q)
                    if (P[r * kWin + q])
                        CHECK(q - r <= 2 * kChain && r - q <= kAdvance + 1 && win_live(r / 16, q / 4),
                              "window factor entry (%d, %d) outside the band (chain %d, t0 %d, l %d, u %d, b %d)", r,
                              q, c, t0, l, u, b);
        }
}

int main() {
    std::vector<int> sizes = {257, 258, 260, 261, 300, 333, 420, 575, 1000, 1023, 1500, 4095};
    for (int na : sizes)
        for (int l : {0, 5}) {
            const int u = l + na - 1;
            const int bd = std::min(64, std::max(1, na / 16));  // the bulge count of a sweep over na rows
            for (int b : {bd, 1, 7, 8, 9, 17, 33, 64}) {
                if (b > bd) continue;
                check_sweep(l, u, b);
                check_band(l, u, b);
            }
        }
    std::printf("%ld checks, %ld failed\n", checks, fails);
    return fails ? 1 : 0;
}
