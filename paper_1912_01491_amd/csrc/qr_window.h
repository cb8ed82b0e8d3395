// Geometry of the windowed multishift QR sweep (spectrum of Q, Fig. 5): which rows and
// columns a chain of bulges touches in a round, how a round's matrix products split into
// the part the next round's chase reads and the rest, and the band of a window's
// orthogonal factor. Shared by the kernels and the host loop of the spectrum, and by a
// host-only check of these rules; the includer provides the __host__ / __device__
// qualifiers (the HIP runtime header in the library).
#pragma once

namespace lb_qr {

constexpr int kSep = 4;                             // rows between neighbouring bulges
constexpr int kWin = 96;                            // window rows and columns
constexpr int kWinLd = kWin + 1;                    // LDS row stride of a window
constexpr int kChain = 8;                           // bulges per chain
constexpr int kAdvance = kWin + 1 - kSep * kChain;  // chain steps per round
constexpr int kChainGap = kWin + 1;                 // steps between the entries of two chains

// Band of a round's window factor: U^T[r][q] = 0 unless -(kAdvance + 1) <= q - r <= 2 kChain.
// A reflector mixes three consecutive rows. A bulge moves one row down per step, so it
// carries an entry at most kAdvance + 1 rows down within a round and at most two rows up
// (its next reflector starts one row lower); an entry moved up is picked up by the next
// bulge of the chain, kSep rows higher, two steps later, so the chain moves it at most
// 2 kChain rows up. The products skip the 16 x 4 blocks of U^T outside the band (30 % of
// them): their terms are exact zeros.
__host__ __device__ constexpr bool win_live(int tile, int kstep) {
    return 4 * kstep - (16 * tile + 15) <= 2 * kChain && 4 * kstep + 3 - 16 * tile >= -(kAdvance + 1);
}

// Columns where rows K..K+2 of U^T can be nonzero while a round runs (the band above for
// those rows; the zero pattern only grows within a round): a reflector at window row K
// changes U^T only there. With the window's columns K.. that is at most
// kWin + 2 kChain + 3 columns for one chase step's left side, two per lane of a wavefront.
__host__ __device__ constexpr int win_ut_lo(int K) { return K > kAdvance + 1 ? K - (kAdvance + 1) : 0; }
__host__ __device__ constexpr int win_ut_hi(int K, int wc) { return K + 2 + 2 * kChain < wc - 1 ? K + 2 + 2 * kChain : wc - 1; }
static_assert(kWin + 2 * kChain + 3 <= 128, "a chase step's left side fits two columns per lane");

// LDS of one chain's chase, in doubles: the window and U^T (kWin rows of stride kWinLd
// each) and a tail of kWin past U^T's last row. A step issues its loads unmasked, lanes
// without work included: the left side reads rows K..K+2 of window columns up to kWin - 1
// and of U^T columns up to kWin - 1 (K <= kWin - 2, so up to row kWin of U^T), the right
// side rows up to 127 of columns K..K+2 and rows K+1..K+3 of those columns; all of it
// lies below kWinLds.
constexpr int kWinLds = 2 * kWin * kWinLd + kWin;

struct WinGeom {
    int ws, we, active;
};

// Window [ws, we] of chain c in the round of steps t0 .. t0 + kAdvance - 1 of a sweep over
// [l, u] with b bulges; bulge j of the chain sits at row l + t - c kChainGap - kSep j in
// step t and is active while that row lies in [l, u - 1]. The window spans the last
// bulge's row at the first step to three rows past the lead bulge's at the last step:
// kAdvance - 1 + kSep (kChain - 1) + 4 = kWin rows at most.
__host__ __device__ inline WinGeom win_geom(int l, int u, int b, int c, int t0) {
    const int left = b - c * kChain;
    const int nbc = left < kChain ? left : kChain;
    const int rel = t0 - c * kChainGap;
    const int klead = l + rel + kAdvance - 1;
    const int ktail = l + rel - kSep * (nbc - 1);
    WinGeom g;
    g.active = klead >= l && ktail <= u - 1;
    g.ws = ktail > l ? ktail : l;
    g.we = klead + 3 < u ? klead + 3 : u;
    return g;
}

// Last column of the near part of chain c's row product: the columns the next round's
// chase of chain c reads (kAdvance past the window), extended to the end of the window of
// the chain ahead (c - 1), so that the block where chain c's rows cross that window's
// columns takes the whole left product before either part of that chain's column product
// (a left product split by columns, or a right one split by rows, is exact only if the
// other one does not fall between its parts).
__host__ __device__ inline int win_row_split(int l, int u, int b, int c, int t0, int we) {
    int nb = we + kAdvance;
    if (c > 0) {
        const WinGeom Ga = win_geom(l, u, b, c - 1, t0);
        if (Ga.active && Ga.we > nb) nb = Ga.we;
    }
    return nb < u ? nb : u;
}

// First row of chain c's column block above its window that the next round's chase of
// chain c + 1 (the chain behind it) reads: rows from there to ws form the near part of
// the column product, rows l.. up to there the far part. Chains further behind never
// reach these columns within a round (their windows end more than kAdvance columns
// before ws).
__host__ __device__ inline int win_split(int l, int u, int b, int c, int t0, int ws) {
    if ((c + 1) * kChain >= b) return ws;
    const WinGeom Gn = win_geom(l, u, b, c + 1, t0 + kAdvance);
    if (!Gn.active) return ws;
    return Gn.ws < ws ? Gn.ws : ws;
}

}  // namespace lb_qr
