// Work items of the pair kernel and the order in which k_apply reads the
// partial sums.  Integer index arithmetic only, built for the device and (for
// the CPU test of the layout) for the host.
//
// The pairs of blocks (I, J), I <= J, of 64 particles are the tiles of the
// upper triangle.  A tile writes the sums its pairs give block J (the j side)
// to block J's slot for column I; the sums they give block I (the i side) go
// to block I's slot for column J0, the first tile of the work item that
// covers (I, J): a row strip of tiles (I, J0), ..., (I, J0 + len - 1) keeps
// the i-side sums of block I in one place and writes them once.  A row K
// (tiles J = K..nb-1, d = nb - K of them) split into strips of S tiles holds
// d / S strips, the first starting at the diagonal, and d mod S items of one
// tile: its last d mod S columns.  The other rows are items of one tile.
// Block K's slots are stored one after the other in k_apply's order
// (apply_offset, item_slot).
#pragma once
#include <cmath>

#ifndef SAKURA_TILES_HD
#define SAKURA_TILES_HD __host__ __device__
#endif

namespace sk {

// The strip length S is a power of two: x / S and x mod S (x >= 0) are a
// shift and a mask, where the kernels form them per tile.
SAKURA_TILES_HD inline long long div_s(long long x, int S) { return x >> __builtin_ctz(S); }
SAKURA_TILES_HD inline long long mod_s(long long x, int S) { return x & (S - 1); }

// Tile t of the one-tile-per-item order: off-diagonal tiles first (twice the
// work of a diagonal one), column by column, then the diagonal.
SAKURA_TILES_HD inline void tile_blocks(int t, int nb, int &I, int &J)
{
    const int noff = nb * (nb - 1) / 2;
    if (t < noff) {
        int j = (int)((1.0 + sqrt(1.0 + 8.0 * (double)t)) * 0.5);
        while (j * (j - 1) / 2 > t) --j;
        while ((j + 1) * j / 2 <= t) ++j;
        J = j;
        I = t - j * (j - 1) / 2;
    } else {
        I = J = t - noff;
    }
}

// Strips of S tiles over all rows: sum over d = 1..nb of d / S.
SAKURA_TILES_HD inline long long strip_count(int nb, int S)
{
    const long long q = div_s(nb, S), rho = mod_s(nb, S);
    return (long long)S * q * (q - 1) / 2 + q * (rho + 1);
}

// Items of one tile over all rows: sum over d = 1..nb of d mod S.
SAKURA_TILES_HD inline long long single_count(int nb, int S)
{
    const long long q = div_s(nb, S), rho = mod_s(nb, S);
    return q * ((long long)S * (S - 1) / 2) + rho * (rho + 1) / 2;
}

// Which rows are split into strips: rows K < kc into strips of S tiles (a
// power of two), the rows K >= kc (the triangle of the last nb - kc blocks)
// into items of one tile, which end the launch.  S <= 1 or kc = 0: one tile
// per item everywhere.
struct StripLayout {
    int S, kc;
};

SAKURA_TILES_HD inline bool strips_on(StripLayout L) { return L.S > 1 && L.kc > 0; }

// Strip length of row K.
SAKURA_TILES_HD inline int row_strip_len(StripLayout L, int K)
{
    return strips_on(L) && K < L.kc ? L.S : 1;
}

SAKURA_TILES_HD inline long long layout_items(int nb, StripLayout L)
{
    if (!strips_on(L)) return (long long)nb * (nb + 1) / 2;
    const int nt = nb - L.kc; // rows of single tiles only
    return strip_count(nb, L.S) - strip_count(nt, L.S) + single_count(nb, L.S) -
           single_count(nt, L.S) + (long long)nt * (nt + 1) / 2;
}

// Work item t of layout L: row I, first tile J0, len tiles.  First the
// strips, by their index m along the row (m = 0 starts at the diagonal) and
// then by row: strip m exists in the rows K < kc with K <= nb - (m + 1) S,
// all kc of them for m < mr = (nb + 1 - kc) / S, and c0 - (m - mr) S of
// them after that (c0 = nb - (mr + 1) S + 1).  Then the single tiles that
// end the strip rows (the last (nb - K) mod S columns of row K), longest rows
// first.  Last the triangle of rows K >= kc in the one-tile order, its
// half-work diagonal tiles at the very end.
SAKURA_TILES_HD inline void layout_item(long long t, int nb, StripLayout L, int &I, int &J0,
                                        int &len)
{
    if (!strips_on(L)) {
        tile_blocks((int)t, nb, I, J0);
        len = 1;
        return;
    }
    const int S = L.S, kc = L.kc, nt = nb - kc;
    const long long ns = strip_count(nb, S) - strip_count(nt, S);
    if (t < ns) {
        const long long mr = div_s(nb + 1 - kc, S); // kc <= nb
        const long long rect = mr * kc;
        len = S;
        if (t < rect) {
            I = (int)(t % kc);
            J0 = I + (int)(t / kc) * S;
            return;
        }
        const long long u = t - rect;
        const long long c0 = nb - (mr + 1) * S + 1; // < kc, and >= 1 here
        auto P = [&](long long k) { return k * c0 - (long long)S * k * (k - 1) / 2; };
        const long long kmax = div_s(c0 - 1, S); // the last index with a row: c0 - k S >= 1
        const double b = (double)c0 + 0.5 * S;
        long long k = (long long)((b - sqrt(fmax(b * b - 2.0 * S * (double)u, 0.0))) / S);
        if (k < 0) k = 0;
        if (k > kmax) k = kmax;
        while (k > 0 && P(k) > u) --k;
        while (k < kmax && P(k + 1) <= u) ++k;
        I = (int)(u - P(k));
        J0 = I + (int)(mr + k) * S;
        return;
    }
    t -= ns;
    const long long nr = single_count(nb, S) - single_count(nt, S);
    len = 1;
    if (t < nr) {
        // v counts the single tiles of all rows from the shortest (d = nb - K
        // = 1, 2, ...): the rows d = a S + rho (rho = 0..S-1) of one period
        // hold rho of them each, S (S - 1) / 2 together; the rows K >= kc
        // (d <= nt) come first in that count and are skipped
        const long long v = single_count(nt, S) + (nr - 1 - t);
        const long long per = (long long)S * (S - 1) / 2;
        const long long a = v / per;
        const int w = (int)(v % per);
        int rho = 1;
        while ((rho + 1) * rho / 2 <= w) ++rho;
        const int idx = w - rho * (rho - 1) / 2;
        const int d = (int)a * S + rho;
        I = nb - d;
        J0 = nb - rho + idx;
        return;
    }
    int i2, j2;
    tile_blocks((int)(t - nr), nt, i2, j2);
    I = kc + i2;
    J0 = kc + j2;
}

// The work items of the pair launch for the plain kernel of one wavefront
// per tile (mode 0 and SPLIT 1; every other launch takes one tile per item).
// Strips of S tiles along a row write one i-side partial per strip instead of
// one per tile (and start a wavefront once per strip), but a launch cannot
// end before its longest item, and long items drain it unevenly.  So the rows
// of the last blocks, a triangle of at least two tiles per wavefront slot
// (slots: the device's wavefront slots), stay single tiles, which the launch
// ends with, and the rows before them are strips of 4 tiles (a strip then
// takes about half of the launch at N = 16384; with 8 tiles, as long as the
// launch, the launch took 10 % longer).  A requested S (a power of two) puts
// strips in every row, of S tiles or of the largest power of two up to nb.
SAKURA_TILES_HD inline StripLayout choose_strips(int requested, bool plain_one_wave, int nb,
                                                 long long slots)
{
    if (!plain_one_wave || nb < 1) return StripLayout{1, 0};
    if (requested > 0) {
        int S = requested;
        while (S > 1 && S > nb) S >>= 1;
        return StripLayout{S, nb};
    }
    long long nt = 0;
    while (nt < nb && nt * (nt + 1) / 2 < 2 * slots) ++nt;
    return StripLayout{4, (int)(nb - nt)};
}

// The partial-sum slots block K receives (by the column L of the tile they
// come from), in k_apply's reduction order:
// slot k < K is the j side of tile (k, K); then the i sides of row K, one per
// strip (L = K, K + S, ...), then one per single tile.  One tile per item:
// L = 0..nb-1.
SAKURA_TILES_HD inline int apply_slots(int K, int nb, StripLayout L)
{
    const int S = row_strip_len(L, K), d = nb - K;
    return K + (int)div_s(d, S) + (int)mod_s(d, S);
}

SAKURA_TILES_HD inline int apply_slot(int k, int K, int nb, StripLayout L)
{
    if (k < K) return k;
    const int S = row_strip_len(L, K);
    const int f = (int)div_s(nb - K, S);
    if (k - K < f) return K + (k - K) * S;
    return K + f * S + (k - K - f);
}

// Storage of the partial sums: block K's slots k = 0..apply_slots(K)-1 in
// k_apply's order, blocks one after the other; block K starts at slot
// apply_offset(K) (the slots of blocks 0..K-1), and apply_offset(nb) is the
// whole buffer.  One tile per item: K nb, the square part[nb][nb].
SAKURA_TILES_HD inline long long apply_offset(int K, int nb, StripLayout L)
{
    const long long k = K;
    if (!strips_on(L)) return k * nb;
    // rows K' < K: K' j sides each, plus their i sides; a row K' >= kc of
    // single tiles has nb - K' i sides, nb slots in all
    const int ms = K < L.kc ? K : L.kc; // strip rows among them
    const long long m = ms;
    return m * (m - 1) / 2 + strip_count(nb, L.S) - strip_count(nb - ms, L.S) +
           single_count(nb, L.S) - single_count(nb - ms, L.S) + (k - m) * nb;
}

// The slot of block I that the i side of the item starting at tile (I, J0)
// goes to: its place among the row's strips and single tiles, after the I j
// sides.  (The j side of tile (I, J) is slot I of block J.)
SAKURA_TILES_HD inline int item_slot(int I, int J0, int nb, StripLayout L)
{
    const int S = row_strip_len(L, I);
    const int f = (int)div_s(nb - I, S);
    const int e = J0 - I;
    return e < f * S ? I + (int)div_s(e, S) : I + f + (e - f * S);
}

} // namespace sk
