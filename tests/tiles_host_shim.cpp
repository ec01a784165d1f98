// Host build of the pair kernel's work-item layout (paper_1402_3325_amd/csrc/
// tiles.hpp), for the CPU test of its coverage (tests/test_tile_layout.py).
#include <cmath>
#include <cstdint>
#include <vector>
using std::fmax;
using std::sqrt;
#define SAKURA_TILES_HD
#include "../paper_1402_3325_amd/csrc/tiles.hpp"

// Rows K < kc in strips of S tiles, the others in items of one tile.
extern "C" long long host_item_count(int nb, int S, int kc)
{
    return sk::layout_items(nb, sk::StripLayout{S, kc});
}

// out[3 t ..] = (I, J0, len) of work item t, t < host_item_count(nb, S, kc)
extern "C" void host_items(int nb, int S, int kc, int *out)
{
    const sk::StripLayout L{S, kc};
    const long long n = sk::layout_items(nb, L);
    for (long long t = 0; t < n; ++t)
        sk::layout_item(t, nb, L, out[3 * t], out[3 * t + 1], out[3 * t + 2]);
}

// out[k] = the k-th slot block K reduces; returns the count
extern "C" int host_apply_slots(int K, int nb, int S, int kc, int *out)
{
    const sk::StripLayout L{S, kc};
    const int n = sk::apply_slots(K, nb, L);
    for (int k = 0; k < n; ++k) out[k] = sk::apply_slot(k, K, nb, L);
    return n;
}

// Start of block K's slots in the compact storage, K = 0..nb (nb: the whole buffer).
extern "C" long long host_apply_offset(int K, int nb, int S, int kc)
{
    return sk::apply_offset(K, nb, sk::StripLayout{S, kc});
}

extern "C" int host_item_slot(int I, int J0, int nb, int S, int kc)
{
    return sk::item_slot(I, J0, nb, sk::StripLayout{S, kc});
}

// The layout the library picks: out[0] = S, out[1] = kc.
extern "C" void host_choose_strips(int requested, int plain_one_wave, int nb, long long slots,
                                   int *out)
{
    const sk::StripLayout L = sk::choose_strips(requested, plain_one_wave != 0, nb, slots);
    out[0] = L.S;
    out[1] = L.kc;
}

// Every tile covered once and every slot of the compact storage written once,
// counted in C++ for large block counts: the number of violations.
extern "C" long long host_check_layout(int nb, int S, int kc)
{
    const sk::StripLayout L{S, kc};
    std::vector<long long> off(nb + 1);
    for (int K = 0; K <= nb; ++K) off[K] = sk::apply_offset(K, nb, L);
    std::vector<unsigned char> cover((size_t)nb * nb, 0), slot((size_t)off[nb], 0);
    long long bad = 0;
    const long long n = sk::layout_items(nb, L);
    for (long long t = 0; t < n; ++t) {
        int I, J0, len;
        sk::layout_item(t, nb, L, I, J0, len);
        if (I < 0 || J0 < I || len < 1 || J0 + len > nb) {
            ++bad;
            continue;
        }
        for (int J = J0; J < J0 + len; ++J) {
            ++cover[(size_t)I * nb + J];
            if (J == I) continue;
            const long long sj = off[J] + I; // the j side
            if (sj >= off[J + 1]) ++bad;
            else ++slot[(size_t)sj];
        }
        const long long si = off[I] + sk::item_slot(I, J0, nb, L);
        if (si < off[I] || si >= off[I + 1]) ++bad;
        else ++slot[(size_t)si];
    }
    for (int I = 0; I < nb; ++I)
        for (int J = 0; J < nb; ++J) bad += cover[(size_t)I * nb + J] != (J >= I ? 1 : 0);
    for (long long k = 0; k < off[nb]; ++k) bad += slot[(size_t)k] != 1;
    return bad;
}
