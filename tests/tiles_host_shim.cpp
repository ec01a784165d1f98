// Host build of the pair kernel's work-item layout (paper_1402_3325_amd/csrc/
// tiles.hpp), for the CPU test of its coverage (tests/test_tile_layout.py).
#include <cmath>
#include <cstdint>
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
