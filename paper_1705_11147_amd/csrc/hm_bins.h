// The bin map and the first partition level's launch shape of the binned path, shared by the
// partition (hm_bins.hip) and by the cardinality pass that can count the first level's
// histogram on its way (hm_card.hip).
#pragma once

#include "hm_device.h"

namespace hm {

// bin map: multiply-shift hashing (any odd constants; the output does not depend on them)
constexpr uint64_t kBinMul1 = 0xC2B2AE3D27D4EB4Full;
constexpr uint64_t kBinMul2 = 0x165667B19E3779F9ull;

__device__ __forceinline__ uint64_t bin_hash(uint64_t hi, uint64_t lo) { return (lo ^ hi * kBinMul1) * kBinMul2; }

// bin of a key: the top `bits` bits of its bin hash (0 when bits == 0)
__device__ __forceinline__ uint32_t bin_of(uint64_t hi, uint64_t lo, int bits) {
    return bits ? (uint32_t)(bin_hash(hi, lo) >> (64 - bits)) : 0u;
}

// host side (hm_bins.hip): argument checks of a bins descriptor, the first level's grid for a
// read set of n_tiles tiles (the pass that counts its histogram and the pass that scatters must
// both use it, as they must use the same tiles), and where that histogram lives in the scratch
int check_bins(const hm_bins_t *b);
int bins_grid1(int64_t n_tiles, uint32_t group_bits);
uint32_t *bins_hist1(const hm_bins_t *b);
// hm_cardinality_bins notes what it counted the histogram for; every hm_bin_kmers takes the note
// and, with HM_BINS_COUNTED, accepts only a note of the same reads, params and bin counts
void bins_note_counted(const hm_bins_t *b, const hm_reads_t *r, const hm_params_t *p);
bool bins_take_counted(const hm_bins_t *b, const hm_reads_t *r, const hm_params_t *p);
void bins_drop_counted(const hm_bins_t *b);  // a partition that does not use the note drops it

}  // namespace hm
