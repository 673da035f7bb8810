// Bitonic compare-exchange networks on (s, key) pairs held one per lane.
#pragma once
#include "famst_common.hpp"

namespace famst {

// Compare-exchange of (s, j) with the lane at distance M (M <= 32): where
// `asc`, the lower lane of the pair keeps the smaller (s, j); keys compare
// as unsigned after s.
template <int M>
__device__ __forceinline__ void cex_lane(float& s, uint32_t& j, bool asc, int lane) {
  const float ps = __shfl_xor(s, M);
  const uint32_t pj = (uint32_t)__shfl_xor((int)j, M);
  const bool lower = (lane & M) == 0;
  const bool pless = (ps < s) | ((ps == s) & (pj < j));
  const bool sless = (s < ps) | ((s == ps) & (j < pj));
  const bool take = (lower == asc) ? pless : sless;
  s = take ? ps : s;
  j = take ? pj : j;
}

// Ascending bitonic sort of the 64 (s, j) of a wave.
__device__ __forceinline__ void sort64_asc(float& s, uint32_t& j, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
    const bool asc = (lane & k) == 0;
    if (k >= 64) cex_lane<32>(s, j, asc, lane);
    if (k >= 32) cex_lane<16>(s, j, asc, lane);
    if (k >= 16) cex_lane<8>(s, j, asc, lane);
    if (k >= 8) cex_lane<4>(s, j, asc, lane);
    if (k >= 4) cex_lane<2>(s, j, asc, lane);
    cex_lane<1>(s, j, asc, lane);
  }
}

}  // namespace famst
