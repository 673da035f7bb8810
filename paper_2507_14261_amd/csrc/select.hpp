// Block-level selection of the k smallest items by (s, id) with float64
// resolution of float32 near-ties at the selection boundary.
#pragma once
#include "famst_common.hpp"

namespace famst {

// Scratch for block_select; lives in LDS.
template <int LMAX>
struct SelectSmem {
  float s[LMAX];      // float32 squared distance of item i
  int id[LMAX];       // unique tie-break id of item i
  int rank[LMAX];     // rank by (s, id)
  int pos[LMAX];      // output: position among the selected, -1 if dropped
  double s64[LMAX];   // float64 squared distance (band items only)
  int band[LMAX];     // compacted list of band items
  float bnd[2];       // s of ranks k-1 and k
  int cnt[4];         // misc counters
};

// Select the k smallest of items [0, L) stored in sm.s / sm.id.  pair(i,
// &a, &b) must return the two points of item i (for the float64 check).
// On return sm.pos[i] is the output slot (ascending (s, id) among the
// selected) or -1.  Returns true (to every thread) if float64 had to be
// consulted.  All NT threads of the block must call it.
template <int NT, int LMAX, class PairFn>
__device__ bool block_select(SelectSmem<LMAX>& sm, int L, int k, float tau, int d,
                             PairFn pair) {
  const int t = threadIdx.x;
  for (int i = t; i < L; i += NT) {
    float si = sm.s[i];
    int ii = sm.id[i];
    int r = 0;
    for (int m = 0; m < L; ++m) r += key_less(sm.s[m], sm.id[m], si, ii) ? 1 : 0;
    sm.rank[i] = r;
    if (r == k - 1) sm.bnd[0] = si;
    if (r == k) sm.bnd[1] = si;
  }
  __syncthreads();
  if (L <= k) {
    for (int i = t; i < L; i += NT) sm.pos[i] = sm.rank[i];
    __syncthreads();
    return false;
  }
  const float hi_keep = sm.bnd[0], lo_drop = sm.bnd[1];
  const float up = 1.0f + 2.0f * tau, dn = 1.0f - 2.0f * tau;
  if (lo_drop * dn > hi_keep * up) {  // float32 order is certain
    for (int i = t; i < L; i += NT) sm.pos[i] = sm.rank[i] < k ? sm.rank[i] : -1;
    __syncthreads();
    return false;
  }
  // band: items whose true value may fall on either side of the boundary
  if (t == 0) { sm.cnt[0] = 0; sm.cnt[1] = 0; }
  __syncthreads();
  for (int i = t; i < L; i += NT) {
    float si = sm.s[i];
    bool inb = si * up >= lo_drop * dn && si * dn <= hi_keep * up;
    if (inb) {
      int p = atomicAdd(&sm.cnt[0], 1);
      sm.band[p] = i;
    } else if (sm.rank[i] < k) {
      atomicAdd(&sm.cnt[1], 1);
    }
    sm.s64[i] = 0.0;
  }
  __syncthreads();
  const int nb = sm.cnt[0], nin = sm.cnt[1];
  // float64 distances of band items, one 16-lane group per item
  const int grp = t >> 4, r16 = t & 15;
  for (int b = grp; b < nb; b += NT / 16) {
    int i = sm.band[b];
    const float* pa;
    const float* pb;
    pair(i, &pa, &pb);
    double v = sq64_group(pa, pb, d, r16);
    if (r16 == 0) sm.s64[i] = v;
  }
  __syncthreads();
  // mark selection: rank >= 0 selected, use pos as a temporary flag
  for (int i = t; i < L; i += NT) {
    bool sel;
    bool inb = false;
    for (int b = 0; b < nb; ++b) inb |= (sm.band[b] == i);
    if (inb) {
      int r = 0;
      for (int b = 0; b < nb; ++b) {
        int m = sm.band[b];
        r += key_less64(sm.s64[m], sm.id[m], sm.s64[i], sm.id[i]) ? 1 : 0;
      }
      sel = r < k - nin;
    } else {
      sel = sm.rank[i] < k;
    }
    sm.pos[i] = sel ? 0 : -1;
  }
  __syncthreads();
  // output order: ascending (s, id) among the selected
  for (int i = t; i < L; i += NT) {
    int p = -1;
    if (sm.pos[i] >= 0) {
      p = 0;
      for (int m = 0; m < L; ++m)
        p += (sm.pos[m] >= 0 && key_less(sm.s[m], sm.id[m], sm.s[i], sm.id[i])) ? 1 : 0;
    }
    sm.rank[i] = p;
  }
  __syncthreads();
  for (int i = t; i < L; i += NT) sm.pos[i] = sm.rank[i];
  __syncthreads();
  return true;
}

}  // namespace famst
