// Pipelined screening with register-resident queries (k' = 32, up to 128 bf16 / 64 fp32 dims).
#pragma once
#include "screen_regs.hpp"

namespace famst {

// Block shape of the pipelined screening: NW waves of 64 queries share tiles
// of 16 NW rows.  Four waves (two blocks per compute unit) suit batches of
// small clouds; eight waves (one block per compute unit) halve the rows
// streamed per query on one large cloud, at the price of a barrier across
// twice as many waves.
template <int NW>
struct V2Shape {
  static constexpr int NT = 64 * NW, BN = 16 * NW, GR = BN / 32;   // threads, tile rows, 32-row groups
  static_assert(NW == 4 || NW == 8, "four or eight waves");
};
template <int NW>
constexpr size_t v2_lds_bytes(int nkb) {
  return (size_t)PIPE * (V2Shape<NW>::BN * nkb * 64 + 4 * V2Shape<NW>::BN);
}

// Tiles at the start of each block's scan whose passing elements are merged
// into the lists a query block at a time (merge_regs) rather than inserted
// one by one.
constexpr int V2_MERGE_TILES = 4;

// BUF: the scan past the merged tiles appends to per-query LDS buffers
// (buffer_regs) instead of inserting one element at a time; for four-wave
// blocks of up to two K-blocks (beyond, the ring leaves no LDS for the
// buffers at two blocks per CU), chosen by the host for short scans.
template <int PREC, int NKB, int NW, bool BUF = false>
__global__ __launch_bounds__(64 * NW, 8 / NW) void dist_topk_v2_kernel(
    const void* __restrict__ Xq_, const float* __restrict__ nq, int nkb,
    const BlockDesc* __restrict__ desc, int* __restrict__ cand_j, float* __restrict__ cand_s,
    int kk, const float* __restrict__ qerr, const unsigned* __restrict__ gstat, float arith_c,
    float tau, float* __restrict__ ubound, const int* __restrict__ perm) {
  using S = Scr<PREC>;
  constexpr int QB = 4, KC = 32, QW = 64, BN = V2Shape<NW>::BN, NT = V2Shape<NW>::NT, GR = V2Shape<NW>::GR;
  constexpr int TILE = BN * NKB * 64;   // BN rows x NKB 64-byte chunks
  constexpr int STG = TILE + 4 * BN;    // tile + its BN norms
  static_assert(GR % 2 == 0, "32-row groups alternate between two accumulator sets");
  const char* Xb = reinterpret_cast<const char*>(Xq_);
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ __attribute__((aligned(16))) float iscratch[NW][INIT_LDS_FLOATS];   // lists from the first rows
  // buffered list updates past the merged tiles
  static_assert(!BUF || (NKB <= 2 && NW == 4), "buffers only where the LDS holds them");
  constexpr bool BUFD = BUF;
  __shared__ __attribute__((aligned(16))) float bufs[BUFD ? NW : 1][BUFD ? 64 * BUF_SLOTS : 4];
  __shared__ __attribute__((aligned(16))) int bufj[BUFD ? NW : 1][BUFD ? 64 * BUF_SLOTS : 4];

  const BlockDesc bd = desc[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, i16 = lane & 15;
  const int wq0 = bd.q0 + wave * QW;
  // instantiated for the exact number of K-blocks: no runtime guards in the
  // tile loop (they would split it into branches and force full waits)
  constexpr int RS = NKB * 64, cpr = NKB * 4;
  constexpr int smask = (cpr & 15) == 0 ? 15 : ((cpr & 7) == 0 ? 7 : 3);

  // resident query fragments, scaled by -2 (exact): the products then
  // accumulate onto the row norms and yield the screened value
  // |y|^2 - 2 x.y directly.  The norm and the band constants of the wave's
  // query l sit in lane l (only insertions read them, by readlane).
  i32x4 qf[QB][NKB];
  float U[QB];
  const Band band{arith_c, __uint_as_float(gstat[1]), __uint_as_float(gstat[2]), tau};
  float nql, bcl0, bcl1;
  {
    const int q = wq0 + lane;
    const bool ok = q < bd.q1;
    nql = ok ? nq[q] : 0.f;
    band.consts(nql, ok ? qerr[q] : 0.f, bcl0, bcl1);
  }
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int q = wq0 + qb * 16 + i16;
    const bool ok = q < bd.q1;
    U[qb] = ok ? F_INF : -F_INF;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      i32x4 v = {0, 0, 0, 0};
      if (ok) v = *reinterpret_cast<const i32x4*>(Xb + (int64_t)q * RS + kb * 64 + g * 16);
      qf[qb][kb] = neg2_fragment<PREC>(v);
    }
  }
  f32x32 ls;
  i32x32 lj;
#pragma unroll
  for (int L = 0; L < 32; ++L) {
    ls[L] = F_INF;
    lj[L] = 0x7FFFFFFF;
  }
  int bcnt[QB];   // buffered elements of the lane's query in each block
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) bcnt[qb] = 0;
  if constexpr (BUFD) {
#pragma unroll
    for (int i = 0; i < BUF_SLOTS / 4; ++i)
      *reinterpret_cast<f32x4*>(&bufs[wave][BUF_SLOTS * lane + 4 * i]) = f32x4{F_INF, F_INF, F_INF, F_INF};
  }

  // Loads of a tile into a stage: chunk slot p of the stage holds chunk
  // (p mod cpr) ^ (row & smask) of row p / cpr (the XOR swizzle of
  // dist_topk_kernel), so lane l of a wave fetches the chunk that lands at
  // its slot; its byte offset from the tile's first row is the same for
  // every tile.  The screening copy and its norms hold at least BN padding
  // rows past the last cloud, so a tile never reads outside them (rows past a
  // cloud never enter a list).  Every thread issues NKB + 1 loads per tile
  // (wave w loads the norms of rows 64 (w mod BN/64) + lane), which keeps the
  // vmcnt bookkeeping static.
  // Scan order: tiles tstart, tstart + 1, ... cyclically.  With a spatial
  // order (perm != null: rows of Xq are the points perm[.], grouped by
  // nearest pivot) tstart is the tile of the block's own first query, so the
  // likely neighbours come first and the thresholds tighten early.  Two
  // scalar counters follow the tile to load and the tile to compute.
  const int ntile = (bd.c1 - bd.c0 + BN - 1) / BN;
  const int tstart = perm ? (bd.q0 - bd.c0) / BN : 0;
  int tl = tstart;   // next tile to load
  unsigned voff[NKB];
#pragma unroll
  for (int i = 0; i < NKB; ++i) {
    const int p = tid + NT * i;
    const int r = p / cpr, sc = p - r * cpr;
    voff[i] = (unsigned)(r * RS + ((sc ^ (r & smask)) << 4));
  }
  auto issue = [&](int stg) {
    const int t0 = bd.c0 + tl * BN;
    tl = tl + 1 == ntile ? 0 : tl + 1;
    char* stage = smem + stg * STG;
    const char* tb = Xb + (int64_t)t0 * RS;
#pragma unroll
    for (int i = 0; i < NKB; ++i)
      __builtin_amdgcn_global_load_lds((gptr_t)(tb + voff[i]), (lptr_t)(stage + (NT * i + 64 * wave) * 16),
                                       16, 0, 0);
    const int nh = wave % (BN / 64);
    __builtin_amdgcn_global_load_lds((gptr_t)(nq + t0 + 64 * nh + lane), (lptr_t)(stage + TILE + 256 * nh), 4, 0,
                                     0);
  };
  // one tile consumed by every thread: wait for the next tile's loads, let
  // every wave pass, and refill the stage the consumed tile used
  auto next_tile = [&](int it) {
    wait_vmcnt<(PIPE - 2) * (NKB + 1)>();   // this thread's loads of tile it are done
    __builtin_amdgcn_s_barrier();           // ... and every thread's; tile it-1 is consumed
    issue((it + PIPE - 1) & (PIPE - 1));    // into the stage tile it-1 used
  };

  // Products of one 32-row group jh of a tile: the accumulators start at the
  // norms of their rows; A fragments double-buffered (the LDS reads of
  // K-step kb + 1 are issued before the products of K-step kb).
  auto products = [&](const char* tile, int jh, f32x4 (&acc)[QB][2]) {
    const float* tn = reinterpret_cast<const float*>(tile + TILE);
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
      const f32x4 v = *reinterpret_cast<const f32x4*>(tn + (2 * jh + jj) * 16 + 4 * g);
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) acc[qb][jj] = v;
    }
    auto lda = [&](int kb, i32x4 (&a)[2]) {
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int r = (2 * jh + jj) * 16 + i16;
        const int cc = kb * 4 + g;
        a[jj] = *reinterpret_cast<const i32x4*>(tile + r * RS + ((cc ^ (r & smask)) << 4));
      }
    };
    i32x4 acur[2], anxt[2];
    lda(0, acur);
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      if (kb + 1 < NKB) lda(kb + 1, anxt);
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const i32x4 a = acur[jj];
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
          if constexpr (PREC == FAMST_FP32) {
            const f32x4 af = __builtin_bit_cast(f32x4, a);
            const f32x4 bf = __builtin_bit_cast(f32x4, qf[qb][kb]);
            acc[qb][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0], bf[0], acc[qb][jj], 0, 0, 0);
            acc[qb][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1], bf[1], acc[qb][jj], 0, 0, 0);
            acc[qb][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[2], bf[2], acc[qb][jj], 0, 0, 0);
            acc[qb][jj] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[3], bf[3], acc[qb][jj], 0, 0, 0);
          } else {
            acc[qb][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, qf[qb][kb]), acc[qb][jj], 0, 0, 0);
          }
        }
      }
      if (kb + 1 < NKB) {
        acur[0] = anxt[0];
        acur[1] = anxt[1];
      }
    }
  };
  // Screening filter of one group: lane holds rows t0h + jj*16 + 4g + r,
  // query qb*16 + i16.  The mode (a compile-time constant) picks the list
  // update: 0 single insertions, 1 whole-block merges, 2 buffered appends.
  auto filter = [&](const f32x4 (&acc)[QB][2], int t0h, auto mode) __attribute__((always_inline)) {
    unsigned qbmask = 0;
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      float m = acc[qb][0][0];
#pragma unroll
      for (int e = 1; e < 8; ++e) m = fminf(m, acc[qb][e >> 2][e & 3]);
      qbmask |= ballot(m <= U[qb]) ? (1u << qb) : 0u;
    }
    auto sv = [&](int qb, int e) { return acc[qb][e >> 2][e & 3]; };
    if (qbmask) {
      constexpr int m = (int)decltype(mode)::value;
      if constexpr (m == 1)
        merge_regs<QB, 8>(ls, lj, qbmask, U, nql, bcl0, bcl1, band, kk, sv, t0h, bd.c1, wq0, lane, g, i16,
                          iscratch[wave]);
      else if constexpr (m == 2)
        buffer_regs<QB>(ls, lj, qbmask, U, bcnt, bufs[wave], bufj[wave], nql, bcl0, bcl1, band, kk, sv, t0h,
                        bd.c1, wq0, lane, g, i16, iscratch[wave]);
      else
        insert_regs<QB, 8>(ls, lj, qbmask, U, nql, bcl0, bcl1, band, kk, sv, t0h, bd.c1, wq0, lane, g, i16);
    }
  };

  // Software pipeline over 32-row groups: the products of the next group
  // are issued before the filter (and any insertion) of the current one, so
  // the matrix cores stay busy meanwhile.  Group h of a tile accumulates in
  // accA for even h, accB for odd h.
#pragma unroll
  for (int it = 0; it < PIPE - 1; ++it) issue(it);
  f32x4 accA[QB][2], accB[QB][2];
  next_tile(0);
  products(smem, 0, accA);
  // the first 32 rows of the scan fill the lists at once
  init_lists<QB>(ls, lj, U, nql, bcl0, bcl1, band, kk, [&](int qb, int e) { return accA[qb][e >> 2][e & 3]; },
                 bd.c0 + tstart * BN, bd.c1, wq0, lane, g, i16, iscratch[wave]);
  int tc = tstart;   // tile being computed
  auto tile_step = [&](int it, auto mode) __attribute__((always_inline)) {
    const char* tile = smem + (it & (PIPE - 1)) * STG;
    const int t0 = bd.c0 + tc * BN;
    tc = tc + 1 == ntile ? 0 : tc + 1;
#pragma unroll
    for (int h = 1; h < GR; h += 2) {
      products(tile, h, accB);
      if (it > 0 || h > 1) filter(accA, t0 + 32 * (h - 1), mode);
      if (h + 1 < GR) {
        products(tile, h + 1, accA);
        filter(accB, t0 + 32 * h, mode);
      }
    }
    if (it + 1 < ntile) {
      next_tile(it + 1);
      products(smem + ((it + 1) & (PIPE - 1)) * STG, 0, accA);
    }
    filter(accB, t0 + 32 * (GR - 1), mode);
  };
  // At four K-blocks the merges run without the software pipeline (the
  // products of a group, then its merge): the second accumulator set is not
  // live across them, which keeps the merge's registers from spilling.
  auto merge_step_serial = [&](int it) __attribute__((always_inline)) {
    const char* tile = smem + (it & (PIPE - 1)) * STG;
    const int t0 = bd.c0 + tc * BN;
    tc = tc + 1 == ntile ? 0 : tc + 1;
    if (it > 0) filter(accA, t0, std::true_type{});   // group 0 of the first tile filled the lists
#pragma unroll
    for (int h = 1; h < GR; ++h) {
      products(tile, h, accA);
      filter(accA, t0 + 32 * h, std::true_type{});
    }
    if (it + 1 < ntile) {
      next_tile(it + 1);
      products(smem + ((it + 1) & (PIPE - 1)) * STG, 0, accA);
    }
  };
  // The scan runs in phases, each its own copy of the tile loop, so that the
  // list registers have one update path per loop: the first tiles, where
  // most rows still pass, merge whole query blocks; the rest append to the
  // LDS buffers (BUF) or insert one element at a time.
  int it = 0;
  const int nmerge = min(ntile, V2_MERGE_TILES);
  if constexpr (NKB < 4) {
    for (; it < nmerge; ++it) tile_step(it, std::true_type{});
  } else {
    for (; it < nmerge; ++it) merge_step_serial(it);
  }
  if constexpr (BUFD) {
    // the rest of the scan appends to the buffers; the last merge empties them
    for (; it < ntile; ++it) tile_step(it, std::integral_constant<int, 2>{});
#pragma unroll
    for (int qb = 0; qb < QB; ++qb)
      if (ballot(bcnt[qb] > 0))
        flush_block(ls, lj, U[qb], qb, bufs[wave], bufj[wave], nql, bcl0, bcl1, band, kk, lane, i16,
                    iscratch[wave]);
  } else {
    for (; it < ntile; ++it) tile_step(it, std::false_type{});
  }
  wait_vmcnt<0>();   // no load may land in LDS after the block ends

  // ---- write the candidate lists and the bound of the rejected elements
  // (rows and ids back in the caller's numbering under a spatial order)
  float nqv[QB];   // norms of the lane's queries (every lane takes part in the shuffles)
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) nqv[qb] = __shfl(nql, qb * 16 + i16);
  if (g == 0) {
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      const int q = wq0 + qb * 16 + i16;
      if (q < bd.q1) ubound[perm ? perm[q] : q] = U[qb] + nqv[qb];
    }
  }
  const int half = lane >> 5, rel = lane & 31;
#pragma unroll
  for (int L = 0; L < 32; ++L) {
    const int q = wq0 + 2 * L + half;
    if (q < bd.q1) {
      const int qo = perm ? perm[q] : q;
      const int jv = lj[L];
      cand_s[(int64_t)qo * KC + rel] = ls[L];
      cand_j[(int64_t)qo * KC + rel] = (perm && jv != 0x7FFFFFFF) ? perm[jv] : jv;
    }
  }
}

}  // namespace famst
