// Phase 1 of FAMST (Alg. 1, GetANNs): exact k nearest neighbours by
// matrix-core distance screening with a fused per-row top-k', float32
// direct-difference re-ranking and exact recomputation of rows the
// screening bound cannot certify.
#include <numeric>

#include "famst_common.hpp"
#include "prims.hpp"
#include "select.hpp"
#include "screen_regs.hpp"
#include "screen_v2.hpp"
#include "screen_hd.hpp"

namespace famst {

// ------------------------------------------------------------------ prep
// One wave per row: padded screening copy (float32 or bfloat16 RNE), its
// squared norm, the norm of the quantisation error and a non-finite flag.
// gstat[0] = non-finite flag, gstat[1] = max norm bits, gstat[2] = max
// quantisation error bits (non-negative floats order like their bits).
template <int PREC>
__global__ __launch_bounds__(256) void prep_kernel(const float* __restrict__ X, int64_t n, int d,
                                                   int DP, void* __restrict__ Xq,
                                                   float* __restrict__ nq, float* __restrict__ qerr,
                                                   unsigned* __restrict__ gstat) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned bad_any = 0, max_nq = 0, max_e = 0;   // meaningful in lane 0
  for (int64_t row = (int64_t)blockIdx.x * 4 + w; row < n; row += (int64_t)gridDim.x * 4) {
    const float* x = X + row * d;
    float acc = 0.f, eacc = 0.f;
    bool bad = false;
    for (int t = lane; t < DP; t += 64) {
      float v = t < d ? x[t] : 0.f;
      bad |= !__builtin_isfinite(v);
      float q;
      if (PREC == FAMST_FP32) {
        q = v;
        reinterpret_cast<float*>(Xq)[row * DP + t] = q;
      } else {
        uint16_t b = f32_to_bf16_rne(v);
        q = bf16_to_f32(b);
        reinterpret_cast<uint16_t*>(Xq)[row * DP + t] = b;
      }
      acc = __builtin_fmaf(q, q, acc);
      float e = q - v;
      eacc = __builtin_fmaf(e, e, eacc);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      acc += __shfl_xor(acc, o);
      eacc += __shfl_xor(eacc, o);
    }
    unsigned long long anybad = ballot(bad);
    if (lane == 0) {
      nq[row] = acc;
      // sqrt rounding and the float32 sum itself: inflate slightly
      float e = eacc > 0.f ? __builtin_sqrtf(eacc) * 1.0001f + 1e-30f : 0.f;
      qerr[row] = e;
      // squared norms must leave headroom: every screened value and every
      // float32 distance stays finite when they are below 1e37
      bad_any |= (anybad || !(acc <= 1e37f)) ? 1u : 0u;
      max_nq = max(max_nq, __float_as_uint(acc));
      max_e = max(max_e, __float_as_uint(e));
    }
  }
  // one set of atomics per block
  __shared__ unsigned red[3][4];
  if (lane == 0) {
    red[0][w] = bad_any;
    red[1][w] = max_nq;
    red[2][w] = max_e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned b = 0, m1 = 0, m2 = 0;
    for (int i = 0; i < 4; ++i) {
      b |= red[0][i];
      m1 = max(m1, red[1][i]);
      m2 = max(m2, red[2][i]);
    }
    if (b) atomicOr(&gstat[0], 1u);
    atomicMax(&gstat[1], m1);
    atomicMax(&gstat[2], m2);
  }
}

// Squared-distance screening of 64*QB queries per wave (4 waves per block)
// against 64-row tiles of the cloud, on the matrix cores:
//   acc(j, q) = x_j . x_q   (16x16 output blocks, db rows x queries)
//   s(j, q)   = |x_j|^2 + |x_q|^2 - 2 acc
// Each wave keeps, for each of its queries, the KC smallest (s, j) in an
// LDS list sorted ascending; a tile element reaches the insertion path only
// if s is within the list's current maximum.
// Insertion of the tile elements that pass the screening filter into the
// per-query sorted lists of one wave (lists at wl, [QW][KC]).  Lane
// (g, i16) holds, for query qb*16 + i16 of the wave, the 16 elements
// e = jb*4 + r at rows t0 + jb*16 + 4g + r; spf(qb, e) returns their
// screened value minus the query's norm.  Elements are pulled one at a time
// (wave-uniform); the whole wave inserts each into its query's list (a
// ballot gives the position, DPP wave_shr:1 shifts the tail).
template <int QB, int KC, class SpFn>
__device__ __forceinline__ void insert_candidates(Cand* wl, unsigned qbmask, float (&U)[QB],
                                                  const float (&nqq)[QB], SpFn spf, int t0, int c1,
                                                  int wq0, int lane, int g, int i16) {
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    if (!(qbmask & (1u << qb))) continue;
    const int q = wq0 + qb * 16 + i16;   // this lane's query in block qb
    f32x16 sp;
    unsigned pm = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      sp[e] = spf(qb, e);
      const int j = t0 + (e >> 2) * 16 + 4 * g + (e & 3);
      const bool ok = (sp[e] <= U[qb]) & (j < c1) & (j != q);
      pm |= (ok ? 1u : 0u) << e;
    }
    while (true) {
      const unsigned long long lanes = ballot(pm != 0);
      if (!lanes) break;
      const int src = __builtin_ctzll(lanes);
      const int e = __builtin_ctz((unsigned)readlane_i((int)pm, src));
      pm = (lane == src) ? (pm & (pm - 1)) : pm;
      const float v = sp[e];   // uniform index into a register vector
      const float spv = readlane_f(v, src);
      if (!(spv <= readlane_f(U[qb], src))) continue;   // list tightened meanwhile
      const int qi = qb * 16 + (src & 15);                 // query within wave
      const int j = t0 + (e >> 2) * 16 + 4 * (src >> 4) + (e & 3);
      const float s = spv + readlane_f(nqq[qb], src);
      Cand* L = wl + qi * KC;
      const Cand c = L[lane & (KC - 1)];
      const bool lt = (lane < KC) & ((c.s < s) | ((c.s == s) & (c.j < j)));
      const int pos = __builtin_popcountll(ballot(lt));
      if (pos >= KC) continue;
      // shift the tail up by one: lane l takes lane l-1's entry (DPP wave_shr:1)
      const float ups = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(c.s), 0x138, 0xF, 0xF, false));
      const int upj = __builtin_amdgcn_update_dpp(0, c.j, 0x138, 0xF, 0xF, false);
      Cand nc;
      nc.s = lane < pos ? c.s : (lane == pos ? s : ups);
      nc.j = lane < pos ? c.j : (lane == pos ? j : upj);
      if (lane < KC) L[lane] = nc;
      const float Tn = readlane_f(nc.s, KC - 1);
      // a few ulps of slack so rounding in U never hides an equal key
      const float Un = (Tn - readlane_f(nqq[qb], src)) + fabsf(Tn) * 2.4e-7f;
      U[qb] = (i16 == (src & 15)) ? Un : U[qb];
    }
  }
}

template <int PREC, int NKB, int QB, int KC>
__global__ __launch_bounds__(256, (NKB <= 4 ? 2 : 1)) void dist_topk_kernel(
    const void* __restrict__ Xq_, const float* __restrict__ nq, int DP, int nkb,
    const BlockDesc* __restrict__ desc, int* __restrict__ cand_j, float* __restrict__ cand_s) {
  using S = Scr<PREC>;
  using T = typename S::T;
  constexpr int QW = 16 * QB;           // queries per wave
  constexpr int QBLK = 4 * QW;          // queries per block
  constexpr int BN = 64;                // tile rows
  const T* Xq = reinterpret_cast<const T*>(Xq_);

  extern __shared__ __attribute__((aligned(16))) char smem[];
  // per-query lists of (s, j), ascending by (s, j): [QBLK][KC]
  Cand* lst = reinterpret_cast<Cand*>(smem);
  char* tile = reinterpret_cast<char*>(lst + QBLK * KC);    // [BN][DP*ESZ], 16-byte chunks swizzled
  const int RS = DP * S::ESZ;                               // row bytes
  const int cpr = RS / 16;                                  // 16-byte chunks per row (multiple of 4)
  // chunk c of row r lives at chunk c ^ (r & smask): the 16 rows read by one
  // lane group then fall in distinct bank groups
  const int smask = (cpr & 15) == 0 ? 15 : ((cpr & 7) == 0 ? 7 : 3);
  const int nchunk = BN * cpr;

  const BlockDesc bd = desc[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, i16 = lane & 15;
  const int wq0 = bd.q0 + wave * QW;   // first query of this wave

  // lists start as (+inf, INT_MAX)
  for (int e = tid; e < QBLK * KC; e += 256) lst[e] = Cand{F_INF, 0x7FFFFFFF};

  // resident query fragments
  i32x4 qf[QB][NKB];
  float nqq[QB], U[QB];
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    int q = wq0 + qb * 16 + i16;
    bool ok = q < bd.q1;
    nqq[qb] = ok ? nq[q] : 0.f;
    U[qb] = ok ? F_INF : -F_INF;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      i32x4 v = {0, 0, 0, 0};
      if (ok && kb < nkb) {
        const char* p = reinterpret_cast<const char*>(Xq + (int64_t)q * DP) +
                        (kb * S::KBW + g * (S::KBW / 4)) * S::ESZ;
        v = *reinterpret_cast<const i32x4*>(p);
      }
      qf[qb][kb] = v;
    }
  }

  // register prefetch of one tile: thread tid owns chunks tid + 256 i
  i32x4 pf[NKB];
  float pnq[4][4];   // norms of the rows this lane filters: t0 + jb*16 + 4g + r
  auto fetch = [&](int t0) {
    if (t0 + BN <= bd.c1) {   // full tile
#pragma unroll
      for (int i = 0; i < NKB; ++i) {
        int c = tid + 256 * i;
        i32x4 v = {0, 0, 0, 0};
        if (i < nkb) {
          int r = c / cpr, cc = c - r * cpr;
          v = *reinterpret_cast<const i32x4*>(reinterpret_cast<const char*>(Xq + (int64_t)(t0 + r) * DP) + cc * 16);
        }
        pf[i] = v;
      }
      const float* np = nq + t0 + 4 * g;
      if ((t0 & 3) == 0) {
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
          f32x4 v = *reinterpret_cast<const f32x4*>(np + jb * 16);
#pragma unroll
          for (int r = 0; r < 4; ++r) pnq[jb][r] = v[r];
        }
      } else {
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
          for (int r = 0; r < 4; ++r) pnq[jb][r] = np[jb * 16 + r];
      }
    } else {                  // ragged last tile
#pragma unroll
      for (int i = 0; i < NKB; ++i) {
        int c = tid + 256 * i;
        i32x4 v = {0, 0, 0, 0};
        if (c < nchunk) {
          int r = c / cpr, cc = c - r * cpr;
          int row = t0 + r;
          if (row < bd.c1)
            v = *reinterpret_cast<const i32x4*>(reinterpret_cast<const char*>(Xq + (int64_t)row * DP) + cc * 16);
        }
        pf[i] = v;
      }
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int row = t0 + jb * 16 + 4 * g + r;
          pnq[jb][r] = row < bd.c1 ? nq[row] : F_INF;
        }
    }
  };
  fetch(bd.c0);

  for (int t0 = bd.c0; t0 < bd.c1; t0 += BN) {
    // ---- publish the prefetched tile, then start fetching the next one
#pragma unroll
    for (int i = 0; i < NKB; ++i) {
      if (i < nkb) {   // chunk tid + 256 i exists iff i < nkb (64 rows x 4 nkb chunks)
        int c = tid + 256 * i;
        int r = c / cpr, cc = c - r * cpr;
        *reinterpret_cast<i32x4*>(tile + r * RS + ((cc ^ (r & smask)) << 4)) = pf[i];
      }
    }
    float nqj[4][4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) nqj[jb][r] = pnq[jb][r];
    __syncthreads();
    if (t0 + BN < bd.c1) fetch(t0 + BN);

    // ---- matrix-core products
    f32x4 acc[QB][4];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) acc[qb][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      if (kb < nkb) {
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
          const int r = jb * 16 + i16;
          const int cc = kb * 4 + g;
          i32x4 a = *reinterpret_cast<const i32x4*>(tile + r * RS + ((cc ^ (r & smask)) << 4));
#pragma unroll
          for (int qb = 0; qb < QB; ++qb) {
            if constexpr (PREC == FAMST_FP32) {
              f32x4 af = __builtin_bit_cast(f32x4, a);
              f32x4 bf = __builtin_bit_cast(f32x4, qf[qb][kb]);
              acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0], bf[0], acc[qb][jb], 0, 0, 0);
              acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1], bf[1], acc[qb][jb], 0, 0, 0);
              acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[2], bf[2], acc[qb][jb], 0, 0, 0);
              acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[3], bf[3], acc[qb][jb], 0, 0, 0);
            } else {
              bf16x8 af = __builtin_bit_cast(bf16x8, a);
              bf16x8 bf = __builtin_bit_cast(bf16x8, qf[qb][kb]);
              acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, acc[qb][jb], 0, 0, 0);
            }
          }
        }
      }
    }

    // ---- screening filter: lane holds rows t0 + jb*16 + 4g + r, query qb*16 + i16
    bool any = false;
    unsigned qbmask = 0;   // query blocks with at least one passing element (wave-uniform)
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      float m = F_INF;
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) m = fminf(m, __builtin_fmaf(-2.f, acc[qb][jb][r], nqj[jb][r]));
      const bool p = m <= U[qb];
      any |= p;
      qbmask |= ballot(p) ? (1u << qb) : 0u;
    }
    if (qbmask)
      insert_candidates<QB, KC>(lst + wave * QW * KC, qbmask, U, nqq,
                                [&](int qb, int e) {
                                  return __builtin_fmaf(-2.f, acc[qb][e >> 2][e & 3], nqj[e >> 2][e & 3]);
                                },
                                t0, bd.c1, wq0, lane, g, i16);
    __syncthreads();
  }

  // ---- write the candidate lists
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    for (int qq = 0; qq < 16; ++qq) {
      int qi = qb * 16 + qq;
      int q = wq0 + qi;
      if (q < bd.q1 && lane < KC) {
        Cand c = lst[(wave * QW + qi) * KC + lane];
        cand_s[(int64_t)q * KC + lane] = c.s;
        cand_j[(int64_t)q * KC + lane] = c.j;
      }
    }
  }
}

// --------------------------------------------- spatial order of the scan
// Every point (row of the screening copy) is assigned to the nearest of
// NPIV pivot rows (rows floor(i n / NPIV)) by screened squared distance
// |p|^2 - 2 x.p, ties to the smaller pivot; sorting by pivot groups nearby
// points, which only changes the order in which the screening visits rows.
// The pivots pass through LDS in chunks of 256.
#ifndef FAMST_NPIV
#define FAMST_NPIV 1024
#endif
constexpr int NPIV = FAMST_NPIV, PCH = 256;
// The streamed screening takes the spatial order for rows of at most this
// many bytes (0: never).  Where the filter and the insertion weigh most
// (short rows) the early tight thresholds pay; on long rows the blocks that
// scan the tiles in the same order share them in L2, which pays more
// (500K x 960 bf16: 470 ms in index order, 490 ms in spatial order; 1M x
// 128 float8: 341 ms against 262 ms).
#ifndef FAMST_HD_SPATIAL_MAXB
#define FAMST_HD_SPATIAL_MAXB 1024
#endif
constexpr int NPIV_BITS = NPIV <= 256 ? 8 : (NPIV <= 1024 ? 10 : (NPIV <= 4096 ? 12 : 16));

template <int PREC, int NKB>
__global__ __launch_bounds__(256) void pivot_assign_kernel(const void* __restrict__ Xq_,
                                                           const float* __restrict__ nq, int n,
                                                           uint32_t* __restrict__ key,
                                                           int* __restrict__ idx) {
  constexpr int QB = 4, RS = NKB * 64, cpr = NKB * 4;
  constexpr int smask = (cpr & 15) == 0 ? 15 : ((cpr & 7) == 0 ? 7 : 3);
  const char* Xb = reinterpret_cast<const char*>(Xq_);
  extern __shared__ __attribute__((aligned(16))) char smem[];
  float* pn = reinterpret_cast<float*>(smem + PCH * RS);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, i16 = lane & 15;
  const int wq0 = blockIdx.x * 256 + wave * 64;
  i32x4 qf[QB][NKB];
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int q = wq0 + qb * 16 + i16;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
      qf[qb][kb] = q < n ? *reinterpret_cast<const i32x4*>(Xb + (int64_t)q * RS + kb * 64 + g * 16)
                         : i32x4{0, 0, 0, 0};
  }
  float best[QB];
  int bi[QB];
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    best[qb] = F_INF;
    bi[qb] = 0;
  }
  for (int p0 = 0; p0 < NPIV; p0 += PCH) {
    __syncthreads();   // the previous chunk is consumed
    for (int c = tid; c < PCH * cpr; c += 256) {
      const int r = c / cpr, sc = c - r * cpr;
      const int64_t prow = (int64_t)(p0 + r) * n / NPIV;
      *reinterpret_cast<i32x4*>(smem + r * RS + ((sc ^ (r & smask)) << 4)) =
          *reinterpret_cast<const i32x4*>(Xb + prow * RS + sc * 16);
    }
    for (int r = tid; r < PCH; r += 256) pn[r] = nq[(int64_t)(p0 + r) * n / NPIV];
    __syncthreads();
    for (int pt = 0; pt < PCH / 64; ++pt) {
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        f32x4 acc[QB];
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) acc[qb] = f32x4{0.f, 0.f, 0.f, 0.f};
        const int r = pt * 64 + jb * 16 + i16;
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) {
          const int cc = kb * 4 + g;
          const i32x4 a = *reinterpret_cast<const i32x4*>(smem + r * RS + ((cc ^ (r & smask)) << 4));
#pragma unroll
          for (int qb = 0; qb < QB; ++qb) {
            if constexpr (PREC == FAMST_FP32) {
              const f32x4 af = __builtin_bit_cast(f32x4, a);
              const f32x4 bf = __builtin_bit_cast(f32x4, qf[qb][kb]);
              acc[qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0], bf[0], acc[qb], 0, 0, 0);
              acc[qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1], bf[1], acc[qb], 0, 0, 0);
              acc[qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[2], bf[2], acc[qb], 0, 0, 0);
              acc[qb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[3], bf[3], acc[qb], 0, 0, 0);
            } else {
              acc[qb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  __builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, qf[qb][kb]), acc[qb], 0, 0, 0);
            }
          }
        }
        // lane holds pivots p0 + pt*64 + jb*16 + 4g + rr for its query qb*16 + i16
#pragma unroll
        for (int qb = 0; qb < QB; ++qb)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int pl = pt * 64 + jb * 16 + 4 * g + rr;
            const float v = __builtin_fmaf(-2.f, acc[qb][rr], pn[pl]);
            if (v < best[qb]) {   // pivots are visited in ascending order per lane
              best[qb] = v;
              bi[qb] = p0 + pl;
            }
          }
      }
    }
  }
  // combine the four lane groups of each query (smaller value, then smaller pivot)
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
#pragma unroll
    for (int o = 16; o <= 32; o <<= 1) {
      const float ov = __shfl_xor(best[qb], o);
      const int oi = __shfl_xor(bi[qb], o);
      if (ov < best[qb] || (ov == best[qb] && oi < bi[qb])) {
        best[qb] = ov;
        bi[qb] = oi;
      }
    }
    const int q = wq0 + qb * 16 + i16;
    if (g == 0 && q < n) {
      key[q] = (uint32_t)bi[qb];
      idx[q] = q;
    }
  }
}

// Permuted copies of the screening rows, norms, rounding norms and (float8)
// row scales (scl null: none).
__global__ __launch_bounds__(256) void gather_rows_kernel(const char* __restrict__ Xq, int RS,
                                                          const float* __restrict__ nq,
                                                          const float* __restrict__ qerr,
                                                          const float* __restrict__ scl,
                                                          const int* __restrict__ perm, int64_t n,
                                                          char* __restrict__ Xp, float* __restrict__ nqp,
                                                          float* __restrict__ qerrp,
                                                          float* __restrict__ sclp) {
  const int cpr = RS / 16;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n * cpr) return;
  const int64_t q = c / cpr;
  const int sc = (int)(c - q * cpr);
  const int src = perm[q];
  *reinterpret_cast<i32x4*>(Xp + q * RS + sc * 16) =
      *reinterpret_cast<const i32x4*>(Xq + (int64_t)src * RS + sc * 16);
  if (sc == 0) {
    nqp[q] = nq[src];
    qerrp[q] = qerr[src];
    if (scl) sclp[q] = scl[src];
  }
}

// Pivot-assignment input for the streamed screening (rows of any length, any
// precision): a 128-coordinate bf16 sketch of each row, coordinate i added
// with sign sg(i) into slot i mod 128 (a sparse random projection; the row
// itself for d <= 128), and the squared norm of the rounded sketch.  It only
// decides the order in which the screening visits the rows.  One wave per row.
__global__ __launch_bounds__(256) void sketch_kernel(const float* __restrict__ X, int64_t n, int d,
                                                     uint16_t* __restrict__ S, float* __restrict__ ns) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  auto sg = [d](int i, float v) {   // top bit of a multiplicative hash of i
    return (d > 128 && ((uint32_t)i * 0x9E3779B1u) >> 31) ? -v : v;
  };
  for (int64_t row = (int64_t)blockIdx.x * 4 + w; row < n; row += (int64_t)gridDim.x * 4) {
    const float* x = X + row * d;
    float s0 = 0.f, s1 = 0.f;
    for (int i0 = 0; i0 < d; i0 += 128) {
      const int i = i0 + lane, j = i0 + 64 + lane;
      if (i < d) s0 += sg(i, x[i]);
      if (j < d) s1 += sg(j, x[j]);
    }
    const uint16_t b0 = f32_to_bf16_rne(s0), b1 = f32_to_bf16_rne(s1);
    S[row * 128 + lane] = b0;
    S[row * 128 + 64 + lane] = b1;
    const float v0 = bf16_to_f32(b0), v1 = bf16_to_f32(b1);
    float t = v0 * v0 + v1 * v1;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
    if (lane == 0) ns[row] = t;
  }
}

// ------------------------------------------------ K-chunked screening
// For any d and for float8: the cloud is streamed in 64-row tiles and the
// dimension in 256-byte chunks; both the tile chunk and the block's query
// chunk are staged in LDS (16-byte chunks XOR-swizzled by row), so no
// operand has to stay resident in registers.  128 queries per block, 32 per
// wave; the filter and the insertion path are those of dist_topk_kernel.

// IEEE float32 -> OCP float8 e4m3 (bias 7, max 448, no infinities), round
// to nearest even, saturating at +-448.
__device__ __forceinline__ uint32_t f32_to_e4m3(float v) {
  const uint32_t sign = v < 0.f ? 0x80u : 0u;
  const float a = fabsf(v);
  if (!(a < 448.f)) return sign | 0x7Eu;
  int e;
  frexpf(a, &e);
  int E = e - 1;                     // floor(log2 a) for a > 0
  if (a == 0.f || E < -6) E = -6;    // subnormal spacing 2^-9
  const float step = ldexpf(1.f, E - 3);
  const float qv = rintf(a / step) * step;
  if (qv == 0.f) return sign;
  int e2;
  frexpf(qv, &e2);
  const int E2 = e2 - 1;
  if (E2 < -6) return sign | (uint32_t)(qv * 512.f);          // m * 2^-9
  const uint32_t mant = (uint32_t)(qv / ldexpf(1.f, E2 - 3)) - 8u;
  return sign | ((uint32_t)(E2 + 7) << 3) | mant;
}

__device__ __forceinline__ float e4m3_to_f32(uint32_t b) {
  const uint32_t ex = (b >> 3) & 15u, m = b & 7u;
  const float mag = ex == 0 ? (float)m * 0.001953125f : ldexpf((float)(8u + m), (int)ex - 10);
  return (b & 0x80u) ? -mag : mag;
}

// One wave per row: per-row scale a = the power of two at or above
// amax / 448 (1 for an all-zero row; at least 2^-126, so that its exponent
// byte is its E8M0 encoding and the matrix cores can apply it), e4m3 codes
// of x / a (every |x / a| <= 448), the norm of the dequantised row and the
// norm of its error; gstat as in prep_kernel.
__global__ __launch_bounds__(256) void prep_fp8_kernel(const float* __restrict__ X, int64_t n, int d,
                                                       int DP, uint8_t* __restrict__ Xq,
                                                       float* __restrict__ scl, float* __restrict__ nq,
                                                       float* __restrict__ qerr,
                                                       unsigned* __restrict__ gstat) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  unsigned bad_any = 0, max_nq = 0, max_e = 0;
  for (int64_t row = (int64_t)blockIdx.x * 4 + w; row < n; row += (int64_t)gridDim.x * 4) {
    const float* x = X + row * d;
    float amax = 0.f;
    bool bad = false;
    for (int t = lane; t < d; t += 64) {
      float v = x[t];
      bad |= !__builtin_isfinite(v);
      amax = fmaxf(amax, fabsf(v));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
    float a = 1.f;
    if (amax > 0.f) {
      int e;
      const float m = frexpf(amax / 448.f, &e);   // amax / 448 = m 2^e, m in [0.5, 1)
      a = ldexpf(1.f, m == 0.5f ? e - 1 : e);
      a = fmaxf(a, 1.17549435e-38f);              // 2^-126
    }
    float acc = 0.f, eacc = 0.f;
    for (int t = lane; t < DP; t += 64) {
      float v = t < d ? x[t] : 0.f;
      uint32_t code = f32_to_e4m3(v / a);
      Xq[row * DP + t] = (uint8_t)code;
      float dq = a * e4m3_to_f32(code);
      acc = __builtin_fmaf(dq, dq, acc);
      float er = dq - v;
      eacc = __builtin_fmaf(er, er, eacc);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      acc += __shfl_xor(acc, o);
      eacc += __shfl_xor(eacc, o);
    }
    unsigned long long anybad = ballot(bad);
    if (lane == 0) {
      nq[row] = acc;
      scl[row] = a;
      float e = eacc > 0.f ? __builtin_sqrtf(eacc) * 1.0001f + 1e-30f : 0.f;
      qerr[row] = e;
      // squared norms must leave headroom: every screened value and every
      // float32 distance stays finite when they are below 1e37
      bad_any |= (anybad || !(acc <= 1e37f)) ? 1u : 0u;
      max_nq = max(max_nq, __float_as_uint(acc));
      max_e = max(max_e, __float_as_uint(e));
    }
  }
  __shared__ unsigned red[3][4];
  if (lane == 0) {
    red[0][w] = bad_any;
    red[1][w] = max_nq;
    red[2][w] = max_e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned b = 0, m1 = 0, m2 = 0;
    for (int i = 0; i < 4; ++i) {
      b |= red[0][i];
      m1 = max(m1, red[1][i]);
      m2 = max(m2, red[2][i]);
    }
    if (b) atomicOr(&gstat[0], 1u);
    atomicMax(&gstat[1], m1);
    atomicMax(&gstat[2], m2);
  }
}

template <int PREC>
struct KcT;
template <>
struct KcT<FAMST_FP32> {
  static constexpr int ESZ = 4, FB = 16;   // FB: bytes of one operand fragment per lane
};
template <>
struct KcT<FAMST_BF16> {
  static constexpr int ESZ = 2, FB = 16;
};
template <>
struct KcT<FAMST_FP8_E4M3> {
  static constexpr int ESZ = 1, FB = 32;
};
constexpr int KCH = 256;   // bytes of a row per K chunk

template <int PREC, int KC>
__global__ __launch_bounds__(256, (KC == 32 ? 2 : 1)) void dist_topk_kc_kernel(
    const void* __restrict__ Xq_, const float* __restrict__ nq, const float* __restrict__ scl, int DP,
    const BlockDesc* __restrict__ desc, int* __restrict__ cand_j, float* __restrict__ cand_s) {
  using T = KcT<PREC>;
  constexpr int QB = 2, QW = 32, QBLK = 128, BN = 64;
  constexpr int NKBC = KCH / (4 * T::FB);   // k-blocks per chunk
  constexpr int CPR = KCH / 16;             // 16-byte chunks per staged row
  const char* Xq = reinterpret_cast<const char*>(Xq_);
  const int RB = DP * T::ESZ;               // bytes per row in HBM
  const int nch = RB / KCH;                 // K chunks

  extern __shared__ __attribute__((aligned(16))) char smem[];
  Cand* lst = reinterpret_cast<Cand*>(smem);                 // [QBLK][KC]
  char* tq = reinterpret_cast<char*>(lst + QBLK * KC);        // [QBLK][KCH] query chunk
  char* tt = tq + QBLK * KCH;                                 // [BN][KCH] tile chunk

  const BlockDesc bd = desc[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, i16 = lane & 15;
  const int wq0 = bd.q0 + wave * QW;
  for (int e = tid; e < QBLK * KC; e += 256) lst[e] = Cand{F_INF, 0x7FFFFFFF};
  float nqq[QB], U[QB], aq[QB];
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    int q = wq0 + qb * 16 + i16;
    bool ok = q < bd.q1;
    nqq[qb] = ok ? nq[q] : 0.f;
    U[qb] = ok ? F_INF : -F_INF;
    aq[qb] = (PREC == FAMST_FP8_E4M3 && ok) ? scl[q] : 1.f;
  }
  __syncthreads();

  for (int t0 = bd.c0; t0 < bd.c1; t0 += BN) {
    f32x4 acc[QB][4];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) acc[qb][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ch = 0; ch < nch; ++ch) {
      // stage the query chunk (128 rows) and the tile chunk (64 rows)
      for (int c = tid; c < (QBLK + BN) * CPR; c += 256) {
        int r = c / CPR, cc = c - r * CPR;
        int64_t row;
        bool ok;
        char* dst;
        if (r < QBLK) {
          row = bd.q0 + r;
          ok = row < bd.q1;
          dst = tq + r * KCH + ((cc ^ (r & 15)) << 4);
        } else {
          int rr = r - QBLK;
          row = t0 + rr;
          ok = row < bd.c1;
          dst = tt + rr * KCH + ((cc ^ (rr & 15)) << 4);
        }
        i32x4 v = {0, 0, 0, 0};
        if (ok) v = *reinterpret_cast<const i32x4*>(Xq + row * RB + (int64_t)ch * KCH + cc * 16);
        *reinterpret_cast<i32x4*>(dst) = v;
      }
      __syncthreads();
#pragma unroll
      for (int kb = 0; kb < NKBC; ++kb) {
        const int c0 = (kb * 4 * T::FB + g * T::FB) >> 4;   // first 16-byte chunk of this lane's fragment
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
          const int ra = jb * 16 + i16;
          if constexpr (T::FB == 16) {
            i32x4 a = *reinterpret_cast<const i32x4*>(tt + ra * KCH + ((c0 ^ (ra & 15)) << 4));
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) {
              const int rq = wave * QW + qb * 16 + i16;
              i32x4 b = *reinterpret_cast<const i32x4*>(tq + rq * KCH + ((c0 ^ (rq & 15)) << 4));
              if constexpr (PREC == FAMST_FP32) {
                f32x4 af = __builtin_bit_cast(f32x4, a), bf = __builtin_bit_cast(f32x4, b);
                acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0], bf[0], acc[qb][jb], 0, 0, 0);
                acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1], bf[1], acc[qb][jb], 0, 0, 0);
                acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[2], bf[2], acc[qb][jb], 0, 0, 0);
                acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[3], bf[3], acc[qb][jb], 0, 0, 0);
              } else {
                acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), acc[qb][jb], 0, 0, 0);
              }
            }
          } else {
            i32x4 a0 = *reinterpret_cast<const i32x4*>(tt + ra * KCH + ((c0 ^ (ra & 15)) << 4));
            i32x4 a1 = *reinterpret_cast<const i32x4*>(tt + ra * KCH + (((c0 + 1) ^ (ra & 15)) << 4));
            i32x8 a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) {
              const int rq = wave * QW + qb * 16 + i16;
              i32x4 b0 = *reinterpret_cast<const i32x4*>(tq + rq * KCH + ((c0 ^ (rq & 15)) << 4));
              i32x4 b1 = *reinterpret_cast<const i32x4*>(tq + rq * KCH + (((c0 + 1) ^ (rq & 15)) << 4));
              i32x8 b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
              acc[qb][jb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[qb][jb], 0, 0, 0, 127, 0, 127);
            }
          }
        }
      }
      __syncthreads();
    }
    // filter: rows t0 + jb*16 + 4g + r of this lane
    float nqj[4][4], cj[4][4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = t0 + jb * 16 + 4 * g + r;
        bool ok = row < bd.c1;
        nqj[jb][r] = ok ? nq[row] : F_INF;
        cj[jb][r] = -2.f * ((PREC == FAMST_FP8_E4M3 && ok) ? scl[row] : 1.f);
      }
    unsigned qbmask = 0;
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      float m = F_INF;
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) m = fminf(m, __builtin_fmaf(cj[jb][r] * aq[qb], acc[qb][jb][r], nqj[jb][r]));
      qbmask |= ballot(m <= U[qb]) ? (1u << qb) : 0u;
    }
    if (qbmask)
      insert_candidates<QB, KC>(lst + wave * QW * KC, qbmask, U, nqq,
                                [&](int qb, int e) {
                                  return __builtin_fmaf(cj[e >> 2][e & 3] * aq[qb], acc[qb][e >> 2][e & 3],
                                                        nqj[e >> 2][e & 3]);
                                },
                                t0, bd.c1, wq0, lane, g, i16);
  }
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    for (int qq = 0; qq < 16; ++qq) {
      int qi = qb * 16 + qq;
      int q = wq0 + qi;
      if (q < bd.q1 && lane < KC) {
        Cand c = lst[(wave * QW + qi) * KC + lane];
        cand_s[(int64_t)q * KC + lane] = c.s;
        cand_j[(int64_t)q * KC + lane] = c.j;
      }
    }
  }
}

// ------------------------------------------------------------- re-rank
// One wave per row (rows taken with a stride of the grid): direct-difference
// float32 distances of the KC
// candidates, selection of the k smallest by (s, j) with float64 at a
// near-tie boundary, and the certificate that no non-candidate is closer.
struct RerankArgs {
  const float* X;
  int64_t n;
  int d;
  const int64_t* offs;
  int B;
  int k, KC;
  const int* cand_j;
  const float* cand_s;
  const float* nq;
  const float* qerr;
  const unsigned* gstat;
  float arith_c;          // screening arithmetic error factor (x 2^-24 folded in)
  const float* ubound;    // per-query bound of the rejected screened values (or null)
  const int* order;       // block i re-ranks row order[i] (null: row i); the spatial order
                          // of the screening, so that neighbouring blocks gather the same rows
  int* nbr;
  float* dist;
  float* kth_s;           // s of the k-th selected (for recomputation)
  int64_t* bad_flag;      // per row: 1 if not certified (listed afterwards by a scan)
  unsigned long long* counters;  // [1] recomputed, [2] near ties
};

__global__ __launch_bounds__(64) void rerank_kernel(RerankArgs a) {
  __shared__ SelectSmem<64> sm;
  __shared__ int invalid;
  const int t = threadIdx.x;
  for (int64_t qi = blockIdx.x; qi < a.n; qi += gridDim.x) {
  const int64_t q = a.order ? (int64_t)a.order[qi] : qi;
  const int cb = find_cloud(a.offs, a.B, q);
  const int64_t nb = a.offs[cb + 1] - a.offs[cb];
  const int Lmax = (int)min<int64_t>(a.KC, nb - 1);
  const float* xq = a.X + q * a.d;
  const float tau = tau32(a.d);
  const int64_t c0 = a.offs[cb];
  // slots the screening never filled hold (+inf, INT_MAX) and sort last
  const int jraw = t < Lmax ? a.cand_j[q * a.KC + t] : 0x7FFFFFFF;
  int L = __builtin_popcountll(ballot(jraw != 0x7FFFFFFF));
  if (t == 0) invalid = 0;
  __syncthreads();
  const int need = (int)min<int64_t>(a.k, nb - 1);
  if (t < max(L, need)) {
    // an id outside the cloud (or too few candidates) is reported: the row is
    // then uncertified, and the id is replaced so that nothing reads out of
    // bounds
    int j = t < L ? jraw : -1;
    if (j < c0 || j >= c0 + nb || j == q) {
      invalid = 1;
      j = q == c0 ? (int)c0 + 1 : (int)c0;
    }
    sm.id[t] = j;
  }
  L = max(L, need);
  __syncthreads();
  const int grp = t >> 4, r16 = t & 15;
  for (int c = grp; c < L; c += 4) {
    float v = sq32_group(xq, a.X + (int64_t)sm.id[c] * a.d, a.d, r16);
    if (r16 == 0) sm.s[c] = v;
  }
  __syncthreads();
  bool tie = block_select<64, 64>(sm, L, a.k, tau, a.d, [&](int i, const float** pa, const float** pb) {
    *pa = xq;
    *pb = a.X + (int64_t)sm.id[i] * a.d;
  });
  float kth = 0.f;
  if (t < L && sm.pos[t] >= 0) {
    a.nbr[q * a.k + sm.pos[t]] = sm.id[t];
    a.dist[q * a.k + sm.pos[t]] = __builtin_sqrtf(sm.s[t]);
    kth = sm.s[t];
  }
  for (int o = 32; o >= 1; o >>= 1) kth = fmaxf(kth, __shfl_xor(kth, o));
  if (t == 0) {
    a.kth_s[q] = kth;
    if (tie) atomicAdd(&a.counters[2], 1ull);
    bool cert = true;
    if (nb - 1 > L) {
      // every non-candidate j has screened value >= S': the list maximum, or
      // the filter bound of the screening kernel when it reports one
      float Sp = a.cand_s[q * a.KC + a.KC - 1];
      if (a.ubound) Sp = fminf(Sp, a.ubound[q]);
      float nmax = __uint_as_float(a.gstat[1]);
      float emax = __uint_as_float(a.gstat[2]);
      float eps = a.arith_c * (a.nq[q] + nmax);
      float lb_scr = Sp - eps;
      float root = lb_scr > 0.f ? __builtin_sqrtf(lb_scr) * (1.0f - 1e-6f) : 0.f;
      float rr = root - (a.qerr[q] + emax);
      float lb = rr > 0.f ? rr * rr * (1.0f - 1e-6f) : 0.f;
      cert = lb > kth * (1.0f + 2.0f * tau);
    }
    a.bad_flag[q] = (!cert || invalid) ? 1 : 0;
  }
  __syncthreads();   // the next row reuses the LDS lists
  }
}

// The uncertified rows, in ascending order, at their exclusive-scan
// positions (a shared counter would serialise on one address when most
// rows are uncertified, as with float8 screening in approximate mode).
__global__ __launch_bounds__(256) void list_flagged_kernel(const int64_t* __restrict__ flag,
                                                          const int64_t* __restrict__ pos, int64_t n,
                                                          int* __restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && flag[i]) rows[pos[i]] = (int)i;
}

// Exact recomputation of a row: collect every point whose float32 distance
// is within the bound of the current k-th, then select as above.  When more
// than FB_CAP points lie under that bound (the screened candidates were far
// from the true neighbours), the k-th smallest float32 distance of the row is
// found exactly by a radix select over its bits (squared distances are
// nonnegative, so their bit patterns order like the values: three histogram
// passes of 11, 11 and 10 bits, with sm.rank as the 2048 bins), and the
// points are collected again under that value's near-tie bound.
constexpr int FB_CAP = 2048;

__device__ __forceinline__ float row_kth_radix(SelectSmem<FB_CAP>& sm, const float* __restrict__ X, int d,
                                               const float* __restrict__ xq, int64_t q, int64_t c0,
                                               int64_t c1, int k) {
  const int t = threadIdx.x, grp = t >> 4, r16 = t & 15;
  uint32_t prefix = 0, pmask = 0;
  int rem = k;   // rank of the wanted value among those matching the prefix (1-based)
  const int shifts[3] = {21, 10, 0}, widths[3] = {11, 11, 10};
  for (int pass = 0; pass < 3; ++pass) {
    const int sh = shifts[pass];
    const uint32_t dmask = (1u << widths[pass]) - 1u;
    for (int b = t; b < FB_CAP; b += 256) sm.rank[b] = 0;
    __syncthreads();
    for (int64_t j0 = c0; j0 < c1; j0 += 16) {
      const int64_t j = j0 + grp;
      if (j < c1 && j != q) {
        const uint32_t bits = __float_as_uint(sq32_group(xq, X + j * d, d, r16));
        if (r16 == 0 && (bits & pmask) == prefix) atomicAdd(&sm.rank[(bits >> sh) & dmask], 1);
      }
    }
    __syncthreads();
    if (t == 0) {
      int cum = 0, sel = (int)dmask;
      for (int b = 0; b <= (int)dmask; ++b) {
        if (cum + sm.rank[b] >= rem) {
          sel = b;
          break;
        }
        cum += sm.rank[b];
      }
      sm.cnt[2] = sel;
      sm.cnt[3] = rem - cum;
    }
    __syncthreads();
    prefix |= (uint32_t)sm.cnt[2] << sh;
    pmask |= dmask << sh;
    rem = sm.cnt[3];
    __syncthreads();
  }
  return __uint_as_float(prefix);
}

__global__ __launch_bounds__(256) void exact_row_kernel(const float* __restrict__ X, int d,
                                                        const int64_t* __restrict__ offs, int B,
                                                        int k, const int* __restrict__ rows,
                                                        const float* __restrict__ kth_s,
                                                        int* __restrict__ nbr, float* __restrict__ dist,
                                                        unsigned long long* __restrict__ counters,
                                                        int* __restrict__ overflow, int64_t nrows) {
  __shared__ SelectSmem<FB_CAP> sm;
  __shared__ int cnt;
  const int t = threadIdx.x, grp = t >> 4, r16 = t & 15;
  for (int64_t ri = blockIdx.x; ri < nrows; ri += gridDim.x) {
  const int64_t q = rows[ri];
  const int cb = find_cloud(offs, B, q);
  const int64_t c0 = offs[cb], c1 = offs[cb + 1];
  const float tau = tau32(d);
  const float up2 = (1.0f + 2.0f * tau) * (1.0f + 2.0f * tau);
  float T = kth_s[q] * up2;
  const float* xq = X + q * d;
  int L = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (t == 0) cnt = 0;
    __syncthreads();
    for (int64_t j0 = c0; j0 < c1; j0 += 16) {
      int64_t j = j0 + grp;
      float v = F_INF;
      if (j < c1 && j != q) v = sq32_group(xq, X + j * d, d, r16);
      if (r16 == 0 && v <= T) {
        int p = atomicAdd(&cnt, 1);
        if (p < FB_CAP) {
          sm.s[p] = v;
          sm.id[p] = (int)j;
        }
      }
    }
    __syncthreads();
    L = cnt;   // uniform: every thread reads the same count
    __syncthreads();
    if (L <= FB_CAP || attempt == 1) break;
    T = row_kth_radix(sm, X, d, xq, q, c0, c1, k) * up2;
  }
  if (L > FB_CAP) {   // more than FB_CAP points within rounding of the k-th
    if (t == 0) atomicOr(overflow, 1);
  } else {
    block_select<256, FB_CAP>(sm, L, k, tau, d, [&](int i, const float** pa, const float** pb) {
      *pa = xq;
      *pb = X + (int64_t)sm.id[i] * d;
    });
    for (int i = t; i < L; i += 256) {
      if (sm.pos[i] >= 0) {
        nbr[q * k + sm.pos[i]] = sm.id[i];
        dist[q * k + sm.pos[i]] = __builtin_sqrtf(sm.s[i]);
      }
    }
    if (t == 0) atomicAdd(&counters[1], 1ull);
  }
  __syncthreads();   // the next row resets the count and reuses the LDS lists
  }
}

// --------------------------------------------------------------- host side
struct KnnPlan {
  int prec, KC, DP, nkb, QB, qblk, esz;
  int nw;         // waves per block of the pipelined kernel
  bool chunked;   // K-chunked kernel (any d, float8) instead of resident queries
  bool piped;     // register lists + pipelined tiles (k' = 32, up to 128 bf16 / 64 fp32 dims)
  bool hd;        // register lists, queries and rows streamed by K-steps (k' = 32, beyond 128 dims)
  bool buffered;  // pipelined kernel with buffered list updates (short scans, up to two K-blocks)
  size_t lds;
};

// Zero rows past the end of the screening copy, its norms and scales: at
// least the largest tile or query block a screening kernel reads whole.
constexpr int PADR = 256;
static_assert(HdShape<4>::BN <= PADR && HdShape<8>::BN <= PADR && hd_qblk<4>() <= PADR && hd_qblk<8>() <= PADR &&
                  V2Shape<8>::BN <= PADR,
              "padding covers every streamed tile and query block");

// Spatial order of the scan for one cloud from this many points: the early
// tight thresholds cut the list insertions (10K x 32 blobs: the screening
// 4.8 -> 2.0 ms in float32, 7.0 -> 2.6 ms in bf16).  Not for batches: with
// pivots per cloud the 256 clouds of 64-dimensional Gaussian clusters took
// 32.8 ms against 22.9 ms in index order.
static constexpr int64_t SPATIAL_MIN = 4096;

// Eight-wave blocks of the pipelined kernel from this many rows of one cloud
// on: they halve the rows streamed per query, which pays where the stream is
// longest (4M x 96: 9 % faster) but not at 1M x 128 (15 % slower: the wider
// barrier leaves a compute unit idle more often)
static constexpr int64_t V2_WIDE_MIN = 2097152;
// Largest cloud whose screening scan buffers its list updates: on longer
// scans under a spatial order few rows pass after the first tiles, and single
// insertions cost less than the buffered loop (1M x 32 bf16: 119.5 against
// 130.8 ms; 200K x 32: 10.6 against 10.8 ms; 10K x 32: 1.29 against 1.80 ms).
static constexpr int64_t V2_BUF_MAX_ROWS = 32768;

static int choose_plan(int prec, int d, int k, int k_cand, int64_t nmax, KnnPlan& p) {
  p.nw = 4;
  p.prec = prec;
  p.KC = k_cand ? k_cand : (k <= 24 ? 32 : 64);
  if (p.KC != 32 && p.KC != 64) return FAMST_EINVAL;
  if (p.KC < k) return FAMST_EINVAL;
  p.esz = prec == FAMST_FP32 ? 4 : (prec == FAMST_BF16 ? 2 : 1);
  const int kbw = prec == FAMST_FP32 ? 16 : 32;
  p.nkb = (d + kbw - 1) / kbw;
  p.chunked = prec == FAMST_FP8_E4M3 || p.nkb > 8;
  p.piped = false;
  p.hd = false;
  p.buffered = false;
  // beyond the register-resident queries (for float32 beyond 64 dims, where
  // the streamed operands cost less than the LDS-list kernel's waits; for
  // float8 at any d)
  if (p.KC == 32 && (prec == FAMST_FP8_E4M3 || d > 128 || (prec == FAMST_FP32 && d > 64))) {
    const int kdim = (prec == FAMST_FP32 ? HdShape<4>::KSB : HdShape<8>::KSB) / p.esz;   // dims per stage
    p.chunked = false;
    p.hd = true;
    p.DP = (d + kdim - 1) / kdim * kdim;
    p.QB = 4;
    p.qblk = prec == FAMST_FP32 ? hd_qblk<4>() : hd_qblk<8>();
    p.lds = prec == FAMST_FP32 ? hd_lds_bytes<4>() : hd_lds_bytes<8>();
  } else if (!p.chunked) {
    p.DP = p.nkb * kbw;
    p.QB = (p.KC == 64) ? 2 : 4;
    p.qblk = 64 * p.QB;
    p.lds = (size_t)p.qblk * p.KC * 8 + (size_t)64 * p.DP * p.esz;
    if (p.KC == 32 && p.nkb <= 4) {
      p.piped = true;
      p.nw = nmax >= V2_WIDE_MIN ? 8 : 4;
      p.buffered = p.nw == 4 && p.nkb <= 2 && nmax <= V2_BUF_MAX_ROWS;
      p.qblk = 64 * p.nw;
      p.lds = p.nw == 8 ? v2_lds_bytes<8>(p.nkb) : v2_lds_bytes<4>(p.nkb);
    }
  } else {
    const int cdim = KCH / p.esz;               // dims per K chunk
    p.DP = (d + cdim - 1) / cdim * cdim;
    p.QB = 2;
    p.qblk = 128;
    p.lds = (size_t)p.qblk * p.KC * 8 + (size_t)(128 + 64) * KCH;
  }
  if (p.lds > 160 * 1024) return FAMST_ENOTIMPL;
  return FAMST_OK;
}

template <int PREC, int KC>
static int launch_kc(const KnnPlan& p, int nblk, hipStream_t s, const void* Xq, const float* nq,
                     const float* scl, const BlockDesc* desc, int* cj, float* cs) {
  auto kern = dist_topk_kc_kernel<PREC, KC>;
  static bool attr = false;
  if (!attr) {
    FAMST_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr = true;
  }
  return launch("dist_topk", kern, dim3(nblk), dim3(256), p.lds, s, Xq, nq, scl, p.DP, desc, cj, cs);
}

static int dispatch_kc(const KnnPlan& p, int nblk, hipStream_t s, const void* Xq, const float* nq,
                       const float* scl, const BlockDesc* desc, int* cj, float* cs) {
  if (p.prec == FAMST_FP32)
    return p.KC == 32 ? launch_kc<FAMST_FP32, 32>(p, nblk, s, Xq, nq, scl, desc, cj, cs)
                      : launch_kc<FAMST_FP32, 64>(p, nblk, s, Xq, nq, scl, desc, cj, cs);
  if (p.prec == FAMST_BF16)
    return p.KC == 32 ? launch_kc<FAMST_BF16, 32>(p, nblk, s, Xq, nq, scl, desc, cj, cs)
                      : launch_kc<FAMST_BF16, 64>(p, nblk, s, Xq, nq, scl, desc, cj, cs);
  return p.KC == 32 ? launch_kc<FAMST_FP8_E4M3, 32>(p, nblk, s, Xq, nq, scl, desc, cj, cs)
                    : launch_kc<FAMST_FP8_E4M3, 64>(p, nblk, s, Xq, nq, scl, desc, cj, cs);
}

template <int PREC, int NKB, int QB, int KC>
static int launch_dt(const KnnPlan& p, int nblk, hipStream_t s, const void* Xq, const float* nq,
                     const BlockDesc* desc, int* cj, float* cs) {
  auto kern = dist_topk_kernel<PREC, NKB, QB, KC>;
  static bool attr = false;
  if (!attr) {
    FAMST_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    attr = true;
  }
  return launch("dist_topk", kern, dim3(nblk), dim3(256), p.lds, s, Xq, nq, p.DP, p.nkb, desc,
                cj, cs);
}

// Inputs of the k-band filter of the pipelined kernel.
struct BandArgs {
  int k;
  const float* qerr;
  const unsigned* gstat;
  float arith_c, tau;
  float* ubound;
  const int* perm;   // spatial order of the rows of Xq (null: identity)
};

template <int PREC, int NKB, int NW, bool BUF = false>
static int launch_v2(const KnnPlan& p, int nblk, hipStream_t s, const void* Xq, const float* nq,
                     const BlockDesc* desc, int* cj, float* cs, const BandArgs& ba) {
  auto kern = dist_topk_v2_kernel<PREC, NKB, NW, BUF>;
  // the kernel also holds static LDS (the list-initialisation scratch): ask
  // for exactly the dynamic bytes this launch uses
  static size_t attr = 0;
  if (attr < p.lds) {
    FAMST_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds));
    attr = p.lds;
  }
  return launch("dist_topk", kern, dim3(nblk), dim3(64 * NW), p.lds, s, Xq, nq, p.nkb, desc, cj, cs,
                ba.k, ba.qerr, ba.gstat, ba.arith_c, ba.tau, ba.ubound, ba.perm);
}

template <int PREC, int SH>
static int launch_hd(const KnnPlan& p, int nblk, hipStream_t s, const void* Xq, const float* nq,
                     const float* scl, const BlockDesc* desc, int* cj, float* cs, const BandArgs& ba) {
  auto kern = dist_topk_hd_kernel<PREC, SH>;
  static bool attr = false;
  if (!attr) {
    // the exact ring size: the kernel's static merge scratch shares the CU's LDS
    FAMST_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)hd_lds_bytes<SH>()));
    attr = true;
  }
  return launch("dist_topk", kern, dim3(nblk), dim3(64 * HdShape<SH>::NW), hd_lds_bytes<SH>(), s, Xq, nq,
                p.DP * p.esz, desc, cj, cs, ba.k, ba.qerr, ba.gstat, ba.arith_c, ba.tau, ba.ubound, scl,
                ba.perm);
}

template <int PREC>
static int dispatch_dt(const KnnPlan& p, int nblk, hipStream_t s, const void* Xq, const float* nq,
                       const BlockDesc* desc, int* cj, float* cs, const BandArgs& ba) {
  if (p.piped) {
#define V2_CASE(NKB)                                                                                        \
  case NKB:                                                                                                 \
    return p.nw == 8 ? launch_v2<PREC, NKB, 8>(p, nblk, s, Xq, nq, desc, cj, cs, ba)                       \
                     : launch_v2<PREC, NKB, 4>(p, nblk, s, Xq, nq, desc, cj, cs, ba);
#define V2_CASE_BUF(NKB)                                                                                    \
  case NKB:                                                                                                 \
    return p.nw == 8 ? launch_v2<PREC, NKB, 8>(p, nblk, s, Xq, nq, desc, cj, cs, ba)                       \
           : p.buffered ? launch_v2<PREC, NKB, 4, true>(p, nblk, s, Xq, nq, desc, cj, cs, ba)               \
                        : launch_v2<PREC, NKB, 4>(p, nblk, s, Xq, nq, desc, cj, cs, ba);
    switch (p.nkb) {
      V2_CASE_BUF(1)
      V2_CASE_BUF(2)
      V2_CASE(3)
      V2_CASE(4)
      default: return FAMST_ENOTIMPL;
    }
#undef V2_CASE
#undef V2_CASE_BUF
  }
#define DT_CASE(NKB)                                                                        \
  if (p.nkb <= NKB) {                                                                       \
    if (p.KC == 32) return launch_dt<PREC, NKB, 4, 32>(p, nblk, s, Xq, nq, desc, cj, cs);   \
    return launch_dt<PREC, NKB, 2, 64>(p, nblk, s, Xq, nq, desc, cj, cs);                   \
  }
  DT_CASE(1)
  DT_CASE(2)
  DT_CASE(4)
  DT_CASE(8)
#undef DT_CASE
  return FAMST_ENOTIMPL;
}

template <int PREC, int NKB>
static int launch_pivots(int64_t n, hipStream_t s, const void* Xq, const float* nq, uint32_t* key,
                         int* idx) {
  auto kern = pivot_assign_kernel<PREC, NKB>;
  const size_t lds = (size_t)PCH * NKB * 64 + PCH * 4;
  static bool attr = false;
  if (!attr) {
    FAMST_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  return launch("pivots", kern, dim3(cdiv(n, 256)), dim3(256), lds, s, Xq, nq, (int)n, key, idx);
}

template <int PREC>
static int pivots_prec(int nkb, int64_t n, hipStream_t s, const void* Xq, const float* nq,
                       uint32_t* key, int* idx) {
  switch (nkb) {
    case 1: return launch_pivots<PREC, 1>(n, s, Xq, nq, key, idx);
    case 2: return launch_pivots<PREC, 2>(n, s, Xq, nq, key, idx);
    case 3: return launch_pivots<PREC, 3>(n, s, Xq, nq, key, idx);
    case 4: return launch_pivots<PREC, 4>(n, s, Xq, nq, key, idx);
    default: return FAMST_ENOTIMPL;
  }
}

static int dispatch_pivots(int prec, int nkb, int64_t n, hipStream_t s, const void* Xq,
                           const float* nq, uint32_t* key, int* idx) {
  return prec == FAMST_FP32 ? pivots_prec<FAMST_FP32>(nkb, n, s, Xq, nq, key, idx)
                            : pivots_prec<FAMST_BF16>(nkb, n, s, Xq, nq, key, idx);
}

// Nearest-pivot assignment (on rows Pq of pprec / pnkb with norms pn), stable
// sort by pivot, permuted screening copy (rows of RS bytes).
static int spatial_order(int pprec, int pnkb, const void* Pq, const float* pn, int64_t n, hipStream_t s,
                         int RS, const void* Xq, const float* nq, const float* qerr, const float* scl,
                         uint32_t* key, uint32_t* key2, int* idx, int* perm, void* tmp, size_t tmpb,
                         char* Xp, float* nqp, float* qerrp, float* sclp) {
  FAMST_TRY(dispatch_pivots(pprec, pnkb, n, s, Pq, pn, key, idx));
  FAMST_TRY(sort_pairs_u32_i32(tmp, tmpb, key, key2, idx, perm, (size_t)n, NPIV_BITS, s));
  return launch("gather_rows", gather_rows_kernel, dim3(cdiv(n * (RS / 16), 256)), dim3(256), 0, s,
                reinterpret_cast<const char*>(Xq), RS, nq, qerr, scl, perm, n, Xp, nqp, qerrp, sclp);
}

// Spatial order of the n rows of X alone (for NN-Descent's initial lists):
// nearest of the NPIV pivot rows on the 128-coordinate bf16 sketch, rows
// stably sorted by pivot; perm[p] = the row at position p.  With ws == NULL
// only the workspace bytes are returned (in *bytes).
int spatial_perm(const float* X, int64_t n, int d, int* perm, void* ws, size_t* bytes, hipStream_t s) {
  Carve cv(ws);
  uint16_t* skx = cv.take<uint16_t>((size_t)n * 128);
  float* sknq = cv.take<float>(n);
  uint32_t* key = cv.take<uint32_t>(n);
  uint32_t* key2 = cv.take<uint32_t>(n);
  int* idx = cv.take<int>(n);
  const size_t tmpb = sort_pairs_u32_i32_bytes(n);
  void* tmp = cv.take<char>(tmpb);
  if (!ws) {
    *bytes = cv.bytes();
    return FAMST_OK;
  }
  const dim3 pgrid(std::min<unsigned>(cdiv(n, 4), 4096));
  FAMST_TRY(launch("sketch", sketch_kernel, pgrid, dim3(256), 0, s, X, n, d, skx, sknq));
  FAMST_TRY(dispatch_pivots(FAMST_BF16, 4, n, s, skx, sknq, key, idx));
  return sort_pairs_u32_i32(tmp, tmpb, key, key2, idx, perm, (size_t)n, NPIV_BITS, s);
}

}  // namespace famst

using namespace famst;

int famst_nndescent_run(const float* X, int64_t n, int32_t d, const int64_t* offs, int32_t B, int32_t k,
                        int32_t* nbr, float* dist, int64_t* stats, void* ws, size_t* ws_bytes, hipStream_t s);

extern "C" int famst_knn_graph(const float* X, int64_t n, int32_t d, const int64_t* offs_h,
                               int32_t B, int32_t k, int32_t precision, int32_t k_cand,
                               int32_t* nbr, float* dist, int64_t* stats, void* ws,
                               size_t* ws_bytes, void* stream) {
  if (!ws_bytes) return FAMST_EINVAL;
  if (n < 2 || d < 1 || k < 1 || k > 64 || B < 1) return FAMST_EINVAL;
  const int prec = precision & 0xFF;
  const bool exact = (precision & FAMST_EXACT) != 0;
  const bool nnd = (precision & FAMST_NNDESCENT) != 0;
  if ((precision & ~(0xFF | FAMST_EXACT | FAMST_NNDESCENT)) != 0) return FAMST_EINVAL;
  if (nnd && (exact || prec != FAMST_FP32)) return FAMST_EINVAL;
  if (prec != FAMST_FP32 && prec != FAMST_BF16 && prec != FAMST_FP8_E4M3) return FAMST_EINVAL;
  int64_t one[2] = {0, n};
  const int64_t* offs = offs_h ? offs_h : one;
  if (!offs_h && B != 1) return FAMST_EINVAL;
  if (offs[0] != 0 || offs[B] != n) return FAMST_EINVAL;
  for (int b = 0; b < B; ++b) {
    int64_t nb = offs[b + 1] - offs[b];
    if (nb < 2 || k > nb - 1) return FAMST_EINVAL;
  }
  if (n >= (int64_t(1) << 31)) return FAMST_EINVAL;
  if (nnd) {
    if (k_cand != 0 && k_cand != 32) return FAMST_EINVAL;
    return famst_nndescent_run(X, n, d, offs, B, k, nbr, dist, stats, ws, ws_bytes, static_cast<hipStream_t>(stream));
  }
  int64_t nmax = 0;
  for (int b = 0; b < B; ++b) nmax = std::max<int64_t>(nmax, offs[b + 1] - offs[b]);
  KnnPlan p;
  FAMST_TRY(choose_plan(prec, d, k, k_cand, nmax, p));
  int nblk = 0;
  for (int b = 0; b < B; ++b) nblk += (int)cdiv(offs[b + 1] - offs[b], p.qblk);
  const int esz = p.esz;

  Carve cv(ws);
  // the screening copy and its norms end with PADR zero rows (tile and query
  // block reads of the screening kernels run up to PADR - 1 rows past a cloud)
  void* Xq = cv.take<char>((size_t)(n + PADR) * p.DP * esz);
  float* nq = cv.take<float>(n + PADR);
  float* scl = cv.take<float>(n + PADR);   // float8 row scales (+ padding, as the norms)
  float* qerr = cv.take<float>(n);
  unsigned* gstat = cv.take<unsigned>(4);
  BlockDesc* desc = cv.take<BlockDesc>(nblk);
  int64_t* offs_d = cv.take<int64_t>(B + 1);
  int* cj = cv.take<int>((size_t)n * p.KC);
  float* cs = cv.take<float>((size_t)n * p.KC);
  float* kth = cv.take<float>(n);
  float* ub = cv.take<float>(n);
  int* bad = cv.take<int>(n);
  int64_t* badf = cv.take<int64_t>(n + 1);
  int64_t* badp = cv.take<int64_t>(n + 1);
  const size_t btmpb = scan_i64_bytes((size_t)n + 1);
  void* btmp = cv.take<char>(btmpb);
  unsigned long long* ctr = cv.take<unsigned long long>(4);
  int* ovf = cv.take<int>(1);
  // spatial order of the scan (one large cloud, pipelined or streamed
  // screening; the streamed one assigns pivots on a 128-coordinate sketch)
  const bool spatial =
      (p.piped || (p.hd && (int64_t)p.DP * esz <= FAMST_HD_SPATIAL_MAXB)) && B == 1 && n >= SPATIAL_MIN;
  const size_t sn = spatial ? (size_t)n : 0;
  const size_t skn = spatial && p.hd ? (size_t)n : 0;
  uint16_t* skx = cv.take<uint16_t>(skn * 128);
  float* sknq = cv.take<float>(skn);
  const bool f8sp = skn && prec == FAMST_FP8_E4M3;   // permuted float8 row scales
  float* sclp = cv.take<float>(f8sp ? skn + PADR : 0);
  char* Xp = cv.take<char>((sn ? sn + PADR : 0) * p.DP * esz);
  float* nqp = cv.take<float>(sn ? sn + PADR : 0);
  float* qerrp = cv.take<float>(sn);
  uint32_t* pkey = cv.take<uint32_t>(sn);
  uint32_t* pkey2 = cv.take<uint32_t>(sn);
  int* pidx = cv.take<int>(sn);
  int* perm = cv.take<int>(sn);
  const size_t ptmpb = spatial ? sort_pairs_u32_i32_bytes(sn) : 0;
  void* ptmp = cv.take<char>(ptmpb);
  if (!ws) {
    *ws_bytes = cv.bytes();
    return FAMST_OK;
  }
  if (*ws_bytes < cv.bytes() || (reinterpret_cast<uintptr_t>(ws) & 255)) return FAMST_EWORKSPACE;
  if (!X || !nbr || !dist) return FAMST_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);

  // block descriptors and offsets (host -> device); the host copy lives
  // until the stream has passed the synchronisation after the non-finite
  // check below (or until any earlier return, which synchronises first)
  struct HostDesc {
    BlockDesc* p;
    hipStream_t s;
    ~HostDesc() {
      if (p) {
        (void)hipStreamSynchronize(s);
        delete[] p;
      }
    }
  } hdesc{new BlockDesc[nblk], s};
  BlockDesc* hd = hdesc.p;
  int bi = 0;
  // blocks of the largest clouds first: a block's work grows with its
  // cloud's size, so late large clouds would leave a tail (ties by index)
  std::vector<int> corder(B);
  std::iota(corder.begin(), corder.end(), 0);
  std::stable_sort(corder.begin(), corder.end(),
                   [&](int a, int b) { return offs[a + 1] - offs[a] > offs[b + 1] - offs[b]; });
  for (int b : corder)
    for (int64_t q0 = offs[b]; q0 < offs[b + 1]; q0 += p.qblk)
      hd[bi++] = BlockDesc{(int)q0, (int)offs[b + 1], (int)offs[b], (int)offs[b + 1]};
  hipError_t e1 = hipMemcpyAsync(desc, hd, sizeof(BlockDesc) * nblk, hipMemcpyHostToDevice, s);
  hipError_t e2 = hipMemcpyAsync(offs_d, offs, sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, s);
  hipError_t e3 = hipMemsetAsync(gstat, 0, 16, s);
  hipError_t e4 = hipMemsetAsync(ctr, 0, 32, s);
  hipError_t e6 = hipMemsetAsync(ovf, 0, sizeof(int), s);
  hipError_t e7 = hipMemsetAsync(static_cast<char*>(Xq) + (size_t)n * p.DP * esz, 0, (size_t)PADR * p.DP * esz, s);
  hipError_t e8 = hipMemsetAsync(nq + n, 0, PADR * sizeof(float), s);
  hipError_t e11 = hipMemsetAsync(scl + n, 0, PADR * sizeof(float), s);
  hipError_t e9 = sn ? hipMemsetAsync(Xp + sn * p.DP * esz, 0, (size_t)PADR * p.DP * esz, s) : hipSuccess;
  hipError_t e10 = sn ? hipMemsetAsync(nqp + sn, 0, PADR * sizeof(float), s) : hipSuccess;
  hipError_t e12 = f8sp ? hipMemsetAsync(sclp + sn, 0, PADR * sizeof(float), s) : hipSuccess;
  if (e1 || e2 || e3 || e4 || e6 || e7 || e8 || e9 || e10 || e11 || e12) return FAMST_EHIP;

  const dim3 pgrid(std::min<unsigned>(cdiv(n, 4), 4096));
  if (prec == FAMST_FP32)
    FAMST_TRY(launch("prep", prep_kernel<FAMST_FP32>, pgrid, dim3(256), 0, s, X, n, d, p.DP, Xq, nq,
                     qerr, gstat));
  else if (prec == FAMST_BF16)
    FAMST_TRY(launch("prep", prep_kernel<FAMST_BF16>, pgrid, dim3(256), 0, s, X, n, d, p.DP, Xq, nq,
                     qerr, gstat));
  else
    FAMST_TRY(launch("prep", prep_fp8_kernel, pgrid, dim3(256), 0, s, X, n, d, p.DP,
                     reinterpret_cast<uint8_t*>(Xq), scl, nq, qerr, gstat));
  unsigned bad_flag = 0;
  FAMST_HIP(hipMemcpyAsync(&bad_flag, gstat, 4, hipMemcpyDeviceToHost, s));
  FAMST_HIP(hipStreamSynchronize(s));
  delete[] hdesc.p;   // its copy has completed
  hdesc.p = nullptr;
  if (bad_flag) return FAMST_ENONFINITE;

  // matrix-core dot products and norms: |err| <= (2d + 8) 2^-24 (|x|^2 + |y|^2)
  const float arith_c = (float)(2 * p.DP + 8) * 5.9604645e-8f;
  BandArgs ba{k, qerr, gstat, arith_c, tau32(d), ub, nullptr};
  const void* Xs = Xq;
  const float* nqs = nq;
  const float* scls = scl;
  if (spatial) {
    if (p.hd) {
      FAMST_TRY(launch("sketch", sketch_kernel, pgrid, dim3(256), 0, s, X, n, d, skx, sknq));
      FAMST_TRY(spatial_order(FAMST_BF16, 4, skx, sknq, n, s, p.DP * esz, Xq, nq, qerr,
                              prec == FAMST_FP8_E4M3 ? scl : nullptr, pkey, pkey2, pidx, perm, ptmp, ptmpb,
                              Xp, nqp, qerrp, sclp));
      if (f8sp) scls = sclp;
    } else {
      FAMST_TRY(spatial_order(prec, p.nkb, Xq, nq, n, s, p.DP * esz, Xq, nq, qerr, nullptr, pkey, pkey2,
                              pidx, perm, ptmp, ptmpb, Xp, nqp, qerrp, nullptr));
    }
    Xs = Xp;
    nqs = nqp;
    ba.qerr = qerrp;
    ba.perm = perm;
  }
  if (p.chunked)
    FAMST_TRY(dispatch_kc(p, nblk, s, Xq, nq, scl, desc, cj, cs));
  else if (p.hd)
    FAMST_TRY((prec == FAMST_FP32   ? launch_hd<FAMST_FP32, 4>(p, nblk, s, Xs, nqs, nullptr, desc, cj, cs, ba)
               : prec == FAMST_BF16 ? launch_hd<FAMST_BF16, 8>(p, nblk, s, Xs, nqs, nullptr, desc, cj, cs, ba)
                                    : launch_hd<FAMST_FP8_E4M3, 8>(p, nblk, s, Xs, nqs, scls, desc, cj, cs, ba)));
  else if (prec == FAMST_FP32)
    FAMST_TRY(dispatch_dt<FAMST_FP32>(p, nblk, s, Xs, nqs, desc, cj, cs, ba));
  else
    FAMST_TRY(dispatch_dt<FAMST_BF16>(p, nblk, s, Xs, nqs, desc, cj, cs, ba));

  RerankArgs ra;
  ra.X = X; ra.n = n; ra.d = d; ra.offs = offs_d; ra.B = B; ra.k = k; ra.KC = p.KC;
  ra.cand_j = cj; ra.cand_s = cs; ra.nq = nq; ra.qerr = qerr; ra.gstat = gstat;
  ra.arith_c = arith_c;
  ra.ubound = (p.piped || p.hd) ? ub : nullptr;
  ra.order = spatial ? perm : nullptr;
  ra.nbr = nbr; ra.dist = dist; ra.kth_s = kth; ra.bad_flag = badf; ra.counters = ctr;
  FAMST_TRY(launch("rerank", rerank_kernel, dim3(stride_grid(n)), dim3(64), 0, s, ra));

  unsigned long long hc[4] = {0, 0, 0, 0};
  int64_t nbad = 0;
  if (exact || stats) {
    FAMST_HIP(hipMemsetAsync(badf + n, 0, sizeof(int64_t), s));
    FAMST_TRY(exclusive_scan_i64(btmp, btmpb, badf, badp, (size_t)n + 1, s));
    if (exact)
      FAMST_TRY(launch("list_flagged", list_flagged_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, badf, badp, n,
                       bad));
    FAMST_HIP(hipMemcpyAsync(&nbad, badp + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FAMST_HIP(hipMemcpyAsync(hc, ctr, 32, hipMemcpyDeviceToHost, s));
    FAMST_HIP(hipStreamSynchronize(s));
    hc[0] = (unsigned long long)nbad;
  }
  if (exact && hc[0] > 0) {
    FAMST_TRY(launch("exact_row", exact_row_kernel, dim3(stride_grid((int64_t)hc[0])), dim3(256), 0, s, X, d,
                     offs_d, B, k, bad, kth, nbr, dist, ctr, ovf, (int64_t)hc[0]));
    int hov = 0;
    FAMST_HIP(hipMemcpyAsync(hc, ctr, 32, hipMemcpyDeviceToHost, s));
    FAMST_HIP(hipMemcpyAsync(&hov, ovf, 4, hipMemcpyDeviceToHost, s));
    FAMST_HIP(hipStreamSynchronize(s));
    hc[0] = (unsigned long long)nbad;
    if (hov) return FAMST_ECAPACITY;
  }
  if (stats) {
    for (int i = 0; i < FAMST_NSTATS; ++i) stats[i] = 0;
    stats[FAMST_STAT_UNCERTIFIED] = (int64_t)hc[0];
    stats[FAMST_STAT_RECOMPUTED] = (int64_t)hc[1];
    stats[FAMST_STAT_NEAR_TIES] = (int64_t)hc[2];
    stats[FAMST_STAT_K_CAND] = p.KC;
  }
  return FAMST_OK;
}
