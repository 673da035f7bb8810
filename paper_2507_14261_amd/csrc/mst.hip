// Phase 4 of FAMST (Alg. 1, GetMST): the spanning tree of the kNN edges and
// the refined inter-component edges.  Edges are keyed by (w, min, max);
// under that strict order the minimum spanning tree is unique, so Boruvka
// (Sec. 2.1) and Kruskal (Sec. 2.1, the paper's choice) give the same tree.
// Also the exact tree of the complete graph by Prim (Sec. 2.1) for k = n-1.
#include <algorithm>
#include <vector>

#include <numeric>

#include <type_traits>

#include "famst_common.hpp"
#include "prims.hpp"

namespace famst {

constexpr uint64_t KEY_NONE = ~uint64_t(0);

// (min << 32 | max) keys with the weight bits as value; invalid entries are
// flagged, self-loops become KEY_NONE (sorted last, dropped).
__global__ void mst_keys_kernel(const int32_t* __restrict__ nbr, const float* __restrict__ dist,
                                int64_t n, int k, const int32_t* __restrict__ eu,
                                const int32_t* __restrict__ ev, const float* __restrict__ ew,
                                int64_t ne, const int64_t* __restrict__ offs, int B,
                                uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                int* __restrict__ bad) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nk = n * k;
  if (e >= nk + ne) return;
  int64_t a, b;
  float w;
  if (e < nk) {
    a = e / k;
    b = nbr[e];
    w = dist[e];
  } else {
    a = eu[e - nk];
    b = ev[e - nk];
    w = ew[e - nk];
  }
  bool ok = a >= 0 && a < n && b >= 0 && b < n && w >= 0.f && __builtin_isfinite(w);
  if (ok && B > 1) ok = find_cloud(offs, B, a) == find_cloud(offs, B, b);
  if (!ok) atomicOr(bad, 1);
  if (!ok || a == b) {
    keys[e] = KEY_NONE;
    vals[e] = 0;
    return;
  }
  int64_t lo = min(a, b), hi = max(a, b);
  keys[e] = ((uint64_t)lo << 32) | (uint64_t)hi;
  vals[e] = __float_as_uint(w + 0.0f);  // -0 -> +0
}

__global__ void edge_unique_kernel(const uint64_t* __restrict__ keys, int64_t m,
                                   int64_t* __restrict__ flag) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  uint64_t kk = keys[p];
  bool keep = kk != KEY_NONE && (p == 0 || keys[p - 1] != kk);
  flag[p] = keep ? 1 : 0;
}

__global__ void edge_compact_kernel(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                    const int64_t* __restrict__ flag, const int64_t* __restrict__ pos,
                                    int64_t m, int32_t* __restrict__ elo, int32_t* __restrict__ ehi,
                                    uint32_t* __restrict__ ewb) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m || !flag[p]) return;
  int64_t o = pos[p];
  elo[o] = (int32_t)(keys[p] >> 32);
  ehi[o] = (int32_t)(uint32_t)keys[p];
  ewb[o] = vals[p];
}

// ------------------------------------------------------------- Boruvka
// Live edges only (ids in `live`): drop edges inside one component, and
// lower the per-component minimum key; a plain read first skips the atomic
// for the (common) edges that cannot improve it.
// The live entries are taken in chunks of 64 (one wave, coalesced reads):
// wave w takes chunk (w * stride) mod nchunk, a bijection for a stride
// coprime to nchunk.  With many small clouds the host passes a large stride,
// so that concurrent waves lower the minima of unrelated clouds rather than
// the few components of one cloud; one cloud is taken in order (stride 1).
// When every active lane of a wave lowers the same component (consecutive
// lambda-edges of one component pair), the wave takes the minimum of its
// keys first and issues one atomic.
__global__ void bv_min_edge_kernel(const int32_t* __restrict__ elo, const int32_t* __restrict__ ehi,
                                   const uint32_t* __restrict__ ewb, const uint32_t* __restrict__ live,
                                   int64_t nlive, uint64_t stride, const int32_t* __restrict__ comp,
                                   unsigned long long* __restrict__ best, int64_t* __restrict__ keep) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nchunk = (nlive + 63) >> 6, w = t >> 6;
  if (w >= nchunk) return;   // uniform per wave
  const int64_t c =
      stride == 1 ? w : (int64_t)(((unsigned __int128)w * stride) % (unsigned __int128)nchunk);
  const int64_t i = (c << 6) + (t & 63);
  bool act = i < nlive;
  int cu = -1, cv = -1;
  unsigned long long key = ~0ull;
  if (act) {
    const uint32_t e = live[i];
    cu = comp[elo[e]];
    cv = comp[ehi[e]];
    act = cu != cv;
    keep[i] = act ? 1 : 0;
    key = ((unsigned long long)ewb[e] << 32) | (unsigned long long)e;
  }
  const unsigned long long am = ballot(act);
  if (!am) return;   // uniform
  const int lead = __builtin_ctzll(am);
  auto lower = [&](int cc) {
    const int c0 = __builtin_amdgcn_readlane(cc, lead);
    if (ballot(act && cc != c0) == 0) {
      // one component for the whole wave: minimum of the keys, one atomic
      unsigned long long m = act ? key : ~0ull;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long om = __shfl_xor(m, o);
        m = om < m ? om : m;
      }
      if ((t & 63) == lead && m < __hip_atomic_load(&best[c0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin(&best[c0], m);
    } else if (act && key < __hip_atomic_load(&best[cc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      atomicMin(&best[cc], key);
    }
  };
  lower(cu);
  lower(cv);
}

__global__ void bv_compact_kernel(const uint32_t* __restrict__ live, const int64_t* __restrict__ keep,
                                  const int64_t* __restrict__ pos, int64_t nlive,
                                  uint32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nlive && keep[i]) out[pos[i]] = live[i];
}

__global__ void bv_hook_kernel(const int32_t* __restrict__ elo, const int32_t* __restrict__ ehi,
                               int64_t n, const int32_t* __restrict__ comp,
                               const unsigned long long* __restrict__ best, int32_t* __restrict__ P,
                               uint8_t* __restrict__ in_tree, int* __restrict__ hooked) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  if (comp[c] != c) return;
  unsigned long long key = best[c];
  if (key == ~0ull) {
    P[c] = (int32_t)c;
    return;
  }
  uint32_t e = (uint32_t)key;
  int cl = comp[elo[e]], ch = comp[ehi[e]];
  int other = (cl == c) ? ch : cl;
  if (best[other] == key && c < other) {
    P[c] = (int32_t)c;   // the smaller root of a mutual pair stays
  } else {
    P[c] = other;
    in_tree[e] = 1;
    *hooked = 1;
  }
}

__global__ void bv_jump_kernel(const int32_t* __restrict__ comp, int64_t n, int32_t* P) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || comp[c] != c) return;
  while (true) {
    int p = __hip_atomic_load(&P[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int pp = __hip_atomic_load(&P[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == pp) break;
    __hip_atomic_store(&P[c], pp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void bv_relabel_kernel(int32_t* __restrict__ comp, const int32_t* __restrict__ P, int64_t n) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  comp[v] = P[comp[v]];
}

// Boruvka for small inputs: every round in one block, with the minimum keys,
// the component labels and the parents in LDS (8 + 2 + 2 bytes per vertex),
// so a call needs no host round trip per round.  Same keys and the same hook
// rule as the kernels above, so the same tree.  Each round scans all m
// edges (an edge inside one component is skipped); the edge count is read
// on the device.
constexpr int BV1_NT = 1024;
constexpr int BV1_MAXN = 13312;           // 12 bytes of LDS per vertex
constexpr int64_t BV1_MAXM = 1 << 18;     // edges scanned per round at most
__global__ __launch_bounds__(BV1_NT) void bv_block_kernel(const int32_t* __restrict__ elo,
                                                         const int32_t* __restrict__ ehi,
                                                         const uint32_t* __restrict__ ewb,
                                                         const int64_t* __restrict__ mptr, int n,
                                                         uint8_t* __restrict__ in_tree) {
  extern __shared__ __attribute__((aligned(16))) unsigned long long bsm[];
  unsigned long long* best = bsm;                               // [n]
  uint16_t* comp = reinterpret_cast<uint16_t*>(best + n);       // [n]
  volatile uint16_t* P = comp + n;                              // [n], roots only
  __shared__ int hooked_s;
  const int t = threadIdx.x;
  const int64_t m = *mptr;
  for (int v = t; v < n; v += BV1_NT) comp[v] = (uint16_t)v;
  for (int round = 0; round < 64; ++round) {
    for (int v = t; v < n; v += BV1_NT) best[v] = ~0ull;
    if (t == 0) hooked_s = 0;
    __syncthreads();
    for (int64_t e = t; e < m; e += BV1_NT) {
      const int cu = comp[elo[e]], cv = comp[ehi[e]];
      if (cu != cv) {
        // a read first: late rounds send most edges to a few components, and
        // atomics on one LDS word run one lane at a time
        const unsigned long long key = ((unsigned long long)ewb[e] << 32) | (unsigned long long)e;
        if (key < best[cu]) atomicMin(&best[cu], key);
        if (key < best[cv]) atomicMin(&best[cv], key);
      }
    }
    __syncthreads();
    for (int c = t; c < n; c += BV1_NT) {
      if (comp[c] != c) continue;
      const unsigned long long key = best[c];
      if (key == ~0ull) {
        P[c] = (uint16_t)c;
        continue;
      }
      const uint32_t e = (uint32_t)key;
      const int cl = comp[elo[e]], ch = comp[ehi[e]];
      const int other = cl == c ? ch : cl;
      if (best[other] == key && c < other) {
        P[c] = (uint16_t)c;   // the smaller root of a mutual pair stays
      } else {
        P[c] = (uint16_t)other;
        in_tree[e] = 1;
        hooked_s = 1;
      }
    }
    __syncthreads();
    if (!hooked_s) break;   // every thread reads it before the next round resets it
    // pointer jumping: parents only move to their own parents' parents, and
    // every chain ends at a root that stays, so each loop ends
    for (int c = t; c < n; c += BV1_NT) {
      if (comp[c] != c) continue;
      while (true) {
        const int p = P[c], pp = P[p];
        if (p == pp) break;
        P[c] = (uint16_t)pp;
      }
    }
    __syncthreads();
    for (int v = t; v < n; v += BV1_NT) comp[v] = P[comp[v]];
    __syncthreads();
  }
}

// ------------------------------------------------------------- Kruskal
__global__ void kr_keys_kernel(const uint32_t* __restrict__ ewb, int64_t m, uint64_t* __restrict__ keys) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) keys[e] = ((uint64_t)ewb[e] << 32) | (uint64_t)e;
}

__device__ int kr_find(int32_t* parent, int x) {
  while (parent[x] != x) {
    parent[x] = parent[parent[x]];
    x = parent[x];
  }
  return x;
}

// sequential union-find scan over the sorted keys (single thread)
__global__ void kr_scan_kernel(const uint64_t* __restrict__ skeys, int64_t m,
                               const int32_t* __restrict__ elo, const int32_t* __restrict__ ehi,
                               int32_t* parent, int64_t target, uint8_t* __restrict__ in_tree) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int64_t cnt = 0;
  for (int64_t i = 0; i < m && cnt < target; ++i) {
    uint32_t e = (uint32_t)skeys[i];
    int a = kr_find(parent, elo[e]), b = kr_find(parent, ehi[e]);
    if (a == b) continue;
    if (a < b) parent[b] = a; else parent[a] = b;
    in_tree[e] = 1;
    ++cnt;
  }
}

// ------------------------------------------------------------ tree output
__global__ void u8_to_i64_kernel(const uint8_t* __restrict__ f, int64_t m, int64_t* __restrict__ o) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < m) o[p] = f[p];
  if (p == m) o[p] = 0;
}

__global__ void tree_compact_kernel(const uint8_t* __restrict__ in_tree, const int64_t* __restrict__ pos,
                                    int64_t m, const int32_t* __restrict__ elo,
                                    const int32_t* __restrict__ ehi, const uint32_t* __restrict__ ewb,
                                    int32_t* __restrict__ tu, int32_t* __restrict__ tv,
                                    float* __restrict__ tw) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m || !in_tree[p]) return;
  int64_t o = pos[p];
  tu[o] = elo[p];
  tv[o] = ehi[p];
  tw[o] = __uint_as_float(ewb[p]);
}

// Per-cloud tree weight: compensated (Neumaier) partial sums in a fixed
// thread order, combined by a fixed tree of error-free additions.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__global__ __launch_bounds__(256) void tree_weight_kernel(const float* __restrict__ tw,
                                                          const int64_t* __restrict__ offs,
                                                          float* __restrict__ W) {
  __shared__ float ss[256], ee[256];
  const int b = blockIdx.x, t = threadIdx.x;
  const int64_t e0 = offs[b] - b, e1 = offs[b + 1] - b - 1;
  // thread t adds elements t, t + 256, t + 512, ... in that order; sixteen
  // loads are issued ahead of the (dependent) compensated additions
  float s = 0.f, c = 0.f;
  constexpr int U = 16;
  for (int64_t i0 = e0 + t; i0 < e1; i0 += 256 * U) {
    float x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = i0 + 256 * u < e1 ? tw[i0 + 256 * u] : 0.f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + 256 * u < e1) {
        float ns, err;
        two_sum(s, x[u], ns, err);
        s = ns;
        c += err;
      }
    }
  }
  ss[t] = s;
  ee[t] = c;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
      float ns, err;
      two_sum(ss[t], ss[t + w], ns, err);
      ss[t] = ns;
      ee[t] = ee[t] + ee[t + w] + err;
    }
    __syncthreads();
  }
  if (t == 0) W[b] = ss[0] + ee[0];
}

// ------------------------------------------------------------ dense Prim
// Exact tree of the complete graph of one cloud: the distances to the newest
// tree vertex are computed on the fly, so nothing of size n^2 is stored.
// Keys are (w, min, max) as everywhere.
constexpr int PRIM_MAX = 16384;   // local ids fit in 14 bits
constexpr int PRIM_NT = 512;      // threads per cloud
constexpr int PRIM_NT_DM = 1024;  // threads per cloud, Prim over the pair matrices

__device__ __forceinline__ bool ekey_less(float w1, int a1, int b1, float w2, int a2, int b2) {
  int l1 = min(a1, b1), h1 = max(a1, b1), l2 = min(a2, b2), h2 = max(a2, b2);
  if (w1 != w2) return w1 < w2;
  if (l1 != l2) return l1 < l2;
  return h1 < h2;
}

// Four lanes (a quad) evaluate one canonical distance (the bits of
// sq32_group): lane c owns partials c, c+4, c+8 and c+12, i.e. the chunks
// congruent to c mod 4, so a quad reads each 64-byte stretch of a row with
// one 16-byte load per lane.  The partials are combined in the lane
// ((pc + pc+8) + (pc+4 + pc+12)), then across the quad by xor 2 and xor 1.
template <int CTRL>
__device__ __forceinline__ float quad_xor_add(float v) {
  const int o = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false);
  return v + __int_as_float(o);
}
constexpr int DPP_QUAD_XOR1 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int DPP_QUAD_XOR2 = 0x4E;   // quad_perm [2, 3, 0, 1]

__device__ __forceinline__ float quad_combine(const float (&p)[4]) {
  const float s4 = (p[0] + p[2]) + (p[1] + p[3]);
  return quad_xor_add<DPP_QUAD_XOR1>(quad_xor_add<DPP_QUAD_XOR2>(s4));
}

// partials of lane c for any d (scalar loads; dimensions past d are skipped)
__device__ __forceinline__ void quad_partials(const float* __restrict__ a, const float* __restrict__ b,
                                              int d, int c, float (&p)[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) p[m] = 0.f;
  for (int base = 0; base < d; base += 64)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int t0 = base + 4 * (c + 4 * m);
      for (int t = t0; t < t0 + 4 && t < d; ++t) {
        const float df = a[t] - b[t];
        p[m] = __builtin_fmaf(df, df, p[m]);
      }
    }
}

// Minimum of a 64-bit key over the wave by DPP (row shifts by 1, 2, 3, then
// 4 and 8 across banks, then the row broadcasts 15 and 31): the minimum
// lands in lane 63.  A lane whose DPP source does not exist keeps its own
// key (the `old` operand), which leaves the minimum unchanged; both halves
// of a key move with the same control, so every lane always holds a whole
// key of some lane.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ uint64_t dpp_min_step(uint64_t v) {
  const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
  const uint32_t olo = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, BANK_MASK, false);
  const uint32_t ohi = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, BANK_MASK, false);
  const uint64_t o = ((uint64_t)ohi << 32) | olo;
  return o < v ? o : v;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
  v = dpp_min_step<0x111, 0xF, 0xF>(v);   // row_shr:1
  v = dpp_min_step<0x112, 0xF, 0xF>(v);   // row_shr:2
  v = dpp_min_step<0x113, 0xF, 0xF>(v);   // row_shr:3
  v = dpp_min_step<0x114, 0xF, 0xE>(v);   // row_shr:4, banks 1-3
  v = dpp_min_step<0x118, 0xF, 0xC>(v);   // row_shr:8, banks 2-3
  v = dpp_min_step<0x142, 0xA, 0xF>(v);   // row_bcast:15 into rows 1 and 3
  v = dpp_min_step<0x143, 0xC, 0xF>(v);   // row_bcast:31 into rows 2 and 3
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}

// Minimum over lanes 0..15 of a row (the row shifts and bank steps of
// wave_min_u64): lane 15 of every row holds its row's minimum.
__device__ __forceinline__ uint64_t row16_min_u64(uint64_t v) {
  v = dpp_min_step<0x111, 0xF, 0xF>(v);
  v = dpp_min_step<0x112, 0xF, 0xF>(v);
  v = dpp_min_step<0x113, 0xF, 0xF>(v);
  v = dpp_min_step<0x114, 0xF, 0xE>(v);
  v = dpp_min_step<0x118, 0xF, 0xC>(v);
  return v;
}

// Selection key of a candidate edge (w, p, j), w >= 0, local ids < 2^14:
// ordered as (w, min, max); the low bit says whether j (the vertex outside
// the tree) is the smaller endpoint.  ~0 marks a dead list entry.
__device__ __forceinline__ uint64_t prim_key(float w, int p, int j) {
  const uint32_t lo = (uint32_t)min(p, j), hi = (uint32_t)max(p, j);
  return ((uint64_t)__float_as_uint(w) << 29) | ((uint64_t)lo << 15) | ((uint64_t)hi << 1) |
         (uint64_t)(j < p);
}
constexpr uint64_t PRIM_DEAD = ~0ull;

// The same minima, first over the 32 weight bits of the keys (bits 29..60;
// a dead key's top word is all ones), with the 64-bit minimum only among
// the lanes that tie on the weight: the same key in about half the
// instructions when the minimum weight is unique.  wave_min_key: all 64
// lanes; row_min_key: lanes 0..15.  Every lane returns the key.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ uint32_t dpp_min_step32(uint32_t v) {
  const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, ROW_MASK, BANK_MASK, false);
  return o < v ? o : v;
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_min_key(uint64_t v) {
  const uint32_t w = (uint32_t)(v >> 29);
  uint32_t m = w;
  m = dpp_min_step32<0x111, 0xF, 0xF>(m);
  m = dpp_min_step32<0x112, 0xF, 0xF>(m);
  m = dpp_min_step32<0x113, 0xF, 0xF>(m);
  m = dpp_min_step32<0x114, 0xF, 0xE>(m);
  m = dpp_min_step32<0x118, 0xF, 0xC>(m);
  m = dpp_min_step32<0x142, 0xA, 0xF>(m);
  m = dpp_min_step32<0x143, 0xC, 0xF>(m);
  m = (uint32_t)__builtin_amdgcn_readlane((int)m, 63);
  const uint64_t tie = __ballot(w == m);
  if (__popcll(tie) == 1) return readlane_u64(v, __builtin_ctzll(tie));
  return wave_min_u64(w == m ? v : PRIM_DEAD);
}
__device__ __forceinline__ uint64_t row_min_key(uint64_t v) {
  const int lane = threadIdx.x & 63;
  const uint32_t w = lane < 16 ? (uint32_t)(v >> 29) : 0xFFFFFFFFu;
  uint32_t m = w;
  m = dpp_min_step32<0x111, 0xF, 0xF>(m);
  m = dpp_min_step32<0x112, 0xF, 0xF>(m);
  m = dpp_min_step32<0x113, 0xF, 0xF>(m);
  m = dpp_min_step32<0x114, 0xF, 0xE>(m);
  m = dpp_min_step32<0x118, 0xF, 0xC>(m);
  m = (uint32_t)__builtin_amdgcn_readlane((int)m, 15);
  const uint64_t tie = __ballot(lane < 16 && w == m);
  if (__popcll(tie) == 1) return readlane_u64(v, __builtin_ctzll(tie));
  return readlane_u64(row16_min_u64(lane < 16 && w == m ? v : PRIM_DEAD), 15);
}
__device__ __forceinline__ float key_w(uint64_t k) { return __uint_as_float((uint32_t)(k >> 29)); }
__device__ __forceinline__ int key_j(uint64_t k) {
  return (k & 1) ? (int)((k >> 15) & 0x3FFF) : (int)((k >> 1) & 0x3FFF);
}
__device__ __forceinline__ int key_p(uint64_t k) {
  return (k & 1) ? (int)((k >> 1) & 0x3FFF) : (int)((k >> 15) & 0x3FFF);
}

// Candidate update of list entry `key` (vertex j outside the tree) by the
// distance s to the newest tree vertex cur.  Skips the square root when
// s > w0^2 (1 + 2^-20): then sqrtf(s) rounds strictly above w0 and the entry
// cannot change.
__device__ __forceinline__ uint64_t prim_relax(uint64_t key, float s, int cur) {
  const float w0 = key_w(key);
  if (s > w0 * w0 * 1.00000095f && w0 > 1e-18f) return key;
  const float w = __builtin_sqrtf(s);
  const int j = key_j(key);
  return ekey_less(w, cur, j, w0, key_p(key), j) ? prim_key(w, cur, j) : key;
}

// Dense Prim over rows c0 .. c0 + nb - 1 by NT threads.  `keys` holds
// one key per vertex outside the tree (its best edge to the tree); slot q
// belongs to quad q mod NQ, whose lane 0 alone writes it, so one barrier
// per step suffices: the per-wave minimum keys go through LDS
// (double-buffered by step parity) and every thread reduces them in the
// same order.  The entry of the vertex that joins the tree is marked dead
// by its owner; every PRIM_COMPACT steps the live entries are packed to the
// front (their order does not matter: the minimum is over unique keys).
// emit(step, p, j, w) is called by thread 0 for each edge, in insertion
// order.  VEC: d == 64 and rows 16-byte aligned; FAMST_PRIM_R rows per
// quad are in flight.  CMAX >= nb / NT.
constexpr int PRIM_COMPACT = 32;

#ifndef FAMST_PRIM_R
#define FAMST_PRIM_R 8
#endif
template <int NT, bool VEC, int CMAX, class Emit>
__device__ void prim_cloud(const float* __restrict__ X, int d, int64_t c0, int nb,
                           uint64_t* __restrict__ keys, uint64_t* __restrict__ wkeys,
                           int* __restrict__ mcount, Emit emit) {
  constexpr int NW = NT / 64, NQ = NT / 4, R = FAMST_PRIM_R;   // rows in flight per lane
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, c = t & 3, g = t >> 2;
  // vertex 0 starts the tree; every other vertex has the placeholder edge
  // (+inf, 0, j), replaced in the first step
  for (int j = 1 + t; j < nb; j += NT) keys[j - 1] = prim_key(F_INF, 0, j);
  if (t == 0) *mcount = 0;
  __syncthreads();
  int m = nb - 1;
  int cur = 0;
  for (int step = 1; step < nb; ++step) {
    const float* __restrict__ xc = X + (c0 + cur) * d;
    uint64_t best = PRIM_DEAD;
    int bslot = -1;
    if constexpr (VEC) {
      f32x4 xa[4];
#pragma unroll
      for (int mm = 0; mm < 4; ++mm) xa[mm] = reinterpret_cast<const f32x4*>(xc)[c + 4 * mm];
      for (int q0 = g; q0 < m; q0 += NQ * R) {
        uint64_t kk[R];
        f32x4 rv[R][4];
#pragma unroll
        for (int u = 0; u < R; ++u) {
          const int q = q0 + u * NQ;
          kk[u] = q < m ? keys[q] : PRIM_DEAD;
          // dead or missing entries read the newest vertex's row (cached),
          // so the loads need no branches
          const int row = kk[u] != PRIM_DEAD ? key_j(kk[u]) : cur;
          const f32x4* rp = reinterpret_cast<const f32x4*>(X + (c0 + row) * 64);
#pragma unroll
          for (int mm = 0; mm < 4; ++mm) rv[u][mm] = rp[c + 4 * mm];
        }
#pragma unroll
        for (int u = 0; u < R; ++u) {
          float pp[4];
#pragma unroll
          for (int mm = 0; mm < 4; ++mm) {
            float acc = 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float df = xa[mm][i] - rv[u][mm][i];
              acc = __builtin_fmaf(df, df, acc);
            }
            pp[mm] = acc;
          }
          const float sq = quad_combine(pp);
          if (kk[u] != PRIM_DEAD) {
            const uint64_t nk = prim_relax(kk[u], sq, cur);
            const int q = q0 + u * NQ;
            if (nk != kk[u] && c == 0) keys[q] = nk;
            if (nk < best) {
              best = nk;
              bslot = q;
            }
          }
        }
      }
    } else {
      for (int q = g; q < m; q += NQ) {
        const uint64_t k0 = keys[q];
        if (k0 == PRIM_DEAD) continue;   // uniform in the quad
        float pp[4];
        quad_partials(xc, X + (c0 + key_j(k0)) * d, d, c, pp);
        const uint64_t nk = prim_relax(k0, quad_combine(pp), cur);
        if (nk != k0 && c == 0) keys[q] = nk;
        if (nk < best) {
          best = nk;
          bslot = q;
        }
      }
    }
    const uint64_t wb = wave_min_u64(best);
    uint64_t* wk = wkeys + (step & 1) * NW;
    if (lane == 0) wk[wave] = wb;
    __syncthreads();
    uint64_t gb = wk[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) gb = wk[w] < gb ? wk[w] : gb;
    const int j = key_j(gb), p = key_p(gb);
    if (t == 0) emit(step, p, j, key_w(gb));
    if (best == gb && c == 0) keys[bslot] = PRIM_DEAD;
    cur = __builtin_amdgcn_readfirstlane(j);
    if (step % PRIM_COMPACT == 0 && step + 1 < nb) {
      if (t == 0) *mcount = 0;
      __syncthreads();   // dead marks and key updates done; counter cleared
      uint64_t e[CMAX];
      int cnt = 0;
#pragma unroll
      for (int i = 0; i < CMAX; ++i) {
        const int q = t + NT * i;
        e[i] = q < m ? keys[q] : PRIM_DEAD;
        cnt += e[i] != PRIM_DEAD;
      }
      __syncthreads();   // every live entry is in registers
      int pos = cnt ? atomicAdd(mcount, cnt) : 0;
#pragma unroll
      for (int i = 0; i < CMAX; ++i)
        if (e[i] != PRIM_DEAD) keys[pos++] = e[i];
      __syncthreads();
      m = *mcount;
    }
  }
  __syncthreads();
}

// Dense Prim over the cloud's pair matrix Dc (row-major nb x nb squared
// distances) by NT threads.  Vertex v >= 1 sits in slot v - 1 for the whole
// run, as entry (v - 1) / NT of thread (v - 1) mod NT, with its key and the
// square below which a distance can change that key (w0^2 (1 + 2^-20), as
// in prim_relax) in registers: a step reads row cur of the matrix with
// consecutive lanes on consecutive entries and compares; only entries under
// the square take the exact relaxation, and slots of tree vertices are
// retired (no compaction: it would scatter the row reads).  The matrices are
// followed by FUSED_MAX zeroed floats, so the reads of the last slots stay
// in the workspace.  Same keys, same minimum and the same emit order as
// prim_cloud, so the same tree.
template <int NT, int CMAX, class Emit>
__device__ void prim_cloud_dm(const float* __restrict__ Dc, int nb, uint64_t* __restrict__ wkeys, Emit emit) {
  static_assert((NT & (NT - 1)) == 0 && NT >= 64 && NT <= 1024, "slot owners by mask, 16 waves at most");
  constexpr int NW = NT / 64;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  uint64_t kr[CMAX];
  float thr[CMAX];
  auto set_slot = [&](int i, uint64_t k) {
    kr[i] = k;
    const float w0 = key_w(k);
    // relax when s <= thr: prim_relax's early exit (none for tiny w0); never
    // for a retired slot
    thr[i] = k == PRIM_DEAD ? -F_INF : (w0 > 1e-18f ? w0 * w0 * 1.00000095f : F_INF);
  };
  auto slots_min = [&]() {
    uint64_t b = PRIM_DEAD;
#pragma unroll
    for (int i = 0; i < CMAX; ++i) b = kr[i] < b ? kr[i] : b;
    return b;
  };
  // vertex 0 starts the tree; every other vertex has the placeholder edge
  // (+inf, 0, v), replaced in the first step
#pragma unroll
  for (int i = 0; i < CMAX; ++i) {
    const int v = t + NT * i + 1;
    set_slot(i, v < nb ? prim_key(F_INF, 0, v) : PRIM_DEAD);
  }
  // the thread's smallest key: keys only fall (relaxation) or retire (the
  // owner of the new tree vertex recomputes it)
  uint64_t best = slots_min();
  int cur = 0, jq = -1;   // jq: the slot that the last step's tree vertex leaves
  for (int step = 1; step < nb; ++step) {
    // entries past the row's end read the next row or the zeroed padding
    // after the last matrix: their slots are retired
    const float* __restrict__ dr = Dc + (int64_t)cur * nb + t + 1;
    float sq[CMAX];
#pragma unroll
    for (int i = 0; i < CMAX; ++i)
      if (NT * i + 1 < nb) sq[i] = dr[NT * i];
    // while the row is in flight: the owner of the last tree vertex retires
    // its slot (it must not be relaxed below)
    if (jq >= 0 && (jq & (NT - 1)) == t) {
#pragma unroll
      for (int i = 0; i < CMAX; ++i)
        if (i == jq / NT) set_slot(i, PRIM_DEAD);
      best = slots_min();
    }
#pragma unroll
    for (int i = 0; i < CMAX; ++i) {
      if (NT * i + 1 < nb && sq[i] <= thr[i]) {
        const uint64_t nk = prim_relax(kr[i], sq[i], cur);
        if (nk != kr[i]) {
          set_slot(i, nk);
          best = nk < best ? nk : best;
        }
      }
    }
    const uint64_t wb = wave_min_key(best);
    uint64_t* wk = wkeys + (step & 1) * NW;
    if (lane == 0) wk[wave] = wb;
    __syncthreads();
    // the NW wave minima: lane l of each wave takes minimum l mod 16 (NW <= 16)
    const uint64_t gb = row_min_key((lane & 15) < NW ? wk[lane & 15] : PRIM_DEAD);
    const int j = key_j(gb), p = key_p(gb);
    if (t == 0) emit(step, p, j, key_w(gb));
    jq = j - 1;
    cur = __builtin_amdgcn_readfirstlane(j);
  }
  __syncthreads();
}

__global__ __launch_bounds__(PRIM_NT) void prim_kernel(const float* __restrict__ X, int d,
                                                       const int64_t* __restrict__ offs, int vec,
                                                       int32_t* __restrict__ ou, int32_t* __restrict__ ov,
                                                       float* __restrict__ ow) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  __shared__ uint64_t wkeys[2 * PRIM_NT / 64];
  __shared__ int mcount;
  const int b = blockIdx.x;
  const int64_t c0 = offs[b];
  const int nb = (int)(offs[b + 1] - c0);
  uint64_t* keys = reinterpret_cast<uint64_t*>(smem);
  const int64_t eo = c0 - b;  // output slot of this cloud's first edge
  auto emit = [&](int step, int p, int j, float w) {
    ou[eo + step - 1] = (int32_t)(c0 + min(p, j));
    ov[eo + step - 1] = (int32_t)(c0 + max(p, j));
    ow[eo + step - 1] = w;
  };
  constexpr int CM = PRIM_MAX / PRIM_NT;
  if (vec) prim_cloud<PRIM_NT, true, CM>(X, d, c0, nb, keys, wkeys, &mcount, emit);
  else prim_cloud<PRIM_NT, false, CM>(X, d, c0, nb, keys, wkeys, &mcount, emit);
}

// ------------------------------------------------ pair distance matrices
// For d <= 64 the squared distance of every pair of a cloud is computed once,
// in the bits of sq32_group, and stored in both orders as the row-major
// nb x nb matrix of the cloud at dmoff[b]; Prim then reads one matrix row
// (4 bytes per vertex outside the tree) per step instead of the rows of
// every such vertex (4 d bytes each).  The matrix is built from 64 x 64
// tiles of the upper triangle of tiles, 256 threads per tile; thread
// (ty, tx) holds the 16 pairs (ty + 16 i, tx + 16 j).  The 16 chunk partials of a pair are combined as
// sq32_group's xor butterfly (over 8, 4, 2, 1), i.e. a binary tree over the
// chunks in bit-reversed order 0, 8, 4, 12, 2, ...; padding dimensions
// (zero in both rows) leave a partial unchanged, as in sq32_group.
constexpr int PD_T = 64, PD_NT = 256, PD_LD = 68;   // tile edge, threads, LDS row stride (floats)
constexpr int DMAT_MAXD = 64;

// chunk partials of chunk c for the thread's 16 pairs: dimensions
// 4 c .. 4 c + 3, fmaf in order
__device__ __forceinline__ void pd_leaf(const float* As, const float* Bs, int ty, int tx, int c, float (&out)[16]) {
  f32x4 xa[4], xb[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    xa[i] = *reinterpret_cast<const f32x4*>(As + (ty + 16 * i) * PD_LD + 4 * c);
    xb[i] = *reinterpret_cast<const f32x4*>(Bs + (tx + 16 * i) * PD_LD + 4 * c);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float acc = 0.f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float df = xa[i][e] - xb[j][e];
        acc = __builtin_fmaf(df, df, acc);
      }
      out[4 * i + j] = acc;
    }
}

// The 16 leaves in bit-reversed chunk order; a finished left subtree at
// level l waits in pend[l] until its right sibling is complete (a binary
// counter over the leaf index).
__device__ __forceinline__ void pd_pairs(const float* As, const float* Bs, int ty, int tx, float (&sq)[16]) {
  float pend[4][16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int c = ((k & 1) << 3) | ((k & 2) << 1) | ((k & 4) >> 1) | ((k & 8) >> 3);
    float v[16];
    pd_leaf(As, Bs, ty, tx, c, v);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      if ((k >> l) & 1) {
#pragma unroll
        for (int p = 0; p < 16; ++p) v[p] = pend[l][p] + v[p];
      } else {
#pragma unroll
        for (int p = 0; p < 16; ++p) pend[l][p] = v[p];
        break;
      }
    }
    if (k == 15) {
#pragma unroll
      for (int p = 0; p < 16; ++p) sq[p] = v[p];
    }
  }
}

// One 64 x 64 tile (ta, tb), ta <= tb, of the upper triangle of tiles of a
// cloud of nb rows starting at row c0, by 256 threads (t = 0 .. 255) with
// their own As and Bs; the matrix of the cloud starts at Dm.  Every thread of
// the block runs the same barriers whether or not its group has a tile
// (valid), so groups of one block may hold tiles of different shapes.
__device__ __forceinline__ void pair_tile(const float* __restrict__ X, int d, int64_t c0, int nb, int64_t li,
                                          bool valid, float* __restrict__ As, float* __restrict__ Bs, int t,
                                          float* __restrict__ Dm) {
  const int ty = t >> 4, tx = t & 15;
  const int T = (nb + PD_T - 1) / PD_T;
  // row ta of the triangle starts at S(ta) = ta T - ta (ta - 1) / 2
  auto S = [&](int r) { return (int64_t)r * T - (int64_t)r * (r - 1) / 2; };
  int ta = 0, tb = 0;
  if (valid) {
    ta = (int)((2.0 * T + 1.0 - sqrt((2.0 * T + 1.0) * (2.0 * T + 1.0) - 8.0 * (double)li)) * 0.5);
    ta = max(0, min(ta, T - 1));
    while (ta > 0 && S(ta) > li) --ta;
    while (ta + 1 < T && S(ta + 1) <= li) ++ta;
    tb = ta + (int)(li - S(ta));
  }
  const int a0 = ta * PD_T, b0 = tb * PD_T;
  // rows of both tiles (rows past the cloud repeat its last row, dimensions
  // past d are zero)
  if (valid)
    for (int e = t; e < PD_T * 16; e += PD_NT) {
      const int r = e >> 4, cc = e & 15;
      const int ra = min(a0 + r, nb - 1), rb = min(b0 + r, nb - 1);
      f32x4 va, vb;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int dim = 4 * cc + i;
        va[i] = dim < d ? X[(c0 + ra) * d + dim] : 0.f;
        vb[i] = dim < d ? X[(c0 + rb) * d + dim] : 0.f;
      }
      *reinterpret_cast<f32x4*>(As + r * PD_LD + 4 * cc) = va;
      *reinterpret_cast<f32x4*>(Bs + r * PD_LD + 4 * cc) = vb;
    }
  __syncthreads();
  float sq[16];
  if (valid) {
    pd_pairs(As, Bs, ty, tx, sq);
    // the values are complete here: the compiler would otherwise sink each
    // pair's arithmetic into its guarded store and read every chunk first
#pragma unroll
    for (int p = 0; p < 16; ++p) __asm__ volatile("" : : "v"(sq[p]));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int a = a0 + ty + 16 * i, c = b0 + tx + 16 * j;
        if (a < nb && c < nb) Dm[(int64_t)a * nb + c] = sq[4 * i + j];
      }
  }
  __syncthreads();   // the tile rows are read; As is reused for the transpose
  const bool mirror = valid && ta != tb;
  if (mirror) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) As[(ty + 16 * i) * PD_LD + tx + 16 * j] = sq[4 * i + j];
  }
  __syncthreads();
  if (mirror) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = b0 + ty + 16 * i, a = a0 + tx + 16 * j;
        if (a < nb && c < nb) Dm[(int64_t)c * nb + a] = As[(tx + 16 * j) * PD_LD + ty + 16 * i];
      }
  }
  __syncthreads();   // the next tile overwrites As and Bs
}

constexpr int FUSED_MAX = 12288;

// After the tree of cloud b (rows c0 .. c0 + nb - 1, edges at eo .. eo + nb
// - 2 in insertion order, par[v] the parent of v): the compensated tree
// weight W[b] in insertion order, the children lists (stable in the child
// id), and the gradient rows, one
// 16-lane group per row: its parent edge first, then its children in
// ascending id, so the result is deterministic.  endp and kid must not
// overlap par.  IT: int, or uint16_t (ids below 2^16) to save LDS.  wv: the
// weight of each vertex's parent edge as Prim emitted it (the square root
// of the canonical squared distance), or null to recompute it per edge.
template <class IT>
__device__ __forceinline__ void lds_count_add(IT* a, int p) {
  if constexpr (sizeof(IT) == 4) {
    atomicAdd(reinterpret_cast<int*>(a) + p, 1);
  } else {
    // the 32-bit word holding a[p]; a count stays below 2^16, so the low
    // half never carries into the high one
    static_assert(sizeof(IT) == 2, "16- or 32-bit lists");
    atomicAdd(reinterpret_cast<unsigned*>(a) + (p >> 1), (p & 1) ? 0x10000u : 1u);
  }
}

template <int NT, class IT>
__device__ void cloud_tail(const float* __restrict__ X, int d, int64_t c0, int nb, int64_t eo, int b,
                           const float* __restrict__ ow, float* __restrict__ W, float* __restrict__ grad,
                           const IT* __restrict__ par, IT* __restrict__ endp, IT* __restrict__ kid,
                           const float* __restrict__ wv, float* __restrict__ ss, float* __restrict__ ee) {
  const int t = threadIdx.x, grp = t >> 4, r16 = t & 15;
  constexpr int NG = NT / 16;
  // ---- tree weight, compensated, in insertion order
  {
    float sacc = 0.f, cacc = 0.f;
    for (int i = t; i < nb - 1; i += NT) {
      float ns, err;
      two_sum(sacc, ow[eo + i], ns, err);
      sacc = ns;
      cacc += err;
    }
    ss[t] = sacc;
    ee[t] = cacc;
    __syncthreads();
    for (int w = NT / 2; w >= 1; w >>= 1) {
      if (t < w) {
        float ns, err;
        two_sum(ss[t], ss[t + w], ns, err);
        ss[t] = ns;
        ee[t] = ee[t] + ee[t + w] + err;
      }
      __syncthreads();
    }
    if (t == 0) W[b] = ss[0] + ee[0];
  }
  // ---- children lists, stable in child id: counts by LDS atomics; then
  // wave 0 scans them (lane l owns a contiguous stretch of parents) and
  // places the children 64 ids at a time, each group of lanes with the same
  // parent by one ballot (rank = lower lanes of the group), so endp[p] ends
  // as the end of p's list
  for (int j = t; j < nb; j += NT) endp[j] = 0;
  __syncthreads();
  for (int c = 1 + t; c < nb; c += NT) lds_count_add(endp, (int)par[c]);
  __syncthreads();
  if (t < 64) {
    const int lane = t, per = (nb + 63) / 64;
    const int a = min(nb, lane * per), e = min(nb, a + per);
    int sum = 0;
    for (int p = a; p < e; ++p) sum += (int)endp[p];
    int incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(incl, o);
      if (lane >= o) incl += v;
    }
    int run = incl - sum;
    for (int p = a; p < e; ++p) {
      const int cnt = (int)endp[p];
      endp[p] = (IT)run;
      run += cnt;
    }
    for (int base = 1; base < nb; base += 64) {
      const int c = base + lane;
      const bool act = c < nb;
      const int P = act ? (int)par[c] : -1;
      uint64_t todo = __ballot(act);
      while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int P0 = __shfl(P, leader);
        const uint64_t m = __ballot(act && P == P0);
        const int start = (int)endp[P0];
        if (act && P == P0) kid[start + __popcll(m & ((1ull << lane) - 1))] = (IT)c;
        if (lane == leader) endp[P0] = (IT)(start + __popcll(m));
        todo &= ~m;
      }
    }
  }
  __syncthreads();
  // ---- gradient rows, one 16-lane group per row: lane r16 owns the
  // dimensions 4 r16 .. 4 r16 + 3 of each 64 (the chunks of sq32_group);
  // per dimension, (x_v - x_o) / w summed over the edges in list order
  for (int v = grp; v < nb; v += NG) {
    const float* xv = X + (c0 + v) * d;
    float* out = grad + (c0 + v) * d;
    const int k0 = v == 0 ? 0 : (int)endp[v - 1], k1 = (int)endp[v];
    const int e0 = v == 0 ? k0 : k0 - 1;   // the parent edge first
    auto other = [&](int e) { return e < k0 ? (int)par[v] : (int)kid[e]; };
    for (int p0 = 0; p0 < d; p0 += 64) {   // every lane of the group takes every pass
      const int t0 = p0 + 4 * r16;
      float a4[4], v4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a4[q] = 0.f;
        v4[q] = t0 + q < d ? xv[t0 + q] : 0.f;
      }
      for (int e = e0; e < k1; ++e) {
        const int o = other(e);
        const float* xo = X + (c0 + o) * d;
        float w;
        if (wv) {
          w = wv[e < k0 ? v : o];
        } else {
          w = __builtin_sqrtf(sq32_group(xv, xo, d, r16));
        }
        if (w == 0.f) continue;
        float o4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) o4[q] = t0 + q < d ? xo[t0 + q] : 0.f;
#pragma unroll
        for (int q = 0; q < 4; ++q) a4[q] += (v4[q] - o4[q]) / w;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (t0 + q < d) out[t0 + q] = a4[q];
    }
  }
  __syncthreads();
}

// Persistent exact-tree kernel for a batch of clouds (d > 64): blocks pull
// clouds from an atomic queue (largest first) and, for each, run dense Prim
// with the distances on the fly, then cloud_tail, all in one launch.  Tree
// edges are written in Prim insertion order as (parent, child).  VEC: d ==
// 64 and rows 16-byte aligned.
template <int NT, bool VEC>
__global__ __launch_bounds__(NT) void prim_fused_kernel(
    const float* __restrict__ X, int d, const int64_t* __restrict__ offs, const int* __restrict__ order,
    int B, int* __restrict__ queue, int32_t* __restrict__ ou, int32_t* __restrict__ ov,
    float* __restrict__ ow, float* __restrict__ W, float* __restrict__ grad) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  uint64_t* keys = reinterpret_cast<uint64_t*>(smem);              // Prim candidate list
  int* par = reinterpret_cast<int*>(keys + FUSED_MAX);            // tree parent of each vertex
  int* endp = reinterpret_cast<int*>(smem);                       // after Prim: list ends ...
  int* kid = endp + FUSED_MAX;                                    // ... and children lists
  __shared__ uint64_t wkeys[2 * NT / 64];
  __shared__ float ss[NT], ee[NT];
  __shared__ int cloud_s, mcount;
  const int t = threadIdx.x;
  while (true) {
    if (t == 0) {
      int idx = atomicAdd(queue, 1);
      cloud_s = idx < B ? order[idx] : -1;
    }
    __syncthreads();
    const int b = cloud_s;
    __syncthreads();   // every thread has read cloud_s before it is rewritten
    if (b < 0) break;
    const int64_t c0 = offs[b];
    const int nb = (int)(offs[b + 1] - c0);
    const int64_t eo = c0 - b;
    if (t == 0) par[0] = -1;
    auto emit = [&](int step, int p, int j, float w) {
      par[j] = p;
      ou[eo + step - 1] = (int32_t)(c0 + p);
      ov[eo + step - 1] = (int32_t)(c0 + j);
      ow[eo + step - 1] = w;
    };
    prim_cloud<NT, VEC, FUSED_MAX / NT>(X, d, c0, nb, keys, wkeys, &mcount, emit);
    __threadfence_block();
    __syncthreads();
    cloud_tail<NT, int>(X, d, c0, nb, eo, b, ow, W, grad, par, endp, kid, nullptr, ss, ee);
  }
}

// Exact trees for d <= 64 in one persistent launch: the pair matrices and
// Prim over them.  The work is a list of items taken from an atomic queue:
// for each cloud, in the processing order (largest first), its tiles in
// items of up to EXACT_TPI tiles, then one Prim item that runs
// prim_cloud_dm over the finished matrix and cloud_tail.  A Prim item waits
// until done[cpos] counts all tiles of its cloud.  The wait always ends:
// every tile item of the cloud sits before it in the list, so it has been
// taken by a block that is running, and tile items wait for nothing.  A
// bounded spin (EXACT_SPIN_MAX sleeps) sets *err instead of waiting on.
// Tiles publish their stores with one agent-scope release per item (an L2
// write-back, costly enough that one per wave per item doubled the launch)
// with the count; the Prim side reads the count and takes an agent-scope
// acquire before its rows, so matrix rows written on another XCD are seen
// (without the pair the trees come out wrong).  No path of the item loop
// leaves thread 0 out of a barrier (a `continue` after its divergent update
// let the compiler send the other threads round the loop without it).
// Item (64 bits): cloud position << 32 | low; low == EXACT_PRIM: the Prim
// item; else tiles s .. s + c of the cloud, low = s << EXACT_TPI_BITS | c.
constexpr uint32_t EXACT_PRIM = 0x80000000u;
constexpr int EXACT_TPI_BITS = 6, EXACT_TPI = 1 << EXACT_TPI_BITS;   // tiles per item at most
// s_waitcnt immediate with vmcnt = 0 and no wait on the other counters
constexpr int WAIT_VMCNT0 = 0x0F70;
constexpr int EXACT_SPIN_MAX = 1 << 22;

// items of the group's clouds from ipre (prefix of the per-cloud item
// counts) and tpre (prefix of the per-cloud tile counts), one thread per item
__global__ void exact_items_kernel(const int64_t* __restrict__ ipre, const int64_t* __restrict__ tpre, int nc,
                                   uint64_t* __restrict__ items) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= ipre[nc]) return;
  int lo = 0, hi = nc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ipre[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  const int64_t li = x - ipre[lo], nit = ipre[lo + 1] - ipre[lo], nt = tpre[lo + 1] - tpre[lo];
  uint32_t low = EXACT_PRIM;
  if (li < nit - 1) {
    const int64_t s = li * EXACT_TPI;
    low = (uint32_t)(s << EXACT_TPI_BITS) | (uint32_t)(min<int64_t>(EXACT_TPI, nt - s) - 1);
  }
  items[x] = ((uint64_t)(uint32_t)lo << 32) | low;
}

constexpr size_t EXACT_LDS = (size_t)2 * PRIM_NT_DM / PD_NT * PD_T * PD_LD * sizeof(float);

__global__ __launch_bounds__(PRIM_NT_DM) void exact_tree_kernel(
    const float* __restrict__ X, int d, const int64_t* __restrict__ offs, const int* __restrict__ order,
    const uint64_t* __restrict__ items, int64_t nitems, const int64_t* __restrict__ dmoff,
    float* __restrict__ D, int* __restrict__ queue, int* __restrict__ done, int* __restrict__ err,
    int32_t* __restrict__ ou, int32_t* __restrict__ ov, float* __restrict__ ow, float* __restrict__ W,
    float* __restrict__ grad) {
  constexpr int NT = PRIM_NT_DM, NGT = NT / PD_NT;   // tiles in flight per block
  static_assert(NGT * 2 * PD_T * PD_LD * sizeof(float) <= EXACT_LDS, "tile buffers fit");
  static_assert(FUSED_MAX * (3 * sizeof(uint16_t) + sizeof(float)) <= EXACT_LDS, "Prim arrays fit");
  static_assert(FUSED_MAX <= 65536, "16-bit local ids");
  extern __shared__ __attribute__((aligned(16))) char smem[];
  float* wv = reinterpret_cast<float*>(smem);                    // weight of each vertex's parent edge
  uint16_t* endp = reinterpret_cast<uint16_t*>(wv + FUSED_MAX);  // after Prim: list ends ...
  uint16_t* kid = endp + FUSED_MAX;                              // ... and children lists
  uint16_t* par = kid + FUSED_MAX;                               // tree parent of each vertex
  __shared__ uint64_t wkeys[2 * NT / 64];
  __shared__ float ss[NT], ee[NT];
  __shared__ uint64_t item_s;
  const int t = threadIdx.x, g = t / PD_NT;
  float* As = reinterpret_cast<float*>(smem) + g * 2 * PD_T * PD_LD;
  float* Bs = As + PD_T * PD_LD;
  // Thread 0 alone talks to the queue and the counters, always right before
  // a barrier of the whole block and never on a path that skips one: the
  // count of a finished tile item is added when the next item is taken.
  int pend_c = -1, pend_n = 0;
  while (true) {
    if (t == 0) {
      if (pend_c >= 0) __hip_atomic_fetch_add(done + pend_c, pend_n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      const int idx = atomicAdd(queue, 1);
      item_s = idx < nitems ? items[idx] : ~0ull;
    }
    __syncthreads();
    const uint64_t it = item_s;
    __syncthreads();   // every thread has read item_s before it is rewritten
    if (it == ~0ull) break;
    const int cpos = (int)(it >> 32);
    const uint32_t low = (uint32_t)it;
    const int b = order[cpos];
    const int64_t c0 = offs[b];
    const int nb = (int)(offs[b + 1] - c0);
    float* Dc = D + dmoff[b];
    if (low != EXACT_PRIM) {
      const int s0 = (int)(low >> EXACT_TPI_BITS), cnt = (int)(low & (EXACT_TPI - 1)) + 1;
      for (int p = 0; p < cnt; p += NGT)
        pair_tile(X, d, c0, nb, s0 + p + g, p + g < cnt, As, Bs, t & (PD_NT - 1), Dc);
      // every wave's matrix stores have reached its XCD's L2 before the
      // barrier (vmcnt(0)); thread 0's agent-scope release then writes that
      // L2 back once per item, before the count is raised
      __builtin_amdgcn_s_waitcnt(WAIT_VMCNT0);
      __syncthreads();
      pend_c = cpos;
      pend_n = cnt;
    } else {
      pend_c = -1;
      if (t == 0) {
        const int T = (nb + PD_T - 1) / PD_T, need = T * (T + 1) / 2;
        int spins = 0;
        while (__hip_atomic_load(done + cpos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          __builtin_amdgcn_s_sleep(8);
          if (++spins == EXACT_SPIN_MAX) {
            atomicOr(err, 1);
            break;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        par[0] = 0xFFFF;
      }
      __syncthreads();
      const int64_t eo = c0 - b;
      auto emit = [&](int step, int p, int j, float w) {
        par[j] = (uint16_t)p;
        wv[j] = w;
        ou[eo + step - 1] = (int32_t)(c0 + p);
        ov[eo + step - 1] = (int32_t)(c0 + j);
        ow[eo + step - 1] = w;
      };
      prim_cloud_dm<NT, FUSED_MAX / NT>(Dc, nb, wkeys, emit);
      __threadfence_block();
      __syncthreads();
      cloud_tail<NT, uint16_t>(X, d, c0, nb, eo, b, ow, W, grad, par, endp, kid, wv, ss, ee);
    }
  }
}

__global__ void pair_keys_kernel(const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                                 const float* __restrict__ w, int64_t m, uint64_t* __restrict__ keys,
                                 uint32_t* __restrict__ vals) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  keys[e] = ((uint64_t)(uint32_t)a[e] << 32) | (uint32_t)b[e];
  vals[e] = __float_as_uint(w[e]);
}

__global__ void unpack_tree_kernel(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                   int64_t m, int32_t* __restrict__ tu, int32_t* __restrict__ tv,
                                   float* __restrict__ tw) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  tu[e] = (int32_t)(keys[e] >> 32);
  tv[e] = (int32_t)(uint32_t)keys[e];
  tw[e] = __uint_as_float(vals[e]);
}

}  // namespace famst

using namespace famst;

extern "C" int famst_mst(const float* X, int64_t n, int32_t d, const int64_t* offs_h, int32_t B,
                         const int32_t* nbr, const float* dist, int32_t k, const int32_t* eu,
                         const int32_t* ev, const float* ew, int64_t n_edges, int32_t algo,
                         int32_t* tu, int32_t* tv, float* tw, float* W, void* ws, size_t* ws_bytes,
                         void* stream) {
  if (!ws_bytes) return FAMST_EINVAL;
  if (n < 2 || B < 1 || k < 0 || n_edges < 0) return FAMST_EINVAL;
  if (algo != FAMST_BORUVKA && algo != FAMST_KRUSKAL && algo != FAMST_DENSE_PRIM) return FAMST_EINVAL;
  if (n >= (int64_t(1) << 31)) return FAMST_EINVAL;
  int64_t one[2] = {0, n};
  const int64_t* offs = offs_h ? offs_h : one;
  if (!offs_h && B != 1) return FAMST_EINVAL;
  if (offs[0] != 0 || offs[B] != n) return FAMST_EINVAL;
  int64_t nbmax = 0;
  for (int b = 0; b < B; ++b) {
    int64_t nb = offs[b + 1] - offs[b];
    if (nb < 2) return FAMST_EINVAL;
    nbmax = std::max(nbmax, nb);
  }
  const int64_t nt = n - B;  // tree edges
  Carve cv(ws);
  int64_t* offs_d = cv.take<int64_t>(B + 1);
  int* bad = cv.take<int>(2);
  if (algo == FAMST_DENSE_PRIM) {
    if (d < 1) return FAMST_EINVAL;
    if (nbmax > PRIM_MAX) return FAMST_ENOTIMPL;
    int32_t* pu = cv.take<int32_t>(nt);
    int32_t* pv = cv.take<int32_t>(nt);
    float* pw = cv.take<float>(nt);
    uint64_t* k1 = cv.take<uint64_t>(nt);
    uint64_t* k2 = cv.take<uint64_t>(nt);
    uint32_t* v1 = cv.take<uint32_t>(nt);
    uint32_t* v2 = cv.take<uint32_t>(nt);
    size_t tmpb = sort_pairs_u64_u32_bytes(nt);
    void* tmp = cv.take<char>(tmpb);
    if (!ws) {
      *ws_bytes = cv.bytes();
      return FAMST_OK;
    }
    if (*ws_bytes < cv.bytes() || (reinterpret_cast<uintptr_t>(ws) & 255)) return FAMST_EWORKSPACE;
    if (!X || !tu || !tv || !tw || !W) return FAMST_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    FAMST_HIP(hipMemcpyAsync(offs_d, offs, sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, s));
    static bool attr = false;
    if (!attr) {
      FAMST_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(prim_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, PRIM_MAX * 8));
      attr = true;
    }
    const int vec = (d == 64) && (reinterpret_cast<uintptr_t>(X) % 16 == 0);
    FAMST_TRY(launch("dense_prim", prim_kernel, dim3(B), dim3(PRIM_NT), (size_t)PRIM_MAX * 8, s, X, d,
                     offs_d, vec, pu, pv, pw));
    FAMST_TRY(launch("pair_keys", pair_keys_kernel, dim3(cdiv(nt, 256)), dim3(256), 0, s, pu, pv, pw,
                     nt, k1, v1));
    FAMST_TRY(sort_pairs_u64_u32(tmp, tmpb, k1, k2, v1, v2, nt, 32 + bits_for(n), s));
    FAMST_TRY(launch("unpack_tree", unpack_tree_kernel, dim3(cdiv(nt, 256)), dim3(256), 0, s, k2, v2,
                     nt, tu, tv, tw));
    FAMST_TRY(launch("tree_weight", tree_weight_kernel, dim3(B), dim3(256), 0, s, tw, offs_d, W));
    return FAMST_OK;
  }

  const int64_t m0 = n * (int64_t)k + n_edges;
  uint64_t* keys = cv.take<uint64_t>(m0);
  uint64_t* skeys = cv.take<uint64_t>(m0);
  uint32_t* vals = cv.take<uint32_t>(m0);
  uint32_t* svals = cv.take<uint32_t>(m0);
  int64_t* flag = cv.take<int64_t>(m0 + 1);
  int64_t* pos = cv.take<int64_t>(m0 + 1);
  int32_t* elo = cv.take<int32_t>(m0);
  int32_t* ehi = cv.take<int32_t>(m0);
  uint32_t* ewb = cv.take<uint32_t>(m0);
  uint8_t* in_tree = cv.take<uint8_t>((m0 + 3) / 4 * 4);   // whole 32-bit words (cleared as such)
  uint32_t* liveA = cv.take<uint32_t>(m0);
  uint32_t* liveB = cv.take<uint32_t>(m0);
  int32_t* comp = cv.take<int32_t>(n);
  int32_t* P = cv.take<int32_t>(n);
  unsigned long long* best = cv.take<unsigned long long>(n);
  int* hooked = cv.take<int>(1);
  size_t tmpb = std::max(sort_pairs_u64_u32_bytes(m0), scan_i64_bytes(m0 + 1));
  tmpb = std::max(tmpb, sort_keys_u64_bytes(m0));
  void* tmp = cv.take<char>(tmpb);
  if (!ws) {
    *ws_bytes = cv.bytes();
    return FAMST_OK;
  }
  if (*ws_bytes < cv.bytes() || (reinterpret_cast<uintptr_t>(ws) & 255)) return FAMST_EWORKSPACE;
  if (!tu || !tv || !tw || !W) return FAMST_EINVAL;
  if (k > 0 && (!nbr || !dist)) return FAMST_EINVAL;
  if (n_edges > 0 && (!eu || !ev || !ew)) return FAMST_EINVAL;
  if (m0 >= (int64_t(1) << 32)) return FAMST_ENOTIMPL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  FAMST_HIP(hipMemcpyAsync(offs_d, offs, sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, s));
  FAMST_HIP(hipMemsetAsync(bad, 0, 2 * sizeof(int), s));
  FAMST_TRY(launch("mst_keys", mst_keys_kernel, dim3(cdiv(m0, 256)), dim3(256), 0, s, nbr, dist, n, k,
                   eu, ev, ew, n_edges, offs_d, B, keys, vals, bad));
  // (min << 32 | max) keys need 32 + bits_for(n) bits; KEY_NONE is all ones
  // there too, so it still sorts after every edge
  FAMST_TRY(sort_pairs_u64_u32(tmp, tmpb, keys, skeys, vals, svals, m0, 32 + bits_for(n), s));
  FAMST_TRY(launch("edge_unique", edge_unique_kernel, dim3(cdiv(m0, 256)), dim3(256), 0, s, skeys, m0,
                   flag));
  FAMST_HIP(hipMemsetAsync(flag + m0, 0, sizeof(int64_t), s));
  FAMST_TRY(exclusive_scan_i64(tmp, tmpb, flag, pos, m0 + 1, s));
  FAMST_TRY(launch("edge_compact", edge_compact_kernel, dim3(cdiv(m0, 256)), dim3(256), 0, s, skeys,
                   svals, flag, pos, m0, elo, ehi, ewb));
  int64_t m = 0;
  int hbad = 0;
  if (algo == FAMST_BORUVKA && n <= BV1_MAXN && m0 <= BV1_MAXM) {
    // small input: all rounds in one block; the edge count stays on the
    // device (the kernels below run over all m0 slots, zero past m), and
    // invalid edges are reported after the tree
    FAMST_TRY(fill_i32(reinterpret_cast<int32_t*>(in_tree), 0, (size_t)(m0 + 3) / 4, s));
    static bool attr = false;
    const size_t lds = (size_t)BV1_MAXN * 12;
    if (!attr) {
      FAMST_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(bv_block_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      attr = true;
    }
    FAMST_TRY(launch("boruvka_block", bv_block_kernel, dim3(1), dim3(BV1_NT), (size_t)n * 12, s, elo, ehi, ewb,
                     pos + m0, (int)n, in_tree));
    FAMST_TRY(launch("tree_flags", u8_to_i64_kernel, dim3(cdiv(m0 + 1, 256)), dim3(256), 0, s, in_tree, m0,
                     flag));
    FAMST_TRY(exclusive_scan_i64(tmp, tmpb, flag, pos, m0 + 1, s));
    int64_t cnt = 0;
    FAMST_HIP(hipMemcpyAsync(&cnt, pos + m0, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FAMST_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    FAMST_HIP(hipStreamSynchronize(s));
    if (hbad) return FAMST_EINVAL;
    if (cnt != nt) return FAMST_EDISCONNECTED;
    FAMST_TRY(launch("tree_compact", tree_compact_kernel, dim3(cdiv(m0, 256)), dim3(256), 0, s, in_tree,
                     pos, m0, elo, ehi, ewb, tu, tv, tw));
    FAMST_TRY(launch("tree_weight", tree_weight_kernel, dim3(B), dim3(256), 0, s, tw, offs_d, W));
    return FAMST_OK;
  }
  FAMST_HIP(hipMemcpyAsync(&m, pos + m0, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  FAMST_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  FAMST_HIP(hipStreamSynchronize(s));
  if (hbad) return FAMST_EINVAL;
  FAMST_HIP(hipMemsetAsync(in_tree, 0, m, s));
  if (algo == FAMST_BORUVKA) {
    FAMST_TRY(iota_i32(comp, n, s));
    FAMST_TRY(iota_i32(reinterpret_cast<int32_t*>(liveA), m, s));
    uint32_t* cur = liveA;
    uint32_t* nxt = liveB;
    int64_t nlive = m;
    for (int round = 0; round < 64 && nlive > 0; ++round) {
      FAMST_TRY(fill_u64(reinterpret_cast<uint64_t*>(best), KEY_NONE, n, s));
      FAMST_HIP(hipMemsetAsync(hooked, 0, sizeof(int), s));
      // chunks of 64 live entries; one cloud: in order; several: a stride
      // coprime to the chunk count (checked)
      const uint64_t nchunk = (uint64_t)(nlive + 63) / 64;
      uint64_t stride = 1;
      if (B > 1) {
        stride = 1009;
        while (std::gcd(stride, nchunk) != 1) stride += 2;
      }
      FAMST_TRY(launch("boruvka_min", bv_min_edge_kernel, dim3(cdiv(nlive, 256)), dim3(256), 0, s, elo,
                       ehi, ewb, cur, nlive, stride % nchunk, comp, best, flag));
      FAMST_TRY(launch("boruvka_hook", bv_hook_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, elo, ehi,
                       n, comp, best, P, in_tree, hooked));
      FAMST_TRY(launch("boruvka_jump", bv_jump_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, comp, n,
                       P));
      FAMST_TRY(launch("boruvka_relabel", bv_relabel_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, comp,
                       P, n));
      // drop edges that were inside one component before this round's hooks
      FAMST_HIP(hipMemsetAsync(flag + nlive, 0, sizeof(int64_t), s));
      FAMST_TRY(exclusive_scan_i64(tmp, tmpb, flag, pos, nlive + 1, s));
      FAMST_TRY(launch("boruvka_compact", bv_compact_kernel, dim3(cdiv(nlive, 256)), dim3(256), 0, s,
                       cur, flag, pos, nlive, nxt));
      int hh = 0;
      int64_t nl = 0;
      FAMST_HIP(hipMemcpyAsync(&hh, hooked, sizeof(int), hipMemcpyDeviceToHost, s));
      FAMST_HIP(hipMemcpyAsync(&nl, pos + nlive, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      FAMST_HIP(hipStreamSynchronize(s));
      std::swap(cur, nxt);
      nlive = nl;
      if (!hh) break;
    }
  } else {
    FAMST_TRY(launch("kruskal_keys", kr_keys_kernel, dim3(cdiv(m, 256)), dim3(256), 0, s, ewb, m,
                     keys));
    FAMST_TRY(sort_keys_u64(tmp, tmpb, keys, skeys, m, 64, s));
    FAMST_TRY(iota_i32(P, n, s));
    FAMST_TRY(launch("kruskal_scan", kr_scan_kernel, dim3(1), dim3(64), 0, s, skeys, m, elo, ehi, P,
                     nt, in_tree));
  }
  FAMST_TRY(launch("tree_flags", u8_to_i64_kernel, dim3(cdiv(m + 1, 256)), dim3(256), 0, s, in_tree, m,
                   flag));
  FAMST_TRY(exclusive_scan_i64(tmp, tmpb, flag, pos, m + 1, s));
  int64_t cnt = 0;
  FAMST_HIP(hipMemcpyAsync(&cnt, pos + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  FAMST_HIP(hipStreamSynchronize(s));
  if (cnt != nt) return FAMST_EDISCONNECTED;
  FAMST_TRY(launch("tree_compact", tree_compact_kernel, dim3(cdiv(m, 256)), dim3(256), 0, s, in_tree,
                   pos, m, elo, ehi, ewb, tu, tv, tw));
  FAMST_TRY(launch("tree_weight", tree_weight_kernel, dim3(B), dim3(256), 0, s, tw, offs_d, W));
  return FAMST_OK;
}

template <int NT, bool VEC>
static int launch_fused(dim3 grid, hipStream_t s, const float* X, int d, const int64_t* offs, const int* order, int nc,
                        int* queue, int32_t* tu, int32_t* tv, float* tw, float* W, float* grad) {
  auto kern = prim_fused_kernel<NT, VEC>;
  const size_t lds = (size_t)3 * FUSED_MAX * 4;
  static bool attr = false;
  if (!attr) {
    FAMST_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds));
    attr = true;
  }
  return launch("dense_prim_fused", kern, grid, dim3(NT), lds, s, X, d, offs, order, nc, queue, tu, tv, tw, W, grad);
}

extern "C" int famst_mst_dense_fused(const float* X, int64_t n, int32_t d, const int64_t* offs_h,
                                     int32_t B, int32_t* tu, int32_t* tv, float* tw, float* W,
                                     float* grad_X, void* ws, size_t* ws_bytes, void* stream) {
  if (!ws_bytes) return FAMST_EINVAL;
  if (n < 2 || d < 1 || B < 1) return FAMST_EINVAL;
  if (n >= (int64_t(1) << 31)) return FAMST_EINVAL;
  int64_t one[2] = {0, n};
  const int64_t* offs = offs_h ? offs_h : one;
  if (!offs_h && B != 1) return FAMST_EINVAL;
  if (offs[0] != 0 || offs[B] != n) return FAMST_EINVAL;
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) {
    int64_t nb = offs[b + 1] - offs[b];
    if (nb < 2) return FAMST_EINVAL;
    if (nb > FUSED_MAX) return FAMST_ENOTIMPL;
    order[b] = b;
  }
  // largest clouds first (longest-processing-time order), ties by index
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return offs[a + 1] - offs[a] > offs[b + 1] - offs[b];
  });
  // d <= 64: pair matrices (nb^2 floats per cloud); the size query asks for
  // all of them at once, and a smaller workspace that still holds the
  // largest cloud's matrix runs the clouds in consecutive groups that fit
  const bool dm = d <= DMAT_MAXD;
  int64_t mtot = 0, mmax = 0, itot = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t nb = offs[b + 1] - offs[b], T = (nb + PD_T - 1) / PD_T;
    mtot += nb * nb;
    mmax = std::max(mmax, nb * nb);
    itot += (T * (T + 1) / 2 + EXACT_TPI - 1) / EXACT_TPI + 1;
  }
  Carve cv(ws);
  int64_t* offs_d = cv.take<int64_t>(B + 1);
  int* order_d = cv.take<int>(B);
  int* queue = cv.take<int>(2);   // queue, error flag
  int64_t* dmoff_d = cv.take<int64_t>(dm ? B : 0);
  // per group: prefixes of the clouds' tile and item counts (B + groups + ... <= 2 B + 1 entries)
  int64_t* tpre_d = cv.take<int64_t>(dm ? 2 * B + 1 : 0);
  int64_t* ipre_d = cv.take<int64_t>(dm ? 2 * B + 1 : 0);
  int* done_d = cv.take<int>(dm ? B : 0);
  uint64_t* items_d = cv.take<uint64_t>(dm ? itot : 0);
  const size_t fixed = cv.bytes();
  // the matrices, then FUSED_MAX zeros that the last Prim slots may read
  float* D = cv.take<float>(dm ? mtot + FUSED_MAX : 0);
  // the queue hands out item indices from a 32-bit counter (each block takes
  // one index past the end)
  if (dm && itot > (int64_t)INT32_MAX - 65536) return FAMST_ENOTIMPL;
  if (!ws) {
    *ws_bytes = cv.bytes();
    return FAMST_OK;
  }
  const size_t need = dm ? fixed + (size_t)(mmax + FUSED_MAX) * 4 : cv.bytes();
  if (*ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255)) return FAMST_EWORKSPACE;
  if (!X || !tu || !tv || !tw || !W || !grad_X) return FAMST_EINVAL;
  // groups of clouds (consecutive in the processing order) whose matrices fit
  const int64_t cap = dm ? (int64_t)((*ws_bytes - fixed) / 4) - FUSED_MAX : 0;
  std::vector<int> gstart{0};
  std::vector<int64_t> dmoff(dm ? B : 0), tpre, ipre, gused;   // gused: matrix floats of each group
  if (dm) {
    int64_t used = 0, tiles = 0, its = 0;
    tpre.push_back(0);
    ipre.push_back(0);
    for (int i = 0; i < B; ++i) {
      const int b = order[i];
      const int64_t nb = offs[b + 1] - offs[b], T = (nb + PD_T - 1) / PD_T, nt = T * (T + 1) / 2;
      if (used + nb * nb > cap) {   // start a new group
        gstart.push_back(i);
        gused.push_back(used);
        used = tiles = its = 0;
        tpre.push_back(0);
        ipre.push_back(0);
      }
      dmoff[b] = used;
      used += nb * nb;
      tiles += nt;
      its += (nt + EXACT_TPI - 1) / EXACT_TPI + 1;
      tpre.push_back(tiles);
      ipre.push_back(its);
    }
    gused.push_back(used);
  }
  gstart.push_back(B);
  hipStream_t s = static_cast<hipStream_t>(stream);
  FAMST_HIP(hipMemcpyAsync(offs_d, offs, sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, s));
  FAMST_HIP(hipMemcpyAsync(order_d, order.data(), sizeof(int) * B, hipMemcpyHostToDevice, s));
  if (dm) {
    FAMST_HIP(hipMemcpyAsync(dmoff_d, dmoff.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice, s));
    FAMST_HIP(hipMemcpyAsync(tpre_d, tpre.data(), sizeof(int64_t) * tpre.size(), hipMemcpyHostToDevice, s));
    FAMST_HIP(hipMemcpyAsync(ipre_d, ipre.data(), sizeof(int64_t) * ipre.size(), hipMemcpyHostToDevice, s));
  }
  FAMST_HIP(hipStreamSynchronize(s));  // host arrays copied before they go out of scope
  int dev = 0, ncu = 256;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  FAMST_TRY(fill_i32(queue, 0, 2, s));
  for (size_t gi = 0; gi + 1 < gstart.size(); ++gi) {
    const int g0 = gstart[gi], nc = gstart[gi + 1] - g0;
    if (dm) {
      // the group's prefixes sit at [g0 + gi .. g0 + gi + nc]
      const int64_t nit = ipre[g0 + gi + nc];
      FAMST_TRY(fill_i32(reinterpret_cast<int32_t*>(D + gused[gi]), 0, FUSED_MAX, s));
      FAMST_TRY(fill_i32(queue, 0, 1, s));
      FAMST_TRY(fill_i32(done_d, 0, nc, s));
      FAMST_TRY(launch("exact_items", exact_items_kernel, dim3(cdiv(nit, 256)), dim3(256), 0, s,
                       ipre_d + g0 + gi, tpre_d + g0 + gi, nc, items_d));
      static bool attr = false;
      if (!attr) {
        FAMST_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(exact_tree_kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)EXACT_LDS));
        attr = true;
      }
      FAMST_TRY(launch("exact_tree", exact_tree_kernel, dim3((unsigned)std::min<int64_t>(nit, ncu)),
                       dim3(PRIM_NT_DM), EXACT_LDS, s, X, d, offs_d, order_d + g0, items_d, nit, dmoff_d, D, queue,
                       done_d, queue + 1, tu, tv, tw, W, grad_X));
      continue;
    }
    FAMST_TRY(fill_i32(queue, 0, 1, s));
    const dim3 grid(std::min(nc, ncu));
    if ((d == 64) && (reinterpret_cast<uintptr_t>(X) % 16 == 0))
      FAMST_TRY((launch_fused<PRIM_NT, true>(grid, s, X, d, offs_d, order_d + g0, nc, queue, tu, tv, tw, W,
                                             grad_X)));
    else
      FAMST_TRY((launch_fused<PRIM_NT, false>(grid, s, X, d, offs_d, order_d + g0, nc, queue, tu, tv, tw, W,
                                              grad_X)));
  }
  if (dm) {
    // the bounded wait of a Prim item ran out: the outputs are not valid
    int e = 0;
    FAMST_HIP(hipMemcpyAsync(&e, queue + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    FAMST_HIP(hipStreamSynchronize(s));
    if (e) return FAMST_ETIMEOUT;
  }
  return FAMST_OK;
}
