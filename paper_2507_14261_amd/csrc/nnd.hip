// Phase 1 by NN-Descent (Dong, Charikar and Li, WWW 2011), the method family
// of the paper's own Phase 1 (PyNNDescent, Sec. 3): approximate k nearest
// neighbours grown by local joins instead of the exact quadratic scan.
// Every point keeps a sorted list of K candidates (squared distance, id,
// "new" flag).  One iteration:
//   sample  each list gives up to S of its new entries (the closest; they
//           turn old) and up to S old ones (a window that moves along the
//           old entries from one iteration to the next), and registers
//           itself in the
//           reverse samples of those points (S hashed buckets each);
//   join    for each point v, with C = its new samples and reverse new
//           samples and D = the old ones, every pair of C x C and C x D is
//           measured (rows staged in LDS) and each endpoint is proposed to
//           the other when it beats that list's current worst entry; a
//           point's proposals go to CB buckets chosen by a hash of the
//           proposed id, each keeping its smallest (s, id) by a 64-bit
//           atomic minimum (repeated ids land in one bucket);
//   merge   every list is merged with its proposals: one wave sorts the 64
//           (s, key) pairs, drops duplicates and keeps the K smallest;
//           entries that came from proposals are new.
// Iterations stop when fewer than delta n K entries change, or at a cap.
// All distances are the canonical float32 direct-difference values, so a
// pair always gets the same bits and duplicates compare equal.
#include "famst_common.hpp"
#include "prims.hpp"
#include "sortnet.hpp"

namespace famst {

constexpr int NND_K = 32;       // list length (k <= 32)
constexpr int NND_S = 8;        // samples per list side, reverse slots per point
constexpr int NND_CB = 32;      // proposal slots per point and iteration
constexpr int NND_MAXD = 256;   // dimensions the local join stages in LDS
constexpr int NND_MAXIT = 32;   // iteration cap
constexpr int NND_EMPTY = 0x7FFFFFFF;

struct NndArgs {
  const float* X;
  int d;
  int64_t n;
  const int64_t* offs;
  int B;
  int* lid;       // [n][K] ids (NND_EMPTY: none)
  float* ls;      // [n][K] squared distances, ascending with the ids
  uint8_t* lnew;  // [n][K] new flags
  float* worst;   // [n] K-th entry (+inf while fewer)
  int* snew;      // [n][S] sampled new entries (-1: none)
  int* sold;      // [n][S] sampled old entries
  // reverse samples: S buckets per point chosen by a hash of the sampling
  // point, each keeping the smallest (hash, id) by a 64-bit atomic minimum,
  // so the choice does not depend on the order of arrival (all ones: empty)
  unsigned long long* rnew;   // [n][S]
  unsigned long long* rold;   // [n][S]
  unsigned long long* cb;   // [n][CB] proposal buckets: s bits << 32 | id (all ones: empty)
  unsigned long long* upd;
};

// Sorted (s, key) of a wave written back as the list: keys are
// id << 2 | from-proposal << 1 | new flag, so equal ids sit next to each
// other after the sort with the list's own copy first; duplicates are
// dropped and the K smallest kept.  Returns the number of kept entries that
// came from proposals (lane-uniform) and stores the K-th distance.
__device__ __forceinline__ int nnd_store(const NndArgs& a, int64_t v, float s, uint32_t key, int lane) {
  const uint32_t pk = (uint32_t)__shfl_up((int)key, 1);
  const float ps = __shfl_up(s, 1);
  const bool dup = lane > 0 && (pk >> 2) == (key >> 2) && ps == s;
  const bool keep = !dup && s < F_INF;
  const unsigned long long km = ballot(keep);
  const int pos = __builtin_popcountll(km & ((1ull << lane) - 1));
  const int cnt = __builtin_popcountll(km);
  const bool fromp = (key & 2u) != 0;
  if (keep && pos < NND_K) {
    a.lid[v * NND_K + pos] = (int)(key >> 2);
    a.ls[v * NND_K + pos] = s;
    a.lnew[v * NND_K + pos] = fromp ? 1 : (uint8_t)(key & 1u);
  }
  if (lane >= cnt && lane < NND_K) {
    a.lid[v * NND_K + lane] = NND_EMPTY;
    a.ls[v * NND_K + lane] = F_INF;
    a.lnew[v * NND_K + lane] = 0;
  }
  const unsigned long long kth = ballot(keep && pos == NND_K - 1);
  const float wst = kth ? readlane_f(s, __builtin_ctzll(kth)) : F_INF;
  if (lane == 0) a.worst[v] = wst;
  return __builtin_popcountll(ballot(keep && fromp && pos < NND_K));
}

// Initial lists of one cloud in spatial order (perm: rows sorted by nearest
// pivot): the point at position p takes the best K of the 64 points at the
// positions around it (a window of 65 positions, shifted inside [0, n)):
// points of its own pivot cell, as a random-projection tree leaf would give.
// One wave per position; lane l measures window slot l (skipping p itself).
__global__ __launch_bounds__(256) void nnd_init_spatial_kernel(NndArgs a, const int* __restrict__ perm) {
  __shared__ float sd[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, grp = lane >> 4, r16 = lane & 15;
  for (int64_t p = (int64_t)blockIdx.x * 4 + w; p < a.n; p += (int64_t)gridDim.x * 4) {
    const int64_t v = perm[p];
    const int64_t p0 = min<int64_t>(max<int64_t>(p - 32, 0), a.n - 65);
    const int64_t q = p0 + lane + (p0 + lane >= p ? 1 : 0);   // the 64 window positions other than p
    const int j = perm[q];
    const float* xv = a.X + v * a.d;
#pragma unroll
    for (int rd = 0; rd < 16; ++rd) {
      const int c = rd * 4 + grp;
      const int jc = __shfl(j, c);
      const float sv = sq32_group(xv, a.X + (int64_t)jc * a.d, a.d, r16);
      if (r16 == 0) sd[w][c] = sv;
    }
    __builtin_amdgcn_wave_barrier();
    float s = sd[w][lane];
    uint32_t key = ((uint32_t)j << 2) | 1u;
    sort64_asc(s, key, lane);
    nnd_store(a, v, s, key, lane);
    __builtin_amdgcn_wave_barrier();
  }
}

// Initial lists: the K points that follow v in its cloud, cyclically
// (distinct, so every list holds min(K, n_b - 1) >= k entries from the
// start), measured and sorted.  One wave per point.
__global__ __launch_bounds__(256) void nnd_init_kernel(NndArgs a) {
  __shared__ float sd[4][NND_K];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, grp = lane >> 4, r16 = lane & 15;
  for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < a.n; v += (int64_t)gridDim.x * 4) {
    const int cb = find_cloud(a.offs, a.B, v);
    const int64_t c0 = a.offs[cb], nb = a.offs[cb + 1] - c0;
    const int m = (int)min<int64_t>(NND_K, nb - 1);
    const int j = lane < m ? (int)(c0 + (v - c0 + 1 + lane) % nb) : -1;
    const float* xv = a.X + v * a.d;
#pragma unroll
    for (int rd = 0; rd < NND_K / 4; ++rd) {
      const int c = rd * 4 + grp;
      const int jc = __shfl(j, c);
      if (jc >= 0) {   // uniform in the group
        const float s = sq32_group(xv, a.X + (int64_t)jc * a.d, a.d, r16);
        if (r16 == 0) sd[w][c] = s;
      }
    }
    __builtin_amdgcn_wave_barrier();
    float s = lane < m ? sd[w][lane] : F_INF;
    uint32_t key = lane < m ? (((uint32_t)j << 2) | 1u) : 0xFFFFFFFFu;
    sort64_asc(s, key, lane);
    nnd_store(a, v, s, key, lane);
    __builtin_amdgcn_wave_barrier();
  }
}

// Samples of one iteration (one wave per point; lane = list entry): the S
// closest new entries, and S old entries taken cyclically from the
// iteration's offset, so every old entry joins within a few iterations.
__global__ __launch_bounds__(256) void nnd_sample_kernel(NndArgs a, int it) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < a.n; v += (int64_t)gridDim.x * 4) {
    int id = NND_EMPTY, fl = 0;
    if (lane < NND_K) {
      id = a.lid[v * NND_K + lane];
      fl = a.lnew[v * NND_K + lane];
    }
    const bool valid = id != NND_EMPTY;
    const bool isn = valid && fl, iso = valid && !fl;
    const unsigned long long below = (1ull << lane) - 1;
    const unsigned long long bn = ballot(isn), bo = ballot(iso);
    const int rn = __builtin_popcountll(bn & below), ro = __builtin_popcountll(bo & below);
    const int nn = __builtin_popcountll(bn), no = __builtin_popcountll(bo);
    const uint32_t hv = (uint32_t)v * 2654435761u;
    const unsigned long long rkey = ((unsigned long long)(hv ^ 0x5bd1e995u) << 32) | (uint32_t)v;
    const int rb = (int)(hv >> 29);   // bucket 0..S-1
    if (isn && rn < NND_S) {
      a.snew[v * NND_S + rn] = id;
      a.lnew[v * NND_K + lane] = 0;   // sampled: old from now on
      atomicMin(&a.rnew[(int64_t)id * NND_S + rb], rkey);
    }
    const int rot = no > NND_S ? (ro - it * NND_S % no + no) % no : ro;   // position in this iteration's window
    if (iso && rot < NND_S) {
      a.sold[v * NND_S + rot] = id;
      atomicMin(&a.rold[(int64_t)id * NND_S + rb], rkey);
    }
    if (lane < NND_S) {
      if (lane >= nn) a.snew[v * NND_S + lane] = -1;
      if (lane >= no) a.sold[v * NND_S + lane] = -1;
    }
  }
}

__device__ __forceinline__ void nnd_propose(const NndArgs& a, int to, int id, float s) {
  if (!(s < a.worst[to])) return;
  // nonnegative floats order like their bit patterns
  const unsigned long long key = ((unsigned long long)__float_as_uint(s) << 32) | (uint32_t)id;
  const uint32_t h = ((uint32_t)id * 2654435761u) >> 27;   // bucket 0..31
  atomicMin(&a.cb[(int64_t)to * NND_CB + h], key);
}

// Local join of one point per 64-lane block (points taken with a stride of
// the grid): slots 0..15 hold the new side (samples, then reverse samples),
// 16..31 the old side; their rows are staged in LDS (dp floats each) and
// every new x new and new x old pair is measured by a 16-lane group.
__global__ __launch_bounds__(64) void nnd_join_kernel(NndArgs a, int dp) {
  extern __shared__ __attribute__((aligned(16))) float rows[];   // [32][dp]
  __shared__ int ids[32];
  const int lane = threadIdx.x, grp = lane >> 4, r16 = lane & 15;
  for (int64_t v = blockIdx.x; v < a.n; v += gridDim.x) {
    if (lane < 32) {
      const int side = lane >> 4, l = lane & 15;
      const int* fw = side ? a.sold : a.snew;
      unsigned long long* rv = side ? a.rold : a.rnew;
      int id = -1;
      if (l < NND_S) {
        id = fw[v * NND_S + l];
      } else {
        unsigned long long& b = rv[v * NND_S + (l - NND_S)];
        if (b != ~0ull) id = (int)(uint32_t)b;
        b = ~0ull;   // empty for the next iteration
      }
      ids[lane] = id;
    }
    __syncthreads();
    for (int r = 0; r < 32; ++r) {
      const int id = ids[r];
      if (id < 0) continue;   // uniform
      const float* src = a.X + (int64_t)id * a.d;
      for (int t = lane; t < dp; t += 64) rows[r * dp + t] = t < a.d ? src[t] : 0.f;
    }
    __syncthreads();
    // pairs: (i, j) with i < j < 16 (120 of them), then i < 16 <= j (256)
    for (int p = grp; p < 120 + 256; p += 4) {
      int i, j;
      if (p < 120) {
        i = 0;
        int rem = p;
        while (rem >= 15 - i) {
          rem -= 15 - i;
          ++i;
        }
        j = i + 1 + rem;
      } else {
        i = (p - 120) >> 4;
        j = 16 + ((p - 120) & 15);
      }
      const int ai = ids[i], bj = ids[j];
      if (ai < 0 || bj < 0 || ai == bj) continue;   // uniform in the group
      const float s = sq32_group(rows + i * dp, rows + j * dp, a.d, r16);
      if (r16 == 0) {
        nnd_propose(a, ai, bj, s);
        nnd_propose(a, bj, ai, s);
      }
    }
    __syncthreads();
  }
}

// Merge of a list with its proposals (one wave per point): lanes 0..31 the
// list, 32..63 the proposal buckets (emptied for the next iteration).
__global__ __launch_bounds__(256) void nnd_merge_kernel(NndArgs a) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < a.n; v += (int64_t)gridDim.x * 4) {
    float s = F_INF;
    uint32_t key = 0xFFFFFFFFu;
    if (lane < NND_K) {
      const int id = a.lid[v * NND_K + lane];
      if (id != NND_EMPTY) {
        s = a.ls[v * NND_K + lane];
        key = ((uint32_t)id << 2) | (uint32_t)a.lnew[v * NND_K + lane];
      }
    } else {
      unsigned long long& slot = a.cb[v * NND_CB + (lane - NND_K)];
      const unsigned long long c = slot;
      if (c != ~0ull) {
        s = __uint_as_float((uint32_t)(c >> 32));
        key = ((uint32_t)c << 2) | 2u;
      }
      slot = ~0ull;   // empty for the next iteration
    }
    sort64_asc(s, key, lane);
    const int ins = nnd_store(a, v, s, key, lane);
    if (lane == 0 && ins) atomicAdd(a.upd, (unsigned long long)ins);
  }
}

// The first k entries of every list as the neighbour lists.
__global__ __launch_bounds__(256) void nnd_output_kernel(const int* __restrict__ lid, const float* __restrict__ ls,
                                                         int64_t n, int k, int32_t* __restrict__ nbr,
                                                         float* __restrict__ dist) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * k) return;
  const int64_t v = i / k, m = i - v * k;
  nbr[i] = lid[v * NND_K + m];
  dist[i] = __builtin_sqrtf(ls[v * NND_K + m]);
}

}  // namespace famst

using namespace famst;

// Workspace layout and run of NN-Descent (called by famst_knn_graph for
// FAMST_NNDESCENT after its argument checks).
namespace famst {
int spatial_perm(const float* X, int64_t n, int d, int* perm, void* ws, size_t* bytes, hipStream_t s);
}

int famst_nndescent_run(const float* X, int64_t n, int32_t d, const int64_t* offs, int32_t B, int32_t k,
                        int32_t* nbr, float* dist, int64_t* stats, void* ws, size_t* ws_bytes, hipStream_t s) {
  if (k > NND_K) return FAMST_ENOTIMPL;
  if (d > NND_MAXD) return FAMST_ENOTIMPL;
  if (n >= (int64_t(1) << 30)) return FAMST_ENOTIMPL;   // ids carry two flag bits in the sort keys
  Carve cv(ws);
  NndArgs a;
  a.X = X;
  a.d = d;
  a.n = n;
  a.B = B;
  int64_t* offs_d = cv.take<int64_t>(B + 1);
  a.offs = offs_d;
  a.lid = cv.take<int>((size_t)n * NND_K);
  a.ls = cv.take<float>((size_t)n * NND_K);
  a.lnew = cv.take<uint8_t>((size_t)n * NND_K);
  a.worst = cv.take<float>(n);
  a.snew = cv.take<int>((size_t)n * NND_S);
  a.sold = cv.take<int>((size_t)n * NND_S);
  a.rnew = cv.take<unsigned long long>((size_t)n * NND_S);
  a.rold = cv.take<unsigned long long>((size_t)n * NND_S);
  a.cb = cv.take<unsigned long long>((size_t)n * NND_CB);
  // one large cloud starts from its spatial order (the pivot cells); batches
  // of clouds from the cyclic successors
  const bool spatial = B == 1 && n >= 4096;
  int* perm = cv.take<int>(spatial ? (size_t)n : 0);
  size_t spb = 0;
  if (spatial) FAMST_TRY(spatial_perm(X, n, d, nullptr, nullptr, &spb, s));
  void* spws = cv.take<char>(spb);
  a.upd = cv.take<unsigned long long>(1);
  if (!ws) {
    *ws_bytes = cv.bytes();
    return FAMST_OK;
  }
  if (*ws_bytes < cv.bytes() || (reinterpret_cast<uintptr_t>(ws) & 255)) return FAMST_EWORKSPACE;
  if (!X || !nbr || !dist) return FAMST_EINVAL;
  FAMST_HIP(hipMemcpyAsync(offs_d, offs, sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, s));
  FAMST_TRY(fill_u64(reinterpret_cast<uint64_t*>(a.cb), ~0ull, (size_t)n * NND_CB, s));
  FAMST_TRY(fill_u64(reinterpret_cast<uint64_t*>(a.rnew), ~0ull, (size_t)n * NND_S, s));
  FAMST_TRY(fill_u64(reinterpret_cast<uint64_t*>(a.rold), ~0ull, (size_t)n * NND_S, s));
  const dim3 wgrid(stride_grid(cdiv(n, 4)));
  if (spatial) {
    FAMST_TRY(spatial_perm(X, n, d, perm, spws, &spb, s));
    FAMST_TRY(launch("nnd_init", nnd_init_spatial_kernel, wgrid, dim3(256), 0, s, a, perm));
  } else {
    FAMST_TRY(launch("nnd_init", nnd_init_kernel, wgrid, dim3(256), 0, s, a));
  }
  const int dp = (d + 3) & ~3;
  const size_t jlds = (size_t)32 * dp * sizeof(float);
  int it = 0;
  unsigned long long last = 0;
  const unsigned long long stop = (unsigned long long)(0.001 * (double)n * NND_K);
  for (; it < NND_MAXIT; ++it) {
    FAMST_TRY(fill_u64(reinterpret_cast<uint64_t*>(a.upd), 0, 1, s));
    FAMST_TRY(launch("nnd_sample", nnd_sample_kernel, wgrid, dim3(256), 0, s, a, it));
    FAMST_TRY(launch("nnd_join", nnd_join_kernel, dim3(stride_grid(n)), dim3(64), jlds, s, a, dp));
    FAMST_TRY(launch("nnd_merge", nnd_merge_kernel, wgrid, dim3(256), 0, s, a));
    FAMST_HIP(hipMemcpyAsync(&last, a.upd, sizeof(last), hipMemcpyDeviceToHost, s));
    FAMST_HIP(hipStreamSynchronize(s));
    if (last <= stop) {
      ++it;
      break;
    }
  }
  FAMST_TRY(launch("nnd_output", nnd_output_kernel, dim3(cdiv(n * k, 256)), dim3(256), 0, s, a.lid, a.ls, n, k,
                   nbr, dist));
  if (stats) {
    FAMST_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < FAMST_NSTATS; ++i) stats[i] = 0;
    stats[FAMST_STAT_K_CAND] = NND_K;
    stats[FAMST_STAT_NND_ITERS] = it;
    stats[FAMST_STAT_NND_UPDATES] = (int64_t)last;
  }
  return FAMST_OK;
}
