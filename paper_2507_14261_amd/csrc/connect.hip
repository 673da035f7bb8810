// Phase 2 of FAMST: the undirected graph G of the neighbour lists and its
// connected components (Alg. 2), then lambda random inter-component edges
// per component pair (Alg. 3).
#include <numeric>
#include <vector>

#include "famst_common.hpp"
#include "prims.hpp"
#include "select.hpp"

namespace famst {

// ---------------------------------------------------------- graph build
// Every neighbour entry gives the two directed keys (i << 32 | j) and
// (j << 32 | i); entries outside the row's cloud are flagged.
__global__ void edge_keys_kernel(const int32_t* __restrict__ nbr, int64_t n, int k,
                                 const int64_t* __restrict__ offs, int B,
                                 uint64_t* __restrict__ keys, int* __restrict__ bad) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  int64_t i = e / k;
  int64_t j = nbr[e];
  bool ok = j >= 0 && j < n;
  if (ok && B > 1) ok = find_cloud(offs, B, i) == find_cloud(offs, B, j);
  if (!ok) {
    atomicOr(bad, 1);
    j = i;  // turned into a self-loop, dropped below
  }
  keys[2 * e] = ((uint64_t)i << 32) | (uint32_t)j;
  keys[2 * e + 1] = ((uint64_t)j << 32) | (uint32_t)i;
}

// keep[p] = first occurrence of a key and not a self-loop
__global__ void unique_flags_kernel(const uint64_t* __restrict__ keys, int64_t m,
                                    int64_t* __restrict__ flag) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  uint64_t kk = keys[p];
  bool keep = (uint32_t)(kk >> 32) != (uint32_t)kk;
  if (p > 0 && keys[p - 1] == kk) keep = false;
  flag[p] = keep ? 1 : 0;
}

// Columns at their scan positions.  The keys are sorted by (row, column),
// so row u starts at the scan position of its first key (kept or not): the
// number of kept keys in the rows before it.  Every row has keys (its own k
// neighbours), and the end is the total.
__global__ void csr_fill_kernel(const uint64_t* __restrict__ keys, const int64_t* __restrict__ flag,
                                const int64_t* __restrict__ pos, int64_t m, int64_t n,
                                int32_t* __restrict__ col, int64_t* __restrict__ row_ptr) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const uint64_t kk = keys[p];
  const uint32_t u = (uint32_t)(kk >> 32);
  if (p == 0 || (uint32_t)(keys[p - 1] >> 32) != u) row_ptr[u] = pos[p];
  if (p == m - 1) row_ptr[n] = pos[m];
  if (flag[p]) col[pos[p]] = (int32_t)(uint32_t)kk;
}

// ------------------------------------------------------ components
// Lock-free union-find: a root is only ever hooked under a smaller root, so
// parent[x] <= x always holds and the final root of a component is its
// minimum vertex.  Finds halve the path: a non-root x is re-pointed to its
// grandparent, an ancestor in the same set.  Hooks only ever replace the
// parent of a root (compare-and-swap against the root itself), and a
// non-root never becomes a root again, so these plain stores cannot undo a
// hook.
__device__ __forceinline__ int uf_find(int* parent, int x) {
  while (true) {
    const int p = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == x) return x;
    const int gp = __hip_atomic_load(&parent[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (gp == p) return p;
    __hip_atomic_store(&parent[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = gp;
  }
}

// The edges are taken in chunks of 64 (one wave, coalesced reads): wave w
// takes chunk (w * stride) mod nchunk, a bijection for a stride coprime to
// nchunk.  Concurrent waves then hook unrelated parts of the graph rather
// than neighbouring vertices whose edges soon share a root (its atomics
// serialise): with many small clouds, and with one cloud whose points are
// grouped by cluster.  The partition does not depend on the order.
#ifndef FAMST_UF_STRIDE
#define FAMST_UF_STRIDE 1009
#endif
__global__ void uf_hook_kernel(const int32_t* __restrict__ nbr, int64_t n, int k, uint64_t stride,
                               int* __restrict__ parent) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nk = n * k, nchunk = (nk + 63) >> 6, w = t >> 6;
  if (w >= nchunk) return;
  const int64_t c = stride == 1 ? w : (int64_t)(((unsigned __int128)w * stride) % (unsigned __int128)nchunk);
  const int64_t e = (c << 6) + (t & 63);
  if (e >= nk) return;
  int a = (int)(e / k), b = nbr[e];
  if (b < 0 || b >= n) return;
  while (true) {
    int ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb) return;
    int hi = max(ra, rb), lo = min(ra, rb);
    if (atomicCAS(&parent[hi], hi, lo) == hi) return;
  }
}

__global__ void uf_roots_kernel(int* __restrict__ parent, int64_t n, int64_t* __restrict__ isroot) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v > n) return;
  if (v == n) {
    isroot[n] = 0;
    return;
  }
  int r = uf_find(parent, (int)v);
  parent[v] = r;
  isroot[v] = (r == v) ? 1 : 0;
}

__global__ void comp_label_kernel(const int* __restrict__ parent, const int64_t* __restrict__ lab,
                                  int64_t n, int32_t* __restrict__ comp, uint32_t* __restrict__ ckey,
                                  int32_t* __restrict__ vidx) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int c = (int)lab[parent[v]];
  comp[v] = c;
  ckey[v] = (uint32_t)c;
  vidx[v] = (int32_t)v;
}

__global__ void comp_ptr_kernel(const uint32_t* __restrict__ skey, int64_t n, int64_t t,
                                int64_t* __restrict__ comp_ptr) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p > n) return;
  if (p == n) {
    comp_ptr[t] = n;
    return;
  }
  if (p == 0 || skey[p] != skey[p - 1]) comp_ptr[skey[p]] = p;
}

__global__ void gather_i64_kernel(const int64_t* __restrict__ src, const int64_t* __restrict__ idx,
                                  int m, int64_t* __restrict__ dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) dst[i] = src[idx[i]];
}

// ------------------------------------------------------ lambda edges
struct CloudPairs {
  int64_t pair_base;   // first pair index of the cloud
  int64_t comp_base;   // first global component id of the cloud
  int64_t t;           // components in the cloud
};

__device__ __forceinline__ int64_t pair_start(int64_t a, int64_t t) {
  return a * t - a * (a + 1) / 2;
}

// One wave per component pair (pairs taken with a stride of the grid):
// lambda^2 samples drawn with Philox, their
// float32 distances, and the lambda smallest by (s, sample).
// CAP >= lambda^2 sample slots in LDS: 64 for lambda <= 8 (small enough for
// many resident waves), 1024 up to lambda = 32.
template <int CAP>
__global__ __launch_bounds__(64) void lambda_edges_kernel(
    const float* __restrict__ X, int d, const CloudPairs* __restrict__ cp, int B, int lam,
    uint32_t key0, uint32_t key1, const int32_t* __restrict__ members,
    const int64_t* __restrict__ comp_ptr, int32_t* __restrict__ eu, int32_t* __restrict__ ev,
    float* __restrict__ ew, int32_t* __restrict__ ea, int32_t* __restrict__ eb, int64_t P) {
  __shared__ SelectSmem<CAP> sm;
  __shared__ int su[CAP], sv[CAP];
  const int t = threadIdx.x, grp = t >> 4, r16 = t & 15;
  for (int64_t p = blockIdx.x; p < P; p += gridDim.x) {
  // cloud of this pair
  int cb = 0;
  {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (cp[mid].pair_base <= p) lo = mid; else hi = mid - 1;
    }
    cb = lo;
  }
  const int64_t tt = cp[cb].t;
  const int64_t pl = p - cp[cb].pair_base;
  int64_t a = 0;
  {
    int64_t lo = 0, hi = tt - 2;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) >> 1;
      if (pair_start(mid, tt) <= pl) lo = mid; else hi = mid - 1;
    }
    a = lo;
  }
  const int64_t b = a + 1 + (pl - pair_start(a, tt));
  const int64_t A = cp[cb].comp_base + a, Bc = cp[cb].comp_base + b;
  const int64_t a0 = comp_ptr[A], b0 = comp_ptr[Bc];
  const uint32_t na = (uint32_t)(comp_ptr[A + 1] - a0), nbb = (uint32_t)(comp_ptr[Bc + 1] - b0);
  const int L = lam * lam;
  for (int q = grp; q < L; q += 4) {
    U4 r = philox4x32_10(U4{(uint32_t)a, (uint32_t)b, (uint32_t)q, (uint32_t)cb}, key0, key1);
    int u = members[a0 + range_map(r.x, na)];
    int v = members[b0 + range_map(r.y, nbb)];
    float s = sq32_group(X + (int64_t)u * d, X + (int64_t)v * d, d, r16);
    if (r16 == 0) {
      sm.s[q] = s;
      sm.id[q] = q;
      su[q] = u;
      sv[q] = v;
    }
  }
  __syncthreads();
  block_select<64, CAP>(sm, L, lam, tau32(d), d, [&](int i, const float** pa, const float** pb) {
    *pa = X + (int64_t)su[i] * d;
    *pb = X + (int64_t)sv[i] * d;
  });
  for (int i = t; i < L; i += 64) {
    int ps = sm.pos[i];
    if (ps >= 0) {
      int64_t o = p * lam + ps;
      eu[o] = su[i];
      ev[o] = sv[i];
      ew[o] = __builtin_sqrtf(sm.s[i]);
      ea[o] = (int32_t)A;
      eb[o] = (int32_t)Bc;
    }
  }
  __syncthreads();   // the next pair reuses the LDS lists
  }
}

}  // namespace famst

using namespace famst;

extern "C" int famst_connect(const float* X, int64_t n, int32_t d, const int64_t* offs_h,
                             int32_t B, const int32_t* nbr, int32_t k, int32_t lambda,
                             uint64_t seed, int64_t* row_ptr, int32_t* col, int64_t* n_col,
                             int32_t* comp, int32_t* members, int64_t* comp_ptr, int32_t* n_comp,
                             int32_t* eu, int32_t* ev, float* ew, int32_t* ea, int32_t* eb,
                             int64_t e_cap, int64_t* n_edges, void* ws, size_t* ws_bytes,
                             void* stream) {
  if (!ws_bytes) return FAMST_EINVAL;
  if (n < 2 || d < 1 || k < 1 || B < 1 || lambda < 1 || lambda > 32) return FAMST_EINVAL;
  if (n >= (int64_t(1) << 31)) return FAMST_EINVAL;
  int64_t one[2] = {0, n};
  const int64_t* offs = offs_h ? offs_h : one;
  if (!offs_h && B != 1) return FAMST_EINVAL;
  if (offs[0] != 0 || offs[B] != n) return FAMST_EINVAL;
  for (int b = 0; b < B; ++b)
    if (offs[b + 1] - offs[b] < 2) return FAMST_EINVAL;
  const int64_t m = 2 * n * (int64_t)k;

  Carve cv(ws);
  uint64_t* keys = cv.take<uint64_t>(m);
  uint64_t* skeys = cv.take<uint64_t>(m);
  int64_t* flag = cv.take<int64_t>(m + 1);
  int64_t* pos = cv.take<int64_t>(m + 1);
  int* parent = cv.take<int>(n);
  int64_t* isroot = cv.take<int64_t>(n + 1);
  int64_t* lab = cv.take<int64_t>(n + 1);
  uint32_t* ckey = cv.take<uint32_t>(n);
  uint32_t* skey = cv.take<uint32_t>(n);
  int32_t* vidx = cv.take<int32_t>(n);
  int64_t* offs_d = cv.take<int64_t>(B + 1);
  int64_t* gath = cv.take<int64_t>(B + 1);
  CloudPairs* cp = cv.take<CloudPairs>(B);
  int* bad = cv.take<int>(1);
  size_t tmpb = sort_keys_u64_bytes(m);
  tmpb = std::max(tmpb, scan_i64_bytes(m + 1));
  tmpb = std::max(tmpb, sort_pairs_u32_i32_bytes(n));
  void* tmp = cv.take<char>(tmpb);
  if (!ws) {
    *ws_bytes = cv.bytes();
    return FAMST_OK;
  }
  if (*ws_bytes < cv.bytes() || (reinterpret_cast<uintptr_t>(ws) & 255)) return FAMST_EWORKSPACE;
  if (!X || !nbr || !row_ptr || !col || !n_col || !comp || !members || !comp_ptr || !n_comp ||
      !n_edges)
    return FAMST_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);

  FAMST_HIP(hipMemcpyAsync(offs_d, offs, sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, s));
  FAMST_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
  // ---- G: sorted, deduplicated symmetric adjacency
  FAMST_TRY(launch("graph_keys", edge_keys_kernel, dim3(cdiv(n * k, 256)), dim3(256), 0, s, nbr, n,
                   k, offs_d, B, keys, bad));
  FAMST_TRY(sort_keys_u64(tmp, tmpb, keys, skeys, m, 32 + bits_for(n), s));
  FAMST_TRY(launch("graph_unique", unique_flags_kernel, dim3(cdiv(m, 256)), dim3(256), 0, s, skeys,
                   m, flag));
  FAMST_HIP(hipMemsetAsync(flag + m, 0, sizeof(int64_t), s));
  FAMST_TRY(exclusive_scan_i64(tmp, tmpb, flag, pos, m + 1, s));
  FAMST_TRY(launch("graph_fill", csr_fill_kernel, dim3(cdiv(m, 256)), dim3(256), 0, s, skeys, flag,
                   pos, m, n, col, row_ptr));
  // ---- components
  FAMST_TRY(iota_i32(parent, n, s));
  // chunk order for the hooks: a stride coprime to the chunk count (checked)
  const uint64_t nchunk = (uint64_t)((n * k + 63) >> 6);
  uint64_t stride = nchunk > 1 ? FAMST_UF_STRIDE : 1;
  if (stride > 1)
    while (std::gcd(stride, nchunk) != 1) ++stride;
  FAMST_TRY(launch("uf_hook", uf_hook_kernel, dim3(cdiv((int64_t)nchunk * 64, 256)), dim3(256), 0, s, nbr, n,
                   k, stride % nchunk, parent));
  FAMST_TRY(launch("uf_roots", uf_roots_kernel, dim3(cdiv(n + 1, 256)), dim3(256), 0, s, parent, n,
                   isroot));
  FAMST_TRY(exclusive_scan_i64(tmp, tmpb, isroot, lab, n + 1, s));
  FAMST_TRY(launch("comp_label", comp_label_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, parent,
                   lab, n, comp, ckey, vidx));
  // per-cloud component counts: lab at the cloud offsets
  FAMST_TRY(launch("gather", gather_i64_kernel, dim3(cdiv(B + 1, 256)), dim3(256), 0, s, lab, offs_d,
                   B + 1, gath));
  std::vector<int64_t> cbase(B + 1);
  int hbad = 0;
  int64_t ncol = 0;
  FAMST_HIP(hipMemcpyAsync(cbase.data(), gath, sizeof(int64_t) * (B + 1), hipMemcpyDeviceToHost, s));
  FAMST_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  FAMST_HIP(hipMemcpyAsync(&ncol, pos + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  // members sorted by (component, vertex): stable sort on the component id
  FAMST_TRY(sort_pairs_u32_i32(tmp, tmpb, ckey, skey, vidx, members, n, bits_for(n + 1), s));
  FAMST_HIP(hipStreamSynchronize(s));
  if (hbad) return FAMST_EINVAL;
  // every cloud holds at least one component and at most its size
  for (int b = 0; b < B; ++b) {
    const int64_t t = cbase[b + 1] - cbase[b];
    if (cbase[b] < 0 || t < 1 || t > offs[b + 1] - offs[b]) return FAMST_EHIP;
  }
  const int64_t T = cbase[B];
  FAMST_TRY(launch("comp_ptr", comp_ptr_kernel, dim3(cdiv(n + 1, 256)), dim3(256), 0, s, skey, n, T,
                   comp_ptr));
  *n_col = ncol;
  std::vector<CloudPairs> hcp(B);
  int64_t P = 0;
  for (int b = 0; b < B; ++b) {
    int64_t t = cbase[b + 1] - cbase[b];
    n_comp[b] = (int32_t)t;
    hcp[b] = CloudPairs{P, cbase[b], t};
    P += t * (t - 1) / 2;
  }
  *n_edges = P * lambda;
  if (!eu) {
    FAMST_HIP(hipStreamSynchronize(s));
    return FAMST_OK;
  }
  if (e_cap < P * lambda || !ev || !ew || !ea || !eb) {
    FAMST_HIP(hipStreamSynchronize(s));
    return e_cap < P * lambda ? FAMST_ECAPACITY : FAMST_EINVAL;
  }
  if (P > 0) {
    FAMST_HIP(hipMemcpyAsync(cp, hcp.data(), sizeof(CloudPairs) * B, hipMemcpyHostToDevice, s));
    auto kern = lambda * lambda <= 64 ? lambda_edges_kernel<64> : lambda_edges_kernel<1024>;
    FAMST_TRY(launch("lambda_edges", kern, dim3(stride_grid(P)), dim3(64), 0, s, X, d, cp, B, lambda,
                     (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), members, comp_ptr, eu, ev,
                     ew, ea, eb, P));
  }
  FAMST_HIP(hipStreamSynchronize(s));
  return FAMST_OK;
}
