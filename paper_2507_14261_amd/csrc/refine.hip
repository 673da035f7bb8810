// Phase 3 of FAMST (Alg. 4): every inter-component edge (u, v) looks at the
// neighbours of u in its own component for a closer endpoint to v, then at
// the neighbours of v for a closer endpoint to the new u.  Rounds repeat
// until no edge changes (Alg. 1).  A round's update of an edge depends only
// on X, the graph, the labels and the edge's own endpoints, so every edge
// runs its rounds on its own, in one launch, until it stops changing; the
// count of edges changed in round r is kept on the device.
#include <vector>

#include "famst_common.hpp"

namespace famst {

// The changed-edge count of round r is spread over REFINE_CSLOTS counters
// (by block index) and summed on the host: one counter per round would
// serialise about a million atomics on one address in the first round of a
// many-component input.
constexpr int REFINE_CSLOTS = 256;

struct Best {
  float s1;   // smallest s
  int id1;    // its id (smallest id among equal s)
  float s2;   // second smallest s (by (s, id))
};

__device__ __forceinline__ void best_push(Best& b, float s, int id) {
  if (key_less(s, id, b.s1, b.id1)) {
    b.s2 = b.s1;
    b.s1 = s;
    b.id1 = id;
  } else if (s < b.s2) {
    b.s2 = s;
  }
}

__device__ __forceinline__ Best best_merge(Best a, Best b) {
  Best r = a;
  if (key_less(b.s1, b.id1, a.s1, a.id1)) {
    r.s1 = b.s1;
    r.id1 = b.id1;
    r.s2 = fminf(a.s1, b.s2);
  } else {
    r.s2 = fminf(a.s2, b.s1);
  }
  return r;
}

// One block of RNT threads per edge: sixteen 16-lane groups measure
// neighbours in parallel; per-wave results meet in LDS.
constexpr int RNT = 256, RNW = RNT / 64;

struct RefineSmem {
  float s1[RNW], s2[RNW];
  int id1[RNW];
  double v64[RNW];
  int i64[RNW];
};

// Smallest (s(x, anchor), x) over neighbours x of `row` in component `c`
// with x != excl; evaluated by the whole block, sixteen 16-lane groups at a
// time.  Near-ties with the runner-up are settled in float64.  Every
// thread of the block returns the same result.
__device__ Best row_argmin(const float* __restrict__ X, int d, const int64_t* __restrict__ row_ptr,
                           const int32_t* __restrict__ col, const int32_t* __restrict__ comp,
                           int row, int c, int excl, int anchor, float tau, bool* used64,
                           double* best64, RefineSmem& sm) {
  const int t = threadIdx.x, grp = t >> 4, r16 = t & 15, lane = t & 63, wave = t >> 6;
  constexpr int NG = RNT / 16;
  const int64_t p0 = row_ptr[row], p1 = row_ptr[row + 1];
  const float* xa = X + (int64_t)anchor * d;
  Best b{F_INF, 0x7FFFFFFF, F_INF};
  for (int64_t p = p0 + grp; p < p1; p += NG) {
    int x = col[p];
    if (comp[x] != c || x == excl) continue;   // uniform within the group
    float s = sq32_group(X + (int64_t)x * d, xa, d, r16);
    best_push(b, s, x);
  }
  // combine the groups: the four of a wave by shuffles, the waves in LDS
#pragma unroll
  for (int o = 16; o <= 32; o <<= 1) {
    Best other;
    other.s1 = __shfl_xor(b.s1, o);
    other.id1 = __shfl_xor(b.id1, o);
    other.s2 = __shfl_xor(b.s2, o);
    b = best_merge(b, other);
  }
  if (lane == 0) {
    sm.s1[wave] = b.s1;
    sm.id1[wave] = b.id1;
    sm.s2[wave] = b.s2;
  }
  __syncthreads();
  b = Best{sm.s1[0], sm.id1[0], sm.s2[0]};
#pragma unroll
  for (int w = 1; w < RNW; ++w) b = best_merge(b, Best{sm.s1[w], sm.id1[w], sm.s2[w]});
  __syncthreads();   // the slots are reused below / by the next call
  *used64 = false;
  const float up = 1.0f + 2.0f * tau, dn = 1.0f - 2.0f * tau;
  if (b.s1 < F_INF && b.s2 * dn <= b.s1 * up) {
    // float32 cannot order the winner against some other candidate
    *used64 = true;
    double m64 = __builtin_inf();
    int mid = 0x7FFFFFFF;
    for (int64_t p = p0 + grp; p < p1; p += NG) {
      int x = col[p];
      if (comp[x] != c || x == excl) continue;
      float s = sq32_group(X + (int64_t)x * d, xa, d, r16);
      if (s * dn <= b.s1 * up) {
        double v = sq64_group(X + (int64_t)x * d, xa, d, r16);
        if (key_less64(v, x, m64, mid)) {
          m64 = v;
          mid = x;
        }
      }
    }
#pragma unroll
    for (int o = 16; o <= 32; o <<= 1) {
      double ov = __shfl_xor(m64, o);
      int oi = __shfl_xor(mid, o);
      if (key_less64(ov, oi, m64, mid)) {
        m64 = ov;
        mid = oi;
      }
    }
    if (lane == 0) {
      sm.v64[wave] = m64;
      sm.i64[wave] = mid;
    }
    __syncthreads();
    m64 = sm.v64[0];
    mid = sm.i64[0];
#pragma unroll
    for (int w = 1; w < RNW; ++w)
      if (key_less64(sm.v64[w], sm.i64[w], m64, mid)) {
        m64 = sm.v64[w];
        mid = sm.i64[w];
      }
    __syncthreads();
    // the winner's float32 value (every group computes it)
    b.id1 = mid;
    b.s1 = sq32_group(X + (int64_t)mid * d, xa, d, r16);
    *best64 = m64;
  }
  return b;
}

// strict "cand < incumbent" with float64 when float32 cannot decide
__device__ bool strictly_less(float sc, float si, const float* ca, const float* cb, const float* ia,
                              const float* ib, int d, float tau, bool have_c64, double c64) {
  const float up = 1.0f + 2.0f * tau, dn = 1.0f - 2.0f * tau;
  if (sc * up < si * dn) return true;
  if (sc * dn > si * up) return false;
  const int r16 = threadIdx.x & 15;
  double vc = have_c64 ? c64 : sq64_group(ca, cb, d, r16);
  double vi = sq64_group(ia, ib, d, r16);
  return vc < vi;
}

__global__ __launch_bounds__(RNT) void refine_kernel(const float* __restrict__ X, int d,
                                                    const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ comp,
                                                    int32_t* __restrict__ eu, int32_t* __restrict__ ev,
                                                    float* __restrict__ ew,
                                                    const int32_t* __restrict__ ea,
                                                    const int32_t* __restrict__ eb, int64_t ne, int max_rounds,
                                                    unsigned long long* __restrict__ cnt) {
  __shared__ RefineSmem sm;
  if ((int64_t)blockIdx.x >= ne) return;
  const int64_t e = blockIdx.x;
  const int r16 = threadIdx.x & 15;
  const float tau = tau32(d);
  const int a = ea[e], b = eb[e];
  int u = eu[e], v = ev[e];
  float wn = 0.f;
  bool any = false;
  for (int r = 0; r < max_rounds; ++r) {   // every thread takes the same path
    const float* xu = X + (int64_t)u * d;
    const float* xv = X + (int64_t)v * d;
    float ds = sq32_group(xu, xv, d, r16);
    int us = u, vs = v;
    // u side: neighbours of u in C_a, measured to v
    bool u64;
    double b64 = 0.0;
    Best bu = row_argmin(X, d, row_ptr, col, comp, u, a, v, v, tau, &u64, &b64, sm);
    if (bu.s1 < F_INF &&
        strictly_less(bu.s1, ds, X + (int64_t)bu.id1 * d, xv, xu, xv, d, tau, u64, b64)) {
      us = bu.id1;
      ds = bu.s1;
    }
    // v side: neighbours of v in C_b (excluding the round's u), measured to u*
    const float* xus = X + (int64_t)us * d;
    Best bv = row_argmin(X, d, row_ptr, col, comp, v, b, u, us, tau, &u64, &b64, sm);
    if (bv.s1 < F_INF &&
        strictly_less(bv.s1, ds, xus, X + (int64_t)bv.id1 * d, xus, X + (int64_t)vs * d, d, tau, u64,
                      b64)) {
      vs = bv.id1;
      ds = bv.s1;
    }
    if (us == u && vs == v) break;
    if (threadIdx.x == 0) atomicAdd(&cnt[r * REFINE_CSLOTS + (blockIdx.x & (REFINE_CSLOTS - 1))], 1ull);
    u = us;
    v = vs;
    wn = __builtin_sqrtf(ds);
    any = true;
  }
  if (any && threadIdx.x == 0) {
    eu[e] = u;
    ev[e] = v;
    ew[e] = wn;
  }
}

// Many edges with short neighbour rows (many components, small k): one
// 16-lane group per edge, sixteen edges per block, each group walking the
// neighbours of u and then of v one at a time.  Same canonical distances,
// (s, id) order and float64 near-tie rule as refine_kernel, so the same
// result; the round's change count takes one atomic per wave.
constexpr int RG_EDGES = RNT / 16;
#ifndef FAMST_REFINE_GROUP_MIN
#define FAMST_REFINE_GROUP_MIN 32768   // edges from which the group-per-edge kernel runs
#endif

__device__ Best row_argmin_group(const float* __restrict__ X, int d, const int64_t* __restrict__ row_ptr,
                                 const int32_t* __restrict__ col, const int32_t* __restrict__ comp,
                                 int row, int c, int excl, int anchor, float tau, bool* used64,
                                 double* best64, int r16) {
  const int64_t p0 = row_ptr[row], p1 = row_ptr[row + 1];
  const float* xa = X + (int64_t)anchor * d;
  Best b{F_INF, 0x7FFFFFFF, F_INF};
  // sixteen neighbours at a time: lane r16 fetches neighbour p0 + r16 and
  // its component, then the group measures the ones that qualify
  const int gsh = threadIdx.x & 48;   // this group's first lane within the wave
  for (int64_t q0 = p0; q0 < p1; q0 += 16) {
    const int64_t p = q0 + r16;
    int x = 0;
    bool ok = false;
    if (p < p1) {
      x = col[p];
      ok = comp[x] == c && x != excl;
    }
    unsigned m = (unsigned)(ballot(ok) >> gsh) & 0xFFFFu;
    while (m) {
      const int j = __builtin_ctz(m);
      m &= m - 1;
      const int xj = __shfl(x, j, 16);
      best_push(b, sq32_group(X + (int64_t)xj * d, xa, d, r16), xj);
    }
  }
  *used64 = false;
  const float up = 1.0f + 2.0f * tau, dn = 1.0f - 2.0f * tau;
  if (b.s1 < F_INF && b.s2 * dn <= b.s1 * up) {
    *used64 = true;
    double m64 = __builtin_inf();
    int mid = 0x7FFFFFFF;
    for (int64_t p = p0; p < p1; ++p) {
      const int x = col[p];
      if (comp[x] != c || x == excl) continue;
      const float s = sq32_group(X + (int64_t)x * d, xa, d, r16);
      if (s * dn <= b.s1 * up) {
        const double v = sq64_group(X + (int64_t)x * d, xa, d, r16);
        if (key_less64(v, x, m64, mid)) {
          m64 = v;
          mid = x;
        }
      }
    }
    b.id1 = mid;
    b.s1 = sq32_group(X + (int64_t)mid * d, xa, d, r16);
    *best64 = m64;
  }
  return b;
}

__global__ __launch_bounds__(RNT) void refine_group_kernel(const float* __restrict__ X, int d,
                                                          const int64_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col,
                                                          const int32_t* __restrict__ comp,
                                                          int32_t* __restrict__ eu, int32_t* __restrict__ ev,
                                                          float* __restrict__ ew,
                                                          const int32_t* __restrict__ ea,
                                                          const int32_t* __restrict__ eb, int64_t ne,
                                                          int max_rounds, unsigned long long* __restrict__ cnt) {
  const int r16 = threadIdx.x & 15, lane = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * RG_EDGES + (threadIdx.x >> 4);
  if (e >= ne) return;   // whole groups
  const float tau = tau32(d);
  const int a = ea[e], b = eb[e];
  int u = eu[e], v = ev[e];
  float wn = 0.f;
  bool any = false;
  // the groups of a wave run their rounds in step: in iteration r every
  // group still running is in its round r, so one atomic per wave counts
  for (int r = 0; r < max_rounds; ++r) {
    const float* xu = X + (int64_t)u * d;
    const float* xv = X + (int64_t)v * d;
    float ds = sq32_group(xu, xv, d, r16);
    int us = u, vs = v;
    bool u64;
    double b64 = 0.0;
    const Best bu = row_argmin_group(X, d, row_ptr, col, comp, u, a, v, v, tau, &u64, &b64, r16);
    if (bu.s1 < F_INF &&
        strictly_less(bu.s1, ds, X + (int64_t)bu.id1 * d, xv, xu, xv, d, tau, u64, b64)) {
      us = bu.id1;
      ds = bu.s1;
    }
    const float* xus = X + (int64_t)us * d;
    const Best bv = row_argmin_group(X, d, row_ptr, col, comp, v, b, u, us, tau, &u64, &b64, r16);
    if (bv.s1 < F_INF &&
        strictly_less(bv.s1, ds, xus, X + (int64_t)bv.id1 * d, xus, X + (int64_t)vs * d, d, tau, u64,
                      b64)) {
      vs = bv.id1;
      ds = bv.s1;
    }
    const bool changed = us != u || vs != v;
    const unsigned long long m = ballot(changed && r16 == 0);
    if (m && lane == __builtin_ctzll(m))
      atomicAdd(&cnt[r * REFINE_CSLOTS + (blockIdx.x & (REFINE_CSLOTS - 1))],
                (unsigned long long)__builtin_popcountll(m));
    if (!changed) break;
    u = us;
    v = vs;
    wn = __builtin_sqrtf(ds);
    any = true;
  }
  if (any && r16 == 0) {
    eu[e] = u;
    ev[e] = v;
    ew[e] = wn;
  }
}

__global__ void zero_u64_kernel(unsigned long long* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace famst

using namespace famst;

extern "C" int famst_refine(const float* X, int64_t n, int32_t d, const int64_t* row_ptr,
                            const int32_t* col, const int32_t* comp, int32_t* eu, int32_t* ev,
                            float* ew, const int32_t* ea, const int32_t* eb, int64_t n_edges,
                            int32_t max_rounds, int32_t* rounds_run, int64_t* deltas, void* ws,
                            size_t* ws_bytes, void* stream) {
  if (!ws_bytes) return FAMST_EINVAL;
  if (n < 2 || d < 1 || n_edges < 0 || max_rounds < 1 || max_rounds > FAMST_REFINE_MAX_ROUNDS) return FAMST_EINVAL;
  if (n_edges >= (int64_t(1) << 31)) return FAMST_ENOTIMPL;
  Carve cv(ws);
  // changed-edge counts of every round (REFINE_CSLOTS per round)
  const int ncnt = max_rounds * REFINE_CSLOTS;
  unsigned long long* cnt = cv.take<unsigned long long>(ncnt);
  if (!ws) {
    *ws_bytes = cv.bytes();
    return FAMST_OK;
  }
  if (*ws_bytes < cv.bytes() || (reinterpret_cast<uintptr_t>(ws) & 255)) return FAMST_EWORKSPACE;
  if (!rounds_run || (n_edges > 0 && (!X || !row_ptr || !col || !comp || !eu || !ev || !ew || !ea || !eb)))
    return FAMST_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  FAMST_TRY(launch("refine_zero", zero_u64_kernel, dim3(cdiv(ncnt, 256)), dim3(256), 0, s, cnt, ncnt));
  if (n_edges >= FAMST_REFINE_GROUP_MIN)
    FAMST_TRY(launch("refine", refine_group_kernel, dim3(cdiv(n_edges, RG_EDGES)), dim3(RNT), 0, s, X, d, row_ptr,
                     col, comp, eu, ev, ew, ea, eb, n_edges, (int)max_rounds, cnt));
  else if (n_edges > 0)
    FAMST_TRY(launch("refine", refine_kernel, dim3((unsigned)n_edges), dim3(RNT), 0, s, X, d, row_ptr, col, comp,
                     eu, ev, ew, ea, eb, n_edges, (int)max_rounds, cnt));
  std::vector<unsigned long long> hs(ncnt), hc(max_rounds, 0);
  FAMST_HIP(hipMemcpyAsync(hs.data(), cnt, sizeof(unsigned long long) * ncnt, hipMemcpyDeviceToHost, s));
  FAMST_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < max_rounds; ++r)
    for (int i = 0; i < REFINE_CSLOTS; ++i) hc[r] += hs[(size_t)r * REFINE_CSLOTS + i];
  // rounds until one changes nothing (a round after an empty one would be empty too)
  int r = 0;
  int64_t last = 0;
  while (r < max_rounds) {
    last = (int64_t)hc[r];
    if (deltas) deltas[r] = last;
    ++r;
    if (last == 0) break;
  }
  *rounds_run = r;
  return last == 0 ? FAMST_OK : FAMST_WNOTCONVERGED;
}
