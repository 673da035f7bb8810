// Screening work units, candidate records and the register-list machinery shared by the pipelined screening kernels.
#pragma once
#include "famst_common.hpp"

namespace famst {

// ------------------------------------------------------ distance + top-k'
// Work unit of one block: queries [q0, q1) of one cloud against the
// cloud's rows [c0, c1).
struct BlockDesc {
  int q0, q1, c0, c1;
};

struct __attribute__((aligned(8))) Cand {
  float s;
  int j;
};

template <int PREC>
struct Scr;
template <>
struct Scr<FAMST_FP32> {
  using T = float;
  static constexpr int KBW = 16;  // k covered by one 16-byte fragment per lane x 4 lane groups
  static constexpr int ESZ = 4;
};
template <>
struct Scr<FAMST_BF16> {
  using T = uint16_t;
  static constexpr int KBW = 32;
  static constexpr int ESZ = 2;
};

// ------------------------------------------- pipelined screening, k' = 32
// The products, filter and insertion rule of dist_topk_kernel, organised
// for memory-level parallelism: the per-query lists live in registers,
// which frees LDS for a ring of PIPE tile stages filled by direct
// global->LDS loads, so PIPE-1 tiles are in flight while one is consumed and
// a single barrier per tile suffices.
//
// Register lists: query qi (0..63) of a wave owns register pair qi/2 of
// (ls, lj), lanes 32 (qi & 1) .. 32 (qi & 1) + 31, ascending by (s, j).
typedef float f32x32 __attribute__((ext_vector_type(32)));
typedef int i32x32 __attribute__((ext_vector_type(32)));
typedef float f32x16v __attribute__((ext_vector_type(16)));
typedef int i32x16v __attribute__((ext_vector_type(16)));
// register lists of a wave with QW queries: QW / 2 register pairs
template <int QW> struct ListRegs;
template <> struct ListRegs<64> { using S = f32x32; using J = i32x32; };
template <> struct ListRegs<32> { using S = f32x16v; using J = i32x16v; };
typedef __attribute__((address_space(1))) const void* gptr_t;
typedef __attribute__((address_space(3))) void* lptr_t;
constexpr int PIPE = 4;
static_assert((PIPE & (PIPE - 1)) == 0, "stage index by mask");

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  // gfx9 s_waitcnt: vmcnt in bits [3:0] and [15:14]; expcnt and lgkmcnt at
  // their maxima (not waited for)
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Screening band above the k-th screened value T of a query: wide enough
// that the re-rank certificate (screening arithmetic error eps, input
// rounding e = e_q + e_max, float32 near-tie factor tau) holds for every
// element the filter rejects:
//   band(T) = (2 eps + 4 e^2) + 4 e sqrt(T) + (8 tau + 1e-5) |T|,
// +inf while fewer than k entries exist.  Only the chance of certifying
// depends on it: the certificate itself uses the final threshold, which
// bounds every rejected element whatever the band was.
struct Band {
  float arith_c, nmax, emax, tau;
  // per-query constants: c0 = 2 eps + 4 e^2, c1 = 4 e
  __device__ __forceinline__ void consts(float nqv, float eqv, float& c0, float& c1) const {
    const float e = eqv + emax;
    c0 = 2.f * arith_c * (nqv + nmax) + 4.f * e * e;
    c1 = 4.f * e;
  }
  __device__ __forceinline__ float operator()(float Tk, float c0, float c1) const {
    if (!(Tk < F_INF)) return F_INF;
    // hardware square root, rounded up by a few ulps
    const float r = c1 > 0.f ? __builtin_amdgcn_sqrtf(fmaxf(Tk, 0.f)) * 1.000001f : 0.f;
    return c0 + c1 * r + (8.f * tau + 1e-5f) * fabsf(Tk);
  }
};

// ------------------------------------------- lists from the first rows
// Per-wave LDS scratch of init_lists and merge_block: a 16 x 32 matrix
// (query of a block, row of the 32-row group), the 16 queries' k-th entries
// and their last entries.
constexpr int INIT_LDS_FLOATS = 16 * 32 + 32;

// The value of lane (lane xor M) of the same half-wave, without the LDS
// crossbar where the VALU can do it: DPP quad permutations for M = 1, 2;
// for M = 4, 8 the row shifts by M in both directions (row_shl:M gives lane
// i the value of lane i + M, row_shr:M that of lane i - M, both inside the
// lane's row of 16), the lane's bit M choosing; ds_swizzle in bit-mask mode
// (xor 16 within 32 lanes) for M = 16.
template <int M>
__device__ __forceinline__ int xor_lane32(int v, int rel) {
  static_assert(M == 1 || M == 2 || M == 4 || M == 8 || M == 16, "a lane distance inside 32 lanes");
  if constexpr (M == 1) {
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1, 0, 3, 2]
  } else if constexpr (M == 2) {
    return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2, 3, 0, 1]
  } else if constexpr (M == 16) {
    return __builtin_amdgcn_ds_swizzle(v, 0x401F);   // and 0x1F, or 0, xor 0x10
  } else {
    const int up = __builtin_amdgcn_update_dpp(0, v, 0x100 + M, 0xF, 0xF, false);   // row_shl:M
    const int dn = __builtin_amdgcn_update_dpp(0, v, 0x110 + M, 0xF, 0xF, false);   // row_shr:M
    return (rel & M) ? dn : up;
  }
}

// Compare-exchange of (s, j) with the lane at distance M of the same
// half-wave: where `asc`, the lower lane of the pair keeps the smaller key.
template <int M>
__device__ __forceinline__ void cex32(float& s, int& j, bool asc, int rel) {
  const float ps = __int_as_float(xor_lane32<M>(__float_as_int(s), rel));
  const int pj = xor_lane32<M>(j, rel);
  const bool lower = (rel & M) == 0;
  const bool pless = (ps < s) | ((ps == s) & (pj < j));
  const bool sless = (s < ps) | ((s == ps) & (j < pj));
  const bool take = (lower == asc) ? pless : sless;
  s = take ? ps : s;
  j = take ? pj : j;
}

// Bitonic sort of the 32 (s, j) of each half-wave into ascending (DESC:
// descending) order.
template <bool DESC = false>
__device__ __forceinline__ void sort32(float& s, int& j, int rel) {
#pragma unroll
  for (int k = 2; k <= 32; k <<= 1) {
    const bool asc = ((rel & k) == 0) != DESC;
    if (k >= 32) cex32<16>(s, j, asc, rel);
    if (k >= 16) cex32<8>(s, j, asc, rel);
    if (k >= 8) cex32<4>(s, j, asc, rel);
    if (k >= 4) cex32<2>(s, j, asc, rel);
    cex32<1>(s, j, asc, rel);
  }
}
__device__ __forceinline__ void sort32_asc(float& s, int& j, int rel) { sort32<false>(s, j, rel); }

// The lists of a wave's queries built from the first 32 rows of the scan at
// once: the first rows of a query all pass an empty list's filter, so
// instead of 32 single insertions per query, each lane writes its 8 values
// of query block qb (+inf where j is the query itself or past the cloud)
// into a 16 x 32 (query, row) matrix, register pair L = 8 qb + c reads the
// rows of its two queries (2c + half) and sorts them by (s, j), and the
// thresholds follow from the new k-th entries.  The lists are then the 32
// smallest (s, j) of those rows, as the single insertions would leave them.
template <int QB, class LS, class LJ, class SpFn>
__device__ __forceinline__ void init_lists(LS& ls, LJ& lj, float (&U)[QB], float nql, float bcl0, float bcl1,
                                           const Band& band, int kk, SpFn spf, int t0, int c1, int wq0, int lane,
                                           int g, int i16, float* mlds) {
  const int half = lane >> 5, rel = lane & 31;
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int q = wq0 + qb * 16 + i16;
    const float nqq = __shfl(nql, qb * 16 + i16);   // |x_q|^2 of the lane's query
    const bool live = U[qb] != -F_INF;                // queries past the block stay empty
    f32x4 w[2];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int j = t0 + (e >> 2) * 16 + 4 * g + (e & 3);
      w[e >> 2][e & 3] = (live & (j < c1) & (j != q)) ? spf(qb, e) + nqq : F_INF;
    }
    *reinterpret_cast<f32x4*>(mlds + i16 * 32 + 4 * g) = w[0];
    *reinterpret_cast<f32x4*>(mlds + i16 * 32 + 16 + 4 * g) = w[1];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      float cs = mlds[(2 * c + half) * 32 + rel];
      int cj = cs < F_INF ? t0 + rel : 0x7FFFFFFF;
      sort32_asc(cs, cj, rel);
      ls[qb * 8 + c] = cs;
      lj[qb * 8 + c] = cj;
      if (rel == kk - 1) mlds[512 + 2 * c + half] = cs;
    }
    __builtin_amdgcn_wave_barrier();
    const float Tk = mlds[512 + i16];
    const float Un = (Tk - nqq) + band(Tk, __shfl(bcl0, qb * 16 + i16), __shfl(bcl1, qb * 16 + i16));
    U[qb] = live ? Un : U[qb];
    __builtin_amdgcn_wave_barrier();   // the scratch is rewritten for the next block
  }
}

// A whole 32-row group merged into the lists of one query block at once:
// where many elements of the block pass the filter (early in the scan, when
// the lists are still far from final), one sort and one merge per register
// pair replace the one-at-a-time insertions.  Each lane writes its passing
// values (+inf elsewhere) into the per-wave 16 x 32 (query, row) matrix;
// register pair L = 8 qb + c reads the rows of its two queries, sorts them
// descending, and keeps the 32 smallest of them and its list (the pairwise
// minimum of an ascending and a descending sequence is bitonic: five more
// compare-exchange steps sort it).  The lists then hold the 32 smallest
// (s, j) of their old entries and the passing elements; the thresholds
// follow from the new k-th entries and never increase.  Elements the
// one-at-a-time rule would have skipped once its threshold tightened can
// stay in the list's tail; they only widen what the re-rank sees.
template <bool CAPK, int NE, class LS, class LJ>
__device__ __forceinline__ void merge_block(LS& ls, LJ& lj, float& Uq, int qb, const float (&sp)[NE],
                                            const bool (&ok)[NE], float nql, float bcl0, float bcl1,
                                            const Band& band, int kk, int t0, int lane, int g, int i16,
                                            float* mlds) {
  static_assert(NE == 8, "a 32-row group: eight elements per lane");
  const int half = lane >> 5, rel = lane & 31;
  const float nqq = __shfl(nql, qb * 16 + i16);   // |x_q|^2 of the lane's query
  f32x4 w[2];
#pragma unroll
  for (int e = 0; e < NE; ++e) w[e >> 2][e & 3] = ok[e] ? sp[e] + nqq : F_INF;
  *reinterpret_cast<f32x4*>(mlds + i16 * 32 + 4 * g) = w[0];
  *reinterpret_cast<f32x4*>(mlds + i16 * 32 + 16 + 4 * g) = w[1];
  __builtin_amdgcn_wave_barrier();
#pragma unroll 1   // one register pair at a time: the merge runs beside the next group's products
  for (int c = 0; c < 8; ++c) {
    float cs = mlds[(2 * c + half) * 32 + rel];
    int cj = cs < F_INF ? t0 + rel : 0x7FFFFFFF;
    sort32<true>(cs, cj, rel);
    const int L = qb * 8 + c;
    const float os = ls[L];
    const int oj = lj[L];
    const bool cl = (cs < os) | ((cs == os) & (cj < oj));
    float ms = cl ? cs : os;
    int mj = cl ? cj : oj;
    cex32<16>(ms, mj, true, rel);
    cex32<8>(ms, mj, true, rel);
    cex32<4>(ms, mj, true, rel);
    cex32<2>(ms, mj, true, rel);
    cex32<1>(ms, mj, true, rel);
    ls[L] = ms;
    lj[L] = mj;
    if (rel == kk - 1) mlds[512 + 2 * c + half] = ms;
    if (CAPK && rel == 31) mlds[528 + 2 * c + half] = ms;
  }
  __builtin_amdgcn_wave_barrier();
  const float Tk = mlds[512 + i16];
  float Un = (Tk - nqq) + band(Tk, __shfl(bcl0, qb * 16 + i16), __shfl(bcl1, qb * 16 + i16));
  if constexpr (CAPK) Un = fminf(Un, mlds[528 + i16] - nqq);
  Uq = Uq != -F_INF ? Un : Uq;   // queries past the block stay empty
  __builtin_amdgcn_wave_barrier();   // the scratch is rewritten for the next block
}

// The filter threshold of a query is U = T_k - |x_q|^2 + band(T_k) with T_k
// the k-th entry of its list (not the last): an element screened above it
// cannot be among the k nearest, and U + |x_q|^2 at the end bounds every
// rejected element for the certificate.  With CAPK, U is also capped at the
// list's last entry minus |x_q|^2 (an element above it cannot enter the
// list): where the band is wide (float8) this keeps most of the filter's
// passes from reaching the insertion only to be dropped there; the bound
// stays valid, as U still never increases.
//
// Elements are taken element-major: for each of the NE elements a lane
// holds (a static register), a ballot gives the lanes whose element passed,
// and each is inserted in turn into its query's list (a ballot gives the
// position, DPP wave_shr:1 shifts the tail, the query's threshold follows
// the new k-th entry).
template <int QB, int NE, bool CAPK = false, class LS, class LJ, class SpFn>
__device__ __forceinline__ void insert_regs(LS& ls, LJ& lj, unsigned qbmask, float (&U)[QB],
                                            float nql, float bcl0, float bcl1,
                                            const Band& band, int kk,
                                            SpFn spf, int t0, int c1, int wq0, int lane, int g,
                                            int i16) {
  const int half = lane >> 5, rel = lane & 31;
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    if (!(qbmask & (1u << qb))) continue;
    const int q = wq0 + qb * 16 + i16;
    float sp[NE];
    bool ok[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      sp[e] = spf(qb, e);
      const int j = t0 + (e >> 2) * 16 + 4 * g + (e & 3);
      ok[e] = (sp[e] <= U[qb]) & (j < c1) & (j != q);
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      unsigned long long lanes = ballot(ok[e]);
      while (lanes) {
        const int src = __builtin_ctzll(lanes);
        lanes &= lanes - 1;
        const float spv = readlane_f(sp[e], src);
        if (!(spv <= readlane_f(U[qb], src))) continue;   // list tightened meanwhile
        const int qi = qb * 16 + (src & 15);
        const int L = qi >> 1, h = qi & 1;
        const int j = t0 + (e >> 2) * 16 + 4 * (src >> 4) + (e & 3);
        const int qw = qb * 16 + (src & 15);   // query within the wave
        const float nqv = readlane_f(nql, qw);
        const float s = spv + nqv;
        const float cs = ls[L];
        const int cjv = lj[L];
        const bool mine = half == h;
        const bool lt = mine & ((cs < s) | ((cs == s) & (cjv < j)));
        const int pos = __builtin_popcountll(ballot(lt));
        if (pos >= 32) continue;
        // shift the tail of the half up by one (DPP wave_shr:1); the first
        // lane of a half never takes the shifted value
        const float ups = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(cs), 0x138, 0xF, 0xF, false));
        const int upj = __builtin_amdgcn_update_dpp(0, cjv, 0x138, 0xF, 0xF, false);
        const bool keep = !mine | (rel < pos);
        const float ns = keep ? cs : (rel == pos ? s : ups);
        const int nj = keep ? cjv : (rel == pos ? j : upj);
        ls[L] = ns;
        lj[L] = nj;
        const float Tk = readlane_f(ns, 32 * h + kk - 1);
        float Un = (Tk - nqv) + band(Tk, readlane_f(bcl0, qw), readlane_f(bcl1, qw));
        if constexpr (CAPK) Un = fminf(Un, readlane_f(ns, 32 * h + 31) - nqv);
        U[qb] = (i16 == (src & 15)) ? Un : U[qb];
      }
    }
  }
}

// The update of merge_block for every query block with a passing element:
// the form for the first groups of a scan, where most rows still pass.
template <int QB, int NE, bool CAPK = false, class LS, class LJ, class SpFn>
__device__ __forceinline__ void merge_regs(LS& ls, LJ& lj, unsigned qbmask, float (&U)[QB], float nql,
                                           float bcl0, float bcl1, const Band& band, int kk, SpFn spf, int t0,
                                           int c1, int wq0, int lane, int g, int i16, float* mlds) {
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    if (!(qbmask & (1u << qb))) continue;
    const int q = wq0 + qb * 16 + i16;
    float sp[NE];
    bool ok[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      sp[e] = spf(qb, e);
      const int j = t0 + (e >> 2) * 16 + 4 * g + (e & 3);
      ok[e] = (sp[e] <= U[qb]) & (j < c1) & (j != q);
    }
    merge_block<CAPK>(ls, lj, U[qb], qb, sp, ok, nql, bcl0, bcl1, band, kk, t0, lane, g, i16, mlds);
  }
}

// ------------------------------------------------ buffered list updates
// Past the merged first tiles most groups pass a few elements per query
// block.  Instead of one insertion pass each, they are appended to a
// per-query LDS buffer of BUF_SLOTS (s, j) slots (bs, bj: query qi of the
// wave owns slots BUF_SLOTS qi ..; empty slots hold +inf) under the
// threshold of the block's last merge, and a block's buffers are merged
// into its lists (flush_block) when one of them would overflow, and at the
// end of the scan.  The threshold only tightens at merges, so more elements
// are appended than the one-at-a-time rule would insert; every element the
// filter rejects is still above the threshold in force, which never
// increases, and every element a merge drops is at or above the list
// maximum of that moment, so the certificate's bounds hold as before.
constexpr int BUF_SLOTS = 16;

template <class LS, class LJ>
__device__ __forceinline__ void flush_block(LS& ls, LJ& lj, float& Uq, int qb, float* bs, int* bj, float nql,
                                            float bcl0, float bcl1, const Band& band, int kk, int lane, int i16,
                                            float* mlds) {
  const int half = lane >> 5, rel = lane & 31;
  const float nqq = __shfl(nql, qb * 16 + i16);
#pragma unroll 1
  for (int c = 0; c < 8; ++c) {
    const int qi = qb * 16 + 2 * c + half;
    float cs = rel < BUF_SLOTS ? bs[qi * BUF_SLOTS + rel] : F_INF;
    int cj = rel < BUF_SLOTS ? bj[qi * BUF_SLOTS + rel] : 0x7FFFFFFF;
    if (!(cs < F_INF)) cj = 0x7FFFFFFF;   // an empty slot
    sort32<true>(cs, cj, rel);
    const int L = qb * 8 + c;
    const float os = ls[L];
    const int oj = lj[L];
    const bool cl = (cs < os) | ((cs == os) & (cj < oj));
    float ms = cl ? cs : os;
    int mj = cl ? cj : oj;
    cex32<16>(ms, mj, true, rel);
    cex32<8>(ms, mj, true, rel);
    cex32<4>(ms, mj, true, rel);
    cex32<2>(ms, mj, true, rel);
    cex32<1>(ms, mj, true, rel);
    ls[L] = ms;
    lj[L] = mj;
    if (rel == kk - 1) mlds[512 + 2 * c + half] = ms;
  }
  __builtin_amdgcn_wave_barrier();
  // empty the block's 16 x BUF_SLOTS slots: four per lane
  static_assert(16 * BUF_SLOTS == 4 * 64, "four slots per lane");
  *reinterpret_cast<f32x4*>(bs + qb * 16 * BUF_SLOTS + 4 * lane) = f32x4{F_INF, F_INF, F_INF, F_INF};
  const float Tk = mlds[512 + i16];
  const float Un = (Tk - nqq) + band(Tk, __shfl(bcl0, qb * 16 + i16), __shfl(bcl1, qb * 16 + i16));
  Uq = Uq != -F_INF ? Un : Uq;
  __builtin_amdgcn_wave_barrier();
}

// Appends of one 32-row group, in two halves of 16 rows (at most 16 passing
// elements per query each, so a half always fits an emptied buffer).  A
// lane's slot: its query's count, plus the passing elements of the same
// query at lower elements of the half, plus those of lower lanes at its own
// element (lanes i16, i16 + 16, i16 + 32, i16 + 48 hold one query).
template <int QB, class LS, class LJ, class SpFn>
__device__ __forceinline__ void buffer_regs(LS& ls, LJ& lj, unsigned qbmask, float (&U)[QB], int (&bc)[QB],
                                            float* bs, int* bj, float nql, float bcl0, float bcl1,
                                            const Band& band, int kk, SpFn spf, int t0, int c1, int wq0,
                                            int lane, int g, int i16, float* mlds) {
  const unsigned long long qm = 0x0001000100010001ull << i16;
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    if (!(qbmask & (1u << qb))) continue;
    const int q = wq0 + qb * 16 + i16;
    const float nqq = __shfl(nql, qb * 16 + i16);
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      float sp[4];
      bool ok[4];
      unsigned long long bl[4];
      int n = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sp[r] = spf(qb, 4 * hh + r);
        const int j = t0 + 16 * hh + 4 * g + r;
        ok[r] = (sp[r] <= U[qb]) & (j < c1) & (j != q);
        bl[r] = ballot(ok[r]);
        n += __builtin_popcountll(bl[r] & qm);
      }
      if ((bl[0] | bl[1] | bl[2] | bl[3]) == 0) continue;
      if (ballot(bc[qb] + n > BUF_SLOTS)) {
        flush_block(ls, lj, U[qb], qb, bs, bj, nql, bcl0, bcl1, band, kk, lane, i16, mlds);
        bc[qb] = 0;
      }
      int base = bc[qb];
      float* rs = bs + (qb * 16 + i16) * BUF_SLOTS;
      int* rj = bj + (qb * 16 + i16) * BUF_SLOTS;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (ok[r]) {
          const int slot = base + __builtin_popcountll(bl[r] & qm & below);
          rs[slot] = sp[r] + nqq;
          rj[slot] = t0 + 16 * hh + 4 * g + r;
        }
        base += __builtin_popcountll(bl[r] & qm);
      }
      bc[qb] = base;
    }
  }
}

// A query fragment (8 bf16 or 4 float32 values) times -2; exact for every
// finite input (a power-of-two scaling, far from overflow for rows that
// passed the norm check).
template <int PREC>
__device__ __forceinline__ i32x4 neg2_fragment(i32x4 v) {
  if constexpr (PREC == FAMST_FP32) {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = __float_as_int(-2.f * __int_as_float(v[i]));
    return v;
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const unsigned u = (unsigned)v[i];
      const unsigned lo = f32_to_bf16_rne(-2.f * bf16_to_f32((uint16_t)(u & 0xFFFFu)));
      const unsigned hi = f32_to_bf16_rne(-2.f * bf16_to_f32((uint16_t)(u >> 16)));
      v[i] = (int)(lo | (hi << 16));
    }
    return v;
  }
}

}  // namespace famst
