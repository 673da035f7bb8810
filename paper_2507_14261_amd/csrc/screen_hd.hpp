// Screening with queries and rows streamed by K-steps (k' = 32, beyond 128 bf16 / 64 fp32 dims).
#pragma once
#include "screen_regs.hpp"

namespace famst {

// ------------------------------------- high-dimensional screening, k' = 32
// For rows longer than the register-resident queries allow (more than 128
// bf16 or 64 float32 dimensions) and for float8: a block of 256 queries (the
// candidate lists in registers as in dist_topk_v2_kernel) against tiles of
// rows.  Queries and rows both stream through LDS in K-steps (KSB bytes) by
// direct global->LDS loads into a ring of stages; each wave accumulates its
// queries x tile rows over all K-steps of a tile, then filters and inserts as
// the pipelined kernel does (same band, same bound of the rejected elements).
// Scan order: tiles tstart, tstart + 1, ... cyclically, where tstart is 0
// for rows in index order and, with a spatial order (perm != null: rows of
// Xq are the points perm[.], grouped by nearest pivot), the tile of the
// block's first query, so that the likely neighbours come first.  In a
// stage, 16-byte chunk c of staged row r sits at slot c ^ swz(r) of the row:
// eight consecutive rows then cover all LDS banks, so the operand reads are
// conflict-free.
// Block shapes (by id): NW waves of 16 QB queries (QBLK = 16 QB NW queries
// per block) against tiles of BN rows, K-steps of KSB bytes in a ring of
// PIPE stages; each wave accumulates QB x BN / 16 fragments (128 VGPRs).
// SC: bytes per tile row beside its staged stretch (the norm, and with
// float8 the row scale).
//   4: float32, 4 waves, 256 x 128, 64-byte steps, three stages, two blocks
//      per CU (four times slower per byte on the matrix cores);
//   8: bf16 and float8, 8 waves, the square 256 x 256 block, 128-byte steps
//      (two bf16 MFMA K-steps or one float8 K-step per barrier), two stages,
//      one block per CU.
template <int SH> struct HdShape;
template <> struct HdShape<4> { static constexpr int NW = 4, QB = 4, BN = 128, PIPE = 3, KSB = 64, SC = 4; };
template <> struct HdShape<8> { static constexpr int NW = 8, QB = 2, BN = 256, PIPE = 2, KSB = 128, SC = 8; };
template <int SH>
constexpr int hd_qblk() { return 16 * HdShape<SH>::QB * HdShape<SH>::NW; }
template <int SH>
constexpr size_t hd_stage_bytes() {
  // query rows, tile rows, the tile's norms (and row scales)
  return (size_t)hd_qblk<SH>() * HdShape<SH>::KSB + (size_t)HdShape<SH>::BN * (HdShape<SH>::KSB + HdShape<SH>::SC);
}
template <int SH>
constexpr size_t hd_lds_bytes() { return (size_t)HdShape<SH>::PIPE * hd_stage_bytes<SH>(); }

template <int PREC, int SH>
__global__ __launch_bounds__(64 * HdShape<SH>::NW, 8 / HdShape<SH>::NW) void dist_topk_hd_kernel(
    const void* __restrict__ Xq_, const float* __restrict__ nq, int RS,
    const BlockDesc* __restrict__ desc, int* __restrict__ cand_j, float* __restrict__ cand_s,
    int kk, const float* __restrict__ qerr, const unsigned* __restrict__ gstat, float arith_c,
    float tau, float* __restrict__ ubound, const float* __restrict__ scl, const int* __restrict__ perm) {
  constexpr int NW = HdShape<SH>::NW, QB = HdShape<SH>::QB, BN = HdShape<SH>::BN, KC = 32, QW = 16 * QB,
                JB = BN / 16, QBLK = hd_qblk<SH>();
  // float8: per-row power-of-two scales applied by the matrix cores (E8M0
  // block scales), so the products come out as a_x a_y codes.codes
  constexpr bool F8 = PREC == FAMST_FP8_E4M3;
  static_assert(!F8 || (HdShape<SH>::KSB == 128 && HdShape<SH>::SC == 8 && BN / 64 < NW),
                "float8: one 128-dim K-step per stage, scales staged by the second half of the waves");
  static_assert(BN / 64 <= NW && (NW & (BN / 64 - 1)) == 0, "norm loads: one wave per 64 tile rows");
  constexpr int HD_PIPE = HdShape<SH>::PIPE, KSB = HdShape<SH>::KSB;
  constexpr int CPR = KSB / 16, KX = KSB / 64;   // 16-byte chunks per staged row; MFMA K-steps per stage
  // chunk c of staged row r sits at slot c ^ swz(r): eight consecutive rows
  // then cover all 32 banks for 64-byte and for 128-byte rows
  auto swz = [](int r) { return CPR == 4 ? ((r >> 1) & 3) : (r & 7); };
  constexpr int NT = 64 * NW;
  constexpr int SQ = QBLK * KSB, SR = BN * KSB, STG = (int)hd_stage_bytes<SH>();
  constexpr int NLQ = QBLK * CPR / NT, NLR = BN * CPR / NT;   // 16-byte query / row chunks per thread
  static_assert(NLQ * NT == QBLK * CPR && NLR * NT == BN * CPR, "whole chunks per thread");
  constexpr int NLD = NLQ + NLR + 1;                  // loads per thread per stage (+ one norm)
  using LS = typename ListRegs<QW>::S;
  using LJ = typename ListRegs<QW>::J;
  const char* Xb = reinterpret_cast<const char*>(Xq_);
  extern __shared__ __attribute__((aligned(16))) char smem[];
  // the first tile's merges: float8 only (its wide band lets most of the
  // first tile's rows pass; in bf16 the extra registers cost more than the
  // merges save), and the four-wave shape has no LDS to spare
  constexpr bool HD_MERGE = SH == 8 && F8;
  __shared__ __attribute__((aligned(16))) float mscratch[HD_MERGE ? NW : 1][INIT_LDS_FLOATS];

  const BlockDesc bd = desc[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, i16 = lane & 15;
  const int wq0 = bd.q0 + wave * QW;
  const int nks = RS / KSB;   // stages per row

  const Band band{arith_c, __uint_as_float(gstat[1]), __uint_as_float(gstat[2]), tau};
  float nql, bcl0, bcl1, U[QB];
  {
    const int q = wq0 + lane;
    const bool ok = lane < QW && q < bd.q1;
    nql = ok ? nq[q] : 0.f;
    band.consts(nql, ok ? qerr[q] : 0.f, bcl0, bcl1);
  }
  int eq[QB];   // E8M0 exponents of the float8 scales of the lane's queries (B operand rows)
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int q = wq0 + qb * 16 + i16;
    U[qb] = q < bd.q1 ? F_INF : -F_INF;
    eq[qb] = (F8 && q < bd.q1) ? (int)((__float_as_uint(scl[q]) >> 23) & 0xFFu) : 127;
  }
  LS ls;
  LJ lj;
#pragma unroll
  for (int L = 0; L < QW / 2; ++L) {
    ls[L] = F_INF;
    lj[L] = 0x7FFFFFFF;
  }

  // this thread's source offsets within the staged query block and row tile
  // (the copy holds PADR >= BN padding rows past its end: no clamps)
  unsigned qoff[NLQ], roff[NLR];
#pragma unroll
  for (int i = 0; i < NLQ; ++i) {
    const int p = tid + NT * i, r = p / CPR;
    qoff[i] = (unsigned)(r * RS + (((p % CPR) ^ swz(r)) << 4));
  }
#pragma unroll
  for (int i = 0; i < NLR; ++i) {
    const int p = tid + NT * i, r = p / CPR;
    roff[i] = (unsigned)(r * RS + (((p % CPR) ^ swz(r)) << 4));
  }
  const int ntile = (bd.c1 - bd.c0 + BN - 1) / BN;
  const char* qbase = Xb + (int64_t)bd.q0 * RS;
  const int tstart = perm ? (bd.q0 - bd.c0) / BN : 0;
  int lt = tstart, lk = 0;   // tile and K-step of the next stage to load
  auto issue = [&](int stg) {
    const int t0 = bd.c0 + lt * BN;
    const int kofs = lk * KSB;
    if (++lk == nks) {
      lk = 0;
      lt = lt + 1 == ntile ? 0 : lt + 1;
    }
    char* stage = smem + stg * STG;
    const char* qb_ = qbase + kofs;
    const char* rb_ = Xb + (int64_t)t0 * RS + kofs;
#pragma unroll
    for (int i = 0; i < NLQ; ++i)
      __builtin_amdgcn_global_load_lds((gptr_t)(qb_ + qoff[i]), (lptr_t)(stage + (NT * i + 64 * wave) * 16),
                                       16, 0, 0);
#pragma unroll
    for (int i = 0; i < NLR; ++i)
      __builtin_amdgcn_global_load_lds((gptr_t)(rb_ + roff[i]),
                                       (lptr_t)(stage + SQ + (NT * i + 64 * wave) * 16), 16, 0, 0);
    // the BN norms: wave w fetches norms 64 (w mod BN/64) .. + 63 (duplicates write equal values);
    // with float8 the second half of the waves fetches the row scales instead
    const int nw = wave & (BN / 64 - 1);
    if (F8 && wave >= BN / 64)
      __builtin_amdgcn_global_load_lds((gptr_t)(scl + t0 + nw * 64 + lane),
                                       (lptr_t)(stage + SQ + SR + BN * 4 + nw * 256), 4, 0, 0);
    else
      __builtin_amdgcn_global_load_lds((gptr_t)(nq + t0 + nw * 64 + lane),
                                       (lptr_t)(stage + SQ + SR + nw * 256), 4, 0, 0);
  };

  // The accumulators of a tile start at -|y|^2 / 2 of their rows, so they
  // end at -s'/2 with s' = |y|^2 - 2 x.y the screened value less |x|^2
  // (scaling by -2 is exact): the filter compares them with -U/2 and needs
  // no arithmetic per element.
  f32x4 acc[QB][JB];

#pragma unroll
  for (int i = 0; i < HD_PIPE - 1; ++i) issue(i);
  const int nst = ntile * nks;
  int cs = 0, ct = tstart, ck = 0;   // stage slot, tile and K-step being computed
  // one stage: its products and, where it completes a tile, the tile's
  // filter and list updates (MERGE: whole-block merges, for the scan's first
  // tile; single insertions otherwise)
  auto stage_step = [&](auto merge) __attribute__((always_inline)) {
    wait_vmcnt<(HD_PIPE - 2) * NLD>();   // this thread's loads of stage st are done
    __builtin_amdgcn_s_barrier();        // ... and every thread's; stage st-1 is consumed
    issue(cs == 0 ? HD_PIPE - 1 : cs - 1);   // into the slot stage st-1 used
    const char* stage = smem + cs * STG;
    if (ck == 0) {
      const float* tn = reinterpret_cast<const float*>(stage + SQ + SR);
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const f32x4 v = *reinterpret_cast<const f32x4*>(tn + jb * 16 + 4 * g);
        const f32x4 h = f32x4{-0.5f * v[0], -0.5f * v[1], -0.5f * v[2], -0.5f * v[3]};
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) acc[qb][jb] = h;
      }
    }
    if constexpr (F8) {
      // one K-step of 128 float8 dimensions: lane (g, i16) holds 32 bytes,
      // chunks 2g and 2g + 1 of its row
      i32x8 bq[QB];
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) {
        const int r = wave * QW + qb * 16 + i16;
        const i32x4 b0 = *reinterpret_cast<const i32x4*>(stage + r * KSB + (((2 * g) ^ swz(r)) << 4));
        const i32x4 b1 = *reinterpret_cast<const i32x4*>(stage + r * KSB + (((2 * g + 1) ^ swz(r)) << 4));
        bq[qb] = i32x8{b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
      }
      const float* tsc = reinterpret_cast<const float*>(stage + SQ + SR + BN * 4);
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const int r = jb * 16 + i16;
        const i32x4 a0 = *reinterpret_cast<const i32x4*>(stage + SQ + r * KSB + (((2 * g) ^ swz(r)) << 4));
        const i32x4 a1 = *reinterpret_cast<const i32x4*>(stage + SQ + r * KSB + (((2 * g + 1) ^ swz(r)) << 4));
        const i32x8 a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
        // lane (g, i16) holds K-block g of row r: the block scale is row r's
        const int ea = (int)((__float_as_uint(tsc[r]) >> 23) & 0xFFu);
#pragma unroll
        for (int qb = 0; qb < QB; ++qb)
          acc[qb][jb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, bq[qb], acc[qb][jb], 0, 0, 0,
                                                                         ea, 0, eq[qb]);
      }
    }
    // query fragments of this wave (B) and row fragments (A), KX K-steps
#pragma unroll
    for (int kx = 0; kx < (F8 ? 0 : KX); ++kx) {
      const int cc = kx * 4 + g;
      i32x4 bq[QB];
#pragma unroll
      for (int qb = 0; qb < QB; ++qb) {
        const int r = wave * QW + qb * 16 + i16;
        bq[qb] = *reinterpret_cast<const i32x4*>(stage + r * KSB + ((cc ^ swz(r)) << 4));
      }
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) {
        const int r = jb * 16 + i16;
        const i32x4 a = *reinterpret_cast<const i32x4*>(stage + SQ + r * KSB + ((cc ^ swz(r)) << 4));
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
          if constexpr (PREC == FAMST_FP32) {
            const f32x4 af = __builtin_bit_cast(f32x4, a);
            const f32x4 bf = __builtin_bit_cast(f32x4, bq[qb]);
            acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0], bf[0], acc[qb][jb], 0, 0, 0);
            acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1], bf[1], acc[qb][jb], 0, 0, 0);
            acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[2], bf[2], acc[qb][jb], 0, 0, 0);
            acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[3], bf[3], acc[qb][jb], 0, 0, 0);
          } else {
            acc[qb][jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, bq[qb]), acc[qb][jb], 0, 0, 0);
          }
        }
      }
    }
    if (++ck == nks) {
      // tile complete: screened value |y|^2 - 2 x.y, filter and insertion in
      // groups of 32 rows (lane holds rows t0h + jj*16 + 4g + r)
      const int t0 = bd.c0 + ct * BN;
#pragma unroll
      for (int h = 0; h < JB / 2; ++h) {
        auto sv = [&](int qb, int e) { return -2.f * acc[qb][2 * h + (e >> 2)][e & 3]; };
        unsigned qbmask = 0;
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
          // sv <= U  <=>  acc >= -U / 2 (exact scaling)
          float m = acc[qb][2 * h][0];
#pragma unroll
          for (int e = 1; e < 8; ++e) m = fmaxf(m, acc[qb][2 * h + (e >> 2)][e & 3]);
          qbmask |= ballot(m >= -0.5f * U[qb]) ? (1u << qb) : 0u;
        }
        if (qbmask) {
          if constexpr (decltype(merge)::value)
            merge_regs<QB, 8, true>(ls, lj, qbmask, U, nql, bcl0, bcl1, band, kk, sv, t0 + 32 * h, bd.c1, wq0,
                                    lane, g, i16, mscratch[wave]);
          else
            insert_regs<QB, 8, true>(ls, lj, qbmask, U, nql, bcl0, bcl1, band, kk, sv, t0 + 32 * h, bd.c1, wq0,
                                     lane, g, i16);
        }
      }
      ck = 0;
      ct = ct + 1 == ntile ? 0 : ct + 1;
    }
    cs = cs + 1 == HD_PIPE ? 0 : cs + 1;
  };
  int st = 0;
  if constexpr (HD_MERGE) {
    const int nfirst = min(nst, nks);   // the stages of the first tile
    for (; st < nfirst; ++st) stage_step(std::true_type{});
  }
  for (; st < nst; ++st) stage_step(std::false_type{});
  wait_vmcnt<0>();   // no load may land in LDS after the block ends

  float nqv[QB];
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
  for (int L = 0; L < QW / 2; ++L) {
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
