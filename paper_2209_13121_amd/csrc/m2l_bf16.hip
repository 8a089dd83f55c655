// m2l_bf16.hip -- multipole-to-local translation on the BF16 matrix cores
// with split operands (mixed precision).
//
// Same operation and work decomposition as m2l.hip (m2l_common.h): per
// parity class and offset d a dense product L~[:, targets] += T_d M~[:, targets - d].
// Every operand x is carried as np BF16 pieces, x = x0 + x1 (+ x2):
// x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1), each rounded to
// nearest even.  For an FP32 value three pieces are exact (8 + 8 + 8
// significant bits).  A product a b is taken as the sum of the piece products
// a_i b_j with i + j < np (6 of 9 for np = 3: the dropped ones are below
// 2^-24 relative; 3 of 4 for np = 2: about 2^-16).  Each piece product of a
// 16 x 32 operator block and a 32 x 16 source block is one
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation; the matrix cores run BF16
// at 16 times the FP32 rate, so np = 3 needs 6 / 16 of the FP32 issue time.
//
//  * Operand layout (16-byte quads of 8 BF16): a row of an operator or a
//    source box holds quad (ks * np + piece) * 4 + g = k values 32 ks + 8 g ..
//    + 7 of that piece, zero past ncoef; lane (col, g) of the MFMA reads
//    exactly one quad per (k step, piece) for A and for B.
//  * Operators: [op][row (16-row blocks)][quads + 1] (the extra zero quad
//    makes the stride odd), generated once per plan from FP64 entries and
//    staged in LDS per offset in k-step chunks, double-buffered.
//  * Sources: the FP32 multipoles of every level, split once per evaluation
//    into BF16 pieces (k_split_mult) so the M2L loop only loads quads.
//  * Accumulation: FP32 chains over kFlush consecutive offsets (smallest
//    piece products first), summed with Kahan compensation.
//  * FP16 form (FMM_M2L_F16X2): operators scaled per row and column, source
//    multipoles per level, by powers of two into the FP16 range, split into 2
//    FP16 pieces (h + l); blocks of low degree take h h + h l + l h, blocks of
//    high degree h h alone (f16_cross); FP32 chains of kGroupF16 offsets
//    summed into the total, unscaled once at the end.
#include <algorithm>

#include "bf16_split.h"
#include "m2l_common.h"

namespace fmm {
namespace {

using m2l::kThreads;

// Tuning (measured at p = 8 on MI355X): row blocks per group of A loads,
// and offsets per FP32 chain -- the chain is added to the compensated sum
// after every kFlush offsets and after the last (chains of 4 offsets are 72
// piece products long; the Kahan update is then a quarter of its per-offset
// cost and the result as accurate).
#ifndef M2LB_RG
#define M2LB_RG 2
#endif
#ifndef M2LB_FLUSH
#define M2LB_FLUSH 4
#endif
#ifndef M2LB_RG_F16
#define M2LB_RG_F16 6
#endif
#ifndef M2LB_PB_KST
#define M2LB_PB_KST 3
#endif
#ifndef M2LB_PB2_KST
#define M2LB_PB2_KST 0
#endif
#ifndef M2LB_OP2
#define M2LB_OP2 1
#endif
constexpr int kFlush = M2LB_FLUSH;
// s_waitcnt operand: vmcnt(n) (n < 64), expcnt and lgkmcnt not waited for
constexpr int vmcnt_op(int n) { return 0x0F70 | (n & 15) | ((n >> 4) << 14); }
constexpr int kVmcntZero = vmcnt_op(0);
// FP16 form: offsets per FP32 partial sum.
constexpr int kGroupF16 = 8;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Piece products (a piece, b piece) with i + j < NP, smallest first.
template <int NP>
struct Prod;
template <>
struct Prod<3> {
  static constexpr int N = 6;
  static constexpr int a[6] = {1, 0, 2, 0, 1, 0};
  static constexpr int b[6] = {1, 2, 0, 1, 0, 0};
};
template <>
struct Prod<2> {
  static constexpr int N = 3;
  static constexpr int a[3] = {0, 1, 0};
  static constexpr int b[3] = {1, 0, 0};
};

// Split every box's FP32 multipole row (stride ms) of levels 2..L into pieces:
// one thread per (box, k step, lane group g) writes the NP quads of its 8 k values.
template <int NP>
__global__ void k_split_mult(const float* __restrict__ m32, int ms, int nc, int kst, int64_t nbox,
                             u32x4* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbox * kst * 4) return;
  const int64_t box = t / (kst * 4);
  const int ks = (int)(t / 4 % kst), g = (int)(t % 4);
  const float* row = m32 + box * ms;
  uint32_t pc[8][NP];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 32 * ks + 8 * g + j;
    split_f32<NP>(k < nc ? row[k] : 0.0f, pc[j]);
  }
  u32x4 q[NP];
  pack_quads<NP>(pc, q);
  u32x4* o = out + box * (kst * NP * 4);
#pragma unroll
  for (int i = 0; i < NP; ++i) o[(ks * NP + i) * 4 + g] = q[i];
}

// FP16 form: boxes of levels 2..L in level order; the work-groups of the
// level-max pass, per level.
struct LevelBlocks {
  int64_t box_off[FMM_DEPTH_MAX + 2];  // first box (row of the expansion arrays) of level l
  int64_t blk_off[FMM_DEPTH_MAX + 2];  // first work-group of level l
  int l0, l1;                          // levels l0..l1
};

__device__ __forceinline__ int level_of_block(const LevelBlocks& lb, int64_t b) {
  int l = lb.l0;
  while (l < lb.l1 && b >= lb.blk_off[l + 1]) ++l;
  return l;
}

// FP16 form, pass 1: per level, the largest |M_k colf_k| over its boxes (the
// FP32 multipoles times the column factors), into lmax[l] as float bits.  The
// work-groups of a level stride over its rows as one flat array of float4
// (ms is a multiple of 4; k >= nc is skipped); each group's maximum joins
// lmax[l] by one atomicMax on the bits (non-negative floats order as their
// bits; a maximum is exact in any order).
constexpr int64_t kLevelMaxGroups = 1024;
constexpr int kMaxColf = 192;  // >= 32 k steps of 32 at the largest p (12), >= its mstride
static_assert(kMaxColf >= 32 * m2lb_ksteps(13 * 13) && kMaxColf >= mstride_of(13 * 13), "column factors fit");
__global__ void k_f16_level_max(const float* __restrict__ m32, int ms, int nc,
                                const float* __restrict__ colf, LevelBlocks lb,
                                uint32_t* __restrict__ lmax) {
  __shared__ float sm[kBlock / 64];
  __shared__ float4 sc4[kMaxColf / 4];  // the column factors, zero past ncoef
  for (int k4 = threadIdx.x; k4 < ms / 4; k4 += kBlock) {
    float4 c;
    c.x = 4 * k4 < nc ? colf[4 * k4] : 0.f;
    c.y = 4 * k4 + 1 < nc ? colf[4 * k4 + 1] : 0.f;
    c.z = 4 * k4 + 2 < nc ? colf[4 * k4 + 2] : 0.f;
    c.w = 4 * k4 + 3 < nc ? colf[4 * k4 + 3] : 0.f;
    sc4[k4] = c;
  }
  __syncthreads();
  const int l = level_of_block(lb, blockIdx.x);
  const int64_t ngrp = lb.blk_off[l + 1] - lb.blk_off[l];
  const int64_t n4 = (lb.box_off[l + 1] - lb.box_off[l]) * ms / 4;
  const float4* v4 = reinterpret_cast<const float4*>(m32 + lb.box_off[l] * ms);
  float m = 0.f;
  // k = 4 t mod ms, advanced by the stride's residue (no division per element)
  const int64_t t0 = (blockIdx.x - lb.blk_off[l]) * kBlock + threadIdx.x, stride = ngrp * kBlock;
  const int kinc = (int)((4 * stride) % ms);
  int k = (int)((4 * t0) % ms);
  for (int64_t t = t0; t < n4; t += stride) {
    const float4 v = v4[t];
    const float4 c = sc4[k >> 2];
    m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x * c.x), fabsf(v.y * c.y)), fmaxf(fabsf(v.z * c.z), fabsf(v.w * c.w))));
    k += kinc;
    if (k >= ms) k -= ms;
  }
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) m = fmaxf(m, __shfl_xor(m, w, 64));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = 0.f;
    for (int w = 0; w < kBlock / 64; ++w) b = fmaxf(b, sm[w]);
    atomicMax(&lmax[l], __float_as_uint(b));
  }
}

// The power of two 2^(14 - e) that puts a level's largest |M_k colf_k| (float
// bits lmax) into [2^13, 2^14); 2^e is returned as the inverse scale.
__device__ __forceinline__ int f16_level_exp(uint32_t lmax_bits) {
  const float m = __uint_as_float(lmax_bits);
  int e = 0;
  if (m > 0.f) frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
  return e;
}

// FP16 form, pass 2: every box's FP32 multipole row times the column factors
// colf_k, scaled by its level's power of two so that the level's largest
// entry lies in [2^13, 2^14), split into 2 FP16 pieces.  lpb (16 or 32)
// lanes per box, lane u holding k = 8 u .. 8 u + 7 (quad (ks * 2 + piece) * 4
// + g, u = 4 ks + g).
__global__ void k_split_mult_h(const float* __restrict__ m32, int ms, int nc, int kst, int lpb,
                               const float* __restrict__ colf, LevelBlocks lb,
                               const uint32_t* __restrict__ lmax, u32x4* __restrict__ out) {
  __shared__ float sColf[kMaxColf];  // the column factors, zero past ncoef
  for (int k = threadIdx.x; k < 32 * kst && k < kMaxColf; k += blockDim.x) sColf[k] = k < nc ? colf[k] : 0.f;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sh = lpb == 16 ? 4 : 5;  // lpb is 16 or 32
  const int64_t box = lb.box_off[lb.l0] + (t >> sh);
  const int u = (int)(t & (lpb - 1));
  if (box >= lb.box_off[lb.l1 + 1] || u >= 4 * kst) return;
  int l = lb.l0;
  while (l < lb.l1 && box >= lb.box_off[l + 1]) ++l;
  // 2^(14 - e): exact, so x colf_k sc equals ldexp(x colf_k, 14 - e)
  const float sc = ldexpf(1.f, 14 - f16_level_exp(lmax[l]));
  // the row's k = 8 u .. 8 u + 7 as two float4 loads (ms is a multiple of 4;
  // quads past the row read as zero)
  const float4* r4 = reinterpret_cast<const float4*>(m32 + box * ms);
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const float4 v0 = 8 * u < ms ? r4[2 * u] : z4, v1 = 8 * u + 4 < ms ? r4[2 * u + 1] : z4;
  const float x[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
  uint32_t pc[8][2];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 8 * u + j;
    split_f16_f32(k < nc ? x[j] * sColf[k] * sc : 0.f, pc[j]);
  }
  u32x4 q[2];
  pack_quads<2>(pc, q);
  u32x4* o = out + box * (kst * 2 * 4);
  const int ks = u / 4, g = u % 4;
  o[(ks * 2 + 0) * 4 + g] = q[0];
  o[(ks * 2 + 1) * 4 + g] = q[1];
}

// FP16 form: a (row block, k step) product block takes all three piece
// products h_a h_b + h_a l_b + l_a h_b when the lowest local degree n of its
// rows plus the lowest multipole degree n' of its k values is below
// kF16Tier, and h_a h_b alone otherwise.  A term of degrees (n, n') reaches a
// target's potential scaled by about (a / |d|)^(n + n'), a the box
// half-diagonal and |d| >= 2 box sizes, so at most (sqrt(3) / 4)^(n + n');
// the dropped piece products are 2^-11 of that term: below 1e-7 relative from
// n + n' = 11 on.
constexpr bool f16_cross(int rb, int ks) { return isqrt_c(16 * rb) + isqrt_c(32 * ks) < kF16Tier; }

// Shape of the kernel for order P and NP pieces.
template <int P, int NP, bool F16 = false, bool AD = false>
struct Shape {
  static constexpr int NC = (P + 1) * (P + 1);
  static constexpr int RB = (NC + 15) / 16;  // 16-row blocks
  static constexpr int RP = RB * 16;
  static constexpr int KST = m2lb_ksteps(NC);       // 32-wide k steps
  static constexpr int QR = m2lb_row_quads(NC, NP);  // quads per source box
  static constexpr int KC = m2lb_kc(NC, NP, AD);     // k steps per staged chunk
  static constexpr int NCH = m2lb_nch(NC, NP, AD);   // chunks per operator
  static constexpr int GQ = m2lb_gq(KC, NP);         // quads between lane groups g
  static constexpr int QCS = m2lb_qcs(KC, NP);       // quads between rows
  static constexpr int CQ = RP * QCS;                // quads per stored chunk
  static constexpr int QD = 4 * GQ;                  // quads of a row the MFMAs read
  static constexpr int NV = NC * QD;                 // quads staged per chunk
  static constexpr int PER_THREAD = (NV + kThreads - 1) / kThreads;
  // row blocks whose MFMA chains are interleaved (per group of A loads):
  // up to 6 in the FP16 form (measured: -7 % time at p = 8), fewer in the
  // BF16 forms, whose extra piece would not fit the registers, and one from
  // 5 (BF16) or 6 (FP16) k steps on, where the accumulators alone take half
  // the registers (p >= 11 still spills a little)
  static constexpr int RGW = F16 ? (KST >= 6 ? 1 : M2LB_RG_F16) : (KST >= 5 ? 1 : M2LB_RG);
  static constexpr int RG = RB < RGW ? RB : RGW;
  // Prefetch the next offset's B quads (a second register set) up to 3 k
  // steps (p <= 8).  From 4 on (p = 9, 10) the second set made the compiler
  // spill (84-112 bytes per lane), and the adaptive p = 10 M2L took 10.3 ms
  // instead of 6.3 ms without it.
  static constexpr bool PREFETCH_B = KST <= M2LB_PB_KST;
  // offsets of B in flight (measured at p = 8: two were no faster than one)
  static constexpr int PBD = !PREFETCH_B ? 0 : (F16 && KST <= M2LB_PB2_KST ? 2 : 1);
  // FP16 form, one chunk per operator: operators loaded two offsets ahead (a
  // second register set for the staged quads; measured at p = 8: M2L 3.17 ->
  // 3.10 ms)
  static constexpr bool OP2 = F16 && M2LB_OP2 && NCH == 1;
};

// F16: FP16 pieces of scaled operands (FMM_M2L_F16X2): FP32 chains of
// kGroupF16 offsets summed into the total, rows times rowf and the level's
// inverse scale (from lmax) at the end; high-degree blocks take one piece
// product (f16_cross).
template <int P, int NP, bool F16, bool AD>
__global__ __launch_bounds__(kThreads) void k_m2l_bf(m2l::Args a, const u32x4* __restrict__ multq,
                                                     const u32x4* __restrict__ zero_q,
                                                     const u32x4* __restrict__ ops,
                                                     float* __restrict__ out,
                                                     const uint32_t* __restrict__ lmax,
                                                     const float* __restrict__ rowf,
                                                     float* __restrict__ half_out) {
  typedef Shape<P, NP, F16, AD> S;
  typedef Prod<NP> PR;
  constexpr int NC = S::NC, RB = S::RB, RP = S::RP, KST = S::KST, QR = S::QR;
  constexpr int KC = S::KC, NCH = S::NCH, GQ = S::GQ, QCS = S::QCS, RG = S::RG;
  __shared__ u32x4 sT[2][RP * QCS];
  __shared__ uint32_t sSlot[AD ? 1 : m2l::kHalo];  // the adaptive form has no halo
  __shared__ int sBox[6];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kg = lane >> 4;
  m2l::TileT<AD, true> tl;  // the tail groups may be split
  if (!tl.setup(a, wave * 16 + col, sSlot, sBox)) return;  // uniform over the work-group
  const int pi = tl.pi;
  // offsets [i0, i1): all of them, or one part of a split group
  const bool whole = tl.part < 0;
  const int i0 = whole ? 0 : tl.part * kIL / kM2lParts;
  const int i1 = whole ? kIL : (tl.part + 1) * kIL / kM2lParts;
  const u32x4* mlev = multq + tl.lvl_off * QR;

  f32x4 sum[RB], comp[RB], acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) sum[r] = comp[r] = acc[r] = f32x4{0, 0, 0, 0};

  // Operator chunk ch of operator op into registers / into an LDS buffer.
  // Chunks are stored in their LDS layout; only the NC real rows and the
  // quads the MFMAs read are staged (loads are clamped so that every lane
  // issues the same loads).  Rows NC..RP-1 of both buffers stay zero.
  auto stage_load = [&](int op, int ch, u32x4* reg) {
    const u32x4* base = ops + ((size_t)op * NCH + ch) * S::CQ;
#pragma unroll
    for (int i = 0; i < S::PER_THREAD; ++i) {
      int e = tid + i * kThreads;
      e = e < S::NV ? e : S::NV - 1;
      reg[i] = base[(e / S::QD) * QCS + e % S::QD];
    }
  };
  auto stage_store = [&](u32x4* buf, const u32x4* reg) {
#pragma unroll
    for (int i = 0; i < S::PER_THREAD; ++i) {
      const int e = tid + i * kThreads;
      if (e < S::NV) buf[(e / S::QD) * QCS + e % S::QD] = reg[i];
    }
  };
  for (int e = tid; e < 2 * (RP - NC) * QCS; e += kThreads) {
    const int b = e / ((RP - NC) * QCS);
    sT[b][NC * QCS + e % ((RP - NC) * QCS)] = u32x4{0, 0, 0, 0};
  }
  auto row_of = [&](m2l::Src src) -> const u32x4* {
    return src.ok ? mlev + (int64_t)src.slot * QR : zero_q;
  };
  // B quads of a source row: this lane group's quad of every (k step, piece).
  auto load_b = [&](const u32x4* ms, u32x4* b) {
#pragma unroll
    for (int i = 0; i < KST * NP; ++i) b[i] = ms[i * 4 + kg];
  };
  // MFMAs of operator chunk ch (staged in buf) against B quads b.
  auto compute_chunk = [&](const u32x4* buf, int ch, const u32x4* b) {
    const u32x4* sa = buf + col * QCS + kg * GQ;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const int ks = ch * KC + kc;
      if (ks >= KST) break;
#pragma unroll
      for (int r0 = 0; r0 < RB; r0 += RG) {
        u32x4 av[RG][NP];
#pragma unroll
        for (int rr = 0; rr < RG; ++rr)
#pragma unroll
          for (int i = 0; i < NP; ++i)
            if (r0 + rr < RB && (!F16 || i == 0 || f16_cross(r0 + rr, ks)))
              av[rr][i] = sa[16 * (r0 + rr) * QCS + kc * NP + i];
#pragma unroll
        for (int t = 0; t < PR::N; ++t)
#pragma unroll
          for (int rr = 0; rr < RG; ++rr)
            if (r0 + rr < RB) {
              if (F16) {
                // blocks of high degree take h_a h_b only (t = N - 1)
                if (t == PR::N - 1 || f16_cross(r0 + rr, ks))
                  acc[r0 + rr] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                      __builtin_bit_cast(f16x8, av[rr][PR::a[t]]),
                      __builtin_bit_cast(f16x8, b[ks * NP + PR::b[t]]), acc[r0 + rr], 0, 0, 0);
              } else {
                acc[r0 + rr] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, av[rr][PR::a[t]]),
                    __builtin_bit_cast(bf16x8, b[ks * NP + PR::b[t]]), acc[r0 + rr], 0, 0, 0);
              }
            }
      }
    }
  };

  constexpr bool PB = S::PREFETCH_B;
  constexpr int FLUSH = kFlush;
  u32x4 reg[S::PER_THREAD], reg2[S::OP2 ? S::PER_THREAD : 1];
  u32x4 b0[KST * NP], b1[PB ? KST * NP : 1], b2[S::PBD > 1 ? KST * NP : 1];
  // Pipeline over the class's offsets: offset i is computed while the
  // operator of the next stage and the B quads of offset i + PBD are loaded
  // and the source slot of offset i + PBD + 1 is looked up (PBD offsets of B
  // in flight: B loads from L2 are the latency the kernel waits on most).
  constexpr int PBD = S::PBD;
  int i = i0, ndx, ndy, ndz;
  int op = m2l::il_offset(pi, i0, ndx, ndy, ndz);
  int nop = m2l::il_offset(pi, i0 + 1 < i1 ? i0 + 1 : i1 - 1, ndx, ndy, ndz);
  auto lookup_at = [&](int k) -> m2l::Src {
    int ldx, ldy, ldz;
    const int kk = k < i1 ? k : i1 - 1;
    m2l::il_offset(pi, kk, ldx, ldy, ldz);
    return tl.lookup(sSlot, kk, ldx, ldy, ldz);
  };
  m2l::Src sw[PBD + 1];  // sources of offsets i .. i + PBD
#pragma unroll
  for (int k = 0; k <= PBD; ++k) sw[k] = lookup_at(i0 + k);
  bool wave_any = false;
  if (PB) {
    load_b(row_of(sw[0]), b0);
    if (PBD > 1) load_b(row_of(sw[1]), b1);
    wave_any = __any(sw[0].ok);
  }
  stage_load(op, 0, reg);
  stage_store(sT[0], reg);
  if (S::OP2) stage_load(nop, 0, reg);  // the operator of offset i0 + 1, stored at offset i0
  __syncthreads();
  int cur = 0;

  // bc: B quads of offset i (loaded); bl: the buffer that receives offset
  // i + PBD.  OP2 (one chunk per operator): rin holds the operator of offset
  // i + 1 (loaded one offset earlier), rout receives that of offset i + 2.
  auto do_offset = [&](u32x4* bc, u32x4* bl, u32x4* rin, u32x4* rout) -> bool {
    const bool more = i + 1 < i1;
    const int fop = m2l::il_offset(pi, i + 2 < i1 ? i + 2 : i1 - 1, ndx, ndy, ndz);
    const m2l::Src s_far = lookup_at(i + PBD + 1);
    if (!PB) {
      load_b(row_of(sw[0]), bc);
      wave_any = __any(sw[0].ok);
    }
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const bool last_chunk = ch == NCH - 1;
      if (S::OP2)
        stage_load(fop, 0, rout);
      else
        stage_load(last_chunk ? (more ? nop : op) : op, last_chunk ? 0 : ch + 1, reg);
      if (PB && ch == 0) load_b(row_of(sw[PBD]), bl);
      if (wave_any) compute_chunk(sT[cur], ch, bc);
      if (F16 && last_chunk && ((i + 1 - i0) % kGroupF16 == 0 || !more)) {
        // one scale per level: the FP32 chain runs over kGroupF16 offsets,
        // then joins the sum (the same two-level summation as a chain per
        // offset scaled into a partial of kGroupF16 offsets)
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          sum[r] += acc[r];
          acc[r] = f32x4{0, 0, 0, 0};
        }
      }
      if (!F16 && last_chunk && (FLUSH == 1 ? wave_any : ((i + 1) % FLUSH == 0 || !more))) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const f32x4 y = acc[r] - comp[r];
          const f32x4 t = sum[r] + y;
          comp[r] = (t - sum[r]) - y;
          sum[r] = t;
          acc[r] = f32x4{0, 0, 0, 0};
        }
      }
      if (last_chunk && !more) return false;
      stage_store(sT[cur ^ 1], S::OP2 ? rin : reg);
      m2l::lds_barrier();
      cur ^= 1;
    }
    ++i;
    op = nop;
    nop = fop;
    if (PB) wave_any = __any(sw[1].ok);
#pragma unroll
    for (int k = 0; k < PBD; ++k) sw[k] = sw[k + 1];
    sw[PBD] = s_far;
    return true;
  };
  if (PBD == 2) {
    while (do_offset(b0, b2, reg, reg2) && do_offset(b1, b0, reg2, reg) && do_offset(b2, b1, reg, reg2) &&
           do_offset(b0, b2, reg2, reg) && do_offset(b1, b0, reg, reg2) && do_offset(b2, b1, reg2, reg)) {
    }
  } else if (PBD == 1) {
    while (do_offset(b0, b1, reg, reg2) && do_offset(b1, b0, reg2, reg)) {
    }
  } else {
    while (do_offset(b0, b0, reg, reg2) && do_offset(b0, b0, reg2, reg)) {
    }
  }

  if (!tl.col_ok) return;
  // parts 1.. of a split group: into their slots of half_out, added to part
  // 0's result by k_m2l_add_half after the launch
  float* o = !whole && tl.part > 0
                 ? half_out + ((tl.sidx * (kM2lParts - 1) + tl.part - 1) * m2l::kTargetsPerGroup + wave * 16 + col) * NC
                 : out + (tl.lvl_off + tl.target_slot(a)) * NC;
  // FP16 form: rows times 2^-ra_r (rowf) and the source level's 2^(e - 14)
  const float lsc = F16 ? ldexpf(1.f, f16_level_exp(lmax[tl.l]) - 14) : 1.f;
  // Accumulator layout of the 16x16 FP32-output MFMAs: lane l holds column
  // l % 16, rows 4 (l / 16) + i.
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * r + 4 * kg + e;
      if (row < NC) o[row] = F16 ? sum[r][e] * (rowf[row] * lsc) : sum[r][e];
    }
}

// Wide FP16 form (p <= kM2lWidePMax): the same products on
// v_mfma_f32_32x32x16_f16.  A work-group of 4 waves owns a 128-target tile
// (the tiles of m2l_common.h); lane (c, h) = (lane % 32, lane / 32) of a wave
// holds target c of its 32 and the k half h of every 16-wide k step.  Each
// 16-byte A read from LDS feeds a 32 x 32 block, and the work-group's LDS (two
// operator buffers and the halo) leaves room for two work-groups per CU.
//  * Operators: the quads the products read (m2lw_*), copied per offset from global
//    memory straight into the LDS buffer not being read (global_load_lds, 64
//    quads per wave instruction), waited for before the offset's barrier.
//  * Sources: the FP16 pieces of k_split_mult_h (quad (ks * 2 + piece) * 4 +
//    g holds k = 32 ks + 8 g ..); lane (c, h) takes quad (ks * 2 + piece) * 4
//    + 2 (s % 2) + h of k step s (ks = s / 2), all loaded one offset ahead.
//  * Source reuse between offsets (uniform tree, whole tiles): the source of
//    target t at offset d is box t - d, so after offset d the source of t at
//    d + D is the one its lattice neighbour t - D held at d.  The 128 targets
//    of a full tile are the class-pi children of an 8 x 4 x 4 block of
//    parents; they are laid out so that each wave holds a 4 x 4 x 2 sub-block,
//    lane c = a + 4 b + 16 c' along the block's axes (A the long one, B, C the
//    others in index order), and every class walks its 189 offsets in an
//    order (kChainOrder) of 3 x 3 snakes in (d_A, d_B) with steps of 2 per
//    d_C: after a step D = +-2 e_A or +-2 e_B a lane takes its neighbour's
//    source quads by a DPP row shift (the rows of 16 lanes hold a 4 x 4 (a,
//    b) layer), and only the lanes on the face the step uncovers load from
//    memory.  39 of the 189 offsets load every row, 150 a quarter of them: the
//    source traffic drops to 40 %.
//  * Accumulator layout (32 x 32 FP32 output): lane l holds column l % 32,
//    element e row 8 (e / 4) + 4 (l / 32) + e % 4.
//  * Rows past ncoef read row ncoef - 1 (their output rows are not stored).
//  * Tiers, chains of kGroupF16 offsets and the final scaling as in k_m2l_bf.
constexpr int kWideWaves = 4;
constexpr int kWideThreads = kWideWaves * 64;
static_assert(kWideWaves * 32 == m2l::kTargetsPerGroup, "a wide work-group covers one tile");

// Offset orders of the reuse form, per long axis A and class: code = op |
// (dx + 4) << 9 | (dy + 4) << 13 | (dz + 4) << 17 | move << 21, move = how the
// offset follows the previous one: 0 none (every lane loads), 1 d_A + 2,
// 2 d_A - 2, 3 d_B + 2, 4 d_B - 2.
struct ChainOrder {
  uint32_t v[3][8][kIL];
};
constexpr int chain_other(int A, int k) { return k == 0 ? (A == 0 ? 1 : 0) : (A == 2 ? 1 : 2); }
constexpr ChainOrder make_chain_order() {
  ChainOrder t{};
  for (int A = 0; A < 3; ++A) {
    const int B = chain_other(A, 0), C = chain_other(A, 1);
    for (int pi = 0; pi < 8; ++pi) {
      const int pa[3] = {(pi >> 2) & 1, (pi >> 1) & 1, pi & 1};
      int n = 0, prev[3] = {0, 0, 0};
      bool have = false;
      for (int dc = pa[C] - 3; dc <= pa[C] + 2; ++dc)
        for (int ra = 0; ra < 2; ++ra)
          for (int rb = 0; rb < 2; ++rb)
            for (int jj = 0; jj < 3; ++jj)
              for (int ii = 0; ii < 3; ++ii) {
                const int i = jj % 2 == 0 ? ii : 2 - ii;  // snake over the 3 x 3 grid
                int d[3] = {0, 0, 0};
                d[A] = pa[A] - 3 + ra + 2 * i;
                d[B] = pa[B] - 3 + rb + 2 * jj;
                d[C] = dc;
                if (d[0] >= -1 && d[0] <= 1 && d[1] >= -1 && d[1] <= 1 && d[2] >= -1 && d[2] <= 1) continue;
                uint32_t move = 0;
                if (have && d[C] == prev[C]) {
                  if (d[B] == prev[B] && d[A] == prev[A] + 2) move = 1;
                  if (d[B] == prev[B] && d[A] == prev[A] - 2) move = 2;
                  if (d[A] == prev[A] && d[B] == prev[B] + 2) move = 3;
                  if (d[A] == prev[A] && d[B] == prev[B] - 2) move = 4;
                }
                t.v[A][pi][n++] = (uint32_t)m2l_op_index(d[0], d[1], d[2]) | (uint32_t)(d[0] + 4) << 9 |
                                  (uint32_t)(d[1] + 4) << 13 | (uint32_t)(d[2] + 4) << 17 | move << 21;
                prev[0] = d[0];
                prev[1] = d[1];
                prev[2] = d[2];
                have = true;
              }
    }
  }
  return t;
}
// every order holds the class's 189 interaction-list offsets once each
constexpr bool chain_order_ok(const ChainOrder& t) {
  for (int A = 0; A < 3; ++A)
    for (int pi = 0; pi < 8; ++pi) {
      bool seen[216] = {};
      for (int k = 0; k < kIL; ++k) {
        const uint32_t c = t.v[A][pi][k];
        const int d[3] = {(int)((c >> 9) & 15u) - 4, (int)((c >> 13) & 15u) - 4, (int)((c >> 17) & 15u) - 4};
        int cell = 0;
        bool near = true;
        for (int q = 0; q < 3; ++q) {
          const int pq = (pi >> (2 - q)) & 1, u = d[q] - (pq - 3);
          if (u < 0 || u > 5) return false;
          cell = cell * 6 + u;
          near = near && d[q] >= -1 && d[q] <= 1;
        }
        if (near || seen[cell] || (int)(c & 511u) != m2l_op_index(d[0], d[1], d[2])) return false;
        seen[cell] = true;
      }
    }
  return true;
}
static_assert(chain_order_ok(make_chain_order()), "offset orders of the reuse form");
static __constant__ ChainOrder kChainOrder = make_chain_order();

template <int P>
struct WShape {
  static constexpr int NC = (P + 1) * (P + 1);
  static constexpr int RB = (NC + 31) / 32;        // 32-row blocks
  static constexpr int KS = m2lw_ksteps(NC);       // 16-wide k steps with data
  static constexpr int QR = m2lb_row_quads(NC, 2);  // quads per source box
  static constexpr int NQ = m2lw_op_quads(NC);     // quads per operator (last: zero)
  static constexpr int NCHUNK = (NQ + 63) / 64;    // 64-quad copies per operator
  static constexpr int NQP = NCHUNK * 64;          // LDS quads per buffer
};

// The 16-byte quad v of the lane that the DPP row shift CTRL names (zero
// where the row has no such lane)
template <int CTRL>
__device__ __forceinline__ u32x4 dpp_quad(u32x4 v) {
  u32x4 r;
#pragma unroll
  for (int w = 0; w < 4; ++w) r[w] = (uint32_t)__builtin_amdgcn_mov_dpp((int)v[w], CTRL, 0xF, 0xF, true);
  return r;
}
template <int CTRL, int KS>
__device__ __forceinline__ void dpp_rows(const u32x4* bh, const u32x4* bl, u32x4* nh, u32x4* nl) {
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    nh[s] = dpp_quad<CTRL>(bh[s]);
    nl[s] = dpp_quad<CTRL>(bl[s]);
  }
}

// One tile of the wide form: logical group lg (part pt, split index si),
// or, with lg < 0, the group the work-group's hardware index names
// (m2l::decode_group).  Uniform over the work-group; contains barriers.
// One tile of the wide form per call of `tile`: logical group lg (whole),
// or, with lg < 0, the group the work-group's hardware index names
// (m2l::decode_group, split parts included).  Plain launch (PERSIST false):
// one tile per work-group.  Persistent form (FMM_SCHED_M2L_PERSISTENT):
// two resident work-groups per CU; those of XCD x (hardware index % 8) take
// the XCD's contiguous range of logical groups in order from counter
// ticket[x], one whole tile at a time (a.ksplit = 0), so each tile is summed
// as in the unsplit form; a work-group leaves when its XCD's range is spent.
template <int P, bool AD, bool PERSIST>
__global__ __launch_bounds__(kWideThreads, 2) void k_m2l_w(m2l::Args a, const u32x4* __restrict__ multq,
                                                         const u32x4* __restrict__ zero_q,
                                                         const u32x4* __restrict__ ops,
                                                         float* __restrict__ out,
                                                         const uint32_t* __restrict__ lmax,
                                                         const float* __restrict__ rowf,
                                                         float* __restrict__ half_out,
                                                         uint32_t* __restrict__ ticket) {
  typedef WShape<P> S;
  __shared__ u32x4 sT0[S::NQP];
  __shared__ u32x4 sT1[S::NQP];
  __shared__ uint32_t sSlot[AD ? 1 : m2l::kHalo];
  __shared__ int sBox[6];
  const int64_t pt = -1, si = 0;
  auto tile = [&](int64_t lg) {
    typedef Prod<2> PR;
    typedef float f32x16 __attribute__((ext_vector_type(16)));
    constexpr int NC = S::NC, RB = S::RB, KS = S::KS, QR = S::QR;
    static_assert(S::NQ <= m2lb_op_quads(S::NC, 2, AD), "the wide operators fit the split-operator array");
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int col = lane & 31, hk = lane >> 5;
    m2l::TileT<AD, true> tl;
    if (lg < 0 ? !tl.setup(a, wave * 32 + col, sSlot, sBox)
               : !tl.setup_at(a, lg, pt, si, wave * 32 + col, sSlot, sBox))
      return;  // uniform over the work-group
    const int pi = tl.pi;
    const bool whole = tl.part < 0;
    const int i0 = whole ? 0 : tl.part * kIL / kM2lParts;
    const int i1 = whole ? kIL : (tl.part + 1) * kIL / kM2lParts;
    const u32x4* mlev = multq + tl.lvl_off * QR;

    // Source reuse: a whole tile of the uniform tree whose parents form an
    // 8 x 4 x 4 block (sBox holds 2 pmin - 2 and 2 pmax + 3 per axis).
    bool chain = false;
    int ax = 0;
    if constexpr (!AD) {
      int ext[3], lo[3], n8 = 0, n4 = 0;
  #pragma unroll
      for (int k = 0; k < 3; ++k) {
        lo[k] = (sBox[k] + 2) / 2;
        ext[k] = (sBox[3 + k] - 3) / 2 - lo[k] + 1;
        n8 += ext[k] == 8;
        n4 += ext[k] == 4;
        if (ext[k] == 8) ax = k;
      }
      chain = __syncthreads_and(whole && n8 == 1 && n4 == 2 && tl.col_ok);  // a full tile
      if (chain) {
        // lane c = a + 4 b + 16 c': parent lo + (4 (w & 1) + a) e_A + b e_B + (2 (w >> 1) + c') e_C
        const int B = chain_other(ax, 0);
        const int ua = 4 * (wave & 1) + (col & 3), ub = (col >> 2) & 3, uc = 2 * (wave >> 1) + (col >> 4);
        int pc[3];
  #pragma unroll
        for (int k = 0; k < 3; ++k) pc[k] = lo[k] + (k == ax ? ua : (k == B ? ub : uc));
        tl.tx = 2 * pc[0] + ((pi >> 2) & 1);
        tl.ty = 2 * pc[1] + ((pi >> 1) & 1);
        tl.tz = 2 * pc[2] + (pi & 1);
        tl.col_ok = true;
      }
    }
    const uint32_t* ord = kChainOrder.v[ax][pi];
    // offset k of this work-group's order: its operator and (dx, dy, dz)
    auto offset_at = [&](int k, int& dx, int& dy, int& dz) -> int {
      if constexpr (AD) return m2l::il_offset(pi, k, dx, dy, dz);  // the source table's order
      const uint32_t c = ord[k];
      dx = (int)((c >> 9) & 15u) - 4;
      dy = (int)((c >> 13) & 15u) - 4;
      dz = (int)((c >> 17) & 15u) - 4;
      return (int)(c & 511u);
    };
    auto move_at = [&](int k) -> int { return chain ? (int)((ord[k] >> 21) & 7u) : 0; };

    f32x16 sum[RB], acc[RB];
  #pragma unroll
    for (int r = 0; r < RB; ++r)
  #pragma unroll
      for (int e = 0; e < 16; ++e) sum[r][e] = acc[r][e] = 0.f;

    // operator op into buf: wave w copies the 64-quad chunks w, w + 4, ...
    // (reads past the operator's end are clamped to its last quad; they land
    // in the buffer's padding)
    auto stage = [&](int op, u32x4* buf) {
      const u32x4* base = ops + (size_t)op * S::NQ;
  #pragma unroll
      for (int j = 0; j < (S::NCHUNK + kWideWaves - 1) / kWideWaves; ++j) {
        const int e0 = (j * kWideWaves + wave) * 64;
        if (e0 < S::NQP) {
          const int e = e0 + lane;
          __builtin_amdgcn_global_load_lds(
              (__attribute__((address_space(1))) void*)(base + (e < S::NQ ? e : S::NQ - 1)),
              (__attribute__((address_space(3))) void*)(buf + e0), 16, 0, 0);
        }
      }
    };
    auto row_of = [&](m2l::Src src) -> const u32x4* {
      return src.ok ? mlev + (int64_t)src.slot * QR : zero_q;
    };
    // B quads of a source row for this lane: all k steps, both pieces (the
    // quads past ncoef hold zeros)
    auto load_b = [&](const u32x4* ms, u32x4* bh, u32x4* bl) {
  #pragma unroll
      for (int s = 0; s < KS; ++s) {
        bh[s] = ms[((s >> 1) * 2 + 0) * 4 + 2 * (s & 1) + hk];
        bl[s] = ms[((s >> 1) * 2 + 1) * 4 + 2 * (s & 1) + hk];
      }
    };
    // B of the next offset from this one's by a row shift
    auto shift_b = [&](int mv, const u32x4* bh, const u32x4* bl, u32x4* nh, u32x4* nl) {
      switch (mv) {
        case 1:  // from lane a - 1 (row_shr:1)
          dpp_rows<0x111, KS>(bh, bl, nh, nl);
          break;
        case 2:  // from lane a + 1 (row_shl:1)
          dpp_rows<0x101, KS>(bh, bl, nh, nl);
          break;
        case 3:  // from lane b - 1 (row_shr:4)
          dpp_rows<0x114, KS>(bh, bl, nh, nl);
          break;
        default:  // from lane b + 1 (row_shl:4)
          dpp_rows<0x104, KS>(bh, bl, nh, nl);
          break;
      }
    };
    // lanes with no neighbour for move mv (they load)
    const int la = col & 3, lb = (col >> 2) & 3;
    auto face = [&](int mv) -> bool {
      return mv == 0 || (mv == 1 && la == 0) || (mv == 2 && la == 3) || (mv == 3 && lb == 0) ||
             (mv == 4 && lb == 3);
    };
    // this lane's operator rows (rows past ncoef read the block's last one),
    // offset by its k half: + 2 h in the steps with both pieces, + h after
    int arc[RB], arn[RB];
  #pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int row = 32 * r + col;
      const int a0 = m2lw_block_base(NC, r) + ((row < NC ? row : NC - 1) - 32 * r) * m2lw_row_len(NC, r);
      arc[r] = a0 + 2 * hk;
      arn[r] = a0 + hk;
    }
    // the lanes whose k half of the last step lies past ncoef read the zero quad
    const bool dead = !m2lw_half_live(NC, KS - 1, 1) && hk == 1;
    auto compute = [&](const u32x4* buf, const u32x4* bh, const u32x4* bl) {
  #pragma unroll
      for (int s = 0; s < KS; ++s) {
        u32x4 ah[RB], al[RB];
  #pragma unroll
        for (int r = 0; r < RB; ++r) {
          const bool cr = s < m2lw_cross_steps(NC, r);
          int q0 = (cr ? arc[r] : arn[r]) + m2lw_pos(NC, r, s, 0, 0);
          if (s == KS - 1 && dead) q0 = S::NQ - 1;
          ah[r] = buf[q0];
          if (f16_cross_w(r, s)) al[r] = buf[s == KS - 1 && dead ? S::NQ - 1 : q0 + 1];
        }
  #pragma unroll
        for (int t = 0; t < PR::N; ++t)
  #pragma unroll
          for (int r = 0; r < RB; ++r)
            if (t == PR::N - 1 || f16_cross_w(r, s))
              acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                  __builtin_bit_cast(f16x8, PR::a[t] ? al[r] : ah[r]),
                  __builtin_bit_cast(f16x8, PR::b[t] ? bl[s] : bh[s]), acc[r], 0, 0, 0);
      }
    };

    u32x4 bh0[KS], bl0[KS], bh1[KS], bl1[KS];
    int i = i0, ndx, ndy, ndz;
    auto lookup_at = [&](int k) -> m2l::Src {
      int ldx, ldy, ldz;
      const int kk = k < i1 ? k : i1 - 1;
      offset_at(kk, ldx, ldy, ldz);
      return tl.lookup(sSlot, kk, ldx, ldy, ldz);
    };
    m2l::Src cur_src = lookup_at(i0), next_src = lookup_at(i0 + 1);
    load_b(row_of(cur_src), bh0, bl0);
    stage(offset_at(i0, ndx, ndy, ndz), sT0);
    __builtin_amdgcn_s_waitcnt(kVmcntZero);
    __syncthreads();
    // offset i: its operator in bufc, its B in (bhc, blc); the next offset's B
    // goes to (bhn, bln) (shifted from this one's and completed by the face
    // lanes' loads, or loaded by every lane) and its operator to bufn.
    auto do_offset = [&](const u32x4* bufc, u32x4* bufn, u32x4* bhc, u32x4* blc, u32x4* bhn,
                         u32x4* bln) -> bool {
      const bool more = i + 1 < i1;
      const m2l::Src far_src = lookup_at(i + 2);
      // this offset's source quads (loaded during the previous one) first: the
      // copy and the loads issued below then need no wait until the barrier
      __builtin_amdgcn_s_waitcnt(kVmcntZero);
      if (more) {
        const int mv = move_at(i + 1);
        if (mv != 0) shift_b(mv, bhc, blc, bhn, bln);
        stage(offset_at(i + 1, ndx, ndy, ndz), bufn);
        if (face(mv)) load_b(row_of(next_src), bhn, bln);
      }
      if (__any(cur_src.ok)) compute(bufc, bhc, blc);
      if ((i + 1 - i0) % kGroupF16 == 0 || !more) {
  #pragma unroll
        for (int r = 0; r < RB; ++r) {
          sum[r] += acc[r];
  #pragma unroll
          for (int e = 0; e < 16; ++e) acc[r][e] = 0.f;
        }
      }
      if (!more) return false;
      // this wave's part of the copy has landed (the next offset's source
      // loads, issued after it, may still be in flight), and every LDS read of
      // this offset has returned (each fed a product); then the work-group's
      // barrier, without the memory fence of __syncthreads (which would wait
      // for the source loads too)
      __builtin_amdgcn_s_waitcnt(vmcnt_op(2 * KS));
      __asm__ volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      __asm__ volatile("" ::: "memory");
      ++i;
      cur_src = next_src;
      next_src = far_src;
      return true;
    };
    while (do_offset(sT0, sT1, bh0, bl0, bh1, bl1) && do_offset(sT1, sT0, bh1, bl1, bh0, bl0)) {
    }

    if (!tl.col_ok) return;
    float* o = !whole && tl.part > 0
                   ? half_out + ((tl.sidx * (kM2lParts - 1) + tl.part - 1) * m2l::kTargetsPerGroup + wave * 32 + col) * NC
                   : out + (tl.lvl_off + tl.target_slot(a)) * NC;
    const float lsc = ldexpf(1.f, f16_level_exp(lmax[tl.l]) - 14);
  #pragma unroll
    for (int r = 0; r < RB; ++r)
  #pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = 32 * r + 8 * (e / 4) + 4 * hk + e % 4;
        if (row < NC) o[row] = sum[r][e] * (rowf[row] * lsc);
      }
  };
  if constexpr (!PERSIST) {
    tile(-1);
  } else {
    __shared__ uint32_t sK;
    const int xcd = (int)(blockIdx.x % 8);
    const int64_t per_xcd = (a.ngroups + 7) / 8;
    for (;;) {
      if (threadIdx.x == 0) sK = atomicAdd(&ticket[xcd], 1u);
      __syncthreads();
      const int64_t k = sK;
      __syncthreads();  // every lane has read sK before the next ticket
      const int64_t lg = xcd * per_xcd + k;
      if (k >= per_xcd || lg >= a.ngroups) return;  // uniform over the work-group
      tile(lg);
    }
  }
}

// Parts 1.. of the split groups into the M2L result: one wave per (split
// group, target of its tile), the lanes along the target's row (the same
// decoding as the M2L kernel); each sum is part 0 + part 1 + ..., in that
// order.
template <bool AD>
__global__ __launch_bounds__(64) void k_m2l_add_half(m2l::Args a, int nc, const float* __restrict__ half_out,
                                                     float* __restrict__ out) {
  const int64_t per_xcd = (a.ngroups + 7) / 8;
  const int64_t sidx = blockIdx.x / m2l::kTargetsPerGroup;
  const int tix = (int)(blockIdx.x % m2l::kTargetsPerGroup);
  const int64_t xcd = sidx / a.ksplit, j = sidx % a.ksplit;
  m2l::TileT<AD, true> tl;
  if (!tl.locate(a, xcd * per_xcd + per_xcd - a.ksplit + j, tix) || !tl.col_ok) return;
  float* o = out + (tl.lvl_off + tl.target_slot(a)) * nc;
  for (int r = threadIdx.x; r < nc; r += 64) {
    float v = o[r];
    for (int q = 1; q < kM2lParts; ++q)
      v += half_out[((sidx * (kM2lParts - 1) + q - 1) * m2l::kTargetsPerGroup + tix) * nc + r];
    o[r] = v;
  }
}

// Work decomposition of the split M2L: the last kM2lSplitPerXcd groups of
// every XCD (fewer when an XCD has fewer) run in kM2lParts parts.  Measured at 2^20 charges, depth 6, p 8 (2,352 groups,
// about 9.2 rounds of the 256 CUs): the nearly empty last round cost 0.36 ms
// of 4.0; two halves took the pass to 3.80 ms.
m2l::Args split_args(fmm_plan_s* Pl) {
  m2l::Args a = m2l::make_args(Pl);
  const int64_t per_xcd = (a.ngroups + 7) / 8;
  a.ksplit = per_xcd < Pl->m2l_split ? per_xcd : Pl->m2l_split;
  return a;
}

void add_halves(fmm_plan_s* Pl, const m2l::Args& a, hipStream_t s) {
  if (a.ksplit == 0) return;
  const unsigned grid = (unsigned)(8 * a.ksplit * m2l::kTargetsPerGroup);
  if (Pl->adaptive)
    k_m2l_add_half<true><<<grid, 64, 0, s>>>(a, Pl->nc, wsp<float>(Pl, Pl->lay.m2l_half),
                                             wsp<float>(Pl, Pl->lay.m2l_out));
  else
    k_m2l_add_half<false><<<grid, 64, 0, s>>>(a, Pl->nc, wsp<float>(Pl, Pl->lay.m2l_half),
                                              wsp<float>(Pl, Pl->lay.m2l_out));
}

template <int P>
struct M2LBfRun {
  template <int NP>
  static hipError_t go(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    const int nc = Pl->nc, kst = m2lb_ksteps(nc);
    // split the multipoles of levels 2..L (levels 0, 1 have no M2L)
    const int64_t box0 = exp_box0(Pl), nbox = exp_nbox(Pl) - box0;
    u32x4* mq = wsp<u32x4>(Pl, lay.multb);
    const int qr = m2lb_row_quads(nc, NP);
    prof_begin(Pl, FMM_PHASE_SPLIT, s);
    k_split_mult<NP><<<grid_for(nbox * kst * 4, kBlock), kBlock, 0, s>>>(
        wsp<float>(Pl, lay.mult32) + box0 * mstride(Pl->p), mstride(Pl->p), nc, kst, nbox,
        mq + box0 * qr);
    prof_end(Pl, s);
    const m2l::Args a = split_args(Pl);
    prof_begin(Pl, FMM_PHASE_M2L, s);
    if (Pl->adaptive)
      k_m2l_bf<P, NP, false, true><<<m2l::grid_of(a), kThreads, 0, s>>>(
          a, mq, wsp<u32x4>(Pl, lay.zero_row), wsp<u32x4>(Pl, lay.op_m2lb), wsp<float>(Pl, lay.m2l_out),
          nullptr, nullptr, wsp<float>(Pl, lay.m2l_half));
    else
      k_m2l_bf<P, NP, false, false><<<m2l::grid_of(a), kThreads, 0, s>>>(
          a, mq, wsp<u32x4>(Pl, lay.zero_row), wsp<u32x4>(Pl, lay.op_m2lb), wsp<float>(Pl, lay.m2l_out),
          nullptr, nullptr, wsp<float>(Pl, lay.m2l_half));
    add_halves(Pl, a, s);
    prof_end(Pl, s);
    return hipGetLastError();
  }
  static hipError_t go_f16(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    const int nc = Pl->nc, kst = m2lb_ksteps(nc);
    const int64_t box0 = exp_box0(Pl), nbox = exp_nbox(Pl) - box0;
    u32x4* mq = wsp<u32x4>(Pl, lay.multb);
    uint32_t* lmax = wsp<uint32_t>(Pl, lay.f16_lmax);
    const int lpb = 4 * kst <= 16 ? 16 : 32;
    // boxes of levels 2..L (adaptive: 2..deepest) and the level-max work-groups
    LevelBlocks lb;
    lb.l0 = 2;
    lb.l1 = Pl->adaptive ? Pl->Ld : Pl->L;
    int64_t nblk = 0;
    for (int l = lb.l0; l <= lb.l1 + 1; ++l) {
      lb.box_off[l] = Pl->adaptive ? Pl->ce_off[l] : lay.lvl_off[l];
      lb.blk_off[l] = nblk;
      if (l <= lb.l1) {
        const int64_t nb = (Pl->adaptive ? Pl->ce_off[l + 1] : lay.lvl_off[l + 1]) - lb.box_off[l];
        const int64_t n4 = nb * mstride(Pl->p) / 4;
        nblk += std::min<int64_t>((n4 + kBlock - 1) / kBlock, kLevelMaxGroups);
      }
    }
    prof_begin(Pl, FMM_PHASE_SPLIT, s);
    hipError_t e = fill_u32(lmax, FMM_DEPTH_MAX + 2, 0u, s);
    if (e != hipSuccess) return e;
    if (nblk > 0) {
      k_f16_level_max<<<(unsigned)nblk, kBlock, 0, s>>>(wsp<float>(Pl, lay.mult32), mstride(Pl->p), nc,
                                                        wsp<float>(Pl, lay.f16_colf), lb, lmax);
      k_split_mult_h<<<grid_for(nbox * lpb, kBlock), kBlock, 0, s>>>(
          wsp<float>(Pl, lay.mult32), mstride(Pl->p), nc, kst, lpb, wsp<float>(Pl, lay.f16_colf), lb,
          lmax, mq);
    }
    prof_end(Pl, s);
    const m2l::Args a = split_args(Pl);
    prof_begin(Pl, FMM_PHASE_M2L, s);
    if constexpr (m2l_f16_wide(P)) {
      if (Pl->m2l_persistent) {
        // two resident work-groups per CU, whole tiles from per-XCD counters
        const m2l::Args ap = m2l::make_args(Pl);
        uint32_t* ticket = wsp<uint32_t>(Pl, lay.m2l_ctl);
        e = fill_u32(ticket, 8, 0u, s);
        if (e != hipSuccess) return e;
        const unsigned grid = 2 * 256;
        if (Pl->adaptive)
          k_m2l_w<P, true, true><<<grid, kWideThreads, 0, s>>>(
              ap, mq, wsp<u32x4>(Pl, lay.zero_row), wsp<u32x4>(Pl, lay.op_m2lb), wsp<float>(Pl, lay.m2l_out),
              lmax, wsp<float>(Pl, lay.f16_rowf), nullptr, ticket);
        else
          k_m2l_w<P, false, true><<<grid, kWideThreads, 0, s>>>(
              ap, mq, wsp<u32x4>(Pl, lay.zero_row), wsp<u32x4>(Pl, lay.op_m2lb), wsp<float>(Pl, lay.m2l_out),
              lmax, wsp<float>(Pl, lay.f16_rowf), nullptr, ticket);
        prof_end(Pl, s);
        return hipGetLastError();
      }
      if (Pl->adaptive)
        k_m2l_w<P, true, false><<<m2l::grid_of(a), kWideThreads, 0, s>>>(
            a, mq, wsp<u32x4>(Pl, lay.zero_row), wsp<u32x4>(Pl, lay.op_m2lb), wsp<float>(Pl, lay.m2l_out),
            lmax, wsp<float>(Pl, lay.f16_rowf), wsp<float>(Pl, lay.m2l_half), nullptr);
      else
        k_m2l_w<P, false, false><<<m2l::grid_of(a), kWideThreads, 0, s>>>(
            a, mq, wsp<u32x4>(Pl, lay.zero_row), wsp<u32x4>(Pl, lay.op_m2lb), wsp<float>(Pl, lay.m2l_out),
            lmax, wsp<float>(Pl, lay.f16_rowf), wsp<float>(Pl, lay.m2l_half), nullptr);
    } else if (Pl->adaptive)
      k_m2l_bf<P, 2, true, true><<<m2l::grid_of(a), kThreads, 0, s>>>(
          a, mq, wsp<u32x4>(Pl, lay.zero_row), wsp<u32x4>(Pl, lay.op_m2lb), wsp<float>(Pl, lay.m2l_out),
          lmax, wsp<float>(Pl, lay.f16_rowf), wsp<float>(Pl, lay.m2l_half));
    else
      k_m2l_bf<P, 2, true, false><<<m2l::grid_of(a), kThreads, 0, s>>>(
          a, mq, wsp<u32x4>(Pl, lay.zero_row), wsp<u32x4>(Pl, lay.op_m2lb), wsp<float>(Pl, lay.m2l_out),
          lmax, wsp<float>(Pl, lay.f16_rowf), wsp<float>(Pl, lay.m2l_half));
    add_halves(Pl, a, s);
    prof_end(Pl, s);
    return hipGetLastError();
  }
  static hipError_t run(fmm_plan_s* Pl, hipStream_t s) {
    if (Pl->m2l_f16) return go_f16(Pl, s);
    return Pl->m2l_np == 2 ? go<2>(Pl, s) : go<3>(Pl, s);
  }
};

}  // namespace

hipError_t launch_m2l_bf16(fmm_plan_s* P, hipStream_t s) { return dispatch_p<M2LBfRun>(P->p, P, s); }

}  // namespace fmm
