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
constexpr int kFlush = M2LB_FLUSH;
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

// FP16 form: every box's FP32 multipole row times the column factors colf_k,
// scaled by a power of two 2^s_b so that its largest entry lies in
// [2^13, 2^14), split into 2 FP16 pieces; mscale_b = 2^-s_b.  lpb (16 or 32)
// lanes per box, lane u holding k = 8 u .. 8 u + 7 (quad (ks * 2 + piece) * 4 + g,
// u = 4 ks + g).
__global__ void k_split_mult_h(const float* __restrict__ m32, int ms, int nc, int kst, int64_t nbox,
                               int lpb, const float* __restrict__ colf, u32x4* __restrict__ out,
                               float* __restrict__ mscale) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t box = t / lpb;
  const int u = (int)(t % lpb);
  const bool live = box < nbox && u < 4 * kst;
  float v[8];
  float m = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 8 * u + j;
    v[j] = (live && k < nc) ? m32[box * ms + k] * colf[k] : 0.f;
    m = fmaxf(m, fabsf(v[j]));
  }
#pragma unroll
  for (int w = 16; w >= 1; w >>= 1)
    if (w < lpb) m = fmaxf(m, __shfl_xor(m, w, lpb));  // box max
  int e = 0;
  if (m > 0.f) frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
  if (!live) return;
  uint32_t pc[8][2];
#pragma unroll
  for (int j = 0; j < 8; ++j) split_f16_f32(ldexpf(v[j], 14 - e), pc[j]);
  u32x4 q[2];
  pack_quads<2>(pc, q);
  u32x4* o = out + box * (kst * 2 * 4);
  const int ks = u / 4, g = u % 4;
  o[(ks * 2 + 0) * 4 + g] = q[0];
  o[(ks * 2 + 1) * 4 + g] = q[1];
  if (u == 0) mscale[box] = ldexpf(1.f, e - 14);
}

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
  static constexpr int RGW = F16 ? (KST >= 6 ? 1 : 6) : (KST >= 5 ? 1 : M2LB_RG);
  static constexpr int RG = RB < RGW ? RB : RGW;
  // Prefetch the next offset's B quads (a second register set) up to 3 k
  // steps (p <= 8).  From 4 on (p = 9, 10) the second set made the compiler
  // spill (84-112 bytes per lane), and the adaptive p = 10 M2L took 10.3 ms
  // instead of 6.3 ms without it.
  static constexpr bool PREFETCH_B = KST <= 3;
};

// F16: FP16 pieces of scaled operands (FMM_M2L_F16X2): per-offset FP32 chains
// times the source box's inverse scale, summed in two levels (partials of
// kGroupF16 offsets), rows times rowf at the end.
template <int P, int NP, bool F16, bool AD>
__global__ __launch_bounds__(kThreads) void k_m2l_bf(m2l::Args a, const u32x4* __restrict__ multq,
                                                     const u32x4* __restrict__ zero_q,
                                                     const u32x4* __restrict__ ops,
                                                     float* __restrict__ out,
                                                     const float* __restrict__ mscale,
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
            if (r0 + rr < RB) av[rr][i] = sa[16 * (r0 + rr) * QCS + kc * NP + i];
#pragma unroll
        for (int t = 0; t < PR::N; ++t)
#pragma unroll
          for (int rr = 0; rr < RG; ++rr)
            if (r0 + rr < RB) {
              if (F16)
                acc[r0 + rr] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                    __builtin_bit_cast(f16x8, av[rr][PR::a[t]]),
                    __builtin_bit_cast(f16x8, b[ks * NP + PR::b[t]]), acc[r0 + rr], 0, 0, 0);
              else
                acc[r0 + rr] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, av[rr][PR::a[t]]),
                    __builtin_bit_cast(bf16x8, b[ks * NP + PR::b[t]]), acc[r0 + rr], 0, 0, 0);
            }
      }
    }
  };

  constexpr bool PB = S::PREFETCH_B;
  constexpr int FLUSH = F16 ? 1 : kFlush;  // FP16: each offset has its own source scale
  u32x4 reg[S::PER_THREAD];
  u32x4 b0[KST * NP], b1[PB ? KST * NP : 1];
  // source box scale (FP16 form): of the current and of the next offset
  auto scale_of = [&](m2l::Src src) -> float { return F16 && src.ok ? mscale[tl.lvl_off + src.slot] : 1.f; };
  // Pipeline over the class's offsets: offset i is computed while the
  // operator of the next stage and the B quads of offset i + 1 are loaded and
  // the source slot of offset i + 2 is looked up.
  int i = i0, dx, dy, dz, ndx, ndy, ndz;
  int op = m2l::il_offset(pi, i0, dx, dy, dz);
  int nop = m2l::il_offset(pi, i0 + 1, ndx, ndy, ndz);
  m2l::Src s_cur = tl.lookup(sSlot, i0, dx, dy, dz);
  m2l::Src s_next = tl.lookup(sSlot, i0 + 1, ndx, ndy, ndz);
  bool wave_any = false;
  float sc_cur = scale_of(s_cur), sc_next = 0.f;
  if (PB) {
    load_b(row_of(s_cur), b0);
    wave_any = __any(s_cur.ok);
  }
  stage_load(op, 0, reg);
  stage_store(sT[0], reg);
  __syncthreads();
  int cur = 0;

  auto do_offset = [&](u32x4* bc, u32x4* bn) -> bool {
    const bool more = i + 1 < i1;
    int fdx, fdy, fdz;
    const int fi = i + 2 < i1 ? i + 2 : i1 - 1;
    const int fop = m2l::il_offset(pi, fi, fdx, fdy, fdz);
    const m2l::Src s_far = tl.lookup(sSlot, fi, fdx, fdy, fdz);
    if (!PB) {
      load_b(row_of(s_cur), bc);
      wave_any = __any(s_cur.ok);
    }
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const bool last_chunk = ch == NCH - 1;
      stage_load(last_chunk ? (more ? nop : op) : op, last_chunk ? 0 : ch + 1, reg);
      if (PB && ch == 0) {
        load_b(row_of(s_next), bn);
        sc_next = scale_of(s_next);
      }
      if (wave_any) compute_chunk(sT[cur], ch, bc);
      if (F16 && last_chunk) {
        // each offset's chain times its source scale into an FP32 partial
        // (fused, exact scaling), the partial into the sum every kGroupF16
        // offsets (emulated at the headline size: 1.9e-7 of phi from the M2L
        // rounding, against 1.35e-7 with Kahan after every offset)
        if (wave_any) {
#pragma unroll
          for (int r = 0; r < RB; ++r) {
#pragma unroll
            for (int e = 0; e < 4; ++e) comp[r][e] = fmaf(acc[r][e], sc_cur, comp[r][e]);
            acc[r] = f32x4{0, 0, 0, 0};
          }
        }
        if ((i + 1 - i0) % kGroupF16 == 0 || !more) {
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            sum[r] += comp[r];
            comp[r] = f32x4{0, 0, 0, 0};
          }
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
      stage_store(sT[cur ^ 1], reg);
      __syncthreads();
      cur ^= 1;
    }
    ++i;
    op = nop;
    dx = ndx;
    dy = ndy;
    dz = ndz;
    nop = fop;
    ndx = fdx;
    ndy = fdy;
    ndz = fdz;
    if (PB) wave_any = __any(s_next.ok);
    sc_cur = PB ? sc_next : scale_of(s_next);
    s_cur = s_next;
    s_next = s_far;
    return true;
  };
  if (PB) {
    while (do_offset(b0, b1) && do_offset(b1, b0)) {
    }
  } else {
    while (do_offset(b0, b0)) {
    }
  }

  if (!tl.col_ok) return;
  // parts 1.. of a split group: into their slots of half_out, added to part
  // 0's result by k_m2l_add_half after the launch
  float* o = !whole && tl.part > 0
                 ? half_out + ((tl.sidx * (kM2lParts - 1) + tl.part - 1) * m2l::kTargetsPerGroup + wave * 16 + col) * NC
                 : out + (tl.lvl_off + tl.target_slot(a)) * NC;
  // Accumulator layout of the 16x16 FP32-output MFMAs: lane l holds column
  // l % 16, rows 4 (l / 16) + i.
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * r + 4 * kg + e;
      if (row < NC) o[row] = F16 ? sum[r][e] * rowf[row] : sum[r][e];
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
  a.ksplit = per_xcd < kM2lSplitPerXcd ? per_xcd : kM2lSplitPerXcd;
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
    const int qr = m2lb_row_quads(nc, 2);
    float* msc = wsp<float>(Pl, lay.f16_mscale);
    const int lpb = 4 * kst <= 16 ? 16 : 32;
    prof_begin(Pl, FMM_PHASE_SPLIT, s);
    k_split_mult_h<<<grid_for(nbox * lpb, kBlock), kBlock, 0, s>>>(
        wsp<float>(Pl, lay.mult32) + box0 * mstride(Pl->p), mstride(Pl->p), nc, kst, nbox, lpb,
        wsp<float>(Pl, lay.f16_colf), mq + box0 * qr, msc + box0);
    prof_end(Pl, s);
    const m2l::Args a = split_args(Pl);
    prof_begin(Pl, FMM_PHASE_M2L, s);
    if (Pl->adaptive)
      k_m2l_bf<P, 2, true, true><<<m2l::grid_of(a), kThreads, 0, s>>>(
          a, mq, wsp<u32x4>(Pl, lay.zero_row), wsp<u32x4>(Pl, lay.op_m2lb), wsp<float>(Pl, lay.m2l_out),
          msc, wsp<float>(Pl, lay.f16_rowf), wsp<float>(Pl, lay.m2l_half));
    else
      k_m2l_bf<P, 2, true, false><<<m2l::grid_of(a), kThreads, 0, s>>>(
          a, mq, wsp<u32x4>(Pl, lay.zero_row), wsp<u32x4>(Pl, lay.op_m2lb), wsp<float>(Pl, lay.m2l_out),
          msc, wsp<float>(Pl, lay.f16_rowf), wsp<float>(Pl, lay.m2l_half));
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
