// m2l.hip -- multipole-to-local translation on the matrix cores.
//
// For a target box t at level l >= 2 the interaction list is every box s of
// level l whose parent is adjacent to t's parent but which is not adjacent to
// t.  With d = t - s (integer box offset), the list depends only on the
// parity pi of t's coordinates: d_a ranges over [pi_a - 3, pi_a + 2] with
// max |d_a| >= 2, 189 offsets per parity class.  Each offset has one unit-box
// operator T_d (316 in all), so the M2L of a level is, per parity class and
// offset, a dense product
//     L~[:, targets] += T_d (NC x NC) * M~[:, targets - d]   (times 1/h later)
// accumulated over the 189 offsets of the class in a fixed order.
//
// Mapping.  One work-group owns 128 targets of one parity class at one level
// (the parity-pi children of 128 consecutive parent slots in Hilbert order);
// each of its 8 waves owns 16 of them and keeps their NC-row local expansions
// in MFMA accumulators (16x16x4) for the whole offset loop.
//  * K order: lane group g at sub-step s of k-quad chunk q works on
//    k = 4V q + V g + s (V elements per 16-byte vector), so each lane's A and B
//    values for a chunk are one 16-byte vector each.
//  * A operand (operator rows): T_d is stored [row][k] and staged in LDS
//    (double-buffered across offsets: the next operator's global loads are in
//    flight while the current one feeds the MFMAs) in a row layout free of
//    LDS bank conflicts (see Shape); one ds_read_b128 gives a lane its V
//    values of a 16-row block, and the reads of chunk q+1 are issued before
//    the MFMAs of chunk q.  All 128 targets share each staged operator.
//  * B operand (source coefficients): 16-byte vectors from global memory; a
//    whole offset's vectors are prefetched while the previous offset's MFMAs
//    run (two register sets used alternately) where the registers allow.
//    Sources outside the domain read a zero row.  All loads are unconditional
//    (clamped addresses) so the waits on them are exact.
//  * FP32: each offset's product is a fresh MFMA chain and the chains are
//    summed across offsets with Kahan compensation (one FP32 chain over all
//    189 x NC/4 steps loses about 4x more accuracy).  FP64: one chain.
// FP64 MFMA in the FP64 mode, FP32 MFMA in the mixed mode.  Offsets with no
// source inside the domain for any of a wave's 16 targets skip their MFMAs.
// Work-groups are assigned to XCDs in contiguous ranges so that neighbouring
// tiles (which share operators and sources) share an L2.
#include "m2l_common.h"

namespace fmm {
namespace {

using m2l::kThreads;
using m2l::kWaves;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Mfma;
// Accumulator lane layout (measured on gfx950): lane l holds column l % 16;
// its four values are rows 4 (l / 16) + i for the f32 form and (l / 16) + 4 i
// for the f64 form.
template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  typedef f32x4 vec_t;  // one 16-byte vector
  static constexpr int V = 4;
  static constexpr bool kChain = true;  // per-offset chains, compensated sum
  static __device__ __forceinline__ int row(int kg, int i) { return 4 * kg + i; }
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void add(acc_t& sum, acc_t& comp, acc_t v) {
    const acc_t y = v - comp;
    const acc_t t = sum + y;
    comp = (t - sum) - y;
    sum = t;
  }
  static __device__ __forceinline__ void add1(float& sum, float& comp, float v) {
    const float y = v - comp;
    const float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
  }
};
template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  typedef f64x2 vec_t;
  static constexpr int V = 2;
  static constexpr bool kChain = false;  // one FP64 chain over all offsets
  static __device__ __forceinline__ int row(int kg, int i) { return kg + 4 * i; }
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void add(acc_t& sum, acc_t&, acc_t v) { sum += v; }
  static __device__ __forceinline__ void add1(double& sum, double&, double v) { sum += v; }
};

constexpr int kLdsBudget = 140 * 1024;  // two operator buffers (plus the slot halo)


// Static shape of the kernel for order P and type T.
template <int P, typename T>
struct Shape {
  static constexpr int NC = (P + 1) * (P + 1);
  static constexpr int RB = (NC + 15) / 16;    // 16-row blocks
  static constexpr int RP = RB * 16;
  // NC = 16 RBM + 1 (p = 6, 8): the last row is a per-lane dot product on the
  // vector ALU instead of a 16-row MFMA block holding one real row.
  static constexpr bool TAIL = NC % 16 == 1 && NC > 16;
  static constexpr int RBM = TAIL ? RB - 1 : RB;  // MFMA row blocks
  static constexpr int ROWS = TAIL ? NC : RP;     // operator rows staged in LDS
  static constexpr int MS = mstride_of(NC);    // multipole row stride
  static constexpr int V = Mfma<T>::V;         // elements per vector
  static constexpr int G = 4 * V;              // k per quad chunk
  static constexpr int NQ = (NC + G - 1) / G;  // quad chunks
  static constexpr int S_LAST = NC - G * (NQ - 1) < V ? NC - G * (NQ - 1) : V;
  static constexpr int KS = m2l_kstride_of(NC, (int)sizeof(T));  // global row stride
  // quad chunks per staged operator chunk: as many as fit two LDS buffers
  // LDS row layout of a staged chunk of n quad chunks, in 16-byte vectors.
  // A 16-byte LDS read serves 32 lanes at a time and is free of bank
  // conflicts when their vectors are distinct modulo 32.
  //  * Conflict-free form: [g][quad chunk], the 4 lane groups g GQ vectors
  //    apart (GQ odd) and rows 4 GQ + 2 apart: 16 rows at a stride of 2 mod 4
  //    fill the even residues, the odd g offset the odd ones.
  //  * Compact form, where the first needs more operator chunks: [quad
  //    chunk][g], rows 4 n + 1 apart (adjacent lane groups share banks).
  static constexpr int gq_of(int n) { return n | 1; }
  static constexpr int row_cf(int n) { return 4 * gq_of(n) + 2; }
  static constexpr int row_compact(int n) { return 4 * n + 1; }
  static constexpr int fit_cf(int n) {
    return n <= 1 ? 1 : (2 * ROWS * row_cf(n) * 16 <= kLdsBudget ? n : fit_cf(n - 1));
  }
  static constexpr int fit_compact(int n) {
    return n <= 1 ? 1 : (2 * ROWS * row_compact(n) * 16 <= kLdsBudget ? n : fit_compact(n - 1));
  }
  static constexpr bool CF = fit_cf(NQ) == fit_compact(NQ);
  static constexpr int fit_nqc(int n) { return CF ? fit_cf(n) : fit_compact(n); }
  static constexpr int NQC = fit_nqc(NQ);
  static constexpr int NCH = (NQ + NQC - 1) / NQC;  // operator chunks
  static constexpr int KC = G * NQC;                // k per operator chunk
  static constexpr int GOFF = CF ? gq_of(NQC) : 1;  // vectors between lane groups
  static constexpr int QOFF = CF ? 1 : 4;            // vectors between quad chunks
  static constexpr int KCS = V * (CF ? row_cf(NQC) : row_compact(NQC));  // LDS row stride
  static constexpr int VPR = KC / V;                // vectors per row per chunk
  static constexpr int NV = ROWS * VPR;             // vectors per chunk
  static constexpr int PER_THREAD = (NV + kThreads - 1) / kThreads;
  // Prefetch the next offset's B vectors (a second register set) only where
  // the registers allow it without spills.
  static constexpr bool PREFETCH_B = P <= (sizeof(T) == 4 ? 8 : 7);
  static_assert(MS % V == 0, "multipole rows must hold whole vectors");
};

template <int P, typename T, bool AD>
__global__ __launch_bounds__(kThreads) void k_m2l(m2l::Args a, const T* __restrict__ mult,
                                                  const T* __restrict__ zero_row,
                                                  const T* __restrict__ ops,
                                                  T* __restrict__ out) {
  typedef Shape<P, T> S;
  constexpr int NC = S::NC, RB = S::RB, RP = S::RP, MS = S::MS, V = S::V, G = S::G;
  constexpr int NQ = S::NQ, NQC = S::NQC, NCH = S::NCH, KC = S::KC, KCS = S::KCS, KS = S::KS;
  constexpr int RBM = S::RBM;
  constexpr bool TAIL = S::TAIL;
  typedef typename Mfma<T>::acc_t acc_t;
  typedef typename Mfma<T>::vec_t vec_t;
  __shared__ __attribute__((aligned(16))) T sT[2][S::ROWS * KCS];
  __shared__ uint32_t sSlot[m2l::kHalo];
  __shared__ int sBox[6];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kg = lane >> 4;
  m2l::TileT<AD> tl;
  if (!tl.setup(a, wave * 16 + col, sSlot, sBox)) return;  // uniform over the work-group
  const int pi = tl.pi;
  const bool col_ok = tl.col_ok;
  const T* mlev = mult + tl.lvl_off * MS;

  acc_t sum[RBM], comp[RBM], acc[RBM];
#pragma unroll
  for (int r = 0; r < RBM; ++r) sum[r] = comp[r] = acc[r] = acc_t{0, 0, 0, 0};
  // Tail row (TAIL): this lane's partial sum over its k values.
  T tsum = T(0), tcomp = T(0), tacc = T(0);

  auto offset_of = [&](int i, int& dx, int& dy, int& dz) {
    return m2l::il_offset(pi, i, dx, dy, dz);
  };
  // Operator chunk ch of operator op into registers / into an LDS buffer.
  // Vector e of a chunk is row e / VPR, k-vector e % VPR; loads are clamped
  // so that every lane issues the same loads.
  auto stage_load = [&](int op, int ch, vec_t* reg) {
    const T* base = ops + (size_t)op * RP * KS + ch * KC;
#pragma unroll
    for (int i = 0; i < S::PER_THREAD; ++i) {
      int e = tid + i * kThreads;
      e = e < S::NV ? e : S::NV - 1;
      const int row = e / S::VPR, kv = e % S::VPR;
      const int k = ch * KC + kv * V;
      // vectors past the operator's stored width (last chunk) read its last vector
      const int kk = k + V <= KS ? kv * V : KS - V - ch * KC;
      reg[i] = *reinterpret_cast<const vec_t*>(base + (size_t)row * KS + kk);
    }
  };
  auto stage_store = [&](T* buf, const vec_t* reg) {
#pragma unroll
    for (int i = 0; i < S::PER_THREAD; ++i) {
      const int e = tid + i * kThreads;
      if (e < S::NV) {
        const int row = e / S::VPR, kv = e % S::VPR;  // kv = 4 (quad chunk) + g
        *reinterpret_cast<vec_t*>(buf + row * KCS + ((kv % 4) * S::GOFF + (kv / 4) * S::QOFF) * V) =
            reg[i];
      }
    }
  };
  typedef m2l::Src Src;
  auto lookup = [&](int k, int dx, int dy, int dz) -> Src { return tl.lookup(sSlot, k, dx, dy, dz); };
  // Source row of a lookup: the zero row outside the domain.
  auto row_of = [&](Src src) -> const T* {
    return src.ok ? mlev + (int64_t)src.slot * MS : zero_row;
  };
  // B vectors of a source row; k-quads past the row read its last vector
  // (they meet zero operator columns).
  auto load_b = [&](const T* ms, vec_t* b) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      int k0 = G * q + V * kg;
      k0 = k0 + V <= MS ? k0 : MS - V;
      b[q] = *reinterpret_cast<const vec_t*>(ms + k0);
    }
  };
  // MFMAs of operator chunk ch (staged in buf) against B vectors b.
  auto compute_chunk = [&](const T* buf, int ch, const vec_t* b) {
    acc_t* dst = Mfma<T>::kChain ? acc : sum;
    T& tdst = Mfma<T>::kChain ? tacc : tsum;
    const T* sa = buf + col * KCS + V * S::GOFF * kg;
    const T* st = buf + (NC - 1) * KCS + V * S::GOFF * kg;  // tail row (same for all 16 columns)
    vec_t av[2][RBM], at[2];
#pragma unroll
    for (int r = 0; r < RBM; ++r) av[0][r] = *reinterpret_cast<const vec_t*>(sa + 16 * r * KCS);
    if (TAIL) at[0] = *reinterpret_cast<const vec_t*>(st);
#pragma unroll
    for (int qc = 0; qc < NQC; ++qc) {
      const int q = ch * NQC + qc;
      if (q >= NQ) break;
      if (qc + 1 < NQC && q + 1 < NQ) {
#pragma unroll
        for (int r = 0; r < RBM; ++r)
          av[(qc + 1) & 1][r] =
              *reinterpret_cast<const vec_t*>(sa + 16 * r * KCS + V * S::QOFF * (qc + 1));
        if (TAIL) at[(qc + 1) & 1] = *reinterpret_cast<const vec_t*>(st + V * S::QOFF * (qc + 1));
      }
      const int ns = (q == NQ - 1) ? S::S_LAST : V;
#pragma unroll
      for (int s = 0; s < V; ++s) {
        if (s >= ns) break;
        const T bv = b[q][s];
#pragma unroll
        for (int r = 0; r < RBM; ++r) dst[r] = Mfma<T>::step(av[qc & 1][r][s], bv, dst[r]);
        if (TAIL) tdst = fma(at[qc & 1][s], bv, tdst);
      }
    }
  };

  constexpr bool PB = S::PREFETCH_B;
  vec_t reg[S::PER_THREAD];
  vec_t b0[NQ], b1[PB ? NQ : 1];
  // Pipeline over the class's offsets: offset i is computed while the
  // operator of the next stage and the B vectors of offset i + 1 are loaded
  // and the source slot of offset i + 2 is looked up.
  int i = 0, dx, dy, dz, ndx, ndy, ndz;
  int op = offset_of(0, dx, dy, dz);
  int nop = offset_of(1, ndx, ndy, ndz);
  Src s_cur = lookup(0, dx, dy, dz);
  Src s_next = lookup(1, ndx, ndy, ndz);
  bool wave_any = false;
  if (PB) {
    load_b(row_of(s_cur), b0);
    wave_any = __any(s_cur.ok);
  }
  stage_load(op, 0, reg);
  stage_store(sT[0], reg);
  __syncthreads();
  int cur = 0;

  // One offset: its NCH operator chunks; stages the next chunk (of this or the
  // next offset) and, at the first chunk, prefetches the next offset's B
  // vectors into bn (or, without prefetch, loads this offset's into bc).
  // Returns false after the last offset.
  auto do_offset = [&](vec_t* bc, vec_t* bn) -> bool {
    const bool more = i + 1 < kIL;
    int fdx, fdy, fdz;
    const int fi = i + 2 < kIL ? i + 2 : kIL - 1;
    const int fop = offset_of(fi, fdx, fdy, fdz);
    const Src s_far = lookup(fi, fdx, fdy, fdz);  // offset i + 2 (clamped at the end)
    if (!PB) {
      load_b(row_of(s_cur), bc);
      wave_any = __any(s_cur.ok);
    }
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const bool last_chunk = ch == NCH - 1;
      stage_load(last_chunk ? (more ? nop : op) : op, last_chunk ? 0 : ch + 1, reg);
      if (PB && ch == 0) load_b(row_of(s_next), bn);
      if (wave_any) compute_chunk(sT[cur], ch, bc);
      if (Mfma<T>::kChain && last_chunk && wave_any) {
#pragma unroll
        for (int r = 0; r < RBM; ++r) {
          Mfma<T>::add(sum[r], comp[r], acc[r]);
          acc[r] = acc_t{0, 0, 0, 0};
        }
        if (TAIL) {
          Mfma<T>::add1(tsum, tcomp, tacc);
          tacc = T(0);
        }
      }
      if (last_chunk && !more) return false;
      stage_store(sT[cur ^ 1], reg);
      m2l::lds_barrier();
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

  // Tail row: combine the four lane groups' partials (fixed order; all lanes
  // take part in the shuffles).
  T tail = T(0);
  if (TAIL) {
    tail = tsum - tcomp;
    tail += __shfl_xor(tail, 16);
    tail += __shfl_xor(tail, 32);
  }
  if (!col_ok) return;
  T* o = out + (tl.lvl_off + tl.target_slot(a)) * NC;
#pragma unroll
  for (int r = 0; r < RBM; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 16 * r + Mfma<T>::row(kg, i);
      if (row < NC) o[row] = sum[r][i];
    }
  if (TAIL && kg == 0) o[NC - 1] = tail;
}

template <int P>
struct M2LRun {
  static hipError_t run(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    const m2l::Args a = m2l::make_args(Pl);
    const unsigned grid = m2l::grid_of(a);
    if (Pl->mixed)
      go<float>(Pl, a, grid, wsp<float>(Pl, lay.mult32), wsp<float>(Pl, lay.zero_row),
                wsp<float>(Pl, lay.op_m2l32), wsp<float>(Pl, lay.m2l_out), s);
    else
      go<double>(Pl, a, grid, wsp<double>(Pl, lay.mult64), wsp<double>(Pl, lay.zero_row),
                 wsp<double>(Pl, lay.op_m2l64), wsp<double>(Pl, lay.m2l_out), s);
    return hipGetLastError();
  }
  template <typename T>
  static void go(fmm_plan_s* Pl, const m2l::Args& a, unsigned grid, const T* mult, const T* zero,
                 const T* ops, T* out, hipStream_t s) {
    if (Pl->adaptive)
      k_m2l<P, T, true><<<grid, kThreads, 0, s>>>(a, mult, zero, ops, out);
    else
      k_m2l<P, T, false><<<grid, kThreads, 0, s>>>(a, mult, zero, ops, out);
  }
};

}  // namespace

hipError_t launch_m2l(fmm_plan_s* P, hipStream_t s) {
  if (P->m2l_np) return launch_m2l_bf16(P, s);  // times its split and M2L kernels apart
  prof_begin(P, FMM_PHASE_M2L, s);
  hipError_t e = dispatch_p<M2LRun>(P->p, P, s);
  prof_end(P, s);
  return e;
}

}  // namespace fmm
