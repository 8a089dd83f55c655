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
//  * A operand (operator rows): T_d is stored [row][k] with an odd stride in
//    16-byte quads and staged in LDS (double-buffered across offsets: the next
//    operator's global loads are in flight while the current one feeds the
//    MFMAs); one ds_read_b128 gives a lane its V values of a 16-row block, and
//    the reads of chunk q+1 are issued before the MFMAs of chunk q.  All 128
//    targets share each staged operator.
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
#include "fmm_internal.h"

namespace fmm {
namespace {

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
};

constexpr int kWaves = 8;  // waves per work-group
constexpr int kThreads = kWaves * 64;
constexpr int kTargetsPerGroup = kWaves * 16;
constexpr int kLdsBudget = 150 * 1024;  // two operator buffers

struct M2LArgs {
  int L;
  int64_t lvl_off[FMM_DEPTH_MAX + 2];    // box offsets per level
  int64_t group_off[FMM_DEPTH_MAX + 2];  // first work-group of each level (levels 2..L)
  int64_t ngroups;
  const uint32_t* c2s;
  const uint32_t* s2c;
};

// Static shape of the kernel for order P and type T.
template <int P, typename T>
struct Shape {
  static constexpr int NC = (P + 1) * (P + 1);
  static constexpr int RB = (NC + 15) / 16;    // 16-row blocks
  static constexpr int RP = RB * 16;
  static constexpr int MS = mstride_of(NC);    // multipole row stride
  static constexpr int V = Mfma<T>::V;         // elements per vector
  static constexpr int G = 4 * V;              // k per quad chunk
  static constexpr int NQ = (NC + G - 1) / G;  // quad chunks
  static constexpr int S_LAST = NC - G * (NQ - 1) < V ? NC - G * (NQ - 1) : V;
  static constexpr int KS = m2l_kstride_of(NC, (int)sizeof(T));  // global row stride
  // quad chunks per staged operator chunk: as many as fit two LDS buffers
  static constexpr int fit_nqc(int n) {
    return n <= 1 ? 1 : (2 * RP * V * (4 * n + 1) * (int)sizeof(T) <= kLdsBudget ? n : fit_nqc(n - 1));
  }
  static constexpr int NQC = fit_nqc(NQ);
  static constexpr int NCH = (NQ + NQC - 1) / NQC;  // operator chunks
  static constexpr int KC = G * NQC;                // k per operator chunk
  static constexpr int KCS = V * (4 * NQC + 1);     // LDS row stride (odd quads)
  static constexpr int VPR = KC / V;                // vectors per row per chunk
  static constexpr int NV = RP * VPR;               // vectors per chunk
  static constexpr int PER_THREAD = (NV + kThreads - 1) / kThreads;
  // Prefetch the next offset's B vectors (a second register set) only where
  // the registers allow it without spills.
  static constexpr bool PREFETCH_B = sizeof(T) == 4 ? P <= 10 : P <= 7;
  static_assert(MS % V == 0, "multipole rows must hold whole vectors");
};

template <int P, typename T>
__global__ __launch_bounds__(kThreads) void k_m2l(M2LArgs a, const T* __restrict__ mult,
                                                  const T* __restrict__ zero_row,
                                                  const T* __restrict__ ops,
                                                  T* __restrict__ out) {
  typedef Shape<P, T> S;
  constexpr int NC = S::NC, RB = S::RB, RP = S::RP, MS = S::MS, V = S::V, G = S::G;
  constexpr int NQ = S::NQ, NQC = S::NQC, NCH = S::NCH, KC = S::KC, KCS = S::KCS, KS = S::KS;
  typedef typename Mfma<T>::acc_t acc_t;
  typedef typename Mfma<T>::vec_t vec_t;
  __shared__ __attribute__((aligned(16))) T sT[2][RP * KCS];

  // XCD-aware order: hardware group b runs on XCD b % 8; each XCD gets a
  // contiguous range of logical groups.
  const int64_t per_xcd = (a.ngroups + 7) / 8;
  const int64_t lg = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (lg >= a.ngroups) return;  // uniform over the work-group

  int l = 2;
  while (l < a.L && lg >= a.group_off[l + 1]) ++l;
  const int64_t np = (int64_t)1 << (3 * (l - 1));  // parents at level l-1
  const int64_t ntile = (np + kTargetsPerGroup - 1) / kTargetsPerGroup;
  const int64_t idx = lg - a.group_off[l];
  const int pi = (int)(idx / ntile);
  const int64_t tile = idx % ntile;
  const int px = (pi >> 2) & 1, py = (pi >> 1) & 1, pz = pi & 1;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kg = lane >> 4;
  const int nb = 1 << l;
  const uint32_t* c2s = a.c2s + a.lvl_off[l];
  const T* mlev = mult + a.lvl_off[l] * MS;

  const int64_t ps = tile * kTargetsPerGroup + wave * 16 + col;
  const bool col_ok = ps < np;
  int tx = 0, ty = 0, tz = 0;
  if (col_ok) {
    unpack_coord(a.s2c[a.lvl_off[l - 1] + ps], tx, ty, tz);
    tx = 2 * tx + px;
    ty = 2 * ty + py;
    tz = 2 * tz + pz;
  }

  acc_t sum[RB], comp[RB], acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) sum[r] = comp[r] = acc[r] = acc_t{0, 0, 0, 0};

  // Offsets of the class in a fixed order: d_a in [pi_a - 3, pi_a + 2] with
  // max |d_a| >= 2 (216 candidates, 27 skipped).
  auto offset_of = [&](int j, int& dx, int& dy, int& dz) {
    dx = px - 3 + j / 36;
    dy = py - 3 + (j / 6) % 6;
    dz = pz - 3 + j % 6;
    return !(dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1);
  };
  auto next_offset = [&](int j, int& dx, int& dy, int& dz) {
    ++j;
    while (j < 216 && !offset_of(j, dx, dy, dz)) ++j;
    return j;
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
        const int row = e / S::VPR, kv = e % S::VPR;
        *reinterpret_cast<vec_t*>(buf + row * KCS + kv * V) = reg[i];
      }
    }
  };
  // This lane's source row for offset (dx, dy, dz): the zero row outside the domain.
  auto source_of = [&](int dx, int dy, int dz, bool& ok) -> const T* {
    const int sx = tx - dx, sy = ty - dy, sz = tz - dz;
    ok = col_ok && sx >= 0 && sy >= 0 && sz >= 0 && sx < nb && sy < nb && sz < nb;
    return ok ? mlev + (int64_t)c2s[lex_index(sx, sy, sz, l)] * MS : zero_row;
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
    const T* sa = buf + col * KCS + V * kg;
    vec_t av[2][RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) av[0][r] = *reinterpret_cast<const vec_t*>(sa + 16 * r * KCS);
#pragma unroll
    for (int qc = 0; qc < NQC; ++qc) {
      const int q = ch * NQC + qc;
      if (q >= NQ) break;
      if (qc + 1 < NQC && q + 1 < NQ) {
#pragma unroll
        for (int r = 0; r < RB; ++r)
          av[(qc + 1) & 1][r] = *reinterpret_cast<const vec_t*>(sa + 16 * r * KCS + G * (qc + 1));
      }
      const int ns = (q == NQ - 1) ? S::S_LAST : V;
#pragma unroll
      for (int s = 0; s < V; ++s) {
        if (s >= ns) break;
        const T bv = b[q][s];
#pragma unroll
        for (int r = 0; r < RB; ++r) dst[r] = Mfma<T>::step(av[qc & 1][r][s], bv, dst[r]);
      }
    }
  };

  constexpr bool PB = S::PREFETCH_B;
  vec_t reg[S::PER_THREAD];
  vec_t b0[NQ], b1[PB ? NQ : 1];
  int dx, dy, dz;
  int j = next_offset(-1, dx, dy, dz);
  bool wave_any = false;
  if (PB) {
    bool ok_cur;
    load_b(source_of(dx, dy, dz, ok_cur), b0);
    wave_any = __any(ok_cur);
  }
  stage_load(m2l_op_index(dx, dy, dz), 0, reg);
  stage_store(sT[0], reg);
  __syncthreads();
  int cur = 0;

  // One offset: its NCH operator chunks; stages the next chunk (of this or the
  // next offset) and, at the first chunk, prefetches the next offset's B
  // vectors into bn (or, without prefetch, loads this offset's into bc).
  // Returns false after the last offset.
  auto do_offset = [&](vec_t* bc, vec_t* bn) -> bool {
    int ndx = dx, ndy = dy, ndz = dz;
    const int jn = next_offset(j, ndx, ndy, ndz);
    const bool more = jn < 216;
    bool ok_next = false;
    if (!PB) {
      bool ok_cur;
      load_b(source_of(dx, dy, dz, ok_cur), bc);
      wave_any = __any(ok_cur);
    }
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      const bool last_chunk = ch == NCH - 1;
      if (!last_chunk)
        stage_load(m2l_op_index(dx, dy, dz), ch + 1, reg);
      else if (more)
        stage_load(m2l_op_index(ndx, ndy, ndz), 0, reg);
      if (PB && ch == 0 && more) load_b(source_of(ndx, ndy, ndz, ok_next), bn);
      if (wave_any) compute_chunk(sT[cur], ch, bc);
      if (Mfma<T>::kChain && last_chunk && wave_any) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          Mfma<T>::add(sum[r], comp[r], acc[r]);
          acc[r] = acc_t{0, 0, 0, 0};
        }
      }
      if (last_chunk && !more) return false;
      stage_store(sT[cur ^ 1], reg);
      __syncthreads();
      cur ^= 1;
    }
    j = jn;
    dx = ndx;
    dy = ndy;
    dz = ndz;
    if (PB) wave_any = __any(ok_next);
    return true;
  };
  if (PB) {
    while (do_offset(b0, b1) && do_offset(b1, b0)) {
    }
  } else {
    while (do_offset(b0, b0)) {
    }
  }

  if (!col_ok) return;
  const int64_t ts = c2s[lex_index(tx, ty, tz, l)];
  T* o = out + (a.lvl_off[l] + ts) * NC;
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 16 * r + Mfma<T>::row(kg, i);
      if (row < NC) o[row] = sum[r][i];
    }
}

template <int P>
struct M2LRun {
  static hipError_t run(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    M2LArgs a;
    a.L = Pl->L;
    for (int l = 0; l <= FMM_DEPTH_MAX + 1; ++l) a.lvl_off[l] = lay.lvl_off[l];
    int64_t g = 0;
    for (int l = 2; l <= Pl->L; ++l) {
      a.group_off[l] = g;
      const int64_t np = (int64_t)1 << (3 * (l - 1));
      g += 8 * ((np + kTargetsPerGroup - 1) / kTargetsPerGroup);
    }
    a.group_off[Pl->L + 1] = g;
    a.ngroups = g;
    a.c2s = wsp<uint32_t>(Pl, lay.coord2slot);
    a.s2c = wsp<uint32_t>(Pl, lay.slot2coord);
    const unsigned grid = (unsigned)(((a.ngroups + 7) / 8) * 8);
    if (Pl->mixed)
      k_m2l<P, float><<<grid, kThreads, 0, s>>>(a, wsp<float>(Pl, lay.mult32),
                                               wsp<float>(Pl, lay.zero_row),
                                               wsp<float>(Pl, lay.op_m2l32),
                                               wsp<float>(Pl, lay.m2l_out));
    else
      k_m2l<P, double><<<grid, kThreads, 0, s>>>(a, wsp<double>(Pl, lay.mult64),
                                                wsp<double>(Pl, lay.zero_row),
                                                wsp<double>(Pl, lay.op_m2l64),
                                                wsp<double>(Pl, lay.m2l_out));
    return hipGetLastError();
  }
};

}  // namespace

hipError_t launch_m2l(fmm_plan_s* P, hipStream_t s) {
  prof_begin(P, FMM_PHASE_M2L, s);
  hipError_t e = dispatch_p<M2LRun>(P->p, P, s);
  prof_end(P, s);
  return e;
}

}  // namespace fmm
