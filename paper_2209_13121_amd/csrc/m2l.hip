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
// in MFMA accumulators for the whole offset loop.
//  * A operand (operator rows): T_d is staged in LDS, in chunks of k-rows,
//    double-buffered so the next chunk's global loads are in flight while the
//    current one feeds the MFMAs; all 128 targets share each staged operator.
//  * B operand (source coefficients): each lane loads its source's
//    coefficients as 16-byte vectors.  The K order of the MFMA steps is
//    permuted so that lane group g at sub-step s of vector chunk q uses
//    k = 4V q + V g + s (V elements per vector); the A read from LDS follows
//    the same order.  A whole offset's B vectors are prefetched into registers
//    while the previous offset's MFMAs run.
//  * Each offset's product is a fresh MFMA chain; chains are summed across
//    offsets with Kahan compensation in FP32 (plainly in FP64).  One FP32
//    chain over all 189 x NC/4 steps loses about 4x more accuracy.
// FP64 MFMA in the FP64 mode, FP32 MFMA in the mixed mode.  Sources outside
// the domain contribute zero; offsets with no valid source for any of a wave's
// 16 targets are skipped.  Work-groups are assigned to XCDs in contiguous
// ranges so that neighbouring tiles (which share operators and sources) share
// an L2.
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
  typedef f32x4 vec_t;  // one 16-byte B vector
  static constexpr int V = 4;
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
  static __device__ __forceinline__ int row(int kg, int i) { return kg + 4 * i; }
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void add(acc_t& sum, acc_t&, acc_t v) { sum += v; }
};

constexpr int kWaves = 8;  // waves per work-group
constexpr int kThreads = kWaves * 64;
constexpr int kTargetsPerGroup = kWaves * 16;

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
  static constexpr int RB = (NC + 15) / 16;      // 16-row blocks
  static constexpr int RP = RB * 16;
  static constexpr int KP = ((NC + 3) / 4) * 4;  // operator k-rows (padded)
  static constexpr int MS = mstride_of(NC);      // multipole row stride
  static constexpr int V = Mfma<T>::V;           // elements per B vector
  static constexpr int G = 4 * V;                // k per vector chunk
  static constexpr int NQ = (NC + G - 1) / G;    // vector chunks
  static constexpr int S_LAST = NC - G * (NQ - 1) < V ? NC - G * (NQ - 1) : V;
  // LDS row stride: >= RP, 16 or 48 mod 64 words, so that the four k-rows one
  // A-fragment read touches fall in distinct bank groups.
  static constexpr int SLD = (RP % 64 == 16 || RP % 64 == 48) ? RP : RP + 16;
  // k-rows staged at a time: all of them if two buffers fit in ~80 KB of LDS,
  // else a multiple of G that does.
  static constexpr int FIT = (80 * 1024) / (2 * SLD * (int)sizeof(T)) / G * G;
  static constexpr int KC = FIT >= KP ? KP : FIT;
  static constexpr int NCH = (KP + KC - 1) / KC;
  static constexpr int PER_THREAD = (KC * RP / V + kThreads - 1) / kThreads;
  static_assert(MS == KP, "multipole stride must equal the operator k padding");
  static_assert(NCH == 1 || KC % G == 0, "operator chunks must hold whole vector chunks");
};

template <int P, typename T>
__global__ __launch_bounds__(kThreads) void k_m2l(M2LArgs a, const T* __restrict__ mult,
                                                  const T* __restrict__ ops,
                                                  T* __restrict__ out) {
  typedef Shape<P, T> S;
  constexpr int NC = S::NC, RB = S::RB, RP = S::RP, KP = S::KP, MS = S::MS, SLD = S::SLD;
  constexpr int V = S::V, G = S::G, NQ = S::NQ, KC = S::KC, NCH = S::NCH;
  typedef typename Mfma<T>::acc_t acc_t;
  typedef typename Mfma<T>::vec_t vec_t;
  __shared__ __attribute__((aligned(16))) T sT[2][KC * SLD];

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
  // Operator chunk ch: global k-rows [ch*KC, min(KP, (ch+1)*KC)).
  auto chunk_vecs = [&](int ch) { return ((ch + 1) * KC <= KP ? KC : KP - ch * KC) * RP / V; };
  auto stage_load = [&](int op, int ch, vec_t* reg) {
    const vec_t* src =
        reinterpret_cast<const vec_t*>(ops + (size_t)op * KP * RP + (size_t)ch * KC * RP);
    const int nvec = chunk_vecs(ch);
#pragma unroll
    for (int i = 0; i < S::PER_THREAD; ++i) {
      const int e = tid + i * kThreads;
      if (e < nvec) reg[i] = src[e];
    }
  };
  auto stage_store = [&](int ch, T* buf, const vec_t* reg) {
    const int nvec = chunk_vecs(ch);
#pragma unroll
    for (int i = 0; i < S::PER_THREAD; ++i) {
      const int e = tid + i * kThreads;
      if (e < nvec) {
        const int k = (e * V) / RP, row = (e * V) % RP;
        *reinterpret_cast<vec_t*>(buf + k * SLD + row) = reg[i];
      }
    }
  };
  // This lane's source box for offset (dx, dy, dz) (nullptr outside the
  // domain) and its B vectors.
  auto source_of = [&](int dx, int dy, int dz) -> const T* {
    const int sx = tx - dx, sy = ty - dy, sz = tz - dz;
    const bool ok = col_ok && sx >= 0 && sy >= 0 && sz >= 0 && sx < nb && sy < nb && sz < nb;
    return ok ? mlev + (int64_t)c2s[lex_index(sx, sy, sz, l)] * MS : nullptr;
  };
  auto load_b = [&](const T* ms, vec_t* b) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k0 = G * q + V * kg;
      b[q] = vec_t{};
      if (ms && k0 < MS) b[q] = *reinterpret_cast<const vec_t*>(ms + k0);
    }
  };

  vec_t reg[S::PER_THREAD];
  vec_t bcur[NQ], bnext[NQ];
  int dx, dy, dz;
  int j = next_offset(-1, dx, dy, dz);
  const T* ms_cur = source_of(dx, dy, dz);
  load_b(ms_cur, bcur);
  stage_load(m2l_op_index(dx, dy, dz), 0, reg);
  stage_store(0, sT[0], reg);
  __syncthreads();
  int cur = 0, ch = 0;
  bool wave_any = __any(ms_cur != nullptr);
  bool ok_next = false;
  while (true) {
    // the stage after (j, ch); its operator chunk is loaded while this one computes
    int jn = j, chn = ch + 1, ndx = dx, ndy = dy, ndz = dz;
    if (chn == NCH) {
      chn = 0;
      jn = next_offset(j, ndx, ndy, ndz);
    }
    const bool more = jn < 216;
    if (more) stage_load(m2l_op_index(ndx, ndy, ndz), chn, reg);
    if (ch == 0) {  // prefetch the next offset's sources
      int fx = dx, fy = dy, fz = dz;
      const int jf = next_offset(j, fx, fy, fz);
      ok_next = false;
      if (jf < 216) {
        const T* ms_next = source_of(fx, fy, fz);
        ok_next = ms_next != nullptr;
        load_b(ms_next, bnext);
      }
    }

    if (wave_any) {
      const T* sTc = sT[cur] + col;
      const int kbase = ch * KC;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (NCH > 1 && (G * q < kbase || G * q >= kbase + KC)) continue;
        const int ns = (q == NQ - 1) ? S::S_LAST : V;
#pragma unroll
        for (int s = 0; s < V; ++s) {
          if (s >= ns) break;
          int k = G * q + V * kg + s;
          k = k < KP ? k : KP - 1;  // rows past KP meet zero B values; keep the read in range
          const T bv = bcur[q][s];
#pragma unroll
          for (int r = 0; r < RB; ++r)
            acc[r] = Mfma<T>::step(sTc[(k - kbase) * SLD + 16 * r], bv, acc[r]);
        }
      }
      if (ch == NCH - 1) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          Mfma<T>::add(sum[r], comp[r], acc[r]);
          acc[r] = acc_t{0, 0, 0, 0};
        }
      }
    }
    if (!more) break;
    stage_store(chn, sT[cur ^ 1], reg);
    __syncthreads();
    cur ^= 1;
    if (chn == 0) {  // moving to the next offset, whose sources are in bnext
#pragma unroll
      for (int q = 0; q < NQ; ++q) bcur[q] = bnext[q];
      wave_any = __any(ok_next);
    }
    j = jn;
    ch = chn;
    dx = ndx;
    dy = ndy;
    dz = ndz;
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
                                               wsp<float>(Pl, lay.op_m2l32),
                                               wsp<float>(Pl, lay.m2l_out));
    else
      k_m2l<P, double><<<grid, kThreads, 0, s>>>(a, wsp<double>(Pl, lay.mult64),
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
