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
// Mapping: one wave64 owns 16 targets of one parity class at one level (the
// parity-pi children of 16 consecutive parent slots in Hilbert order) and keeps
// their NC-row local expansions in MFMA accumulators for the whole offset
// loop.  Each 16x16x4 MFMA takes 16 operator rows x 4 input coefficients (A)
// and 4 input coefficients x 16 targets (B); the B fragment of a k-step is
// reused by every 16-row block.  FP64 MFMA in the FP64 mode, FP32 MFMA with
// FP32 accumulation in the mixed mode.  Sources outside the domain contribute
// zero.  Work-groups are assigned to XCDs in contiguous ranges so that
// neighbouring tiles (which share operators and sources) share an L2.
#include "fmm_internal.h"

namespace fmm {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Accumulator lane layout (measured on gfx950): lane l holds column l % 16;
// its four values are rows 4 (l / 16) + i for the f32 form and (l / 16) + 4 i
// for the f64 form.
// Results of one offset's MFMA chain are added to the running sum across
// offsets: compensated (Kahan) in FP32, plainly in FP64.  One FP32 accumulator
// chained over all 189 x NC/4 steps loses about 4x more accuracy.
template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ int row(int kg, int i) { return 4 * kg + i; }
  static __device__ __forceinline__ void add(acc_t& sum, acc_t& comp, acc_t v) {
    const acc_t y = v - comp;
    const acc_t t = sum + y;
    comp = (t - sum) - y;
    sum = t;
  }
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ int row(int kg, int i) { return kg + 4 * i; }
  static __device__ __forceinline__ void add(acc_t& sum, acc_t&, acc_t v) { sum += v; }
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

constexpr int kWaves = 4;  // waves per work-group

struct M2LArgs {
  int L;
  int64_t lvl_off[FMM_DEPTH_MAX + 2];  // box offsets per level
  int64_t wave_off[FMM_DEPTH_MAX + 2];  // first wave of each level (levels 2..L)
  int64_t total_waves;
  int64_t nblocks;
  const uint32_t* c2s;
  const uint32_t* s2c;
};

template <int P, typename T>
__global__ __launch_bounds__(kWaves * 64) void k_m2l(M2LArgs a, const T* __restrict__ mult,
                                                     const T* __restrict__ ops,
                                                     T* __restrict__ out) {
  constexpr int NC = (P + 1) * (P + 1);
  constexpr int RB = (NC + 15) / 16;
  constexpr int RP = RB * 16;
  constexpr int KP = ((NC + 3) / 4) * 4;
  typedef typename Mfma<T>::acc_t acc_t;

  // XCD-aware block order: hardware block b runs on XCD b % 8; give each XCD a
  // contiguous range of logical blocks.
  const int64_t per_xcd = (a.nblocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  const int64_t gw = lb * kWaves + (threadIdx.x >> 6);
  if (lb >= a.nblocks || gw >= a.total_waves) return;

  int l = 2;
  while (l < a.L && gw >= a.wave_off[l + 1]) ++l;
  const int64_t np = (int64_t)1 << (3 * (l - 1));  // parents
  const int64_t ntile = (np + 15) / 16;
  const int64_t idx = gw - a.wave_off[l];
  const int pi = (int)(idx / ntile);
  const int64_t tile = idx % ntile;
  const int px = (pi >> 2) & 1, py = (pi >> 1) & 1, pz = pi & 1;

  const int lane = threadIdx.x & 63;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t ps = tile * 16 + col;
  const bool col_ok = ps < np;
  int tx = 0, ty = 0, tz = 0;
  if (col_ok) {
    unpack_coord(a.s2c[a.lvl_off[l - 1] + ps], tx, ty, tz);
    tx = 2 * tx + px;
    ty = 2 * ty + py;
    tz = 2 * tz + pz;
  }
  const int nb = 1 << l;
  const uint32_t* c2s = a.c2s + a.lvl_off[l];
  const T* mlev = mult + a.lvl_off[l] * NC;

  acc_t sum[RB], comp[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) sum[r] = comp[r] = acc_t{0, 0, 0, 0};

  for (int dx = px - 3; dx <= px + 2; ++dx)
    for (int dy = py - 3; dy <= py + 2; ++dy)
      for (int dz = pz - 3; dz <= pz + 2; ++dz) {
        if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) continue;
        const int sx = tx - dx, sy = ty - dy, sz = tz - dz;
        const bool ok = col_ok && sx >= 0 && sy >= 0 && sz >= 0 && sx < nb && sy < nb && sz < nb;
        const T* ms = mlev + (ok ? (int64_t)c2s[lex_index(sx, sy, sz, l)] * NC : 0);
        const T* op = ops + (size_t)m2l_op_index(dx, dy, dz) * KP * RP + col;
        acc_t acc[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r] = acc_t{0, 0, 0, 0};
#pragma unroll 2
        for (int kk = 0; kk < KP / 4; ++kk) {
          const int k = 4 * kk + kg;
          const T b = (ok && k < NC) ? ms[k] : T(0);
          const T* opk = op + (size_t)k * RP;
#pragma unroll
          for (int r = 0; r < RB; ++r) acc[r] = Mfma<T>::step(opk[16 * r], b, acc[r]);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) Mfma<T>::add(sum[r], comp[r], acc[r]);
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
    int64_t w = 0;
    for (int l = 2; l <= Pl->L; ++l) {
      a.wave_off[l] = w;
      const int64_t np = (int64_t)1 << (3 * (l - 1));
      w += 8 * ((np + 15) / 16);
    }
    a.wave_off[Pl->L + 1] = w;
    a.total_waves = w;
    a.nblocks = (w + kWaves - 1) / kWaves;
    a.c2s = wsp<uint32_t>(Pl, lay.coord2slot);
    a.s2c = wsp<uint32_t>(Pl, lay.slot2coord);
    const unsigned grid = (unsigned)(((a.nblocks + 7) / 8) * 8);
    if (Pl->mixed)
      k_m2l<P, float><<<grid, kWaves * 64, 0, s>>>(a, wsp<float>(Pl, lay.mult32),
                                                  wsp<float>(Pl, lay.op_m2l32),
                                                  wsp<float>(Pl, lay.m2l_out));
    else
      k_m2l<P, double><<<grid, kWaves * 64, 0, s>>>(a, wsp<double>(Pl, lay.mult64),
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
