// shift.hip -- M2M and L2L on the FP64 matrix cores.
//
// Both translations use the 8 level-free octant matrices (operators.hip), so
// each level is a set of dense products batched by octant:
//   M2M  M~p[:, parents]          = sum_o A_o * M~[:, child of octant o]
//   L2L  L~[:, children of oct o] = (1/h) M2L[:, ...] + B_o * L~[:, parents]
// FP64 in both precision modes.  One work-group owns 128 targets (parents for
// M2M; the octant-o children of 128 parent slots for L2L), one wave 16 of
// them; the operator of each octant is staged in LDS (in chunks of k-rows when
// it does not fit) and shared by the 128 targets.  The B operand is read as
// 16-byte vectors (two coefficients), the K order of the MFMA steps being
// permuted to match (lane group g at sub-step s of chunk q uses k = 8q + 2g + s).
#include "fmm_internal.h"

namespace fmm {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int kWaves = 8;
constexpr int kThreads = kWaves * 64;
constexpr int kTargets = kWaves * 16;

template <int P>
struct ShiftShape {
  static constexpr int NC = (P + 1) * (P + 1);
  static constexpr int RB = (NC + 15) / 16;
  static constexpr int RP = RB * 16;
  static constexpr int KP = ((NC + 3) / 4) * 4;
  static constexpr int MS = mstride_of(NC);
  static constexpr int G = 8;                   // k per vector chunk (4 lane groups x 2)
  static constexpr int NQ = (NC + G - 1) / G;
  static constexpr int S_LAST = NC - G * (NQ - 1) < 2 ? NC - G * (NQ - 1) : 2;
  static constexpr int SLD = (RP % 64 == 16 || RP % 64 == 48) ? RP : RP + 16;
  static constexpr int FIT = (80 * 1024) / (SLD * 8) / G * G;
  static constexpr int KC = FIT >= KP ? KP : FIT;
  static constexpr int NCH = (KP + KC - 1) / KC;
  static constexpr int PER_THREAD = (KC * RP / 2 + kThreads - 1) / kThreads;
  static_assert(NCH == 1 || KC % G == 0, "operator chunks must hold whole vector chunks");
};

struct ShiftArgs {
  int mode;            // 0 = M2M, 1 = L2L
  int l;               // level of the targets
  int mixed;           // source (M2M) / destination (L2L leaf) is FP32
  int leaf;            // L2L: this level is the leaf level
  int64_t ntargets;    // M2M: parents at level l; L2L: parents at level l-1 (per octant)
  int64_t ntile;       // tiles of 128 per octant (L2L) or in all (M2M)
  const uint32_t* s2c_child;  // slot -> coord of the child level
  const double* ops;          // 8 padded operators [oct][KP][RP]
  const void* src;            // M2M: child multipoles (stride MS); L2L: parent locals (stride MS)
  double* dst64;              // M2M: parent multipoles; L2L: child locals (stride MS)
  float* dst32;               // M2M mixed: FP32 copy of the parents; L2L mixed leaf: leaf locals
  const void* m2l;            // L2L: M2L results of the children (stride NC, FP32 if mixed)
  const DevParams* dp;
};

template <int P>
__global__ __launch_bounds__(kThreads) void k_shift(ShiftArgs a) {
  typedef ShiftShape<P> S;
  constexpr int NC = S::NC, RB = S::RB, RP = S::RP, KP = S::KP, MS = S::MS, SLD = S::SLD;
  constexpr int G = S::G, NQ = S::NQ, KC = S::KC, NCH = S::NCH;
  __shared__ __attribute__((aligned(16))) double sT[KC * SLD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t g = blockIdx.x;
  const int oct_l2l = a.mode == 1 ? (int)(g / a.ntile) : 0;
  const int64_t tile = a.mode == 1 ? g % a.ntile : g;
  const int64_t ps = tile * kTargets + wave * 16 + col;  // parent slot of this column
  const bool ok = ps < a.ntargets;

  // child of each octant: children of slot ps are slots 8 ps .. 8 ps + 7
  int child_of[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) child_of[o] = 0;
  if (ok) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      int x, y, z;
      unpack_coord(a.s2c_child[8 * ps + c], x, y, z);
      child_of[((x & 1) << 2) | ((y & 1) << 1) | (z & 1)] = c;
    }
  }

  f64x4 acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = f64x4{0, 0, 0, 0};

  const int nops = a.mode == 0 ? 8 : 1;
  for (int o = 0; o < nops; ++o) {
    const int oct = a.mode == 0 ? o : oct_l2l;
    // this lane's B operand: the octant-oct child (M2M) or the parent (L2L)
    f64x2 b[NQ];
    {
      int64_t row_of_src = -1;
      if (ok) row_of_src = a.mode == 0 ? 8 * ps + child_of[oct] : ps;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int k0 = G * q + 2 * kg;
        b[q] = f64x2{0.0, 0.0};
        if (row_of_src >= 0 && k0 < MS) {
          if (a.mode == 0 && a.mixed) {
            const f32x2 v = *reinterpret_cast<const f32x2*>(
                static_cast<const float*>(a.src) + row_of_src * MS + k0);
            b[q] = f64x2{(double)v[0], (double)v[1]};
          } else {
            b[q] = *reinterpret_cast<const f64x2*>(static_cast<const double*>(a.src) +
                                                   row_of_src * MS + k0);
          }
        }
      }
    }
    for (int ch = 0; ch < NCH; ++ch) {
      // stage k-rows [ch*KC, ...) of the operator
      const int rows = (ch + 1) * KC <= KP ? KC : KP - ch * KC;
      const f64x2* srcv =
          reinterpret_cast<const f64x2*>(a.ops + (size_t)oct * KP * RP + (size_t)ch * KC * RP);
      __syncthreads();
      for (int e = tid; e < rows * RP / 2; e += kThreads) {
        const int k = (2 * e) / RP, row = (2 * e) % RP;
        *reinterpret_cast<f64x2*>(sT + k * SLD + row) = srcv[e];
      }
      __syncthreads();
      const double* sTc = sT + col;
      const int kbase = ch * KC;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (NCH > 1 && (G * q < kbase || G * q >= kbase + KC)) continue;
        const int ns = (q == NQ - 1) ? S::S_LAST : 2;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          if (s >= ns) break;
          int k = G * q + 2 * kg + s;
          k = k < KP ? k : KP - 1;  // rows past KP meet zero B values
          const double bv = b[q][s];
#pragma unroll
          for (int r = 0; r < RB; ++r)
            acc[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(sTc[(k - kbase) * SLD + 16 * r], bv,
                                                          acc[r], 0, 0, 0);
        }
      }
    }
  }

  if (!ok) return;
  // f64 accumulator layout: lane holds column col, rows 16 r + kg + 4 i
  if (a.mode == 0) {
    double* o64 = a.dst64 + ps * MS;
    float* o32 = a.dst32 ? a.dst32 + ps * MS : nullptr;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * r + kg + 4 * i;
        if (row < MS) {  // rows NC..MS-1 are zero (zero operator rows)
          o64[row] = acc[r][i];
          if (o32) o32[row] = (float)acc[r][i];
        }
      }
  } else {
    const int64_t cs = 8 * ps + child_of[oct_l2l];
    const double inv_h = (double)(1 << a.l) / a.dp->side;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * r + kg + 4 * i;
        if (row >= MS) continue;
        double v = acc[r][i];
        if (row < NC)
          v += inv_h * (a.mixed ? (double)static_cast<const float*>(a.m2l)[cs * NC + row]
                                : static_cast<const double*>(a.m2l)[cs * NC + row]);
        if (a.leaf && a.mixed)
          a.dst32[cs * MS + row] = (float)v;
        else
          a.dst64[cs * MS + row] = v;
      }
  }
}

template <int P>
struct ShiftRun {
  static hipError_t run(ShiftArgs a, int64_t groups, hipStream_t s) {
    k_shift<P><<<(unsigned)groups, kThreads, 0, s>>>(a);
    return hipGetLastError();
  }
};

// Level 2 locals: L~ = (1/h) * M2L result (no parent contribution).
template <typename TM>
__global__ void k_l2l_top(int nc, int ms, int l, int64_t nbox, const DevParams* __restrict__ dp,
                          const TM* __restrict__ m2l, double* __restrict__ dst64,
                          float* __restrict__ dst32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nbox * ms) return;
  const int64_t b = e / ms;
  const int row = (int)(e % ms);
  const double v = row < nc ? (double)(1 << l) / dp->side * (double)m2l[b * nc + row] : 0.0;
  if (dst32)
    dst32[e] = (float)v;
  else
    dst64[e] = v;
}

}  // namespace

hipError_t launch_m2m(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  const int ms = mstride(P->p);
  double* m64 = wsp<double>(P, lay.mult64);
  float* m32 = P->mixed ? wsp<float>(P, lay.mult32) : nullptr;
  for (int l = P->L - 1; l >= 2; --l) {
    ShiftArgs a = {};
    a.mode = 0;
    a.l = l;
    a.mixed = (l + 1 == P->L && P->mixed) ? 1 : 0;  // leaf multipoles are FP32 in the mixed mode
    a.ntargets = (int64_t)1 << (3 * l);
    a.ntile = (a.ntargets + kTargets - 1) / kTargets;
    a.s2c_child = wsp<uint32_t>(P, lay.slot2coord) + lay.lvl_off[l + 1];
    a.ops = wsp<double>(P, lay.op_m2m);
    a.src = a.mixed ? (const void*)(m32 + lay.lvl_off[l + 1] * ms)
                    : (const void*)(m64 + lay.lvl_off[l + 1] * ms);
    a.dst64 = m64 + lay.lvl_off[l] * ms;
    a.dst32 = m32 ? m32 + lay.lvl_off[l] * ms : nullptr;
    a.dp = wsp<DevParams>(P, lay.params);
    hipError_t e = dispatch_p<ShiftRun>(P->p, a, a.ntile, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_l2l(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  const int nc = P->nc, ms = mstride(P->p), L = P->L;
  double* l64 = wsp<double>(P, lay.loc_exp64);
  float* leaf32 = P->mixed ? wsp<float>(P, lay.leaf_loc32) : nullptr;
  const DevParams* dp = wsp<DevParams>(P, lay.params);
  {
    const int64_t nb = 64;  // level 2
    float* d32 = (L == 2 && P->mixed) ? leaf32 : nullptr;
    if (P->mixed)
      k_l2l_top<float><<<grid_for(nb * ms, kBlock), kBlock, 0, s>>>(
          nc, ms, 2, nb, dp, wsp<float>(P, lay.m2l_out) + lay.lvl_off[2] * nc,
          l64 + lay.lvl_off[2] * ms, d32);
    else
      k_l2l_top<double><<<grid_for(nb * ms, kBlock), kBlock, 0, s>>>(
          nc, ms, 2, nb, dp, wsp<double>(P, lay.m2l_out) + lay.lvl_off[2] * nc,
          l64 + lay.lvl_off[2] * ms, nullptr);
  }
  for (int l = 3; l <= L; ++l) {
    ShiftArgs a = {};
    a.mode = 1;
    a.l = l;
    a.mixed = P->mixed ? 1 : 0;
    a.leaf = l == L ? 1 : 0;
    a.ntargets = (int64_t)1 << (3 * (l - 1));
    a.ntile = (a.ntargets + kTargets - 1) / kTargets;
    a.s2c_child = wsp<uint32_t>(P, lay.slot2coord) + lay.lvl_off[l];
    a.ops = wsp<double>(P, lay.op_l2l);
    a.src = l64 + lay.lvl_off[l - 1] * ms;
    a.dst64 = l64 + lay.lvl_off[l] * ms;
    a.dst32 = (l == L && P->mixed) ? leaf32 : nullptr;
    a.m2l = P->mixed ? (const void*)(wsp<float>(P, lay.m2l_out) + lay.lvl_off[l] * nc)
                     : (const void*)(wsp<double>(P, lay.m2l_out) + lay.lvl_off[l] * nc);
    a.dp = dp;
    hipError_t e = dispatch_p<ShiftRun>(P->p, a, 8 * a.ntile, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace fmm
