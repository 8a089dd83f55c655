// upward.hip -- charges into Hilbert order, P2M at the leaves, M2M up to
// level 2.
//
// P2M: M~_n^m = sum_j q_j conj(R_n^m(u_j)) with u_j the box-unit offset of
// particle j from its leaf centre (computed by the tree pass), accumulated in
// FP64 in both precision modes from the FP64 offsets.  (An FP32 sum of
// neutral clusters of charges, one cluster after another, rounds every
// cluster's partial sums the same way, so the leaf monopoles would drift by an
// amount proportional to the particle count: a smooth, density-shaped error
// charge.  FP64 adds cost the same issue slots as FP32 ones here.)  The mixed
// mode stores the sum rounded to FP32 only, read by the M2L pass and,
// converted back, by the M2M pass: one rounding of the final value, with no
// drift.
// M2M (shift.hip): M~p = sum over the 8 children of A[octant] M~c with the
// level-free octant matrices, always in FP64; in the mixed mode each parent is
// also stored rounded to FP32 for the M2L pass.
#include "fmm_internal.h"

namespace fmm {
namespace {

template <typename T>
__global__ void k_gather_q(const double* __restrict__ q, const int32_t* __restrict__ perm, int64_t n,
                           double* __restrict__ q64, Rec<T>* __restrict__ src,
                           Rec<double>* __restrict__ src64) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double v = q[perm[s]];
  q64[s] = v;
  src[s].q = (T)v;
  if (src64) src64[s].q = v;
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_p2m(const uint32_t* __restrict__ start,
                                                const Rec<double>* __restrict__ src, int64_t nleaf,
                                                double* __restrict__ mult, float* __restrict__ mult32) {
  typedef double T;
  constexpr int NC = (P + 1) * (P + 1);
  constexpr int MS = mstride_of(NC);
  constexpr int NT = (P + 1) * (P + 2) / 2;
  const int64_t leaf = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (leaf >= nleaf) return;
  T acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = T(0);
  const uint32_t b = start[leaf], e = start[leaf + 1];
  for (uint32_t s = b; s < e; ++s) {
    T re[NT], im[NT];
    const Rec<T> r = src[s];
    regular_harmonics<P, T>(r.x, r.y, r.z, re, im);
    const T qq = r.q;
#pragma unroll
    for (int nn = 0; nn <= P; ++nn) {
      acc[cidx_re(nn, 0)] += qq * re[tri(nn, 0)];
#pragma unroll
      for (int m = 1; m <= nn; ++m) {
        acc[cidx_re(nn, m)] += qq * re[tri(nn, m)];
        acc[cidx_im(nn, m)] -= qq * im[tri(nn, m)];
      }
    }
  }
  if (mult) {
    T* out = mult + leaf * MS;
#pragma unroll
    for (int c = 0; c < MS; ++c) out[c] = c < NC ? acc[c] : T(0);
  }
  if (mult32) {
    float* o32 = mult32 + leaf * MS;
#pragma unroll
    for (int c = 0; c < MS; ++c) o32[c] = c < NC ? (float)acc[c] : 0.f;
  }
}

template <int P>
struct P2MRun {
  static hipError_t run(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    const int64_t nleaf = lay.nleaf, row0 = lay.lvl_off[Pl->L] * mstride(Pl->p);
    k_p2m<P><<<grid_for(nleaf, 64), 64, 0, s>>>(
        wsp<uint32_t>(Pl, lay.leaf_start), wsp<Rec<double>>(Pl, Pl->mixed ? lay.src64 : lay.src), nleaf,
        Pl->mixed ? nullptr : wsp<double>(Pl, lay.mult64) + row0,
        Pl->mixed ? wsp<float>(Pl, lay.mult32) + row0 : nullptr);
    return hipGetLastError();
  }
};

}  // namespace

hipError_t launch_upward(fmm_plan_s* P, const double* d_q, hipStream_t s) {
  const Layout& lay = P->lay;
  const int64_t n = P->n;
  if (d_q) {  // NULL: reuse the sorted charges of the last evaluation (adjoint)
    if (P->mixed)
      k_gather_q<float><<<grid_for(n, kBlock), kBlock, 0, s>>>(
          d_q, wsp<int32_t>(P, lay.perm), n, wsp<double>(P, lay.q64), wsp<Rec<float>>(P, lay.src),
          wsp<Rec<double>>(P, lay.src64));
    else
      k_gather_q<double><<<grid_for(n, kBlock), kBlock, 0, s>>>(
          d_q, wsp<int32_t>(P, lay.perm), n, wsp<double>(P, lay.q64), wsp<Rec<double>>(P, lay.src),
          nullptr);
  }
  if (P->adaptive) return launch_adaptive_upward(P, s);
  if (P->L < 2) return hipGetLastError();
  prof_begin(P, FMM_PHASE_P2M, s);
  hipError_t e = dispatch_p<P2MRun>(P->p, P, s);
  prof_end(P, s);
  if (e != hipSuccess) return e;
  prof_begin(P, FMM_PHASE_M2M, s);
  e = launch_m2m(P, s);
  prof_end(P, s);
  return e;
}

}  // namespace fmm
