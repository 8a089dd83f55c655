// downward.hip -- L2L from level 2 down to the leaves and L2P.
//
// L2L (shift.hip, FP64 in both modes): at level l the local expansion of box c
// is L~c = (1/h_l) * (M2L result of c) + B[octant(c)] L~parent(c) (l > 2) with
// the level-free octant matrices B; the 1/h_l of the unit-box M2L operators is
// applied there.  The leaf level is written in the compute precision for L2P.
// L2P: phi(c + u) = sum_n [L~_n^0 R_n^0(u/h) + 2 sum_{m>0} Re(L~_n^m R_n^m(u/h))]
// and its gradient from d/dz R_n^m = R_{n-1}^m,
// d/dx R_n^m = (R_{n-1}^{m+1} - R_{n-1}^{m-1})/2,
// d/dy R_n^m = -i (R_{n-1}^{m-1} + R_{n-1}^{m+1})/2, with R_{n-1}^{-1} =
// -conj(R_{n-1}^1), scaled by 1/h.
#include "fmm_internal.h"

namespace fmm {
namespace {

// level: adaptive tree, the level of each (compact) leaf row, whose local
// expansion is zero above level 2; null: every leaf is of level L.
template <int P, typename T>
__global__ __launch_bounds__(kBlock) void k_l2p(const uint32_t* __restrict__ sorted_leaf,
                                                const Rec<T>* __restrict__ src, int64_t n, int L,
                                                const int32_t* __restrict__ level,
                                                const DevParams* __restrict__ dp,
                                                const T* __restrict__ leafloc,
                                                double* __restrict__ far_phi,
                                                double* __restrict__ far_grad) {
  constexpr int MS = mstride_of((P + 1) * (P + 1));
  constexpr int NT = (P + 1) * (P + 2) / 2;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const uint32_t leaf = sorted_leaf[s];
  if (level) {
    L = level[leaf];
    if (L < 2) {
      far_phi[s] = 0.0;
      far_grad[s] = far_grad[n + s] = far_grad[2 * n + s] = 0.0;
      return;
    }
  }
  const T* Lc = leafloc + (int64_t)leaf * MS;
  T re[NT], im[NT];
  const Rec<T> r = src[s];
  regular_harmonics<P, T>(r.x, r.y, r.z, re, im);
  T f = T(0), gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
  for (int nn = 0; nn <= P; ++nn) {
    // m = 0
    {
      const T c = Lc[cidx_re(nn, 0)];
      f += c * re[tri(nn, 0)];
      if (nn >= 1) {
        gz += c * re[tri(nn - 1, 0)];
        if (nn >= 2) {
          gx += c * re[tri(nn - 1, 1)];
          gy += c * im[tri(nn - 1, 1)];
        }
      }
    }
#pragma unroll
    for (int m = 1; m <= nn; ++m) {
      const T cr = T(2) * Lc[cidx_re(nn, m)], ci = T(2) * Lc[cidx_im(nn, m)];
      f += cr * re[tri(nn, m)] - ci * im[tri(nn, m)];
      // R_{n-1}^{m-1} (m-1 >= 0), R_{n-1}^{m+1} (zero unless m+1 <= n-1), R_{n-1}^m
      const T ar = re[tri(nn - 1, m - 1)], ai = im[tri(nn - 1, m - 1)];
      T br = T(0), bi = T(0), zr = T(0), zi = T(0);
      if (m + 1 <= nn - 1) {
        br = re[tri(nn - 1, m + 1)];
        bi = im[tri(nn - 1, m + 1)];
      }
      if (m <= nn - 1) {
        zr = re[tri(nn - 1, m)];
        zi = im[tri(nn - 1, m)];
      }
      // Re(c X) = cr Xr - ci Xi, with X the derivative's combination
      gx += T(0.5) * (cr * (br - ar) - ci * (bi - ai));
      gy += T(0.5) * (cr * (ai + bi) + ci * (ar + br));
      gz += cr * zr - ci * zi;
    }
  }
  const double inv_h = (double)(1 << L) / dp->side;
  far_phi[s] = (double)f;
  far_grad[s] = inv_h * (double)gx;
  far_grad[n + s] = inv_h * (double)gy;
  far_grad[2 * n + s] = inv_h * (double)gz;
}

template <int P>
struct L2PRun {
  static hipError_t run(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    const int64_t n = Pl->n;
    const DevParams* dp = wsp<DevParams>(Pl, lay.params);
    if (Pl->mixed)
      k_l2p<P, float><<<grid_for(n, kBlock), kBlock, 0, s>>>(
          wsp<uint32_t>(Pl, lay.sorted_leaf), wsp<Rec<float>>(Pl, lay.src), n, Pl->L, nullptr, dp,
          wsp<float>(Pl, lay.leaf_loc32), wsp<double>(Pl, lay.far_phi),
          wsp<double>(Pl, lay.far_grad));
    else
      k_l2p<P, double><<<grid_for(n, kBlock), kBlock, 0, s>>>(
          wsp<uint32_t>(Pl, lay.sorted_leaf), wsp<Rec<double>>(Pl, lay.src), n, Pl->L, nullptr, dp,
          wsp<double>(Pl, lay.loc_exp64) + lay.lvl_off[Pl->L] * mstride(Pl->p),
          wsp<double>(Pl, lay.far_phi), wsp<double>(Pl, lay.far_grad));
    return hipGetLastError();
  }
};

}  // namespace

// Adaptive tree: L2P at every particle from its leaf's local expansion
// (FP32 copy in the mixed mode), zero above level 2.
template <int P>
struct L2PAdaptiveRun {
  static hipError_t run(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    const int64_t n = Pl->n;
    const DevParams* dp = wsp<DevParams>(Pl, lay.params);
    const int32_t* lev = wsp<int32_t>(Pl, lay.a_level);
    if (Pl->mixed)
      k_l2p<P, float><<<grid_for(n, kBlock), kBlock, 0, s>>>(
          wsp<uint32_t>(Pl, lay.sorted_leaf), wsp<Rec<float>>(Pl, lay.src), n, Pl->L, lev, dp,
          wsp<float>(Pl, lay.leaf_loc32), wsp<double>(Pl, lay.far_phi), wsp<double>(Pl, lay.far_grad));
    else
      k_l2p<P, double><<<grid_for(n, kBlock), kBlock, 0, s>>>(
          wsp<uint32_t>(Pl, lay.sorted_leaf), wsp<Rec<double>>(Pl, lay.src), n, Pl->L, lev, dp,
          wsp<double>(Pl, lay.loc_exp64), wsp<double>(Pl, lay.far_phi), wsp<double>(Pl, lay.far_grad));
    return hipGetLastError();
  }
};

hipError_t launch_l2p_adaptive(fmm_plan_s* P, hipStream_t s) { return dispatch_p<L2PAdaptiveRun>(P->p, P, s); }

hipError_t launch_downward(fmm_plan_s* P, hipStream_t s) {
  if (P->adaptive) return launch_adaptive_downward(P, s);
  prof_begin(P, FMM_PHASE_L2L, s);
  hipError_t e = launch_l2l(P, s);
  prof_end(P, s);
  if (e != hipSuccess) return e;
  prof_begin(P, FMM_PHASE_L2P, s);
  e = dispatch_p<L2PRun>(P->p, P, s);
  prof_end(P, s);
  return e;
}

}  // namespace fmm
