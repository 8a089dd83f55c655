// downward.hip -- L2L from level 2 down to the leaves and L2P.
//
// L2L (FP64 in both modes): at level l the local expansion of box c is
//   L~c = (1/h_l) * (M2L result of c) + B[octant(c)] L~parent(c)   (l > 2)
// with the level-free octant matrices B; the 1/h_l of the unit-box M2L
// operators is applied here.  The leaf level is written in the compute
// precision for L2P.
// L2P: phi(c + u) = sum_n [L~_n^0 R_n^0(u/h) + 2 sum_{m>0} Re(L~_n^m R_n^m(u/h))]
// and its gradient from d/dz R_n^m = R_{n-1}^m,
// d/dx R_n^m = (R_{n-1}^{m+1} - R_{n-1}^{m-1})/2,
// d/dy R_n^m = -i (R_{n-1}^{m-1} + R_{n-1}^{m+1})/2, with R_{n-1}^{-1} =
// -conj(R_{n-1}^1), scaled by 1/h.
#include "fmm_internal.h"

namespace fmm {
namespace {

template <typename TM, typename TO>
__global__ void k_l2l(int nc, int l, int64_t nbox, const DevParams* __restrict__ dp,
                      const uint32_t* __restrict__ s2c, const TM* __restrict__ m2l,
                      const double* __restrict__ parent, const double* __restrict__ B,
                      TO* __restrict__ outl) {
  extern __shared__ double sp[];  // parent coefficients
  const int64_t cs = blockIdx.x;
  if (cs >= nbox) return;
  if (parent)
    for (int e = threadIdx.x; e < nc; e += blockDim.x) sp[e] = parent[(cs >> 3) * nc + e];
  __syncthreads();
  const int row = threadIdx.x;
  if (row >= nc) return;
  const double inv_h = (double)(1 << l) / dp->side;
  double v = inv_h * (double)m2l[cs * nc + row];
  if (parent) {
    int x, y, z;
    unpack_coord(s2c[cs], x, y, z);
    const double* Bo = B + (size_t)(((x & 1) << 2) | ((y & 1) << 1) | (z & 1)) * nc * nc;
    for (int k = 0; k < nc; ++k) v += Bo[(size_t)k * nc + row] * sp[k];
  }
  outl[cs * nc + row] = (TO)v;
}

template <int P, typename T>
__global__ __launch_bounds__(kBlock) void k_l2p(const uint32_t* __restrict__ sorted_leaf,
                                                const T* __restrict__ loc, int64_t n, int L,
                                                const DevParams* __restrict__ dp,
                                                const T* __restrict__ leafloc,
                                                double* __restrict__ far_phi,
                                                double* __restrict__ far_grad) {
  constexpr int NC = (P + 1) * (P + 1);
  constexpr int NT = (P + 1) * (P + 2) / 2;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const T* Lc = leafloc + (int64_t)sorted_leaf[s] * NC;
  T re[NT], im[NT];
  regular_harmonics<P, T>(loc[s], loc[n + s], loc[2 * n + s], re, im);
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
          wsp<uint32_t>(Pl, lay.sorted_leaf), wsp<float>(Pl, lay.loc32), n, Pl->L, dp,
          wsp<float>(Pl, lay.leaf_loc32), wsp<double>(Pl, lay.far_phi),
          wsp<double>(Pl, lay.far_grad));
    else
      k_l2p<P, double><<<grid_for(n, kBlock), kBlock, 0, s>>>(
          wsp<uint32_t>(Pl, lay.sorted_leaf), wsp<double>(Pl, lay.loc64), n, Pl->L, dp,
          wsp<double>(Pl, lay.loc_exp64) + lay.lvl_off[Pl->L] * Pl->nc,
          wsp<double>(Pl, lay.far_phi), wsp<double>(Pl, lay.far_grad));
    return hipGetLastError();
  }
};

}  // namespace

hipError_t launch_downward(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  const int nc = P->nc, L = P->L;
  const int threads = ((nc + 63) / 64) * 64;
  const size_t shm = sizeof(double) * nc;
  const DevParams* dp = wsp<DevParams>(P, lay.params);
  const uint32_t* s2c = wsp<uint32_t>(P, lay.slot2coord);
  double* l64 = wsp<double>(P, lay.loc_exp64);
  const double* B = wsp<double>(P, lay.op_l2l);
  prof_begin(P, FMM_PHASE_L2L, s);
  for (int l = 2; l <= L; ++l) {
    const int64_t nb = (int64_t)1 << (3 * l);
    const double* parent = l > 2 ? l64 + lay.lvl_off[l - 1] * nc : nullptr;
    const uint32_t* s2cl = s2c + lay.lvl_off[l];
    if (P->mixed) {
      const float* m2l = wsp<float>(P, lay.m2l_out) + lay.lvl_off[l] * nc;
      if (l == L)
        k_l2l<float, float><<<(unsigned)nb, threads, shm, s>>>(nc, l, nb, dp, s2cl, m2l, parent, B,
                                                              wsp<float>(P, lay.leaf_loc32));
      else
        k_l2l<float, double><<<(unsigned)nb, threads, shm, s>>>(nc, l, nb, dp, s2cl, m2l, parent, B,
                                                               l64 + lay.lvl_off[l] * nc);
    } else {
      const double* m2l = wsp<double>(P, lay.m2l_out) + lay.lvl_off[l] * nc;
      k_l2l<double, double><<<(unsigned)nb, threads, shm, s>>>(nc, l, nb, dp, s2cl, m2l, parent, B,
                                                              l64 + lay.lvl_off[l] * nc);
    }
  }
  prof_end(P, s);
  prof_begin(P, FMM_PHASE_L2P, s);
  hipError_t e = dispatch_p<L2PRun>(P->p, P, s);
  prof_end(P, s);
  return e;
}

}  // namespace fmm
