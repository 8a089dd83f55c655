// upward.hip -- charges into Hilbert order, P2M at the leaves, M2M up to
// level 2.
//
// P2M: M~_n^m = sum_j q_j conj(R_n^m(u_j)) with u_j the box-unit offset of
// particle j from its leaf centre (computed by the tree pass), in the
// compute precision (FP32 for the mixed mode, FP64 otherwise).
// M2M: M~p = sum over the 8 children of A[octant] M~c with the level-free
// octant matrices, always in FP64; in the mixed mode each parent is also
// stored rounded to FP32 for the M2L pass.
#include "fmm_internal.h"

namespace fmm {
namespace {

__global__ void k_gather_q(const double* __restrict__ q, const int32_t* __restrict__ perm, int64_t n,
                           double* __restrict__ q64, float* __restrict__ q32) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double v = q[perm[s]];
  q64[s] = v;
  if (q32) q32[s] = (float)v;
}

template <int P, typename T>
__global__ __launch_bounds__(kBlock) void k_p2m(const uint32_t* __restrict__ start,
                                                const T* __restrict__ loc, const T* __restrict__ q,
                                                int64_t n, int64_t nleaf, T* __restrict__ mult) {
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
    regular_harmonics<P, T>(loc[s], loc[n + s], loc[2 * n + s], re, im);
    const T qq = q[s];
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
  T* out = mult + leaf * MS;
#pragma unroll
  for (int c = 0; c < NC; ++c) out[c] = acc[c];
#pragma unroll
  for (int c = NC; c < MS; ++c) out[c] = T(0);
}

// One block per parent box of level l; thread = output coefficient.  Child
// and parent rows have stride ms (zero padding written for rows nc..ms-1).
template <typename TC>
__global__ void k_m2m(int nc, int ms, int64_t nparent, const uint32_t* __restrict__ s2c_child,
                      const TC* __restrict__ child, const double* __restrict__ A,
                      double* __restrict__ parent64, float* __restrict__ parent32) {
  extern __shared__ double sm[];  // 8 * nc child coefficients
  const int64_t ps = blockIdx.x;
  if (ps >= nparent) return;
  int oct[8];
  for (int c = 0; c < 8; ++c) {
    int x, y, z;
    unpack_coord(s2c_child[8 * ps + c], x, y, z);
    oct[c] = ((x & 1) << 2) | ((y & 1) << 1) | (z & 1);
  }
  for (int e = threadIdx.x; e < 8 * nc; e += blockDim.x)
    sm[e] = (double)child[(8 * ps + e / nc) * ms + e % nc];
  __syncthreads();
  const int row = threadIdx.x;
  if (row >= nc) {
    if (row < ms) {
      parent64[ps * ms + row] = 0.0;
      if (parent32) parent32[ps * ms + row] = 0.0f;
    }
    return;
  }
  double acc = 0.0;
  for (int c = 0; c < 8; ++c) {
    const double* Ac = A + (size_t)oct[c] * nc * nc;
    const double* Mc = sm + c * nc;
    for (int k = 0; k < nc; ++k) acc += Ac[(size_t)k * nc + row] * Mc[k];
  }
  parent64[ps * ms + row] = acc;
  if (parent32) parent32[ps * ms + row] = (float)acc;
}

template <int P>
struct P2MRun {
  template <typename T>
  static hipError_t go(fmm_plan_s* Pl, const T* loc, const T* q, T* mult_leaf, hipStream_t s) {
    const int64_t nleaf = Pl->lay.nleaf;
    k_p2m<P, T><<<grid_for(nleaf, 64), 64, 0, s>>>(wsp<uint32_t>(Pl, Pl->lay.leaf_start), loc, q,
                                                   Pl->n, nleaf, mult_leaf);
    return hipGetLastError();
  }
  static hipError_t run(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    if (Pl->mixed)
      return go<float>(Pl, wsp<float>(Pl, lay.loc32), wsp<float>(Pl, lay.q32),
                       wsp<float>(Pl, lay.mult32) + lay.lvl_off[Pl->L] * mstride(Pl->p), s);
    return go<double>(Pl, wsp<double>(Pl, lay.loc64), wsp<double>(Pl, lay.q64),
                      wsp<double>(Pl, lay.mult64) + lay.lvl_off[Pl->L] * mstride(Pl->p), s);
  }
};

}  // namespace

hipError_t launch_upward(fmm_plan_s* P, const double* d_q, hipStream_t s) {
  const Layout& lay = P->lay;
  const int64_t n = P->n;
  k_gather_q<<<grid_for(n, kBlock), kBlock, 0, s>>>(
      d_q, wsp<int32_t>(P, lay.perm), n, wsp<double>(P, lay.q64),
      P->mixed ? wsp<float>(P, lay.q32) : nullptr);
  if (P->L < 2) return hipGetLastError();
  prof_begin(P, FMM_PHASE_P2M, s);
  hipError_t e = dispatch_p<P2MRun>(P->p, P, s);
  prof_end(P, s);
  if (e != hipSuccess) return e;
  const int nc = P->nc, ms = mstride(P->p);
  const int threads = ((ms + 63) / 64) * 64;
  const size_t shm = sizeof(double) * 8 * nc;
  const uint32_t* s2c = wsp<uint32_t>(P, lay.slot2coord);
  double* m64 = wsp<double>(P, lay.mult64);
  float* m32 = P->mixed ? wsp<float>(P, lay.mult32) : nullptr;
  const double* A = wsp<double>(P, lay.op_m2m);
  prof_begin(P, FMM_PHASE_M2M, s);
  for (int l = P->L - 1; l >= 2; --l) {
    const int64_t np = (int64_t)1 << (3 * l);
    const uint32_t* s2c_child = s2c + lay.lvl_off[l + 1];
    double* p64 = m64 + lay.lvl_off[l] * ms;
    float* p32 = m32 ? m32 + lay.lvl_off[l] * ms : nullptr;
    if (l + 1 == P->L && P->mixed)
      k_m2m<float><<<(unsigned)np, threads, shm, s>>>(nc, ms, np, s2c_child,
                                                      m32 + lay.lvl_off[l + 1] * ms, A, p64, p32);
    else
      k_m2m<double><<<(unsigned)np, threads, shm, s>>>(nc, ms, np, s2c_child,
                                                       m64 + lay.lvl_off[l + 1] * ms, A, p64, p32);
  }
  prof_end(P, s);
  return hipGetLastError();
}

}  // namespace fmm
