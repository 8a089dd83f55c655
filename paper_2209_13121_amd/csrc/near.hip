// near.hip -- P2P near field, combination with the far field, return to the
// caller's particle order, and the FP64 energy.
//
// For target i in leaf t the near field sums every j != i in the 27 leaves at
// Chebyshev distance <= 1 from t (adaptive tree: the leaves of U(t)).
// Distances are formed in box units from the box-local coordinates,
// x_i - x_j = h ((u_i - u_j) - o) with o the leaf offset, in FP64 and then
// rounded once, so even the mixed (FP32) form keeps the relative accuracy of a
// close pair's offset; r^2, 1/r and the sums run in the compute precision.
// Then phi_i = phi_near + phi_far, F_i = -q_i grad phi_i (FP64), written at the
// particle's user index.  In the adjoint form the same pass writes
// g dE/dq_i = g phi_i and g dE/dx_i = g q_i grad phi_i: with every
// (local <= p, multipole <= p) pair kept, the FMM energy is a symmetric
// quadratic form in q, and while no particle crosses a box face its gradient
// in x_i is q_i grad phi_i.  E = 1/2 sum q_i phi_i is reduced in FP64 in a fixed
// tree order: per-block partials, then one block over the partials.
#include <math.h>

#include "fmm_internal.h"

namespace fmm {
namespace {

__device__ __forceinline__ float inv_sqrt(float x) { return rsqrtf(x); }
__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }

template <typename T>
struct NearAcc {
  T f, gx, gy, gz;
  bool coincident;
};

// Sum over sources j in [b, e), j != i, with (ox, oy, oz) the target's offset
// from the source box centre in the target's box units: pair offset
// r = o - sg u_j.  SCALED: the sources' own offsets are in units sg times the
// target's (an exact power of two; adaptive tree).  The box-unit offsets are
// FP64 in both precision modes: the pair offset is formed in FP64 and rounded
// once to T, so a close pair keeps its relative accuracy; r^2, 1/r and the
// sums run in T.
template <bool SCALED, typename T>
__device__ __forceinline__ void near_pair(NearAcc<T>& a, double ox, double oy, double oz, double sg,
                                          const Rec<double>& rj, bool self) {
  const T rx = (T)(SCALED ? fma(-sg, rj.x, ox) : ox - rj.x);
  const T ry = (T)(SCALED ? fma(-sg, rj.y, oy) : oy - rj.y);
  const T rz = (T)(SCALED ? fma(-sg, rj.z, oz) : oz - rj.z);
  const T r2 = rx * rx + ry * ry + rz * rz;
  // the target itself and coincident points contribute nothing (the latter
  // are flagged); selects rather than branches keep the loop straight
  const bool skip = self || r2 == T(0);
  a.coincident |= !self && r2 == T(0);
  const T rinv = inv_sqrt(skip ? T(1) : r2);
  const T qr = (skip ? T(0) : (T)rj.q) * rinv;
  const T qr3 = qr * rinv * rinv;
  a.f += qr;
  a.gx -= qr3 * rx;
  a.gy -= qr3 * ry;
  a.gz -= qr3 * rz;
}

// Sum over sources j in [b, e), j != i, with (ox, oy, oz) the target's offset
// from the source box centre in the target's box units: pair offset
// r = o - sg u_j.  SCALED: the sources' own offsets are in units sg times the
// target's (an exact power of two; adaptive tree).  The box-unit offsets are
// FP64 in both precision modes: the pair offset is formed in FP64 and rounded
// once to T, so a close pair keeps its relative accuracy; r^2, 1/r and the
// sums run in T.  Four source records are loaded ahead of their use.
template <bool SCALED, typename T>
__device__ __forceinline__ void near_pairs(NearAcc<T>& a, double ox, double oy, double oz, double sg,
                                           const Rec<double>* __restrict__ src, uint32_t b,
                                           uint32_t e, int64_t i) {
  uint32_t j = b;
  for (; j + 4 <= e; j += 4) {
    const Rec<double> r0 = src[j], r1 = src[j + 1], r2 = src[j + 2], r3 = src[j + 3];
    near_pair<SCALED, T>(a, ox, oy, oz, sg, r0, (int64_t)j == i);
    near_pair<SCALED, T>(a, ox, oy, oz, sg, r1, (int64_t)j + 1 == i);
    near_pair<SCALED, T>(a, ox, oy, oz, sg, r2, (int64_t)j + 2 == i);
    near_pair<SCALED, T>(a, ox, oy, oz, sg, r3, (int64_t)j + 3 == i);
  }
  for (; j < e; ++j) near_pair<SCALED, T>(a, ox, oy, oz, sg, src[j], (int64_t)j == i);
}

struct FinishArgs {
  int64_t n;
  const double* q64;
  const int32_t* perm;
  int has_far;
  const double* far_phi;
  const double* far_grad;
  double* phi_out;
  double* force_out;
  const double* adj_g;
  double* dEdq;
  double* dEdx;
  int32_t* flags;
};

// phi_i = near + far, F_i = -q_i grad phi_i (or the adjoint outputs), at the
// particle's user index; returns q_i phi_i for the energy.
template <typename T>
__device__ __forceinline__ double finish_particle(const FinishArgs& fa, int64_t i, double inv_h,
                                                  const NearAcc<T>& acc) {
  if (acc.coincident) atomicOr(fa.flags, kFlagCoincident);
  double phi = inv_h * (double)acc.f;
  double g[3] = {inv_h * inv_h * (double)acc.gx, inv_h * inv_h * (double)acc.gy,
                 inv_h * inv_h * (double)acc.gz};
  const int64_t n = fa.n;
  if (fa.has_far) {
    phi += fa.far_phi[i];
    for (int a = 0; a < 3; ++a) g[a] += fa.far_grad[a * n + i];
  }
  const double qi = fa.q64[i];
  const int64_t u = fa.perm[i];
  if (fa.phi_out) fa.phi_out[u] = phi;
  if (fa.force_out)
    for (int a = 0; a < 3; ++a) fa.force_out[3 * u + a] = -qi * g[a];
  if (fa.adj_g) {  // adjoint: dE/dq_i = phi_i, dE/dx_i = q_i grad phi_i, times g
    const double gs = fa.adj_g[0];
    if (fa.dEdq) fa.dEdq[u] = gs * phi;
    if (fa.dEdx)
      for (int a = 0; a < 3; ++a) fa.dEdx[3 * u + a] = gs * (qi * g[a]);
  }
  return qi * phi;
}

// Deterministic block partial of q_i phi_i.
__device__ __forceinline__ void energy_partial(double e_i, double* epart) {
  __shared__ double red[kBlock];
  red[threadIdx.x] = e_i;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) epart[blockIdx.x] = red[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_near(
    int L, const DevParams* __restrict__ dp, const uint32_t* __restrict__ sorted_leaf,
    const uint32_t* __restrict__ start, const uint32_t* __restrict__ c2s,
    const uint32_t* __restrict__ s2c, const Rec<double>* __restrict__ src, FinishArgs fa,
    double* __restrict__ epart) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e_i = 0.0;
  if (i < fa.n) {
    const uint32_t leaf = sorted_leaf[i];
    int cx, cy, cz;
    unpack_coord(s2c[leaf], cx, cy, cz);
    const Rec<double> ri = src[i];
    NearAcc<T> acc = {T(0), T(0), T(0), T(0), false};
    const int nb = 1 << L;
    for (int dx = -1; dx <= 1; ++dx) {
      const int sx = cx + dx;
      if (sx < 0 || sx >= nb) continue;
      for (int dy = -1; dy <= 1; ++dy) {
        const int sy = cy + dy;
        if (sy < 0 || sy >= nb) continue;
        for (int dz = -1; dz <= 1; ++dz) {
          const int sz = cz + dz;
          if (sz < 0 || sz >= nb) continue;
          const uint32_t sl = c2s[lex_index(sx, sy, sz, L)];
          near_pairs<false, T>(acc, ri.x - dx, ri.y - dy, ri.z - dz, 1.0, src, start[sl],
                               start[sl + 1], i);
        }
      }
    }
    e_i = finish_particle(fa, i, (double)(1 << L) / dp->side, acc);
  }
  if (epart) energy_partial(e_i, epart);
}

// Adaptive tree: the sources are the leaves of U(leaf of i); a source leaf c
// sits at offset (c_c - c_t)/h_t = (cc + 1/2) 2^(lt - lc) - (ct + 1/2) from
// the target leaf t in t's units, its offsets scaled by 2^(lt - lc) (exact).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_near_list(
    const DevParams* __restrict__ dp, const uint32_t* __restrict__ sorted_leaf,
    const int32_t* __restrict__ level, const uint32_t* __restrict__ coord,
    const uint32_t* __restrict__ range, const uint32_t* __restrict__ uoff,
    const uint32_t* __restrict__ uidx, const Rec<double>* __restrict__ src, FinishArgs fa,
    double* __restrict__ epart) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e_i = 0.0;
  if (i < fa.n) {
    const uint32_t leaf = sorted_leaf[i];
    const int lt = level[leaf];
    int ct[3];
    unpack_coord(coord[leaf], ct[0], ct[1], ct[2]);
    const Rec<double> ri = src[i];
    NearAcc<T> acc = {T(0), T(0), T(0), T(0), false};
    for (uint32_t k = uoff[leaf]; k < uoff[leaf + 1]; ++k) {
      const uint32_t c = uidx[k];
      const int lc = level[c];
      int cc[3];
      unpack_coord(coord[c], cc[0], cc[1], cc[2]);
      const double sc = lt >= lc ? (double)(1 << (lt - lc)) : 1.0 / (double)(1 << (lc - lt));
      const double ox = ri.x - (((double)cc[0] + 0.5) * sc - ((double)ct[0] + 0.5));
      const double oy = ri.y - (((double)cc[1] + 0.5) * sc - ((double)ct[1] + 0.5));
      const double oz = ri.z - (((double)cc[2] + 0.5) * sc - ((double)ct[2] + 0.5));
      near_pairs<true, T>(acc, ox, oy, oz, sc, src, range[2 * c], range[2 * c] + range[2 * c + 1], i);
    }
    e_i = finish_particle(fa, i, (double)(1 << lt) / dp->side, acc);
  }
  if (epart) energy_partial(e_i, epart);
}

__global__ void k_energy(const double* __restrict__ part, int64_t nparts, double* __restrict__ e) {
  __shared__ double red[kBlock];
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nparts; b += kBlock) s += part[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) e[0] = 0.5 * red[0];
}

}  // namespace

hipError_t launch_near_and_finish(fmm_plan_s* P, double* d_phi, double* d_force,
                                  double* d_energy, const double* adj_g, double* dEdq,
                                  double* dEdx, hipStream_t s) {
  const Layout& lay = P->lay;
  const int64_t n = P->n;
  const int L = P->L;
  double* epart = d_energy ? wsp<double>(P, lay.energy_part) : nullptr;
  const uint32_t* c2s = wsp<uint32_t>(P, lay.coord2slot) + lay.lvl_off[L];
  const uint32_t* s2c = wsp<uint32_t>(P, lay.slot2coord) + lay.lvl_off[L];
  prof_begin(P, FMM_PHASE_P2P, s);
  FinishArgs fa;
  fa.n = n;
  fa.q64 = wsp<double>(P, lay.q64);
  fa.perm = wsp<int32_t>(P, lay.perm);
  fa.has_far = (P->adaptive || L >= 2) ? 1 : 0;  // the adaptive L2P pass always writes far_*
  fa.far_phi = wsp<double>(P, lay.far_phi);
  fa.far_grad = wsp<double>(P, lay.far_grad);
  fa.phi_out = d_phi;
  fa.force_out = d_force;
  fa.adj_g = adj_g;
  fa.dEdq = dEdq;
  fa.dEdx = dEdx;
  fa.flags = wsp<int32_t>(P, lay.flags);
  const DevParams* dp = wsp<DevParams>(P, lay.params);
  const uint32_t* sl = wsp<uint32_t>(P, lay.sorted_leaf);
  if (P->adaptive) {
    const int32_t* lev = wsp<int32_t>(P, lay.a_level);
    const uint32_t* crd = wsp<uint32_t>(P, lay.a_coord);
    const uint32_t* rng = wsp<uint32_t>(P, lay.a_range);
    const uint32_t* uoff = wsp<uint32_t>(P, lay.a_off);
    const uint32_t* uidx = wsp<uint32_t>(P, lay.a_uidx);
    if (P->mixed)
      k_near_list<float><<<grid_for(n, kBlock), kBlock, 0, s>>>(
          dp, sl, lev, crd, rng, uoff, uidx, wsp<Rec<double>>(P, lay.src64), fa, epart);
    else
      k_near_list<double><<<grid_for(n, kBlock), kBlock, 0, s>>>(
          dp, sl, lev, crd, rng, uoff, uidx, wsp<Rec<double>>(P, lay.src), fa, epart);
  } else if (P->mixed) {
    k_near<float><<<grid_for(n, kBlock), kBlock, 0, s>>>(
        L, dp, sl, wsp<uint32_t>(P, lay.leaf_start), c2s, s2c, wsp<Rec<double>>(P, lay.src64), fa, epart);
  } else {
    k_near<double><<<grid_for(n, kBlock), kBlock, 0, s>>>(
        L, dp, sl, wsp<uint32_t>(P, lay.leaf_start), c2s, s2c, wsp<Rec<double>>(P, lay.src), fa, epart);
  }
  prof_end(P, s);
  if (d_energy) {
    prof_begin(P, FMM_PHASE_ENERGY, s);
    k_energy<<<1, kBlock, 0, s>>>(epart, lay.n_energy_part, d_energy);
    prof_end(P, s);
  }
  return hipGetLastError();
}

}  // namespace fmm
