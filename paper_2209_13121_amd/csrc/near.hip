// near.hip -- P2P near field, combination with the far field, return to the
// caller's particle order, and the FP64 energy.
//
// For target i in leaf t the near field sums every j != i in the 27 leaves at
// Chebyshev distance <= 1 from t.  Distances are formed in box units from the
// box-local coordinates, x_i - x_j = h ((u_i - u_j) - o) with o the integer
// leaf offset, so FP32 keeps the full relative accuracy of the local offsets.
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
__global__ __launch_bounds__(kBlock) void k_near(
    int64_t n, int L, const DevParams* __restrict__ dp, const uint32_t* __restrict__ sorted_leaf,
    const uint32_t* __restrict__ start, const uint32_t* __restrict__ c2s,
    const uint32_t* __restrict__ s2c, const Rec<T>* __restrict__ src,
    const double* __restrict__ q64, const int32_t* __restrict__ perm, int has_far,
    const double* __restrict__ far_phi, const double* __restrict__ far_grad,
    double* __restrict__ phi_out, double* __restrict__ force_out, double* __restrict__ epart,
    const double* __restrict__ adj_g, double* __restrict__ dEdq, double* __restrict__ dEdx,
    int32_t* __restrict__ flags) {
  __shared__ double red[kBlock];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e_i = 0.0;
  if (i < n) {
    const uint32_t leaf = sorted_leaf[i];
    int cx, cy, cz;
    unpack_coord(s2c[leaf], cx, cy, cz);
    const Rec<T> ri = src[i];
    const T xi = ri.x, yi = ri.y, zi = ri.z;
    T f = T(0), gx = T(0), gy = T(0), gz = T(0);
    bool coincident = false;
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
          const uint32_t b = start[sl], e = start[sl + 1];
          const T ox = xi - T(dx), oy = yi - T(dy), oz = zi - T(dz);
          for (uint32_t j = b; j < e; ++j) {
            if ((int64_t)j == i) continue;
            const Rec<T> rj = src[j];
            const T rx = ox - rj.x, ry = oy - rj.y, rz = oz - rj.z;
            const T r2 = rx * rx + ry * ry + rz * rz;
            if (r2 == T(0)) {
              coincident = true;
              continue;
            }
            const T rinv = inv_sqrt(r2);
            const T qr = rj.q * rinv;
            const T qr3 = qr * rinv * rinv;
            f += qr;
            gx -= qr3 * rx;
            gy -= qr3 * ry;
            gz -= qr3 * rz;
          }
        }
      }
    }
    if (coincident) atomicOr(flags, kFlagCoincident);
    const double inv_h = (double)(1 << L) / dp->side;
    double phi = inv_h * (double)f;
    double g[3] = {inv_h * inv_h * (double)gx, inv_h * inv_h * (double)gy,
                   inv_h * inv_h * (double)gz};
    if (has_far) {
      phi += far_phi[i];
      for (int a = 0; a < 3; ++a) g[a] += far_grad[a * n + i];
    }
    const double qi = q64[i];
    const int64_t u = perm[i];
    if (phi_out) phi_out[u] = phi;
    if (force_out)
      for (int a = 0; a < 3; ++a) force_out[3 * u + a] = -qi * g[a];
    if (adj_g) {  // adjoint: dE/dq_i = phi_i, dE/dx_i = q_i grad phi_i, times g
      const double gs = adj_g[0];
      if (dEdq) dEdq[u] = gs * phi;
      if (dEdx)
        for (int a = 0; a < 3; ++a) dEdx[3 * u + a] = gs * (qi * g[a]);
    }
    e_i = qi * phi;
  }
  if (!epart) return;
  red[threadIdx.x] = e_i;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) epart[blockIdx.x] = red[0];
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
  if (P->mixed)
    k_near<float><<<grid_for(n, kBlock), kBlock, 0, s>>>(
        n, L, wsp<DevParams>(P, lay.params), wsp<uint32_t>(P, lay.sorted_leaf),
        wsp<uint32_t>(P, lay.leaf_start), c2s, s2c, wsp<Rec<float>>(P, lay.src),
        wsp<double>(P, lay.q64), wsp<int32_t>(P, lay.perm), L >= 2,
        wsp<double>(P, lay.far_phi), wsp<double>(P, lay.far_grad), d_phi, d_force, epart, adj_g,
        dEdq, dEdx, wsp<int32_t>(P, lay.flags));
  else
    k_near<double><<<grid_for(n, kBlock), kBlock, 0, s>>>(
        n, L, wsp<DevParams>(P, lay.params), wsp<uint32_t>(P, lay.sorted_leaf),
        wsp<uint32_t>(P, lay.leaf_start), c2s, s2c, wsp<Rec<double>>(P, lay.src),
        wsp<double>(P, lay.q64), wsp<int32_t>(P, lay.perm), L >= 2,
        wsp<double>(P, lay.far_phi), wsp<double>(P, lay.far_grad), d_phi, d_force, epart, adj_g,
        dEdq, dEdx, wsp<int32_t>(P, lay.flags));
  prof_end(P, s);
  if (d_energy) {
    prof_begin(P, FMM_PHASE_ENERGY, s);
    k_energy<<<1, kBlock, 0, s>>>(epart, lay.n_energy_part, d_energy);
    prof_end(P, s);
  }
  return hipGetLastError();
}

}  // namespace fmm
