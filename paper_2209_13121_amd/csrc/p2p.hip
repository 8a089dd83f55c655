// p2p.hip -- P2P near field on source tiles staged in LDS, combination with
// the far field, return to the caller's particle order, and the FP64 energy.
//
// One wave per target leaf t.  The sources of t are the particles of its
// neighbour leaves (uniform tree: the 27 leaves at Chebyshev distance <= 1;
// adaptive tree: the leaves of U(t), t included).  They are staged in LDS in
// tiles of TILE (kTile by default, 128 or 512 by schedule), each source as its
// offset from t's centre in t's box units,
// s_j = o_c + sc_c u_j (o_c the source leaf's centre offset, sc_c its size in
// t's units, u_j the particle's offset in its own leaf, all exact in FP64),
// then every lane reads the tile:
//   * T <= 32 targets: lane = t + T' g (T' the power of two >= T, G = 64 / T'
//     groups); group g takes sources g, g + G, ... of each tile, and the
//     groups' sums are combined by xor shuffles over the lane bits of g, in a
//     fixed order;
//   * T > 32: every lane holds K = ceil(T / 64) <= kKMax targets (lane +
//     64 m) and reads every source of the tile (one LDS broadcast read
//     serves K pairs); leaves above 64 kKMax targets run in groups.
// Mixed precision: s_j and the target's u_i are carried as FP32 pairs
// hi + lo (hi = fp32(x), lo = fp32(x - hi)), so the pair offset
// (u_hi - s_hi) + (u_lo - s_lo) keeps FP32 relative accuracy however close
// the pair; r^2, 1/r and the sums run in FP32.  FP64: the offset u_i - s_j in
// FP64.  The target's own leaf is staged first: its pairs at distance 0 (the
// target itself, or a coincident point, which always shares the leaf)
// contribute nothing, and more than one per target raises the coincident
// flag; pairs with the other leaves skip that check.
// Then phi_i = phi_near + phi_far, F_i = -q_i grad phi_i (FP64), written at
// the particle's user index.  In the adjoint form the same pass writes
// g dE/dq_i = g phi_i and g dE/dx_i = g q_i grad phi_i: with every
// (local <= p, multipole <= p) pair kept, the FMM energy is a symmetric
// quadratic form in q, and while no particle crosses a box face its gradient
// in x_i is q_i grad phi_i.  E = 1/2 sum q_i phi_i is reduced in FP64 in a
// fixed tree order over the per-particle terms.
#include <math.h>

#include <type_traits>

#include "fmm_internal.h"

namespace fmm {
namespace {

constexpr int kTile = 256;   // sources per staged tile (FMM_SCHED_P2P_TILE: 128, 256, 512)
constexpr int kNbBatch = 64;  // neighbour leaves handled per batch (one per lane)
constexpr int kKMax = 4;      // targets per lane of a large leaf (groups of 64 kKMax targets)
// occupancy the register budget is held to: FP32 4 waves per SIMD (128 VGPRs),
// FP64 2 (its targets and sums take twice the registers)
template <typename T>
constexpr int waves_per_simd() { return sizeof(T) == 4 ? 4 : 2; }

// Staged source: mixed, {s_hi, q} and {s_lo, unused}; FP64, {s, q}.
template <typename T>
struct SSrc;
template <>
struct SSrc<float> {
  float4 hq, lo;
};
template <>
struct SSrc<double> {
  double x, y, z, q;
};

// A target in registers: its offset from its leaf centre (box units).
template <typename T>
struct Tgt;
template <>
struct Tgt<float> {
  float xh, yh, zh, xl, yl, zl;
};
template <>
struct Tgt<double> {
  double x, y, z;
};

template <typename T>
struct Acc {
  T f, gx, gy, gz;
  int nz;  // pairs at distance 0 (the target itself included)
};

__device__ __forceinline__ void split2(double v, float& hi, float& lo) {
  hi = (float)v;
  lo = (float)(v - (double)hi);
}

template <typename T>
__device__ __forceinline__ Tgt<T> make_tgt(const Rec<double>& r);
template <>
__device__ __forceinline__ Tgt<float> make_tgt<float>(const Rec<double>& r) {
  Tgt<float> t;
  split2(r.x, t.xh, t.xl);
  split2(r.y, t.yh, t.yl);
  split2(r.z, t.zh, t.zl);
  return t;
}
template <>
__device__ __forceinline__ Tgt<double> make_tgt<double>(const Rec<double>& r) {
  return Tgt<double>{r.x, r.y, r.z};
}

__device__ __forceinline__ float inv_sqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }

// One pair.  SELF: the source may be the target itself or coincide with it
// (sources of the target's own leaf: coincident points share a leaf), so a
// zero distance contributes nothing and is counted; otherwise no check (a
// zero distance there would make the sums non-finite, which finish_particle
// flags).
template <typename T, bool SELF>
__device__ __forceinline__ void pair(Acc<T>& a, const Tgt<T>& t, const SSrc<T>& s) {
  T dx, dy, dz, q;
  if constexpr (sizeof(T) == 4) {
    dx = (t.xh - s.hq.x) + (t.xl - s.lo.x);
    dy = (t.yh - s.hq.y) + (t.yl - s.lo.y);
    dz = (t.zh - s.hq.z) + (t.zl - s.lo.z);
    q = s.hq.w;
  } else {
    dx = t.x - s.x;
    dy = t.y - s.y;
    dz = t.z - s.z;
    q = s.q;
  }
  const T r2 = dx * dx + dy * dy + dz * dz;
  T rinv;
  if constexpr (SELF) {
    const bool z = r2 == T(0);
    rinv = z ? T(0) : inv_sqrt(r2);
    a.nz += z ? 1 : 0;
  } else {
    rinv = inv_sqrt(r2);
  }
  const T qr = q * rinv;
  const T qr3 = qr * rinv * rinv;
  a.f += qr;
  a.gx -= qr3 * dx;
  a.gy -= qr3 * dy;
  a.gz -= qr3 * dz;
}

// One neighbour leaf: particle range and its centre offset / scale in the
// target's box units.
struct Nb {
  uint32_t start, count;
  double ox, oy, oz, sc;
};

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
  double* eterm;  // q_i phi_i per sorted particle (energy), or NULL
};

// phi_i = near + far, F_i = -q_i grad phi_i (or the adjoint outputs), at the
// particle's user index; q_i phi_i into the energy terms.
template <typename T>
__device__ __forceinline__ void finish_particle(const FinishArgs& fa, int64_t i, double inv_h,
                                                const Acc<T>& acc) {
  if (acc.nz > 1 || !isfinite((double)acc.f)) atomicOr(fa.flags, kFlagCoincident);
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
  if (fa.eterm) fa.eterm[i] = qi * phi;
}

// Neighbour leaves of a target leaf.
struct UniformNbs {
  int L;
  const uint32_t* start;  // leaf particle ranges (Hilbert slot order), 8^L + 1
  const uint32_t* c2s;    // leaf level: lexicographic cell -> slot
  const uint32_t* s2c;    // leaf level: slot -> packed cell
  // Target leaf b: its particle range and level; false for no particles.
  __device__ bool target(int64_t b, uint32_t& t0, uint32_t& nt, int& lt) const {
    t0 = start[b];
    nt = start[b + 1] - t0;
    lt = L;
    return nt > 0;
  }
  __device__ int count(int64_t) const { return 27; }
  // neighbour k: the leaf itself first (k = 0), then the other 26
  __device__ Nb get(int64_t b, int k) const {
    int cx, cy, cz;
    unpack_coord(s2c[b], cx, cy, cz);
    const int kk = k == 0 ? 13 : (k <= 13 ? k - 1 : k);  // 13 = (0, 0, 0)
    const int dx = kk / 9 - 1, dy = (kk / 3) % 3 - 1, dz = kk % 3 - 1;
    const int sx = cx + dx, sy = cy + dy, sz = cz + dz, nb = 1 << L;
    Nb r{0, 0, (double)dx, (double)dy, (double)dz, 1.0};
    if (sx >= 0 && sy >= 0 && sz >= 0 && sx < nb && sy < nb && sz < nb) {
      const uint32_t sl = c2s[lex_index(sx, sy, sz, L)];
      r.start = start[sl];
      r.count = start[sl + 1] - r.start;
    }
    return r;
  }
};

// Adaptive tree: boxes in compact order; a leaf's sources are the leaves of
// U(b).  A source leaf c sits at (c_c - c_t) / h_t = (cc + 1/2) 2^(lt - lc) -
// (ct + 1/2) from t in t's units, its offsets scaled by 2^(lt - lc) (exact).
struct AdaptiveNbs {
  const int32_t* level;
  const uint32_t* coord;
  const uint32_t* range;  // {first sorted particle, count} per box
  const int32_t* child0;  // -1 for a leaf
  const uint32_t* uoff;
  const uint32_t* uidx;
  __device__ bool target(int64_t b, uint32_t& t0, uint32_t& nt, int& lt) const {
    if (child0[b] >= 0) return false;
    t0 = range[2 * b];
    nt = range[2 * b + 1];
    lt = level[b];
    return nt > 0;
  }
  __device__ int count(int64_t b) const { return (int)(uoff[b + 1] - uoff[b]); }
  // entry k of U(b) with b itself moved to the front (swapped with entry 0)
  __device__ Nb get(int64_t b, int k) const {
    uint32_t c = uidx[uoff[b] + k];
    if (k == 0)
      c = (uint32_t)b;
    else if (c == (uint32_t)b)
      c = uidx[uoff[b]];
    const int lt = level[b], lc = level[c];
    int ct[3], cc[3];
    unpack_coord(coord[b], ct[0], ct[1], ct[2]);
    unpack_coord(coord[c], cc[0], cc[1], cc[2]);
    const double sc = lt >= lc ? (double)(1 << (lt - lc)) : 1.0 / (double)(1 << (lc - lt));
    Nb r;
    r.start = range[2 * c];
    r.count = range[2 * c + 1];
    r.ox = ((double)cc[0] + 0.5) * sc - ((double)ct[0] + 0.5);
    r.oy = ((double)cc[1] + 0.5) * sc - ((double)ct[1] + 0.5);
    r.oz = ((double)cc[2] + 0.5) * sc - ((double)ct[2] + 0.5);
    r.sc = sc;
    return r;
  }
};

template <typename T>
__device__ __forceinline__ SSrc<T> stage_one(const Rec<double>& r, const Nb& nb);
template <>
__device__ __forceinline__ SSrc<float> stage_one<float>(const Rec<double>& r, const Nb& nb) {
  SSrc<float> s;
  split2(fma(nb.sc, r.x, nb.ox), s.hq.x, s.lo.x);
  split2(fma(nb.sc, r.y, nb.oy), s.hq.y, s.lo.y);
  split2(fma(nb.sc, r.z, nb.oz), s.hq.z, s.lo.z);
  s.hq.w = (float)r.q;
  s.lo.w = 0.f;
  return s;
}
template <>
__device__ __forceinline__ SSrc<double> stage_one<double>(const Rec<double>& r, const Nb& nb) {
  return SSrc<double>{fma(nb.sc, r.x, nb.ox), fma(nb.sc, r.y, nb.oy), fma(nb.sc, r.z, nb.oz), r.q};
}

// Pairs of K targets per lane (targets lane + 64 m) with sources [0, ns) of
// the tile, the first nself of them from the target's own leaf.
template <typename T, int K>
__device__ __forceinline__ void tile_big(Acc<T> (&acc)[kKMax], const Tgt<T> (&tg)[kKMax], const SSrc<T>* sS,
                                         int nself, int ns) {
  for (int j = 0; j < nself; ++j) {
    const SSrc<T> s = sS[j];
#pragma unroll
    for (int m = 0; m < K; ++m) pair<T, true>(acc[m], tg[m], s);
  }
  for (int j = nself; j < ns; ++j) {
    const SSrc<T> s = sS[j];
#pragma unroll
    for (int m = 0; m < K; ++m) pair<T, false>(acc[m], tg[m], s);
  }
}

// LDS of one wave's leaf (TILE sources per staged tile).
template <typename T, int TILE>
struct P2PShared {
  SSrc<T> sS[TILE];
  Nb sNb[kNbBatch];
  uint32_t sPre[kNbBatch + 1];
};

// The near field of target leaf b (one wave).
template <typename T, typename NBS, int TILE>
__device__ __forceinline__ void p2p_leaf(const NBS& nbs, int64_t b, P2PShared<T, TILE>& sh,
                                         const DevParams* __restrict__ dp,
                                         const Rec<double>* __restrict__ src, const FinishArgs& fa) {
  SSrc<T>* sS = sh.sS;
  Nb* sNb = sh.sNb;
  uint32_t* sPre = sh.sPre;
  const int lane = threadIdx.x;
  uint32_t t0, nt;
  int lt;
  if (!nbs.target(b, t0, nt, lt)) return;  // uniform over the wave
  // target layout: small leaves split the sources over lane groups, large
  // ones take up to kKMax targets per lane, in groups of 64 kKMax targets
  // (each group stages the sources again)
  const bool small = nt <= 32;
  int tp = 1;
  while (tp < (int)nt) tp <<= 1;
  const int G = small ? 64 / tp : 1;
  const int gi = small ? lane / tp : 0;  // source group of this lane
  const int nn = nbs.count(b);
  Acc<T> acc[kKMax];
  Tgt<T> tg[kKMax];
  constexpr uint32_t kGrp = 64 * kKMax;
  for (uint32_t g0 = 0; g0 < nt; g0 += kGrp) {
    const int ng = (int)(nt - g0 < kGrp ? nt - g0 : kGrp);  // targets of this group
    const int K = small ? 1 : (ng + 63) / 64;               // targets per lane
#pragma unroll
    for (int m = 0; m < kKMax; ++m) {
      acc[m] = Acc<T>{T(0), T(0), T(0), T(0), 0};
      const int t = small ? lane % tp : lane + 64 * m;
      if (m < K) tg[m] = make_tgt<T>(src[t0 + g0 + (t < ng ? t : 0)]);
    }
    for (int n0 = 0; n0 < nn; n0 += kNbBatch) {
      // neighbour batch: one leaf per lane, the inclusive scan of counts
      const int k = n0 + lane;
      Nb me{0, 0, 0.0, 0.0, 0.0, 1.0};
      if (k < nn) me = nbs.get(b, k);
      uint32_t c = me.count;
#pragma unroll
      for (int w = 1; w < 64; w <<= 1) {
        const uint32_t v = __shfl_up(c, w, 64);
        if (lane >= w) c += v;
      }
      __syncthreads();  // the previous batch's tables and tile are no longer read
      sNb[lane] = me;
      sPre[lane + 1] = c;
      if (lane == 0) sPre[0] = 0;
      const uint32_t total = __shfl(c, 63, 64);
      __syncthreads();
      for (uint32_t c0 = 0; c0 < total; c0 += TILE) {
        const int ns = (int)(total - c0 < (uint32_t)TILE ? total - c0 : (uint32_t)TILE);
        // stage: lane stages sources c0 + lane + 64 m of the batch
        for (int m = lane; m < ns; m += 64) {
          const uint32_t q = c0 + m;
          int lo = 0, hi = kNbBatch;  // sPre[lo] <= q < sPre[hi]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (sPre[mid] <= q)
              lo = mid;
            else
              hi = mid;
          }
          const Nb& nb = sNb[lo];
          sS[m] = stage_one<T>(src[nb.start + (q - sPre[lo])], nb);
        }
        __syncthreads();
        // the target leaf's own sources lead batch 0 (neighbour 0)
        int nself = 0;
        if (n0 == 0 && c0 < nt) nself = nt - c0 < (uint32_t)ns ? (int)(nt - c0) : ns;
        if (small) {
          int j = gi;
          for (; j < nself; j += G) pair<T, true>(acc[0], tg[0], sS[j]);
          for (; j < ns; j += G) pair<T, false>(acc[0], tg[0], sS[j]);
        } else if (K == 1) {
          tile_big<T, 1>(acc, tg, sS, nself, ns);
        } else if (K == 2) {
          tile_big<T, 2>(acc, tg, sS, nself, ns);
        } else {
          tile_big<T, kKMax>(acc, tg, sS, nself, ns);
        }
        __syncthreads();
      }
    }
    if (!small) {
      const double inv_h = (double)(1 << lt) / dp->side;
#pragma unroll
      for (int m = 0; m < kKMax; ++m)
        if (m < K && lane + 64 * m < ng)
          finish_particle<T>(fa, (int64_t)t0 + g0 + lane + 64 * m, inv_h, acc[m]);
    }
  }
  if (!small) return;
  // small leaf: the G groups' sums, combined by xor shuffles over the group bits
  for (int w = tp; w < 64; w <<= 1) {
    acc[0].f += __shfl_xor(acc[0].f, w, 64);
    acc[0].gx += __shfl_xor(acc[0].gx, w, 64);
    acc[0].gy += __shfl_xor(acc[0].gy, w, 64);
    acc[0].gz += __shfl_xor(acc[0].gz, w, 64);
    acc[0].nz += __shfl_xor(acc[0].nz, w, 64);
  }
  if (lane < (int)nt) finish_particle<T>(fa, (int64_t)t0 + lane, (double)(1 << lt) / dp->side, acc[0]);
}

// One wave per box (boxes that are no leaf, or empty, return at once).
template <typename T, typename NBS, int TILE>
__global__ __launch_bounds__(64, waves_per_simd<T>()) void k_p2p(NBS nbs, int64_t nbox, const DevParams* __restrict__ dp,
                                            const Rec<double>* __restrict__ src, FinishArgs fa) {
  __shared__ P2PShared<T, TILE> sh;
  if ((int64_t)blockIdx.x >= nbox) return;
  p2p_leaf<T, NBS, TILE>(nbs, blockIdx.x, sh, dp, src, fa);
}

// Persistent form over a work-list: the non-empty leaves in order of
// decreasing pair count (built at plan time by k_p2p_worklist), taken one at a
// time by resident waves through a ticket counter (zeroed before the launch),
// so the costliest leaves start first and no wave waits for an empty box.
// Every wave leaves once the tickets pass the list's length.  Each leaf's
// outputs are written by its one task in a fixed order, so the result does
// not depend on which wave takes it.
template <typename T, typename NBS, int TILE>
__global__ __launch_bounds__(64, waves_per_simd<T>()) void k_p2p_persistent(
    NBS nbs, const uint32_t* __restrict__ worklist, const uint32_t* __restrict__ ntasks,
    uint32_t* __restrict__ ticket, const DevParams* __restrict__ dp, const Rec<double>* __restrict__ src,
    FinishArgs fa) {
  __shared__ P2PShared<T, TILE> sh;
  const uint32_t n = ntasks[0];
  for (;;) {
    uint32_t t = 0;
    if (threadIdx.x == 0) t = atomicAdd(ticket, 1u);
    t = __shfl(t, 0, 64);
    if (t >= n) break;  // uniform over the wave
    p2p_leaf<T, NBS, TILE>(nbs, worklist[t], sh, dp, src, fa);
    __syncthreads();  // the tile of this leaf is no longer read
  }
}

// Work-list of the adaptive tree's non-empty leaves by decreasing pair count
// n_b sum_{c in U(b)} n_c: a leaf's bucket is the bit length of its count
// (64 buckets, costliest first).  Counts and positions are taken per
// work-group in LDS and reserved in the global buckets by one atomic per
// (work-group, bucket); the order within a bucket only steers the schedule.
__global__ void k_p2p_cost(AdaptiveNbs nbs, int64_t nbox, uint8_t* __restrict__ bucket,
                           uint32_t* __restrict__ hist) {
  __shared__ uint32_t sh[64];
  if (threadIdx.x < 64) sh[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint8_t k = 255;  // not a task
  uint32_t t0, nt;
  int lt;
  if (b < nbox && nbs.target(b, t0, nt, lt)) {
    uint64_t ns = 0;
    const int nn = nbs.count(b);
    for (int j = 0; j < nn; ++j) ns += nbs.range[2 * nbs.uidx[nbs.uoff[b] + j] + 1];
    const uint64_t cost = (uint64_t)nt * ns;
    k = (uint8_t)(63 - __clzll(cost | 1ull));
    atomicAdd(&sh[63 - k], 1u);  // bucket 63 - k: the costliest first
  }
  if (b < nbox) bucket[b] = k;
  __syncthreads();
  if (threadIdx.x < 64 && sh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], sh[threadIdx.x]);
}

// Exclusive scan of the 64 bucket counts (one wave) and the list length.
__global__ void k_p2p_hist_scan(uint32_t* __restrict__ hist, uint32_t* __restrict__ ntasks) {
  const int lane = threadIdx.x;
  uint32_t c = hist[lane];
#pragma unroll
  for (int w = 1; w < 64; w <<= 1) {
    const uint32_t v = __shfl_up(c, w, 64);
    if (lane >= w) c += v;
  }
  hist[lane] = c - hist[lane];  // exclusive
  if (lane == 63) ntasks[0] = c;
}

__global__ void k_p2p_worklist(int64_t nbox, const uint8_t* __restrict__ bucket,
                               uint32_t* __restrict__ hist, uint32_t* __restrict__ worklist) {
  __shared__ uint32_t cnt[64], base[64];
  if (threadIdx.x < 64) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = b < nbox && bucket[b] != 255 ? 63 - bucket[b] : -1;
  const uint32_t r = k >= 0 ? atomicAdd(&cnt[k], 1u) : 0u;
  __syncthreads();
  if (threadIdx.x < 64) base[threadIdx.x] = cnt[threadIdx.x] ? atomicAdd(&hist[threadIdx.x], cnt[threadIdx.x]) : 0u;
  __syncthreads();
  if (k >= 0) worklist[base[k] + r] = (uint32_t)b;
}

// Uniform tree with small leaves: one wave per parent box P (level L - 1),
// the targets being the particles of its 8 children (consecutive Hilbert
// slots 8P .. 8P + 7, so a contiguous particle range).  The sources of all 8
// are the 4 x 4 x 4 leaves around P, staged once in LDS (tiles of
// kGroupTile) as offsets from P's centre in leaf units, leaf by leaf in
// lexicographic order; each target reads the 27 leaves around its own as 9
// runs of 3 leaves adjacent in z, each run's sources contiguous in LDS.  With
// at most 32 targets, lanes t and t + 32 share a target, taking runs 0..4 and
// 5..8, combined by one xor shuffle.  Tiles of 256 sources (8 KB
// of LDS in mixed mode) leave the occupancy to the registers (4 waves per
// SIMD); tiles of 512 held all 64 leaves of a typical block at once but
// limited it to 9 waves per CU: 0.37 -> 0.26 ms at 2^20 charges, depth 6.
constexpr int kGroupTile = 256;
template <typename T>
__global__ __launch_bounds__(64, waves_per_simd<T>()) void k_p2p_group(
    int L, const uint32_t* __restrict__ start, const uint32_t* __restrict__ c2s,
    const uint32_t* __restrict__ s2c, const uint32_t* __restrict__ sorted_leaf,
    const DevParams* __restrict__ dp, const Rec<double>* __restrict__ src, FinishArgs fa) {
  __shared__ SSrc<T> sS[kGroupTile];
  __shared__ uint32_t sPre[65];  // staged order: block leaf k holds [sPre[k], sPre[k + 1])
  __shared__ uint32_t sStart[64];
  const int64_t P = blockIdx.x;
  const int lane = threadIdx.x;
  const uint32_t t0 = start[8 * P], nt = start[8 * P + 8] - t0;
  if (nt == 0) return;  // uniform over the wave
  int px, py, pz;
  unpack_coord(s2c[8 * P], px, py, pz);
  px >>= 1;
  py >>= 1;
  pz >>= 1;
  const int nb = 1 << L;
  // block leaf k = 16 a + 4 b + c at cell (2 px - 1 + a, ...), centre offset
  // from P's centre (a - 1.5, b - 1.5, c - 1.5) leaf units
  const int ba = lane >> 4, bb = (lane >> 2) & 3, bc = lane & 3;
  {
    const int sx = 2 * px - 1 + ba, sy = 2 * py - 1 + bb, sz = 2 * pz - 1 + bc;
    uint32_t st = 0, cnt = 0;
    if (sx >= 0 && sy >= 0 && sz >= 0 && sx < nb && sy < nb && sz < nb) {
      const uint32_t sl = c2s[lex_index(sx, sy, sz, L)];
      st = start[sl];
      cnt = start[sl + 1] - st;
    }
    uint32_t c = cnt;
#pragma unroll
    for (int w = 1; w < 64; w <<= 1) {
      const uint32_t v = __shfl_up(c, w, 64);
      if (lane >= w) c += v;
    }
    sStart[lane] = st;
    sPre[lane + 1] = c;
    if (lane == 0) sPre[0] = 0;
  }
  __syncthreads();
  const uint32_t total = sPre[64];
  const bool split = nt <= 32;
  for (uint32_t g0 = 0; g0 < nt; g0 += (split ? 32u : 64u)) {
    const int t = split ? (lane & 31) : lane;
    const int h = split ? (lane >> 5) : 0;
    const bool live = g0 + t < nt;
    const int64_t i = (int64_t)t0 + g0 + (live ? t : 0);
    // this target's leaf in the block and its offset from P's centre
    int lx, ly, lz;
    unpack_coord(s2c[sorted_leaf[i]], lx, ly, lz);
    lx -= 2 * px - 1;
    ly -= 2 * py - 1;
    lz -= 2 * pz - 1;
    Rec<double> r = src[i];
    r.x += (double)lx - 1.5;
    r.y += (double)ly - 1.5;
    r.z += (double)lz - 1.5;
    const Tgt<T> tg = make_tgt<T>(r);
    const int kown = 16 * lx + 4 * ly + lz;
    Acc<T> acc = {T(0), T(0), T(0), T(0), 0};
    for (uint32_t c0 = 0; c0 < total; c0 += kGroupTile) {
      const uint32_t ns = total - c0 < (uint32_t)kGroupTile ? total - c0 : (uint32_t)kGroupTile;
      __syncthreads();  // the previous tile is no longer read
      for (uint32_t m = lane; m < ns; m += 64) {
        const uint32_t q = c0 + m;
        int lo = 0, hi = 64;  // sPre[lo] <= q < sPre[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (sPre[mid] <= q)
            lo = mid;
          else
            hi = mid;
        }
        const Nb nbk{0, 0, (double)(lo >> 4) - 1.5, (double)((lo >> 2) & 3) - 1.5, (double)(lo & 3) - 1.5, 1.0};
        sS[m] = stage_one<T>(src[sStart[lo] + (q - sPre[lo])], nbk);
      }
      __syncthreads();
      if (live) {
        // the 27 neighbour leaves as 9 runs of 3 consecutive block leaves (dz =
        // -1, 0, 1 for each (dx, dy)), whose sources are contiguous in the
        // staged order; split lanes take runs 0..4 and 5..8
        const int r0 = split ? 5 * h : 0, r1 = split ? (h ? 9 : 5) : 9;
        for (int r = r0; r < r1; ++r) {
          const int k = kown + 16 * (r / 3 - 1) + 4 * (r % 3 - 1) - 1;  // first leaf of the run
          // the run's sources within this tile: [a, e) (empty when e <= a)
          const int a = (int)(sPre[k] > c0 ? sPre[k] : c0) - (int)c0;
          const int e = (int)(sPre[k + 3] < c0 + ns ? sPre[k + 3] : c0 + ns) - (int)c0;
          if (r == 4)  // the run through the target's own leaf (zero distances only there)
            for (int j = a; j < e; ++j) pair<T, true>(acc, tg, sS[j]);
          else
            for (int j = a; j < e; ++j) pair<T, false>(acc, tg, sS[j]);
        }
      }
    }
    if (split) {
      acc.f += __shfl_xor(acc.f, 32, 64);
      acc.gx += __shfl_xor(acc.gx, 32, 64);
      acc.gy += __shfl_xor(acc.gy, 32, 64);
      acc.gz += __shfl_xor(acc.gz, 32, 64);
      acc.nz += __shfl_xor(acc.nz, 32, 64);
    }
    if (live && h == 0) finish_particle<T>(fa, i, (double)nb / dp->side, acc);
  }
}

// E = 1/2 sum q_i phi_i: per-block sums of 4 * kBlock consecutive terms in a
// fixed tree order, then one block over the block sums.
__global__ void k_energy_blocks(const double* __restrict__ eterm, int64_t n, double* __restrict__ part) {
  __shared__ double red[kBlock];
  double s = 0.0;
  const int64_t base = (int64_t)blockIdx.x * 4 * kBlock;
  for (int r = 0; r < 4; ++r) {
    const int64_t i = base + r * kBlock + threadIdx.x;
    if (i < n) s += eterm[i];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
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

namespace {
AdaptiveNbs adaptive_nbs(fmm_plan_s* P) {
  const Layout& lay = P->lay;
  return AdaptiveNbs{wsp<int32_t>(P, lay.a_level), wsp<uint32_t>(P, lay.a_coord),
                     wsp<uint32_t>(P, lay.a_range), wsp<int32_t>(P, lay.a_child0),
                     wsp<uint32_t>(P, lay.a_off), wsp<uint32_t>(P, lay.a_uidx)};
}
// Calls f with std::integral_constant<int, TILE> for the plan's P2P tile.
template <typename F>
void launch_tile(int tile, F&& f) {
  if (tile == 128)
    f(std::integral_constant<int, 128>{});
  else if (tile == 512)
    f(std::integral_constant<int, 512>{});
  else
    f(std::integral_constant<int, kTile>{});
}
}  // namespace

// Plan time (adaptive tree, after its lists): the P2P work-list of the
// persistent form.  Device work only; no read-back.
hipError_t launch_p2p_worklist(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  const int64_t nbox = P->ce_off[P->Ld + 1];
  uint32_t* ctl = wsp<uint32_t>(P, lay.a_p2p_ctl);  // [64] bucket counts, [64] tasks, [65] ticket
  uint8_t* bucket = wsp<uint8_t>(P, lay.a_p2p_bucket);
  hipError_t e = fill_u32(ctl, 66, 0u, s);
  if (e != hipSuccess) return e;
  if (nbox > 0) k_p2p_cost<<<grid_for(nbox, kBlock), kBlock, 0, s>>>(adaptive_nbs(P), nbox, bucket, ctl);
  k_p2p_hist_scan<<<1, 64, 0, s>>>(ctl, ctl + 64);
  if (nbox > 0)
    k_p2p_worklist<<<grid_for(nbox, kBlock), kBlock, 0, s>>>(nbox, bucket, ctl,
                                                               wsp<uint32_t>(P, lay.a_p2p_list));
  return hipGetLastError();
}

hipError_t launch_near_and_finish(fmm_plan_s* P, double* d_phi, double* d_force,
                                  double* d_energy, const double* adj_g, double* dEdq,
                                  double* dEdx, hipStream_t s) {
  const Layout& lay = P->lay;
  const int64_t n = P->n;
  const int L = P->L;
  double* eterm = d_energy ? wsp<double>(P, lay.energy_part) : nullptr;
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
  fa.eterm = eterm;
  const DevParams* dp = wsp<DevParams>(P, lay.params);
  const Rec<double>* src = wsp<Rec<double>>(P, P->mixed ? lay.src64 : lay.src);
  if (P->adaptive) {
    const AdaptiveNbs nb = adaptive_nbs(P);
    const int64_t nbox = P->ce_off[P->Ld + 1];
    if (P->p2p_persistent) {
      // resident waves over the work-list (16 per CU cover the occupancy of
      // both forms; surplus waves find no ticket and leave)
      uint32_t* ticket = wsp<uint32_t>(P, lay.a_p2p_ctl) + 65;
      hipError_t e = fill_u32(ticket, 1, 0u, s);
      if (e != hipSuccess) return e;
      const uint32_t* wl = wsp<uint32_t>(P, lay.a_p2p_list);
      const uint32_t* nt = wsp<uint32_t>(P, lay.a_p2p_ctl) + 64;
      launch_tile(P->p2p_tile, [&](auto tile) {
        constexpr int TL = decltype(tile)::value;
        const unsigned grid = 256 * 16;
        if (P->mixed)
          k_p2p_persistent<float, AdaptiveNbs, TL><<<grid, 64, 0, s>>>(nb, wl, nt, ticket, dp, src, fa);
        else
          k_p2p_persistent<double, AdaptiveNbs, TL><<<grid, 64, 0, s>>>(nb, wl, nt, ticket, dp, src, fa);
      });
    } else {
      launch_tile(P->p2p_tile, [&](auto tile) {
        constexpr int TL = decltype(tile)::value;
        if (P->mixed)
          k_p2p<float, AdaptiveNbs, TL><<<(unsigned)nbox, 64, 0, s>>>(nb, nbox, dp, src, fa);
        else
          k_p2p<double, AdaptiveNbs, TL><<<(unsigned)nbox, 64, 0, s>>>(nb, nbox, dp, src, fa);
      });
    }
  } else {
    UniformNbs nb{L, wsp<uint32_t>(P, lay.leaf_start), wsp<uint32_t>(P, lay.coord2slot) + lay.lvl_off[L],
                  wsp<uint32_t>(P, lay.slot2coord) + lay.lvl_off[L]};
    const int64_t nleaf = lay.nleaf;
    if (L >= 1 && n <= 8 * nleaf) {
      // small leaves (at most 8 particles on average): a wave per parent box
      const int64_t npar = nleaf / 8;
      const uint32_t* sl = wsp<uint32_t>(P, lay.sorted_leaf);
      if (P->mixed)
        k_p2p_group<float><<<(unsigned)npar, 64, 0, s>>>(L, nb.start, nb.c2s, nb.s2c, sl, dp, src, fa);
      else
        k_p2p_group<double><<<(unsigned)npar, 64, 0, s>>>(L, nb.start, nb.c2s, nb.s2c, sl, dp, src, fa);
    } else {
      launch_tile(P->p2p_tile, [&](auto tile) {
        constexpr int TL = decltype(tile)::value;
        if (P->mixed)
          k_p2p<float, UniformNbs, TL><<<(unsigned)nleaf, 64, 0, s>>>(nb, nleaf, dp, src, fa);
        else
          k_p2p<double, UniformNbs, TL><<<(unsigned)nleaf, 64, 0, s>>>(nb, nleaf, dp, src, fa);
      });
    }
  }
  prof_end(P, s);
  if (d_energy) {
    prof_begin(P, FMM_PHASE_ENERGY, s);
    const int64_t nparts = (n + 4 * kBlock - 1) / (4 * kBlock);
    double* part = eterm + n;
    k_energy_blocks<<<(unsigned)nparts, kBlock, 0, s>>>(eterm, n, part);
    k_energy<<<1, kBlock, 0, s>>>(part, nparts, d_energy);
    prof_end(P, s);
  }
  return hipGetLastError();
}

}  // namespace fmm
