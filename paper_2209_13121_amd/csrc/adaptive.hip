// adaptive.hip -- the adaptive octree: which boxes exist, their compact
// numbering, the U, W and X lists, and the passes only the adaptive tree has
// (P2M at leaves of any level, P2L over X, M2P over W; L2P at leaves of any
// level is the uniform kernel given each leaf's level, downward.hip).
//
// Tree (Cheng, Greengard & Rokhlin, J. Comput. Phys. 155:468 (1999), sec. 4):
// a box holding more than leaf_max particles is divided into its 8 children
// while its level is below the depth cap L.  The particles are sorted once by
// their level-L Hilbert key (tree.hip), so the box of level l with Hilbert slot
// s holds the sorted range of level-L slots [s 8^(L-l), (s+1) 8^(L-l)), and a
// box exists when every one of its ancestors holds more than leaf_max.  All 8
// children of a divided box exist (an empty child is an empty leaf).  The
// existing boxes are numbered level by level in Hilbert order by an exclusive
// scan over the dense existence flags, so each level is one contiguous block of
// the expansion arrays and the children of a divided box are 8 consecutive
// boxes, in the same order as the uniform tree's slots 8s .. 8s+7.
//
// Lists of a box b ("adjacent": the closed cubes touch, any sizes):
//   U(b), b a leaf: the leaves adjacent to b, b included          -> P2P
//   V(b): existing same-level boxes at the interaction-list offsets -> M2L
//         (looked up by the M2L kernels in the dense map)
//   W(b), b a leaf: boxes finer than b, not adjacent to b, whose parent is
//         adjacent to b                                            -> M2P
//   X(b): leaves coarser than b, adjacent to b's parent, not to b  -> P2L
// Scaling as in the uniform passes: a box's multipole is stored in units of
// its own size h (M~_n = M_n / h^n) and its local expansion as L~_n = L_n h^n,
// so with v = (y - c)/h:
//   P2L  L~_n^m += (1/h) q conj(I_n^m(v))      (added to the M2L result,
//                                                whose 1/h the L2L applies)
//   M2P  phi(x)  = (1/h) sum M~_n^m I_n^m(w),  w = (x - c)/h, gradient 1/h^2
//        from dI_n^m/dz = -I_{n+1}^m, dI_n^m/dx = (I_{n+1}^{m+1} - I_{n+1}^{m-1})/2,
//        dI_n^m/dy = -i (I_{n+1}^{m+1} + I_{n+1}^{m-1})/2.
#include <math.h>

#include <algorithm>

#include "fmm_internal.h"
#include "m2l_common.h"

namespace fmm {
namespace {

struct ATree {
  int L;         // depth cap
  int leaf_max;
  int l0;        // batch level: boxes of level l0 are independent systems (0: one system)
  int64_t nbox;  // existing boxes
  int64_t ls;    // stride of the three lists' count and offset arrays
  int64_t lvl_off[FMM_DEPTH_MAX + 2];  // dense level offsets
  int64_t ce_off[FMM_DEPTH_MAX + 2];   // compact level offsets
  const uint32_t* start;    // level-L slot starts (8^L + 1)
  const uint32_t* c2s;      // dense: lexicographic cell -> Hilbert slot
  const uint32_t* s2c;      // dense: Hilbert slot -> packed cell
  const uint32_t* present;  // dense: the box exists
  const uint32_t* scan;     // dense: compact index of an existing box
  const int32_t* level;     // compact
  const uint32_t* coord;    // compact: packed cell
  const uint32_t* range;    // compact: {first sorted particle, count}
  const int32_t* child0;    // compact: first child or -1
};

__device__ __forceinline__ uint32_t count_of(const uint32_t* start, int L, int l, uint32_t slot) {
  const int sh = 3 * (L - l);
  return start[(uint64_t)(slot + 1) << sh] - start[(uint64_t)slot << sh];
}

// Compact index of the box of level l at cell (x, y, z), or -1.
__device__ __forceinline__ int64_t find_box(const ATree& t, int l, int x, int y, int z) {
  const int nb = 1 << l;
  if (x < 0 || y < 0 || z < 0 || x >= nb || y >= nb || z >= nb) return -1;
  const int64_t g = t.lvl_off[l] + t.c2s[t.lvl_off[l] + lex_index(x, y, z, l)];
  return t.present[g] ? (int64_t)t.scan[g] : -1;
}

// A box of level l holding cnt particles is divided (cnt > leaf_max, or it lies
// above the batch level and is not empty) unless l is the cap.
__device__ __forceinline__ bool divided(const ATree& t, int l, uint32_t cnt) {
  return l < t.L && (cnt > (uint32_t)t.leaf_max || (l < t.l0 && cnt > 0));
}

// Boxes a (level la) and b (level lb) belong to one system: always for a single
// system; for a batch, both at or below the batch level with one ancestor there.
__device__ __forceinline__ bool same_system(const ATree& t, int la, int ax, int ay, int az, int lb,
                                            int bx, int by, int bz) {
  if (t.l0 == 0) return true;
  if (la < t.l0 || lb < t.l0) return false;
  const int sa = la - t.l0, sb = lb - t.l0;
  return (ax >> sa) == (bx >> sb) && (ay >> sa) == (by >> sb) && (az >> sa) == (bz >> sb);
}

// Closed cubes of box a (level la) and box b (level lb >= la) touch.
__device__ __forceinline__ bool touches(int la, int ax, int ay, int az, int lb, int bx, int by, int bz) {
  const int s = lb - la;
  return (ax << s) <= bx + 1 && bx <= ((ax + 1) << s) && (ay << s) <= by + 1 &&
         by <= ((ay + 1) << s) && (az << s) <= bz + 1 && bz <= ((az + 1) << s);
}

// ---- tree ------------------------------------------------------------------

__global__ void k_present(ATree t, int64_t nd, uint32_t* __restrict__ present) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nd) return;
  int l = 0;
  while (l < t.L && g >= t.lvl_off[l + 1]) ++l;
  const uint32_t slot = (uint32_t)(g - t.lvl_off[l]);
  uint32_t ok = 1;
  for (int m = 0; m < l && ok; ++m)
    if (!divided(t, m, count_of(t.start, t.L, m, slot >> (3 * (l - m))))) ok = 0;
  present[g] = ok;
}

__global__ void k_level_offsets(ATree t, uint32_t* __restrict__ out) {
  const int l = threadIdx.x;
  if (l <= t.L + 1) out[l] = t.scan[t.lvl_off[l]];
}

__global__ void k_compact(ATree t, int64_t nd, uint32_t* __restrict__ slot_of,
                          int32_t* __restrict__ level, uint32_t* __restrict__ coord,
                          uint32_t* __restrict__ range, int32_t* __restrict__ child0,
                          uint32_t* __restrict__ parent_of) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nd || !t.present[g]) return;
  int l = 0;
  while (l < t.L && g >= t.lvl_off[l + 1]) ++l;
  const uint32_t slot = (uint32_t)(g - t.lvl_off[l]);
  const int64_t c = t.scan[g];
  const uint32_t cnt = count_of(t.start, t.L, l, slot);
  slot_of[c] = slot;
  level[c] = l;
  coord[c] = t.s2c[g];
  range[2 * c] = t.start[(uint64_t)slot << (3 * (t.L - l))];
  range[2 * c + 1] = cnt;
  int32_t ch = -1;
  if (divided(t, l, cnt)) {
    ch = (int32_t)t.scan[t.lvl_off[l + 1] + 8 * (int64_t)slot];
    parent_of[ch] = (uint32_t)(c - t.ce_off[l]);
  }
  child0[c] = ch;
}

// Leaf of every sorted particle (the first box on its path that is not
// divided) and its offset from the leaf centre in units of the leaf size.
template <typename T>
__global__ void k_gather_adaptive(ATree t, const double* __restrict__ pos,
                                  const int32_t* __restrict__ perm, const uint32_t* __restrict__ keys,
                                  int64_t n, const DevParams* __restrict__ dp,
                                  uint32_t* __restrict__ sorted_leaf, Rec<T>* __restrict__ src,
                                  Rec<double>* __restrict__ src64) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int32_t i = perm[s];
  const uint32_t key = keys[i];
  int l = 0;
  uint32_t slot = 0;
  for (; l <= t.L; ++l) {
    slot = key >> (3 * (t.L - l));
    if (!divided(t, l, count_of(t.start, t.L, l, slot))) break;
  }
  if (l > t.L) l = t.L;
  const int64_t g = t.lvl_off[l] + slot;
  sorted_leaf[s] = t.scan[g];
  int c[3];
  unpack_coord(t.s2c[g], c[0], c[1], c[2]);
  const double h = dp->side / (double)(1 << l);
  double u[3];
  for (int a = 0; a < 3; ++a) {
    double x = pos[3 * (int64_t)i + a];
    if (!isfinite(x)) x = dp->lo[a];
    u[a] = (x - (dp->lo[a] + ((double)c[a] + 0.5) * h)) / h;
  }
  Rec<T> r;
  r.x = (T)u[0];
  r.y = (T)u[1];
  r.z = (T)u[2];
  r.q = T(0);
  src[s] = r;
  if (src64) src64[s] = Rec<double>{u[0], u[1], u[2], 0.0};
}

// ---- M2L work lists -------------------------------------------------------------

struct VLevels {
  int64_t ndiv[FMM_DEPTH_MAX + 2];     // divided parents of level l - 1 (targets per class)
  int64_t tgt_off[FMM_DEPTH_MAX + 2];
  int64_t vt_off[FMM_DEPTH_MAX + 2];
};

// Class pi of a box is the parity of its cell; the k-th divided parent of
// level l - 1 owns rows 8k .. 8k+7 of level l, one of each class.
__global__ void k_m2l_targets(ATree t, VLevels v, uint32_t* __restrict__ tgt) {
  const int64_t r = t.ce_off[2] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= t.nbox) return;
  const int l = t.level[r];
  int x, y, z;
  unpack_coord(t.coord[r], x, y, z);
  const int pi = ((x & 1) << 2) | ((y & 1) << 1) | (z & 1);
  const int64_t rel = r - t.ce_off[l];
  tgt[v.tgt_off[l] + pi * v.ndiv[l] + rel / 8] = (uint32_t)rel;
}

// Source row of every (tile, class, offset, target) of level l: the existing
// box of level l at target - d (d the class's offset), or kAbsent.
__global__ void k_m2l_sources(ATree t, VLevels v, int l, int64_t nent, const uint32_t* __restrict__ tgt,
                              uint32_t* __restrict__ vtab) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nent) return;
  const int tix = (int)(e % m2l::kTargetsPerGroup);
  int64_t rest = e / m2l::kTargetsPerGroup;
  const int i = (int)(rest % kIL);
  rest /= kIL;
  const int pi = (int)(rest % 8);
  const int64_t tile = rest / 8;
  const int64_t ps = tile * m2l::kTargetsPerGroup + tix;
  uint32_t out = m2l::kAbsent;
  if (ps < v.ndiv[l]) {
    const uint32_t trow = tgt[v.tgt_off[l] + pi * v.ndiv[l] + ps];
    int x, y, z, dx, dy, dz;
    unpack_coord(t.coord[t.ce_off[l] + trow], x, y, z);
    m2l::il_offset(pi, i, dx, dy, dz);
    if (same_system(t, l, x - dx, y - dy, z - dz, l, x, y, z)) {
      const int64_t c = find_box(t, l, x - dx, y - dy, z - dz);
      if (c >= 0) out = (uint32_t)(c - t.ce_off[l]);
    }
  }
  vtab[v.vt_off[l] + e] = out;
}

// ---- lists -------------------------------------------------------------------

constexpr int kStack = 80;  // depth-first stack: at most 7 per level below the leaf + 8

// FILL = false: counts per box into cnt[list * ls + b];
// FILL = true: entries at off[...] (the exclusive scan of the counts).
template <bool FILL>
__global__ void k_lists(ATree t, uint32_t* __restrict__ cnt, const uint32_t* __restrict__ off,
                        uint32_t* __restrict__ uidx, uint32_t* __restrict__ widx,
                        uint32_t* __restrict__ xidx, int32_t* __restrict__ flags) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= t.nbox) return;
  const int64_t nb1 = t.ls;
  const int l = t.level[b];
  int bx, by, bz;
  unpack_coord(t.coord[b], bx, by, bz);
  uint32_t nu = 0, nw = 0, nx = 0;
  uint32_t *pu = nullptr, *pw = nullptr, *px = nullptr;
  if (FILL) {
    pu = uidx + off[b];
    pw = widx + off[nb1 + b];
    px = xidx + off[2 * nb1 + b];
  }
  if (t.child0[b] < 0) {
    // coarser leaves touching b: at level m the candidates per axis are
    // (c - 1) >> s .. (c + 1) >> s, s = l - m
    for (int m = 0; m < l; ++m) {
      const int s = l - m, top = (1 << m) - 1;
      const int x0 = max(0, (bx - 1) >> s), x1 = min(top, (bx + 1) >> s);
      const int y0 = max(0, (by - 1) >> s), y1 = min(top, (by + 1) >> s);
      const int z0 = max(0, (bz - 1) >> s), z1 = min(top, (bz + 1) >> s);
      for (int x = x0; x <= x1; ++x)
        for (int y = y0; y <= y1; ++y)
          for (int z = z0; z <= z1; ++z) {
            if (!same_system(t, m, x, y, z, l, bx, by, bz)) continue;
            const int64_t c = find_box(t, m, x, y, z);
            if (c < 0 || t.child0[c] >= 0 || !touches(m, x, y, z, l, bx, by, bz)) continue;
            if (FILL) pu[nu] = (uint32_t)c;
            ++nu;
          }
    }
    // same level, then the finer boxes below divided neighbours
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          if (!same_system(t, l, bx + dx, by + dy, bz + dz, l, bx, by, bz)) continue;
          const int64_t c = find_box(t, l, bx + dx, by + dy, bz + dz);
          if (c < 0) continue;
          if (t.child0[c] < 0) {
            if (FILL) pu[nu] = (uint32_t)c;
            ++nu;
            continue;
          }
          int32_t stack[kStack];
          int sp = 0;
          stack[sp++] = (int32_t)c;
          while (sp > 0) {
            const int32_t d = stack[--sp];
            for (int k = 0; k < 8; ++k) {
              const int32_t e = t.child0[d] + k;
              int ex, ey, ez;
              unpack_coord(t.coord[e], ex, ey, ez);
              if (!touches(l, bx, by, bz, t.level[e], ex, ey, ez)) {
                if (FILL) pw[nw] = (uint32_t)e;
                ++nw;
              } else if (t.child0[e] < 0) {
                if (FILL) pu[nu] = (uint32_t)e;
                ++nu;
              } else if (sp < kStack) {
                stack[sp++] = e;
              } else {
                atomicOr(flags, kFlagListOverflow);
              }
            }
          }
        }
  }
  if (l >= 2) {
    // coarser leaves touching the parent but not b
    const int px0 = bx >> 1, py0 = by >> 1, pz0 = bz >> 1;
    for (int m = 0; m < l; ++m) {
      const int s = l - 1 - m, top = (1 << m) - 1;
      const int x0 = max(0, (px0 - 1) >> s), x1 = min(top, (px0 + 1) >> s);
      const int y0 = max(0, (py0 - 1) >> s), y1 = min(top, (py0 + 1) >> s);
      const int z0 = max(0, (pz0 - 1) >> s), z1 = min(top, (pz0 + 1) >> s);
      for (int x = x0; x <= x1; ++x)
        for (int y = y0; y <= y1; ++y)
          for (int z = z0; z <= z1; ++z) {
            if (!same_system(t, m, x, y, z, l, bx, by, bz)) continue;
            const int64_t c = find_box(t, m, x, y, z);
            if (c < 0 || t.child0[c] >= 0 || touches(m, x, y, z, l, bx, by, bz)) continue;
            if (FILL) px[nx] = (uint32_t)c;
            ++nx;
          }
    }
  }
  if (!FILL) {
    cnt[b] = nu;
    cnt[nb1 + b] = nw;
    cnt[2 * nb1 + b] = nx;
  }
}

__global__ void k_flag_nonzero(const uint32_t* __restrict__ cnt, int64_t n, uint32_t* __restrict__ flag) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n) flag[b] = cnt[b] ? 1u : 0u;
}

__global__ void k_compact_nonzero(const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ pos,
                                  int64_t n, uint32_t* __restrict__ list) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n && cnt[b]) list[pos[b]] = (uint32_t)b;
}

// Tree statistics: [0] leaves, [1] V entries, [2] M2L pairs of non-empty
// boxes, [3] ordered P2P pairs + n (sum over leaves of n_b * sum_U n_c).
__global__ void k_stats(ATree t, const uint32_t* __restrict__ off, const uint32_t* __restrict__ uidx,
                        unsigned long long* __restrict__ st) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= t.nbox) return;
  const int l = t.level[b];
  const uint32_t nb_ = t.range[2 * b + 1];
  int x, y, z;
  unpack_coord(t.coord[b], x, y, z);
  if (l >= 2) {
    unsigned long long v = 0, vn = 0;
    for (int dx = -3; dx <= 3; ++dx)
      for (int dy = -3; dy <= 3; ++dy)
        for (int dz = -3; dz <= 3; ++dz) {
          if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) continue;
          const int sx = x + dx, sy = y + dy, sz = z + dz;
          if (abs((sx >> 1) - (x >> 1)) > 1 || abs((sy >> 1) - (y >> 1)) > 1 ||
              abs((sz >> 1) - (z >> 1)) > 1)
            continue;
          if (!same_system(t, l, sx, sy, sz, l, x, y, z)) continue;
          const int64_t c = find_box(t, l, sx, sy, sz);
          if (c < 0) continue;
          ++v;
          if (nb_ && t.range[2 * c + 1]) ++vn;
        }
    atomicAdd(&st[1], v);
    atomicAdd(&st[2], vn);
  }
  if (t.child0[b] < 0) {
    atomicAdd(&st[0], 1ull);
    unsigned long long src = 0;
    for (uint32_t k = off[b]; k < off[b + 1]; ++k) src += t.range[2 * uidx[k] + 1];
    atomicAdd(&st[3], (unsigned long long)nb_ * src);
  }
}

__global__ void k_zero_stats(unsigned long long* st) {
  if (threadIdx.x < 8) st[threadIdx.x] = 0ull;
}

// ---- harmonics -------------------------------------------------------------

// Irregular solid harmonics I_n^m(x) = (n-m)! P_n^m(cos t) e^{i m f} / r^{n+1}
// (Condon-Shortley phase; Epton & Dembart, SIAM J. Sci. Comput. 16:865 (1995))
// for 0 <= m <= n <= Q, by the recurrences
//   I_0^0 = 1/r,  I_m^m = -(2m-1)(x + i y)/r^2 I_{m-1}^{m-1},
//   I_{m+1}^m = (2m+1) z/r^2 I_m^m,
//   r^2 I_n^m = (2n-1) z I_{n-1}^m - (n+m-1)(n-m-1) I_{n-2}^m;
// outputs indexed by tri(n, m).
template <int Q, typename T>
__device__ __forceinline__ void irregular_harmonics(T x, T y, T z, T* re, T* im) {
  const T r2 = x * x + y * y + z * z;
  const T ir2 = T(1) / r2;
  re[0] = T(1) / sqrt(r2);
  im[0] = T(0);
#pragma unroll
  for (int m = 0; m <= Q; ++m) {
    if (m > 0) {
      const T s = T(-(2.0 * m - 1.0)) * ir2;
      const T pr = re[tri(m - 1, m - 1)], pi = im[tri(m - 1, m - 1)];
      re[tri(m, m)] = s * (x * pr - y * pi);
      im[tri(m, m)] = s * (x * pi + y * pr);
    }
    if (m + 1 <= Q) {
      const T s = T(2.0 * m + 1.0) * z * ir2;
      re[tri(m + 1, m)] = s * re[tri(m, m)];
      im[tri(m + 1, m)] = s * im[tri(m, m)];
    }
#pragma unroll
    for (int n = m + 2; n <= Q; ++n) {
      const T a = T(2.0 * n - 1.0) * z, b = T((double)(n + m - 1) * (double)(n - m - 1));
      re[tri(n, m)] = (a * re[tri(n - 1, m)] - b * re[tri(n - 2, m)]) * ir2;
      im[tri(n, m)] = (a * im[tri(n - 1, m)] - b * im[tri(n - 2, m)]) * ir2;
    }
  }
}

// The same values, in the same order and arithmetic, handed to f(n, m, re, im)
// as the recurrence produces them, so that only its last two terms stay live.
template <int Q, typename T, typename F>
__device__ __forceinline__ void irregular_harmonics_each(T x, T y, T z, F&& f) {
  const T r2 = x * x + y * y + z * z;
  const T ir2 = T(1) / r2;
  T dre = T(1) / sqrt(r2), dim = T(0);  // I_m^m
  f(0, 0, dre, dim);
#pragma unroll
  for (int m = 0; m <= Q; ++m) {
    if (m > 0) {
      const T s = T(-(2.0 * m - 1.0)) * ir2;
      const T nre = s * (x * dre - y * dim);
      const T nim = s * (x * dim + y * dre);
      dre = nre;
      dim = nim;
      f(m, m, dre, dim);
    }
    if (m + 1 <= Q) {
      const T s = T(2.0 * m + 1.0) * z * ir2;
      T p1re = s * dre, p1im = s * dim, p0re = dre, p0im = dim;
      f(m + 1, m, p1re, p1im);
#pragma unroll
      for (int n = m + 2; n <= Q; ++n) {
        const T a = T(2.0 * n - 1.0) * z, b = T((double)(n + m - 1) * (double)(n - m - 1));
        const T cre = (a * p1re - b * p0re) * ir2;
        const T cim = (a * p1im - b * p0im) * ir2;
        f(n, m, cre, cim);
        p0re = p1re;
        p0im = p1im;
        p1re = cre;
        p1im = cim;
      }
    }
  }
}

// ---- passes ------------------------------------------------------------------

// P2M at the leaves of levels >= 2, accumulated in FP64 from the FP64
// offsets (as in the uniform pass); the mixed mode also stores it in FP32.
template <int P>
__global__ __launch_bounds__(64) void k_p2m_adaptive(ATree t, const Rec<double>* __restrict__ src,
                                                     double* __restrict__ mult64, float* __restrict__ mult32) {
  typedef double T;
  constexpr int NC = (P + 1) * (P + 1);
  constexpr int MS = mstride_of(NC);
  constexpr int NT = (P + 1) * (P + 2) / 2;
  const int64_t b = t.ce_off[2] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= t.nbox || t.child0[b] >= 0) return;
  T acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = T(0);
  const uint32_t s0 = t.range[2 * b], s1 = s0 + t.range[2 * b + 1];
  for (uint32_t s = s0; s < s1; ++s) {
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
  double* out = mult64 + b * MS;
#pragma unroll
  for (int c = 0; c < MS; ++c) out[c] = c < NC ? acc[c] : T(0);
  if (mult32) {
    float* o32 = mult32 + b * MS;
#pragma unroll
    for (int c = 0; c < MS; ++c) o32[c] = c < NC ? (float)acc[c] : 0.f;
  }
}

// Sum over the 64 lanes of a wave of N values per lane (N a power of two,
// >= 64), by halving: at each step the lanes exchange half of what they still
// hold with the partner lane w apart, the lanes with bit w set keeping the
// upper half.  Afterwards lane L holds in v[0 .. N/64) the sums of the values
// N/64 L .. N/64 L + N/64 - 1.  N - 2 shuffles instead of 6 N, in a fixed order.
template <int H, int W, typename T>
__device__ __forceinline__ void halve_exchange(T* v) {
  const bool up = (threadIdx.x & W) != 0;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const T send = up ? v[i] : v[i + H];
    const T keep = up ? v[i + H] : v[i];
    v[i] = keep + __shfl_xor(send, W);
  }
}
template <int N, typename T>
__device__ __forceinline__ void wave_sum_split(T* v) {
  static_assert(N >= 64 && (N & (N - 1)) == 0, "N must be a power of two >= 64");
  halve_exchange<N / 2, 32>(v);
  halve_exchange<N / 4, 16>(v);
  halve_exchange<N / 8, 8>(v);
  halve_exchange<N / 16, 4>(v);
  halve_exchange<N / 32, 2>(v);
  halve_exchange<N / 64, 1>(v);
}

// Coefficients of degree <= p whose order m lies in [m0, m1), in the order of
// the global index (cidx_re / cidx_im): their number, and the position of one
// of them in that list.
__host__ __device__ constexpr int orders_count(int p, int m0, int m1) {
  int c = 0;
  for (int n = 0; n <= p; ++n)
    for (int m = m0; m < m1 && m <= n; ++m) c += m ? 2 : 1;
  return c;
}
__host__ __device__ constexpr int orders_pos(int m0, int m1, int n, int m, bool im) {
  int c = 0;
  for (int nn = 0; nn < n; ++nn)
    for (int mm = m0; mm < m1 && mm <= nn; ++mm) c += mm ? 2 : 1;
  for (int mm = m0; mm < m; ++mm) c += mm ? 2 : 1;
  return c + (im ? 1 : 0);
}
// Split of the orders 0..p into [0, m) and [m, p]: the m that halves the
// coefficients most evenly.
__host__ __device__ constexpr int orders_split(int p) {
  int best = 1;
  for (int m = 1; m <= p; ++m) {
    const int a = 2 * orders_count(p, 0, m) - (p + 1) * (p + 1);
    const int b = 2 * orders_count(p, 0, best) - (p + 1) * (p + 1);
    if ((a < 0 ? -a : a) < (b < 0 ? -b : b)) best = m;
  }
  return best;
}

// P2L over X(b), added to the M2L result of b (units before the 1/h of L2L):
// q conj(I_n^m(v)) with v the source's offset from b's centre in b's units,
// for the orders m in [M0, M1) (the coefficients are split over two launches
// by order, so that a lane holds fewer sums and more waves fit a SIMD).
// One wave per box of the compact list xbox (the boxes whose X list is not
// empty).  The lanes take the (X entry, particle) pairs of the list in order,
// 64 at a time, so a short leaf does not leave lanes idle; each lane keeps its
// own partial expansion, and the wave sums them at the end (wave_sum_split).
template <int P, typename T, int M0, int M1>
__global__ __launch_bounds__(64) void k_p2l(ATree t, const uint32_t* __restrict__ xbox,
                                            const uint32_t* __restrict__ xoff,
                                            const uint32_t* __restrict__ xidx,
                                            const Rec<T>* __restrict__ src, T* __restrict__ m2l) {
  constexpr int NC = (P + 1) * (P + 1);
  constexpr int NA = orders_count(P, M0, M1);
  constexpr int N = NA <= 64 ? 64 : (NA <= 128 ? 128 : 256);
  constexpr int R = N / 64;
  const int lane = threadIdx.x;
  const int64_t b = xbox[blockIdx.x];
  const uint32_t k0 = xoff[b], k1 = xoff[b + 1];
  const int l = t.level[b];
  int bc[3];
  unpack_coord(t.coord[b], bc[0], bc[1], bc[2]);
  T acc[N];
#pragma unroll
  for (int c = 0; c < N; ++c) acc[c] = T(0);
  // lane state: the X entry k of its current pair and the pairs before entry k
  uint32_t k = k0, before = 0;
  uint32_t cnt = k < k1 ? t.range[2 * xidx[k] + 1] : 0;
  for (uint32_t base = 0;; base += 64) {
    const uint32_t j = base + lane;
    while (k < k1 && j >= before + cnt) {
      before += cnt;
      ++k;
      cnt = k < k1 ? t.range[2 * xidx[k] + 1] : 0;
    }
    const bool active = k < k1;
    if (!__any(active)) break;
    if (active) {
      const uint32_t c = xidx[k];
      const int lc = t.level[c];  // < l
      int cc[3];
      unpack_coord(t.coord[c], cc[0], cc[1], cc[2]);
      // centre offset in b's units: ((cc + 1/2) 2^(l - lc) - (bc + 1/2)), exact
      const double sc = (double)(1 << (l - lc));
      const T ox = (T)(((double)cc[0] + 0.5) * sc - ((double)bc[0] + 0.5));
      const T oy = (T)(((double)cc[1] + 0.5) * sc - ((double)bc[1] + 0.5));
      const T oz = (T)(((double)cc[2] + 0.5) * sc - ((double)bc[2] + 0.5));
      const T sg = (T)sc;
      const Rec<T> r = src[t.range[2 * c] + (j - before)];
      irregular_harmonics_each<P, T>(
          ox + sg * r.x, oy + sg * r.y, oz + sg * r.z, [&](int nn, int m, T re, T im) {
            if (m < M0 || m >= M1) return;
            acc[orders_pos(M0, M1, nn, m, false)] += r.q * re;
            if (m) acc[orders_pos(M0, M1, nn, m, true)] -= r.q * im;
          });
    }
  }
  wave_sum_split<N>(acc);
  // local index u -> global coefficient index
  T* o = m2l + b * NC;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int u = R * lane + i;
    if (u >= NA) continue;
    int c = 0, seen = 0;
    for (int nn = 0; nn <= P; ++nn) {
      const int here = orders_count(nn, M0, M1) - orders_count(nn - 1, M0, M1);
      if (u < seen + here) {
        const int v = u - seen;  // position within degree nn: m0 (re[, im]), m0 + 1 ...
        const int m = M0 == 0 ? (v + 1) / 2 : M0 + v / 2;
        const bool im = M0 == 0 ? (v > 0 && v % 2 == 0) : (v % 2 == 1);
        c = im ? cidx_im(nn, m) : cidx_re(nn, m);
        break;
      }
      seen += here;
    }
    o[c] += acc[i];
  }
}

// M2P over the W list of a leaf, added to the far field L2P wrote: one
// work-group of kM2pWaves waves per leaf of the compact list wbox (the leaves
// whose W list is not empty), a lane per particle (64 at a time).  Wave v
// takes the W entries v, v + kM2pWaves, ... in list order, so all lanes of a
// wave read the same multipole at once; the waves' sums are added in wave
// order through LDS.
constexpr int kM2pWaves = 4;
template <int P, typename T>
__global__ __launch_bounds__(64 * kM2pWaves, sizeof(T) == 4 && P <= 10 ? 2 : 1) void k_m2p(ATree t, const uint32_t* __restrict__ wbox,
                                            const Rec<T>* __restrict__ src, int64_t n,
                                            const DevParams* __restrict__ dp,
                                            const T* __restrict__ mult,
                                            const uint32_t* __restrict__ woff,
                                            const uint32_t* __restrict__ widx,
                                            double* __restrict__ far_phi,
                                            double* __restrict__ far_grad) {
  constexpr int MS = mstride_of((P + 1) * (P + 1));
  constexpr int NT1 = (P + 2) * (P + 3) / 2;
  __shared__ double red[kM2pWaves][4][64];
  // the wave index, uniform over the wave (so the multipole reads stay scalar)
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t leaf = wbox[blockIdx.x];  // a leaf whose W list is not empty
  const uint32_t k0 = woff[leaf], k1 = woff[leaf + 1];
  const uint32_t s0 = t.range[2 * leaf], cnt = t.range[2 * leaf + 1];
  const int l = t.level[leaf];
  for (uint32_t base = 0; base < cnt; base += 64) {
    const uint32_t j = base + lane;
    const bool active = j < cnt;
    const int64_t s = s0 + (active ? j : 0);
    const Rec<T> r = src[s];
    double phi = 0.0, g[3] = {0.0, 0.0, 0.0};
    int lc[3];
    unpack_coord(t.coord[leaf], lc[0], lc[1], lc[2]);
    for (uint32_t k = k0 + wv; k < k1; k += kM2pWaves) {
      const uint32_t w = widx[k];
      const int lw = t.level[w];  // > l
      int wc[3];
      unpack_coord(t.coord[w], wc[0], wc[1], wc[2]);
      // the particle's offset from w's centre in w's units, from the leaf-unit
      // offset u: (leaf centre - w centre)/h_w + u h_leaf/h_w, the centre part exact
      const double sc = (double)(1 << (lw - l));
      const T vx = (T)(((double)lc[0] + 0.5) * sc - ((double)wc[0] + 0.5)) + (T)sc * r.x;
      const T vy = (T)(((double)lc[1] + 0.5) * sc - ((double)wc[1] + 0.5)) + (T)sc * r.y;
      const T vz = (T)(((double)lc[2] + 0.5) * sc - ((double)wc[2] + 0.5)) + (T)sc * r.z;
      T re[NT1], im[NT1];
      irregular_harmonics<P + 1, T>(vx, vy, vz, re, im);
      const T* Mw = mult + (int64_t)w * MS;
      T f = T(0), gx = T(0), gy = T(0), gz = T(0);
      // I_{n+1}^{m-1} at m = 0 is I_{n+1}^{-1} = -conj(I_{n+1}^1)
      auto ir = [&](int nn, int m) { return m >= 0 ? re[tri(nn, m)] : -re[tri(nn, 1)]; };
      auto ii = [&](int nn, int m) { return m >= 0 ? im[tri(nn, m)] : im[tri(nn, 1)]; };
  #pragma unroll
      for (int nn = 0; nn <= P; ++nn) {
  #pragma unroll
        for (int m = 0; m <= nn; ++m) {
          const T mr = Mw[cidx_re(nn, m)];
          const T mi = m ? Mw[cidx_im(nn, m)] : T(0);
          const T wgt = m ? T(2) : T(1);  // the negative orders are the conjugates
          // Re(M I_n^m)
          f += wgt * (mr * re[tri(nn, m)] - mi * im[tri(nn, m)]);
          // d/dx: M (I_{n+1}^{m+1} - I_{n+1}^{m-1}) / 2
          const T dxr = T(0.5) * (re[tri(nn + 1, m + 1)] - ir(nn + 1, m - 1));
          const T dxi = T(0.5) * (im[tri(nn + 1, m + 1)] - ii(nn + 1, m - 1));
          gx += wgt * (mr * dxr - mi * dxi);
          // d/dy: M (-i/2)(I_{n+1}^{m+1} + I_{n+1}^{m-1}); (-i/2)(a + i b) = b/2 - i a/2
          const T sr = re[tri(nn + 1, m + 1)] + ir(nn + 1, m - 1);
          const T si = im[tri(nn + 1, m + 1)] + ii(nn + 1, m - 1);
          gy += wgt * (mr * (T(0.5) * si) - mi * (T(-0.5) * sr));
          // d/dz: -M I_{n+1}^m
          gz -= wgt * (mr * re[tri(nn + 1, m)] - mi * im[tri(nn + 1, m)]);
        }
      }
      const double inv_hw = (double)(1 << lw) / dp->side;
      phi += inv_hw * (double)f;
      g[0] += inv_hw * inv_hw * (double)gx;
      g[1] += inv_hw * inv_hw * (double)gy;
      g[2] += inv_hw * inv_hw * (double)gz;
    }
    red[wv][0][lane] = phi;
    red[wv][1][lane] = g[0];
    red[wv][2][lane] = g[1];
    red[wv][3][lane] = g[2];
    __syncthreads();
    if (wv == 0 && active) {
      double v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v[q] = red[0][q][lane];
#pragma unroll
        for (int w = 1; w < kM2pWaves; ++w) v[q] += red[w][q][lane];
      }
      far_phi[s] += v[0];
      far_grad[s] += v[1];
      far_grad[n + s] += v[2];
      far_grad[2 * n + s] += v[3];
    }
    __syncthreads();
  }
}

ATree tree_view(fmm_plan_s* P) {
  const Layout& lay = P->lay;
  ATree t;
  t.L = P->L;
  t.leaf_max = P->cfg.leaf_max;
  t.l0 = P->cfg.batch_level;
  t.nbox = P->ce_off[P->L + 1];
  t.ls = lay.bmax + 1;
  for (int l = 0; l <= FMM_DEPTH_MAX + 1; ++l) {
    t.lvl_off[l] = lay.lvl_off[l];
    t.ce_off[l] = P->ce_off[l];
  }
  t.start = wsp<uint32_t>(P, lay.leaf_start);
  t.c2s = wsp<uint32_t>(P, lay.coord2slot);
  t.s2c = wsp<uint32_t>(P, lay.slot2coord);
  t.present = wsp<uint32_t>(P, lay.a_present);
  t.scan = wsp<uint32_t>(P, lay.a_scan);
  t.level = wsp<int32_t>(P, lay.a_level);
  t.coord = wsp<uint32_t>(P, lay.a_coord);
  t.range = wsp<uint32_t>(P, lay.a_range);
  t.child0 = wsp<int32_t>(P, lay.a_child0);
  return t;
}

template <int P>
struct P2MAdaptiveRun {
  static hipError_t run(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    const ATree t = tree_view(Pl);
    const int64_t nb = t.nbox - t.ce_off[2];
    if (nb <= 0) return hipGetLastError();
    k_p2m_adaptive<P><<<grid_for(nb, 64), 64, 0, s>>>(
        t, wsp<Rec<double>>(Pl, Pl->mixed ? lay.src64 : lay.src), wsp<double>(Pl, lay.mult64),
        Pl->mixed ? wsp<float>(Pl, lay.mult32) : nullptr);
    return hipGetLastError();
  }
};

template <int P>
struct P2LRun {
  static hipError_t run(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    const ATree t = tree_view(Pl);
    const uint32_t* xoff = wsp<uint32_t>(Pl, lay.a_off) + 2 * (lay.bmax + 1);
    if (Pl->nxbox == 0) return hipGetLastError();
    const unsigned nx = (unsigned)Pl->nxbox;  // one wave per box with an X list
    const uint32_t* xbox = wsp<uint32_t>(Pl, lay.a_xbox);
    // FP32: two launches, over the orders below and from the split (p >= 6),
    // which took the clusters P2L at p = 10 from 1 to 3 waves per SIMD and
    // 1.6 to 1.4 ms; FP64 stays at one wave per SIMD either way, and there the
    // second pass over the pairs made it slower (2.3 -> 4.4 ms), so one launch
    constexpr int MS = P >= 6 ? orders_split(P) : P + 1;
    if (Pl->mixed) {
      k_p2l<P, float, 0, MS><<<nx, 64, 0, s>>>(t, xbox, xoff, wsp<uint32_t>(Pl, lay.a_xidx),
                                               wsp<Rec<float>>(Pl, lay.src), wsp<float>(Pl, lay.m2l_out));
      if (MS <= P)
        k_p2l<P, float, MS, P + 1><<<nx, 64, 0, s>>>(t, xbox, xoff, wsp<uint32_t>(Pl, lay.a_xidx),
                                                     wsp<Rec<float>>(Pl, lay.src), wsp<float>(Pl, lay.m2l_out));
    } else {
      k_p2l<P, double, 0, P + 1><<<nx, 64, 0, s>>>(t, xbox, xoff, wsp<uint32_t>(Pl, lay.a_xidx),
                                                   wsp<Rec<double>>(Pl, lay.src), wsp<double>(Pl, lay.m2l_out));
    }
    return hipGetLastError();
  }
};

template <int P>
struct M2PRun {
  static hipError_t run(fmm_plan_s* Pl, hipStream_t s) {
    const Layout& lay = Pl->lay;
    if (Pl->nlist[1] == 0) return hipGetLastError();
    const ATree t = tree_view(Pl);
    const uint32_t* woff = wsp<uint32_t>(Pl, lay.a_off) + (lay.bmax + 1);
    const int64_t n = Pl->n;
    const DevParams* dp = wsp<DevParams>(Pl, lay.params);
    const unsigned nb = (unsigned)Pl->nwbox;  // one work-group per leaf with a W list
    const uint32_t* wbox = wsp<uint32_t>(Pl, lay.a_wbox);
    if (Pl->mixed)
      k_m2p<P, float><<<nb, 64 * kM2pWaves, 0, s>>>(t, wbox, wsp<Rec<float>>(Pl, lay.src), n, dp,
                                        wsp<float>(Pl, lay.mult32), woff, wsp<uint32_t>(Pl, lay.a_widx),
                                        wsp<double>(Pl, lay.far_phi), wsp<double>(Pl, lay.far_grad));
    else
      k_m2p<P, double><<<nb, 64 * kM2pWaves, 0, s>>>(t, wbox, wsp<Rec<double>>(Pl, lay.src), n, dp,
                                         wsp<double>(Pl, lay.mult64), woff, wsp<uint32_t>(Pl, lay.a_widx),
                                         wsp<double>(Pl, lay.far_phi), wsp<double>(Pl, lay.far_grad));
    return hipGetLastError();
  }
};

}  // namespace

hipError_t launch_adaptive_tree(fmm_plan_s* P, const double* d_pos, hipStream_t s) {
  const Layout& lay = P->lay;
  const int64_t nd = lay.nbox;
  uint32_t* present = wsp<uint32_t>(P, lay.a_present);
  uint32_t* scan = wsp<uint32_t>(P, lay.a_scan);
  uint32_t* small = wsp<uint32_t>(P, lay.a_small);
  uint32_t* tmp = wsp<uint32_t>(P, lay.scan_tmp);
  prof_begin(P, FMM_PHASE_TREE, s);
  for (int l = 0; l <= FMM_DEPTH_MAX + 1; ++l) P->ce_off[l] = 0;
  ATree t = tree_view(P);
  k_present<<<grid_for(nd, kBlock), kBlock, 0, s>>>(t, nd, present);
  hipError_t e = scan_exclusive(present, nd, nd + 1, scan, tmp, s);
  if (e != hipSuccess) return e;
  k_level_offsets<<<1, 64, 0, s>>>(t, small);
  uint32_t h[FMM_DEPTH_MAX + 2];
  e = hipMemcpyAsync(h, small, sizeof(uint32_t) * (P->L + 2), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (int l = 0; l <= P->L + 1; ++l) P->ce_off[l] = h[l];
  for (int l = P->L + 2; l <= FMM_DEPTH_MAX + 1; ++l) P->ce_off[l] = h[P->L + 1];
  P->Ld = 0;
  for (int l = 0; l <= P->L; ++l)
    if (P->ce_off[l + 1] > P->ce_off[l]) P->Ld = l;
  for (int l = 0; l <= FMM_DEPTH_MAX; ++l)
    P->nsplit[l] = l < P->L ? (P->ce_off[l + 2] - P->ce_off[l + 1]) / 8 : 0;
  const int64_t nbox = P->ce_off[P->L + 1];
  if (nbox > lay.bmax) return hipErrorInvalidValue;  // cannot happen: bmax bounds the tree
  t = tree_view(P);
  k_compact<<<grid_for(nd, kBlock), kBlock, 0, s>>>(
      t, nd, wsp<uint32_t>(P, lay.a_slot), wsp<int32_t>(P, lay.a_level), wsp<uint32_t>(P, lay.a_coord),
      wsp<uint32_t>(P, lay.a_range), wsp<int32_t>(P, lay.a_child0), wsp<uint32_t>(P, lay.a_parent_of));
  {  // M2L targets per class and their source rows, level by level
    VLevels v = {};
    int64_t to = 0, vo = 0;
    for (int l = 0; l <= FMM_DEPTH_MAX + 1; ++l) {
      P->a_tgt_off[l] = v.tgt_off[l] = to;
      P->a_vt_off[l] = v.vt_off[l] = vo;
      v.ndiv[l] = l >= 1 ? P->nsplit[l - 1] : 0;  // l - 1 <= FMM_DEPTH_MAX
      if (l >= 2 && l <= P->Ld) {
        to += 8 * v.ndiv[l];
        vo += ((v.ndiv[l] + m2l::kTargetsPerGroup - 1) / m2l::kTargetsPerGroup) * m2l::kTargetsPerGroup *
              8 * kIL;
      }
    }
    if (to > lay.bmax || vo > lay.vtcap) return hipErrorInvalidValue;  // cannot happen (bounds)
    uint32_t* tgt = wsp<uint32_t>(P, lay.a_tgt);
    const int64_t nb2 = t.nbox - t.ce_off[2];
    if (nb2 > 0) k_m2l_targets<<<grid_for(nb2, kBlock), kBlock, 0, s>>>(t, v, tgt);
    for (int l = 2; l <= P->Ld; ++l) {
      const int64_t nent = P->a_vt_off[l + 1] - P->a_vt_off[l];
      if (nent > 0)
        k_m2l_sources<<<grid_for(nent, kBlock), kBlock, 0, s>>>(t, v, l, nent, tgt,
                                                                 wsp<uint32_t>(P, lay.a_vtab));
    }
  }
  const DevParams* dp = wsp<DevParams>(P, lay.params);
  if (P->mixed)
    k_gather_adaptive<float><<<grid_for(P->n, kBlock), kBlock, 0, s>>>(
        t, d_pos, wsp<int32_t>(P, lay.perm), wsp<uint32_t>(P, lay.keys), P->n, dp,
        wsp<uint32_t>(P, lay.sorted_leaf), wsp<Rec<float>>(P, lay.src), wsp<Rec<double>>(P, lay.src64));
  else
    k_gather_adaptive<double><<<grid_for(P->n, kBlock), kBlock, 0, s>>>(
        t, d_pos, wsp<int32_t>(P, lay.perm), wsp<uint32_t>(P, lay.keys), P->n, dp,
        wsp<uint32_t>(P, lay.sorted_leaf), wsp<Rec<double>>(P, lay.src), nullptr);
  // lists: count, scan each list over nbox + 1 entries, read the totals, fill
  uint32_t* cnt = wsp<uint32_t>(P, lay.a_cnt);
  uint32_t* off = wsp<uint32_t>(P, lay.a_off);
  const int64_t nb1 = lay.bmax + 1;
  int32_t* flags = wsp<int32_t>(P, lay.flags);
  k_lists<false><<<grid_for(nbox, kBlock), kBlock, 0, s>>>(t, cnt, off, nullptr, nullptr, nullptr,
                                                          flags);
  for (int k = 0; k < 3; ++k) {
    e = scan_exclusive(cnt + k * nb1, nbox, nbox + 1, off + k * nb1, tmp, s);
    if (e != hipSuccess) return e;
  }
  // compact lists of the boxes with a W (list 1) or X (list 2) list
  uint32_t* flag = wsp<uint32_t>(P, lay.a_flag);
  uint32_t* fscan = wsp<uint32_t>(P, lay.a_fscan);
  for (int k = 1; k <= 2; ++k) {
    k_flag_nonzero<<<grid_for(nbox, kBlock), kBlock, 0, s>>>(cnt + k * nb1, nbox, flag);
    e = scan_exclusive(flag, nbox, nbox + 1, fscan + (k - 1) * nb1, tmp, s);
    if (e != hipSuccess) return e;
    k_compact_nonzero<<<grid_for(nbox, kBlock), kBlock, 0, s>>>(
        cnt + k * nb1, fscan + (k - 1) * nb1, nbox, wsp<uint32_t>(P, k == 1 ? lay.a_wbox : lay.a_xbox));
  }
  uint32_t tot[5];
  for (int k = 0; k < 5; ++k) {
    const uint32_t* at = k < 3 ? off + k * nb1 + nbox : fscan + (k - 3) * nb1 + nbox;
    e = hipMemcpyAsync(&tot[k], at, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  for (int k = 0; k < 3; ++k) P->nlist[k] = tot[k];
  P->nwbox = tot[3];
  P->nxbox = tot[4];
  if (P->nlist[0] > lay.ucap || P->nlist[1] > lay.wcap || P->nlist[2] > lay.xcap) {
    prof_end(P, s);
    return hipSuccess;  // the caller reports FMM_E_WORKSPACE
  }
  k_lists<true><<<grid_for(nbox, kBlock), kBlock, 0, s>>>(
      t, cnt, off, wsp<uint32_t>(P, lay.a_uidx), wsp<uint32_t>(P, lay.a_widx),
      wsp<uint32_t>(P, lay.a_xidx), flags);
  prof_end(P, s);
  return hipGetLastError();
}

hipError_t launch_adaptive_upward(fmm_plan_s* P, hipStream_t s) {
  if (P->Ld < 2) return hipGetLastError();
  prof_begin(P, FMM_PHASE_P2M, s);
  hipError_t e = dispatch_p<P2MAdaptiveRun>(P->p, P, s);
  prof_end(P, s);
  if (e != hipSuccess) return e;
  prof_begin(P, FMM_PHASE_M2M, s);
  e = launch_m2m_adaptive(P, s);
  prof_end(P, s);
  return e;
}

hipError_t launch_adaptive_p2l(fmm_plan_s* P, hipStream_t s) {
  if (P->Ld < 2) return hipGetLastError();
  return dispatch_p<P2LRun>(P->p, P, s);
}

hipError_t launch_adaptive_downward(fmm_plan_s* P, hipStream_t s) {
  hipError_t e = hipSuccess;
  if (P->Ld >= 2) {
    prof_begin(P, FMM_PHASE_L2L, s);
    e = launch_l2l_adaptive(P, s);
    prof_end(P, s);
    if (e != hipSuccess) return e;
  }
  prof_begin(P, FMM_PHASE_L2P, s);
  e = launch_l2p_adaptive(P, s);
  if (e == hipSuccess) e = dispatch_p<M2PRun>(P->p, P, s);
  prof_end(P, s);
  return e;
}

hipError_t launch_adaptive_stats(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  const ATree t = tree_view(P);
  unsigned long long* st = wsp<unsigned long long>(P, lay.a_stats);
  k_zero_stats<<<1, 64, 0, s>>>(st);
  if (t.nbox > 0)
    k_stats<<<grid_for(t.nbox, kBlock), kBlock, 0, s>>>(t, wsp<uint32_t>(P, lay.a_off),
                                                        wsp<uint32_t>(P, lay.a_uidx), st);
  return hipGetLastError();
}

}  // namespace fmm
