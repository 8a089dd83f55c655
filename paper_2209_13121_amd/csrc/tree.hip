// tree.hip -- tree construction for a uniform octree of depth L.
//
// Per particle: leaf cell of the root cube (FP64, correctly rounded division,
// floor, clamp), validity flags, 3L-bit Hilbert key.  A counting sort over the
// 8^L leaf slots puts particles in Hilbert order: for 3 <= L <= 7 in two levels
// with LDS counters only (k_keys_hist .. k_fine), otherwise in one (histogram by
// global atomics, exclusive scan, scatter); a per-leaf rank by user index makes
// the order inside each leaf, and so every later summation order, deterministic.  Per level, maps between box
// coordinates and Hilbert slots give neighbour lookups; a box's Hilbert slot at
// level l is the top 3l bits of the leaf key of any of its cells, so children of
// slot s are slots 8s .. 8s+7 and every box owns a contiguous range of leaves.
#include <math.h>

#include <algorithm>

#include "fmm_internal.h"

namespace fmm {
namespace {

__global__ void k_fill_u32(uint32_t* a, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_set_params(DevParams* dp, int32_t* flags, double lo0, double lo1, double lo2,
                             double side) {
  dp->lo[0] = lo0;
  dp->lo[1] = lo1;
  dp->lo[2] = lo2;
  dp->side = side;
  flags[0] = 0;
}

// Derived cube: per-block min / max of each axis over finite coordinates.
__global__ void k_bbox_partial(const double* __restrict__ pos, int64_t n, double* __restrict__ part) {
  __shared__ double smin[3][kBlock], smax[3][kBlock];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int a = 0; a < 3; ++a) {
      const double v = pos[3 * i + a];
      if (isfinite(v)) {
        mn[a] = fmin(mn[a], v);
        mx[a] = fmax(mx[a], v);
      }
    }
  }
  for (int a = 0; a < 3; ++a) {
    smin[a][threadIdx.x] = mn[a];
    smax[a][threadIdx.x] = mx[a];
  }
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int a = 0; a < 3; ++a) {
        smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + w]);
        smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a) {
      part[6 * blockIdx.x + a] = smin[a][0];
      part[6 * blockIdx.x + 3 + a] = smax[a][0];
    }
}

// One block of kBlock threads: each folds a strided share of the partials,
// then a tree reduction in LDS (min / max are exact in any order).
__global__ void k_bbox_final(const double* __restrict__ part, int nparts, DevParams* dp,
                             int32_t* flags) {
  __shared__ double smin[3][kBlock], smax[3][kBlock];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nparts; b += kBlock)
    for (int a = 0; a < 3; ++a) {
      mn[a] = fmin(mn[a], part[6 * b + a]);
      mx[a] = fmax(mx[a], part[6 * b + 3 + a]);
    }
  for (int a = 0; a < 3; ++a) {
    smin[a][threadIdx.x] = mn[a];
    smax[a][threadIdx.x] = mx[a];
  }
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int a = 0; a < 3; ++a) {
        smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + w]);
        smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  for (int a = 0; a < 3; ++a) {
    mn[a] = smin[a][0];
    mx[a] = smax[a][0];
  }
  double side = 0.0;
  for (int a = 0; a < 3; ++a) {
    if (!isfinite(mn[a])) mn[a] = 0.0, mx[a] = 0.0;  // no finite coordinate at all
    dp->lo[a] = mn[a];
    side = fmax(side, mx[a] - mn[a]);
  }
  dp->side = side > 0.0 ? side : 1.0;
  flags[0] = 0;
}

__device__ __forceinline__ int leaf_cell(double x, double lo, double side, int L, bool check_cube,
                                         int32_t& flag) {
  if (!isfinite(x)) {
    flag |= kFlagNonFinite;
    return 0;
  }
  const double t = (x - lo) / side;
  if (check_cube && !(t >= 0.0 && t <= 1.0)) flag |= kFlagOutOfCube;
  const double nb = (double)(1 << L);
  double f = floor(t * nb);
  f = fmin(fmax(f, 0.0), nb - 1.0);
  return (int)f;
}

__global__ void k_keys(const double* __restrict__ pos, int64_t n, int L, int check_cube,
                       const DevParams* __restrict__ dp, uint32_t* __restrict__ keys,
                       uint32_t* __restrict__ count, int32_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t flag = 0;
  const double side = dp->side;
  const int cx = leaf_cell(pos[3 * i + 0], dp->lo[0], side, L, check_cube, flag);
  const int cy = leaf_cell(pos[3 * i + 1], dp->lo[1], side, L, check_cube, flag);
  const int cz = leaf_cell(pos[3 * i + 2], dp->lo[2], side, L, check_cube, flag);
  if (flag) atomicOr(flags, flag);
  const uint32_t key = (uint32_t)hilbert_index(cx, cy, cz, L);
  keys[i] = key;
  atomicAdd(&count[key], 1u);
}

// Two-level counting sort of the leaf keys (3 <= L <= 7), with no global
// atomics: the coarse digit c = key >> (3L - 9) (the level-3 box) and the fine
// digit f = the key's low 3L - 9 bits (the leaf inside it).
//  1. k_keys_hist: keys as k_keys, and each work-group's count of every coarse
//     value (LDS atomics) at hist[c * nblk + block];
//  2. an exclusive scan of hist (coarse value major): the first position of
//     each (coarse value, work-group) pair;
//  3. k_coarse_scatter: each particle to its pair's range (LDS atomics give
//     positions within the work-group), key and index;
//  4. k_fine: one work-group per coarse value counts its fine digits in LDS,
//     scans them into the leaf counts and starts, and places each particle in
//     its leaf's range.
// The order inside a leaf is then arbitrary, as after k_scatter, and k_rank
// sorts it by user index: the tree is the same as the one-level sort's.
__global__ __launch_bounds__(kBlock) void k_keys_hist(const double* __restrict__ pos, int64_t n, int L,
                                                      int check_cube, const DevParams* __restrict__ dp,
                                                      uint32_t* __restrict__ keys, int32_t* flags,
                                                      uint32_t* __restrict__ hist, int64_t nblk) {
  __shared__ uint32_t h[kSortCoarse];
  for (int c = threadIdx.x; c < kSortCoarse; c += kBlock) h[c] = 0;
  __syncthreads();
  const int sh = 3 * L - 9;
  const double side = dp->side;
  int32_t flag = 0;
  constexpr int R = kSortChunk / kBlock;
  double x[R][3];  // every position of the thread in flight before the first key
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = (int64_t)blockIdx.x * kSortChunk + r * kBlock + threadIdx.x;
#pragma unroll
    for (int a = 0; a < 3; ++a) x[r][a] = i < n ? pos[3 * i + a] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = (int64_t)blockIdx.x * kSortChunk + r * kBlock + threadIdx.x;
    if (i >= n) break;
    const int cx = leaf_cell(x[r][0], dp->lo[0], side, L, check_cube, flag);
    const int cy = leaf_cell(x[r][1], dp->lo[1], side, L, check_cube, flag);
    const int cz = leaf_cell(x[r][2], dp->lo[2], side, L, check_cube, flag);
    const uint32_t key = (uint32_t)hilbert_index(cx, cy, cz, L);
    keys[i] = key;
    atomicAdd(&h[key >> sh], 1u);
  }
  if (flag) atomicOr(flags, flag);
  __syncthreads();
  for (int c = threadIdx.x; c < kSortCoarse; c += kBlock) hist[(int64_t)c * nblk + blockIdx.x] = h[c];
}

__global__ __launch_bounds__(kBlock) void k_coarse_scatter(const uint32_t* __restrict__ keys, int64_t n, int L,
                                                           const uint32_t* __restrict__ off, int64_t nblk,
                                                           uint32_t* __restrict__ key_tmp,
                                                           int32_t* __restrict__ idx_tmp) {
  __shared__ uint32_t base[kSortCoarse];
  for (int c = threadIdx.x; c < kSortCoarse; c += kBlock) base[c] = off[(int64_t)c * nblk + blockIdx.x];
  __syncthreads();
  const int sh = 3 * L - 9;
  constexpr int R = kSortChunk / kBlock;
  uint32_t kk[R];  // every key of the thread in flight before the first placement
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = (int64_t)blockIdx.x * kSortChunk + r * kBlock + threadIdx.x;
    kk[r] = i < n ? keys[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t i = (int64_t)blockIdx.x * kSortChunk + r * kBlock + threadIdx.x;
    if (i >= n) break;
    const uint32_t at = atomicAdd(&base[kk[r] >> sh], 1u);
    key_tmp[at] = kk[r];
    idx_tmp[at] = (int32_t)i;
  }
}

// One work-group of kFineThreads per coarse value: a value can hold most of
// the particles (a dense system of a batch), and its two passes over them
// are the longest work-group of the launch.
constexpr int kFineThreads = 1024;
__global__ __launch_bounds__(kFineThreads) void k_fine(int64_t n, int L, const uint32_t* __restrict__ off, int64_t nblk,
                                                 const uint32_t* __restrict__ key_tmp,
                                                 const int32_t* __restrict__ idx_tmp,
                                                 uint32_t* __restrict__ count, uint32_t* __restrict__ start,
                                                 int32_t* __restrict__ perm_tmp) {
  __shared__ uint32_t cnt[1 << 12];  // fine values: 2^(3L - 9) <= 4096
  __shared__ uint32_t ssum[kFineThreads];
  const int tid = threadIdx.x;
  const int64_t c = blockIdx.x;
  const int fb = 1 << (3 * L - 9);
  const uint32_t b0 = off[c * nblk], b1 = off[(c + 1) * nblk];
  for (int f = tid; f < fb; f += kFineThreads) cnt[f] = 0;
  __syncthreads();
  for (uint32_t j = b0 + tid; j < b1; j += kFineThreads) atomicAdd(&cnt[key_tmp[j] & (uint32_t)(fb - 1)], 1u);
  __syncthreads();
  // exclusive scan of cnt: a chunk of consecutive values per thread, the
  // chunk sums scanned across the work-group
  const int per = (fb + kFineThreads - 1) / kFineThreads;
  const int f0 = min(fb, tid * per), f1 = min(fb, f0 + per);
  uint32_t mine = 0;
  for (int f = f0; f < f1; ++f) mine += cnt[f];
  ssum[tid] = mine;
  __syncthreads();
  for (int w = 1; w < kFineThreads; w <<= 1) {
    const uint32_t add = tid >= w ? ssum[tid - w] : 0u;
    __syncthreads();
    ssum[tid] += add;
    __syncthreads();
  }
  uint32_t run = b0 + ssum[tid] - mine;
  const int64_t leaf0 = c * fb;
  for (int f = f0; f < f1; ++f) {
    const uint32_t k = cnt[f];
    count[leaf0 + f] = k;
    start[leaf0 + f] = run;
    cnt[f] = run;  // now the next free position of leaf f
    run += k;
  }
  if (c == kSortCoarse - 1 && tid == 0) start[(int64_t)kSortCoarse * fb] = (uint32_t)n;
  __syncthreads();
  for (uint32_t j = b0 + tid; j < b1; j += kFineThreads) {
    const uint32_t at = atomicAdd(&cnt[key_tmp[j] & (uint32_t)(fb - 1)], 1u);
    perm_tmp[at] = idx_tmp[j];
  }
}

// Exclusive scan, 1024 elements per block of 256 threads; elements at index
// >= n_valid read as 0.  Block totals go to bsum.
__global__ void k_scan_block(const uint32_t* __restrict__ in, int64_t n_valid, int64_t n,
                             uint32_t* __restrict__ out, uint32_t* __restrict__ bsum) {
  __shared__ uint32_t s[kBlock];
  const int64_t base = (int64_t)blockIdx.x * 1024 + 4 * threadIdx.x;
  uint32_t v[4], tsum = 0;
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k;
    v[k] = (i < n_valid) ? in[i] : 0u;
    tsum += v[k];
  }
  s[threadIdx.x] = tsum;
  __syncthreads();
  for (int w = 1; w < kBlock; w <<= 1) {
    const uint32_t add = (int)threadIdx.x >= w ? s[threadIdx.x - w] : 0u;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - tsum;  // exclusive prefix of this thread
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = s[kBlock - 1];
}

__global__ void k_scan_add(uint32_t* __restrict__ out, int64_t n, const uint32_t* __restrict__ boff) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += boff[i / 1024];
}

}  // namespace

// out[0..n) = exclusive scan of in[0..n_valid) padded with zeros.
hipError_t scan_exclusive(const uint32_t* in, int64_t n_valid, int64_t n, uint32_t* out,
                          uint32_t* tmp, hipStream_t s) {
  const int64_t nblk = (n + 1023) / 1024;
  k_scan_block<<<(unsigned)nblk, kBlock, 0, s>>>(in, n_valid, n, out, tmp);
  if (nblk > 1) {
    hipError_t e = scan_exclusive(tmp, nblk, nblk, tmp, tmp + nblk, s);
    if (e != hipSuccess) return e;
    k_scan_add<<<grid_for(n, kBlock), kBlock, 0, s>>>(out, n, tmp);
  }
  return hipGetLastError();
}

namespace {

__global__ void k_scatter(const uint32_t* __restrict__ keys, int64_t n,
                          const uint32_t* __restrict__ start, uint32_t* __restrict__ fill,
                          int32_t* __restrict__ perm_tmp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i];
  perm_tmp[start[k] + atomicAdd(&fill[k], 1u)] = (int32_t)i;
}

// Inside each leaf, order particles by user index (rank = number of smaller
// indices in the same leaf).
__global__ void k_rank(const int32_t* __restrict__ perm_tmp, const uint32_t* __restrict__ keys,
                       int64_t n, const uint32_t* __restrict__ start,
                       const uint32_t* __restrict__ count, int32_t* __restrict__ perm) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int32_t me = perm_tmp[s];
  const uint32_t leaf = keys[me];
  const uint32_t b = start[leaf], c = count[leaf];
  uint32_t rank = 0;
  for (uint32_t t = b; t < b + c; ++t) rank += (perm_tmp[t] < me) ? 1u : 0u;
  perm[b + rank] = me;
}

__global__ void k_luts(int L, int64_t nbox, Layout lay,
                       uint32_t* __restrict__ c2s, uint32_t* __restrict__ s2c) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nbox) return;
  int l = 0;
  while (l < L && g >= lay.lvl_off[l + 1]) ++l;
  const int64_t lex = g - lay.lvl_off[l];
  const uint32_t nb = 1u << l;
  const uint32_t x = (uint32_t)(lex >> (2 * l)), y = (uint32_t)((lex >> l) & (nb - 1)),
                 z = (uint32_t)(lex & (nb - 1));
  const int sh = L - l;
  const uint32_t slot = (uint32_t)(hilbert_index(x << sh, y << sh, z << sh, L) >> (3 * sh));
  c2s[lay.lvl_off[l] + lex] = slot;
  s2c[lay.lvl_off[l] + slot] = pack_coord(x, y, z);
}

// The particle record of sorted position d: box-unit offset from its leaf
// centre (FP64; rounded to T), charge slot zero (filled by each evaluation).
template <typename T>
__device__ __forceinline__ void write_record(const double* __restrict__ pos, int32_t i, uint32_t leaf,
                                             int64_t d, int L, const DevParams* __restrict__ dp,
                                             const uint32_t* __restrict__ s2c_leaf,
                                             Rec<T>* __restrict__ src, Rec<double>* __restrict__ src64) {
  int c[3];
  unpack_coord(s2c_leaf[leaf], c[0], c[1], c[2]);
  const double h = dp->side / (double)(1 << L);
  double u[3];
  for (int a = 0; a < 3; ++a) {
    double x = pos[3 * (int64_t)i + a];
    if (!isfinite(x)) x = dp->lo[a];
    const double centre = dp->lo[a] + ((double)c[a] + 0.5) * h;
    u[a] = (x - centre) / h;
  }
  Rec<T> r;
  r.x = (T)u[0];
  r.y = (T)u[1];
  r.z = (T)u[2];
  r.q = T(0);
  src[d] = r;
  if (src64) src64[d] = Rec<double>{u[0], u[1], u[2], 0.0};
}

// k_rank and k_gather in one pass (uniform tree): the particle's place in its
// leaf, then its index, leaf and record at that sorted position.
template <typename T>
__global__ void k_rank_gather(const int32_t* __restrict__ perm_tmp, const uint32_t* __restrict__ keys,
                              int64_t n, const uint32_t* __restrict__ start,
                              const uint32_t* __restrict__ count, int32_t* __restrict__ perm,
                              const double* __restrict__ pos, int L, const DevParams* __restrict__ dp,
                              const uint32_t* __restrict__ s2c_leaf, uint32_t* __restrict__ sorted_leaf,
                              Rec<T>* __restrict__ src, Rec<double>* __restrict__ src64) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int32_t me = perm_tmp[s];
  const uint32_t leaf = keys[me];
  const uint32_t b = start[leaf], c = count[leaf];
  uint32_t rank = 0;
  for (uint32_t t = b; t < b + c; ++t) rank += (perm_tmp[t] < me) ? 1u : 0u;
  const int64_t d = (int64_t)b + rank;
  perm[d] = me;
  sorted_leaf[d] = leaf;
  write_record<T>(pos, me, leaf, d, L, dp, s2c_leaf, src, src64);
}

__global__ void k_leaves_out(const uint32_t* __restrict__ keys, int64_t n,
                             const uint32_t* __restrict__ s2c_leaf, int32_t* __restrict__ cells,
                             uint32_t* __restrict__ leaf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i];
  if (leaf) leaf[i] = k;
  if (cells) {
    int x, y, z;
    unpack_coord(s2c_leaf[k], x, y, z);
    cells[3 * i] = x;
    cells[3 * i + 1] = y;
    cells[3 * i + 2] = z;
  }
}

__device__ __forceinline__ uint32_t box_count(const uint32_t* start, uint32_t slot, int sh) {
  return start[(uint64_t)(slot + 1) << (3 * sh)] - start[(uint64_t)slot << (3 * sh)];
}

// Work counts: M2L pairs of non-empty boxes (levels 2..L) and ordered P2P pairs.
__global__ void k_work(int L, Layout lay, const uint32_t* __restrict__ start,
                       const uint32_t* __restrict__ c2s, const uint32_t* __restrict__ s2c,
                       unsigned long long* __restrict__ work) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= lay.nbox) return;
  int l = 0;
  while (l < L && g >= lay.lvl_off[l + 1]) ++l;
  const uint32_t slot = (uint32_t)(g - lay.lvl_off[l]);
  const int sh = L - l;
  const uint32_t nt = box_count(start, slot, sh);
  if (nt == 0) return;
  int x, y, z;
  unpack_coord(s2c[lay.lvl_off[l] + slot], x, y, z);
  const int nb = 1 << l;
  if (l >= 2) {
    unsigned long long pairs = 0;
    for (int dx = -3; dx <= 3; ++dx)
      for (int dy = -3; dy <= 3; ++dy)
        for (int dz = -3; dz <= 3; ++dz) {
          const int sx = x + dx, sy = y + dy, sz = z + dz;
          if (sx < 0 || sy < 0 || sz < 0 || sx >= nb || sy >= nb || sz >= nb) continue;
          if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) continue;
          if (abs((sx >> 1) - (x >> 1)) > 1 || abs((sy >> 1) - (y >> 1)) > 1 ||
              abs((sz >> 1) - (z >> 1)) > 1)
            continue;
          const uint32_t ss = c2s[lay.lvl_off[l] + lex_index(sx, sy, sz, l)];
          if (box_count(start, ss, sh) > 0) ++pairs;
        }
    if (pairs) atomicAdd(&work[0], pairs);
  }
  if (l == L) {
    unsigned long long src = 0;
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          const int sx = x + dx, sy = y + dy, sz = z + dz;
          if (sx < 0 || sy < 0 || sz < 0 || sx >= nb || sy >= nb || sz >= nb) continue;
          src += box_count(start, c2s[lay.lvl_off[l] + lex_index(sx, sy, sz, l)], 0);
        }
    atomicAdd(&work[1], (unsigned long long)nt * (src - 1ull));
  }
}

__global__ void k_zero_work(unsigned long long* work) {
  if (threadIdx.x < 2) work[threadIdx.x] = 0ull;
}

}  // namespace

hipError_t fill_u32(uint32_t* a, int64_t n, uint32_t v, hipStream_t s) {
  if (n > 0) k_fill_u32<<<grid_for(n, kBlock), kBlock, 0, s>>>(a, n, v);
  return hipGetLastError();
}

hipError_t launch_tree(fmm_plan_s* P, const double* d_pos, hipStream_t s) {
  const Layout& lay = P->lay;
  const int64_t n = P->n;
  const int L = P->L;
  DevParams* dp = wsp<DevParams>(P, lay.params);
  int32_t* flags = wsp<int32_t>(P, lay.flags);
  uint32_t* keys = wsp<uint32_t>(P, lay.keys);
  uint32_t* count = wsp<uint32_t>(P, lay.leaf_count);
  uint32_t* start = wsp<uint32_t>(P, lay.leaf_start);
  uint32_t* fill = wsp<uint32_t>(P, lay.leaf_fill);
  uint32_t* c2s = wsp<uint32_t>(P, lay.coord2slot);
  uint32_t* s2c = wsp<uint32_t>(P, lay.slot2coord);

  prof_begin(P, FMM_PHASE_TREE, s);
  const bool given = P->cfg.root_side > 0.0;
  if (given) {
    k_set_params<<<1, 1, 0, s>>>(dp, flags, P->cfg.root_lo[0], P->cfg.root_lo[1],
                                 P->cfg.root_lo[2], P->cfg.root_side);
  } else {
    double* part = wsp<double>(P, lay.bbox);
    const int nparts = (int)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
    k_bbox_partial<<<nparts, kBlock, 0, s>>>(d_pos, n, part);
    k_bbox_final<<<1, kBlock, 0, s>>>(part, nparts, dp, flags);
  }
  if (!P->ops_ready) {  // the zero row M2L reads for sources outside the domain (kept by a re-plan)
    const int64_t words = (int64_t)(zero_row_bytes(P->p, P->m2l_np) / 4);
    k_fill_u32<<<grid_for(words, kBlock), kBlock, 0, s>>>(wsp<uint32_t>(P, lay.zero_row), words, 0u);
  }
  k_luts<<<grid_for(lay.nbox, kBlock), kBlock, 0, s>>>(L, lay.nbox, lay, c2s, s2c);
  int32_t* perm_tmp = wsp<int32_t>(P, lay.perm_tmp);
  int32_t* perm = wsp<int32_t>(P, lay.perm);
  if (sort_two_level(L)) {
    // key and index by coarse digit in the sorted-leaf array and the
    // permutation (both written again below)
    const int64_t nblk = (n + kSortChunk - 1) / kSortChunk;
    uint32_t* hist = wsp<uint32_t>(P, lay.sort_hist);
    uint32_t* key_tmp = wsp<uint32_t>(P, lay.sorted_leaf);
    k_keys_hist<<<(unsigned)nblk, kBlock, 0, s>>>(d_pos, n, L, given ? 1 : 0, dp, keys, flags, hist, nblk);
    const int64_t nh = sort_hist_elems(n);  // the last element (0) becomes the total
    k_fill_u32<<<1, 1, 0, s>>>(hist + nh - 1, 1, 0u);
    hipError_t e = scan_exclusive(hist, nh, nh, hist, wsp<uint32_t>(P, lay.scan_tmp), s);
    if (e != hipSuccess) return e;
    k_coarse_scatter<<<(unsigned)nblk, kBlock, 0, s>>>(keys, n, L, hist, nblk, key_tmp, perm);
    k_fine<<<kSortCoarse, kFineThreads, 0, s>>>(n, L, hist, nblk, key_tmp, perm, count, start, perm_tmp);
  } else {
    k_fill_u32<<<grid_for(lay.nleaf, kBlock), kBlock, 0, s>>>(count, lay.nleaf, 0u);
    k_fill_u32<<<grid_for(lay.nleaf, kBlock), kBlock, 0, s>>>(fill, lay.nleaf, 0u);
    k_keys<<<grid_for(n, kBlock), kBlock, 0, s>>>(d_pos, n, L, given ? 1 : 0, dp, keys, count, flags);
    hipError_t e = scan_exclusive(count, lay.nleaf, lay.nleaf + 1, start,
                                  wsp<uint32_t>(P, lay.scan_tmp), s);
    if (e != hipSuccess) return e;
    k_scatter<<<grid_for(n, kBlock), kBlock, 0, s>>>(keys, n, start, fill, perm_tmp);
  }
  if (P->adaptive) {
    // leaves and box-unit offsets come from the adaptive tree (adaptive.hip)
    k_rank<<<grid_for(n, kBlock), kBlock, 0, s>>>(perm_tmp, keys, n, start, count, perm);
  } else if (P->mixed) {
    k_rank_gather<float><<<grid_for(n, kBlock), kBlock, 0, s>>>(
        perm_tmp, keys, n, start, count, perm, d_pos, L, dp, s2c + lay.lvl_off[L],
        wsp<uint32_t>(P, lay.sorted_leaf), wsp<Rec<float>>(P, lay.src), wsp<Rec<double>>(P, lay.src64));
  } else {
    k_rank_gather<double><<<grid_for(n, kBlock), kBlock, 0, s>>>(
        perm_tmp, keys, n, start, count, perm, d_pos, L, dp, s2c + lay.lvl_off[L],
        wsp<uint32_t>(P, lay.sorted_leaf), wsp<Rec<double>>(P, lay.src), nullptr);
  }
  prof_end(P, s);
  return hipGetLastError();
}

hipError_t launch_leaves_out(fmm_plan_s* P, int32_t* d_cells, uint32_t* d_leaf, hipStream_t s) {
  const Layout& lay = P->lay;
  k_leaves_out<<<grid_for(P->n, kBlock), kBlock, 0, s>>>(
      wsp<uint32_t>(P, lay.keys), P->n, wsp<uint32_t>(P, lay.slot2coord) + lay.lvl_off[P->L],
      d_cells, d_leaf);
  return hipGetLastError();
}

hipError_t launch_work_count(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  unsigned long long* work = wsp<unsigned long long>(P, lay.work);
  k_zero_work<<<1, 64, 0, s>>>(work);
  k_work<<<grid_for(lay.nbox, kBlock), kBlock, 0, s>>>(
      P->L, lay, wsp<uint32_t>(P, lay.leaf_start), wsp<uint32_t>(P, lay.coord2slot),
      wsp<uint32_t>(P, lay.slot2coord), work);
  return hipGetLastError();
}

}  // namespace fmm
