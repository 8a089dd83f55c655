// m2l_common.h -- work decomposition shared by the M2L kernels (FP32/FP64
// MFMA in m2l.hip, split-BF16 MFMA in m2l_bf16.hip).
//
// For a target box t at level l >= 2 the interaction list is every box s of
// level l whose parent is adjacent to t's parent but which is not adjacent to
// t (well-separatedness 1; Greengard 1988, ch. 3; Cheng, Greengard & Rokhlin
// 1999, sec. 3).  With d = t - s the list depends only on the parity pi of t's
// coordinates: d_a ranges over [pi_a - 3, pi_a + 2] with max |d_a| >= 2, 189
// offsets per class, one unit-box operator per offset (316 in all).
//
// One work-group owns 128 targets of one parity class at one level: the
// parity-pi children of 128 consecutive, aligned parent slots in Hilbert
// order, 8 waves of 16 targets (one MFMA column block each).
#ifndef FMM_M2L_COMMON_H_
#define FMM_M2L_COMMON_H_

#include "fmm_internal.h"

namespace fmm {
namespace m2l {

constexpr int kWaves = 8;  // waves per work-group
constexpr int kThreads = kWaves * 64;
constexpr int kTargetsPerGroup = kWaves * 16;

// Interaction-list offsets of each parity class pi in a fixed order, with
// their operator numbers: code = op | (dx + 4) << 9 | (dy + 4) << 13 | (dz + 4) << 17.
struct ILTable {
  uint32_t v[8][kIL];
};
constexpr ILTable make_il_table() {
  ILTable t{};
  for (int pi = 0; pi < 8; ++pi) {
    const int px = (pi >> 2) & 1, py = (pi >> 1) & 1, pz = pi & 1;
    int i = 0;
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b)
        for (int c = 0; c < 6; ++c) {
          const int dx = px - 3 + a, dy = py - 3 + b, dz = pz - 3 + c;
          if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) continue;
          t.v[pi][i++] = (uint32_t)m2l_op_index(dx, dy, dz) | (uint32_t)(dx + 4) << 9 |
                         (uint32_t)(dy + 4) << 13 | (uint32_t)(dz + 4) << 17;
        }
  }
  return t;
}
static __constant__ ILTable kILTable = make_il_table();

// Work-group barrier of the double-buffered operator staging: this wave's
// LDS reads and writes have completed (lgkmcnt(0)), then s_barrier.  Unlike
// __syncthreads it does not wait for outstanding global loads (the next
// offset's source prefetch stays in flight across it).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt not waited for
  __asm__ volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
}

// Offset i of class pi and its operator number.
__device__ __forceinline__ int il_offset(int pi, int i, int& dx, int& dy, int& dz) {
  const uint32_t c = kILTable.v[pi][i];
  dx = (int)((c >> 9) & 15u) - 4;
  dy = (int)((c >> 13) & 15u) - 4;
  dz = (int)((c >> 17) & 15u) - 4;
  return (int)(c & 511u);
}

struct Args {
  int L;                                 // deepest level with targets
  int64_t lvl_off[FMM_DEPTH_MAX + 2];    // dense box offsets per level (c2s, s2c)
  int64_t exp_off[FMM_DEPTH_MAX + 2];    // first row of each level in the expansion arrays
  int64_t group_off[FMM_DEPTH_MAX + 2];  // first work-group of each level (levels 2..L)
  int64_t ngroups;
  int64_t ksplit;  // work-groups per XCD run as two halves (0: none)
  const uint32_t* c2s;
  const uint32_t* s2c;
  // Adaptive tree only.  The targets of level l
  // and class pi are the class-pi children of the level's divided parents,
  // ndiv[l] of them, rows tgt[tgt_off[l] + pi ndiv[l] + k] of the level; a
  // work-group owns 128 of them (tile t) and reads the row of each target's
  // source at offset i of its class from
  // vtab[vt_off[l] + ((t * 8 + pi) * kIL + i) * 128 + target] (kAbsent where
  // the tree has no such box, and for the padding of the last tile).
  const uint32_t* tgt;
  const uint32_t* vtab;
  int64_t ndiv[FMM_DEPTH_MAX + 2];
  int64_t tgt_off[FMM_DEPTH_MAX + 2];
  int64_t vt_off[FMM_DEPTH_MAX + 2];
};

inline Args make_args(fmm_plan_s* Pl) {
  const Layout& lay = Pl->lay;
  Args a;
  a.L = Pl->adaptive ? Pl->Ld : Pl->L;
  for (int l = 0; l <= FMM_DEPTH_MAX + 1; ++l) {
    a.lvl_off[l] = lay.lvl_off[l];
    a.exp_off[l] = Pl->adaptive ? Pl->ce_off[l] : lay.lvl_off[l];
  }
  int64_t g = 0;
  for (int l = 2; l <= a.L; ++l) {
    a.group_off[l] = g;
    const int64_t np = Pl->adaptive ? Pl->nsplit[l - 1] : (int64_t)1 << (3 * (l - 1));
    g += 8 * ((np + kTargetsPerGroup - 1) / kTargetsPerGroup);
  }
  a.group_off[a.L + 1] = g;
  a.ngroups = g;
  a.ksplit = 0;
  a.c2s = wsp<uint32_t>(Pl, lay.coord2slot);
  a.s2c = wsp<uint32_t>(Pl, lay.slot2coord);
  a.tgt = Pl->adaptive ? wsp<uint32_t>(Pl, lay.a_tgt) : nullptr;
  a.vtab = Pl->adaptive ? wsp<uint32_t>(Pl, lay.a_vtab) : nullptr;
  for (int l = 0; l <= FMM_DEPTH_MAX + 1; ++l) {
    a.ndiv[l] = Pl->adaptive && l >= 1 ? Pl->nsplit[l - 1] : 0;
    a.tgt_off[l] = Pl->a_tgt_off[l];
    a.vt_off[l] = Pl->a_vt_off[l];
  }
  return a;
}
inline unsigned grid_of(const Args& a) {
  return (unsigned)(((a.ngroups + 7) / 8 + (kM2lParts - 1) * a.ksplit) * 8);
}

// Hardware group b -> logical group lg.  XCD-aware order: group b runs on XCD
// b % 8, and each XCD gets a contiguous range of per_xcd logical groups.  With
// ksplit > 0 the last ksplit of them are each run by kM2lParts consecutive
// hardware groups, parts 0 .. kM2lParts - 1 (split index sidx = xcd * ksplit
// + j for the j-th); part = -1 for a whole group.
__host__ __device__ inline void decode_group(const Args& a, int64_t b, int64_t& lg, int& part,
                                             int64_t& sidx) {
  const int64_t per_xcd = (a.ngroups + 7) / 8, xcd = b % 8, r = b / 8, full = per_xcd - a.ksplit;
  if (r < full) {
    lg = xcd * per_xcd + r;
    part = -1;
    sidx = 0;
  } else {
    const int64_t h = r - full;
    lg = xcd * per_xcd + full + h / kM2lParts;
    part = (int)(h % kM2lParts);
    sidx = xcd * a.ksplit + h / kM2lParts;
  }
}

// Slots of every source box a work-group can touch: 128 consecutive aligned
// Hilbert slots of the parent level are two face-adjacent 4^3 blocks, so the
// targets span at most 15 x 7 x 7 boxes and their sources (targets - d,
// d in [pi - 3, pi + 2]) at most 20 x 12 x 12.
constexpr int kHalo = 20 * 12 * 12;

struct Src {
  uint32_t slot;
  bool ok;  // inside the domain (else the source is a zero row)
};

// Source-table entry of the adaptive tree: no box there.
constexpr uint32_t kAbsent = 0x80000000u;

// A lane's view of its work-group's tile.  AD: adaptive tree (targets from the
// per-class lists, sources from the table; no halo), fixed at compile time so
// that the uniform form carries none of it.
// SPLIT: the work-group may be one part of a split group (decode_group);
// otherwise the plain XCD-aware mapping.
template <bool AD, bool SPLIT = false>
struct TileT {
  int l, pi, nb;
  int tx, ty, tz;  // this lane's target box (meaningful when col_ok)
  bool col_ok;
  int hx0, hy0, hz0, hx1, hy1, hz1, hey, hez;  // halo box (clamped to the level)
  int64_t lvl_off;                             // first row of level l in the expansion arrays
  int64_t dense_off;                           // first box of level l in the dense tables
  int64_t tile;                                // tile number within the level and class
  const uint32_t* vt;                          // adaptive: this lane's source-row column
  int64_t trow;                                // adaptive: this lane's target row
  int part;                                    // -1 whole group, else its part (split M2L)
  int64_t sidx;                                // split index of a part group

  // Decode the group, find this lane's target (number tix of the tile's 128)
  // and (uniform tree) stage the halo's slots in sSlot.  Returns false,
  // uniformly over the work-group, for a group past the end.  The uniform form
  // contains barriers.
  __device__ __forceinline__ bool setup(const Args& a, int tix, uint32_t* sSlot, int* sBox) {
    int64_t lg;
    if constexpr (SPLIT) {
      int pt;
      int64_t si;
      decode_group(a, blockIdx.x, lg, pt, si);
      return setup_at(a, lg, pt, si, tix, sSlot, sBox);
    } else {
      // (the same steps as locate, written out: the FP32 / FP64 kernel's main
      // loop was measured 7 % slower when they were shared)
      part = -1;
      sidx = 0;
      const int64_t per_xcd = (a.ngroups + 7) / 8;
      lg = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
      if (lg >= a.ngroups) return false;
      l = 2;
      while (l < a.L && lg >= a.group_off[l + 1]) ++l;
      if constexpr (AD) {
        const int64_t idx = lg - a.group_off[l];
        pi = (int)(idx % 8);
        tile = idx / 8;
        lvl_off = a.exp_off[l];
        retarget(a, tix);
        return true;
      }
      const int64_t idx = lg - a.group_off[l];
      pi = (int)(idx % 8);
      tile = idx / 8;
    }
    if constexpr (AD) return true;  // no halo, the source rows come from the table
    const int px = (pi >> 2) & 1, py = (pi >> 1) & 1, pz = pi & 1;
    if constexpr (!SPLIT) {
      nb = 1 << l;
      lvl_off = a.exp_off[l];
      dense_off = a.lvl_off[l];
      retarget(a, tix);
    }
    const int tid = threadIdx.x;
    if (tid < 6) sBox[tid] = tid < 3 ? nb : -1;
    __syncthreads();
    if (col_ok) {
      atomicMin(&sBox[0], tx - px - 2);
      atomicMin(&sBox[1], ty - py - 2);
      atomicMin(&sBox[2], tz - pz - 2);
      atomicMax(&sBox[3], tx - px + 3);
      atomicMax(&sBox[4], ty - py + 3);
      atomicMax(&sBox[5], tz - pz + 3);
    }
    __syncthreads();
    hx0 = sBox[0] < 0 ? 0 : sBox[0];
    hy0 = sBox[1] < 0 ? 0 : sBox[1];
    hz0 = sBox[2] < 0 ? 0 : sBox[2];
    hx1 = sBox[3] >= nb ? nb - 1 : sBox[3];
    hy1 = sBox[4] >= nb ? nb - 1 : sBox[4];
    hz1 = sBox[5] >= nb ? nb - 1 : sBox[5];
    hey = hy1 - hy0 + 1;
    hez = hz1 - hz0 + 1;
    const int hn = (hx1 - hx0 + 1) * hey * hez;  // <= kHalo by the bound above
    const uint32_t* c2s = a.c2s + dense_off;
    for (int e = tid; e < hn && e < kHalo; e += (int)blockDim.x) {
      const int x = hx0 + e / (hey * hez), y = hy0 + (e / hez) % hey, z = hz0 + e % hez;
      sSlot[e] = c2s[lex_index(x, y, z, l)];
    }
    __syncthreads();
    return true;
  }

  // setup for logical group lg given by the caller (part pt, split index si;
  // pt = -1 for a whole group): the persistent launches.
  __device__ __forceinline__ bool setup_at(const Args& a, int64_t lg, int pt, int64_t si, int tix,
                                           uint32_t* sSlot, int* sBox) {
    part = pt;
    sidx = si;
    if (!locate(a, lg, tix)) return false;
    if constexpr (!AD) stage_halo(a, sSlot, sBox);  // the adaptive tree's sources come from its table
    return true;
  }

  // Uniform tree: the slots of the tile's halo into sSlot (barriers).
  __device__ __forceinline__ void stage_halo(const Args& a, uint32_t* sSlot, int* sBox) {
    const int px = (pi >> 2) & 1, py = (pi >> 1) & 1, pz = pi & 1;
    const int tid = threadIdx.x;
    if (tid < 6) sBox[tid] = tid < 3 ? nb : -1;
    __syncthreads();
    if (col_ok) {
      atomicMin(&sBox[0], tx - px - 2);
      atomicMin(&sBox[1], ty - py - 2);
      atomicMin(&sBox[2], tz - pz - 2);
      atomicMax(&sBox[3], tx - px + 3);
      atomicMax(&sBox[4], ty - py + 3);
      atomicMax(&sBox[5], tz - pz + 3);
    }
    __syncthreads();
    hx0 = sBox[0] < 0 ? 0 : sBox[0];
    hy0 = sBox[1] < 0 ? 0 : sBox[1];
    hz0 = sBox[2] < 0 ? 0 : sBox[2];
    hx1 = sBox[3] >= nb ? nb - 1 : sBox[3];
    hy1 = sBox[4] >= nb ? nb - 1 : sBox[4];
    hz1 = sBox[5] >= nb ? nb - 1 : sBox[5];
    hey = hy1 - hy0 + 1;
    hez = hz1 - hz0 + 1;
    const int hn = (hx1 - hx0 + 1) * hey * hez;  // <= kHalo by the bound above
    const uint32_t* c2s = a.c2s + dense_off;
    for (int e = tid; e < hn && e < kHalo; e += (int)blockDim.x) {
      const int x = hx0 + e / (hey * hez), y = hy0 + (e / hez) % hey, z = hz0 + e % hez;
      sSlot[e] = c2s[lex_index(x, y, z, l)];
    }
    __syncthreads();
  }

  // Level, class and tile of logical group lg, and this lane's target (number
  // tix of the tile); false past the last group.  No barriers, no halo.
  // The 8 parity classes of a tile are consecutive groups, so they run close
  // together on one XCD and share its L2 for the tile's sources.
  __device__ __forceinline__ bool locate(const Args& a, int64_t lg, int tix) {
    if (lg >= a.ngroups) return false;
    l = 2;
    while (l < a.L && lg >= a.group_off[l + 1]) ++l;
    const int64_t idx = lg - a.group_off[l];
    pi = (int)(idx % 8);
    tile = idx / 8;
    nb = 1 << l;
    lvl_off = a.exp_off[l];
    dense_off = a.lvl_off[l];
    retarget(a, tix);
    return true;
  }

  // This lane's target: number tix of the tile (no barriers).
  __device__ __forceinline__ void retarget(const Args& a, int tix) {
    const int64_t ps = tile * kTargetsPerGroup + tix;
    if constexpr (AD) {
      col_ok = ps < a.ndiv[l];
      trow = col_ok ? (int64_t)a.tgt[a.tgt_off[l] + pi * a.ndiv[l] + ps] : 0;
      vt = a.vtab + a.vt_off[l] + (tile * 8 + pi) * (int64_t)kIL * kTargetsPerGroup + tix;
    } else {
      col_ok = ps < ((int64_t)1 << (3 * (l - 1)));
      tx = ty = tz = 0;
      if (col_ok) {
        unpack_coord(a.s2c[a.lvl_off[l - 1] + ps], tx, ty, tz);
        tx = 2 * tx + ((pi >> 2) & 1);
        ty = 2 * ty + ((pi >> 1) & 1);
        tz = 2 * tz + (pi & 1);
      }
    }
  }

  // This lane's source for offset k = (dx, dy, dz) of its class: its row,
  // read from the staged halo at coordinates clamped into it (so the read is
  // unconditional) or, on the adaptive tree, from the source table; and
  // whether the source exists.
  __device__ __forceinline__ Src lookup(const uint32_t* sSlot, int k, int dx, int dy, int dz) const {
    if constexpr (AD) {
      const uint32_t v = vt[(int64_t)k * kTargetsPerGroup];
      return Src{v & ~kAbsent, !(v & kAbsent)};
    }
    int sx = tx - dx, sy = ty - dy, sz = tz - dz;
    const bool ok = col_ok && sx >= 0 && sy >= 0 && sz >= 0 && sx < nb && sy < nb && sz < nb;
    sx = sx < hx0 ? hx0 : (sx > hx1 ? hx1 : sx);
    sy = sy < hy0 ? hy0 : (sy > hy1 ? hy1 : sy);
    sz = sz < hz0 ? hz0 : (sz > hz1 ? hz1 : sz);
    return Src{sSlot[((sx - hx0) * hey + (sy - hy0)) * hez + (sz - hz0)], ok};
  }

  // Row of this lane's target within its level (col_ok only).
  __device__ __forceinline__ int64_t target_slot(const Args& a) const {
    if constexpr (AD) return trow;
    return a.c2s[dense_off + lex_index(tx, ty, tz, l)];
  }
};

}  // namespace m2l
}  // namespace fmm

#endif  // FMM_M2L_COMMON_H_
