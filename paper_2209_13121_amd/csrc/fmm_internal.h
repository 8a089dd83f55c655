// fmm_internal.h -- plan object, workspace layout and device helpers shared by
// the library's HIP sources.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fmm.h"

namespace fmm {

constexpr int kBlock = 256;          // default work-group size (4 wave64)
// Leaf sort of the uniform tree (3 <= L <= 7): particles per work-group of
// the coarse pass, and the coarse digit's 512 values (the key's top 9 bits)
constexpr int kSortChunk = 4 * kBlock;
constexpr int kSortCoarse = 512;
inline bool sort_two_level(int L) { return L >= 3 && L <= 7; }
inline int64_t sort_hist_elems(int64_t n) {
  return (int64_t)kSortCoarse * ((n + kSortChunk - 1) / kSortChunk) + 1;
}
constexpr int kNumM2LOps = 316;      // offsets in [-3,3]^3 \ [-1,1]^3
constexpr int kIL = 189;             // interaction-list offsets per parity class
// Split M2L (split forms): at most this many work-groups per XCD, the
// last ones dispatched, each run as kM2lParts part work-groups over offsets
// [q kIL / kM2lParts, (q + 1) kIL / kM2lParts) (the launch's last round then
// ends nearly full instead of nearly empty).
constexpr int kM2lSplitPerXcd = 16;
constexpr int kM2lParts = 4;
constexpr int kMaxProfile = 8192;    // recorded launches between profile reads

// Error bits raised by kernels (atomicOr into Plan::d_flags).
enum : int32_t { kFlagOutOfCube = 1, kFlagNonFinite = 2, kFlagCoincident = 4, kFlagListOverflow = 8 };

// Device-resident parameters of a plan (written by kernels, so that a derived
// cube never needs a host round trip).
struct DevParams {
  double lo[3];
  double side;
};

inline int ncoef(int p) { return (p + 1) * (p + 1); }
// Row stride of the multipole arrays: ncoef rounded up to a multiple of 4
// (zero padded), so that a box's coefficients start 16-byte aligned.
__host__ __device__ constexpr int mstride_of(int nc) { return ((nc + 3) / 4) * 4; }
inline int mstride(int p) { return mstride_of(ncoef(p)); }
// Operator tile sizes: rows padded to 16-row MFMA blocks, K to 4-deep steps.
inline int m2l_rows_pad(int p) { return ((ncoef(p) + 15) / 16) * 16; }
inline int m2l_k_pad(int p) { return ((ncoef(p) + 3) / 4) * 4; }
// M2M / L2L octant operators are stored [octant][row (16-row blocks)][k], k
// padded to a multiple of 8 (zero).
__host__ __device__ constexpr int shift_kpad(int nc) { return ((nc + 7) / 8) * 8; }
// M2L operators are stored [row][k] with k-stride V (4 V nq + 1) elements, V
// the elements per 16-byte vector and nq = ceil(ncoef / 4V): every 16-byte
// k-quad a lane reads is inside the row (zero padded), and the odd quad stride
// keeps 16 consecutive rows in distinct LDS bank groups.
__host__ __device__ constexpr int m2l_kstride_of(int nc, int elem) {
  return (16 / elem) * (4 * ((nc + 4 * (16 / elem) - 1) / (4 * (16 / elem))) + 1);
}

// Split-BF16 M2L: k runs in steps of 32 (16x16x32 BF16 MFMA), each split into
// 4 lane groups g of 8 k values (k = 32 ks + 8 g + j, zero past ncoef).
//  * A source box holds quad (ks * np + piece) * 4 + g for every k step and
//    piece (m2lb_row_quads quads).
//  * An operator is stored in chunks of kc k steps (as many as two LDS
//    buffers hold), each chunk [row][g][k step][piece] with the g blocks gq
//    quads apart (gq = kc * np made odd) and rows 4 gq + 2 quads apart.  A
//    16-byte LDS read serves 32 lanes at a time and is free of bank conflicts
//    when their quads are distinct modulo 32: 16 rows at a stride of 2 mod 4
//    fill the even residues and the odd g offset the odd ones.
__host__ __device__ constexpr int m2lb_ksteps(int nc) { return (nc + 31) / 32; }
__host__ __device__ constexpr int m2lb_row_quads(int nc, int np) { return m2lb_ksteps(nc) * np * 4; }
// LDS for the two operator chunk buffers: the uniform tree's kernels also hold
// the halo's slot table (11.5 KB), the adaptive tree's (ad) do not.
constexpr int kM2lbLdsBudget = 140 * 1024;
constexpr int kM2lbLdsBudgetAd = 156 * 1024;
__host__ __device__ constexpr int m2lb_gq(int kc, int np) { return (kc * np) | 1; }
__host__ __device__ constexpr int m2lb_qcs(int kc, int np) { return 4 * m2lb_gq(kc, np) + 2; }
__host__ __device__ constexpr int m2lb_rows(int nc) { return ((nc + 15) / 16) * 16; }
// Wide FP16 form (p <= kM2lWidePMax; 32 x 32 x 16 MFMA, a wave per 32
// targets).  Its operators hold only the quads its products read: row block
// rb (32 rows) takes both FP16 pieces for its first m2lw_cross_steps k steps
// (16 k values each) and the leading piece alone for the others (the product
// tiers: h h + h l + l h while the lowest local degree of the block plus the
// lowest multipole degree of the step is below kF16Tier, h h alone after),
// and no quad whose 8 k values all lie past ncoef.  A row of block rb holds
// its quads in k order (quad 4 s + 2 h + piece while s is below the cross
// steps S, then 4 S + 2 (s - S) + h), padded to an odd count so that the 32
// rows of a 16-byte LDS read fall on distinct quads modulo 32; the blocks
// follow each other, and one zero quad ends the operator (read by the lanes
// whose k half lies past ncoef).  Staged into LDS as one contiguous copy.
#ifndef M2L_WIDE_PMAX
#define M2L_WIDE_PMAX 8
#endif
#ifndef M2LB_TIER
#define M2LB_TIER 11
#endif
constexpr int kM2lWidePMax = M2L_WIDE_PMAX;
constexpr int kF16Tier = M2LB_TIER;
__host__ __device__ constexpr bool m2l_f16_wide(int p) { return p <= kM2lWidePMax; }
__host__ __device__ constexpr int isqrt_c(int v) {
  int r = 0;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}
// 32-row block rb and 16-wide k step s take all three piece products
__host__ __device__ constexpr bool f16_cross_w(int rb, int s) {
  return isqrt_c(32 * rb) + isqrt_c(16 * s) < kF16Tier;
}
__host__ __device__ constexpr int m2lw_ksteps(int nc) { return (nc + 15) / 16; }
__host__ __device__ constexpr int m2lw_cross_steps(int nc, int rb) {
  int n = 0;
  while (n < m2lw_ksteps(nc) && f16_cross_w(rb, n)) ++n;
  return n;
}
// k half (s, h) holds data
__host__ __device__ constexpr bool m2lw_half_live(int nc, int s, int h) { return 16 * s + 8 * h < nc; }
// position of (k step s, half h, piece i) in a row of block rb
__host__ __device__ constexpr int m2lw_pos(int nc, int rb, int s, int h, int i) {
  return s < m2lw_cross_steps(nc, rb) ? 4 * s + 2 * h + i
                                      : 4 * m2lw_cross_steps(nc, rb) + 2 * (s - m2lw_cross_steps(nc, rb)) + h;
}
__host__ __device__ constexpr int m2lw_row_len(int nc, int rb) {
  int len = 0;
  for (int s = 0; s < m2lw_ksteps(nc); ++s)
    for (int h = 0; h < 2; ++h)
      if (m2lw_half_live(nc, s, h)) {
        const int top = m2lw_pos(nc, rb, s, h, s < m2lw_cross_steps(nc, rb) ? 1 : 0) + 1;
        len = len > top ? len : top;
      }
  return len | 1;
}
__host__ __device__ constexpr int m2lw_rows_in(int nc, int rb) { return nc - 32 * rb < 32 ? nc - 32 * rb : 32; }
__host__ __device__ constexpr int m2lw_block_base(int nc, int rb) {
  int b = 0;
  for (int r = 0; r < rb; ++r) b += m2lw_rows_in(nc, r) * m2lw_row_len(nc, r);
  return b;
}
// quads of one operator (the last is the zero quad)
__host__ __device__ constexpr int m2lw_op_quads(int nc) { return m2lw_block_base(nc, (nc + 31) / 32) + 1; }
__host__ __device__ constexpr int m2lb_kc_fit(int nc, int np, int n, bool ad) {
  return n <= 1 ? 1
                : (2 * m2lb_rows(nc) * m2lb_qcs(n, np) * 16 <= (ad ? kM2lbLdsBudgetAd : kM2lbLdsBudget)
                       ? n
                       : m2lb_kc_fit(nc, np, n - 1, ad));
}
__host__ __device__ constexpr int m2lb_kc(int nc, int np, bool ad = false) {
  return m2lb_kc_fit(nc, np, m2lb_ksteps(nc), ad);
}
__host__ __device__ constexpr int m2lb_nch(int nc, int np, bool ad = false) {
  return (m2lb_ksteps(nc) + m2lb_kc(nc, np, ad) - 1) / m2lb_kc(nc, np, ad);
}
// Quads of one operator (all chunks).
__host__ __device__ constexpr int m2lb_op_quads(int nc, int np, bool ad = false) {
  return m2lb_nch(nc, np, ad) * m2lb_rows(nc) * m2lb_qcs(m2lb_kc(nc, np, ad), np);
}

// Bytes of the all-zero source row that M2L reads outside the domain (large
// enough for the FP64, FP32 and split-BF16 row forms).
inline size_t zero_row_bytes(int p, int np) {
  const size_t zb = sizeof(double) * (size_t)mstride(p);
  const size_t zq = (size_t)16 * m2lb_row_quads(ncoef(p), np ? np : 1);
  return zb > zq ? zb : zq;
}

struct Layout {  // byte offsets into the workspace, every one 256-aligned
  size_t params, flags, energy_part, bbox, zero_row;
  size_t keys, perm, perm_tmp, sorted_leaf;
  size_t sort_hist;        // leaf sort: per-block counts of the coarse key digit, then their offsets
  size_t leaf_count, leaf_start, leaf_fill, scan_tmp;
  size_t coord2slot, slot2coord;
  size_t src;              // particle records {u_x, u_y, u_z, q} in the compute precision
  size_t src64;            // mixed: the same records in FP64 (P2P pair offsets)
  size_t q64;              // sorted charges (FP64)
  size_t far_phi, far_grad;  // far-field results per sorted particle (FP64)
  size_t mult64, mult32;   // multipole expansions, all levels (row stride mstride)
  size_t m2l_out;          // M2L results, all levels (compute precision)
  size_t loc_exp64;        // local expansions FP64, all levels (row stride mstride)
  size_t leaf_loc32;       // leaf local expansions FP32 (mixed; row stride mstride)
  size_t op_m2m, op_l2l;   // 8 octant operators each, FP64 [oct][row][k] (shift_kpad)
  size_t op_m2l64, op_m2l32;
  size_t multb;            // split M2L: multipoles as BF16 / FP16 pieces, all boxes
  size_t op_m2lb;          // split M2L: operators as BF16 / FP16 pieces
  size_t m2l_half;         // split M2L: parts 1.. of the split tail groups
  size_t m2l_ctl;          // persistent M2L: per-XCD tile counters (8)
  size_t f16_lmax;         // FP16 M2L: per level, max |M_k colf_k| (float bits; the level's scale)
  size_t f16_rowf;         // FP16 M2L: per operator row, the inverse row scale
  size_t f16_colf;         // FP16 M2L: per k, the inverse column scale (applied to multipoles)
  size_t f16_tbl;          // FP16 M2L: per (row, k), max |entry| over the operators (float bits)
  size_t op_m2l_scratch;   // FP16 M2L: FP64 operator entries [op][row][k] at plan time
  size_t work;             // 2 x int64 counters
  // Adaptive tree (leaf_max > 0).  Dense over every box of levels 0..L:
  size_t a_present;        // 1 where the box exists (all its ancestors were divided)
  size_t a_scan;           // exclusive scan of a_present: the box's compact index
  // Compact, one entry per existing box, level by level in Hilbert order:
  size_t a_slot;           // Hilbert slot within the level
  size_t a_level;          // level
  size_t a_coord;          // packed cell coordinates
  size_t a_range;          // {first sorted particle, count}
  size_t a_child0;         // compact index of the first of the 8 children, or -1 (leaf)
  size_t a_parent_of;      // at child0: the parent's index within its level
  size_t a_cnt, a_off;     // list sizes and offsets: 3 lists (U, W, X) x (bmax + 1)
  size_t a_uidx, a_widx, a_xidx;  // list entries (compact box indices)
  size_t a_wbox, a_xbox;   // compact lists of the boxes whose W / X list is not empty
  size_t a_flag, a_fscan;  // scratch of the compaction (bmax + 1 each)
  size_t a_tgt;            // M2L targets per level and parity class (rows within the level)
  size_t a_vtab;           // M2L source rows per (tile, class, offset, target); vtcap entries
  size_t a_p2p_bucket;     // P2P work-list: per box its cost bucket (255: no task)
  size_t a_p2p_list;       // P2P work-list: leaves by decreasing pair count
  size_t a_p2p_ctl;        // P2P work-list: 64 bucket offsets, the length, the ticket
  size_t a_small;          // per-level offsets and totals read back by the host
  size_t a_stats;          // 8 x int64 counters of the tree statistics
  int64_t bmax, ucap, wcap, xcap, vtcap, nbox_exp;  // bounds; nbox_exp = rows of the expansion arrays
  size_t total;
  int64_t n, nleaf, nbox, n_energy_part, scan_tmp_elems;
  int64_t lvl_off[FMM_DEPTH_MAX + 2];
};

bool make_layout(const fmm_config& cfg, int64_t n, Layout* lay);
// BF16 / FP16 pieces per operand of the M2L (2 or 3), or 0 for FP32/FP64 MFMA.
int m2l_pieces(const fmm_config& cfg);
bool m2l_is_f16(const fmm_config& cfg);  // FMM_M2L_F16X2

struct ProfileRec {
  int phase;
  hipEvent_t start, stop;
};

}  // namespace fmm

struct fmm_plan_s {
  fmm_config cfg;
  fmm::Layout lay;
  int64_t n;
  int L, p, nc;
  bool mixed;
  int m2l_np;    // m2l_pieces(cfg)
  bool m2l_f16;  // m2l_is_f16(cfg): the pieces are scaled FP16
  // Adaptive tree: L is the depth cap, Ld the deepest level that exists.
  bool adaptive;
  int Ld;
  int64_t ce_off[FMM_DEPTH_MAX + 2];  // compact index of the first box of each level
  int64_t nsplit[FMM_DEPTH_MAX + 1];  // divided boxes per level
  int64_t nlist[3];                   // U, W, X entries
  int64_t nwbox, nxbox;               // boxes with a non-empty W / X list
  int64_t a_tgt_off[FMM_DEPTH_MAX + 2];  // M2L target lists per level (entries)
  int64_t a_vt_off[FMM_DEPTH_MAX + 2];   // M2L source tables per level (entries)
  char* ws;
  hipStream_t last_stream;
  bool has_charges;  // fmm_evaluate has run: sorted charges are in the workspace
  // profiling
  uint32_t profile_mask;  // passes (bit 1 << FMM_PHASE_*) whose launches are timed
  bool prof_open;         // prof_begin recorded a start event not yet closed
  int nrec;
  fmm::ProfileRec* rec;  // kMaxProfile entries, events created lazily
  int nevents_created;
  bool is_static;  // the per-device plan of fmm_evaluate_static (not freed by fmm_destroy)
  bool ops_ready;  // the workspace holds the translation operators of (p, kind)
  // schedule (fmm_plan_set_schedule): work distribution only
  int p2p_persistent;  // adaptive P2P as a persistent kernel over the work-list
  int m2l_split;       // split-M2L tail work-groups per XCD (0 .. kM2lSplitPerXcd)
  int m2l_persistent;  // wide FP16 M2L as a persistent launch over per-XCD tile counters
  int p2p_tile;        // P2P sources per staged LDS tile (128, 256 or 512)
};

namespace fmm {

template <typename T>
inline T* wsp(fmm_plan_s* P, size_t off) {
  return reinterpret_cast<T*>(P->ws + off);
}

// ---- plan set-up and evaluation (defined in fmm_api.hip) ------------------
fmm_status validate_config_for(const fmm_config* cfg);
fmm_status plan_into(fmm_plan_s* P, const fmm_config& cfg, const Layout& lay, int64_t n,
                     const double* d_pos, char* ws, hipStream_t s, ProfileRec* rec,
                     bool keep_operators);
fmm_status evaluate_into(fmm_plan_s* P, const double* d_q, double* d_phi, double* d_force,
                         double* d_energy, hipStream_t s);

// ---- launch helpers (defined in fmm_api.hip) -------------------------------
void prof_begin(fmm_plan_s* P, int phase, hipStream_t s);
void prof_end(fmm_plan_s* P, hipStream_t s);

// ---- passes (each file defines its launchers) ------------------------------
hipError_t fill_u32(uint32_t* a, int64_t n, uint32_t v, hipStream_t s);  // a[0..n) = v
hipError_t launch_tree(fmm_plan_s* P, const double* d_pos, hipStream_t s);
hipError_t launch_operators(fmm_plan_s* P, hipStream_t s);
hipError_t launch_upward(fmm_plan_s* P, const double* d_q, hipStream_t s);
hipError_t launch_m2l(fmm_plan_s* P, hipStream_t s);
hipError_t launch_m2l_bf16(fmm_plan_s* P, hipStream_t s);  // split-BF16 form (P->m2l_np > 0)
hipError_t launch_m2m(fmm_plan_s* P, hipStream_t s);
hipError_t launch_l2l(fmm_plan_s* P, hipStream_t s);
hipError_t launch_downward(fmm_plan_s* P, hipStream_t s);
hipError_t launch_near_and_finish(fmm_plan_s* P, double* d_phi, double* d_force,
                                  double* d_energy, const double* adj_g, double* dEdq,
                                  double* dEdx, hipStream_t s);
hipError_t launch_leaves_out(fmm_plan_s* P, int32_t* d_cells, uint32_t* d_leaf, hipStream_t s);
hipError_t launch_work_count(fmm_plan_s* P, hipStream_t s);
hipError_t scan_exclusive(const uint32_t* in, int64_t n_valid, int64_t n, uint32_t* out,
                          uint32_t* tmp, hipStream_t s);
// adaptive tree (adaptive.hip)
hipError_t launch_adaptive_tree(fmm_plan_s* P, const double* d_pos, hipStream_t s);  // synchronises s
hipError_t launch_adaptive_upward(fmm_plan_s* P, hipStream_t s);
hipError_t launch_adaptive_p2l(fmm_plan_s* P, hipStream_t s);
hipError_t launch_adaptive_downward(fmm_plan_s* P, hipStream_t s);
hipError_t launch_adaptive_stats(fmm_plan_s* P, hipStream_t s);
hipError_t launch_p2p_worklist(fmm_plan_s* P, hipStream_t s);  // p2p.hip
hipError_t launch_l2p_adaptive(fmm_plan_s* P, hipStream_t s);  // downward.hip
// M2M / L2L over the divided boxes of the adaptive tree (shift.hip)
hipError_t launch_m2m_adaptive(fmm_plan_s* P, hipStream_t s);
hipError_t launch_l2l_adaptive(fmm_plan_s* P, hipStream_t s);
// First box and number of boxes (levels 2..) of the expansion arrays.
inline int64_t exp_box0(const fmm_plan_s* P) { return P->adaptive ? P->ce_off[2] : P->lay.lvl_off[2]; }
inline int64_t exp_nbox(const fmm_plan_s* P) {
  return P->adaptive ? P->ce_off[P->Ld + 1] : P->lay.nbox;
}

// ---- device helpers --------------------------------------------------------

// 3-D Hilbert index of cell (x, y, z) on a 2^bits grid: Skilling's transpose
// method (AIP Conf. Proc. 707:381, 2004) -- undo excess work from the top bit
// down, Gray-encode, then interleave the transposed bits, most significant
// first, in the order x, y, z.
__host__ __device__ inline uint64_t hilbert_index(uint32_t x, uint32_t y, uint32_t z, int bits) {
  if (bits <= 0) return 0;
  uint32_t X[3] = {x, y, z};
  const uint32_t top = 1u << (bits - 1);
  for (uint32_t Q = top; Q > 1; Q >>= 1) {
    const uint32_t Pm = Q - 1;
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= Pm;
      } else {
        const uint32_t t = (X[0] ^ X[i]) & Pm;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0;
  for (uint32_t Q = top; Q > 1; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1;
  X[0] ^= t;
  X[1] ^= t;
  X[2] ^= t;
  uint64_t h = 0;
  for (int b = bits - 1; b >= 0; --b)
    for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> b) & 1u);
  return h;
}

__host__ __device__ inline uint32_t pack_coord(uint32_t x, uint32_t y, uint32_t z) {
  return (x << 20) | (y << 10) | z;
}
__host__ __device__ inline void unpack_coord(uint32_t c, int& x, int& y, int& z) {
  x = (int)(c >> 20);
  y = (int)((c >> 10) & 1023u);
  z = (int)(c & 1023u);
}
__host__ __device__ inline int64_t lex_index(int x, int y, int z, int l) {
  return ((int64_t)x << (2 * l)) | ((int64_t)y << l) | (int64_t)z;
}

// Per sorted particle: its box-unit offset from its leaf centre and its
// charge, one 16-byte (FP32) or 32-byte (FP64) record.
template <typename T>
struct alignas(4 * sizeof(T)) Rec {
  T x, y, z, q;
};

// Real packing of the coefficients of a real-valued expansion: degree n owns
// entries n^2 .. n^2 + 2n as [Re c_n^0, Re c_n^1, Im c_n^1, ..., Re c_n^n, Im c_n^n];
// negative orders follow from c_n^{-m} = (-1)^m conj(c_n^m).
__host__ __device__ constexpr int cidx_re(int n, int m) { return m == 0 ? n * n : n * n + 2 * m - 1; }
__host__ __device__ constexpr int cidx_im(int n, int m) { return n * n + 2 * m; }
__host__ __device__ constexpr int tri(int n, int m) { return n * (n + 1) / 2 + m; }

// Regular solid harmonics R_n^m(x) = r^n P_n^m(cos t) e^{i m f} / (n+m)!
// (Condon-Shortley phase) for 0 <= m <= n <= P, by the three-term recurrences
//   R_m^m = -(x + i y)/(2m) R_{m-1}^{m-1},  R_{m+1}^m = z R_m^m,
//   (n-m)(n+m) R_n^m = (2n-1) z R_{n-1}^m - r^2 R_{n-2}^m.
// Outputs are indexed by tri(n, m).
template <int P, typename T>
__device__ __forceinline__ void regular_harmonics(T x, T y, T z, T* re, T* im) {
  const T r2 = x * x + y * y + z * z;
  re[0] = T(1);
  im[0] = T(0);
#pragma unroll
  for (int m = 0; m <= P; ++m) {
    if (m > 0) {
      const T s = T(-1.0 / (2.0 * m));
      const T pr = re[tri(m - 1, m - 1)], pi = im[tri(m - 1, m - 1)];
      re[tri(m, m)] = s * (x * pr - y * pi);
      im[tri(m, m)] = s * (x * pi + y * pr);
    }
    if (m + 1 <= P) {
      re[tri(m + 1, m)] = z * re[tri(m, m)];
      im[tri(m + 1, m)] = z * im[tri(m, m)];
    }
#pragma unroll
    for (int n = m + 2; n <= P; ++n) {
      const T a = T((2.0 * n - 1.0) / ((double)(n - m) * (double)(n + m)));
      const T b = T(1.0 / ((double)(n - m) * (double)(n + m)));
      re[tri(n, m)] = a * z * re[tri(n - 1, m)] - b * r2 * re[tri(n - 2, m)];
      im[tri(n, m)] = a * z * im[tri(n - 1, m)] - b * r2 * im[tri(n - 2, m)];
    }
  }
}

// M2L operators are numbered lexicographically over the offsets o in
// [-3,3]^3 with max |o_a| >= 2 (the 316 possible target-minus-source offsets of
// interaction-list boxes).
__host__ __device__ inline void m2l_offset(int op, int o[3]) {
  int idx = 0;
  for (int a = -3; a <= 3; ++a)
    for (int b = -3; b <= 3; ++b)
      for (int c = -3; c <= 3; ++c) {
        if (a >= -1 && a <= 1 && b >= -1 && b <= 1 && c >= -1 && c <= 1) continue;
        if (idx == op) {
          o[0] = a;
          o[1] = b;
          o[2] = c;
        }
        ++idx;
      }
}

__host__ __device__ constexpr int clamp03(int v) { return v < 0 ? 0 : (v > 3 ? 3 : v); }

// Inverse of m2l_offset: lexicographic position in [-3,3]^3 minus the number
// of inner ([-1,1]^3) offsets that precede it.
__host__ __device__ constexpr int m2l_op_index(int ox, int oy, int oz) {
  const int a = ox + 3, b = oy + 3, c = oz + 3;
  int before = 9 * clamp03(a - 2);
  if (a >= 2 && a <= 4) {
    before += 3 * clamp03(b - 2);
    if (b >= 2 && b <= 4) before += clamp03(c - 2);
  }
  return a * 49 + b * 7 + c - before;
}

// Dispatch a templated functor on the expansion order p (0..FMM_P_MAX).
template <template <int> class F, typename... Args>
inline hipError_t dispatch_p(int p, Args&&... args) {
  switch (p) {
    case 0: return F<0>::run(args...);
    case 1: return F<1>::run(args...);
    case 2: return F<2>::run(args...);
    case 3: return F<3>::run(args...);
    case 4: return F<4>::run(args...);
    case 5: return F<5>::run(args...);
    case 6: return F<6>::run(args...);
    case 7: return F<7>::run(args...);
    case 8: return F<8>::run(args...);
    case 9: return F<9>::run(args...);
    case 10: return F<10>::run(args...);
    case 11: return F<11>::run(args...);
    case 12: return F<12>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace fmm
