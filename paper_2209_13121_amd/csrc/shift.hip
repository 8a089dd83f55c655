// shift.hip -- M2M and L2L on the FP64 matrix cores.
//
// Both translations use the 8 level-free octant matrices (operators.hip), so
// each level is a set of dense products batched by octant:
//   M2M  M~p[:, parents]          = sum_o A_o * M~[:, child of octant o]
//   L2L  L~[:, children of oct o] = (1/h) M2L[:, ...] + B_o * L~[:, parents]
// FP64 in both precision modes.  Three forms:
//  * k_shift (row-block form): one work-group owns one 16-row block of the
//    expansions and 8 tiles of 16 targets, one tile per wave: 128 parents for
//    M2M, the octant-o children of 128 parents for L2L.  The row block's rows
//    of the operators it needs (all 8 octants for M2M, octant o for L2L) are
//    staged in LDS once and shared by the 8 waves; the grid runs over (row
//    block, tiles), so even the coarse levels spread over many work-groups.
//    L2L's coarse levels (and M2M at p >= 12) run here.
//  * k_shift_oct (coarse M2M, p <= 11): as above, but the 8 waves take the 8
//    octants of 1-4 column tiles, whose partials are added through LDS.
//  * k_shift_rows (fine levels, p <= 8): a work-group computes every row
//    block of 128 columns, so each source column is loaded once.
//  * The translations are triangular in degree: a parent multipole of degree
//    n takes child degrees <= n only, a child local of degree n parent
//    degrees >= n only (the addition theorems of the solid harmonics;
//    Greengard 1988, ch. 3).  A row block stages and runs only the k steps
//    that can be non-zero for its rows; the skipped products are exact zeros.
//  * K order: step t of pair q uses k = 8 q + 2 g + t in lane group g, so a
//    lane's A and B values of a pair are one 16-byte load each.  LDS rows are
//    a multiple of 2 mod 4 16-byte units apart, which keeps the 32 lanes a
//    16-byte read serves at once on distinct banks.
#include "fmm_internal.h"

namespace fmm {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
// 16-byte operator loads a thread has in flight while staging rows in LDS:
// the loads of a batch are all issued before its first LDS store, so a
// staging pass costs a memory round trip per batch, not per load.
constexpr int kStageBatch = 8;
// s_waitcnt operand: vector memory count 0, the other counters unconstrained
// (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kVmcntZero = 0x0F70;
template <int N>
constexpr int kVmcntNQ = 0x0F70 | (N & 15) | ((N >> 4) << 14);  // vector memory count N (< 64)

template <int P, int MODE>
struct ShiftShape {
  static constexpr int NC = (P + 1) * (P + 1);
  static constexpr int RB = (NC + 15) / 16;
  static constexpr int MS = mstride_of(NC);
  static constexpr int KP = shift_kpad(NC);
  static constexpr int NQ = KP / 8;  // k pairs of steps
  static constexpr int RS = (KP / 2) % 4 == 2 ? KP / 2 : KP / 2 + (6 - (KP / 2) % 4) % 4;  // row stride (16 B)
  static constexpr int NOCT = MODE == 0 ? 8 : 1;  // octants staged
  // M2M at large orders stages the octants in two halves (LDS size)
  static constexpr int OCT_STAGE = NOCT * 16 * RS * 16 <= 150 * 1024 ? NOCT : NOCT / 2;
  static_assert(RS % 4 == 2 && RS >= KP / 2, "LDS row stride");
};
// LDS units (16 bytes) of the all-rows form: every row of one octant, in
// whole wave copies of 64 units
template <int P>
constexpr int kRowsUnits = ((ShiftShape<P, 0>::RB * 16 * ShiftShape<P, 0>::RS + 63) / 64) * 64;

// Degree of packed coefficient index c (c = n^2 .. n^2 + 2n).
__device__ __forceinline__ int degree_of(int c) {
  int n = (int)sqrtf((float)c);
  while (n * n > c) --n;
  while ((n + 1) * (n + 1) <= c) ++n;
  return n;
}

struct ShiftArgs {
  int l;               // level of the targets
  int mixed;           // source (M2M) / destination (L2L leaf) is FP32
  int leaf;            // L2L: this level is the leaf level
  int64_t nparent;     // M2M: parents at level l; L2L: parents at level l-1
  int64_t ngroups;     // work-groups in the launch
  const uint32_t* s2c_child;  // slot -> coord of the child level
  const double* ops;          // 8 operators [oct][row][KP]
  const void* src;            // M2M: child multipoles (stride MS); L2L: parent locals (stride MS)
  double* dst64;              // M2M: parent multipoles; L2L: child locals (stride MS)
  float* dst32;               // M2M mixed: FP32 copy of the parents; L2L mixed leaf: leaf locals
  const void* m2l;            // L2L: M2L results of the children (stride NC, FP32 if mixed)
  const DevParams* dp;
  // Adaptive tree: target column ps is the ps-th divided parent, whose row
  // within its level is parent_of[8 ps] (children 8 ps .. 8 ps + 7 of the
  // child level); null for the uniform tree (row ps).
  const uint32_t* parent_of;
};

// TM: the L2L's M2L results' type (float in the mixed mode).
template <int P, int MODE, typename TM = double>
__global__ __launch_bounds__(kThreads) void k_shift(ShiftArgs a) {
  typedef ShiftShape<P, MODE> S;
  constexpr int NC = S::NC, RB = S::RB, MS = S::MS, KP = S::KP, NQ = S::NQ, RS = S::RS;
  constexpr int OCT_STAGE = S::OCT_STAGE;
  __shared__ f64x2 sA[OCT_STAGE * 16 * RS];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kg = lane >> 4;
  // group -> (row block, 8 tiles); L2L groups of the 8 octants of the same
  // parents are adjacent (they read the same parent locals).  XCD-aware
  // order: hardware group b runs on XCD b % 8 and each XCD gets a contiguous
  // range of logical groups, so the groups that read the same sources share
  // an L2.
  const int64_t per_xcd = (a.ngroups + 7) / 8;
  const int64_t g = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (g >= a.ngroups) return;  // uniform over the work-group
  const int rb = (int)(g % RB);
  const int64_t rest = g / RB;
  const int oct_l2l = MODE == 1 ? (int)(rest % 8) : 0;
  const int64_t pgroup = MODE == 1 ? rest / 8 : rest;
  const int64_t ps = (pgroup * kWaves + wave) * 16 + col;  // parent slot of this column
  const bool ok = ps < a.nparent;
  const int64_t prow = !ok ? 0 : (a.parent_of ? (int64_t)a.parent_of[8 * ps] : ps);

  // child slot of each octant (children of slot ps are slots 8 ps .. 8 ps + 7),
  // packed 3 bits per octant
  uint32_t child_bits = 0;
  if (ok) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      int x, y, z;
      unpack_coord(a.s2c_child[8 * ps + c], x, y, z);
      child_bits |= (uint32_t)c << (3 * (((x & 1) << 2) | ((y & 1) << 1) | (z & 1)));
    }
  }
  auto child_of = [&](int oct) { return (int)((child_bits >> (3 * oct)) & 7u); };

  // k pairs this row block can touch (exact zeros outside)
  const int row0 = 16 * rb;
  int q0, q1;
  if (MODE == 0) {  // lower: k of degree <= deg(last row)
    const int d = degree_of(min(row0 + 15, NC - 1));
    q0 = 0;
    q1 = ((d + 1) * (d + 1) + 7) / 8;
  } else {  // upper: k of degree >= deg(first row)
    const int d = degree_of(row0);
    q0 = (d * d) / 8;
    q1 = NQ;
  }

  f64x4 acc0 = f64x4{0, 0, 0, 0}, acc1 = f64x4{0, 0, 0, 0};
  for (int o0 = 0; o0 < S::NOCT; o0 += OCT_STAGE) {
    // stage rows row0..row0+15, pairs q0..q1-1, of octants o0.. (M2M) or oct_l2l (L2L)
    if (o0 > 0) __syncthreads();
    const int npair = q1 - q0;  // 16-byte units per row = 4 per pair
    const int ne = OCT_STAGE * 16 * 4 * npair;
    for (int e0 = 0; e0 < ne; e0 += kStageBatch * kThreads) {
      f64x2 st[kStageBatch];  // every load of the batch in flight before the first store
#pragma unroll
      for (int i = 0; i < kStageBatch; ++i) {
        const int e = e0 + tid + i * kThreads;
        const int u = e % (4 * npair), r = e / (4 * npair) % 16, oo = e / (4 * npair * 16);
        const int oct = MODE == 0 ? o0 + oo : oct_l2l;
        if (e < ne)
          st[i] = *reinterpret_cast<const f64x2*>(a.ops + ((size_t)oct * (RB * 16) + row0 + r) * KP +
                                                  8 * q0 + 2 * u);
      }
#pragma unroll
      for (int i = 0; i < kStageBatch; ++i) {
        const int e = e0 + tid + i * kThreads;
        const int u = e % (4 * npair), r = e / (4 * npair) % 16, oo = e / (4 * npair * 16);
        if (e < ne) sA[(oo * 16 + r) * RS + 4 * q0 + u] = st[i];
      }
    }
    __syncthreads();
    // B pairs of octant oct: unconditional loads at clamped addresses (so
    // a whole octant's loads are in flight together), then zeroed where the
    // source does not exist or k is past the row
    auto load_b = [&](int oct, f64x2* bv) {
      const bool have = ok;
      const int64_t srow = !have ? 0 : (MODE == 0 ? 8 * ps + child_of(oct) : prow);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int k = 8 * q + 2 * kg;
        const int k0 = k < MS ? k : MS - 2;
        f64x2 v;
        if (MODE == 0 && a.mixed) {
          const f32x2 w = *reinterpret_cast<const f32x2*>(static_cast<const float*>(a.src) +
                                                          srow * MS + k0);
          v = f64x2{(double)w[0], (double)w[1]};
        } else {
          v = *reinterpret_cast<const f64x2*>(static_cast<const double*>(a.src) + srow * MS + k0);
        }
        bv[q] = (have && k < MS) ? v : f64x2{0.0, 0.0};
      }
    };
    f64x2 bcur[NQ], bnext[NQ];
    load_b(MODE == 0 ? o0 : oct_l2l, bcur);
#pragma unroll
    for (int oo = 0; oo < OCT_STAGE; ++oo) {
      if (oo + 1 < OCT_STAGE) load_b(o0 + oo + 1, bnext);  // M2M: next octant in flight
      const f64x2* sa = sA + (oo * 16 + col) * RS + kg;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (q < q0 || q >= q1) continue;  // uniform over the work-group
        const f64x2 av = sa[4 * q];
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0], bcur[q][0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1], bcur[q][1], acc1, 0, 0, 0);
      }
      if (oo + 1 < OCT_STAGE) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) bcur[q] = bnext[q];
      }
    }
  }
  const f64x4 acc = acc0 + acc1;

  // The f64 accumulator gives lane (col, kg) rows 16 rb + kg + 4 i.  Transpose
  // across the 4 lanes of a column so that it holds rows 16 rb + 4 kg + j,
  // j = 0..3, and writes them as one 16- or 32-byte vector: in round t lane
  // (col, j) offers its value i = (j - t) mod 4 and lane (col, kg) takes it
  // from lane (col, (kg + t) mod 4), which is row 4 kg + (kg + t) mod 4.
  double v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int i_send = (kg - t) & 3;
    const double send = i_send == 0 ? acc[0] : i_send == 1 ? acc[1] : i_send == 2 ? acc[2] : acc[3];
    const int from = ((kg + t) & 3) * 16 + col;
    const double got = __shfl(send, from);
    const int j = (kg + t) & 3;
    if (j == 0) v[0] = got;
    if (j == 1) v[1] = got;
    if (j == 2) v[2] = got;
    if (j == 3) v[3] = got;
  }
  const int rr = row0 + 4 * kg;  // this lane's 4 rows; MS % 4 == 0, so all or none < MS
  if (!ok || rr >= MS) return;
  if (MODE == 0) {  // rows NC..MS-1 are zero (zero operator rows)
    *reinterpret_cast<f64x2*>(a.dst64 + prow * MS + rr) = f64x2{v[0], v[1]};
    *reinterpret_cast<f64x2*>(a.dst64 + prow * MS + rr + 2) = f64x2{v[2], v[3]};
    if (a.dst32)
      *reinterpret_cast<f32x4*>(a.dst32 + prow * MS + rr) =
          f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  } else {
    const int64_t cs = 8 * ps + child_of(oct_l2l);
    const double inv_h = (double)(1 << a.l) / a.dp->side;
    TM w[4];  // all four loads in flight before the first use
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = static_cast<const TM*>(a.m2l)[cs * NC + (rr + j < NC ? rr + j : 0)];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (rr + j < NC) v[j] += inv_h * (double)w[j];
    // uniform leaf level (mixed): FP32 only; otherwise FP64, plus an FP32 copy
    // where dst32 is given (adaptive, mixed: every level holds leaves)
    if (!(a.leaf && a.mixed)) {
      *reinterpret_cast<f64x2*>(a.dst64 + cs * MS + rr) = f64x2{v[0], v[1]};
      *reinterpret_cast<f64x2*>(a.dst64 + cs * MS + rr + 2) = f64x2{v[2], v[3]};
    }
    if (a.dst32)
      *reinterpret_cast<f32x4*>(a.dst32 + cs * MS + rr) =
          f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  }
}

// Coarse M2M levels (few parents): the 8 waves of a work-group take the 8
// octants of one 16-row block for NT column tiles of 16 parents, so a level
// spreads over (parents / 16 NT) x RB work-groups instead of k_shift's
// (parents / 128) x RB, each wave running NT octant products instead of 8.
// The octant partials of every column are then added in octant order through
// LDS (the staged rows' space).  For p with all 8 octants' rows in LDS.
template <int P, int NT, typename TS>
__global__ __launch_bounds__(kThreads) void k_shift_oct(ShiftArgs a) {
  typedef ShiftShape<P, 0> S;
  typedef TS TS2 __attribute__((ext_vector_type(2)));  // the sources' type, as loaded
  constexpr int NC = S::NC, RB = S::RB, MS = S::MS, KP = S::KP, NQ = S::NQ, RS = S::RS;
  static_assert(S::OCT_STAGE == 8, "every octant's rows staged at once");
  // 16-byte LDS units: the staged rows, then the partials (8 NT tiles of 64
  // lanes x 32 bytes)
  constexpr int kUnits = 8 * 16 * RS > 8 * NT * 64 * 2 ? 8 * 16 * RS : 8 * NT * 64 * 2;
  __shared__ f64x2 sA[kUnits];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kg = lane >> 4;
  const int64_t per_xcd = (a.ngroups + 7) / 8;
  const int64_t g = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (g >= a.ngroups) return;  // uniform over the work-group
  const int rb = (int)(g % RB);
  const int64_t pgroup = g / RB;
  const int row0 = 16 * rb;
  const int d = degree_of(min(row0 + 15, NC - 1));
  const int q1 = ((d + 1) * (d + 1) + 7) / 8;  // k pairs the block can touch (lower in degree)

  // stage rows row0 .. row0 + 15 of the 8 octants, pairs 0 .. q1 - 1, by DMA
  // from global memory into LDS, 64 units per wave instruction: LDS unit e is
  // octant row e / RS (octant (e / RS) / 16, row row0 + (e / RS) % 16),
  // 16-byte unit e % RS; units past the block's pairs (never read) fetch the
  // row's first unit.  In flight together with the first tile's sources.
  for (int e0 = wave * 64; e0 < 8 * 16 * RS; e0 += kThreads) {
    const int e = e0 + lane;
    const int orow = e / RS, u = e % RS;
    const bool v = u < 4 * q1;
    __builtin_amdgcn_global_load_lds(
        (__attribute__((address_space(1))) void*)(a.ops + ((size_t)(orow >> 4) * (RB * 16) + row0 + (orow & 15)) * KP +
                                                  (v ? 2 * u : 0)),
        (__attribute__((address_space(3))) void*)(sA + e0), 16, 0, 0);
  }

  // this wave's octant: the child of each parent in that octant
  const int oct = wave;
  auto load_b = [&](int t, TS2* bv) {
    const int64_t ps = (pgroup * NT + t) * 16 + col;
    const bool ok = ps < a.nparent;
    int child = 0;
    if (ok)
      for (int c = 0; c < 8; ++c) {
        int x, y, z;
        unpack_coord(a.s2c_child[8 * ps + c], x, y, z);
        if ((((x & 1) << 2) | ((y & 1) << 1) | (z & 1)) == oct) child = c;
      }
    const int64_t srow = ok ? 8 * ps + child : 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = 8 * q + 2 * kg;
      const int k0 = k < MS ? k : MS - 2;
      const TS2 v = *reinterpret_cast<const TS2*>(static_cast<const TS*>(a.src) + srow * MS + k0);
      bv[q] = (ok && k < MS) ? v : TS2{TS(0), TS(0)};
    }
  };
  TS2 bcur[NQ], bnext[NQ];
  load_b(0, bcur);
  __builtin_amdgcn_s_waitcnt(kVmcntZero);  // this wave's copies have landed
  __syncthreads();
  f64x4 part[NT];
  const f64x2* sa = sA + (oct * 16 + col) * RS + kg;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t + 1 < NT) load_b(t + 1, bnext);  // the next tile's sources in flight
    f64x4 acc0 = f64x4{0, 0, 0, 0}, acc1 = f64x4{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (q >= q1) continue;  // uniform over the work-group
      const f64x2 av = sa[4 * q];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0], (double)bcur[q][0], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1], (double)bcur[q][1], acc1, 0, 0, 0);
    }
    part[t] = acc0 + acc1;
    if (t + 1 < NT) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) bcur[q] = bnext[q];
    }
  }
  // the octant partials through LDS, added in octant order by waves 0 .. NT - 1
  __syncthreads();  // every wave is done with the staged rows
  f64x4* sP = reinterpret_cast<f64x4*>(sA);
#pragma unroll
  for (int t = 0; t < NT; ++t) sP[(wave * NT + t) * 64 + lane] = part[t];
  __syncthreads();
  if (wave >= NT) return;  // uniform over the wave
  const int t = wave;
  f64x4 acc = sP[t * 64 + lane];
#pragma unroll
  for (int o = 1; o < 8; ++o) acc += sP[(o * NT + t) * 64 + lane];
  // transpose across the 4 lanes of a column (as in k_shift): this lane then
  // holds rows 16 rb + 4 kg + j, j = 0..3
  double v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i_send = (kg - r) & 3;
    const double send = i_send == 0 ? acc[0] : i_send == 1 ? acc[1] : i_send == 2 ? acc[2] : acc[3];
    const double got = __shfl(send, ((kg + r) & 3) * 16 + col);
    const int j = (kg + r) & 3;
    if (j == 0) v[0] = got;
    if (j == 1) v[1] = got;
    if (j == 2) v[2] = got;
    if (j == 3) v[3] = got;
  }
  const int64_t ps = (pgroup * NT + t) * 16 + col;
  const int rr = row0 + 4 * kg;  // MS % 4 == 0: all 4 rows or none < MS
  if (ps >= a.nparent || rr >= MS) return;
  const int64_t prow = a.parent_of ? (int64_t)a.parent_of[8 * ps] : ps;
  *reinterpret_cast<f64x2*>(a.dst64 + prow * MS + rr) = f64x2{v[0], v[1]};
  *reinterpret_cast<f64x2*>(a.dst64 + prow * MS + rr + 2) = f64x2{v[2], v[3]};
  if (a.dst32)
    *reinterpret_cast<f32x4*>(a.dst32 + prow * MS + rr) = f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
}

// Fine levels: one work-group per 128 target columns computes every row
// block, so each source column is loaded once (the kernel above re-reads it
// once per row block) and each target's rows are written together.  The
// operator rows of one octant (all row blocks, only the k steps each row
// block can touch) are staged in LDS per octant; M2M runs the 8 octants in
// turn with the next octant's sources in flight, L2L one octant per
// work-group.  Used where the row blocks' accumulators and the source
// registers fit (at most 6 row blocks, p <= 8) and the level has enough
// columns to fill the chip.
// TS: the sources' type (float: the FP32 leaf multipoles of the mixed uniform
// tree, kept as loaded until their products, so their loads stay in flight);
// TM: the L2L's M2L results' type (float in the mixed mode), likewise.
template <int P, int MODE, typename TS, typename TM = double>
__global__ __launch_bounds__(kThreads) void k_shift_rows(ShiftArgs a) {
  typedef ShiftShape<P, MODE> S;
  typedef TS TS2 __attribute__((ext_vector_type(2)));
  constexpr int NC = S::NC, RB = S::RB, MS = S::MS, KP = S::KP, NQ = S::NQ, RS = S::RS;
  // M2M: two operator buffers (one work-group per CU); L2L: one (two per CU)
  __shared__ f64x2 sA[(MODE == 0 ? 2 : 1) * kRowsUnits<P>];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, kg = lane >> 4;
  // group -> (8 tiles of 16 parents[, octant]), XCD-aware as above
  const int64_t per_xcd = (a.ngroups + 7) / 8;
  const int64_t g = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (g >= a.ngroups) return;  // uniform over the work-group
  const int oct_l2l = MODE == 1 ? (int)(g % 8) : 0;
  const int64_t pgroup = MODE == 1 ? g / 8 : g;
  const int64_t ps = (pgroup * kWaves + wave) * 16 + col;
  const bool ok = ps < a.nparent;
  const int64_t prow = !ok ? 0 : (a.parent_of ? (int64_t)a.parent_of[8 * ps] : ps);
  uint32_t child_bits = 0;
  if (ok) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      int x, y, z;
      unpack_coord(a.s2c_child[8 * ps + c], x, y, z);
      child_bits |= (uint32_t)c << (3 * (((x & 1) << 2) | ((y & 1) << 1) | (z & 1)));
    }
  }
  auto child_of = [&](int oct) { return (int)((child_bits >> (3 * oct)) & 7u); };
  // k pairs row block rb can touch (exact zeros outside): M2M lower, L2L upper
  auto qrange = [&](int rb, int& q0, int& q1) {
    if (MODE == 0) {
      const int d = degree_of(min(16 * rb + 15, NC - 1));
      q0 = 0;
      q1 = ((d + 1) * (d + 1) + 7) / 8;
    } else {
      const int d = degree_of(16 * rb);
      q0 = (d * d) / 8;
      q1 = NQ;
    }
  };
  auto load_b = [&](int oct, TS2* bv) {
    const int64_t srow = !ok ? 0 : (MODE == 0 ? 8 * ps + child_of(oct) : prow);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = 8 * q + 2 * kg;
      const int k0 = k < MS ? k : MS - 2;
      const TS2 v = *reinterpret_cast<const TS2*>(static_cast<const TS*>(a.src) + srow * MS + k0);
      bv[q] = (ok && k < MS) ? v : TS2{TS(0), TS(0)};
    }
  };
  // stage every row of octant oct, the k pairs of its row block only, by DMA
  // from global memory into LDS buffer buf, 64 units per wave instruction: LDS
  // unit e is row e / RS, 16-byte unit e % RS; units outside the block's k
  // pairs (never read) fetch the row's first unit.
  auto stage = [&](int oct, f64x2* buf) {
    for (int e0 = wave * 64; e0 < kRowsUnits<P>; e0 += kThreads) {
      const int e = e0 + lane;
      const int row = e / RS < RB * 16 ? e / RS : 0, u = e % RS, q = u / 4;
      int q0, q1;
      qrange(row / 16, q0, q1);
      const bool v = u < 4 * NQ && q >= q0 && q < q1;
      __builtin_amdgcn_global_load_lds(
          (__attribute__((address_space(1))) void*)(a.ops + ((size_t)oct * (RB * 16) + row) * KP + (v ? 2 * u : 0)),
          (__attribute__((address_space(3))) void*)(buf + e0), 16, 0, 0);
    }
  };
  // the products of one octant: rows of LDS buffer buf times sources b
  f64x4 acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = f64x4{0, 0, 0, 0};
  auto products = [&](const f64x2* buf, const TS2* b) {
    f64x2 bq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) bq[q] = f64x2{(double)b[q][0], (double)b[q][1]};
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      int q0, q1;
      qrange(rb, q0, q1);
      const f64x2* sa = buf + (16 * rb + col) * RS + kg;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (q < q0 || q >= q1) continue;  // uniform over the work-group
        const f64x2 av = sa[4 * q];
        acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0], bq[q][0], acc[rb], 0, 0, 0);
        acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1], bq[q][1], acc[rb], 0, 0, 0);
      }
    }
  };
  const int64_t cs = MODE == 1 && ok ? 8 * ps + child_of(oct_l2l) : 0;
  if constexpr (MODE == 1) {
    TS2 b[NQ];
    load_b(oct_l2l, b);
    // L2L: the child's (1/h) M2L result starts the accumulators (lane (col, kg)
    // holds rows 16 rb + kg + 4 i of its column); loaded here, so the loads are
    // in flight while the operator rows are staged (rows past ncoef, or a
    // column past the level, read row 0 and are not used)
    TM m2lv[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * rb + kg + 4 * i;
        m2lv[rb][i] = static_cast<const TM*>(a.m2l)[cs * NC + (ok && row < NC ? row : 0)];
      }
    stage(oct_l2l, sA);
    __builtin_amdgcn_s_waitcnt(kVmcntZero);  // this wave's copies have landed
    __syncthreads();
    const double inv_h = (double)(1 << a.l) / a.dp->side;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (ok && 16 * rb + kg + 4 * i < NC) acc[rb][i] = inv_h * (double)m2lv[rb][i];
    products(sA, b);
  } else {
    // M2M, the 8 octants in turn: octant o + 1's rows are copied into the
    // other LDS buffer while octant o's products run, and each octant's
    // sources are loaded two octants ahead (three register buffers).  The wait
    // at the end of octant o leaves only octant o + 2's source loads, issued
    // after the copy, in flight.
    TS2 b[3][NQ];
    stage(0, sA);
    load_b(0, b[0]);
    load_b(1, b[1]);
    __builtin_amdgcn_s_waitcnt(kVmcntZero);
    __syncthreads();
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      if (o + 1 < 8) stage(o + 1, sA + ((o + 1) & 1) * kRowsUnits<P>);
      __builtin_amdgcn_sched_barrier(0);  // the copy is issued before the source loads
      if (o + 2 < 8) load_b(o + 2, b[(o + 2) % 3]);
      products(sA + (o & 1) * kRowsUnits<P>, b[o % 3]);
      if (o + 1 < 8) {
        if (o + 2 < 8)
          __builtin_amdgcn_s_waitcnt(kVmcntNQ<NQ>);  // all but octant o + 2's NQ source loads
        else
          __builtin_amdgcn_s_waitcnt(kVmcntZero);
        __syncthreads();  // octant o + 1's rows are in; octant o's buffer is free
      }
    }
  }
  if (!ok) return;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const f64x4 acc_rb = acc[rb];
    // transpose across the 4 lanes of a column (as in k_shift): this lane then
    // holds rows 16 rb + 4 kg + j, j = 0..3
    double v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i_send = (kg - t) & 3;
      const double send = i_send == 0 ? acc_rb[0] : i_send == 1 ? acc_rb[1] : i_send == 2 ? acc_rb[2] : acc_rb[3];
      const double got = __shfl(send, ((kg + t) & 3) * 16 + col);
      const int j = (kg + t) & 3;
      if (j == 0) v[0] = got;
      if (j == 1) v[1] = got;
      if (j == 2) v[2] = got;
      if (j == 3) v[3] = got;
    }
    const int rr = 16 * rb + 4 * kg;
    if (rr >= MS) continue;
    if (MODE == 0) {
      *reinterpret_cast<f64x2*>(a.dst64 + prow * MS + rr) = f64x2{v[0], v[1]};
      *reinterpret_cast<f64x2*>(a.dst64 + prow * MS + rr + 2) = f64x2{v[2], v[3]};
      if (a.dst32)
        *reinterpret_cast<f32x4*>(a.dst32 + prow * MS + rr) =
            f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    } else {
      if (!(a.leaf && a.mixed)) {
        *reinterpret_cast<f64x2*>(a.dst64 + cs * MS + rr) = f64x2{v[0], v[1]};
        *reinterpret_cast<f64x2*>(a.dst64 + cs * MS + rr + 2) = f64x2{v[2], v[3]};
      }
      if (a.dst32)
        *reinterpret_cast<f32x4*>(a.dst32 + cs * MS + rr) =
            f32x4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
    }
  }
}

// Columns from which a level runs the all-rows form (64 work-groups of 128
// columns: below that the per-row-block form spreads the level over more
// work-groups).
constexpr int64_t kRowsMinColumns = 64 * 128;

template <int P>
struct ShiftRun {
  static hipError_t run(ShiftArgs a, int mode, hipStream_t s) {
    typedef ShiftShape<P, 0> S;
    const int64_t pgroups = (a.nparent + 16 * kWaves - 1) / (16 * kWaves);
    if constexpr (S::RB <= 6) {
      if (a.nparent * (mode == 1 ? 8 : 1) >= kRowsMinColumns) {
        a.ngroups = pgroups * (mode == 1 ? 8 : 1);
        const unsigned grid = (unsigned)(((a.ngroups + 7) / 8) * 8);
        if (mode == 1 && a.mixed)
          k_shift_rows<P, 1, double, float><<<grid, kThreads, 0, s>>>(a);
        else if (mode == 1)
          k_shift_rows<P, 1, double, double><<<grid, kThreads, 0, s>>>(a);
        else if (a.mixed)
          k_shift_rows<P, 0, float><<<grid, kThreads, 0, s>>>(a);
        else
          k_shift_rows<P, 0, double><<<grid, kThreads, 0, s>>>(a);
        return hipGetLastError();
      }
    }
    if constexpr (S::OCT_STAGE == 8) {
      if (mode == 0) {  // coarse M2M: octants over the waves, NT column tiles each
        const int nt = a.nparent >= 2048 ? 4 : a.nparent >= 256 ? 2 : 1;
        a.ngroups = ((a.nparent + 16 * nt - 1) / (16 * nt)) * S::RB;
        const unsigned grid = (unsigned)(((a.ngroups + 7) / 8) * 8);
        auto go = [&](auto ts) {
          typedef decltype(ts) TS;
          if (nt == 4)
            k_shift_oct<P, 4, TS><<<grid, kThreads, 0, s>>>(a);
          else if (nt == 2)
            k_shift_oct<P, 2, TS><<<grid, kThreads, 0, s>>>(a);
          else
            k_shift_oct<P, 1, TS><<<grid, kThreads, 0, s>>>(a);
        };
        if (a.mixed)
          go(float{});
        else
          go(double{});
        return hipGetLastError();
      }
    }
    a.ngroups = pgroups * S::RB * (mode == 1 ? 8 : 1);
    const unsigned grid = (unsigned)(((a.ngroups + 7) / 8) * 8);
    if (mode == 0)
      k_shift<P, 0><<<grid, kThreads, 0, s>>>(a);
    else if (a.mixed)
      k_shift<P, 1, float><<<grid, kThreads, 0, s>>>(a);
    else
      k_shift<P, 1, double><<<grid, kThreads, 0, s>>>(a);
    return hipGetLastError();
  }
};

// Level 2 locals: L~ = (1/h) * M2L result (no parent contribution), into
// dst64 and / or dst32 (whichever is given).
template <typename TM>
__global__ void k_l2l_top(int nc, int ms, int l, int64_t nbox, const DevParams* __restrict__ dp,
                          const TM* __restrict__ m2l, double* __restrict__ dst64,
                          float* __restrict__ dst32) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nbox * ms) return;
  const int64_t b = e / ms;
  const int row = (int)(e % ms);
  const double v = row < nc ? (double)(1 << l) / dp->side * (double)m2l[b * nc + row] : 0.0;
  if (dst32) dst32[e] = (float)v;
  if (dst64) dst64[e] = v;
}

}  // namespace

hipError_t launch_m2m(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  const int ms = mstride(P->p);
  double* m64 = wsp<double>(P, lay.mult64);
  float* m32 = P->mixed ? wsp<float>(P, lay.mult32) : nullptr;
  for (int l = P->L - 1; l >= 2; --l) {
    ShiftArgs a = {};
    a.l = l;
    // mixed: the leaf multipoles exist in FP32 only (the P2M pass sums them in
    // FP64 and rounds once); every level above is kept in FP64 as well
    const bool leaf32 = m32 && l == P->L - 1;
    a.mixed = leaf32 ? 1 : 0;
    a.nparent = (int64_t)1 << (3 * l);
    a.s2c_child = wsp<uint32_t>(P, lay.slot2coord) + lay.lvl_off[l + 1];
    a.ops = wsp<double>(P, lay.op_m2m);
    a.src = leaf32 ? static_cast<const void*>(m32 + lay.lvl_off[l + 1] * ms)
                   : static_cast<const void*>(m64 + lay.lvl_off[l + 1] * ms);
    a.dst64 = m64 + lay.lvl_off[l] * ms;
    a.dst32 = m32 ? m32 + lay.lvl_off[l] * ms : nullptr;
    a.dp = wsp<DevParams>(P, lay.params);
    hipError_t e = dispatch_p<ShiftRun>(P->p, a, 0, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_l2l(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  const int nc = P->nc, ms = mstride(P->p), L = P->L;
  double* l64 = wsp<double>(P, lay.loc_exp64);
  float* leaf32 = P->mixed ? wsp<float>(P, lay.leaf_loc32) : nullptr;
  const DevParams* dp = wsp<DevParams>(P, lay.params);
  {
    const int64_t nb = 64;  // level 2
    float* d32 = (L == 2 && P->mixed) ? leaf32 : nullptr;
    if (P->mixed)
      k_l2l_top<float><<<grid_for(nb * ms, kBlock), kBlock, 0, s>>>(
          nc, ms, 2, nb, dp, wsp<float>(P, lay.m2l_out) + lay.lvl_off[2] * nc,
          d32 ? nullptr : l64 + lay.lvl_off[2] * ms, d32);
    else
      k_l2l_top<double><<<grid_for(nb * ms, kBlock), kBlock, 0, s>>>(
          nc, ms, 2, nb, dp, wsp<double>(P, lay.m2l_out) + lay.lvl_off[2] * nc,
          l64 + lay.lvl_off[2] * ms, nullptr);
  }
  for (int l = 3; l <= L; ++l) {
    ShiftArgs a = {};
    a.l = l;
    a.mixed = P->mixed ? 1 : 0;
    a.leaf = l == L ? 1 : 0;
    a.nparent = (int64_t)1 << (3 * (l - 1));
    a.s2c_child = wsp<uint32_t>(P, lay.slot2coord) + lay.lvl_off[l];
    a.ops = wsp<double>(P, lay.op_l2l);
    a.src = l64 + lay.lvl_off[l - 1] * ms;
    a.dst64 = l64 + lay.lvl_off[l] * ms;
    a.dst32 = (l == L && P->mixed) ? leaf32 : nullptr;
    a.m2l = P->mixed ? (const void*)(wsp<float>(P, lay.m2l_out) + lay.lvl_off[l] * nc)
                     : (const void*)(wsp<double>(P, lay.m2l_out) + lay.lvl_off[l] * nc);
    a.dp = dp;
    hipError_t e = dispatch_p<ShiftRun>(P->p, a, 1, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

// Adaptive tree: the same kernels over the divided boxes of each level (the
// compact rows of a level are contiguous; children of the k-th divided box of
// level l are rows 8k .. 8k+7 of level l + 1).  Every multipole is read in
// FP64; every local is written in FP64.
hipError_t launch_m2m_adaptive(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  const int ms = mstride(P->p);
  double* m64 = wsp<double>(P, lay.mult64);
  float* m32 = P->mixed ? wsp<float>(P, lay.mult32) : nullptr;
  for (int l = P->Ld - 1; l >= 2; --l) {
    if (P->nsplit[l] == 0) continue;
    ShiftArgs a = {};
    a.l = l;
    a.mixed = 0;
    a.nparent = P->nsplit[l];
    a.s2c_child = wsp<uint32_t>(P, lay.a_coord) + P->ce_off[l + 1];
    a.parent_of = wsp<uint32_t>(P, lay.a_parent_of) + P->ce_off[l + 1];
    a.ops = wsp<double>(P, lay.op_m2m);
    a.src = m64 + P->ce_off[l + 1] * ms;
    a.dst64 = m64 + P->ce_off[l] * ms;
    a.dst32 = m32 ? m32 + P->ce_off[l] * ms : nullptr;
    a.dp = wsp<DevParams>(P, lay.params);
    hipError_t e = dispatch_p<ShiftRun>(P->p, a, 0, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t launch_l2l_adaptive(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  const int nc = P->nc, ms = mstride(P->p);
  double* l64 = wsp<double>(P, lay.loc_exp64);
  const DevParams* dp = wsp<DevParams>(P, lay.params);
  const int64_t nb2 = P->ce_off[3] - P->ce_off[2];
  if (nb2 > 0) {
    if (P->mixed)
      k_l2l_top<float><<<grid_for(nb2 * ms, kBlock), kBlock, 0, s>>>(
          nc, ms, 2, nb2, dp, wsp<float>(P, lay.m2l_out) + P->ce_off[2] * nc,
          l64 + P->ce_off[2] * ms, wsp<float>(P, lay.leaf_loc32) + P->ce_off[2] * ms);
    else
      k_l2l_top<double><<<grid_for(nb2 * ms, kBlock), kBlock, 0, s>>>(
          nc, ms, 2, nb2, dp, wsp<double>(P, lay.m2l_out) + P->ce_off[2] * nc,
          l64 + P->ce_off[2] * ms, nullptr);
  }
  for (int l = 3; l <= P->Ld; ++l) {
    if (P->nsplit[l - 1] == 0) continue;
    ShiftArgs a = {};
    a.l = l;
    a.mixed = P->mixed ? 1 : 0;
    a.leaf = 0;
    a.nparent = P->nsplit[l - 1];
    a.s2c_child = wsp<uint32_t>(P, lay.a_coord) + P->ce_off[l];
    a.parent_of = wsp<uint32_t>(P, lay.a_parent_of) + P->ce_off[l];
    a.ops = wsp<double>(P, lay.op_l2l);
    a.src = l64 + P->ce_off[l - 1] * ms;
    a.dst64 = l64 + P->ce_off[l] * ms;
    a.dst32 = P->mixed ? wsp<float>(P, lay.leaf_loc32) + P->ce_off[l] * ms : nullptr;
    a.m2l = P->mixed ? (const void*)(wsp<float>(P, lay.m2l_out) + P->ce_off[l] * nc)
                     : (const void*)(wsp<double>(P, lay.m2l_out) + P->ce_off[l] * nc);
    a.dp = dp;
    hipError_t e = dispatch_p<ShiftRun>(P->p, a, 1, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace fmm
