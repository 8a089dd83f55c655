// operators.hip -- translation operators as dense real matrices.
//
// Expansions are kept in box-scaled form: at level l with box side h,
//   multipole  M~_n^m = sum_j q_j conj(R_n^m((y_j - c)/h))
//   local      phi(c + u) = sum L~_k^l R_k^l(u/h)
// with the regular / irregular solid harmonics
//   R_n^m = r^n P_n^m(cos t) e^{imf} / (n+m)!,   I_n^m = (n-m)! P_n^m(cos t) e^{imf} / r^{n+1}
// (Epton & Dembart, SIAM J. Sci. Comput. 16:865 (1995)), whose addition
// theorems give, after the scaling, translations that do not depend on the
// level:
//   M2M  M~p_n^m = sum_{k<=n,l} 2^{-k} M~c_k^l conj(R_{n-k}^{m-l}(w))
//   L2L  L~c_j^i = sum_{k>=j,l} 2^{-j} L~p_k^l R_{k-j}^{l-i}(w)
//   M2L  L~t_k^l = (1/h) (-1)^{k+l} sum_{n,m} M~s_n^m I_{n+k}^{m-l}(o)
// where w = (c_child - c_parent)/h_parent = (+-1/4, +-1/4, +-1/4) and o is the
// integer offset (c_t - c_s)/h.  Summing over m = -n..n with the real-charge
// symmetry c^{-m} = (-1)^m conj(c^m) turns each translation into a real matrix
// acting on the packed real coefficient vector (fmm_internal.h).  The 1/h of
// M2L is applied when its result is promoted (L2L pass).
//
// Tables, zero padded: M2M and L2L, 8 octants each, FP64, stored
// [octant][input k (padded to KP)][output row (padded to RP)]; M2L, 316
// offsets in the M2L precision, stored [offset][output row (padded to RP)]
// [input k (stride m2l_kstride_of)].
#include "bf16_split.h"

namespace fmm {
namespace {

struct Cd {
  double re, im;
};

// Entry of a real matrix from the two complex coefficients X1 (order m - l
// partner) and X2 (the partner of the negative input order), given the packed
// positions of input and output.
__host__ __device__ inline double real_entry(int in_m, bool in_im, bool out_im, Cd X1, Cd X2) {
  if (in_m == 0) return out_im ? X1.im : X1.re;
  const double sg = (in_m & 1) ? -1.0 : 1.0;
  if (!in_im) {
    const Cd c = {X1.re + sg * X2.re, X1.im + sg * X2.im};
    return out_im ? c.im : c.re;
  }
  const Cd d = {X1.re - sg * X2.re, X1.im - sg * X2.im};
  return out_im ? d.re : -d.im;  // coefficient of i * b
}

__host__ __device__ inline void unpack_index(int c, int& n, int& m, bool& is_im) {
  n = 0;
  while ((n + 1) * (n + 1) <= c) ++n;
  const int r = c - n * n;
  m = (r + 1) / 2;
  is_im = (r != 0) && ((r & 1) == 0);
}

// Harmonic table entry of order mm (any sign) from the m >= 0 table.
__host__ __device__ inline Cd harm(const double* re, const double* im, int nmax, int n, int mm) {
  if (n < 0 || n > nmax || mm > n || -mm > n) return {0.0, 0.0};
  if (mm >= 0) return {re[tri(n, mm)], im[tri(n, mm)]};
  const double sg = ((-mm) & 1) ? -1.0 : 1.0;
  return {sg * re[tri(n, -mm)], -sg * im[tri(n, -mm)]};
}

// Regular harmonics in FP64, table of m >= 0 (runtime degree).
__host__ __device__ void regular_table(double x, double y, double z, int p, double* re, double* im) {
  const double r2 = x * x + y * y + z * z;
  re[0] = 1.0;
  im[0] = 0.0;
  for (int m = 0; m <= p; ++m) {
    if (m > 0) {
      const double pr = re[tri(m - 1, m - 1)], pi = im[tri(m - 1, m - 1)];
      re[tri(m, m)] = -(x * pr - y * pi) / (2.0 * m);
      im[tri(m, m)] = -(x * pi + y * pr) / (2.0 * m);
    }
    if (m + 1 <= p) {
      re[tri(m + 1, m)] = z * re[tri(m, m)];
      im[tri(m + 1, m)] = z * im[tri(m, m)];
    }
    for (int n = m + 2; n <= p; ++n) {
      const double d = (double)(n - m) * (double)(n + m);
      re[tri(n, m)] = ((2.0 * n - 1.0) * z * re[tri(n - 1, m)] - r2 * re[tri(n - 2, m)]) / d;
      im[tri(n, m)] = ((2.0 * n - 1.0) * z * im[tri(n - 1, m)] - r2 * im[tri(n - 2, m)]) / d;
    }
  }
}

// Irregular harmonics I_n^m, m >= 0, n <= p:
//   I_0^0 = 1/r,  I_m^m = -(2m-1)(x + i y)/r^2 I_{m-1}^{m-1},
//   I_{m+1}^m = (2m+1) z / r^2 I_m^m,
//   r^2 I_n^m = (2n-1) z I_{n-1}^m - (n+m-1)(n-m-1) I_{n-2}^m.
__host__ __device__ void irregular_table(double x, double y, double z, int p, double* re, double* im) {
  const double r2 = x * x + y * y + z * z;
  re[0] = 1.0 / sqrt(r2);
  im[0] = 0.0;
  for (int m = 0; m <= p; ++m) {
    if (m > 0) {
      const double pr = re[tri(m - 1, m - 1)], pi = im[tri(m - 1, m - 1)];
      const double f = -(2.0 * m - 1.0) / r2;
      re[tri(m, m)] = f * (x * pr - y * pi);
      im[tri(m, m)] = f * (x * pi + y * pr);
    }
    if (m + 1 <= p) {
      const double f = (2.0 * m + 1.0) * z / r2;
      re[tri(m + 1, m)] = f * re[tri(m, m)];
      im[tri(m + 1, m)] = f * im[tri(m, m)];
    }
    for (int n = m + 2; n <= p; ++n) {
      const double c1 = (2.0 * n - 1.0) * z, c2 = (double)(n + m - 1) * (double)(n - m - 1);
      re[tri(n, m)] = (c1 * re[tri(n - 1, m)] - c2 * re[tri(n - 2, m)]) / r2;
      im[tri(n, m)] = (c1 * im[tri(n - 1, m)] - c2 * im[tri(n - 2, m)]) / r2;
    }
  }
}

constexpr int kTabMax = (2 * FMM_P_MAX + 1) * (2 * FMM_P_MAX + 2) / 2;

// Column m (all degrees n = m..p) of the irregular table, by the same
// recurrences, with the diagonal entry in closed form
// I_m^m = (-1)^m (2m-1)!! (x + i y)^m / r^{2m+1}; one thread per order m.
__host__ __device__ void irregular_column(double x, double y, double z, int p, int m, double* re,
                                 double* im) {
  const double r2 = x * x + y * y + z * z;
  double dr = 1.0 / sqrt(r2), di = 0.0;  // I_0^0
  for (int k = 1; k <= m; ++k) {
    const double f = -(2.0 * k - 1.0) / r2;
    const double nr = f * (x * dr - y * di), ni = f * (x * di + y * dr);
    dr = nr;
    di = ni;
  }
  re[tri(m, m)] = dr;
  im[tri(m, m)] = di;
  if (m + 1 <= p) {
    const double f = (2.0 * m + 1.0) * z / r2;
    re[tri(m + 1, m)] = f * dr;
    im[tri(m + 1, m)] = f * di;
  }
  for (int n = m + 2; n <= p; ++n) {
    const double c1 = (2.0 * n - 1.0) * z, c2 = (double)(n + m - 1) * (double)(n - m - 1);
    re[tri(n, m)] = (c1 * re[tri(n - 1, m)] - c2 * re[tri(n - 2, m)]) / r2;
    im[tri(n, m)] = (c1 * im[tri(n - 1, m)] - c2 * im[tri(n - 2, m)]) / r2;
  }
}

__host__ __device__ inline void octant_vector(int oct, double w[3]) {
  w[0] = (oct & 4) ? 0.25 : -0.25;
  w[1] = (oct & 2) ? 0.25 : -0.25;
  w[2] = (oct & 1) ? 0.25 : -0.25;
}

// Entry (row, col) of the M2M (is_l2l false) or L2L matrix of one octant,
// from that octant's regular-harmonic table of w.
__host__ __device__ inline double shift_entry(int p, bool is_l2l, int row, int col, const double* tre,
                                              const double* tim) {
  int n, m, k, l;
  bool oim, iim;
  unpack_index(row, n, m, oim);
  unpack_index(col, k, l, iim);
  if (!is_l2l) {
    // output (n, m): multipole of the parent; input (k, l): multipole of the child
    if (k > n) return 0.0;
    Cd x1 = harm(tre, tim, p, n - k, m - l), x2 = harm(tre, tim, p, n - k, m + l);
    x1.im = -x1.im;  // conjugates
    x2.im = -x2.im;
    return ldexp(real_entry(l, iim, oim, x1, x2), -k);
  }
  // output (n, m) = (j, i): local of the child; input (k, l): local of the parent
  if (k < n) return 0.0;
  const Cd x1 = harm(tre, tim, p, k - n, l - m), x2 = harm(tre, tim, p, k - n, -l - m);
  return ldexp(real_entry(l, iim, oim, x1, x2), -n);
}

// Entry (row, col) of the unit-box M2L matrix from the irregular-harmonic
// table (degrees <= 2p) of the offset (c_t - c_s)/h.
__host__ __device__ inline double m2l_entry(int p, int row, int col, const double* tre,
                                            const double* tim) {
  int kd, l, n, m;
  bool oim, iim;
  unpack_index(row, kd, l, oim);
  unpack_index(col, n, m, iim);
  Cd x1 = harm(tre, tim, 2 * p, n + kd, m - l), x2 = harm(tre, tim, 2 * p, n + kd, -m - l);
  if ((kd + l) & 1) {
    x1.re = -x1.re, x1.im = -x1.im;
    x2.re = -x2.re, x2.im = -x2.im;
  }
  return real_entry(m, iim, oim, x1, x2);
}

// M2M and L2L tables: blocks 8 s + b (s < kShiftSplit) build rows of the
// M2M of octant b, blocks 8 (kShiftSplit + s) + b those of the L2L, stored
// [octant][row (padded to rp)][k (padded to kp)], zero padded.
constexpr int kShiftSplit = 8;
__global__ void k_gen_shift(int p, int kp, int rp, double* __restrict__ m2m,
                            double* __restrict__ l2l) {
  __shared__ double tre[kTabMax], tim[kTabMax];
  const int oct = blockIdx.x & 7;
  const bool is_l2l = (int)(blockIdx.x >> 3) >= kShiftSplit;
  const int part = (blockIdx.x >> 3) % kShiftSplit;
  if (threadIdx.x == 0) {
    double w[3];
    octant_vector(oct, w);
    regular_table(w[0], w[1], w[2], p, tre, tim);
  }
  __syncthreads();
  const int nc = (p + 1) * (p + 1);
  double* out = (is_l2l ? l2l : m2m) + (size_t)oct * kp * rp;
  const int rows = (rp + kShiftSplit - 1) / kShiftSplit, r0 = part * rows;
  const int r1 = r0 + rows < rp ? r0 + rows : rp;
  for (int e = r0 * kp + threadIdx.x; e < r1 * kp; e += blockDim.x) {  // [row][k]
    const int row = e / kp, col = e % kp;
    out[e] = (col < nc && row < nc) ? shift_entry(p, is_l2l, row, col, tre, tim) : 0.0;
  }
}

template <typename T>
__global__ void k_gen_m2l(int p, int rp, int ks, T* __restrict__ ops) {
  __shared__ double tre[kTabMax], tim[kTabMax];
  const int op = blockIdx.x;
  if ((int)threadIdx.x <= 2 * p) {
    int o[3];
    m2l_offset(op, o);
    // o is the target-minus-source offset (c_t - c_s)/h
    irregular_column((double)o[0], (double)o[1], (double)o[2], 2 * p, threadIdx.x, tre, tim);
  }
  __syncthreads();
  const int nc = (p + 1) * (p + 1);
  T* out = ops + (size_t)op * rp * ks;
  for (int e = threadIdx.x; e < rp * ks; e += blockDim.x) {
    const int row = e / ks, col = e % ks;
    const double v = (col < nc && row < nc) ? m2l_entry(p, row, col, tre, tim) : 0.0;
    out[e] = (T)v;
  }
}

// Operators in pieces, in the chunked LDS layout of the split-BF16 M2L: one
// thread per (operator row, k step, lane group) computes its 8 FP64 entries
// and writes their NP quads.  Pad quads are zeroed beforehand.
template <int NP>
__global__ void k_gen_m2l_bf(int p, bool ad, u32x4* __restrict__ ops) {
  __shared__ double tre[kTabMax], tim[kTabMax];
  const int op = blockIdx.x;
  if ((int)threadIdx.x <= 2 * p) {
    int o[3];
    m2l_offset(op, o);
    // o is the target-minus-source offset (c_t - c_s)/h
    irregular_column((double)o[0], (double)o[1], (double)o[2], 2 * p, threadIdx.x, tre, tim);
  }
  __syncthreads();
  const int nc = (p + 1) * (p + 1);
  const int kst = m2lb_ksteps(nc), rp = m2lb_rows(nc), kc = m2lb_kc(nc, NP, ad);
  const int gq = m2lb_gq(kc, NP), qcs = m2lb_qcs(kc, NP);
  u32x4* out = ops + (size_t)op * m2lb_op_quads(nc, NP, ad);
  for (int e = threadIdx.x; e < rp * kst * 4; e += blockDim.x) {
    const int row = e / (kst * 4), ks = e / 4 % kst, g = e % 4;
    uint32_t pc[8][NP];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 32 * ks + 8 * g + j;
      split_f64<NP>((k < nc && row < nc) ? m2l_entry(p, row, k, tre, tim) : 0.0, pc[j]);
    }
    u32x4 q[NP];
    pack_quads<NP>(pc, q);
    u32x4* o = out + ((size_t)(ks / kc) * rp + row) * qcs + g * gq + (ks % kc) * NP;
#pragma unroll
    for (int i = 0; i < NP; ++i) o[i] = q[i];
  }
}

// ---- FP16 split M2L operators (FMM_M2L_F16X2) --------------------------
// The entries span many decades (|I_j^m(d)| grows like (j - m)! / |d|^(j+1)),
// more than FP16 holds, so each row r and column k gets a power-of-two scale,
// shared by all 316 operators: T'[r][k] = T[r][k] 2^(ra_r + cb_k), rows
// normalised first (max over k and operators -> 1), then columns, then all
// rows shifted so that the largest entry is just below 2^14.  The column
// scale is applied to the multipoles (times 2^-cb_k) and the row scale undone
// on the M2L results (times 2^-ra_r); both are exact.

// Pass 1: FP64 entries of every operator into scratch [op][row][k] (rows
// padded to 16, k to 32, zero outside); kGenSplit blocks per operator, each
// a range of rows.
constexpr int kGenSplit = 4;
__global__ void k_gen_m2l_f64(int p, double* __restrict__ scratch) {
  __shared__ double tre[kTabMax], tim[kTabMax];
  const int op = blockIdx.x / kGenSplit, part = blockIdx.x % kGenSplit;
  if ((int)threadIdx.x <= 2 * p) {
    int o[3];
    m2l_offset(op, o);
    irregular_column((double)o[0], (double)o[1], (double)o[2], 2 * p, threadIdx.x, tre, tim);
  }
  __syncthreads();
  const int nc = (p + 1) * (p + 1);
  const int rp = m2lb_rows(nc), kp = 32 * m2lb_ksteps(nc);
  double* out = scratch + (size_t)op * rp * kp;
  const int rows = (rp + kGenSplit - 1) / kGenSplit, r0 = part * rows;
  const int r1 = r0 + rows < rp ? r0 + rows : rp;
  for (int e = r0 * kp + threadIdx.x; e < r1 * kp; e += blockDim.x) {
    const int row = e / kp, k = e % kp;
    out[e] = (row < nc && k < nc) ? m2l_entry(p, row, k, tre, tim) : 0.0;
  }
}

// Pass 2: tbl[row][k] = max over operators of |entry| (FP32).
__global__ void k_f16_table(int rpkp, const double* __restrict__ scratch, float* __restrict__ tbl) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rpkp) return;
  double m = 0.0;
  for (int op = 0; op < kNumM2LOps; ++op) m = fmax(m, fabs(scratch[(size_t)op * rpkp + e]));
  tbl[e] = (float)m;
}

// Pass 3 (one work-group): the row and column exponents, as inverse factors
// rowf_r = 2^-ra_r and colf_k = 2^-cb_k.
__global__ void k_f16_fit(int rp, int kp, const float* __restrict__ tbl, float* __restrict__ rowf,
                          float* __restrict__ colf) {
  __shared__ int ra[256];
  for (int r = threadIdx.x; r < rp; r += blockDim.x) {
    float m = 0.f;
    for (int k = 0; k < kp; ++k) m = fmaxf(m, tbl[r * kp + k]);
    int e = 0;
    if (m > 0.f) frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
    ra[r] = -e;                  // max of the row times 2^ra in [0.5, 1)
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kp; k += blockDim.x) {
    float m = 0.f;
    for (int r = 0; r < rp; ++r) m = fmaxf(m, ldexpf(tbl[r * kp + k], ra[r]));
    int e = 0;
    if (m > 0.f) frexpf(m, &e);
    colf[k] = ldexpf(1.f, e);  // cb_k = -e
  }
  __syncthreads();
  // every scaled entry is now below 1: shift all rows by 2^14
  for (int r = threadIdx.x; r < rp; r += blockDim.x) rowf[r] = ldexpf(1.f, -(ra[r] + 14));
}

// Pass 4: scaled entries split into 2 FP16 pieces, in the split-M2L operator
// layout (m2lb_* with np = 2) or the wide form's (m2lw_*); one thread per
// (op, row, k step, lane group).
// The wide form's operator layout for one p (row blocks of 32), from the
// m2lw_* rules on the host.
struct WideOps {
  int base[4], len[4], cross[4], quads;
};
inline WideOps wide_ops(int nc) {
  WideOps w{};
  for (int rb = 0; rb < 4; ++rb) {
    w.base[rb] = m2lw_block_base(nc, rb < (nc + 31) / 32 ? rb : 0);
    w.len[rb] = m2lw_row_len(nc, rb);
    w.cross[rb] = m2lw_cross_steps(nc, rb);
  }
  w.quads = m2lw_op_quads(nc);
  return w;
}

__global__ void k_f16_split_ops(int p, bool ad, bool wide, WideOps wl, int64_t nitems, const double* __restrict__ scratch,
                                const float* __restrict__ rowf, const float* __restrict__ colf,
                                u32x4* __restrict__ ops) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nitems) return;
  const int nc = (p + 1) * (p + 1);
  const int kst = m2lb_ksteps(nc), rp = m2lb_rows(nc), kp = 32 * kst, kc = m2lb_kc(nc, 2, ad);
  const int gq = m2lb_gq(kc, 2), qcs = m2lb_qcs(kc, 2);
  const int g = (int)(t % 4), ks = (int)(t / 4 % kst), row = (int)(t / (4 * kst) % rp);
  const int op = (int)(t / (4 * kst * rp));
  if (wide && row >= nc) return;  // the wide form stores the ncoef real rows only
  // wide form: this thread's 8 k values are half h of 16-wide step sw; its
  // row block's products may need the leading piece only, or none
  const int sw = 2 * ks + g / 2, hw = g % 2, rbw = row / 32;
  if (wide && !m2lw_half_live(nc, sw, hw)) return;
  const double* src = scratch + ((size_t)op * rp + row) * kp;
  const double rs = 1.0 / (double)rowf[row];
  uint32_t pc[8][2];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 32 * ks + 8 * g + j;
    split_f16_f64(src[k] * rs / (double)colf[k], pc[j]);
  }
  u32x4 q[2];
  pack_quads<2>(pc, q);
  if (wide) {
    // m2lw_pos with the row block's values from the host
    const int cs = wl.cross[rbw];
    u32x4* o = ops + (size_t)op * wl.quads + wl.base[rbw] + (row - 32 * rbw) * wl.len[rbw];
    if (sw < cs) {
      o[4 * sw + 2 * hw] = q[0];
      o[4 * sw + 2 * hw + 1] = q[1];
    } else {
      o[4 * cs + 2 * (sw - cs) + hw] = q[0];
    }
    return;
  }
  u32x4* o = ops + (size_t)op * m2lb_op_quads(nc, 2, ad) + ((size_t)(ks / kc) * rp + row) * qcs + g * gq +
             (ks % kc) * 2;
  o[0] = q[0];
  o[1] = q[1];
}

}  // namespace

hipError_t launch_operators(fmm_plan_s* P, hipStream_t s) {
  const Layout& lay = P->lay;
  prof_begin(P, FMM_PHASE_OPERATORS, s);
  const int kp = shift_kpad(P->nc), rp = m2l_rows_pad(P->p);
  k_gen_shift<<<16 * kShiftSplit, kBlock, 0, s>>>(P->p, kp, rp, wsp<double>(P, lay.op_m2m),
                                    wsp<double>(P, lay.op_l2l));
  if (P->m2l_f16) {
    const int nc = P->nc, rpp = m2lb_rows(nc), kp = 32 * m2lb_ksteps(nc);
    const int64_t words = (int64_t)kNumM2LOps * m2lb_op_quads(nc, 2, P->adaptive) * 4;
    hipError_t e = fill_u32(wsp<uint32_t>(P, lay.op_m2lb), words, 0u, s);  // pad quads
    if (e != hipSuccess) return e;
    double* scratch = wsp<double>(P, lay.op_m2l_scratch);
    float* tbl = wsp<float>(P, lay.f16_tbl);
    float* rowf = wsp<float>(P, lay.f16_rowf);
    float* colf = wsp<float>(P, lay.f16_colf);
    k_gen_m2l_f64<<<kNumM2LOps * kGenSplit, kBlock, 0, s>>>(P->p, scratch);
    k_f16_table<<<grid_for(rpp * kp, kBlock), kBlock, 0, s>>>(rpp * kp, scratch, tbl);
    k_f16_fit<<<1, kBlock, 0, s>>>(rpp, kp, tbl, rowf, colf);
    const int64_t items = (int64_t)kNumM2LOps * rpp * m2lb_ksteps(nc) * 4;
    k_f16_split_ops<<<grid_for(items, kBlock), kBlock, 0, s>>>(P->p, P->adaptive, m2l_f16_wide(P->p),
                                                               wide_ops(nc), items, scratch, rowf,
                                                               colf, wsp<u32x4>(P, lay.op_m2lb));
  } else if (P->m2l_np) {
    const int np = P->m2l_np;
    const int64_t words = (int64_t)kNumM2LOps * m2lb_op_quads(P->nc, np, P->adaptive) * 4;
    hipError_t e = fill_u32(wsp<uint32_t>(P, lay.op_m2lb), words, 0u, s);  // pad quads
    if (e != hipSuccess) return e;
    u32x4* ob = wsp<u32x4>(P, lay.op_m2lb);
    if (np == 2)
      k_gen_m2l_bf<2><<<kNumM2LOps, kBlock, 0, s>>>(P->p, P->adaptive, ob);
    else
      k_gen_m2l_bf<3><<<kNumM2LOps, kBlock, 0, s>>>(P->p, P->adaptive, ob);
  } else if (P->mixed)
    k_gen_m2l<float><<<kNumM2LOps, kBlock, 0, s>>>(P->p, rp, m2l_kstride_of(P->nc, 4),
                                                   wsp<float>(P, lay.op_m2l32));
  else
    k_gen_m2l<double><<<kNumM2LOps, kBlock, 0, s>>>(P->p, rp, m2l_kstride_of(P->nc, 8),
                                                    wsp<double>(P, lay.op_m2l64));
  prof_end(P, s);
  return hipGetLastError();
}

}  // namespace fmm
