/*
 * fmm_oracle.c -- CPU reference ("oracle") for the 3-D Laplace fast multipole
 * method.  TEST INFRASTRUCTURE ONLY: this file is compiled into liboracle.so,
 * which only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load.  The GPU library never links, includes or calls it, and it
 * shares no code, header, table or generator with the GPU library.
 *
 * What is computed
 * ----------------
 *   Exact sum (the quantity the method approximates):
 *       phi_i = sum_{j != i} q_j / |x_i - x_j|,    F_i = -q_i grad phi_i,
 *       E     = 1/2 sum_i q_i phi_i.
 *   Open boundary, pure 1/r kernel (no Coulomb constant), no softening.
 *
 *   FMM result: a uniform octree of depth L over a cube (root = level 0,
 *   leaves = level L), well-separatedness 1 (near list = the 27 boxes at
 *   Chebyshev index distance <= 1, interaction list = children of the parent's
 *   near list that are not in the box's own near list), multipole and local
 *   expansions of degree <= p about box centres, every (local degree <= p,
 *   multipole degree <= p) pair kept in the multipole-to-local translation.
 *   Steps in the method's order (Greengard, "The Rapid Evaluation of Potential
 *   Fields in Particle Systems", MIT Press 1988, ch. 3; Cheng, Greengard &
 *   Rokhlin, J. Comput. Phys. 155:468 (1999), sec. 2-3):
 *       P2M -> M2M (leaf level up to level 2) -> M2L (levels 2..L)
 *       -> L2L (level 2 down to the leaves) -> L2P, plus the P2P near sum.
 *
 * Basis
 * -----
 *   Complex solid harmonics with the Epton-Dembart normalisation
 *   (SIAM J. Sci. Comput. 16:865 (1995)):
 *       R_n^m(x) = r^n P_n^m(cos t) e^{i m f} / (n+m)!       (regular)
 *       I_n^m(x) = (n-m)! P_n^m(cos t) e^{i m f} / r^{n+1}    (irregular)
 *   with the Condon-Shortley phase in P_n^m and, for negative orders,
 *   R_n^{-m} = (-1)^m conj(R_n^m), I_n^{-m} = (-1)^m conj(I_n^m).
 *   All orders -n..n are stored and summed (no real-charge symmetry is used),
 *   so each sum below is the textbook formula written out.
 *   Addition theorems used:
 *     (A1) 1/|x-y|      = sum_{n,m} conj(R_n^m(y)) I_n^m(x),           |y|<|x|
 *     (A2) R_n^m(x+y)   = sum_{k<=n,l} R_k^l(x) R_{n-k}^{m-l}(y)
 *     (A3) I_n^m(x-y)   = sum_{k,l} conj(R_k^l(y)) I_{n+k}^{m+l}(x),    |y|<|x|
 *     (A4) d/dz R_n^m = R_{n-1}^m,  d/dx R_n^m = (R_{n-1}^{m+1} - R_{n-1}^{m-1})/2,
 *          d/dy R_n^m = -i (R_{n-1}^{m-1} + R_{n-1}^{m+1})/2
 *   giving the operators
 *     P2M  M_n^m  = sum_j q_j conj(R_n^m(y_j - c))
 *     M2P  phi(x) = sum M_n^m I_n^m(x - c)
 *     M2M  M'_n^m = sum_{k,l} M_k^l conj(R_{n-k}^{m-l}(c - c'))          (A2)
 *     M2L  L_k^l  = (-1)^{k+l} sum_{n,m} M_n^m I_{n+k}^{m-l}(c_t - c_s)   (A3)
 *     L2L  L'_j^i = sum_{k>=j,l} L_k^l R_{k-j}^{l-i}(c' - c)              (A2)
 *     L2P  phi(x) = Re sum L_k^l R_k^l(x - c), gradient by (A4).
 *
 * Tree conventions (readings where the problem statement is silent)
 * -----------------------------------------------------------------
 *   cube: [lo, lo+side]^3 as given; if side <= 0 it is derived as
 *         lo_a = min_i x_ia, side = max_a (max_i x_ia - lo_a) (1 if that is 0).
 *   leaf cell per axis: floor(((x - lo)/side) * 2^L), clamped to [0, 2^L - 1]
 *         (a point on an internal face belongs to the upper cell; the top face
 *         is clamped into the last cell).  A given cube that does not contain
 *         a point is an error (ORACLE_E_OUT_OF_CUBE).
 *   particles are ordered by lexicographic leaf index (ix, iy, iz), stable.
 *   box centre at level l: lo + (i + 1/2) side / 2^l.
 *
 * Parity status: every function here is pinned by tests that do not re-use
 * its formulas (brute-force truncated Taylor kernel, Legendre closed forms,
 * direct-sum invariants, finite differences); none is "parity unpinned".
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum {
  ORACLE_OK = 0,
  ORACLE_E_INVALID_ARG = 1,
  ORACLE_E_OUT_OF_CUBE = 3,
  ORACLE_E_NONFINITE = 4,
  ORACLE_E_COINCIDENT = 5,
  ORACLE_E_NOMEM = 8
};

#define ORACLE_PMAX 20
#define ORACLE_LMAX 10

static inline int hidx(int n, int m) { return n * n + n + m; }
static inline int nharm(int p) { return (p + 1) * (p + 1); }

/* ------------------------------------------------------------------------ */
/* Solid harmonics by the three-term Legendre recurrences.                   */
/* ------------------------------------------------------------------------ */

/* R_n^m(x) for 0 <= n <= p, -n <= m <= n. */
static void regular_harmonics(double x, double y, double z, int p, cplx *R) {
  const double r2 = x * x + y * y + z * z;
  const cplx xy = x + I * y;
  R[hidx(0, 0)] = 1.0;
  for (int m = 0; m <= p; ++m) {
    if (m > 0) R[hidx(m, m)] = -xy / (2.0 * m) * R[hidx(m - 1, m - 1)];
    if (m + 1 <= p) R[hidx(m + 1, m)] = z * R[hidx(m, m)];
    for (int n = m + 2; n <= p; ++n)
      R[hidx(n, m)] = ((2.0 * n - 1.0) * z * R[hidx(n - 1, m)] - r2 * R[hidx(n - 2, m)]) /
                      ((double)(n - m) * (double)(n + m));
  }
  for (int n = 1; n <= p; ++n)
    for (int m = 1; m <= n; ++m)
      R[hidx(n, -m)] = ((m & 1) ? -1.0 : 1.0) * conj(R[hidx(n, m)]);
}

/* I_n^m(x) for 0 <= n <= p, -n <= m <= n; x != 0. */
static void irregular_harmonics(double x, double y, double z, int p, cplx *Ih) {
  const double r2 = x * x + y * y + z * z;
  const cplx xy = x + I * y;
  Ih[hidx(0, 0)] = 1.0 / sqrt(r2);
  for (int m = 0; m <= p; ++m) {
    if (m > 0) Ih[hidx(m, m)] = -(2.0 * m - 1.0) * xy / r2 * Ih[hidx(m - 1, m - 1)];
    if (m + 1 <= p) Ih[hidx(m + 1, m)] = (2.0 * m + 1.0) * z / r2 * Ih[hidx(m, m)];
    for (int n = m + 2; n <= p; ++n)
      Ih[hidx(n, m)] = ((2.0 * n - 1.0) * z * Ih[hidx(n - 1, m)] -
                        (double)(n + m - 1) * (double)(n - m - 1) * Ih[hidx(n - 2, m)]) / r2;
  }
  for (int n = 1; n <= p; ++n)
    for (int m = 1; m <= n; ++m)
      Ih[hidx(n, -m)] = ((m & 1) ? -1.0 : 1.0) * conj(Ih[hidx(n, m)]);
}

static inline cplx harm_get(const cplx *H, int pmax, int n, int m) {
  if (n < 0 || n > pmax || m < -n || m > n) return 0.0;
  return H[hidx(n, m)];
}

/* ------------------------------------------------------------------------ */
/* The six operators, one call = one translation (no batching or fusion).    */
/* ------------------------------------------------------------------------ */

/* P2M: M += q conj(R(y - c)). */
static void op_p2m(int p, const double y[3], double q, const double c[3], cplx *M) {
  cplx R[(ORACLE_PMAX + 1) * (ORACLE_PMAX + 1)];
  regular_harmonics(y[0] - c[0], y[1] - c[1], y[2] - c[2], p, R);
  for (int i = 0; i < nharm(p); ++i) M[i] += q * conj(R[i]);
}

/* M2M: multipole M about c -> added into Mp about cp. */
static void op_m2m(int p, const cplx *M, const double c[3], const double cp[3], cplx *Mp) {
  cplx R[(ORACLE_PMAX + 1) * (ORACLE_PMAX + 1)];
  regular_harmonics(c[0] - cp[0], c[1] - cp[1], c[2] - cp[2], p, R);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) {
      cplx acc = 0.0;
      for (int k = 0; k <= n; ++k)
        for (int l = -k; l <= k; ++l)
          acc += M[hidx(k, l)] * conj(harm_get(R, p, n - k, m - l));
      Mp[hidx(n, m)] += acc;
    }
}

/* M2L: multipole M about cs -> added into local L about ct. */
static void op_m2l(int p, const cplx *M, const double cs[3], const double ct[3], cplx *L) {
  cplx Ih[(2 * ORACLE_PMAX + 1) * (2 * ORACLE_PMAX + 1)];
  irregular_harmonics(ct[0] - cs[0], ct[1] - cs[1], ct[2] - cs[2], 2 * p, Ih);
  for (int k = 0; k <= p; ++k)
    for (int l = -k; l <= k; ++l) {
      cplx acc = 0.0;
      for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m)
          acc += M[hidx(n, m)] * harm_get(Ih, 2 * p, n + k, m - l);
      L[hidx(k, l)] += (((k + l) & 1) ? -1.0 : 1.0) * acc;
    }
}

/* L2L: local L about c -> added into local Lc about cc. */
static void op_l2l(int p, const cplx *L, const double c[3], const double cc[3], cplx *Lc) {
  cplx R[(ORACLE_PMAX + 1) * (ORACLE_PMAX + 1)];
  regular_harmonics(cc[0] - c[0], cc[1] - c[1], cc[2] - c[2], p, R);
  for (int j = 0; j <= p; ++j)
    for (int i = -j; i <= j; ++i) {
      cplx acc = 0.0;
      for (int k = j; k <= p; ++k)
        for (int l = -k; l <= k; ++l)
          acc += L[hidx(k, l)] * harm_get(R, p, k - j, l - i);
      Lc[hidx(j, i)] += acc;
    }
}

/* L2P: potential and gradient of the local expansion L about c at x. */
static void op_l2p(int p, const cplx *L, const double c[3], const double x[3], double *phi,
                   double grad[3]) {
  cplx R[(ORACLE_PMAX + 1) * (ORACLE_PMAX + 1)];
  regular_harmonics(x[0] - c[0], x[1] - c[1], x[2] - c[2], p, R);
  cplx f = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) {
      const cplx a = L[hidx(n, m)];
      f += a * R[hidx(n, m)];
      if (n == 0) continue;
      const cplx rm = harm_get(R, p, n - 1, m - 1), rp = harm_get(R, p, n - 1, m + 1);
      gz += a * harm_get(R, p, n - 1, m);
      gx += a * 0.5 * (rp - rm);
      gy += a * (-0.5 * I) * (rm + rp);
    }
  *phi = creal(f);
  grad[0] = creal(gx);
  grad[1] = creal(gy);
  grad[2] = creal(gz);
}

/* M2P: potential of the multipole M about c at x (used by the operator pins). */
static double op_m2p(int p, const cplx *M, const double c[3], const double x[3]) {
  cplx Ih[(ORACLE_PMAX + 1) * (ORACLE_PMAX + 1)];
  irregular_harmonics(x[0] - c[0], x[1] - c[1], x[2] - c[2], p, Ih);
  cplx f = 0.0;
  for (int i = 0; i < nharm(p); ++i) f += M[i] * Ih[i];
  return creal(f);
}

/* ------------------------------------------------------------------------ */
/* Neumaier-compensated accumulation.                                        */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } ksum;
static inline void ksum_add(ksum *k, double v) {
  const double t = k->s + v;
  if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
  else k->c += (v - t) + k->s;
  k->s = t;
}
static inline double ksum_val(const ksum *k) { return k->s + k->c; }

/* ------------------------------------------------------------------------ */
/* Direct sum.                                                               */
/* ------------------------------------------------------------------------ */

/* phi/force for the targets listed (all particles when targets == NULL);
 * energy (when non-NULL and targets == NULL) = 1/2 sum q_i phi_i. */
int oracle_direct(int64_t n, const double *pos, const double *q, int64_t nt,
                  const int64_t *targets, double *phi, double *force, double *energy) {
  if (n < 0 || !pos || !q) return ORACLE_E_INVALID_ARG;
  if (!targets) nt = n;
  double *phi_tmp = NULL;
  if (!phi && energy && !targets) {
    phi_tmp = malloc(sizeof(double) * (n ? n : 1));
    if (!phi_tmp) return ORACLE_E_NOMEM;
    phi = phi_tmp;
  }
  int status = ORACLE_OK;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t i = targets ? targets[t] : t;
    ksum f = {0, 0}, gx = {0, 0}, gy = {0, 0}, gz = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dx = pos[3 * i] - pos[3 * j], dy = pos[3 * i + 1] - pos[3 * j + 1],
                   dz = pos[3 * i + 2] - pos[3 * j + 2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 == 0.0) {
#pragma omp atomic write
        status = ORACLE_E_COINCIDENT;
        continue;
      }
      const double r = sqrt(r2);
      const double qr = q[j] / r, qr3 = qr / r2;
      ksum_add(&f, qr);
      /* grad phi_i = -sum_j q_j (x_i - x_j) / r^3 */
      ksum_add(&gx, -qr3 * dx);
      ksum_add(&gy, -qr3 * dy);
      ksum_add(&gz, -qr3 * dz);
    }
    if (phi) phi[t] = ksum_val(&f);
    if (force) {
      force[3 * t] = -q[i] * ksum_val(&gx);
      force[3 * t + 1] = -q[i] * ksum_val(&gy);
      force[3 * t + 2] = -q[i] * ksum_val(&gz);
    }
  }
  if (energy && !targets) {
    ksum e = {0, 0};
    for (int64_t i = 0; i < n; ++i) ksum_add(&e, q[i] * phi[i]);
    *energy = 0.5 * ksum_val(&e);
  }
  free(phi_tmp);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Tree.                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  int L, p, nh;
  double lo[3], side;
  int64_t n;
  int32_t *cell;    /* n x 3 leaf cell per particle (user order) */
  int64_t *order;   /* particles sorted by lexicographic leaf index */
  int64_t *start;   /* leaf start in order[], 8^L + 1 entries */
  int64_t lvl_off[ORACLE_LMAX + 2]; /* box offset of each level in the arrays below */
  cplx *M, *Lc;     /* expansions for every box of every level */
} otree;

static inline int64_t box_lin(int l, int ix, int iy, int iz) {
  const int64_t nb = (int64_t)1 << l;
  return ((int64_t)ix * nb + iy) * nb + iz;
}

static void box_centre(const otree *T, int l, int ix, int iy, int iz, double c[3]) {
  const double h = T->side / (double)((int64_t)1 << l);
  c[0] = T->lo[0] + (ix + 0.5) * h;
  c[1] = T->lo[1] + (iy + 0.5) * h;
  c[2] = T->lo[2] + (iz + 0.5) * h;
}

static int resolve_cube(int64_t n, const double *pos, const double lo_in[3], double side_in,
                        double lo[3], double *side) {
  for (int64_t i = 0; i < 3 * n; ++i)
    if (!isfinite(pos[i])) return ORACLE_E_NONFINITE;
  if (side_in > 0) {
    if (!lo_in) return ORACLE_E_INVALID_ARG;
    for (int a = 0; a < 3; ++a) lo[a] = lo_in[a];
    *side = side_in;
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < 3; ++a) {
        const double t = (pos[3 * i + a] - lo[a]) / side_in;
        if (!(t >= 0.0 && t <= 1.0)) return ORACLE_E_OUT_OF_CUBE;
      }
    return ORACLE_OK;
  }
  double hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = n ? pos[a] : 0.0;
    hi[a] = lo[a];
  }
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      if (pos[3 * i + a] < lo[a]) lo[a] = pos[3 * i + a];
      if (pos[3 * i + a] > hi[a]) hi[a] = pos[3 * i + a];
    }
  double s = 0.0;
  for (int a = 0; a < 3; ++a)
    if (hi[a] - lo[a] > s) s = hi[a] - lo[a];
  *side = (s > 0.0) ? s : 1.0;
  return ORACLE_OK;
}

static int leaf_cell_axis(double x, double lo, double side, int L) {
  const double t = (x - lo) / side;
  const int64_t nb = (int64_t)1 << L;
  double f = floor(t * (double)nb);
  int64_t c = (int64_t)f;
  if (c < 0) c = 0;
  if (c > nb - 1) c = nb - 1;
  return (int)c;
}

static void otree_free(otree *T) {
  free(T->cell);
  free(T->order);
  free(T->start);
  free(T->M);
  free(T->Lc);
}

static int otree_build(otree *T, int64_t n, const double *pos, int L, int p,
                       const double lo_in[3], double side_in) {
  memset(T, 0, sizeof(*T));
  T->L = L;
  T->p = p;
  T->nh = nharm(p);
  T->n = n;
  int st = resolve_cube(n, pos, lo_in, side_in, T->lo, &T->side);
  if (st) return st;
  const int64_t nleaf = (int64_t)1 << (3 * L);
  T->cell = malloc(sizeof(int32_t) * 3 * (n ? n : 1));
  T->order = malloc(sizeof(int64_t) * (n ? n : 1));
  T->start = calloc(nleaf + 1, sizeof(int64_t));
  if (!T->cell || !T->order || !T->start) return ORACLE_E_NOMEM;
  int64_t *leaf = malloc(sizeof(int64_t) * (n ? n : 1));
  if (!leaf) return ORACLE_E_NOMEM;
  for (int64_t i = 0; i < n; ++i) {
    int c[3];
    for (int a = 0; a < 3; ++a) {
      c[a] = leaf_cell_axis(pos[3 * i + a], T->lo[a], T->side, L);
      T->cell[3 * i + a] = c[a];
    }
    leaf[i] = box_lin(L, c[0], c[1], c[2]);
    T->start[leaf[i] + 1]++;
  }
  for (int64_t b = 0; b < nleaf; ++b) T->start[b + 1] += T->start[b];
  int64_t *fill = malloc(sizeof(int64_t) * nleaf);
  if (!fill) { free(leaf); return ORACLE_E_NOMEM; }
  memcpy(fill, T->start, sizeof(int64_t) * nleaf);
  for (int64_t i = 0; i < n; ++i) T->order[fill[leaf[i]]++] = i; /* stable */
  free(fill);
  free(leaf);
  int64_t off = 0;
  for (int l = 0; l <= L; ++l) {
    T->lvl_off[l] = off;
    off += (int64_t)1 << (3 * l);
  }
  T->lvl_off[L + 1] = off;
  T->M = calloc((size_t)off * T->nh, sizeof(cplx));
  T->Lc = calloc((size_t)off * T->nh, sizeof(cplx));
  if (!T->M || !T->Lc) return ORACLE_E_NOMEM;
  return ORACLE_OK;
}

static inline cplx *exp_at(const otree *T, cplx *base, int l, int64_t b) {
  return base + (size_t)(T->lvl_off[l] + b) * T->nh;
}

/* Upward pass: P2M at the leaves, then M2M from level L-1 up to level 2. */
static void upward_pass(otree *T, const double *pos, const double *q) {
  const int L = T->L, p = T->p;
  const int nb = 1 << L;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t b = 0; b < (int64_t)nb * nb * nb; ++b) {
    const int ix = (int)(b / ((int64_t)nb * nb)), iy = (int)((b / nb) % nb), iz = (int)(b % nb);
    double c[3];
    box_centre(T, L, ix, iy, iz, c);
    cplx *M = exp_at(T, T->M, L, b);
    for (int64_t k = T->start[b]; k < T->start[b + 1]; ++k) {
      const int64_t j = T->order[k];
      op_p2m(p, pos + 3 * j, q[j], c, M);
    }
  }
  for (int l = L - 1; l >= 2; --l) {
    const int nl = 1 << l;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < (int64_t)nl * nl * nl; ++b) {
      const int ix = (int)(b / ((int64_t)nl * nl)), iy = (int)((b / nl) % nl), iz = (int)(b % nl);
      double cp[3];
      box_centre(T, l, ix, iy, iz, cp);
      cplx *Mp = exp_at(T, T->M, l, b);
      for (int ch = 0; ch < 8; ++ch) {
        const int cx = 2 * ix + (ch >> 2), cy = 2 * iy + ((ch >> 1) & 1), cz = 2 * iz + (ch & 1);
        double cc[3];
        box_centre(T, l + 1, cx, cy, cz, cc);
        op_m2m(p, exp_at(T, T->M, l + 1, box_lin(l + 1, cx, cy, cz)), cc, cp, Mp);
      }
    }
  }
}

static inline int iabs_(int a) { return a < 0 ? -a : a; }

/* Interaction list of box (ix,iy,iz) at level l >= 2: children of the
 * parent's near boxes that are not adjacent to the box.  M2L of each of them
 * into the box's local expansion. */
static void m2l_box(otree *T, int l, int ix, int iy, int iz) {
  const int nl = 1 << l, p = T->p;
  double ct[3];
  box_centre(T, l, ix, iy, iz, ct);
  cplx *Lt = exp_at(T, T->Lc, l, box_lin(l, ix, iy, iz));
  const int px = ix >> 1, py = iy >> 1, pz = iz >> 1;
  for (int ax = px - 1; ax <= px + 1; ++ax)
    for (int ay = py - 1; ay <= py + 1; ++ay)
      for (int az = pz - 1; az <= pz + 1; ++az) {
        if (ax < 0 || ay < 0 || az < 0 || 2 * ax >= nl || 2 * ay >= nl || 2 * az >= nl) continue;
        for (int ch = 0; ch < 8; ++ch) {
          const int sx = 2 * ax + (ch >> 2), sy = 2 * ay + ((ch >> 1) & 1), sz = 2 * az + (ch & 1);
          if (iabs_(sx - ix) <= 1 && iabs_(sy - iy) <= 1 && iabs_(sz - iz) <= 1) continue;
          double cs[3];
          box_centre(T, l, sx, sy, sz, cs);
          op_m2l(p, exp_at(T, T->M, l, box_lin(l, sx, sy, sz)), cs, ct, Lt);
        }
      }
}

/* Near field at point x of leaf (cx,cy,cz) from the 27 neighbour leaves,
 * skipping particle `skip' (the target itself; -1 for none). */
static int p2p_point(const otree *T, const double *pos, const double *q, int cx, int cy, int cz,
                     const double x[3], int64_t skip, double *phi, double grad[3]) {
  const int L = T->L, nb = 1 << L;
  ksum f = {0, 0}, gx = {0, 0}, gy = {0, 0}, gz = {0, 0};
  int status = ORACLE_OK;
  for (int ax = cx - 1; ax <= cx + 1; ++ax)
    for (int ay = cy - 1; ay <= cy + 1; ++ay)
      for (int az = cz - 1; az <= cz + 1; ++az) {
        if (ax < 0 || ay < 0 || az < 0 || ax >= nb || ay >= nb || az >= nb) continue;
        const int64_t b = box_lin(L, ax, ay, az);
        for (int64_t k = T->start[b]; k < T->start[b + 1]; ++k) {
          const int64_t j = T->order[k];
          if (j == skip) continue;
          const double dx = x[0] - pos[3 * j], dy = x[1] - pos[3 * j + 1], dz = x[2] - pos[3 * j + 2];
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 == 0.0) {
            status = ORACLE_E_COINCIDENT;
            continue;
          }
          const double r = sqrt(r2), qr = q[j] / r, qr3 = qr / r2;
          ksum_add(&f, qr);
          ksum_add(&gx, -qr3 * dx);
          ksum_add(&gy, -qr3 * dy);
          ksum_add(&gz, -qr3 * dz);
        }
      }
  *phi = ksum_val(&f);
  grad[0] = ksum_val(&gx);
  grad[1] = ksum_val(&gy);
  grad[2] = ksum_val(&gz);
  return status;
}

/* Near field of particle i: the sum over its leaf's 27 neighbours, j != i. */
static int p2p_particle(const otree *T, const double *pos, const double *q, int64_t i,
                        double *phi, double grad[3]) {
  return p2p_point(T, pos, q, T->cell[3 * i], T->cell[3 * i + 1], T->cell[3 * i + 2], pos + 3 * i,
                   i, phi, grad);
}

/* Which boxes need a local expansion: the ancestors (levels 2..L) of the
 * leaves of the listed particles (all particles when list is NULL). */
static unsigned char *need_of(const otree *T, int64_t nt, const int64_t *list) {
  const int L = T->L;
  unsigned char *need = calloc(T->lvl_off[L + 1] ? T->lvl_off[L + 1] : 1, 1);
  if (!need) return NULL;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t i = list ? list[t] : t;
    for (int l = 2; l <= L; ++l) {
      const int s = L - l;
      need[T->lvl_off[l] + box_lin(l, T->cell[3 * i] >> s, T->cell[3 * i + 1] >> s,
                                   T->cell[3 * i + 2] >> s)] = 1;
    }
  }
  return need;
}

/* Upward pass, then M2L (levels 2..L) and L2L into every needed box. */
static void expansions(otree *T, const double *pos, const double *q, const unsigned char *need) {
  const int L = T->L, p = T->p;
  if (L < 2) return;
  upward_pass(T, pos, q);
  /* M2L, every level 2..L */
  for (int l = 2; l <= L; ++l) {
    const int nl = 1 << l;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t b = 0; b < (int64_t)nl * nl * nl; ++b) {
      if (!need[T->lvl_off[l] + b]) continue;
      m2l_box(T, l, (int)(b / ((int64_t)nl * nl)), (int)((b / nl) % nl), (int)(b % nl));
    }
  }
  /* L2L, level 2 down to L-1 into their children */
  for (int l = 2; l < L; ++l) {
    const int nl = 1 << (l + 1);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < (int64_t)nl * nl * nl; ++b) {
      if (!need[T->lvl_off[l + 1] + b]) continue;
      const int cx = (int)(b / ((int64_t)nl * nl)), cy = (int)((b / nl) % nl), cz = (int)(b % nl);
      double cp[3], cc[3];
      box_centre(T, l, cx >> 1, cy >> 1, cz >> 1, cp);
      box_centre(T, l + 1, cx, cy, cz, cc);
      op_l2l(p, exp_at(T, T->Lc, l, box_lin(l, cx >> 1, cy >> 1, cz >> 1)), cp, cc,
             exp_at(T, T->Lc, l + 1, b));
    }
  }
}

/* Full FMM (targets == NULL) or the FMM result at the listed targets only.
 * In the second form the upward pass is done in full and the downward pass
 * only along the ancestors of the targets' leaves; the values are the same as
 * the full run's. */
int oracle_fmm(int64_t n, const double *pos, const double *q, int depth, int p,
               const double lo[3], double side, int64_t nt, const int64_t *targets, double *phi,
               double *force, double *energy) {
  if (n < 0 || !pos || !q || depth < 0 || depth > ORACLE_LMAX || p < 0 || p > ORACLE_PMAX)
    return ORACLE_E_INVALID_ARG;
  if (!targets) nt = n;
  for (int64_t t = 0; t < nt; ++t)
    if (targets && (targets[t] < 0 || targets[t] >= n)) return ORACLE_E_INVALID_ARG;
  otree T;
  int st = otree_build(&T, n, pos, depth, p, lo, side);
  if (st) { otree_free(&T); return st; }
  const int L = depth;

  unsigned char *need = need_of(&T, nt, targets);
  if (!need) { otree_free(&T); return ORACLE_E_NOMEM; }
  expansions(&T, pos, q, need);

  int status = ORACLE_OK;
  double *phi_all = phi;
  double *phi_tmp = NULL;
  if (!phi) {
    phi_tmp = malloc(sizeof(double) * (nt ? nt : 1));
    phi_all = phi_tmp;
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t i = targets ? targets[t] : t;
    double fn, gn[3], ff = 0.0, gf[3] = {0.0, 0.0, 0.0};
    int s = p2p_particle(&T, pos, q, i, &fn, gn);
    if (s) {
#pragma omp atomic write
      status = s;
    }
    if (L >= 2) {
      double c[3];
      box_centre(&T, L, T.cell[3 * i], T.cell[3 * i + 1], T.cell[3 * i + 2], c);
      op_l2p(p, exp_at(&T, T.Lc, L, box_lin(L, T.cell[3 * i], T.cell[3 * i + 1], T.cell[3 * i + 2])),
             c, pos + 3 * i, &ff, gf);
    }
    phi_all[t] = fn + ff;
    if (force)
      for (int a = 0; a < 3; ++a) force[3 * t + a] = -q[i] * (gn[a] + gf[a]);
  }
  if (energy && !targets) {
    ksum e = {0, 0};
    for (int64_t i = 0; i < n; ++i) ksum_add(&e, q[i] * phi_all[i]);
    *energy = 0.5 * ksum_val(&e);
  }
  free(phi_tmp);
  free(need);
  otree_free(&T);
  return status;
}

/* Potential of the FMM at displaced target positions.  For probe k the
 * particle i = idx[k] is taken to sit at y_k (3 values), which must lie in the
 * same leaf as x_i: phi_k = sum over the 27 neighbour leaves of q_j / |y_k -
 * x_j| (j != i) plus the leaf's local expansion evaluated at y_k.  The tree,
 * every multipole and every local expansion are those of the unmoved system:
 * with every (local <= p, multipole <= p) pair kept, the FMM energy is the
 * symmetric form E = 1/2 sum_{j,k} q_j q_k K_jk, and the only entries that move
 * with x_i are K_ij = K_ji, so E(x_i -> y) - E(x_i -> y') = q_i (phi(y) -
 * phi(y')) exactly (central differences of the energy in x_i).
 * Errors: ORACLE_E_INVALID_ARG (an index out of range, or y_k outside x_i's
 * leaf). */
int oracle_fmm_probe(int64_t n, const double *pos, const double *q, int depth, int p,
                     const double lo[3], double side, int64_t m, const int64_t *idx,
                     const double *y, double *phi) {
  if (n < 0 || !pos || !q || !idx || !y || !phi || depth < 0 || depth > ORACLE_LMAX || p < 0 ||
      p > ORACLE_PMAX)
    return ORACLE_E_INVALID_ARG;
  for (int64_t k = 0; k < m; ++k)
    if (idx[k] < 0 || idx[k] >= n) return ORACLE_E_INVALID_ARG;
  otree T;
  int st = otree_build(&T, n, pos, depth, p, lo, side);
  if (st) { otree_free(&T); return st; }
  for (int64_t k = 0; k < m && st == ORACLE_OK; ++k)
    for (int a = 0; a < 3; ++a)
      if (leaf_cell_axis(y[3 * k + a], T.lo[a], T.side, depth) != T.cell[3 * idx[k] + a])
        st = ORACLE_E_INVALID_ARG;
  unsigned char *need = st ? NULL : need_of(&T, m, idx);
  if (!st && !need) st = ORACLE_E_NOMEM;
  if (st) { free(need); otree_free(&T); return st; }
  expansions(&T, pos, q, need);
  int status = ORACLE_OK;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t k = 0; k < m; ++k) {
    const int64_t i = idx[k];
    const int cx = T.cell[3 * i], cy = T.cell[3 * i + 1], cz = T.cell[3 * i + 2];
    double fn, gn[3], ff = 0.0, gf[3] = {0.0, 0.0, 0.0};
    int s = p2p_point(&T, pos, q, cx, cy, cz, y + 3 * k, i, &fn, gn);
    if (s) {
#pragma omp atomic write
      status = s;
    }
    if (depth >= 2) {
      double c[3];
      box_centre(&T, depth, cx, cy, cz, c);
      op_l2p(p, exp_at(&T, T.Lc, depth, box_lin(depth, cx, cy, cz)), c, y + 3 * k, &ff, gf);
    }
    phi[k] = fn + ff;
  }
  free(need);
  otree_free(&T);
  return status;
}

/* Leaf cell (ix, iy, iz) of every particle, and the resolved cube. */
int oracle_leaf_cells(int64_t n, const double *pos, int depth, const double lo_in[3],
                      double side_in, int32_t *cells, double lo_out[3], double *side_out) {
  if (n < 0 || !pos || depth < 0 || depth > ORACLE_LMAX) return ORACLE_E_INVALID_ARG;
  double lo[3], side;
  int st = resolve_cube(n, pos, lo_in, side_in, lo, &side);
  if (st) return st;
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) cells[3 * i + a] = leaf_cell_axis(pos[3 * i + a], lo[a], side, depth);
  if (lo_out)
    for (int a = 0; a < 3; ++a) lo_out[a] = lo[a];
  if (side_out) *side_out = side;
  return ORACLE_OK;
}

/* Operator chains for the single-operator pins.  Sources (ns points, charges
 * q) are expanded about c1, then:
 *   chain 0: M2P at x                          (P2M, M2P)
 *   chain 1: M2M to c2, M2P at x               (P2M, M2M, M2P)
 *   chain 2: M2L to c2, L2P at x               (P2M, M2L, L2P)
 *   chain 3: M2L to c2, L2L to c3, L2P at x    (P2M, M2L, L2L, L2P)
 * phi (nx) receives the potential, grad (nx x 3, may be NULL) the gradient
 * (chains 2 and 3 only). */
int oracle_chain(int chain, int p, int64_t ns, const double *src, const double *q,
                 const double c1[3], const double c2[3], const double c3[3], int64_t nx,
                 const double *x, double *phi, double *grad) {
  if (p < 0 || p > ORACLE_PMAX || chain < 0 || chain > 3) return ORACLE_E_INVALID_ARG;
  const int nh = nharm(p);
  cplx *A = calloc(nh, sizeof(cplx)), *B = calloc(nh, sizeof(cplx)), *C = calloc(nh, sizeof(cplx));
  if (!A || !B || !C) { free(A); free(B); free(C); return ORACLE_E_NOMEM; }
  for (int64_t j = 0; j < ns; ++j) op_p2m(p, src + 3 * j, q[j], c1, A);
  for (int64_t i = 0; i < nx; ++i) {
    double g[3] = {0, 0, 0};
    switch (chain) {
      case 0: phi[i] = op_m2p(p, A, c1, x + 3 * i); break;
      case 1:
        if (i == 0) op_m2m(p, A, c1, c2, B);
        phi[i] = op_m2p(p, B, c2, x + 3 * i);
        break;
      case 2:
        if (i == 0) op_m2l(p, A, c1, c2, B);
        op_l2p(p, B, c2, x + 3 * i, phi + i, g);
        break;
      case 3:
        if (i == 0) {
          op_m2l(p, A, c1, c2, B);
          op_l2l(p, B, c2, c3, C);
        }
        op_l2p(p, C, c3, x + 3 * i, phi + i, g);
        break;
    }
    if (grad)
      for (int a = 0; a < 3; ++a) grad[3 * i + a] = g[a];
  }
  free(A);
  free(B);
  free(C);
  return ORACLE_OK;
}

/* ======================================================================== */
/* Adaptive octree FMM.                                                      */
/* ======================================================================== */
/*
 * Tree (Cheng, Greengard & Rokhlin 1999, sec. 4; Carrier, Greengard &
 * Rokhlin, SIAM J. Sci. Stat. Comput. 9:669 (1988)): the root is the cube; a
 * box holding more than leaf_max particles is divided into its 8 children
 * while its level is below max_depth.  All 8 children of a divided box are
 * kept (an empty child is an empty leaf: it holds nothing and receives
 * nothing, so the result is the same as with empty children dropped).  A
 * particle's box at level l is its cell at max_depth shifted right by
 * max_depth - l (the uniform tree's cell rule).
 *
 * "Adjacent" means the closed cubes touch; boxes may differ in size.
 * Lists of a box b:
 *   U(b), b a leaf: every leaf adjacent to b, b included        -> P2P
 *   V(b): children of the colleagues (adjacent same-level boxes) of b's
 *         parent that are not adjacent to b                      -> M2L
 *   W(b), b a leaf: boxes finer than b, not adjacent to b, whose parent is
 *         adjacent to b                                         -> M2P
 *   X(b): leaves coarser than b, adjacent to b's parent and not adjacent to
 *         b (b is in W of each of them)                         -> P2L
 * Passes in the method's order: P2M at every leaf; M2M from the deepest level
 * up to level 2; for levels 2, 3, ...: L2L from the parent (level >= 3), M2L
 * over V, P2L over X; at every leaf: L2P (level >= 2), M2P over W, P2P over U.
 *
 * Two extra operators:
 *   P2L  L_n^m += q conj(I_n^m(y - c))                 (A1 with the roles of
 *        the two points exchanged, since 1/|x - y| is symmetric)
 *   M2P with gradient: the multipole field's value and gradient at x are the
 *        degree-0 and degree-1 coefficients of its local expansion about x
 *        itself, i.e. (A3) with c_t = x and local degree <= 1.
 */

typedef struct {
  int level, c[3];
  int64_t parent, child0; /* child0 < 0: leaf; else children child0 .. child0+7 */
  int64_t start, count;   /* particles order[start .. start+count) */
} abox;

typedef struct {
  int p, nh, Lmax, leaf_max;
  double lo[3], side;
  int64_t n, nbox, cap;
  abox *box;
  int64_t lvl_first[ORACLE_LMAX + 2]; /* boxes are level-sorted (breadth first) */
  int64_t *order;
  int32_t *cell; /* n x 3, cell at Lmax */
  cplx *M, *Lc;
} atree;

static void atree_free(atree *T) {
  free(T->box);
  free(T->order);
  free(T->cell);
  free(T->M);
  free(T->Lc);
}

static int atree_push(atree *T, const abox *b) {
  if (T->nbox == T->cap) {
    const int64_t nc = T->cap ? 2 * T->cap : 64;
    abox *nb = realloc(T->box, sizeof(abox) * nc);
    if (!nb) return ORACLE_E_NOMEM;
    T->box = nb;
    T->cap = nc;
  }
  T->box[T->nbox++] = *b;
  return ORACLE_OK;
}

static int atree_build(atree *T, int64_t n, const double *pos, int leaf_max, int Lmax, int p,
                       const double lo_in[3], double side_in) {
  memset(T, 0, sizeof(*T));
  T->p = p;
  T->nh = nharm(p);
  T->Lmax = Lmax;
  T->leaf_max = leaf_max;
  T->n = n;
  int st = resolve_cube(n, pos, lo_in, side_in, T->lo, &T->side);
  if (st) return st;
  T->cell = malloc(sizeof(int32_t) * 3 * (n ? n : 1));
  T->order = malloc(sizeof(int64_t) * (n ? n : 1));
  int64_t *tmp = malloc(sizeof(int64_t) * (n ? n : 1));
  if (!T->cell || !T->order || !tmp) { free(tmp); return ORACLE_E_NOMEM; }
  for (int64_t i = 0; i < n; ++i) {
    T->order[i] = i;
    for (int a = 0; a < 3; ++a) T->cell[3 * i + a] = leaf_cell_axis(pos[3 * i + a], T->lo[a], T->side, Lmax);
  }
  abox root = {0, {0, 0, 0}, -1, -1, 0, n};
  st = atree_push(T, &root);
  /* Breadth first, so the boxes come out sorted by level. */
  for (int64_t b = 0; st == ORACLE_OK && b < T->nbox; ++b) {
    const abox B = T->box[b];
    if (B.count <= leaf_max || B.level >= Lmax) continue;
    const int s = Lmax - (B.level + 1);
    int64_t cnt[8] = {0}, off[8];
    for (int64_t k = B.start; k < B.start + B.count; ++k) {
      const int32_t *c = T->cell + 3 * T->order[k];
      cnt[(((c[0] >> s) & 1) << 2) | (((c[1] >> s) & 1) << 1) | ((c[2] >> s) & 1)]++;
    }
    off[0] = B.start;
    for (int ch = 1; ch < 8; ++ch) off[ch] = off[ch - 1] + cnt[ch - 1];
    int64_t fill[8];
    memcpy(fill, off, sizeof(fill));
    for (int64_t k = B.start; k < B.start + B.count; ++k) { /* stable */
      const int32_t *c = T->cell + 3 * T->order[k];
      tmp[fill[(((c[0] >> s) & 1) << 2) | (((c[1] >> s) & 1) << 1) | ((c[2] >> s) & 1)]++] = T->order[k];
    }
    memcpy(T->order + B.start, tmp + B.start, sizeof(int64_t) * B.count);
    T->box[b].child0 = T->nbox;
    for (int ch = 0; ch < 8 && st == ORACLE_OK; ++ch) {
      abox C = {B.level + 1,
                {2 * B.c[0] + (ch >> 2), 2 * B.c[1] + ((ch >> 1) & 1), 2 * B.c[2] + (ch & 1)},
                b, -1, off[ch], cnt[ch]};
      st = atree_push(T, &C);
    }
  }
  free(tmp);
  if (st) return st;
  for (int l = 0; l <= ORACLE_LMAX + 1; ++l) T->lvl_first[l] = T->nbox;
  for (int64_t b = T->nbox - 1; b >= 0; --b) T->lvl_first[T->box[b].level] = b;
  for (int l = ORACLE_LMAX; l >= 0; --l)
    if (T->lvl_first[l] > T->lvl_first[l + 1]) T->lvl_first[l] = T->lvl_first[l + 1];
  T->M = calloc((size_t)T->nbox * T->nh, sizeof(cplx));
  T->Lc = calloc((size_t)T->nbox * T->nh, sizeof(cplx));
  if (!T->M || !T->Lc) return ORACLE_E_NOMEM;
  return ORACLE_OK;
}

/* Closed cubes of boxes a and b touch (any levels). */
static int aadjacent(const abox *a, const abox *b) {
  const int f = a->level > b->level ? a->level : b->level;
  const int sa = f - a->level, sb = f - b->level;
  for (int k = 0; k < 3; ++k) {
    const int64_t alo = (int64_t)a->c[k] << sa, ahi = (int64_t)(a->c[k] + 1) << sa;
    const int64_t blo = (int64_t)b->c[k] << sb, bhi = (int64_t)(b->c[k] + 1) << sb;
    if (alo > bhi || blo > ahi) return 0;
  }
  return 1;
}

static void abox_centre(const atree *T, const abox *b, double c[3]) {
  const double h = T->side / (double)((int64_t)1 << b->level);
  for (int a = 0; a < 3; ++a) c[a] = T->lo[a] + (b->c[a] + 0.5) * h;
}

/* Box of level l at cell c, or -1 when the tree has no such box. */
static int64_t abox_find(const atree *T, int l, const int c[3]) {
  for (int a = 0; a < 3; ++a)
    if (c[a] < 0 || c[a] >= (1 << l)) return -1;
  int64_t b = 0;
  for (int m = 1; m <= l; ++m) {
    if (T->box[b].child0 < 0) return -1;
    const int s = l - m;
    b = T->box[b].child0 + ((((c[0] >> s) & 1) << 2) | (((c[1] >> s) & 1) << 1) | ((c[2] >> s) & 1));
  }
  return b;
}

/* List sink: a growable array of box indices. */
typedef struct { int64_t *v; int64_t n, cap; int err; } alist;
static void alist_add(alist *L, int64_t b) {
  if (L->n == L->cap) {
    const int64_t nc = L->cap ? 2 * L->cap : 32;
    int64_t *nv = realloc(L->v, sizeof(int64_t) * nc);
    if (!nv) { L->err = 1; return; }
    L->v = nv;
    L->cap = nc;
  }
  L->v[L->n++] = b;
}

/* U and W of leaf b: descend from the root through boxes adjacent to b; an
 * adjacent leaf is in U, a non-adjacent box whose parent is adjacent and which
 * is finer than b is in W. */
static void collect_uw(const atree *T, int64_t b, int64_t c, alist *U, alist *W) {
  const abox *B = T->box + b, *C = T->box + c;
  if (!aadjacent(B, C)) {
    if (C->level > B->level) alist_add(W, c);
    return;
  }
  if (C->child0 < 0) { alist_add(U, c); return; }
  for (int ch = 0; ch < 8; ++ch) collect_uw(T, b, C->child0 + ch, U, W);
}

/* V of box b (level >= 2). */
static void collect_v(const atree *T, int64_t b, alist *V) {
  const abox *B = T->box + b, *P = T->box + B->parent;
  for (int dx = -1; dx <= 1; ++dx)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dz = -1; dz <= 1; ++dz) {
        if (!dx && !dy && !dz) continue;
        const int cc[3] = {P->c[0] + dx, P->c[1] + dy, P->c[2] + dz};
        const int64_t col = abox_find(T, P->level, cc);
        if (col < 0 || T->box[col].child0 < 0) continue;
        for (int ch = 0; ch < 8; ++ch)
          if (!aadjacent(B, T->box + T->box[col].child0 + ch)) alist_add(V, T->box[col].child0 + ch);
      }
}

/* X of box b: descend from the root through boxes adjacent to b's parent,
 * above b's level; a leaf there that is not adjacent to b is in X. */
static void collect_x(const atree *T, int64_t b, int64_t c, alist *X) {
  const abox *B = T->box + b, *C = T->box + c;
  if (C->level >= B->level || !aadjacent(T->box + B->parent, C)) return;
  if (C->child0 < 0) {
    if (!aadjacent(B, C)) alist_add(X, c);
    return;
  }
  for (int ch = 0; ch < 8; ++ch) collect_x(T, b, C->child0 + ch, X);
}

/* P2L: local expansion about c of the charge q at y. */
static void op_p2l(int p, const double y[3], double q, const double c[3], cplx *L) {
  cplx Ih[(ORACLE_PMAX + 1) * (ORACLE_PMAX + 1)];
  irregular_harmonics(y[0] - c[0], y[1] - c[1], y[2] - c[2], p, Ih);
  for (int i = 0; i < nharm(p); ++i) L[i] += q * conj(Ih[i]);
}

/* M2P with gradient: local coefficients of degree 0 and 1 about x of the
 * multipole M about c (A3 with c_t = x), read as value and gradient. */
static void op_m2p_grad(int p, const cplx *M, const double c[3], const double x[3], double *phi,
                        double grad[3]) {
  cplx Ih[(ORACLE_PMAX + 2) * (ORACLE_PMAX + 2)];
  irregular_harmonics(x[0] - c[0], x[1] - c[1], x[2] - c[2], p + 1, Ih);
  cplx Lk[4] = {0, 0, 0, 0}; /* (k, l) = (0,0), (1,-1), (1,0), (1,1) */
  for (int k = 0; k <= 1; ++k)
    for (int l = -k; l <= k; ++l) {
      cplx acc = 0.0;
      for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) acc += M[hidx(n, m)] * harm_get(Ih, p + 1, n + k, m - l);
      Lk[hidx(k, l)] = (((k + l) & 1) ? -1.0 : 1.0) * acc;
    }
  *phi = creal(Lk[0]);
  /* gradient of a local expansion at its own centre (A4 at R(0)) */
  grad[0] = creal(0.5 * (Lk[hidx(1, -1)] - Lk[hidx(1, 1)]));
  grad[1] = creal(-0.5 * I * (Lk[hidx(1, 1)] + Lk[hidx(1, -1)]));
  grad[2] = creal(Lk[hidx(1, 0)]);
}

/* Tree statistics reported by oracle_fmm_adaptive (integer, exact):
 *   [0] boxes, [1] leaves, [2] deepest level, [3] sum |U| over leaves,
 *   [4] sum |V|, [5] sum |W| over leaves, [6] sum |X|,
 *   [7] ordered P2P pairs (sum over leaves b of n_b * sum_{c in U(b)} n_c, minus N),
 *   [8] M2L pairs between non-empty boxes. */
#define ORACLE_ASTATS 9

int oracle_fmm_adaptive(int64_t n, const double *pos, const double *q, int leaf_max,
                        int max_depth, int p, const double lo[3], double side, double *phi,
                        double *force, double *energy, int64_t *stats) {
  if (n < 0 || !pos || !q || leaf_max < 1 || max_depth < 0 || max_depth > ORACLE_LMAX || p < 0 ||
      p > ORACLE_PMAX)
    return ORACLE_E_INVALID_ARG;
  atree T;
  int st = atree_build(&T, n, pos, leaf_max, max_depth, p, lo, side);
  if (st) { atree_free(&T); return st; }
  const int nh = T.nh;
  int deepest = 0;
  for (int64_t b = 0; b < T.nbox; ++b)
    if (T.box[b].level > deepest) deepest = T.box[b].level;
  int64_t s_leaf = 0, s_u = 0, s_v = 0, s_w = 0, s_x = 0, s_p2p = 0, s_m2l = 0;
  int fail = 0;

  /* P2M at every leaf. */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t b = 0; b < T.nbox; ++b) {
    const abox *B = T.box + b;
    if (B->child0 >= 0) continue;
    double c[3];
    abox_centre(&T, B, c);
    for (int64_t k = B->start; k < B->start + B->count; ++k) {
      const int64_t j = T.order[k];
      op_p2m(p, pos + 3 * j, q[j], c, T.M + (size_t)b * nh);
    }
  }
  /* M2M, deepest level first, up to level 2. */
  for (int l = deepest - 1; l >= 2; --l) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = T.lvl_first[l]; b < T.lvl_first[l + 1]; ++b) {
      const abox *B = T.box + b;
      if (B->child0 < 0) continue;
      double cp[3];
      abox_centre(&T, B, cp);
      for (int ch = 0; ch < 8; ++ch) {
        const abox *C = T.box + B->child0 + ch;
        double cc[3];
        abox_centre(&T, C, cc);
        op_m2m(p, T.M + (size_t)(B->child0 + ch) * nh, cc, cp, T.M + (size_t)b * nh);
      }
    }
  }
  /* Downward: level by level, L2L from the parent, then M2L over V, P2L over X. */
  for (int l = 2; l <= deepest; ++l) {
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : s_v, s_x, s_m2l) reduction(| : fail)
    for (int64_t b = T.lvl_first[l]; b < T.lvl_first[l + 1]; ++b) {
      const abox *B = T.box + b;
      cplx *Lb = T.Lc + (size_t)b * nh;
      double ct[3];
      abox_centre(&T, B, ct);
      if (l >= 3) {
        double cp[3];
        abox_centre(&T, T.box + B->parent, cp);
        op_l2l(p, T.Lc + (size_t)B->parent * nh, cp, ct, Lb);
      }
      alist V = {0}, X = {0};
      collect_v(&T, b, &V);
      collect_x(&T, b, 0, &X);
      fail |= V.err | X.err;
      for (int64_t k = 0; k < V.n; ++k) {
        double cs[3];
        abox_centre(&T, T.box + V.v[k], cs);
        op_m2l(p, T.M + (size_t)V.v[k] * nh, cs, ct, Lb);
        if (B->count && T.box[V.v[k]].count) s_m2l++;
      }
      for (int64_t k = 0; k < X.n; ++k) {
        const abox *C = T.box + X.v[k];
        for (int64_t m = C->start; m < C->start + C->count; ++m) {
          const int64_t j = T.order[m];
          op_p2l(p, pos + 3 * j, q[j], ct, Lb);
        }
      }
      s_v += V.n;
      s_x += X.n;
      free(V.v);
      free(X.v);
    }
  }
  /* Leaves: L2P, M2P over W, P2P over U. */
  double *phi_all = phi ? phi : malloc(sizeof(double) * (n ? n : 1));
  if (!phi_all) { atree_free(&T); return ORACLE_E_NOMEM; }
  int status = ORACLE_OK;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : s_leaf, s_u, s_w, s_p2p) reduction(| : fail)
  for (int64_t b = 0; b < T.nbox; ++b) {
    const abox *B = T.box + b;
    if (B->child0 >= 0) continue;
    s_leaf++;
    alist U = {0}, W = {0};
    collect_uw(&T, b, 0, &U, &W);
    fail |= U.err | W.err;
    s_u += U.n;
    s_w += W.n;
    int64_t nu = 0;
    for (int64_t k = 0; k < U.n; ++k) nu += T.box[U.v[k]].count;
    s_p2p += B->count * nu;
    double c[3];
    abox_centre(&T, B, c);
    for (int64_t k = B->start; k < B->start + B->count; ++k) {
      const int64_t i = T.order[k];
      const double *x = pos + 3 * i;
      double f = 0.0, g[3] = {0.0, 0.0, 0.0};
      if (B->level >= 2) op_l2p(p, T.Lc + (size_t)b * nh, c, x, &f, g);
      for (int64_t w = 0; w < W.n; ++w) {
        double cw[3], fw, gw[3];
        abox_centre(&T, T.box + W.v[w], cw);
        op_m2p_grad(p, T.M + (size_t)W.v[w] * nh, cw, x, &fw, gw);
        f += fw;
        for (int a = 0; a < 3; ++a) g[a] += gw[a];
      }
      ksum fn = {0, 0}, gx = {0, 0}, gy = {0, 0}, gz = {0, 0};
      for (int64_t u = 0; u < U.n; ++u) {
        const abox *C = T.box + U.v[u];
        for (int64_t m = C->start; m < C->start + C->count; ++m) {
          const int64_t j = T.order[m];
          if (j == i) continue;
          const double dx = x[0] - pos[3 * j], dy = x[1] - pos[3 * j + 1], dz = x[2] - pos[3 * j + 2];
          const double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 == 0.0) {
#pragma omp atomic write
            status = ORACLE_E_COINCIDENT;
            continue;
          }
          const double r = sqrt(r2), qr = q[j] / r, qr3 = qr / r2;
          ksum_add(&fn, qr);
          ksum_add(&gx, -qr3 * dx);
          ksum_add(&gy, -qr3 * dy);
          ksum_add(&gz, -qr3 * dz);
        }
      }
      phi_all[i] = f + ksum_val(&fn);
      if (force) {
        force[3 * i] = -q[i] * (g[0] + ksum_val(&gx));
        force[3 * i + 1] = -q[i] * (g[1] + ksum_val(&gy));
        force[3 * i + 2] = -q[i] * (g[2] + ksum_val(&gz));
      }
    }
    free(U.v);
    free(W.v);
  }
  if (energy) {
    ksum e = {0, 0};
    for (int64_t i = 0; i < n; ++i) ksum_add(&e, q[i] * phi_all[i]);
    *energy = 0.5 * ksum_val(&e);
  }
  if (stats) {
    stats[0] = T.nbox;
    stats[1] = s_leaf;
    stats[2] = deepest;
    stats[3] = s_u;
    stats[4] = s_v;
    stats[5] = s_w;
    stats[6] = s_x;
    stats[7] = s_p2p - n;
    stats[8] = s_m2l;
  }
  if (!phi) free(phi_all);
  atree_free(&T);
  if (fail) return ORACLE_E_NOMEM;
  return status;
}
