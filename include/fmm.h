/*
 * fmm.h -- C ABI of libfmm.so, a fast multipole method (FMM) for the 3-D
 * Coulomb / Laplace sum on AMD Instinct MI355X (gfx950).
 *
 * Problem (the exact result the method approximates; open boundary, pure 1/r
 * kernel with no Coulomb constant, i = j excluded, no softening):
 *     phi_i = sum_{j != i} q_j / |x_i - x_j|
 *     F_i   = -q_i grad phi_i = q_i sum_{j != i} q_j (x_i - x_j) / |x_i - x_j|^3
 *     E     = 1/2 sum_i q_i phi_i
 *
 * Method: uniform octree of depth L (root = level 0) over a cube, boxes kept in
 * Hilbert order; well-separatedness 1 (near list = 27 boxes at Chebyshev index
 * distance <= 1; interaction list = children of the parent's near list that are
 * not in the box's near list); multipole and local expansions of degree <= p
 * about box centres with every (local degree <= p, multipole degree <= p) pair
 * kept in the multipole-to-local (M2L) translation.  The passes are P2M, M2M
 * (leaves up to level 2), M2L (levels 2..L), L2L (level 2 down to the leaves),
 * L2P and the P2P near-field direct sum (Greengard, "The Rapid Evaluation of
 * Potential Fields in Particle Systems", MIT Press 1988, ch. 3; Cheng, Greengard
 * & Rokhlin, J. Comput. Phys. 155:468 (1999), sec. 2-3).
 *
 * Conventions shared by every call
 *   - Memory: the caller owns every device buffer, the workspace included; the
 *     library allocates no device memory.  It owns only the host-side plan
 *     object, freed by fmm_destroy.  Input arrays are read-only.
 *   - Layouts: positions are n x 3 row-major FP64 (x0 y0 z0 x1 ...); charges,
 *     potentials n FP64; forces n x 3 row-major FP64; all in the caller's
 *     ("user") particle order.  Pointers marked "device" must be device memory.
 *   - Streams: every call that takes a hipStream_t only enqueues work on that
 *     stream and returns; a plan must not be used from two streams at once.
 *   - Determinism: every sum is taken in a fixed order (no floating-point
 *     atomics), so repeated runs on the same inputs are bitwise identical.
 *   - Errors: argument errors are detected on the host, returned at once and
 *     leave every output untouched.  Errors found by kernels (a point outside a
 *     given cube, a non-finite coordinate, two distinct particles at the same
 *     point) raise a flag in the workspace; fmm_check waits for the stream and
 *     reports it.  Outputs of a call whose flag is raised are unspecified (but
 *     every kernel stays in bounds).  HIP runtime failures map to FMM_E_DEVICE.
 *     No call aborts or throws.
 */
#ifndef FMM_H_
#define FMM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMM_ABI_VERSION 2
#define FMM_P_MAX 12     /* largest expansion order */
#define FMM_DEPTH_MAX 9  /* deepest uniform tree (8^9 leaves) */

typedef struct ihipStream_t *fmm_stream_t; /* a hipStream_t; NULL = the null stream */

typedef enum {
  FMM_OK = 0,
  FMM_E_INVALID_ARG = 1, /* a NULL pointer, size or config field out of range */
  FMM_E_WORKSPACE = 2,   /* workspace NULL, misaligned (256 B) or too small */
  FMM_E_OUT_OF_CUBE = 3, /* device: a position outside the given root cube */
  FMM_E_NONFINITE = 4,   /* device: a non-finite coordinate */
  FMM_E_COINCIDENT = 5,  /* device: two distinct particles at the same point */
  FMM_E_UNSUPPORTED = 6, /* a valid request this build does not implement */
  FMM_E_DEVICE = 7       /* a HIP runtime call failed */
} fmm_status;

typedef enum {
  FMM_PREC_FP64 = 0,  /* every pass in FP64 */
  FMM_PREC_MIXED = 1  /* P2M, L2P, P2P in FP32, M2L on the FP32 matrix cores or on split
                         FP16 / BF16 operands with FP32 accumulation (fmm_m2l_kind); M2M,
                         L2L, the combination of results and the energy in FP64 */
} fmm_precision;

typedef enum {
  FMM_M2L_AUTO = 0,   /* FMM_M2L_F64 for FMM_PREC_FP64, FMM_M2L_F16X2 for FMM_PREC_MIXED */
  FMM_M2L_F64 = 1,    /* FP64 matrix cores (FMM_PREC_FP64 only) */
  FMM_M2L_F32 = 2,    /* FP32 matrix cores (FMM_PREC_MIXED only) */
  FMM_M2L_BF16X2 = 3, /* BF16 matrix cores, operands split into 2 BF16 pieces, 3 piece
                         products, FP32 accumulation (FMM_PREC_MIXED only; about
                         16 significant bits per product, below the FP32 modes) */
  FMM_M2L_BF16X3 = 4, /* BF16 matrix cores, operands split into 3 BF16 pieces (exact for
                         FP32 values), the 6 piece products of total order <= 2, FP32
                         accumulation (FMM_PREC_MIXED only; FP32-level products) */
  FMM_M2L_F16X2 = 5   /* FP16 matrix cores: operators and multipoles scaled by powers of
                         two (per operator row and column, and per source box) into the
                         FP16 range and split into 2 FP16 pieces, the 3 piece products
                         of total order <= 1, FP32 accumulation (FMM_PREC_MIXED only;
                         about 22 significant bits per product) */
} fmm_m2l_kind;

typedef struct {
  uint32_t abi_version; /* must equal FMM_ABI_VERSION */
  int32_t p;            /* expansion order, 0..FMM_P_MAX */
  int32_t depth;        /* uniform tree (leaf_max == 0): the leaf level L,
                           0..FMM_DEPTH_MAX; L <= 1 has no well-separated pairs,
                           so the result is the direct sum.
                           adaptive tree (leaf_max > 0): the deepest level a box
                           may be divided down to (depth cap), 0..FMM_DEPTH_MAX */
  int32_t leaf_max;     /* 0: uniform tree of leaf level depth.
                           > 0: adaptive tree (Cheng, Greengard & Rokhlin 1999,
                           sec. 4): a box holding more than leaf_max particles is
                           divided into its 8 children while its level is below
                           depth; U, V, W, X lists (P2P, M2L, M2P, P2L).  The
                           workspace holds list capacities of 40, 16 and 16
                           entries per possible box for U, W and X; a tree whose
                           lists exceed them fails fmm_plan with
                           FMM_E_WORKSPACE.  < 0: FMM_E_INVALID_ARG. */
  int32_t ws;           /* well-separatedness; must be 1 */
  int32_t precision;    /* fmm_precision */
  int32_t m2l_kind;     /* fmm_m2l_kind; must agree with precision or be AUTO
                           (else FMM_E_UNSUPPORTED) */
  double root_lo[3];    /* root cube corner */
  double root_side;     /* > 0: the cube [root_lo, root_lo + root_side]^3, which
                           must contain every position (else FMM_E_OUT_OF_CUBE);
                           <= 0: derived on the device as lo_a = min_i x_ia,
                           side = max_a (max_i x_ia - lo_a), or 1 if that is 0 */
  int32_t batch_level;  /* adaptive tree only: 0 for one system; b > 0: every box of
                           level b is an independent system (a batch of systems,
                           one per box of level b, e.g. each in its own cell of
                           the root cube).  Boxes above level b that hold
                           particles are always divided, and no pair of
                           particles in different level-b boxes interacts: the
                           result per system is that of a plan for the system
                           alone with its level-b box as the root cube, and the
                           energy is the sum over the systems.  0..depth, else
                           FMM_E_INVALID_ARG; > 0 with leaf_max == 0:
                           FMM_E_UNSUPPORTED. */
  int32_t reserved;     /* must be 0 */
} fmm_config;

typedef struct fmm_plan_s fmm_plan_t; /* opaque */

/* Fill *cfg with defaults: p = 8, depth = 3, ws = 1, FP64, unit cube at 0. */
void fmm_config_default(fmm_config *cfg);

/* Bytes of device workspace a plan for n particles under cfg needs.
 * Pure host computation.  Errors: FMM_E_INVALID_ARG (cfg or bytes NULL, a field
 * out of range, n < 1 or n > 2^31 - 1). */
fmm_status fmm_workspace_size(const fmm_config *cfg, int64_t n, size_t *bytes);

/* Build the tree for n particles at d_pos (device, n x 3 FP64, user order):
 * quantise to leaf cells of the root cube, Hilbert keys, counting sort into
 * Hilbert order (ties kept in user order), leaf ranges, per-level box maps,
 * box-local coordinates, and the translation operators for order p.
 * d_workspace (device, 256-byte aligned, >= fmm_workspace_size bytes) is owned
 * by the caller and must stay valid and unused by others until fmm_destroy.
 * On FMM_OK *out receives a new plan (host object); work is only enqueued,
 * except for an adaptive tree (leaf_max > 0), whose box and list counts are
 * read back: the call then synchronises the stream twice.
 * Errors: FMM_E_INVALID_ARG, FMM_E_WORKSPACE (also: adaptive lists over
 * capacity), FMM_E_DEVICE (*out is left unchanged on any error). */
fmm_status fmm_plan(const fmm_config *cfg, int64_t n, const double *d_pos, void *d_workspace,
                    size_t workspace_bytes, fmm_stream_t stream, fmm_plan_t **out);

/* Build the tree of plan for new positions d_pos (device, n x 3 FP64, user
 * order; the same n and configuration), keeping the translation operators
 * already in the plan's workspace: they depend on p and the M2L form only, so
 * a sequence of position sets (time steps of a simulation) generates them
 * once.  Everything else is as for fmm_plan (the tree build, the adaptive
 * tree's read-backs); charges of an earlier fmm_evaluate are forgotten; the
 * profiling selection and unread profile records are kept.  Errors: FMM_E_INVALID_ARG (plan or
 * d_pos NULL), FMM_E_WORKSPACE (adaptive lists over capacity), FMM_E_DEVICE. */
fmm_status fmm_replan(fmm_plan_t *plan, const double *d_pos, fmm_stream_t stream);

/* Schedule of a plan's passes: how work is spread over the GPU, never what
 * is computed.  Keys:
 *   FMM_SCHED_P2P_PERSISTENT: 0 (default) one wave per box; 1 (adaptive tree
 *     only, else FMM_E_UNSUPPORTED) a persistent launch whose resident waves
 *     take the non-empty leaves from a work-list built at plan time, costliest
 *     (most ordered pairs) first.  Results are bitwise the same.
 *   FMM_SCHED_M2L_SPLIT: 0..16 (default 16), split M2L forms: how many of the
 *     last work-groups of each XCD run as four parts over the offsets, added in
 *     part order afterwards (a shorter last round; the summation order of those
 *     tiles changes, within rounding).
 *   FMM_SCHED_M2L_PERSISTENT: 0 (default) one work-group per M2L tile; 1 (the
 *     scaled FP16 form at p <= 8 with an M2L pass, else FMM_E_UNSUPPORTED) a
 *     persistent launch of two work-groups per CU, those of each XCD taking
 *     the XCD's tiles in order from a counter; no tile is split, so results
 *     equal bitwise those of FMM_SCHED_M2L_SPLIT 0 (which it overrides).
 *   FMM_SCHED_P2P_TILE: 128, 256 or 512 (default 128 in mixed precision, 256
 *     in FP64): sources a P2P wave stages in LDS at a time (the per-leaf
 *     kernels; the uniform tree's kernel for small leaves keeps its own).
 *     Results are bitwise the same.
 * Kept by fmm_replan.  Errors: FMM_E_INVALID_ARG (plan NULL, unknown key or
 * value out of range), FMM_E_UNSUPPORTED. */
enum {
  FMM_SCHED_P2P_PERSISTENT = 0,
  FMM_SCHED_M2L_SPLIT = 1,
  FMM_SCHED_M2L_PERSISTENT = 2,
  FMM_SCHED_P2P_TILE = 3
};
fmm_status fmm_plan_set_schedule(fmm_plan_t *plan, int key, int value);

/* Evaluate the FMM for charges d_q (device, n FP64, user order).  Any of
 * d_phi (n), d_force (n x 3), d_energy (1 FP64) may be NULL; all are device
 * pointers in user order.  The positions of the plan are those passed to
 * fmm_plan.  Errors: FMM_E_INVALID_ARG (plan or d_q NULL), FMM_E_DEVICE. */
fmm_status fmm_evaluate(fmm_plan_t *plan, const double *d_q, double *d_phi, double *d_force,
                        double *d_energy, fmm_stream_t stream);

/* Adjoint of the energy E = 1/2 q^T K q of the last fmm_evaluate on this plan.
 * Given the upstream gradient d_grad_energy (device, one FP64 g = dL/dE),
 * writes d_dE_dq = g dE/dq = g phi (n) and d_dE_dx = g dE/dx = g q_i grad phi_i
 * = -g F_i (n x 3), both device, user order, either may be NULL.  Every pass
 * is recomputed from the stored charges (nothing of the forward call is
 * kept).  The FMM energy is exactly symmetric in the charges (every (local <=
 * p, multipole <= p) pair is kept), and differentiable in x_i wherever no
 * particle crosses a box face (Greengard 1988, ch. 3; the expansions are
 * polynomials in the box-local offsets).  Same precision mode as the plan.
 * Errors: FMM_E_INVALID_ARG (plan or d_grad_energy NULL, or no fmm_evaluate
 * on the plan yet), FMM_E_DEVICE. */
fmm_status fmm_backward(fmm_plan_t *plan, const double *d_grad_energy, double *d_dE_dx,
                        double *d_dE_dq, fmm_stream_t stream);

/* Wait for the plan's last stream and report a device-detected error
 * (FMM_E_OUT_OF_CUBE, FMM_E_NONFINITE, FMM_E_COINCIDENT) or FMM_OK. */
fmm_status fmm_check(fmm_plan_t *plan);

/* Free the host plan object (waits for its last stream first).  NULL is a no-op. */
fmm_status fmm_destroy(fmm_plan_t *plan);

/* Static text for a status code. */
const char *fmm_status_string(fmm_status status);

/* ---- a variant that allocates nothing ------------------------------------ */

/* Bytes of the device scratch array fmm_evaluate_static works in (one array
 * per GPU the library runs on, held until the process ends). */
#define FMM_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): fmm_plan followed
 * by fmm_evaluate, with the workspace taken from a device scratch array of
 * FMM_STATIC_SCRATCH_BYTES that the library holds on the current device, and
 * the plan object a static of the library's too.  The call allocates no device
 * or host memory.  Arguments as for fmm_plan and fmm_evaluate; the caller
 * still passes d_pos, d_q and the outputs (device, user order).
 * *out_plan (if out_plan is not NULL) receives the library's plan for this
 * device, usable with fmm_check, fmm_backward, fmm_plan_work and
 * fmm_plan_tree_stats until the next fmm_evaluate_static call on the device;
 * fmm_destroy on it only waits for its stream; fmm_profile_enable on it
 * returns FMM_E_UNSUPPORTED.
 * Every call on one GPU shares that GPU's array and plan: calls that overlap
 * on one GPU (different streams, or host threads) race.  The array keeps the
 * last call's contents; every pass clears what it needs.
 * Errors: FMM_E_INVALID_ARG, FMM_E_UNSUPPORTED (as fmm_plan),
 * FMM_E_WORKSPACE (the plan needs more than FMM_STATIC_SCRATCH_BYTES, see
 * fmm_workspace_size; or adaptive lists over capacity), FMM_E_DEVICE. */
fmm_status fmm_evaluate_static(const fmm_config *cfg, int64_t n, const double *d_pos,
                               const double *d_q, double *d_phi, double *d_force,
                               double *d_energy, fmm_stream_t stream, fmm_plan_t **out_plan);

/* ---- introspection (tests and measurement) ------------------------------- */

/* Leaf cell (ix, iy, iz) of every particle in user order (d_cells: device,
 * n x 3 int32) and the Hilbert slot of its leaf (d_leaf: device, n uint32); either
 * may be NULL.  Enqueued on stream.  Errors: FMM_E_INVALID_ARG, FMM_E_DEVICE. */
fmm_status fmm_plan_leaves(fmm_plan_t *plan, int32_t *d_cells, uint32_t *d_leaf,
                           fmm_stream_t stream);

/* The resolved root cube (waits for the stream). */
fmm_status fmm_plan_cube(fmm_plan_t *plan, double lo[3], double *side);

/* 3-D Hilbert index (3 * bits bits) of cell (ix, iy, iz) on a 2^bits grid, the
 * curve the library sorts by (Skilling, AIP Conf. Proc. 707:381 (2004)).  Host
 * function; returns 0 for arguments out of range. */
uint64_t fmm_hilbert_index(uint32_t ix, uint32_t iy, uint32_t iz, int32_t bits);

/* Kernel-duration recording.  fmm_profile_enable(plan, mask) selects the
 * passes to time: bit (1 << FMM_PHASE_x) for pass x, FMM_PROFILE_ALL for every
 * pass, 0 for none (the default).  For each selected pass the library records
 * HIP events on the call's stream around its launches (each event pair costs
 * a few microseconds of stream time).  fmm_profile_read waits for them, writes
 * for each pass (FMM_PHASE_*) the summed duration in ms and the number of
 * launches, and clears the record.  Capacity: 8192 launches between reads
 * (later launches are not recorded). */
enum {
  FMM_PHASE_TREE = 0,   /* quantise, keys, count, scan, scatter, leaf sort, gather */
  FMM_PHASE_OPERATORS,  /* translation-operator tables */
  FMM_PHASE_P2M,
  FMM_PHASE_M2M,
  FMM_PHASE_M2L,        /* the M2L kernel alone */
  FMM_PHASE_L2L,        /* adaptive tree: P2L included */
  FMM_PHASE_L2P,        /* adaptive tree: M2P included */
  FMM_PHASE_P2P,        /* near field, combination, unpermute, energy partials */
  FMM_PHASE_ENERGY,
  FMM_PHASE_SPLIT,      /* split forms of M2L: multipoles into BF16 / FP16 pieces */
  FMM_PHASE_COUNT
};
#define FMM_PROFILE_ALL 0x3ff
fmm_status fmm_profile_enable(fmm_plan_t *plan, int phase_mask);
fmm_status fmm_profile_read(fmm_plan_t *plan, double ms[FMM_PHASE_COUNT],
                            int32_t launches[FMM_PHASE_COUNT]);

/* Algorithmic work of the plan's tree (after the stream has finished the
 * plan): number of M2L (target, source) box pairs with both boxes non-empty,
 * summed over levels 2..L, and number of ordered P2P particle pairs (i != j).
 * Synchronises the plan's stream. */
fmm_status fmm_plan_work(fmm_plan_t *plan, int64_t *m2l_pairs, int64_t *p2p_pairs);

/* Integer statistics of an adaptive plan's tree (Cheng, Greengard & Rokhlin
 * 1999, sec. 4; all 8 children of a divided box counted, empty ones included):
 *   stats[0] boxes, [1] leaves, [2] deepest level, [3] sum over leaves of |U|
 *   (the leaf itself included), [4] sum over boxes of |V|, [5] sum of |W|,
 *   [6] sum of |X|, [7] ordered P2P particle pairs (i != j), [8] M2L (V) pairs
 *   with both boxes non-empty.
 * Synchronises the plan's stream.  Errors: FMM_E_INVALID_ARG (NULL),
 * FMM_E_UNSUPPORTED (uniform plan), FMM_E_DEVICE. */
#define FMM_TREE_STATS 9
fmm_status fmm_plan_tree_stats(fmm_plan_t *plan, int64_t stats[FMM_TREE_STATS]);

#ifdef __cplusplus
}
#endif
#endif /* FMM_H_ */
