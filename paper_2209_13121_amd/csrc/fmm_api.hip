// fmm_api.hip -- the C ABI of libfmm.so: argument validation, workspace
// layout, plan lifetime, pass sequencing and kernel-duration recording.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "fmm_internal.h"

namespace fmm {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int m2l_pieces(const fmm_config& cfg) {
  if (cfg.precision != FMM_PREC_MIXED) return 0;
  if (cfg.m2l_kind == FMM_M2L_BF16X2 || cfg.m2l_kind == FMM_M2L_F16X2 ||
      cfg.m2l_kind == FMM_M2L_AUTO)
    return 2;
  if (cfg.m2l_kind == FMM_M2L_BF16X3) return 3;
  return 0;
}

bool m2l_is_f16(const fmm_config& cfg) {  // FMM_M2L_F16X2, the mixed AUTO choice
  return cfg.precision == FMM_PREC_MIXED &&
         (cfg.m2l_kind == FMM_M2L_F16X2 || cfg.m2l_kind == FMM_M2L_AUTO);
}

bool make_layout(const fmm_config& cfg, int64_t n, Layout* lay) {
  memset(lay, 0, sizeof(*lay));
  const int L = cfg.depth, p = cfg.p, nc = ncoef(p);
  const bool mixed = cfg.precision == FMM_PREC_MIXED;
  lay->n = n;
  lay->nleaf = (int64_t)1 << (3 * L);
  int64_t off = 0;
  for (int l = 0; l <= L; ++l) {
    lay->lvl_off[l] = off;
    off += (int64_t)1 << (3 * l);
  }
  lay->lvl_off[L + 1] = off;
  lay->nbox = off;
  // energy: q_i phi_i per particle, then sums of 4 kBlock terms
  lay->n_energy_part = n + (n + 4 * kBlock - 1) / (4 * kBlock);
  const bool adaptive = cfg.leaf_max > 0;
  if (adaptive) {
    // Every existing box but the root is one of 8 children of a divided box.
    // Below the batch level a divided box holds more than leaf_max particles,
    // so such a level has at most min(8^l, n / (leaf_max + 1)) of them; above
    // it (batch_level > 0) every non-empty box is divided: min(8^l, n).
    int64_t div = 0;
    for (int l = 0; l < L; ++l)
      div += std::min<int64_t>((int64_t)1 << (3 * l),
                               l < cfg.batch_level ? n : n / ((int64_t)cfg.leaf_max + 1));
    lay->bmax = 1 + 8 * div;
    lay->ucap = 40 * lay->bmax;
    lay->wcap = 16 * lay->bmax;
    lay->xcap = 16 * lay->bmax;
    // M2L source table: 8 x 189 entries per divided parent, tiles of 128
    // padded, at most L + 1 partly filled tiles per class
    lay->vtcap = ((lay->bmax + 7) / 8 + 128 * (int64_t)(L + 1)) * 8 * kIL;
  }
  lay->nbox_exp = adaptive ? lay->bmax : lay->nbox;
  // scan scratch: block sums of every level of the recursive scan, for the
  // longest scan (leaf counts; adaptive: also the dense box flags and lists)
  int64_t longest = lay->nleaf + 1;
  if (sort_two_level(L)) longest = std::max(longest, sort_hist_elems(n));
  if (adaptive) longest = std::max(longest, std::max(lay->nbox + 1, lay->bmax + 1));
  int64_t tmp = 0, m = longest;
  while (m > 1) {
    m = (m + 1023) / 1024;
    tmp += m;
  }
  lay->scan_tmp_elems = tmp + 1;

  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t at = cur;
    cur = align256(cur + (bytes ? bytes : 1));
    return at;
  };
  const size_t N = (size_t)n, NB = (size_t)lay->nbox_exp, NL = (size_t)lay->nleaf;
  const size_t ND = (size_t)lay->nbox;  // dense boxes of every level
  lay->params = take(sizeof(DevParams));
  lay->flags = take(sizeof(int32_t) * 4);
  lay->energy_part = take(sizeof(double) * (size_t)lay->n_energy_part);
  lay->bbox = take(sizeof(double) * 6 * 1024);
  const int np = m2l_pieces(cfg);
  lay->zero_row = take(zero_row_bytes(p, np));
  lay->keys = take(sizeof(uint32_t) * N);
  lay->perm = take(sizeof(int32_t) * N);
  lay->perm_tmp = take(sizeof(int32_t) * N);
  lay->sorted_leaf = take(sizeof(uint32_t) * N);
  lay->sort_hist = sort_two_level(L) ? take(sizeof(uint32_t) * (size_t)sort_hist_elems(n)) : 0;
  lay->leaf_count = take(sizeof(uint32_t) * NL);
  lay->leaf_start = take(sizeof(uint32_t) * (NL + 1));
  lay->leaf_fill = take(sizeof(uint32_t) * NL);
  lay->scan_tmp = take(sizeof(uint32_t) * (size_t)lay->scan_tmp_elems);
  lay->coord2slot = take(sizeof(uint32_t) * ND);
  lay->slot2coord = take(sizeof(uint32_t) * ND);
  lay->src = take((mixed ? sizeof(Rec<float>) : sizeof(Rec<double>)) * N);
  lay->src64 = mixed ? take(sizeof(Rec<double>) * N) : 0;
  lay->q64 = take(sizeof(double) * N);
  lay->far_phi = take(sizeof(double) * N);
  lay->far_grad = take(sizeof(double) * 3 * N);
  const size_t nce = (size_t)nc;
  if (L >= 2) {
    const size_t ms = (size_t)mstride(p);
    lay->mult64 = take(sizeof(double) * NB * ms);
    lay->mult32 = mixed ? take(sizeof(float) * NB * ms) : 0;
    lay->m2l_out = take((mixed ? sizeof(float) : sizeof(double)) * NB * nce);
    lay->loc_exp64 = take(sizeof(double) * NB * ms);
    // mixed: FP32 leaf locals for L2P (adaptive: a copy of every box's local)
    lay->leaf_loc32 = mixed ? take(sizeof(float) * (adaptive ? NB : NL) * ms) : 0;
    const size_t tile = (size_t)shift_kpad(nc) * m2l_rows_pad(p);
    lay->op_m2m = take(sizeof(double) * 8 * tile);
    lay->op_l2l = take(sizeof(double) * 8 * tile);
    const size_t el = mixed ? sizeof(float) : sizeof(double);
    const size_t opsz = (size_t)kNumM2LOps * m2l_rows_pad(p) * m2l_kstride_of(nc, (int)el);
    lay->op_m2l64 = mixed ? 0 : take(sizeof(double) * opsz);
    lay->op_m2l32 = (mixed && !np) ? take(sizeof(float) * opsz) : 0;
    if (np) {
      const size_t rq = (size_t)m2lb_row_quads(nc, np);
      lay->multb = take(16 * NB * rq);
      lay->op_m2lb = take(16 * (size_t)kNumM2LOps * m2lb_op_quads(nc, np, adaptive));
      lay->m2l_half = take(sizeof(float) * 8 * kM2lSplitPerXcd * (kM2lParts - 1) * 128 * (size_t)nc);
      lay->m2l_ctl = take(sizeof(uint32_t) * 8);
    }
    if (m2l_is_f16(cfg)) {
      const size_t rp = (size_t)m2lb_rows(nc), kp = (size_t)32 * m2lb_ksteps(nc);
      lay->f16_lmax = take(sizeof(uint32_t) * (FMM_DEPTH_MAX + 2));
      lay->f16_rowf = take(sizeof(float) * rp);
      lay->f16_colf = take(sizeof(float) * kp);
      lay->f16_tbl = take(sizeof(uint32_t) * rp * kp);
      lay->op_m2l_scratch = take(sizeof(double) * (size_t)kNumM2LOps * rp * kp);
    }
  }
  lay->work = take(sizeof(int64_t) * 2);
  if (adaptive) {
    const size_t BM = (size_t)lay->bmax;
    lay->a_present = take(sizeof(uint32_t) * (ND + 1));
    lay->a_scan = take(sizeof(uint32_t) * (ND + 1));
    lay->a_slot = take(sizeof(uint32_t) * BM);
    lay->a_level = take(sizeof(int32_t) * BM);
    lay->a_coord = take(sizeof(uint32_t) * BM);
    lay->a_range = take(sizeof(uint32_t) * 2 * BM);
    lay->a_child0 = take(sizeof(int32_t) * BM);
    lay->a_parent_of = take(sizeof(uint32_t) * BM);
    lay->a_cnt = take(sizeof(uint32_t) * 3 * (BM + 1));
    lay->a_off = take(sizeof(uint32_t) * 3 * (BM + 1));
    lay->a_uidx = take(sizeof(uint32_t) * (size_t)lay->ucap);
    lay->a_widx = take(sizeof(uint32_t) * (size_t)lay->wcap);
    lay->a_xidx = take(sizeof(uint32_t) * (size_t)lay->xcap);
    lay->a_wbox = take(sizeof(uint32_t) * BM);
    lay->a_xbox = take(sizeof(uint32_t) * BM);
    lay->a_flag = take(sizeof(uint32_t) * (BM + 1));
    lay->a_fscan = take(sizeof(uint32_t) * 2 * (BM + 1));
    lay->a_tgt = take(sizeof(uint32_t) * BM);
    lay->a_vtab = take(sizeof(uint32_t) * (size_t)lay->vtcap);
    lay->a_p2p_bucket = take(BM);
    lay->a_p2p_list = take(sizeof(uint32_t) * BM);
    lay->a_p2p_ctl = take(sizeof(uint32_t) * 66);
    lay->a_small = take(sizeof(uint32_t) * 64);
    lay->a_stats = take(sizeof(int64_t) * 8);
  }
  lay->total = cur;
  return true;
}

static inline fmm_status from_hip(hipError_t e) { return e == hipSuccess ? FMM_OK : FMM_E_DEVICE; }

void prof_begin(fmm_plan_s* P, int phase, hipStream_t s) {
  P->prof_open = false;
  if (!P->rec || !((P->profile_mask >> phase) & 1u) || P->nrec >= kMaxProfile) return;
  ProfileRec& r = P->rec[P->nrec];
  if (P->nrec >= P->nevents_created) {
    if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) return;
    P->nevents_created = P->nrec + 1;
  }
  r.phase = phase;
  hipEventRecord(r.start, s);
  P->prof_open = true;
}

void prof_end(fmm_plan_s* P, hipStream_t s) {
  if (!P->prof_open) return;
  P->prof_open = false;
  hipEventRecord(P->rec[P->nrec].stop, s);
  P->nrec++;
}

// Every pass before the near field: upward, M2L (+ P2L on the adaptive tree),
// downward.
static hipError_t run_passes(fmm_plan_s* P, const double* d_q, hipStream_t s) {
  hipError_t e = launch_upward(P, d_q, s);
  if (P->Ld >= 2) {
    if (e == hipSuccess) e = launch_m2l(P, s);
    if (e == hipSuccess && P->adaptive) {
      prof_begin(P, FMM_PHASE_L2L, s);  // P2L builds local expansions: timed with L2L
      e = launch_adaptive_p2l(P, s);
      prof_end(P, s);
    }
  }
  if (e == hipSuccess && (P->Ld >= 2 || P->adaptive)) e = launch_downward(P, s);
  return e;
}

static fmm_status validate_config(const fmm_config* cfg) {
  if (!cfg) return FMM_E_INVALID_ARG;
  if (cfg->abi_version != FMM_ABI_VERSION) return FMM_E_INVALID_ARG;
  if (cfg->p < 0 || cfg->p > FMM_P_MAX) return FMM_E_INVALID_ARG;
  if (cfg->depth < 0 || cfg->depth > FMM_DEPTH_MAX) return FMM_E_INVALID_ARG;
  if (cfg->ws != 1) return FMM_E_INVALID_ARG;
  if (cfg->leaf_max < 0) return FMM_E_INVALID_ARG;
  if (cfg->batch_level < 0 || cfg->batch_level > cfg->depth || cfg->reserved != 0)
    return FMM_E_INVALID_ARG;
  if (cfg->batch_level > 0 && cfg->leaf_max == 0) return FMM_E_UNSUPPORTED;
  if (cfg->precision != FMM_PREC_FP64 && cfg->precision != FMM_PREC_MIXED) return FMM_E_INVALID_ARG;
  if (cfg->m2l_kind < FMM_M2L_AUTO || cfg->m2l_kind > FMM_M2L_F16X2) return FMM_E_INVALID_ARG;
  if (cfg->m2l_kind == FMM_M2L_F64 && cfg->precision != FMM_PREC_FP64) return FMM_E_UNSUPPORTED;
  if (cfg->m2l_kind >= FMM_M2L_F32 && cfg->precision != FMM_PREC_MIXED) return FMM_E_UNSUPPORTED;
  for (int a = 0; a < 3; ++a)
    if (!(cfg->root_lo[a] == cfg->root_lo[a]) || cfg->root_lo[a] - cfg->root_lo[a] != 0.0)
      return FMM_E_INVALID_ARG;  // NaN or infinite corner
  if (!(cfg->root_side == cfg->root_side) || cfg->root_side - cfg->root_side != 0.0)
    return FMM_E_INVALID_ARG;
  return FMM_OK;
}

// Fill plan P (host object owned by the caller) for n particles at d_pos with
// workspace ws laid out as lay, and enqueue the tree build and the operator
// tables on s.  rec: kMaxProfile profile records, or NULL (no profiling).
fmm_status plan_into(fmm_plan_s* P, const fmm_config& cfg, const Layout& lay, int64_t n,
                     const double* d_pos, char* ws, hipStream_t s, ProfileRec* rec,
                     bool keep_operators) {
  // what a re-plan keeps: the operator tables in the workspace, profiling state
  const bool ops_ready = keep_operators && P->ops_ready;
  const uint32_t mask = keep_operators ? P->profile_mask : 0u;
  const int nevents = keep_operators ? P->nevents_created : 0;
  const int nrec = keep_operators ? P->nrec : 0;
  const bool is_static = keep_operators && P->is_static;
  const int p2p_persistent = keep_operators ? P->p2p_persistent : 0;
  const int m2l_split = keep_operators ? P->m2l_split : kM2lSplitPerXcd;
  const int m2l_persistent = keep_operators ? P->m2l_persistent : 0;
  // P2P tile: 128 sources in mixed precision (the occupancy stays with the
  // registers), 256 in FP64
  const int p2p_tile = keep_operators ? P->p2p_tile : (cfg.precision == FMM_PREC_MIXED ? 128 : 256);
  memset(P, 0, sizeof(*P));
  P->p2p_tile = p2p_tile;
  P->p2p_persistent = p2p_persistent;
  P->m2l_split = m2l_split;
  P->m2l_persistent = m2l_persistent;
  P->ops_ready = ops_ready;
  P->profile_mask = mask;
  P->nevents_created = nevents;
  P->nrec = nrec;
  P->is_static = is_static;
  P->cfg = cfg;
  P->lay = lay;
  P->n = n;
  P->L = cfg.depth;
  P->p = cfg.p;
  P->nc = ncoef(cfg.p);
  P->mixed = cfg.precision == FMM_PREC_MIXED;
  P->m2l_np = m2l_pieces(cfg);
  P->m2l_f16 = m2l_is_f16(cfg);
  P->adaptive = cfg.leaf_max > 0;
  P->Ld = P->L;
  P->ws = ws;
  P->last_stream = s;
  P->rec = rec;
  hipError_t e = launch_tree(P, d_pos, s);
  if (e == hipSuccess && P->adaptive) e = launch_adaptive_tree(P, d_pos, s);
  if (e != hipSuccess) return FMM_E_DEVICE;
  if (P->adaptive && (P->nlist[0] > lay.ucap || P->nlist[1] > lay.wcap || P->nlist[2] > lay.xcap))
    return FMM_E_WORKSPACE;  // the tree's lists do not fit the workspace's list capacity
  if (P->adaptive && launch_p2p_worklist(P, s) != hipSuccess) return FMM_E_DEVICE;
  if (P->Ld >= 2 && !P->ops_ready) {
    if (launch_operators(P, s) != hipSuccess) return FMM_E_DEVICE;
    P->ops_ready = true;
  }
  return FMM_OK;
}

// Every pass of an evaluation of charges d_q (NULL: the stored sorted charges)
// and the outputs.
fmm_status evaluate_into(fmm_plan_s* P, const double* d_q, double* d_phi, double* d_force,
                         double* d_energy, hipStream_t s) {
  P->last_stream = s;
  hipError_t e = run_passes(P, d_q, s);
  if (e == hipSuccess)
    e = launch_near_and_finish(P, d_phi, d_force, d_energy, nullptr, nullptr, nullptr, s);
  if (e == hipSuccess) P->has_charges = true;
  return from_hip(e);
}

fmm_status validate_config_for(const fmm_config* cfg) { return validate_config(cfg); }

}  // namespace fmm

using namespace fmm;

extern "C" {

void fmm_config_default(fmm_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->abi_version = FMM_ABI_VERSION;
  cfg->p = 8;
  cfg->depth = 3;
  cfg->ws = 1;
  cfg->precision = FMM_PREC_FP64;
  cfg->m2l_kind = FMM_M2L_AUTO;
  cfg->root_side = 1.0;
}

fmm_status fmm_workspace_size(const fmm_config* cfg, int64_t n, size_t* bytes) {
  if (!bytes) return FMM_E_INVALID_ARG;
  fmm_status st = validate_config(cfg);
  if (st != FMM_OK) return st;
  if (n < 1 || n > INT32_MAX) return FMM_E_INVALID_ARG;
  Layout lay;
  make_layout(*cfg, n, &lay);
  *bytes = lay.total;
  return FMM_OK;
}

fmm_status fmm_plan(const fmm_config* cfg, int64_t n, const double* d_pos, void* d_workspace,
                    size_t workspace_bytes, fmm_stream_t stream, fmm_plan_t** out) {
  fmm_status st = validate_config(cfg);
  if (st != FMM_OK) return st;
  if (!out || !d_pos || n < 1 || n > INT32_MAX) return FMM_E_INVALID_ARG;
  if (!d_workspace || ((uintptr_t)d_workspace & 255u)) return FMM_E_WORKSPACE;
  Layout lay;
  make_layout(*cfg, n, &lay);
  if (workspace_bytes < lay.total) return FMM_E_WORKSPACE;

  fmm_plan_s* P = new (std::nothrow) fmm_plan_s;
  if (!P) return FMM_E_DEVICE;
  ProfileRec* rec = static_cast<ProfileRec*>(calloc(kMaxProfile, sizeof(ProfileRec)));
  if (!rec) {
    delete P;
    return FMM_E_DEVICE;
  }
  memset(P, 0, sizeof(*P));
  st = plan_into(P, *cfg, lay, n, d_pos, static_cast<char*>(d_workspace),
                 reinterpret_cast<hipStream_t>(stream), rec, false);
  if (st != FMM_OK) {
    free(rec);
    delete P;
    return st;
  }
  *out = P;
  return FMM_OK;
}

fmm_status fmm_plan_set_schedule(fmm_plan_t* P, int key, int value) {
  if (!P) return FMM_E_INVALID_ARG;
  switch (key) {
    case FMM_SCHED_P2P_PERSISTENT:
      if (value != 0 && value != 1) return FMM_E_INVALID_ARG;
      if (value && !P->adaptive) return FMM_E_UNSUPPORTED;
      P->p2p_persistent = value;
      return FMM_OK;
    case FMM_SCHED_M2L_SPLIT:
      if (value < 0 || value > kM2lSplitPerXcd) return FMM_E_INVALID_ARG;
      P->m2l_split = value;
      return FMM_OK;
    case FMM_SCHED_P2P_TILE:
      if (value != 128 && value != 256 && value != 512) return FMM_E_INVALID_ARG;
      P->p2p_tile = value;
      return FMM_OK;
    case FMM_SCHED_M2L_PERSISTENT:
      if (value != 0 && value != 1) return FMM_E_INVALID_ARG;
      if (value && !(P->m2l_f16 && m2l_f16_wide(P->p) && P->L >= 2)) return FMM_E_UNSUPPORTED;
      P->m2l_persistent = value;
      return FMM_OK;
  }
  return FMM_E_INVALID_ARG;
}

fmm_status fmm_replan(fmm_plan_t* P, const double* d_pos, fmm_stream_t stream) {
  if (!P || !d_pos) return FMM_E_INVALID_ARG;
  const fmm_config cfg = P->cfg;
  const Layout lay = P->lay;
  return plan_into(P, cfg, lay, P->n, d_pos, P->ws, reinterpret_cast<hipStream_t>(stream), P->rec,
                   true);
}

fmm_status fmm_evaluate(fmm_plan_t* P, const double* d_q, double* d_phi, double* d_force,
                        double* d_energy, fmm_stream_t stream) {
  if (!P || !d_q) return FMM_E_INVALID_ARG;
  return evaluate_into(P, d_q, d_phi, d_force, d_energy, reinterpret_cast<hipStream_t>(stream));
}

fmm_status fmm_backward(fmm_plan_t* P, const double* d_grad_energy, double* d_dE_dx,
                        double* d_dE_dq, fmm_stream_t stream) {
  if (!P || !d_grad_energy) return FMM_E_INVALID_ARG;
  if (!P->has_charges) return FMM_E_INVALID_ARG;  // no fmm_evaluate on this plan yet
  if (!d_dE_dx && !d_dE_dq) return FMM_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  P->last_stream = s;
  // Recompute every pass from the stored sorted charges (no expansion of the
  // forward call is reused), then write the scaled gradients.
  hipError_t e = run_passes(P, nullptr, s);
  if (e == hipSuccess)
    e = launch_near_and_finish(P, nullptr, nullptr, nullptr, d_grad_energy, d_dE_dq, d_dE_dx, s);
  return from_hip(e);
}

fmm_status fmm_check(fmm_plan_t* P) {
  if (!P) return FMM_E_INVALID_ARG;
  if (hipStreamSynchronize(P->last_stream) != hipSuccess) return FMM_E_DEVICE;
  int32_t flags = 0;
  if (hipMemcpy(&flags, P->ws + P->lay.flags, sizeof(flags), hipMemcpyDeviceToHost) != hipSuccess)
    return FMM_E_DEVICE;
  if (flags & kFlagNonFinite) return FMM_E_NONFINITE;
  if (flags & kFlagOutOfCube) return FMM_E_OUT_OF_CUBE;
  if (flags & kFlagCoincident) return FMM_E_COINCIDENT;
  if (flags & kFlagListOverflow) return FMM_E_WORKSPACE;
  return FMM_OK;
}

fmm_status fmm_destroy(fmm_plan_t* P) {
  if (!P) return FMM_OK;
  fmm_status st = FMM_OK;
  if (hipStreamSynchronize(P->last_stream) != hipSuccess) st = FMM_E_DEVICE;
  if (P->is_static) return st;  // the library's own plan of fmm_evaluate_static: kept
  for (int i = 0; i < P->nevents_created; ++i) {
    hipEventDestroy(P->rec[i].start);
    hipEventDestroy(P->rec[i].stop);
  }
  free(P->rec);
  delete P;
  return st;
}

const char* fmm_status_string(fmm_status st) {
  switch (st) {
    case FMM_OK: return "ok";
    case FMM_E_INVALID_ARG: return "invalid argument";
    case FMM_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case FMM_E_OUT_OF_CUBE: return "a position lies outside the given root cube";
    case FMM_E_NONFINITE: return "a coordinate is not finite";
    case FMM_E_COINCIDENT: return "two distinct particles share a position";
    case FMM_E_UNSUPPORTED: return "not supported by this build";
    case FMM_E_DEVICE: return "HIP runtime error";
  }
  return "unknown status";
}

fmm_status fmm_plan_leaves(fmm_plan_t* P, int32_t* d_cells, uint32_t* d_leaf, fmm_stream_t stream) {
  if (!P) return FMM_E_INVALID_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  P->last_stream = s;
  return from_hip(launch_leaves_out(P, d_cells, d_leaf, s));
}

fmm_status fmm_plan_cube(fmm_plan_t* P, double lo[3], double* side) {
  if (!P || !lo || !side) return FMM_E_INVALID_ARG;
  if (hipStreamSynchronize(P->last_stream) != hipSuccess) return FMM_E_DEVICE;
  DevParams dp;
  if (hipMemcpy(&dp, P->ws + P->lay.params, sizeof(dp), hipMemcpyDeviceToHost) != hipSuccess)
    return FMM_E_DEVICE;
  for (int a = 0; a < 3; ++a) lo[a] = dp.lo[a];
  *side = dp.side;
  return FMM_OK;
}

uint64_t fmm_hilbert_index(uint32_t ix, uint32_t iy, uint32_t iz, int32_t bits) {
  if (bits < 0 || bits > 21) return 0;
  if (bits < 32 && (ix >> bits || iy >> bits || iz >> bits)) return 0;
  return hilbert_index(ix, iy, iz, bits);
}

fmm_status fmm_profile_enable(fmm_plan_t* P, int phase_mask) {
  if (!P) return FMM_E_INVALID_ARG;
  if (!P->rec) return FMM_E_UNSUPPORTED;  // the plan of fmm_evaluate_static records nothing
  P->profile_mask = (uint32_t)phase_mask & ((1u << FMM_PHASE_COUNT) - 1u);
  P->prof_open = false;
  return FMM_OK;
}

fmm_status fmm_profile_read(fmm_plan_t* P, double ms[FMM_PHASE_COUNT],
                            int32_t launches[FMM_PHASE_COUNT]) {
  if (!P || !ms || !launches) return FMM_E_INVALID_ARG;
  for (int i = 0; i < FMM_PHASE_COUNT; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  fmm_status st = FMM_OK;
  for (int i = 0; i < P->nrec; ++i) {
    const ProfileRec& r = P->rec[i];
    if (hipEventSynchronize(r.stop) != hipSuccess) {
      st = FMM_E_DEVICE;
      break;
    }
    float t = 0.0f;
    if (hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) {
      st = FMM_E_DEVICE;
      break;
    }
    ms[r.phase] += t;
    launches[r.phase] += 1;
  }
  P->nrec = 0;
  return st;
}

fmm_status fmm_plan_tree_stats(fmm_plan_t* P, int64_t stats[FMM_TREE_STATS]) {
  if (!P || !stats) return FMM_E_INVALID_ARG;
  if (!P->adaptive) return FMM_E_UNSUPPORTED;
  hipStream_t s = P->last_stream;
  if (launch_adaptive_stats(P, s) != hipSuccess) return FMM_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return FMM_E_DEVICE;
  int64_t w[4];
  if (hipMemcpy(w, P->ws + P->lay.a_stats, sizeof(w), hipMemcpyDeviceToHost) != hipSuccess)
    return FMM_E_DEVICE;
  stats[0] = P->ce_off[P->L + 1];  // boxes
  stats[1] = w[0];                 // leaves
  stats[2] = P->Ld;                // deepest level
  stats[3] = P->nlist[0];          // U entries
  stats[4] = w[1];                 // V entries
  stats[5] = P->nlist[1];          // W entries
  stats[6] = P->nlist[2];          // X entries
  stats[7] = w[3] - P->n;          // ordered P2P pairs
  stats[8] = w[2];                 // M2L pairs of non-empty boxes
  return FMM_OK;
}

fmm_status fmm_plan_work(fmm_plan_t* P, int64_t* m2l_pairs, int64_t* p2p_pairs) {
  if (!P || !m2l_pairs || !p2p_pairs) return FMM_E_INVALID_ARG;
  if (P->adaptive) {
    int64_t st[FMM_TREE_STATS];
    fmm_status r = fmm_plan_tree_stats(P, st);
    if (r != FMM_OK) return r;
    *m2l_pairs = st[8];
    *p2p_pairs = st[7];
    return FMM_OK;
  }
  hipStream_t s = P->last_stream;
  if (launch_work_count(P, s) != hipSuccess) return FMM_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return FMM_E_DEVICE;
  int64_t w[2];
  if (hipMemcpy(w, P->ws + P->lay.work, sizeof(w), hipMemcpyDeviceToHost) != hipSuccess)
    return FMM_E_DEVICE;
  *m2l_pairs = w[0];
  *p2p_pairs = w[1];
  return FMM_OK;
}

}  // extern "C"
