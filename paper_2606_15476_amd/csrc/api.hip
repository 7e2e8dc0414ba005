// api.hip -- the C ABI (include/farm.h): argument checks, device memory
// ownership, metadata staging and the launch sequence of each entry point.
//
// Launch sequence of a scoring call (all on the caller's stream):
//   1. host metadata (classes, CSR relation offsets, predicates) is checked on
//      the host, written to a pinned staging block and copied to the device;
//   2. target and anchor vectors are L2-normalised into the workspace;
//   3. the similarity GEMM fills sim[q + R][n] (clamped cosine, class factor
//      on target rows);
//   4. the relational pass produces s(i) (and optionally t_r, b_r);
//   5. (fused path) TopK, then the ScoredCandidate breakdown of the winners.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <type_traits>

#include "farm_internal.h"

// Scratch of farm_query_topk_static (see include/farm.h): one copy per device,
// held until the process ends.  Host code never passes this name to a kernel
// or a copy -- on the host it is a stand-in, not a device address -- but the
// address hipGetSymbolAddress returns for the current device (static_scratch).
static __device__ __align__(256) unsigned char scratch[FARM_STATIC_SCRATCH_BYTES];

namespace farm {

static thread_local std::string g_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}

farm_status hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return FARM_ERR_HIP;
}

namespace {

template <class T>
farm_status dalloc(std::vector<void*>& allocs, size_t& bytes, T** p, size_t count, const char* what) {
  *p = nullptr;
  if (count == 0) count = 1;
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of %zu bytes for %s failed: %s", count * sizeof(T), what, hipGetErrorString(e));
    return FARM_ERR_OOM;
  }
  allocs.push_back(v);
  bytes += count * sizeof(T);
  *p = static_cast<T*>(v);
  return FARM_OK;
}

void free_all(std::vector<void*>& allocs) {
  for (void* p : allocs) (void)hipFree(p);
  allocs.clear();
}

#define FARM_TRY(expr)                  \
  do {                                  \
    farm_status st_ = (expr);           \
    if (st_ != FARM_OK) return st_;     \
  } while (0)

#define FARM_TRY_OR(expr, on_fail)      \
  do {                                  \
    farm_status st_ = (expr);           \
    if (st_ != FARM_OK) return on_fail(st_); \
  } while (0)

#define FARM_HIP(expr, what)                     \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Marks a workspace as inside a library call for the claim's lifetime; a
// second host thread that enters a call on the same workspace meanwhile is
// turned away with FARM_ERR_BUSY instead of racing on its host state.
struct WorkspaceClaim {
  farm_workspace* ws;
  bool ok;
  explicit WorkspaceClaim(farm_workspace* w) : ws(w), ok(!w || !w->in_call.exchange(true, std::memory_order_acquire)) {}
  ~WorkspaceClaim() {
    if (ws && ok) ws->in_call.store(false, std::memory_order_release);
  }
};

#define FARM_CLAIM(ws_)                                                                  \
  WorkspaceClaim claim_(ws_);                                                            \
  if (!claim_.ok) {                                                                      \
    set_error("workspace is in use by another call (one caller at a time)");             \
    return FARM_ERR_BUSY;                                                                \
  }

// The workspace's device buffers, in one place for the three ways a workspace
// is laid out: hipMalloc per buffer (farm_workspace_create), a byte count
// (farm_workspace_estimate) and bump allocation inside the library's static
// scratch array (farm_query_topk_static).  alloc(T** p, size_t count, const
// char* what) returns a farm_status.
template <class Alloc>
farm_status layout_workspace(farm_workspace* ws, const farm_memory* mem, int32_t max_q, int32_t max_rel,
                             int32_t max_k, Alloc&& alloc) {
  ws->mem = mem;
  ws->device = mem->device;
  ws->max_q = max_q;
  ws->max_rel = max_rel;
  ws->ld_s = round_up(mem->n, kRowAlign);
  const size_t rows = (size_t)max_q + (size_t)max_rel;
  const size_t rel1 = (size_t)(max_rel > 0 ? max_rel : 1);
  FARM_TRY(alloc(&ws->qn, rows * mem->ldk, "query vectors"));
  if (mem->dn_bf16) {
    FARM_TRY(alloc(&ws->qn_bf16, rows * mem->ldk, "BF16 query vectors"));
    FARM_TRY(alloc(&ws->qerr_bf16, rows, "BF16 query error norms"));
    FARM_TRY(alloc(&ws->qnrm_bf16, rows, "BF16 query norms"));
  }
  if (mem->dn_fp8) {
    FARM_TRY(alloc(&ws->qn_fp8, rows * mem->ldk, "FP8 query vectors"));
    FARM_TRY(alloc(&ws->qn_scale, rows, "FP8 query scales"));
    FARM_TRY(alloc(&ws->qerr_fp8, rows, "FP8 query error norms"));
    FARM_TRY(alloc(&ws->qnrm_fp8, rows, "FP8 query norms"));
  }
  FARM_TRY(alloc(&ws->sim, rows * ws->ld_s, "similarity matrix"));
  FARM_TRY(alloc(&ws->lsim, rel1 * ws->ld_s, "log similarities"));
  FARM_TRY(alloc(&ws->scores, (size_t)max_q * ws->ld_s, "scores"));
  if (mem->dn_bf16 || mem->dn_fp8) FARM_TRY(alloc(&ws->scores_hi, (size_t)max_q * ws->ld_s, "score bounds"));
  ws->meta_len = 2 * (int64_t)max_q + 1 + 3 * (int64_t)max_rel;
  FARM_TRY(alloc(&ws->d_meta, (size_t)ws->meta_len, "metadata"));
  FARM_TRY(alloc(&ws->status, 1, "status"));
  ws->cand_cap = topk_candidate_capacity(mem->n, max_q, max_k + 1);
  for (int b = 0; b < 2; ++b) {
    FARM_TRY(alloc(&ws->cand_key[b], (size_t)ws->cand_cap, "TopK keys"));
    FARM_TRY(alloc(&ws->cand_idx[b], (size_t)ws->cand_cap, "TopK indices"));
  }
  ws->max_k = max_k;
  ws->rs_cap = max_k > kBoundCap ? max_k : kBoundCap;
  const size_t nk = (size_t)max_q * ws->rs_cap;
  FARM_TRY(alloc(&ws->cand_count, (size_t)max_q, "candidate counts"));
  FARM_TRY(alloc(&ws->rs_idx, nk, "winner indices"));
  FARM_TRY(alloc(&ws->rs_score, nk, "rescored scores"));
  FARM_TRY(alloc(&ws->rs_terms, nk * kMaxRel, "rescored terms"));
  FARM_TRY(alloc(&ws->rs_anchor, nk * kMaxRel, "rescored anchors"));
  FARM_TRY(alloc(&ws->sem_idx, rel1 * kSemMax, "semantic sets"));
  FARM_TRY(alloc(&ws->sem_cnt, rel1, "semantic set sizes"));
  FARM_TRY(alloc(&ws->sem_tau, rel1, "semantic bounds"));
  FARM_TRY(alloc(&ws->sem_sim, rel1 * kSemMax, "semantic similarities"));
  FARM_TRY(alloc(&ws->btw_idx, rel1 * kBetweenSetSize, "Between candidate sets"));
  FARM_TRY(alloc(&ws->btw_sim, rel1 * kBetweenSetSize, "Between candidate similarities"));
  FARM_TRY(alloc(&ws->btw_cnt, rel1, "Between candidate counts"));
  FARM_TRY(alloc(&ws->prop_stats, 4, "proposal counters"));
  ws->fb_cap = fallback_cap(max_q);
  FARM_TRY(alloc(&ws->fb_list, (size_t)ws->fb_cap, "fallback worklist"));
  FARM_TRY(alloc(&ws->fb_count, 1, "fallback count"));
  return FARM_OK;
}

// Device bytes of a workspace of this shape (what farm_workspace_create allocates).
size_t workspace_bytes_for(const farm_memory* mem, int32_t max_q, int32_t max_rel, int32_t max_k) {
  farm_workspace tmp;
  size_t b = 0;
  (void)layout_workspace(&tmp, mem, max_q, max_rel, max_k, [&](auto** p, size_t count, const char*) {
    b += (count ? count : 1) * sizeof(**p);
    *p = nullptr;
    return FARM_OK;
  });
  return b;
}

// Relation rows whose terms k_scan_rows takes in the exhaustive method: the
// rank predicates, Inside, the entity-geometry predicates and the first slot
// of a Between invocation.
bool entity_geo_pred(int32_t p) { return p >= FARM_NEAR_HELLINGER && p <= FARM_BEHIND_VIEW; }
bool scanned_row(int32_t p) {
  return p == FARM_CLOSEST || p == FARM_FARTHEST || p == FARM_INSIDE || p == FARM_BETWEEN || entity_geo_pred(p);
}

farm_status check_meta(const farm_memory* mem, const farm_workspace* ws, int32_t q, const int32_t* rel_off,
                       const int32_t* rel_pred, int32_t* r_tot);

farm_status check_queries(const farm_memory* mem, const farm_workspace* ws, int32_t q, int32_t d,
                          const float* target, const int32_t* rel_off, const int32_t* rel_pred,
                          const float* rel_anchor, int32_t* r_tot) {
  if (!mem || !ws) { set_error("null memory or workspace"); return FARM_ERR_INVALID_ARG; }
  if (ws->mem != mem) { set_error("workspace was created for another memory"); return FARM_ERR_INVALID_ARG; }
  if (q < 0 || q > ws->max_q) { set_error("q = %d outside [0, %d]", q, ws->max_q); return FARM_ERR_INVALID_ARG; }
  if (d != mem->d) { set_error("query width %d != memory width %d", d, mem->d); return FARM_ERR_INVALID_ARG; }
  if (q > 0 && !target) { set_error("null target"); return FARM_ERR_INVALID_ARG; }
  FARM_TRY(check_meta(mem, ws, q, rel_off, rel_pred, r_tot));
  if (*r_tot > 0 && !rel_anchor) { set_error("null rel_anchor"); return FARM_ERR_INVALID_ARG; }
  return FARM_OK;
}

// The host metadata of a query batch: CSR offsets, predicate ids, Between
// pairing, the entity geometry the predicates need.  *r_tot: the relations.
farm_status check_meta(const farm_memory* mem, const farm_workspace* ws, int32_t q, const int32_t* rel_off,
                       const int32_t* rel_pred, int32_t* r_tot) {
  if (q > 0 && !rel_off) { set_error("null rel_off"); return FARM_ERR_INVALID_ARG; }
  if (q == 0) { *r_tot = 0; return FARM_OK; }
  if (rel_off[0] != 0) { set_error("rel_off[0] = %d, expected 0", rel_off[0]); return FARM_ERR_INVALID_ARG; }
  for (int32_t k = 0; k < q; ++k) {
    int32_t r = rel_off[k + 1] - rel_off[k];
    if (r < 0 || r > kMaxRel) {
      set_error("query %d has %d relations (allowed 0..%d)", k, r, kMaxRel);
      return FARM_ERR_INVALID_ARG;
    }
  }
  int32_t R = rel_off[q];
  if (R > ws->max_rel) { set_error("%d relations exceed the workspace's %d", R, ws->max_rel); return FARM_ERR_INVALID_ARG; }
  if (R > 0 && !rel_pred) { set_error("null rel_pred"); return FARM_ERR_INVALID_ARG; }
  for (int32_t r = 0; r < R; ++r)
    if (rel_pred[r] < 0 || rel_pred[r] >= FARM_NUM_PRED) {
      set_error("relation %d has predicate id %d", r, rel_pred[r]);
      return FARM_ERR_INVALID_ARG;
    }
  for (int32_t r = 0; r < R; ++r) {
    if (rel_pred[r] == FARM_NEAR_HELLINGER && !mem->cov) {
      set_error("relation %d (FARM_NEAR_HELLINGER) needs entity Gaussians (farm_set_entity_geometry)", r);
      return FARM_ERR_UNSUPPORTED;
    }
    if (rel_pred[r] >= FARM_LEFT_OF_VIEW && rel_pred[r] <= FARM_BEHIND_VIEW && !mem->view) {
      set_error("relation %d (predicate %d) needs stored views (farm_set_entity_geometry)", r, rel_pred[r]);
      return FARM_ERR_UNSUPPORTED;
    }
  }
  // a Between slot is followed by its second anchor's FARM_AND slot in the same query, and only there
  for (int32_t k = 0; k < q; ++k)
    for (int32_t r = rel_off[k]; r < rel_off[k + 1]; ++r) {
      if (rel_pred[r] == FARM_BETWEEN && (r + 1 >= rel_off[k + 1] || rel_pred[r + 1] != FARM_AND)) {
        set_error("relation %d (FARM_BETWEEN) is not followed by FARM_AND in its query", r);
        return FARM_ERR_INVALID_ARG;
      }
      if (rel_pred[r] == FARM_AND && (r == rel_off[k] || rel_pred[r - 1] != FARM_BETWEEN)) {
        set_error("relation %d (FARM_AND) does not follow a FARM_BETWEEN of its query", r);
        return FARM_ERR_INVALID_ARG;
      }
    }
  *r_tot = R;
  return FARM_OK;
}

bool has_between(const int32_t* rel_pred, int32_t R) {
  for (int32_t r = 0; r < R; ++r)
    if (rel_pred[r] == FARM_BETWEEN) return true;
  return false;
}

// Phase timer: brackets a phase with events on the call's stream when enabled.
struct PhaseTimer {
  farm_workspace* ws;
  hipStream_t s;
  int phase;
  hipEvent_t a = nullptr, b = nullptr;
  static hipEvent_t take(farm_workspace* w) {
    if (!w->ev_pool.empty()) {
      hipEvent_t e = w->ev_pool.back();
      w->ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  PhaseTimer(farm_workspace* w, hipStream_t st, int ph) : ws(w), s(st), phase(ph) {
    if (!ws->timing) return;
    a = take(ws);
    b = take(ws);
    if (a) (void)hipEventRecord(a, s);
  }
  ~PhaseTimer() {
    if (!ws->timing || !a || !b) return;
    (void)hipEventRecord(b, s);
    ws->pending.push_back({phase, a, b});
  }
};

// Stage the per-call metadata and return device views of it.
farm_status stage_meta(farm_workspace* ws, int32_t q, int32_t R, const int32_t* target_cls, const int32_t* rel_off,
                       const int32_t* rel_pred, hipStream_t s, MetaView* view) {
  if (ws->meta_pending) {
    FARM_HIP(hipEventSynchronize(ws->meta_done), "waiting for the previous metadata copy");
    ws->meta_pending = false;
  }
  int32_t* h = ws->h_meta;
  for (int32_t k = 0; k < q; ++k) h[k] = target_cls ? target_cls[k] : -1;
  memcpy(h + q, rel_off, sizeof(int32_t) * (size_t)(q + 1));
  if (R) memcpy(h + 2 * q + 1, rel_pred, sizeof(int32_t) * (size_t)R);
  int32_t* rq = h + 2 * q + 1 + R;
  for (int32_t k = 0; k < q; ++k)
    for (int32_t r = rel_off[k]; r < rel_off[k + 1]; ++r) rq[r] = k;
  int32_t* rk = h + 2 * q + 1 + 2 * R;  // rows of the scanned predicates (Closest, Farthest, Inside)
  int32_t nrank = 0, ngeo = 0;
  for (int32_t r = 0; r < R; ++r)
    if (scanned_row(rel_pred[r])) {
      rk[nrank++] = r;
      ngeo += entity_geo_pred(rel_pred[r]) ? 1 : 0;
    }
  size_t len = (size_t)(2 * q + 1 + 2 * R + nrank);
  FARM_HIP(hipMemcpyAsync(ws->d_meta, h, len * sizeof(int32_t), hipMemcpyHostToDevice, s), "metadata copy");
  FARM_HIP(hipEventRecord(ws->meta_done, s), "metadata event");
  ws->meta_pending = true;
  view->tcls = ws->d_meta;
  view->rel_off = ws->d_meta + q;
  view->rel_pred = ws->d_meta + 2 * q + 1;
  view->rel_query = ws->d_meta + 2 * q + 1 + R;
  view->scan_rows = ws->d_meta + 2 * q + 1 + 2 * R;
  view->scan_n = nrank;
  view->geo_n = ngeo;
  return FARM_OK;
}

// Error-bound accumulation term of a reduced-precision similarity: FP32
// accumulation of the GEMM and of the FP32 reference dot products (each at
// most ldk * 2^-24 for unit vectors), with margin for the normalisation.
float accumulation_bound(int32_t ldk) { return 2.02f * (float)ldk * 5.9604645e-8f + 1e-6f; }

// Steps 2 and 3: normalised query rows and the similarity matrix in `dtype`.
// need_log: also write lsim (the exhaustive relational pass stages it; the
// candidate methods take logarithms of the few similarities they gather).
farm_status similarity_tail(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t R, const MetaView& meta,
                            int32_t dtype, bool need_log, bool between, hipStream_t s);

farm_status similarities(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t R, const float* target,
                         const float* rel_anchor, const MetaView& meta, int32_t dtype, SimBound* bound,
                         bool need_log, bool between, hipStream_t s) {
  const int32_t ldk = mem->ldk;
  LowPrecRows lt, la;
  if (dtype == FARM_BF16) {
    lt.bf16 = ws->qn_bf16;
    lt.err_bf16 = ws->qerr_bf16;
    lt.nrm_bf16 = ws->qnrm_bf16;
  } else if (dtype == FARM_FP8_E4M3) {
    lt.fp8 = ws->qn_fp8;
    lt.fp8_scale = ws->qn_scale;
    lt.err_fp8 = ws->qerr_fp8;
    lt.nrm_fp8 = ws->qnrm_fp8;
  }
  la = lt;
  const int64_t off = (int64_t)q * ldk;
  if (la.bf16) la.bf16 += off;
  if (la.fp8) la.fp8 += off;
  if (la.fp8_scale) la.fp8_scale += q;
  if (la.err_bf16) { la.err_bf16 += q; la.nrm_bf16 += q; }
  if (la.err_fp8) { la.err_fp8 += q; la.nrm_fp8 += q; }
  {
    PhaseTimer t(ws, s, FARM_PHASE_NORMALIZE);
    FARM_HIP(launch_normalize_rows(target, q, mem->d, ldk, ws->qn, lt, ws->status, s), "normalize targets");
    FARM_HIP(launch_normalize_rows(rel_anchor, R, mem->d, ldk, ws->qn + off, la, ws->status, s),
             "normalize anchors");
  }
  PhaseTimer t(ws, s, FARM_PHASE_GEMM);
  *bound = SimBound{};
  const int64_t rows = (int64_t)q + R;
  if (dtype == FARM_F32) {
    FARM_HIP(launch_sim_gemm_f32(ws->qn, mem->dn, rows, mem->n, ldk, ws->sim, ws->ld_s, meta.tcls, q, mem->cls, s),
             "similarity GEMM");
  } else if (dtype == FARM_BF16) {
    FARM_HIP(launch_sim_gemm_bf16(ws->qn_bf16, mem->dn_bf16, rows, mem->n, ldk, ws->sim, ws->ld_s, meta.tcls, q,
                                  mem->cls, s),
             "BF16 similarity GEMM");
    *bound = SimBound{ws->qnrm_bf16, ws->qerr_bf16, mem->err_bf16, mem->err_max, accumulation_bound(ldk)};
  } else {
    FARM_HIP(launch_sim_gemm_fp8(ws->qn_fp8, ws->qn_scale, mem->dn_fp8, mem->dn_scale, rows, mem->n, ldk, ws->sim,
                                 ws->ld_s, meta.tcls, q, mem->cls, s),
             "FP8 similarity GEMM");
    *bound = SimBound{ws->qnrm_fp8, ws->qerr_fp8, mem->err_fp8, mem->err_max + 1, accumulation_bound(ldk)};
  }
  return similarity_tail(mem, ws, q, R, meta, dtype, need_log, between, s);
}

// What every form derives from the similarity rows: their logarithms (the
// exhaustive relational pass) and Between's candidate sets.
farm_status similarity_tail(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t R, const MetaView& meta,
                            int32_t dtype, bool need_log, bool between, hipStream_t s) {
  if (need_log)
    FARM_HIP(launch_log_rows(ws->sim + (int64_t)q * ws->ld_s, ws->ld_s, R, mem->n, ws->lsim, s), "log similarities");
  if (between) {
    // Between's rows exact in FP32 whatever the GEMM's dtype, then its candidate sets
    if (dtype != FARM_F32)
      FARM_HIP(launch_exact_rows(mem, ws->qn, ws->sim, ws->ld_s, q, meta, R, s), "Between exact rows");
    FARM_HIP(launch_between_sets(mem, ws->sim, ws->ld_s, q, meta, R, ws->btw_idx, ws->btw_sim, ws->btw_cnt, s),
             "Between candidate sets");
  }
  return FARM_OK;
}

// Options of the fused path, checked against the memory: dtype, method, flags
// and the number c of candidates that leave the first TopK (rescore_mult * k
// for the reduced-precision exhaustive form, else k).
struct TopkPlan {
  int32_t dtype = FARM_F32, method = FARM_METHOD_EXHAUSTIVE, opt_flags = 0, c = 0;
  int32_t* certified = nullptr;
  bool between = false;  // the batch has Between invocations
  bool presim = false;   // ws->sim already holds the unary rows (fused); only derive from them
};

farm_status plan_topk(const farm_memory* mem, const farm_score_opts* opts, int32_t k, TopkPlan* plan) {
  if (k < 1 || k > FARM_MAX_K) { set_error("k = %d outside [1, %d]", k, FARM_MAX_K); return FARM_ERR_INVALID_ARG; }
  const int32_t dtype = opts ? opts->dtype : FARM_F32;
  const int32_t method = opts ? opts->method : FARM_METHOD_EXHAUSTIVE;
  if (method != FARM_METHOD_EXHAUSTIVE && method != FARM_METHOD_BOUNDED && method != FARM_METHOD_PROPOSAL) {
    set_error("unknown method %d", method);
    return FARM_ERR_INVALID_ARG;
  }
  if (method == FARM_METHOD_PROPOSAL && mem->prop_m == 0 && mem->n >= 2) {
    set_error("method PROPOSAL needs farm_build_proposals on this memory");
    return FARM_ERR_UNSUPPORTED;
  }
  const int32_t opt_flags = opts ? opts->flags : 0;
  if (opt_flags & ~FARM_OPT_GLOBAL_PROPOSAL_PASS) {
    set_error("unknown option flags 0x%x", opt_flags);
    return FARM_ERR_INVALID_ARG;
  }
  if (dtype != FARM_F32 && dtype != FARM_BF16 && dtype != FARM_FP8_E4M3) {
    set_error("unknown dtype %d", dtype);
    return FARM_ERR_INVALID_ARG;
  }
  if ((dtype == FARM_BF16 && !mem->dn_bf16) || (dtype == FARM_FP8_E4M3 && !mem->dn_fp8)) {
    set_error("memory was built without the %s copy", dtype == FARM_BF16 ? "BF16" : "FP8");
    return FARM_ERR_UNSUPPORTED;
  }
  int32_t c = k;
  if (dtype != FARM_F32 && method == FARM_METHOD_EXHAUSTIVE) {
    const int32_t mult = opts->rescore_mult;
    if (mult < 1) { set_error("rescore_mult = %d must be >= 1", mult); return FARM_ERR_INVALID_ARG; }
    if ((int64_t)mult * k > FARM_MAX_K) {
      set_error("rescore_mult * k = %lld exceeds %d", (long long)mult * k, FARM_MAX_K);
      return FARM_ERR_INVALID_ARG;
    }
    c = mult * k;
  }
  plan->dtype = dtype;
  plan->method = method;
  plan->opt_flags = opt_flags;
  plan->c = c;
  plan->certified = opts ? opts->certified : nullptr;
  return FARM_OK;
}

// Steps 2-5 of the fused path once the metadata is on the device: shared by
// farm_query_topk (a created workspace) and farm_query_topk_static (a
// workspace laid out in the static scratch array).
farm_status query_topk_core(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t R, const float* target,
                            const float* rel_anchor, const MetaView& meta, const TopkPlan& plan, int32_t k,
                            uint32_t* out_id, float* out_score, float* out_terms, uint32_t* out_anchor_id,
                            hipStream_t s) {
  const int32_t dtype = plan.dtype, method = plan.method, opt_flags = plan.opt_flags, c = plan.c;
  int32_t* certified = plan.certified;
  SimBound bound;
  if (plan.presim)
    FARM_TRY(similarity_tail(mem, ws, q, R, meta, dtype, method == FARM_METHOD_EXHAUSTIVE, plan.between, s));
  else
    FARM_TRY(similarities(mem, ws, q, R, target, rel_anchor, meta, dtype, &bound, method == FARM_METHOD_EXHAUSTIVE,
                          plan.between, s));
  if (method == FARM_METHOD_BOUNDED || method == FARM_METHOD_PROPOSAL) {
    {
      PhaseTimer t(ws, s, FARM_PHASE_TOPK);
      FARM_HIP(launch_bound_candidates(mem, ws->sim, ws->ld_s, q, meta, bound, k, kBoundCap, ws->rs_idx,
                                       ws->cand_count, certified, s),
               "bound candidates");
    }
    PropView pv;
    pv.stats = ws->prop_stats;  // term and dot counters (full scans of BOUNDED too)
    if (method == FARM_METHOD_PROPOSAL && mem->prop_m > 0) {
      const bool in_lds = !(opt_flags & FARM_OPT_GLOBAL_PROPOSAL_PASS) && proposal_pass_in_lds(mem, dtype != FARM_F32);
      if (!in_lds) {
        // the LDS-staged pass selects the semantic sets itself; otherwise a scan per relation row
        PhaseTimer t(ws, s, FARM_PHASE_PROPOSE);
        FARM_HIP(launch_semantic_sets(ws->sim, ws->ld_s, q, R, mem->n, ws->sem_idx, ws->sem_cnt, ws->sem_tau, s),
                 "semantic sets");
        if (dtype != FARM_F32) FARM_HIP(launch_semantic_exact(mem, ws, q, R, s), "semantic similarities");
      }
      pv.m = mem->prop_m;
      pv.idx = mem->prop_idx;
      pv.val = mem->prop_val;
      pv.out = mem->prop_out;
      pv.sem_idx = ws->sem_idx;
      pv.sem_cnt = ws->sem_cnt;
      pv.sem_tau = ws->sem_tau;
      pv.sem_sim = dtype != FARM_F32 ? ws->sem_sim : nullptr;
      pv.stats = ws->prop_stats;
      pv.fb_list = ws->fb_list;
      pv.fb_count = ws->fb_count;
      pv.fb_cap = ws->fb_cap;
      pv.rel_total = R;
      pv.in_lds = in_lds;
      // the survivor queue suits BF16's error bound; FP8's leaves too many survivors per relation
      pv.queue = dtype == FARM_BF16;
      pv.sem_idx_out = ws->sem_idx;
      pv.sem_cnt_out = ws->sem_cnt;
      pv.sem_tau_out = ws->sem_tau;
      pv.sem_sim_out = ws->sem_sim;
    }
    {
      PhaseTimer t(ws, s, FARM_PHASE_RESCORE);
      FARM_HIP(launch_rescore_terms(mem, ws, ws->sim, ws->ld_s, q, meta, bound, ws->rs_idx, ws->cand_count,
                                    kBoundCap, pv, false, s),
               "candidate terms");
    }
    if (pv.m > 0) {
      PhaseTimer t(ws, s, FARM_PHASE_FALLBACK);
      FARM_HIP(launch_rescore_terms(mem, ws, ws->sim, ws->ld_s, q, meta, bound, ws->rs_idx, ws->cand_count,
                                    kBoundCap, pv, true, s),
               "fallback terms");
    }
    PhaseTimer t(ws, s, FARM_PHASE_SELECT);
    FARM_HIP(launch_rescore_combine(mem, ws, ws->sim, ws->ld_s, q, meta, bound, ws->rs_idx, ws->cand_count,
                                    kBoundCap, s),
             "candidate scores");
    FARM_HIP(launch_rescore_select(ws, q, kBoundCap, k, nullptr, nullptr, ws->cand_count, mem->n, out_id, out_score,
                                   out_terms, out_anchor_id, nullptr, s),
             "candidate select");
    return FARM_OK;
  }
  {
    PhaseTimer t(ws, s, FARM_PHASE_PAIR);
    FARM_HIP(launch_pair_exhaustive(mem, ws, ws->sim, ws->lsim, ws->ld_s, q, meta, bound, ws->scores, ws->ld_s, nullptr, nullptr,
                                    dtype == FARM_F32 ? nullptr : ws->scores_hi, s),
             "relational pass");
  }
  uint64_t* key;
  int32_t* idx;
  {
    PhaseTimer t(ws, s, FARM_PHASE_TOPK);
    FARM_HIP(launch_topk(mem, ws, ws->scores, ws->ld_s, q, c, &key, &idx, s), "topk");
    if (dtype == FARM_F32)
      FARM_HIP(launch_topk_emit(key, idx, q, k, out_id, out_score, ws->rs_idx, s), "topk emit");
    else
      FARM_HIP(launch_topk_emit(key, idx, q, c, nullptr, nullptr, ws->rs_idx, s), "candidate emit");
  }
  if (dtype == FARM_F32) {
    PhaseTimer t(ws, s, FARM_PHASE_EXPLAIN);
    FARM_HIP(launch_explain(mem, ws, ws->sim, ws->ld_s, q, meta, ws->rs_idx, k, out_terms, out_anchor_id, s), "explain");
    if (certified) FARM_HIP(launch_fill_i32(certified, q, 1, s), "certificate");
    return FARM_OK;
  }
  uint64_t* hi_key = nullptr;
  int32_t* hi_idx = nullptr;
  if (certified) {  // the c + 1 largest upper bounds (the first non-candidate among them bounds the rest)
    PhaseTimer t(ws, s, FARM_PHASE_TOPK);
    FARM_HIP(launch_topk(mem, ws, ws->scores_hi, ws->ld_s, q, c + 1, &hi_key, &hi_idx, s), "bound topk");
  }
  {
    PhaseTimer t(ws, s, FARM_PHASE_RESCORE);
    FARM_HIP(launch_rescore_terms(mem, ws, ws->sim, ws->ld_s, q, meta, bound, ws->rs_idx, nullptr, c, PropView{},
                                  false, s),
             "rescore terms");
  }
  PhaseTimer t(ws, s, FARM_PHASE_SELECT);
  FARM_HIP(launch_rescore_combine(mem, ws, ws->sim, ws->ld_s, q, meta, bound, ws->rs_idx, nullptr, c, s),
           "rescore scores");
  FARM_HIP(launch_rescore_select(ws, q, c, k, hi_key, hi_idx, nullptr, mem->n, out_id, out_score, out_terms,
                                 out_anchor_id, certified, s),
           "rescore select");
  return FARM_OK;
}

// ---- farm_query_topk_static: the workspace laid out in a static device array.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// ---- reciprocal-rank fusion of the unary scores (farm_query_topk_rrf)
constexpr int32_t kMaxAddedSpaces = 7;
constexpr int32_t kMaxChannels = 8;
constexpr int32_t kRrfMaxBlocks = 1024;

struct SpaceView {
  int32_t d = 0, ldk = 0;
  const float* dn = nullptr;
};

bool space_view(const farm_memory* mem, int32_t sp, SpaceView* v) {
  if (sp == 0) {
    *v = SpaceView{mem->d, mem->ldk, mem->dn};
    return true;
  }
  if (sp < 0 || sp > (int32_t)mem->spaces.size()) return false;
  const farm_memory::Space& e = mem->spaces[(size_t)sp - 1];
  *v = SpaceView{e.d, e.ldk, e.dn};
  return true;
}

farm_status check_channels(const farm_memory* mem, int32_t q, int32_t R, int32_t nch, const farm_rrf_channel* ch) {
  if (nch < 1 || nch > kMaxChannels || !ch) {
    set_error("n_channels = %d outside [1, %d] or no channel array", nch, kMaxChannels);
    return FARM_ERR_INVALID_ARG;
  }
  for (int32_t c = 0; c < nch; ++c) {
    SpaceView v;
    if (!space_view(mem, ch[c].space, &v)) {
      set_error("channel %d names embedding space %d (the memory has %d)", c, ch[c].space, 1 + (int)mem->spaces.size());
      return FARM_ERR_INVALID_ARG;
    }
    if (!(ch[c].weight > 0.0f) || !std::isfinite(ch[c].weight)) {
      set_error("channel %d has weight %g (must be positive and finite)", c, (double)ch[c].weight);
      return FARM_ERR_INVALID_ARG;
    }
    if ((q > 0 && !ch[c].target) || (R > 0 && !ch[c].anchor)) {
      set_error("channel %d lacks its target or anchor vectors", c);
      return FARM_ERR_INVALID_ARG;
    }
  }
  return FARM_OK;
}

// The workspace's fusion buffers, sized for its shape and the memory's widest space.
farm_status ensure_rrf(const farm_memory* mem, farm_workspace* ws) {
  int32_t ldk = mem->ldk;
  for (const farm_memory::Space& e : mem->spaces) ldk = std::max(ldk, e.ldk);
  if (ws->rrf_cos && ws->rrf_ldk >= ldk) return FARM_OK;
  free_all(ws->rrf_allocs);
  ws->rrf_qn = ws->rrf_cos = ws->rrf_val = nullptr;
  ws->rrf_idx = nullptr;
  ws->rrf_ldk = ws->rrf_blocks = 0;
  const int64_t rows = (int64_t)ws->max_q + ws->max_rel;
  const int32_t blocks = (int32_t)std::min<int64_t>(rows, kRrfMaxBlocks);
  const int64_t n = std::max<int64_t>(mem->n, 1);
  size_t bytes = 0;
  farm_status st = dalloc(ws->rrf_allocs, bytes, &ws->rrf_qn, (size_t)(rows * ldk), "fusion query vectors");
  if (!st) st = dalloc(ws->rrf_allocs, bytes, &ws->rrf_cos, (size_t)(rows * ws->ld_s), "fusion cosines");
  if (!st) st = dalloc(ws->rrf_allocs, bytes, &ws->rrf_val, (size_t)(blocks * n), "ranking scratch");
  if (!st) st = dalloc(ws->rrf_allocs, bytes, &ws->rrf_idx, (size_t)(blocks * n), "ranking scratch");
  if (st) {
    free_all(ws->rrf_allocs);
    ws->rrf_qn = ws->rrf_cos = ws->rrf_val = nullptr;
    ws->rrf_idx = nullptr;
    return st;
  }
  ws->rrf_ldk = ldk;
  ws->rrf_blocks = blocks;
  ws->bytes += bytes;
  return FARM_OK;
}

// ws->sim rows [q + R][n] := the fused unary scores of the channels (targets: with the class factor).
farm_status rrf_fuse(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t R, int32_t nch,
                     const farm_rrf_channel* ch, const MetaView& meta, hipStream_t s) {
  const int32_t rows = q + R;
  const int64_t n = mem->n;
  PhaseTimer t(ws, s, FARM_PHASE_GEMM);
  FARM_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(ws->sim), (int64_t)rows * ws->ld_s, 0, s), "fused rows clear");
  float total = 0.0f;
  for (int32_t c = 0; c < nch; ++c) {
    SpaceView v;
    space_view(mem, ch[c].space, &v);
    FARM_HIP(launch_normalize_rows(ch[c].target, q, v.d, v.ldk, ws->rrf_qn, LowPrecRows{}, ws->status, s),
             "normalize channel targets");
    FARM_HIP(launch_normalize_rows(ch[c].anchor, R, v.d, v.ldk, ws->rrf_qn + (int64_t)q * v.ldk, LowPrecRows{},
                                   ws->status, s),
             "normalize channel anchors");
    FARM_HIP(launch_gemm_nt_f32(ws->rrf_qn, v.dn, rows, n, v.ldk, ws->rrf_cos, ws->ld_s, s), "channel cosines");
    FARM_HIP(launch_rrf_rank(ws->rrf_cos, ws->ld_s, rows, n, mem->id, ch[c].weight, ws->sim, ws->rrf_val, ws->rrf_idx,
                             ws->rrf_blocks, s),
             "channel ranks");
    total += ch[c].weight;
  }
  // divided by the largest fused value sum(w) / (5 + 1)
  FARM_HIP(launch_rrf_finish(ws->sim, ws->ld_s, q, rows, n, meta.tcls, mem->cls, 6.0f / total, s), "fused rows");
  return FARM_OK;
}

// Shared checks and preparation of the two fusion entry points.
farm_status rrf_begin(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t nch, const farm_rrf_channel* ch,
                      const int32_t* rel_off, const int32_t* rel_pred, int32_t* R) {
  if (!mem || !ws) { set_error("null memory or workspace"); return FARM_ERR_INVALID_ARG; }
  if (ws->mem != mem) { set_error("workspace was created for another memory"); return FARM_ERR_INVALID_ARG; }
  if (q < 0 || q > ws->max_q) { set_error("q = %d outside [0, %d]", q, ws->max_q); return FARM_ERR_INVALID_ARG; }
  FARM_TRY(check_meta(mem, ws, q, rel_off, rel_pred, R));
  if (q == 0) return FARM_OK;
  return check_channels(mem, q, *R, nch, ch);
}

// Device address of `scratch` on `device`, which must be current: looked up
// once per device (hipGetSymbolAddress) and kept.
farm_status static_scratch(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device %d outside the %d the static scratch table covers", device, kMaxDevices);
    return FARM_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch address");
    g_scratch_ptr[device] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return FARM_OK;
}

// Per-call metadata of the static path travels in kernel arguments (no host
// staging buffer to allocate or keep alive): one launch per chunk.
constexpr int kMetaChunk = 248;
struct MetaChunk {
  int32_t off, cnt;
  int32_t v[kMetaChunk];
};

__global__ void k_meta_chunk(int32_t* __restrict__ dst, MetaChunk c) {
  for (int i = threadIdx.x; i < c.cnt; i += blockDim.x) dst[c.off + i] = c.v[i];
}

// The metadata block of stage_meta, written through kernel arguments.
farm_status stage_meta_args(farm_workspace* ws, int32_t q, int32_t R, const int32_t* target_cls,
                            const int32_t* rel_off, const int32_t* rel_pred, hipStream_t s, MetaView* view) {
  MetaChunk ch;
  ch.off = 0;
  ch.cnt = 0;
  hipError_t err = hipSuccess;
  auto flush = [&]() {
    if (ch.cnt == 0 || err != hipSuccess) return;
    hipLaunchKernelGGL(k_meta_chunk, dim3(1), dim3(256), 0, s, ws->d_meta, ch);
    err = hipGetLastError();
    ch.off += ch.cnt;
    ch.cnt = 0;
  };
  auto push = [&](int32_t v) {
    ch.v[ch.cnt++] = v;
    if (ch.cnt == kMetaChunk) flush();
  };
  for (int32_t k = 0; k < q; ++k) push(target_cls ? target_cls[k] : -1);
  for (int32_t k = 0; k <= q; ++k) push(rel_off[k]);
  for (int32_t r = 0; r < R; ++r) push(rel_pred[r]);
  for (int32_t k = 0; k < q; ++k)
    for (int32_t r = rel_off[k]; r < rel_off[k + 1]; ++r) push(k);
  int32_t nrank = 0, ngeo = 0;
  for (int32_t r = 0; r < R; ++r)
    if (scanned_row(rel_pred[r])) {
      push(r);
      ++nrank;
      ngeo += entity_geo_pred(rel_pred[r]) ? 1 : 0;
    }
  flush();
  if (err != hipSuccess) return hip_fail(err, "metadata launch");
  view->tcls = ws->d_meta;
  view->rel_off = ws->d_meta + q;
  view->rel_pred = ws->d_meta + 2 * q + 1;
  view->rel_query = ws->d_meta + 2 * q + 1 + R;
  view->scan_rows = ws->d_meta + 2 * q + 1 + 2 * R;
  view->scan_n = nrank;
  view->geo_n = ngeo;
  return FARM_OK;
}

}  // namespace
}  // namespace farm

using namespace farm;

extern "C" {

const char* farm_last_error(void) { return g_error.c_str(); }

const char* farm_version(void) { return "farm-mi355x 0.1 (gfx950)"; }

farm_status farm_build_memory(int64_t n, int32_t d, const float* desc, const float* center, const float* extent,
                              const uint32_t* id, const int32_t* cls, float view_right_x, float view_right_y,
                              uint32_t flags, void* stream, farm_memory** out) {
  try {
    if (!out) { set_error("out is NULL"); return FARM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (n < 1 || n >= (int64_t(1) << 31)) { set_error("n = %lld outside [1, 2^31)", (long long)n); return FARM_ERR_INVALID_ARG; }
    if (d < 1 || d > 8192) { set_error("d = %d outside [1, 8192]", d); return FARM_ERR_INVALID_ARG; }
    if (!desc || !center || !extent || !id) { set_error("null input pointer"); return FARM_ERR_INVALID_ARG; }
    if (!std::isfinite(view_right_x) || !std::isfinite(view_right_y)) {
      set_error("viewer right vector is not finite");
      return FARM_ERR_INVALID_ARG;
    }
    if (flags & ~(FARM_BUILD_BF16 | FARM_BUILD_FP8)) { set_error("unknown build flags 0x%x", flags); return FARM_ERR_INVALID_ARG; }
    hipStream_t s = (hipStream_t)stream;
    int device = 0;
    FARM_HIP(hipGetDevice(&device), "hipGetDevice");
    auto* mem = new (std::nothrow) farm_memory();
    if (!mem) { set_error("host allocation failed"); return FARM_ERR_OOM; }
    mem->device = device;
    mem->n = n;
    mem->d = d;
    mem->ldk = (int32_t)round_up(d, kKPad);
    mem->flags = flags;
    mem->rx = view_right_x;
    mem->ry = view_right_y;
    auto fail = [&](farm_status st) {
      (void)hipStreamSynchronize(s);
      free_all(mem->allocs);
      delete mem;
      return st;
    };
    farm_status st = FARM_OK;
    const size_t nn = (size_t)n;
    if ((st = dalloc(mem->allocs, mem->bytes, &mem->dn, nn * mem->ldk, "descriptors"))) return fail(st);
    if (flags & FARM_BUILD_BF16) {
      if ((st = dalloc(mem->allocs, mem->bytes, &mem->dn_bf16, nn * mem->ldk, "BF16 descriptors"))) return fail(st);
      if ((st = dalloc(mem->allocs, mem->bytes, &mem->err_bf16, nn, "BF16 error norms"))) return fail(st);
      if ((st = dalloc(mem->allocs, mem->bytes, &mem->nrm_bf16, nn, "BF16 norms"))) return fail(st);
    }
    if (flags & FARM_BUILD_FP8) {
      if ((st = dalloc(mem->allocs, mem->bytes, &mem->dn_fp8, nn * mem->ldk, "FP8 descriptors"))) return fail(st);
      if ((st = dalloc(mem->allocs, mem->bytes, &mem->dn_scale, nn, "FP8 scales"))) return fail(st);
      if ((st = dalloc(mem->allocs, mem->bytes, &mem->err_fp8, nn, "FP8 error norms"))) return fail(st);
      if ((st = dalloc(mem->allocs, mem->bytes, &mem->nrm_fp8, nn, "FP8 norms"))) return fail(st);
    }
    if ((st = dalloc(mem->allocs, mem->bytes, &mem->err_max, 2, "error maxima"))) return fail(st);
    if ((st = dalloc(mem->allocs, mem->bytes, &mem->x, nn, "x"))) return fail(st);
    if ((st = dalloc(mem->allocs, mem->bytes, &mem->y, nn, "y"))) return fail(st);
    if ((st = dalloc(mem->allocs, mem->bytes, &mem->z, nn, "z"))) return fail(st);
    if ((st = dalloc(mem->allocs, mem->bytes, &mem->hr_hi, 2 * nn, "lateral/depth hi"))) return fail(st);
    if ((st = dalloc(mem->allocs, mem->bytes, &mem->hr_lo, 2 * nn, "lateral/depth lo"))) return fail(st);
    if ((st = dalloc(mem->allocs, mem->bytes, &mem->ext, nn * 3, "extents"))) return fail(st);
    if ((st = dalloc(mem->allocs, mem->bytes, &mem->vz, 2 * nn, "bottom/top faces"))) return fail(st);
    if ((st = dalloc(mem->allocs, mem->bytes, &mem->id, nn, "ids"))) return fail(st);
    if (cls)
      if ((st = dalloc(mem->allocs, mem->bytes, &mem->cls, nn, "classes"))) return fail(st);

    // validation scratch: flags + id hash table (freed before returning)
    std::vector<void*> tmp;
    size_t tmp_bytes = 0;
    int* d_flags = nullptr;
    uint32_t* table = nullptr;
    int64_t tsize = 2;
    while (tsize < 2 * n) tsize <<= 1;
    if ((st = dalloc(tmp, tmp_bytes, &d_flags, 1, "validation flags"))) return fail(st);
    if ((st = dalloc(tmp, tmp_bytes, &table, (size_t)tsize, "id table"))) { free_all(tmp); return fail(st); }
    auto fail_tmp = [&](farm_status st2) { (void)hipStreamSynchronize(s); free_all(tmp); return fail(st2); };
    hipError_t e;
    if ((e = hipMemsetAsync(d_flags, 0, sizeof(int), s)) != hipSuccess) return fail_tmp(hip_fail(e, "memset"));
    if ((e = launch_validate_memory(desc, center, extent, id, n, d, d_flags, table, tsize, s)) != hipSuccess)
      return fail_tmp(hip_fail(e, "validate"));
    LowPrecRows lp;
    lp.bf16 = mem->dn_bf16;
    lp.err_bf16 = mem->err_bf16;
    lp.nrm_bf16 = mem->nrm_bf16;
    lp.fp8 = mem->dn_fp8;
    lp.fp8_scale = mem->dn_scale;
    lp.err_fp8 = mem->err_fp8;
    lp.nrm_fp8 = mem->nrm_fp8;
    if ((e = launch_normalize_rows(desc, n, d, mem->ldk, mem->dn, lp, d_flags, s)) != hipSuccess)
      return fail_tmp(hip_fail(e, "normalize descriptors"));
    if (mem->err_bf16 && (e = launch_max_reduce(mem->err_bf16, n, mem->err_max, s)) != hipSuccess)
      return fail_tmp(hip_fail(e, "error maximum"));
    if (mem->err_fp8 && (e = launch_max_reduce(mem->err_fp8, n, mem->err_max + 1, s)) != hipSuccess)
      return fail_tmp(hip_fail(e, "error maximum"));
    if ((e = launch_geometry(center, extent, n, view_right_x, view_right_y, mem->vz, mem->x, mem->y, mem->z,
                             mem->hr_hi, mem->hr_lo, mem->ext, s)) != hipSuccess)
      return fail_tmp(hip_fail(e, "geometry"));
    if ((e = hipMemcpyAsync(mem->id, id, nn * sizeof(uint32_t), hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return fail_tmp(hip_fail(e, "copy ids"));
    if (cls && (e = hipMemcpyAsync(mem->cls, cls, nn * sizeof(int32_t), hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return fail_tmp(hip_fail(e, "copy classes"));
    int h_flags = 0;
    if ((e = hipMemcpyAsync(&h_flags, d_flags, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return fail_tmp(hip_fail(e, "read flags"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_tmp(hip_fail(e, "build synchronize"));
    free_all(tmp);
    if (!h_flags && cls && n > 0) {
      // class order (host sort of n ints, once per memory)
      std::vector<int32_t> hc((size_t)n), order((size_t)n);
      if ((e = hipMemcpy(hc.data(), mem->cls, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost)) != hipSuccess)
        return fail(hip_fail(e, "read classes"));
      for (int64_t i = 0; i < n; ++i) order[(size_t)i] = (int32_t)i;
      std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return hc[a] < hc[b]; });
      std::vector<int32_t> sorted((size_t)n);
      for (int64_t i = 0; i < n; ++i) sorted[(size_t)i] = hc[order[(size_t)i]];
      if ((st = dalloc(mem->allocs, mem->bytes, &mem->cls_order, nn, "class order"))) return fail(st);
      if ((st = dalloc(mem->allocs, mem->bytes, &mem->cls_sorted, nn, "sorted classes"))) return fail(st);
      if ((e = hipMemcpy(mem->cls_order, order.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice)) !=
              hipSuccess ||
          (e = hipMemcpy(mem->cls_sorted, sorted.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice)) !=
              hipSuccess)
        return fail(hip_fail(e, "class order"));
    }
    if (h_flags) {
      set_error("invalid scene:%s%s%s%s%s%s", (h_flags & kBadDesc) ? " non-finite descriptor;" : "",
                (h_flags & kZeroNorm) ? " zero-norm descriptor;" : "",
                (h_flags & kBadCenter) ? " non-finite center;" : "",
                (h_flags & kBadExtent) ? " non-positive or non-finite extent;" : "",
                (h_flags & kBadId) ? " reserved id 0xFFFFFFFF;" : "", (h_flags & kDupId) ? " duplicate id;" : "");
      return fail(FARM_ERR_INVALID_ARG);
    }
    *out = mem;
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_build_memory");
    return FARM_ERR_OOM;
  }
}

farm_status farm_set_entity_geometry(farm_memory* mem, const float* cov, const float* view, void* stream) {
  try {
    if (!mem) { set_error("null memory"); return FARM_ERR_INVALID_ARG; }
    if (!cov && !view) return FARM_OK;
    DeviceGuard g(mem->device);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = mem->n;
    std::vector<void*> cov_allocs, view_allocs, tmp;
    size_t cov_bytes = 0, view_bytes = 0, tmp_bytes = 0;
    float* c = nullptr;
    double* ld = nullptr;
    float* v = nullptr;
    int* flags = nullptr;
    auto fail = [&](farm_status st) {
      free_all(cov_allocs);
      free_all(view_allocs);
      free_all(tmp);
      return st;
    };
    if (cov) {
      FARM_TRY_OR(dalloc(cov_allocs, cov_bytes, &c, (size_t)n * 6, "entity covariances"), fail);
      FARM_TRY_OR(dalloc(cov_allocs, cov_bytes, &ld, (size_t)n, "covariance log determinants"), fail);
    }
    if (view) FARM_TRY_OR(dalloc(view_allocs, view_bytes, &v, (size_t)n * 12, "stored views"), fail);
    FARM_TRY_OR(dalloc(tmp, tmp_bytes, &flags, 2, "validation flags"), fail);
    hipError_t e = launch_fill_i32(flags, 1, 0, s);
    if (e == hipSuccess) e = launch_fill_i32(flags + 1, 1, INT32_MAX, s);
    if (e == hipSuccess) e = launch_entity_geometry(cov, view, n, c, ld, v, flags, flags + 1, s);
    int h[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(hip_fail(e, "entity geometry"));
    if (h[0]) {
      set_error("invalid entity geometry at object %d:%s%s", h[1],
                (h[0] & kBadCov) ? " covariance not finite or not positive definite;" : "",
                (h[0] & kBadView) ? " view not finite or its rotation rows not orthonormal;" : "");
      return fail(FARM_ERR_INVALID_ARG);
    }
    free_all(tmp);
    if (cov) {
      mem->bytes -= std::min(mem->bytes, (size_t)n * (6 * sizeof(float) + sizeof(double)) * (mem->cov ? 1 : 0));
      free_all(mem->cov_allocs);
      mem->cov_allocs = cov_allocs;
      mem->cov = c;
      mem->cov_ld = ld;
      mem->bytes += cov_bytes;
    }
    if (view) {
      mem->bytes -= std::min(mem->bytes, (size_t)n * 12 * sizeof(float) * (mem->view ? 1 : 0));
      free_all(mem->view_allocs);
      mem->view_allocs = view_allocs;
      mem->view = v;
      mem->bytes += view_bytes;
    }
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_set_entity_geometry");
    return FARM_ERR_OOM;
  }
}

farm_status farm_free_memory(farm_memory* mem) {
  if (!mem) return FARM_OK;
  if (const int32_t u = mem->users.load(std::memory_order_acquire)) {
    set_error("memory still has %d workspace(s) or server registration(s); free those first", u);
    return FARM_ERR_BUSY;
  }
  DeviceGuard g(mem->device);
  (void)hipDeviceSynchronize();
  free_all(mem->allocs);
  free_all(mem->prop_allocs);
  free_all(mem->cov_allocs);
  free_all(mem->view_allocs);
  free_all(mem->space_allocs);
  delete mem;
  return FARM_OK;
}

farm_status farm_memory_info(const farm_memory* mem, int64_t* n, int32_t* d, size_t* bytes) {
  if (!mem) { set_error("null memory"); return FARM_ERR_INVALID_ARG; }
  if (n) *n = mem->n;
  if (d) *d = mem->d;
  if (bytes) *bytes = mem->bytes;
  return FARM_OK;
}

farm_status farm_workspace_estimate(const farm_memory* mem, int32_t max_q, int32_t max_rel, int32_t max_k,
                                    size_t* bytes) {
  if (!mem || !bytes || max_q < 1 || max_rel < 0 || max_k < 1 || max_k > FARM_MAX_K) {
    set_error("invalid workspace shape");
    return FARM_ERR_INVALID_ARG;
  }
  *bytes = workspace_bytes_for(mem, max_q, max_rel, max_k);
  return FARM_OK;
}

farm_status farm_workspace_create(const farm_memory* mem, int32_t max_q, int32_t max_rel, int32_t max_k,
                                  farm_workspace** out) {
  try {
    if (!out) { set_error("out is NULL"); return FARM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (!mem || max_q < 1 || max_rel < 0 || max_k < 1 || max_k > FARM_MAX_K) {
      set_error("invalid workspace shape (max_q %d, max_rel %d, max_k %d)", max_q, max_rel, max_k);
      return FARM_ERR_INVALID_ARG;
    }
    DeviceGuard g(mem->device);
    auto* ws = new (std::nothrow) farm_workspace();
    if (!ws) { set_error("host allocation failed"); return FARM_ERR_OOM; }
    auto fail = [&](farm_status st) {
      free_all(ws->allocs);
      if (ws->h_meta) (void)hipHostFree(ws->h_meta);
      if (ws->meta_done) (void)hipEventDestroy(ws->meta_done);
      delete ws;
      return st;
    };
    farm_status st = layout_workspace(ws, mem, max_q, max_rel, max_k, [&](auto** p, size_t count, const char* what) {
      return dalloc(ws->allocs, ws->bytes, p, count, what);
    });
    if (st) return fail(st);
    hipError_t e = hipHostMalloc((void**)&ws->h_meta, (size_t)ws->meta_len * sizeof(int32_t), hipHostMallocDefault);
    if (e != hipSuccess) { ws->h_meta = nullptr; return fail(hip_fail(e, "pinned metadata staging")); }
    e = hipEventCreateWithFlags(&ws->meta_done, hipEventDisableTiming);
    if (e != hipSuccess) { ws->meta_done = nullptr; return fail(hip_fail(e, "event")); }
    e = hipMemset(ws->status, 0, sizeof(int));
    if (e != hipSuccess) return fail(hip_fail(e, "status clear"));
    e = hipMemset(ws->prop_stats, 0, 4 * sizeof(unsigned long long));
    if (e != hipSuccess) return fail(hip_fail(e, "counter clear"));
    mem->users.fetch_add(1, std::memory_order_acq_rel);
    *out = ws;
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_workspace_create");
    return FARM_ERR_OOM;
  }
}

farm_status farm_workspace_set_timing(farm_workspace* ws, int32_t enable) {
  if (!ws) { set_error("null workspace"); return FARM_ERR_INVALID_ARG; }
  FARM_CLAIM(ws);
  ws->timing = enable != 0;
  return FARM_OK;
}

farm_status farm_workspace_timings(farm_workspace* ws, double* ms, int64_t* count, int32_t reset) {
  if (!ws) { set_error("null workspace"); return FARM_ERR_INVALID_ARG; }
  FARM_CLAIM(ws);
  DeviceGuard g(ws->device);
  for (auto& p : ws->pending) {
    FARM_HIP(hipEventSynchronize(p.b), "timer synchronize");
    float t = 0.f;
    FARM_HIP(hipEventElapsedTime(&t, p.a, p.b), "timer elapsed");
    ws->phase_ms[p.phase] += t;
    ws->phase_count[p.phase] += 1;
    ws->ev_pool.push_back(p.a);
    ws->ev_pool.push_back(p.b);
  }
  ws->pending.clear();
  for (int i = 0; i < FARM_PHASE_COUNT; ++i) {
    if (ms) ms[i] = ws->phase_ms[i];
    if (count) count[i] = ws->phase_count[i];
    if (reset) {
      ws->phase_ms[i] = 0;
      ws->phase_count[i] = 0;
    }
  }
  return FARM_OK;
}

farm_status farm_workspace_free(farm_workspace* ws) {
  if (!ws) return FARM_OK;
  if (ws->in_call.load(std::memory_order_acquire)) {
    set_error("workspace is in use by another call");
    return FARM_ERR_BUSY;
  }
  ws->mem->users.fetch_sub(1, std::memory_order_acq_rel);
  DeviceGuard g(ws->device);
  (void)hipDeviceSynchronize();
  for (auto& p : ws->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : ws->ev_pool) (void)hipEventDestroy(e);
  free_all(ws->allocs);
  free_all(ws->rrf_allocs);
  if (ws->h_meta) (void)hipHostFree(ws->h_meta);
  if (ws->meta_done) (void)hipEventDestroy(ws->meta_done);
  delete ws;
  return FARM_OK;
}

farm_status farm_workspace_bytes(const farm_workspace* ws, size_t* bytes) {
  if (!ws || !bytes) { set_error("null argument"); return FARM_ERR_INVALID_ARG; }
  *bytes = ws->bytes;
  return FARM_OK;
}

farm_status farm_proposal_pass_form(const farm_memory* mem, int32_t dtype, int32_t* in_lds) {
  if (!mem || !in_lds) { set_error("null memory or output"); return FARM_ERR_INVALID_ARG; }
  DeviceGuard g(mem->device);
  *in_lds = proposal_pass_in_lds(mem, dtype != FARM_F32) ? 1 : 0;
  return FARM_OK;
}

farm_status farm_workspace_proposal_stats(farm_workspace* ws, int64_t* stats, int32_t reset, void* stream) {
  if (!ws || !stats) { set_error("null workspace or output"); return FARM_ERR_INVALID_ARG; }
  FARM_CLAIM(ws);
  DeviceGuard g(ws->device);
  hipStream_t s = (hipStream_t)stream;
  unsigned long long h[4] = {0, 0, 0, 0};
  FARM_HIP(hipMemcpyAsync(h, ws->prop_stats, sizeof(h), hipMemcpyDeviceToHost, s), "read counters");
  FARM_HIP(hipStreamSynchronize(s), "counter synchronize");
  for (int i = 0; i < 4; ++i) stats[i] = (int64_t)h[i];
  if (reset) {
    FARM_HIP(hipMemsetAsync(ws->prop_stats, 0, sizeof(h), s), "counter clear");
    FARM_HIP(hipStreamSynchronize(s), "counter synchronize");
  }
  return FARM_OK;
}

farm_status farm_workspace_status(farm_workspace* ws, void* stream) {
  if (!ws) { set_error("null workspace"); return FARM_ERR_INVALID_ARG; }
  FARM_CLAIM(ws);
  DeviceGuard g(ws->device);
  hipStream_t s = (hipStream_t)stream;
  int h = 0;
  FARM_HIP(hipMemcpyAsync(&h, ws->status, sizeof(int), hipMemcpyDeviceToHost, s), "read status");
  FARM_HIP(hipStreamSynchronize(s), "status synchronize");
  if (h) {
    FARM_HIP(hipMemsetAsync(ws->status, 0, sizeof(int), s), "status clear");
    FARM_HIP(hipStreamSynchronize(s), "status synchronize");
    set_error("a scoring call saw a%s%s query vector", (h & kBadDesc) ? " non-finite" : "",
              (h & kZeroNorm) ? " zero-norm" : "");
    return FARM_ERR_INVALID_ARG;
  }
  return FARM_OK;
}

farm_status farm_score_query(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t d, const float* target,
                             const int32_t* target_cls, const int32_t* rel_off, const int32_t* rel_pred,
                             const float* rel_anchor, float* scores, float* rel_terms, uint32_t* rel_anchor_id,
                             void* stream) {
  try {
    FARM_CLAIM(ws);
    int32_t R = 0;
    FARM_TRY(check_queries(mem, ws, q, d, target, rel_off, rel_pred, rel_anchor, &R));
    if (q > 0 && !scores) { set_error("scores is NULL"); return FARM_ERR_INVALID_ARG; }
    if (q == 0) return FARM_OK;
    DeviceGuard g(mem->device);
    hipStream_t s = (hipStream_t)stream;
    MetaView meta;
    FARM_TRY(stage_meta(ws, q, R, target_cls, rel_off, rel_pred, s, &meta));
    SimBound none;
    FARM_TRY(similarities(mem, ws, q, R, target, rel_anchor, meta, FARM_F32, &none, true, has_between(rel_pred, R), s));
    PhaseTimer t(ws, s, FARM_PHASE_PAIR);
    FARM_HIP(launch_pair_exhaustive(mem, ws, ws->sim, ws->lsim, ws->ld_s, q, meta, none, scores, mem->n, rel_terms, rel_anchor_id,
                                    nullptr, s),
             "relational pass");
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_score_query");
    return FARM_ERR_HIP;
  }
}

farm_status farm_similarity(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t d, const float* target,
                            const int32_t* target_cls, int32_t dtype, float* out, void* stream) {
  try {
    FARM_CLAIM(ws);
    if (dtype != FARM_F32 && dtype != FARM_BF16 && dtype != FARM_FP8_E4M3) {
      set_error("unknown dtype %d", dtype);
      return FARM_ERR_INVALID_ARG;
    }
    std::vector<int32_t> rel_off((size_t)std::max(q, 0) + 1, 0);
    int32_t R = 0;
    FARM_TRY(check_queries(mem, ws, q, d, target, rel_off.data(), nullptr, nullptr, &R));
    if (q == 0) return FARM_OK;
    if (!out) { set_error("out is NULL"); return FARM_ERR_INVALID_ARG; }
    if ((dtype == FARM_BF16 && !mem->dn_bf16) || (dtype == FARM_FP8_E4M3 && !mem->dn_fp8)) {
      set_error("the memory was built without the %s copy", dtype == FARM_BF16 ? "BF16" : "FP8");
      return FARM_ERR_UNSUPPORTED;
    }
    DeviceGuard g(mem->device);
    hipStream_t s = (hipStream_t)stream;
    MetaView meta;
    FARM_TRY(stage_meta(ws, q, 0, target_cls, rel_off.data(), nullptr, s, &meta));
    SimBound bound;
    FARM_TRY(similarities(mem, ws, q, 0, target, nullptr, meta, dtype, &bound, false, false, s));
    FARM_HIP(hipMemcpy2DAsync(out, (size_t)mem->n * sizeof(float), ws->sim, (size_t)ws->ld_s * sizeof(float),
                              (size_t)mem->n * sizeof(float), (size_t)q, hipMemcpyDeviceToDevice, s),
             "similarity copy");
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_similarity");
    return FARM_ERR_HIP;
  }
}

farm_status farm_topk(const farm_memory* mem, farm_workspace* ws, const float* scores, int32_t q, int32_t k,
                      uint32_t* out_id, float* out_score, int32_t* out_index, void* stream) {
  try {
    FARM_CLAIM(ws);
    if (!mem || !ws || ws->mem != mem) { set_error("null or mismatched memory/workspace"); return FARM_ERR_INVALID_ARG; }
    if (q < 0 || q > ws->max_q) { set_error("q = %d outside [0, %d]", q, ws->max_q); return FARM_ERR_INVALID_ARG; }
    if (k < 1 || k > FARM_MAX_K) { set_error("k = %d outside [1, %d]", k, FARM_MAX_K); return FARM_ERR_INVALID_ARG; }
    if (q == 0) return FARM_OK;
    if (!scores || !out_id || !out_score) { set_error("null pointer"); return FARM_ERR_INVALID_ARG; }
    if (k > ws->max_k) { set_error("k = %d exceeds the workspace's max_k %d", k, ws->max_k); return FARM_ERR_INVALID_ARG; }
    DeviceGuard g(mem->device);
    hipStream_t s = (hipStream_t)stream;
    uint64_t* key;
    int32_t* idx;
    PhaseTimer t(ws, s, FARM_PHASE_TOPK);
    FARM_HIP(launch_topk(mem, ws, scores, mem->n, q, k, &key, &idx, s), "topk");
    FARM_HIP(launch_topk_emit(key, idx, q, k, out_id, out_score, out_index, s), "topk emit");
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_topk");
    return FARM_ERR_HIP;
  }
}

farm_status farm_query_topk(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t d, const float* target,
                            const int32_t* target_cls, const int32_t* rel_off, const int32_t* rel_pred,
                            const float* rel_anchor, const farm_score_opts* opts, int32_t k, uint32_t* out_id,
                            float* out_score, float* out_terms, uint32_t* out_anchor_id, void* stream) {
  try {
    FARM_CLAIM(ws);
    int32_t R = 0;
    FARM_TRY(check_queries(mem, ws, q, d, target, rel_off, rel_pred, rel_anchor, &R));
    TopkPlan plan;
    FARM_TRY(plan_topk(mem, opts, k, &plan));
    if (q == 0) return FARM_OK;
    plan.between = has_between(rel_pred, R);
    if (!out_id || !out_score) { set_error("null output pointer"); return FARM_ERR_INVALID_ARG; }
    if (plan.c > ws->max_k) {
      set_error("%s = %d exceeds the workspace's max_k %d", plan.c > k ? "rescore_mult * k" : "k", plan.c, ws->max_k);
      return FARM_ERR_INVALID_ARG;
    }
    DeviceGuard g(mem->device);
    hipStream_t s = (hipStream_t)stream;
    MetaView meta;
    FARM_TRY(stage_meta(ws, q, R, target_cls, rel_off, rel_pred, s, &meta));
    return query_topk_core(mem, ws, q, R, target, rel_anchor, meta, plan, k, out_id, out_score, out_terms,
                           out_anchor_id, s);
  } catch (...) {
    set_error("unexpected host exception in farm_query_topk");
    return FARM_ERR_HIP;
  }
}

farm_status farm_query_topk_static(const farm_memory* mem, int32_t q, int32_t d, const float* target,
                                   const int32_t* target_cls, const int32_t* rel_off, const int32_t* rel_pred,
                                   const float* rel_anchor, const farm_score_opts* opts, int32_t k, uint32_t* out_id,
                                   float* out_score, float* out_terms, uint32_t* out_anchor_id, void* stream) {
  try {
    if (!mem) { set_error("null memory"); return FARM_ERR_INVALID_ARG; }
    farm_workspace ws;  // host-side descriptor only: its buffers point into the static scratch
    ws.mem = mem;
    ws.max_q = q > 0 ? q : 0;
    ws.max_rel = INT32_MAX;
    int32_t R = 0;
    FARM_TRY(check_queries(mem, &ws, q, d, target, rel_off, rel_pred, rel_anchor, &R));
    TopkPlan plan;
    FARM_TRY(plan_topk(mem, opts, k, &plan));
    if (q == 0) return FARM_OK;
    plan.between = has_between(rel_pred, R);
    if (!out_id || !out_score) { set_error("null output pointer"); return FARM_ERR_INVALID_ARG; }
    DeviceGuard g(mem->device);
    if (!g.ok) { set_error("cannot make device %d current", mem->device); return FARM_ERR_HIP; }
    unsigned char* base = nullptr;
    FARM_TRY(static_scratch(mem->device, &base));
    size_t used = 0;
    farm_status st = layout_workspace(&ws, mem, q, R, plan.c, [&](auto** p, size_t count, const char*) {
      const size_t bytes = (count ? count : 1) * sizeof(**p);
      const size_t off = (size_t)round_up((int64_t)used, 256);
      used = off + bytes;
      *p = used <= FARM_STATIC_SCRATCH_BYTES ? reinterpret_cast<std::decay_t<decltype(*p)>>(base + off) : nullptr;
      return FARM_OK;
    });
    if (st) return st;
    if (used > FARM_STATIC_SCRATCH_BYTES) {
      set_error("farm_query_topk_static: q = %d, R = %d, k = %d over n = %lld objects needs %zu bytes of scratch; "
                "the static scratch holds %zu",
                q, R, plan.c, (long long)mem->n, used, (size_t)FARM_STATIC_SCRATCH_BYTES);
      return FARM_ERR_INVALID_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    // the array keeps the previous call's contents: clear the flags and counters
    // this call accumulates into (fill kernels, no memset nodes)
    FARM_HIP(launch_fill_i32(ws.status, 1, 0, s), "status clear");
    FARM_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(ws.prop_stats), 8, 0, s), "counter clear");
    MetaView meta;
    FARM_TRY(stage_meta_args(&ws, q, R, target_cls, rel_off, rel_pred, s, &meta));
    return query_topk_core(mem, &ws, q, R, target, rel_anchor, meta, plan, k, out_id, out_score, out_terms,
                           out_anchor_id, s);
  } catch (...) {
    set_error("unexpected host exception in farm_query_topk_static");
    return FARM_ERR_HIP;
  }
}

farm_status farm_add_embedding_space(farm_memory* mem, int32_t d, const float* desc, void* stream, int32_t* space_out) {
  try {
    if (!mem || !desc || !space_out) { set_error("null memory, descriptors or output"); return FARM_ERR_INVALID_ARG; }
    if (d < 1 || d > 8192) { set_error("width %d outside [1, 8192]", d); return FARM_ERR_INVALID_ARG; }
    if ((int32_t)mem->spaces.size() >= kMaxAddedSpaces) {
      set_error("the memory already holds %d added embedding spaces", kMaxAddedSpaces);
      return FARM_ERR_INVALID_ARG;
    }
    DeviceGuard g(mem->device);
    hipStream_t s = (hipStream_t)stream;
    farm_memory::Space sp;
    sp.d = d;
    sp.ldk = (int32_t)round_up(d, kKPad);
    std::vector<void*> allocs, tmp;
    size_t bytes = 0, tmp_bytes = 0;
    int* flags = nullptr;
    auto fail = [&](farm_status st) {
      free_all(allocs);
      free_all(tmp);
      return st;
    };
    FARM_TRY_OR(dalloc(allocs, bytes, &sp.dn, (size_t)(std::max<int64_t>(mem->n, 1) * sp.ldk), "embedding space"),
                fail);
    FARM_TRY_OR(dalloc(tmp, tmp_bytes, &flags, 1, "validation flag"), fail);
    hipError_t e = launch_fill_i32(flags, 1, 0, s);
    if (e == hipSuccess) e = launch_normalize_rows(desc, mem->n, d, sp.ldk, sp.dn, LowPrecRows{}, flags, s);
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flags, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(hip_fail(e, "embedding space"));
    if (h) {
      set_error("invalid embedding space:%s%s", (h & kBadDesc) ? " non-finite value;" : "",
                (h & kZeroNorm) ? " zero-norm row;" : "");
      return fail(FARM_ERR_INVALID_ARG);
    }
    free_all(tmp);
    mem->spaces.push_back(sp);
    mem->space_allocs.insert(mem->space_allocs.end(), allocs.begin(), allocs.end());
    mem->bytes += bytes;
    *space_out = (int32_t)mem->spaces.size();
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_add_embedding_space");
    return FARM_ERR_OOM;
  }
}

farm_status farm_rrf_similarity(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t n_channels,
                                const farm_rrf_channel* channels, const int32_t* target_cls, const int32_t* rel_off,
                                const int32_t* rel_pred, float* out, void* stream) {
  try {
    FARM_CLAIM(ws);
    int32_t R = 0;
    FARM_TRY(rrf_begin(mem, ws, q, n_channels, channels, rel_off, rel_pred, &R));
    if (q == 0) return FARM_OK;
    if (!out) { set_error("out is NULL"); return FARM_ERR_INVALID_ARG; }
    DeviceGuard g(mem->device);
    hipStream_t s = (hipStream_t)stream;
    FARM_TRY(ensure_rrf(mem, ws));
    MetaView meta;
    FARM_TRY(stage_meta(ws, q, R, target_cls, rel_off, rel_pred, s, &meta));
    FARM_TRY(rrf_fuse(mem, ws, q, R, n_channels, channels, meta, s));
    FARM_HIP(hipMemcpy2DAsync(out, (size_t)mem->n * sizeof(float), ws->sim, (size_t)ws->ld_s * sizeof(float),
                              (size_t)mem->n * sizeof(float), (size_t)(q + R), hipMemcpyDeviceToDevice, s),
             "fused rows copy");
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_rrf_similarity");
    return FARM_ERR_HIP;
  }
}

farm_status farm_query_topk_rrf(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t n_channels,
                                const farm_rrf_channel* channels, const int32_t* target_cls, const int32_t* rel_off,
                                const int32_t* rel_pred, const farm_score_opts* opts, int32_t k, uint32_t* out_id,
                                float* out_score, float* out_terms, uint32_t* out_anchor_id, void* stream) {
  try {
    FARM_CLAIM(ws);
    int32_t R = 0;
    FARM_TRY(rrf_begin(mem, ws, q, n_channels, channels, rel_off, rel_pred, &R));
    TopkPlan plan;
    FARM_TRY(plan_topk(mem, opts, k, &plan));
    if (plan.dtype != FARM_F32) {
      set_error("fused unary scores need the FP32 form (dtype FARM_F32)");
      return FARM_ERR_UNSUPPORTED;
    }
    if (q == 0) return FARM_OK;
    plan.between = has_between(rel_pred, R);
    plan.presim = true;
    if (!out_id || !out_score) { set_error("null output pointer"); return FARM_ERR_INVALID_ARG; }
    if (plan.c > ws->max_k) { set_error("k = %d exceeds the workspace's max_k %d", plan.c, ws->max_k); return FARM_ERR_INVALID_ARG; }
    DeviceGuard g(mem->device);
    hipStream_t s = (hipStream_t)stream;
    FARM_TRY(ensure_rrf(mem, ws));
    MetaView meta;
    FARM_TRY(stage_meta(ws, q, R, target_cls, rel_off, rel_pred, s, &meta));
    FARM_TRY(rrf_fuse(mem, ws, q, R, n_channels, channels, meta, s));
    return query_topk_core(mem, ws, q, R, nullptr, nullptr, meta, plan, k, out_id, out_score, out_terms,
                           out_anchor_id, s);
  } catch (...) {
    set_error("unexpected host exception in farm_query_topk_rrf");
    return FARM_ERR_HIP;
  }
}

}  // extern "C"
