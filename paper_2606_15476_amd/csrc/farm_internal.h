// farm_internal.h -- private declarations shared by libfarm's translation units.
// Not installed; the public ABI is include/farm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include <string>
#include <vector>

#include "../../include/farm.h"

namespace farm {

constexpr int kMaxRel = FARM_MAX_REL;
constexpr int kKPad = 128;         // descriptor rows are zero-padded to a multiple of this
constexpr int kRowAlign = 64;      // similarity-matrix rows are padded to a multiple of this
constexpr float kW = 0.5f;         // soft-blend weight of the relational factor
constexpr float kClassFactor = 0.3f;
constexpr float kFp8Max = 448.0f;  // largest finite OCP e4m3 value
constexpr int32_t kBoundCap = 2048;  // candidates per query kept by the bound-pruned TopK
constexpr int32_t kSemMax = 64;      // semantic anchor set per relation in the proposal pass
constexpr int32_t kBetweenSetSize = 64;  // candidate set of each of Between's anchor variables
// Uncertified terms listed for the block-wide fallback scan (more are still
// found and scanned by a sweep over the terms).
inline int64_t fallback_cap(int32_t max_q) {
  const int64_t c = (int64_t)max_q * 256 + 1024;
  return c < (1 << 20) ? c : (1 << 20);
}

// Validation flag bits raised by device-side checks.
enum : int {
  kBadDesc = 1 << 0,
  kZeroNorm = 1 << 1,
  kBadCenter = 1 << 2,
  kBadExtent = 1 << 3,
  kBadId = 1 << 4,
  kDupId = 1 << 5,
  kBadQuery = 1 << 6,
  kBadCov = 1 << 7,   // non-finite or not positive definite covariance
  kBadView = 1 << 8,  // non-finite view or rotation rows not orthonormal
};

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

}  // namespace farm

struct farm_memory {
  int64_t n = 0;
  int32_t d = 0;
  int32_t ldk = 0;  // padded descriptor row length (elements)
  int device = 0;
  uint32_t flags = 0;
  float rx = 0.f, ry = 0.f;
  // descriptors, L2-normalised, zero-padded to ldk
  float* dn = nullptr;        // [n][ldk] FP32 master
  uint16_t* dn_bf16 = nullptr;  // [n][ldk] BF16 (RNE)
  uint8_t* dn_fp8 = nullptr;    // [n][ldk] OCP e4m3, scaled by 1/dn_scale
  float* dn_scale = nullptr;    // [n] per-row FP32 scale (amax / 448)
  // reduced-precision error norms ||d~ - d||_2 and norms ||d~||_2 per row
  float* err_bf16 = nullptr;
  float* nrm_bf16 = nullptr;
  float* err_fp8 = nullptr;
  float* nrm_fp8 = nullptr;
  float* err_max = nullptr;  // [2] max over rows of err_bf16, err_fp8
  // geometry, structure of arrays
  float* x = nullptr;
  float* y = nullptr;
  float* z = nullptr;
  // [2][n]: lateral coordinate c . r (first n), then depth c . f along the
  // viewing direction f = (-r_y, r_x), each as an unevaluated sum hi + lo
  float* hr_hi = nullptr;
  float* hr_lo = nullptr;
  float* ext = nullptr;    // [3][n] extents
  // [2][n]: On's vertical coordinates, 4 * bottom face (first n) and 4 * top
  // face (z -+ extent_z / 2); the factor 4 = sigma_h / sigma_v (0.5 m / 0.125 m)
  // turns On's exponent into Near's form with a single coefficient (a power of
  // two, so exact)
  float* vz = nullptr;
  uint32_t* id = nullptr;
  int32_t* cls = nullptr;
  // objects ordered by class (stable): indices and their classes, so that the
  // candidate set of Closest/Farthest (one class) is a contiguous range
  int32_t* cls_order = nullptr;
  int32_t* cls_sorted = nullptr;
  // learned anchor proposals (farm_build_proposals): per predicate p and
  // target o a list of M anchors (target-major: one target's list is contiguous)
  int32_t prop_m = 0;
  int32_t* prop_idx = nullptr;  // [P][n][M] anchor indices (P = FARM_NUM_PROP_PRED)
  float* prop_val = nullptr;    // [P][n][M] predicate value (Near family: log P, others: P)
  float* prop_out = nullptr;    // [P][n] largest predicate value over anchors left out (same domain)
  std::vector<void*> prop_allocs;
  // entity Gaussians and stored views (farm_set_entity_geometry), structure of
  // arrays; null when the memory has none
  float* cov = nullptr;      // [6][n] packed covariances (xx, xy, xz, yy, yz, zz)
  double* cov_ld = nullptr;  // [n] log det of each covariance
  float* view = nullptr;     // [12][n] camera center, then its right, down and forward axes
  std::vector<void*> cov_allocs, view_allocs;
  // further embedding spaces (farm_add_embedding_space): normalised FP32 rows,
  // zero-padded like dn; spaces[s - 1] is space s (space 0 is dn)
  struct Space {
    int32_t d = 0, ldk = 0;
    float* dn = nullptr;  // [n][ldk]
  };
  std::vector<Space> spaces;
  std::vector<void*> space_allocs;
  size_t bytes = 0;
  std::vector<void*> allocs;
  // workspaces created on this memory plus servers it is registered with:
  // farm_free_memory refuses (FARM_ERR_BUSY) while any remain
  mutable std::atomic<int32_t> users{0};
};

struct farm_workspace {
  const farm_memory* mem = nullptr;
  // set while a library call runs on this workspace (WorkspaceClaim): a second
  // host thread entering meanwhile gets FARM_ERR_BUSY
  std::atomic<bool> in_call{false};
  int device = 0;
  int32_t max_q = 0, max_rel = 0;
  int64_t ld_s = 0;          // row stride of the similarity / score matrices
  float* qn = nullptr;        // [max_q + max_rel][ldk] normalised query vectors
  uint16_t* qn_bf16 = nullptr;
  uint8_t* qn_fp8 = nullptr;
  float* qn_scale = nullptr;
  float* qerr_bf16 = nullptr;   // [rows] ||q~ - q||_2 and ||q~||_2 of the reduced-precision copies
  float* qnrm_bf16 = nullptr;
  float* qerr_fp8 = nullptr;
  float* qnrm_fp8 = nullptr;
  float* sim = nullptr;       // [max_q + max_rel][ld_s] clamped similarities (target rows x kappa)
  float* lsim = nullptr;      // [max_rel][ld_s] log of the relation rows' similarities
  float* scores = nullptr;    // [max_q][ld_s] composite scores (fused path)
  float* scores_hi = nullptr; // [max_q][ld_s] upper bounds of the scores (reduced-precision form)
  int32_t* d_meta = nullptr;  // device copy of the metadata block below
  int32_t* h_meta = nullptr;  // pinned host staging of the metadata block
  int64_t meta_len = 0;       // int32 elements in the metadata block
  hipEvent_t meta_done = nullptr;
  bool meta_pending = false;
  int* status = nullptr;      // device validation flags
  // TopK candidate ping-pong buffers
  uint64_t* cand_key[2] = {nullptr, nullptr};
  int32_t* cand_idx[2] = {nullptr, nullptr};
  int64_t cand_cap = 0;       // elements per buffer
  int32_t max_k = 0;
  int32_t rs_cap = 0;            // candidate slots per query: max(max_k, kBoundCap)
  // winners / rescoring candidates: object indices, FP32 scores, terms, bound anchors
  int32_t* rs_idx = nullptr;     // [max_q][rs_cap]
  float* rs_score = nullptr;     // [max_q][rs_cap]
  float* rs_terms = nullptr;     // [max_q][rs_cap][FARM_MAX_REL]
  uint32_t* rs_anchor = nullptr; // [max_q][rs_cap][FARM_MAX_REL]
  int32_t* cand_count = nullptr; // [max_q]
  // proposal pass: semantic anchor set per relation, certificate counters
  int32_t* sem_idx = nullptr;    // [max_rel][kSemMax]
  int32_t* sem_cnt = nullptr;    // [max_rel]
  float* sem_tau = nullptr;      // [max_rel] largest similarity of an anchor outside the set
  float* sem_sim = nullptr;      // [max_rel][kSemMax] FP32 similarity of each set member (reduced precision)
  int32_t* btw_idx = nullptr;    // [max_rel][64] Between's candidate sets (relation rows of Between invocations)
  float* btw_sim = nullptr;      // [max_rel][64] their similarities
  int32_t* btw_cnt = nullptr;    // [max_rel]
  unsigned long long* prop_stats = nullptr;  // [4] terms checked, fell back, FP32 dots (subset, fallback)
  unsigned long long* fb_list = nullptr;     // [fb_cap] terms the proposals could not certify: query << 32 | term
  uint32_t* fb_count = nullptr;              // [1]
  int64_t fb_cap = 0;
  // optional phase timer: pending (start, stop) event pairs per phase
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  struct PendingPhase { int phase; hipEvent_t a, b; };
  std::vector<PendingPhase> pending;
  double phase_ms[FARM_PHASE_COUNT] = {0};
  int64_t phase_count[FARM_PHASE_COUNT] = {0};
  // reciprocal-rank fusion buffers, allocated on first use (farm_query_topk_rrf)
  float* rrf_qn = nullptr;       // [max_q + max_rel][rrf_ldk] one channel's normalised query vectors
  int32_t rrf_ldk = 0;
  float* rrf_cos = nullptr;      // [max_q + max_rel][ld_s] one channel's cosines
  float* rrf_val = nullptr;      // [rrf_blocks][n] ranking scratch: cosines in bucket order ...
  int32_t* rrf_idx = nullptr;    // [rrf_blocks][n] ... and their object indices
  int32_t rrf_blocks = 0;
  std::vector<void*> rrf_allocs;
  size_t bytes = 0;
  std::vector<void*> allocs;
};

// The anchor proposal network (mlp.hip): FP32 masters, BF16 copies, batch buffers.
struct farm_mlp {
  int device = 0;
  int32_t d = 0, dp = 0, ldx = 0, h = 0, bmax = 0, bpad = 0;
  int64_t step = 0;
  // FP32 master parameters, gradients, AdamW moments: one block of floats
  float* par = nullptr;
  float* grad = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  int64_t n_par = 0;
  float *W1, *b1, *W2, *b2, *W3, *b3;      // views into par
  float *gW1, *gb1, *gW2, *gb2, *gW3, *gb3;  // views into grad
  // BF16 copies used by the GEMMs; W3 rounded to BF16 values kept as floats
  uint16_t* W1b = nullptr;   // [h][ldx]
  uint16_t* W2b = nullptr;   // [h][h]
  uint16_t* W2bT = nullptr;  // [h][h] transpose
  float* W3r = nullptr;      // [P][h]
  // batch activations
  uint16_t* X = nullptr;     // [bpad][ldx]
  uint16_t* XT = nullptr;    // [ldx][bpad]
  float* Z1 = nullptr;       // [bpad][h]
  float* Z2 = nullptr;
  uint16_t* A1 = nullptr;    // [bpad][h]
  uint16_t* A1T = nullptr;   // [h][bpad]
  uint16_t* A2 = nullptr;
  float* Y = nullptr;        // [bpad][P]
  float* dY = nullptr;       // [bpad][P]
  float* dA = nullptr;       // [bpad][h]
  uint16_t* dZ = nullptr;    // [bpad][h] dZ2 of the last step
  uint16_t* dZ1 = nullptr;   // [bpad][h] dZ1 of the last step
  uint16_t* dZT = nullptr;   // [h][bpad]
  float* loss_part = nullptr;
  float* red_part = nullptr;  // partial sums of the chunked batch reductions
  std::vector<void*> allocs;
  size_t bytes = 0;
};

// Metadata block layout (int32), written by the host per call:
//   [0, q)                 target class per query
//   [q, 2q + 1)            rel_off
//   [2q + 1, 2q + 1 + R)   rel_pred
//   [.., + R)              query index of each relation
struct MetaView {
  const int32_t* tcls;
  const int32_t* rel_off;
  const int32_t* rel_pred;
  const int32_t* rel_query;
  const int32_t* scan_rows = nullptr;  // relation rows of the scanned predicates (scan_n of them)
  int32_t scan_n = 0;
  int32_t geo_n = 0;  // how many of them name an entity-geometry predicate (Gaussians, stored views)
};

namespace farm {

// Outputs of row normalisation for the reduced-precision copies (any may be null).
struct LowPrecRows {
  uint16_t* bf16 = nullptr;
  uint8_t* fp8 = nullptr;
  float* fp8_scale = nullptr;
  float* err_bf16 = nullptr;
  float* nrm_bf16 = nullptr;
  float* err_fp8 = nullptr;
  float* nrm_fp8 = nullptr;
};

// Error bound of a reduced-precision similarity matrix, before the clamp and
// the class factor:  |sim~(row, j) - sim(row, j)| <= q_nrm[row] * o_err[j] + q_err[row] + acc.
// (Cauchy-Schwarz on q~.d~ - q.d = q~.(d~ - d) + (q~ - q).d with |d| <= 1, plus
// FP32 accumulation of both the GEMM and the FP32 reference dot products.)
// A null q_nrm means the matrix is the FP32 one (bound 0).
struct SimBound {
  const float* q_nrm = nullptr;
  const float* q_err = nullptr;
  const float* o_err = nullptr;
  const float* o_err_max = nullptr;  // device scalar: max_j o_err[j]
  float acc = 0.f;
};

// Anchor proposals seen by the rescoring kernel; m == 0 means full anchor scans.
struct PropView {
  int32_t m = 0;
  const int32_t* idx = nullptr;      // [P][n][m]
  const float* val = nullptr;        // [P][n][m]
  const float* out = nullptr;        // [P][n]
  const int32_t* sem_idx = nullptr;  // [R][kSemMax]
  const int32_t* sem_cnt = nullptr;  // [R]
  const float* sem_tau = nullptr;    // [R]
  const float* sem_sim = nullptr;    // [R][kSemMax] exact similarities of the set, or null (FP32 matrix)
  unsigned long long* stats = nullptr;
  unsigned long long* fb_list = nullptr;  // worklist of uncertified terms (query << 32 | term index)
  uint32_t* fb_count = nullptr;
  int64_t fb_cap = 0;
  int32_t rel_total = 0;  // relation rows of the call (one LDS-staged block each)
  bool in_lds = false;    // run the proposal pass with the rows staged in LDS
  bool queue = false;     // LDS pass: queue the survivors' dot products per block (BF16 similarities)
  // Between's candidate sets (scanned terms of Between invocations)
  const int32_t* btw_idx = nullptr;
  const float* btw_sim = nullptr;
  const int32_t* btw_cnt = nullptr;
  // where the LDS-staged pass publishes the semantic sets it selects
  int32_t* sem_idx_out = nullptr;
  int32_t* sem_cnt_out = nullptr;
  float* sem_tau_out = nullptr;
  float* sem_sim_out = nullptr;
};

// Entity Gaussians and stored views of a memory, passed to kernels by value
// (null pointers when the memory has none).
struct EntityGeo {
  const float* cov = nullptr;      // [6][n]
  const double* cov_ld = nullptr;  // [n]
  const float* view = nullptr;     // [12][n]
};
inline EntityGeo entity_geo(const farm_memory* m) { return EntityGeo{m->cov, m->cov_ld, m->view}; }

// Whether the proposal pass stages similarity rows of this memory in LDS
// (and then selects the semantic sets itself).
bool proposal_pass_in_lds(const farm_memory* mem, bool bounded);

// Makes `dev` current for the guard's lifetime.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

void set_error(const char* fmt, ...);
farm_status hip_fail(hipError_t e, const char* what);

// ---- prep.hip
hipError_t launch_validate_memory(const float* desc, const float* center, const float* extent,
                                  const uint32_t* id, int64_t n, int32_t d, int* flags,
                                  uint32_t* table, int64_t table_size, hipStream_t s);
hipError_t launch_normalize_rows(const float* src, int64_t rows, int32_t d, int32_t ldk, float* dst_f32,
                                 const LowPrecRows& lp, int* flags, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// Validate and lay out entity Gaussians (cov_in [n][6] -> cov [6][n] and
// cov_ld [n]) and stored views (view_in [n][12] -> view [12][n]); either
// input may be null.  Raises kBadCov / kBadView in flags and lowers
// first_bad[0] to the first offending object.
hipError_t launch_entity_geometry(const float* cov_in, const float* view_in, int64_t n, float* cov, double* cov_ld,
                                  float* view, int* flags, int* first_bad, hipStream_t s);
hipError_t launch_geometry(const float* center, const float* extent, int64_t n, float rx, float ry, float* vz,
                           float* x, float* y, float* z, float* hr_hi, float* hr_lo, float* ext,
                           hipStream_t s);

// ---- gemm.hip: sim[row][col] = kappa(row, col) * max(0, <a_row, b_col>)
hipError_t launch_sim_gemm_f32(const float* a, const float* b, int64_t m, int64_t n, int32_t ldk,
                               float* c, int64_t ldc, const int32_t* row_cls, int64_t n_cls_rows,
                               const int32_t* col_cls, hipStream_t s);
hipError_t launch_sim_gemm_bf16(const uint16_t* a, const uint16_t* b, int64_t m, int64_t n, int32_t ldk,
                                float* c, int64_t ldc, const int32_t* row_cls, int64_t n_cls_rows,
                                const int32_t* col_cls, hipStream_t s);
hipError_t launch_sim_gemm_fp8(const uint8_t* a, const float* a_scale, const uint8_t* b, const float* b_scale,
                               int64_t m, int64_t n, int32_t ldk, float* c, int64_t ldc,
                               const int32_t* row_cls, int64_t n_cls_rows, const int32_t* col_cls,
                               hipStream_t s);

// Plain FP32 "NT" GEMM without epilogue: C[m][n] = <A row, B row> (k a multiple of 32).
hipError_t launch_gemm_nt_f32(const float* a, const float* b, int64_t m, int64_t n, int32_t ldk, float* c, int64_t ldc,
                              hipStream_t s);

// Plain BF16 "NT" GEMM for the proposal network: C[m][n] = A[m][k] . B[n][k]^T
// (+ bias[n]) in FP32, or BF16 GELU(A . B^T + bias) when gelu_bf16_out; k a
// multiple of 64, leading dimensions in elements (rows 16-byte aligned).
hipError_t launch_gemm_nt_bf16(const uint16_t* a, int64_t lda, const uint16_t* b, int64_t ldb, int64_t m, int64_t n,
                               int64_t k, void* c, int64_t ldc, const float* bias, bool gelu_bf16_out, hipStream_t s);

// ---- pair.hip
// With a SimBound (bound.q_nrm != null) the pass also writes scores_hi >= s:
// the target similarity raised by its error bound and every relation term by
// the largest similarity error bound of its row.
// lsim[r][j] = log(sim[q + r][j]) of the relation rows (large negative for 0),
// shared by the Near family of every relational kernel.
hipError_t launch_log_rows(const float* sim, int64_t ld_s, int64_t rows, int64_t n, float* lsim, hipStream_t s);
hipError_t launch_pair_exhaustive(const farm_memory* mem, const farm_workspace* ws, const float* sim,
                                  const float* lsim, int64_t ld_s, int32_t q, MetaView meta, const SimBound& bound,
                                  float* scores, int64_t ld_out, float* rel_terms, uint32_t* rel_anchor_id,
                                  float* scores_hi, hipStream_t s);
// ScoredCandidate breakdown for selected objects: t_r and b_r recomputed for
// each (query, rank) entry of idx[q][k].
hipError_t launch_explain(const farm_memory* mem, const farm_workspace* ws, const float* sim, int64_t ld_s, int32_t q,
                          MetaView meta, const int32_t* idx, int32_t k, float* out_terms, uint32_t* out_anchor_id,
                          hipStream_t s);

// Between's candidate sets (scan_math.h): for every relation row of a Between
// invocation (FARM_BETWEEN / FARM_AND) the 64 anchors of largest similarity
// (ties by id) and their similarities into bidx/bsim [R][64], bcnt [R].
hipError_t launch_between_sets(const farm_memory* mem, const float* sim, int64_t ld_s, int32_t q, MetaView meta,
                               int32_t R, int32_t* bidx, float* bsim, int32_t* bcnt, hipStream_t s);

// ---- rescore.hip
// Exact FP32 similarities of the Between rows, in place (reduced-precision GEMMs).
hipError_t launch_exact_rows(const farm_memory* mem, const float* qn, float* sim, int64_t ld_s, int32_t q,
                             MetaView meta, int32_t R, hipStream_t s);
// FP32 scores of the candidates cand[q][c] (object indices, -1 = none): exact
// target similarity and, per relation, the exact maximum over anchors, where
// only anchors whose bounded value can reach the best lower bound get an FP32
// dot product.  Writes rs_score[q][c], rs_terms/rs_anchor[q][c][8].
// Candidate scoring in two steps.  launch_rescore_terms: every (candidate,
// relation) term into rs_terms / rs_anchor in the family's domain.  With
// proposals (prop.m > 0) a first pass takes each term over the target's anchor
// list and the relation's semantic set and keeps it when it exceeds the bound
// on every anchor outside both; the second pass (fallback_pass) scans all
// anchors for the others.  Without proposals one pass scans all anchors.
// launch_rescore_combine: s_sem (FP32 dot for reduced precision) and the
// composite into rs_score, linear terms into rs_terms.
hipError_t launch_rescore_terms(const farm_memory* mem, const farm_workspace* ws, const float* sim, int64_t ld_s,
                                int32_t q, MetaView meta, const SimBound& bound, const int32_t* cand,
                                const int32_t* cand_count, int32_t c, const PropView& prop, bool fallback_pass,
                                hipStream_t s);
hipError_t launch_rescore_combine(const farm_memory* mem, const farm_workspace* ws, const float* sim, int64_t ld_s,
                                  int32_t q, MetaView meta, const SimBound& bound, const int32_t* cand,
                                  const int32_t* cand_count, int32_t c, hipStream_t s);

// ---- bounded.hip
// Candidates of the exact bound-pruned TopK: per query every object whose
// s_sem upper bound reaches the K-th largest lower bound (1 - w) s_sem_lo,
// in index order, into cand[q][cap] (-1 padded), count[q]; certified[q] = 0
// when more than cap objects qualified (the cap best upper bounds are kept).
hipError_t launch_bound_candidates(const farm_memory* mem, const float* sim, int64_t ld_s, int32_t q, MetaView meta,
                                   const SimBound& bound, int32_t k, int32_t cap, int32_t* cand, int32_t* count,
                                   int32_t* certified, hipStream_t s);
// Final TopK among rescored candidates; certified[q] (optional) = 1 when the
// K-th rescored score exceeds, by the FP32 value tolerance, the largest upper
// bound of any object outside the candidates, or every object was a
// candidate.  hi_key/hi_idx [q][c + 1] are the top c + 1 objects by upper
// bound: the first of them that is not a candidate carries that largest bound.
// cand_count (optional): per query, the number of filled candidate slots.
hipError_t launch_rescore_select(const farm_workspace* ws, int32_t q, int32_t c, int32_t k,
                                 const uint64_t* hi_key, const int32_t* hi_idx, const int32_t* cand_count, int64_t n,
                                 uint32_t* out_id, float* out_score, float* out_terms, uint32_t* out_anchor_id,
                                 int32_t* certified, hipStream_t s);
hipError_t launch_max_reduce(const float* v, int64_t n, float* out, hipStream_t s);
// FP32 similarity max(0, q.d) of every semantic-set member (reduced-precision
// matrices), with the rescoring kernel's own dot product so that the values
// are the ones a full scan would compute.
hipError_t launch_semantic_exact(const farm_memory* mem, const farm_workspace* ws, int32_t q, int32_t R, hipStream_t s);

// ---- proposal.hip
// Per relation row: a semantic anchor set (at most kSemMax anchors with the
// largest similarities) and the largest similarity of the anchors outside it.
hipError_t launch_semantic_sets(const float* sim, int64_t ld_s, int32_t q, int32_t R, int64_t n, int32_t* sem_idx,
                                int32_t* sem_cnt, float* sem_tau, hipStream_t s);

// ---- rrf.hip
// Reciprocal-rank fusion: out[row][i] += w / (5 + rank of cos[row][i] in its row), ranks by
// (cosine descending, id ascending); val/idx: blocks x n scratch.
hipError_t launch_rrf_rank(const float* cos, int64_t ld, int32_t rows, int64_t n, const uint32_t* ids, float w,
                           float* out, float* val, int32_t* idx, int32_t blocks, hipStream_t s);
// out[row][i] *= inv_norm, times the class factor on target rows (row < q).
hipError_t launch_rrf_finish(float* out, int64_t ld, int32_t q, int32_t rows, int64_t n, const int32_t* tcls,
                             const int32_t* cls, float inv_norm, hipStream_t s);

// ---- topk.hip
// Select the top k of each score row.  Writes (key, index) of the winners in
// order into out_key/out_idx [q][k]; candidate buffers come from the workspace.
hipError_t launch_topk(const farm_memory* mem, farm_workspace* ws, const float* scores, int64_t ld_scores,
                       int32_t q, int32_t k, uint64_t** out_key, int32_t** out_idx, hipStream_t s);
hipError_t launch_topk_emit(const uint64_t* key, const int32_t* idx, int32_t q, int32_t k, uint32_t* out_id,
                            float* out_score, int32_t* out_index, hipStream_t s);
int64_t topk_candidate_capacity(int64_t n, int32_t max_q, int32_t max_k);

}  // namespace farm
