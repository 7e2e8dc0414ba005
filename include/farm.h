/*
 * farm.h -- C ABI of libfarm, the MI355X (gfx950) library for FARM's
 * query-time relational retrieval over an object-level spatial memory.
 *
 * The operation (paper, Section 2.3 "Robust Relational Object Retrieval";
 * Appendix "Robust Relational Retrieval Formulation" and Appendix "Retrieval
 * Details", steps 3-5 and 7):
 *
 *   memory   : n objects, each with a descriptor (d floats), a 3-D box
 *              (center, full extents), a unique id and an optional class id;
 *              one viewer frame per scene (its right vector in the x-y plane).
 *   query    : a target embedding q_t, an optional target class, and R <= 8
 *              relations (predicate p_r, anchor embedding q_r).
 *   sim(i,v) = max(0, cos(desc_i, v))
 *   s_sem(i) = kappa_i * sim(i, q_t)      kappa_i = 0.3 if both classes are
 *                                          known (>= 0) and differ, else 1
 *   t_r(i)   = max_{j != i} sim(j, q_r) * P_{p_r}(i, j)
 *   b_r(i)   = id of the maximising anchor (smallest id on ties)
 *   s(i)     = s_sem(i) * (0.5 + 0.5 * (prod_r t_r(i))^(1/R))   (1 if R = 0)
 *   TopK     = first min(K, n) objects by (s desc, id asc)
 *
 *   predicates, D = c_i - c_j (target minus anchor box center), sig = logistic,
 *   r = the scene's viewer right axis, f = (-r_y, r_x) its viewing direction
 *   (Appendix "Retrieval Details": closed-form evaluators; one viewer frame
 *   per scene stands in for the stored camera views):
 *   FARM_NEAR        exp(-|D|^2 / (2 * 0.5^2))
 *   FARM_NEXT_TO     exp(-|D|^2 / (2 * 1.0^2))
 *   FARM_ABOVE       sig(D_z / 0.1)            FARM_BELOW    sig(-D_z / 0.1)
 *   FARM_RIGHT_OF    sig((D_x r_x + D_y r_y) / 0.1)
 *   FARM_LEFT_OF     sig(-(D_x r_x + D_y r_y) / 0.1)
 *   FARM_IN_FRONT_OF sig(-(D_x f_x + D_y f_y) / 0.1)   (nearer the viewer)
 *   FARM_BEHIND      sig((D_x f_x + D_y f_y) / 0.1)
 *   FARM_ON          exp(-(D_x^2 + D_y^2) / (2 * 0.5^2)) * exp(-g^2 / (2 * 0.125^2))
 *                    g = (c_i,z - e_i,z / 2) - (c_j,z + e_j,z / 2): the target's
 *                    bottom face minus the anchor's top face (e = full extents);
 *                    a horizontal gate times a vertical band
 *   FARM_CLOSEST     1 / rank             FARM_FARTHEST  1 / (m + 2 - rank)
 *                    rank of i among the query's candidates (objects of its
 *                    target class; all objects without a class), by distance
 *                    to j: 1 + #{c in C, c != i, j : |c_c - c_j| < |c_i - c_j|,
 *                    equal distances by id}, m = |C minus i and j|; squared
 *                    distances summed in FP32 from FP32 center differences
 *                    (within 5 * 2^-24 relative of the exact ones, so two
 *                    candidates closer than that may take either order).  A rank within
 *                    the candidate set, scored 1 / (|rank - r*| + 1).  Cost
 *                    O(|C|) per evaluated anchor (O(N) without a class)
 *   FARM_INSIDE      prod_k sig((e_j,k / 2 - |D_k|) / 0.1): the target's center
 *                    within the anchor's box (e = full extents), a soft
 *                    containment test
 *   FARM_BETWEEN     ternary, anchors j1 and j2 (a FARM_BETWEEN relation slot
 *                    holds j1's description and must be followed by a
 *                    FARM_AND slot holding j2's; the pair is one predicate
 *                    invocation, counted once in the geometric mean):
 *                    sig(s / 0.1) sig((L - s) / 0.1) exp(-h^2 / (2 * 0.5^2)),
 *                    L = |c_j2 - c_j1|, s the offset of c_i along the axis
 *                    from c_j1 to c_j2, h the distance of c_i from that axis
 *                    (0 when L = 0): the target's center projects inside the
 *                    segment joining the anchors and lies near it.  Term
 *                    max over j1 != j2 (both != i) of sim(j1, q_j1)
 *                    sim(j2, q_j2) Between; both slots report it, the first
 *                    binds j1 and the second j2 (smaller id pair on ties;
 *                    FARM_NO_ID when the term is 0).  Exact by bucket
 *                    elimination of the two anchor variables per target: the
 *                    pairs of the two relations' semantic sets first, then,
 *                    unless they certify the term, every pair whose bound
 *                    reaches the best value
 *
 *   over the entity Gaussians and stored views of farm_set_entity_geometry
 *   (Section "Memory Construction": a 3D Gaussian and representative posed
 *   views per entity; Section "Robust Relational Object Retrieval",
 *   implementation paragraph: Hellinger distance for Near; Appendix
 *   "Retrieval Details", step 4: the viewpoint-dependent predicates in stored
 *   camera views of the target candidate).  A memory without them answers
 *   FARM_ERR_UNSUPPORTED to queries that name these:
 *   FARM_NEAR_HELLINGER  1 - H(N_i, N_j), H^2 = 1 - BC, BC = det(A)^(1/4)
 *                    det(B)^(1/4) / det(M)^(1/2) exp(-D^T M^-1 D / 8),
 *                    M = (A + B) / 2, A and B the covariances (means = centers)
 *   FARM_LEFT_OF_VIEW    sig((u_j - u_i) / 0.05)   FARM_RIGHT_OF_VIEW sig((u_i - u_j) / 0.05)
 *   FARM_IN_FRONT_OF_VIEW sig((z_j - z_i) / 0.1)   FARM_BEHIND_VIEW   sig((z_i - z_j) / 0.1)
 *                    (x, y, z) = R_i (c - p_i) the camera coordinates of a
 *                    center in target i's stored view (camera center p_i,
 *                    rotation rows right, down, forward), u = x / z its
 *                    horizontal image-plane coordinate; 0 unless both centers
 *                    are in the view: z >= 0.1 m, |x| <= z, |y| <= 0.75 z
 *   These five are evaluated in FP64 and scanned per anchor like Inside.
 *
 * Conventions shared by every entry point:
 *   - Every function returns a farm_status; farm_last_error() gives a message
 *     for the calling thread's last failure.  Nothing aborts and no C++
 *     exception crosses the ABI.
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary process memory.  All arrays are dense,
 *     row-major, without padding.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls are stream-ordered and return before the GPU work finishes,
 *     except where stated.  Input pointers are borrowed for the duration of
 *     the call's GPU work; output buffers are owned by the caller.
 *   - Floating point is FP32 throughout the scoring path (no FP64 on the GPU).
 */
#ifndef FARM_H
#define FARM_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define FARM_API __attribute__((visibility("default")))
#else
#define FARM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FARM_OK = 0,
  FARM_ERR_INVALID_ARG = -1, /* bad pointer, size, predicate id, R > 8, K < 1,
                                non-finite or zero-norm vector, duplicate id */
  FARM_ERR_OOM = -2,         /* device allocation failed or exceeds a budget */
  FARM_ERR_HIP = -3,         /* a HIP runtime call failed */
  FARM_ERR_UNSUPPORTED = -4, /* valid request outside what the library supports */
  FARM_ERR_BUSY = -5         /* the object is in use: a workspace entered by a
                                second host thread during a call on it, or a
                                memory freed while workspaces or servers still
                                use it; nothing was done, retry later */
} farm_status;

typedef enum { FARM_F32 = 0, FARM_BF16 = 1, FARM_FP8_E4M3 = 2 } farm_dtype;

typedef enum {
  FARM_NEAR = 0,
  FARM_ABOVE = 1,
  FARM_BELOW = 2,
  FARM_LEFT_OF = 3,
  FARM_RIGHT_OF = 4,
  FARM_NEXT_TO = 5,
  FARM_IN_FRONT_OF = 6,
  FARM_BEHIND = 7,
  FARM_ON = 8,
  FARM_CLOSEST = 9,
  FARM_FARTHEST = 10,
  FARM_INSIDE = 11,
  FARM_BETWEEN = 12,
  FARM_AND = 13,          /* the second anchor of the FARM_BETWEEN slot before it */
  FARM_NEAR_HELLINGER = 14,
  FARM_LEFT_OF_VIEW = 15,
  FARM_RIGHT_OF_VIEW = 16,
  FARM_IN_FRONT_OF_VIEW = 17,
  FARM_BEHIND_VIEW = 18
} farm_pred;
#define FARM_NUM_PRED 19        /* predicate ids 0 .. FARM_NUM_PRED - 1 */
#define FARM_NUM_PROP_PRED 9    /* predicates with learned anchor lists (network outputs): 0 .. 8 */

#define FARM_MAX_REL 8          /* relations per query */
#define FARM_MAX_K 1024         /* TopK size */
#define FARM_NO_ID 0xFFFFFFFFu  /* padding id (reserved: never a valid object id) */

/* build flags: which reduced-precision descriptor copies to keep */
#define FARM_BUILD_BF16 0x1u
#define FARM_BUILD_FP8 0x2u

typedef struct farm_memory farm_memory;       /* device-resident scene, immutable once built */
typedef struct farm_workspace farm_workspace; /* per-stream scratch for scoring calls */

/*
 * Build the device-resident memory of one scene (memory representation of
 * Section 2.2: per-entity geometry and retrieval embedding; one viewer frame).
 *   n            number of objects, 1 <= n < 2^31
 *   d            descriptor width, 1 <= d <= 8192
 *   desc         device [n][d] FP32 descriptors, any non-zero norm
 *   center       device [n][3] FP32 box centers (metres, z up)
 *   extent       device [n][3] FP32 full box side lengths, > 0
 *   id           device [n] uint32 object ids, unique, != FARM_NO_ID
 *   cls          device [n] int32 class ids (-1 = unknown) or NULL (all unknown)
 *   view_right_x/y  the scene viewer's right vector in the ground plane
 *   flags        FARM_BUILD_* bits
 *   out          receives the handle
 * The library copies everything it needs; the inputs can be freed afterwards.
 * Synchronises `stream` to validate the inputs (finite values, non-zero
 * norms, positive extents, unique ids): FARM_ERR_INVALID_ARG names the first
 * violation.  With classes it also keeps the objects in class order (two
 * int32 arrays of n; a host sort of the class ids), the candidate sets of
 * FARM_CLOSEST / FARM_FARTHEST.  Free with farm_free_memory.
 */
FARM_API farm_status farm_build_memory(int64_t n, int32_t d, const float* desc, const float* center,
                              const float* extent, const uint32_t* id, const int32_t* cls,
                              float view_right_x, float view_right_y, uint32_t flags, void* stream,
                              farm_memory** out);

/*
 * Attach entity Gaussians and stored views to a built memory (Section "Memory
 * Construction": each entity's 3D Gaussian N(mu, Sigma), mu its center, and
 * its representative posed views), for FARM_NEAR_HELLINGER and the
 * FARM_*_VIEW predicates.
 *   cov    device [n][6] FP32 covariances, packed (xx, xy, xz, yy, yz, zz),
 *          positive definite; or NULL (keep the current ones, if any)
 *   view   device [n][12] FP32 stored views: camera center (3), then the
 *          camera's right, down and forward axes in world coordinates (the
 *          rows of the world-to-camera rotation, orthonormal within 1e-3);
 *          or NULL (keep the current ones)
 * The library copies them.  Synchronises `stream` to validate: INVALID_ARG
 * (naming the first bad object) leaves the memory as it was.  Must not run
 * while scoring calls on the memory are in flight.
 */
FARM_API farm_status farm_set_entity_geometry(farm_memory* mem, const float* cov, const float* view, void* stream);

/* Release a memory handle (synchronises the device first). NULL is a no-op.
   FARM_ERR_BUSY while workspaces created on it or servers it was added to
   have not been freed; the handle then stays valid. */
FARM_API farm_status farm_free_memory(farm_memory* mem);

/* n, d and the device bytes the handle holds (any out pointer may be NULL). */
FARM_API farm_status farm_memory_info(const farm_memory* mem, int64_t* n, int32_t* d, size_t* bytes);

/*
 * Scratch for scoring calls on one memory: normalised query vectors, the
 * similarity matrix, metadata staging and TopK candidate buffers, sized for up
 * to max_q queries, max_rel relations (all queries together) and TopK size
 * max_k (1..FARM_MAX_K; with reduced-precision rescoring the candidate count
 * rescore_mult*k must fit too) per call.  A workspace serves one stream at a
 * time: calls that share it must be ordered on one stream.  It serves one host
 * thread at a time too: a call entered while another call on the same
 * workspace runs returns FARM_ERR_BUSY without doing anything.  Allocates
 * device memory and one pinned host staging block; free with
 * farm_workspace_free.
 */
FARM_API farm_status farm_workspace_create(const farm_memory* mem, int32_t max_q, int32_t max_rel, int32_t max_k,
                                  farm_workspace** out);
FARM_API farm_status farm_workspace_free(farm_workspace* ws);
FARM_API farm_status farm_workspace_bytes(const farm_workspace* ws, size_t* bytes);

/* Projected device bytes of a workspace of this shape (for admission). */
FARM_API farm_status farm_workspace_estimate(const farm_memory* mem, int32_t max_q, int32_t max_rel, int32_t max_k,
                                    size_t* bytes);

/*
 * Score every (query, object) pair exhaustively (the plain method): for each
 * target candidate o, the score of its best witnessing binding (Section
 * "Robust Relational Object Retrieval", the score and TopK definition; the
 * same definition in Appendix "Robust Relational Retrieval Formulation",
 * "Soft verification").  Conditioning on o separates the anchors of a star
 * query ("Query-time complexity" paragraph), so each relation r contributes
 * its own best anchor:
 *   s_sem(o) = kappa_o * max(0, cos(target, u_o))   (kappa_o the class factor)
 *   t_r(o)   = max over a != o of max(0, cos(anchor_r, u_a)) * P_r(o, a)
 *   s(o)     = s_sem(o) * (1/2 + 1/2 * geometric mean of the t_r(o))
 * with Between's two anchors bound jointly over their candidate sets.  The
 * per-predicate P are the closed-form evaluators of Appendix "Retrieval
 * Details", step 4; the blend and the class factor are its step 5.
 *   q, d         number of queries; d must equal the memory's d
 *   target       device [q][d] FP32 target embeddings (any non-zero norm)
 *   target_cls   host [q] int32 parsed target classes (-1 = none) or NULL
 *   rel_off      host [q+1] int32 CSR offsets, rel_off[0] = 0, non-decreasing,
 *                at most FARM_MAX_REL relations per query
 *   rel_pred     host [rel_off[q]] int32 farm_pred values (FARM_BETWEEN is
 *                followed by FARM_AND in the same query, and only there)
 *   rel_anchor   device [rel_off[q]][d] FP32 anchor embeddings
 *   scores       device [q][n] FP32 out: s(i)
 *   rel_terms    device [rel_off[q]][n] FP32 out: t_r(i), or NULL
 *   rel_anchor_id device [rel_off[q]][n] uint32 out: b_r(i), or NULL
 *                (FARM_NO_ID when n = 1)
 * Host arguments are read before the call returns.  Device input vectors
 * that are non-finite or have zero norm are reported by the next
 * farm_workspace_status call; their rows' outputs are unspecified.
 */
FARM_API farm_status farm_score_query(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t d,
                             const float* target, const int32_t* target_cls, const int32_t* rel_off,
                             const int32_t* rel_pred, const float* rel_anchor, float* scores,
                             float* rel_terms, uint32_t* rel_anchor_id, void* stream);

/*
 * The target similarity s_sem alone, as the similarity GEMM of `dtype`
 * produces it: out[j][i] = kappa_i * max(0, cos(target_j, u_i)) with the
 * class factor of Appendix "Retrieval Details", step 5 (kappa = 0.3 when the
 * object's class differs from target_cls[j], else 1; the target similarity of
 * its step 3, one embedding channel).  FARM_BF16 / FARM_FP8_E4M3 return the
 * reduced-precision estimate the precision form starts from (before any FP32
 * rescoring), for measuring its error.
 *   q, d, target, target_cls   as in farm_score_query (no relations)
 *   dtype        farm_dtype; UNSUPPORTED when the memory lacks that copy
 *   out          device [q][n] FP32
 */
FARM_API farm_status farm_similarity(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t d,
                                     const float* target, const int32_t* target_cls, int32_t dtype, float* out,
                                     void* stream);

/*
 * TopK of precomputed score rows: the K highest-scoring candidates, the
 * retrieval output (Section "Robust Relational Object Retrieval", the TopK
 * over the entity set; the ranked candidate list of Appendix "Retrieval
 * Details", step 7).
 *   scores       device [q][n] FP32 (n = the memory's n; NaN not allowed)
 *   k            1 <= k <= FARM_MAX_K; k > n returns n entries, then padding
 *   out_id       device [q][k] uint32 ids (FARM_NO_ID padding)
 *   out_score    device [q][k] FP32 scores (-INFINITY padding)
 *   out_index    device [q][k] int32 object indices (-1 padding) or NULL
 * Order: score descending, then id ascending.
 */
FARM_API farm_status farm_topk(const farm_memory* mem, farm_workspace* ws, const float* scores, int32_t q,
                      int32_t k, uint32_t* out_id, float* out_score, int32_t* out_index, void* stream);

/* How the fused path finds the TopK. */
typedef enum {
  /* score every object over every anchor (the plain method); with a reduced
     precision dtype, the top rescore_mult*k by estimate are rescored in FP32 */
  FARM_METHOD_EXHAUSTIVE = 0,
  /* exact bound-pruned TopK: the soft blend keeps each score in
     [(1-w) s_sem, s_sem], so only objects whose s_sem upper bound reaches the
     K-th largest lower bound (1-w) s_sem can enter the TopK; those (at most
     2048 per query) are scored exactly in FP32 */
  FARM_METHOD_BOUNDED = 1,
  /* BOUNDED, with each candidate's relation terms taken over its learned
     anchor list and the relation's semantic anchor set, certified against a
     bound on every other anchor, else over all anchors (needs
     farm_build_proposals); the result equals BOUNDED's */
  FARM_METHOD_PROPOSAL = 2
} farm_method;

/* Option bits of farm_score_opts.flags. */
typedef enum {
  /* FARM_METHOD_PROPOSAL: run the proposal pass on similarities gathered from
     global memory even when a similarity row fits in LDS (the form used
     for scenes too large to stage); results are identical */
  FARM_OPT_GLOBAL_PROPOSAL_PASS = 1
} farm_opt_flags;

/* Options of the fused path. */
typedef struct {
  int32_t dtype;        /* farm_dtype of the similarity GEMM (FARM_F32 = exact path) */
  int32_t method;       /* farm_method */
  int32_t rescore_mult; /* EXHAUSTIVE with reduced precision: rescore the top rescore_mult*k (>= 1) */
  int32_t flags;        /* farm_opt_flags bits (0 = defaults) */
  int32_t* certified;   /* device [q] out or NULL: 1 when the returned set is provably
                           the exact TopK, else 0 */
} farm_score_opts;

/*
 * Fused score + TopK, returning ScoredCandidate records (Appendix "Retrieval
 * Details", output step: target, composite score, per-predicate breakdown,
 * bound landmarks).
 *   query arguments as in farm_score_query
 *   opts         NULL = FP32 exact path
 *   k            1 <= k <= FARM_MAX_K
 *   out_id, out_score     device [q][k]
 *   out_terms     device [q][k][FARM_MAX_REL] FP32 t_r of each returned
 *                 object (0 beyond the query's R), or NULL
 *   out_anchor_id device [q][k][FARM_MAX_REL] uint32 b_r (FARM_NO_ID beyond R),
 *                 or NULL
 * With a reduced-precision dtype the similarity GEMM runs in BF16 or FP8
 * e4m3 (per-row scales); the relational pass then scores every object with an
 * upper bound of its score (each similarity raised by a proven bound on its
 * rounding error), the top rescore_mult*k objects by that bound are rescored
 * in FP32 (exact target similarity; per relation, FP32 similarities for every
 * anchor that could attain the maximum) and the TopK is taken among them.
 * The memory must have been built with the matching FARM_BUILD_* flag and the
 * workspace's max_k must cover rescore_mult*k.
 * With FARM_METHOD_BOUNDED / FARM_METHOD_PROPOSAL the candidates (objects
 * whose score can still reach the TopK, at most 2048 per query) are scored
 * exactly -- FP32 similarities, or for a reduced-precision dtype FP32 dot
 * products wherever the error bound leaves the maximum open -- so the result
 * is the exact TopK whenever certified[q] = 1; certified[q] = 0 only when more
 * than 2048 objects qualified (then the 2048 with the largest upper bounds
 * were scored).  PROPOSAL returns the same records as BOUNDED, bit for bit;
 * its tables cover predicates 0..FARM_NUM_PROP_PRED-1, and terms of the other
 * predicates are scanned over all anchors.
 * Errors: INVALID_ARG (shapes, pointers, k, unknown dtype/method/flag bits,
 * host metadata), UNSUPPORTED (missing reduced-precision copy; PROPOSAL
 * without farm_build_proposals), HIP.
 */
FARM_API farm_status farm_query_topk(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t d,
                            const float* target, const int32_t* target_cls, const int32_t* rel_off,
                            const int32_t* rel_pred, const float* rel_anchor,
                            const farm_score_opts* opts, int32_t k, uint32_t* out_id, float* out_score,
                            float* out_terms, uint32_t* out_anchor_id, void* stream);

/* ------------------------------------------------------------------------
 * Multi-channel reciprocal-rank fusion of the unary scores (Appendix
 * "Retrieval Details", step 3: the whole pool ranked per query channel, each
 * channel adding w / (mu + rank), mu = 5; Section "Robust Relational Object
 * Retrieval", implementation paragraph: unary scores fused over the
 * retrieval embeddings stored per entity).  The memory holds several
 * embedding spaces (space 0 is its descriptor table); a query channel is a
 * query vector in one space with a weight.  For every row (targets, then the
 * relations' anchors, analogously):
 *   rank_c(i) = 1 + #{j != i : cos_c(j) > cos_c(i), or equal and id_j < id_i}
 *   fused(i)  = sum_c w_c / (5 + rank_c(i)) / (sum_c w_c / 6)    in (0, 1]
 * and the fused target row takes the class factor; the fused rows replace
 * the clamped cosines as s_sem and sim(a, q_r), and scoring proceeds as in
 * farm_query_topk.  Cosines are FP32 (the FP32 GEMM); the ranks are exact
 * for those values.  Cost per channel: one FP32 GEMM over the space, one
 * bucketed ranking pass per row (quadratic only in the size of groups of
 * equal-bucket cosines).
 * ---------------------------------------------------------------------- */

/* Add an embedding space: desc device [n][d] FP32 (any non-zero norms; n =
   the memory's).  Copies and normalises it.  space_out receives its index
   (1, 2, ...).  At most 7 added spaces.  Errors: INVALID_ARG (non-finite or
   zero-norm row, d out of 1..8192), OOM, HIP. */
FARM_API farm_status farm_add_embedding_space(farm_memory* mem, int32_t d, const float* desc, void* stream,
                                              int32_t* space_out);

typedef struct {
  int32_t space;          /* embedding space (0 = the memory's descriptor table) */
  float weight;           /* w_c > 0 */
  const float* target;    /* device [q][d_space] the targets' query vectors */
  const float* anchor;    /* device [R][d_space] the relations' anchor query vectors, or NULL when R = 0 */
} farm_rrf_channel;

/* The fused rows alone: out device [q + R][n] FP32 (targets, then the relation
   rows).  channels: host array of n_channels (1..8) entries; other arguments
   as in farm_query_topk_rrf. */
FARM_API farm_status farm_rrf_similarity(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t n_channels,
                                         const farm_rrf_channel* channels, const int32_t* target_cls,
                                         const int32_t* rel_off, const int32_t* rel_pred, float* out, void* stream);

/* farm_query_topk with fused unary scores.  opts->dtype must be FARM_F32
   (the fused rows are exact functions of the FP32 cosines; reduced-precision
   forms are UNSUPPORTED); every method works.  The workspace allocates its
   fusion buffers on the first call (one cosine matrix of the workspace's
   shape and per-row ranking scratch). */
FARM_API farm_status farm_query_topk_rrf(const farm_memory* mem, farm_workspace* ws, int32_t q, int32_t n_channels,
                                         const farm_rrf_channel* channels, const int32_t* target_cls,
                                         const int32_t* rel_off, const int32_t* rel_pred, const farm_score_opts* opts,
                                         int32_t k, uint32_t* out_id, float* out_score, float* out_terms,
                                         uint32_t* out_anchor_id, void* stream);

/*
 * farm_query_topk without a workspace and without any allocation, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Arguments, options,
 * results and errors as farm_query_topk (q, d, the query arrays, opts, k and
 * the outputs), minus the workspace.  The call calls no hipMalloc, hipFree,
 * pinned-host or other allocating routine: the scratch it needs (query
 * vectors, similarity matrix, candidate buffers, counters, metadata) is laid
 * out in a static device array of FARM_STATIC_SCRATCH_BYTES that the library
 * holds on every device it runs on until the process ends, and the per-call
 * metadata reaches the device in kernel arguments.
 * Limit: a call whose layout does not fit FARM_STATIC_SCRATCH_BYTES (about
 * q + 2R rows of n floats plus 150 KB per query, e.g. q = 32, R = 96 at
 * n = 20,000) fails with FARM_ERR_INVALID_ARG and a message giving the bytes
 * it needs.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents: calls that overlap on one device (on different streams or
 * from different host threads) race; the caller orders them.  Device query
 * vectors are not validated here (there is no workspace status to report
 * to): a non-finite or zero-norm vector leaves its query's results
 * unspecified.
 */
#define FARM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
FARM_API farm_status farm_query_topk_static(const farm_memory* mem, int32_t q, int32_t d, const float* target,
                                            const int32_t* target_cls, const int32_t* rel_off,
                                            const int32_t* rel_pred, const float* rel_anchor,
                                            const farm_score_opts* opts, int32_t k, uint32_t* out_id,
                                            float* out_score, float* out_terms, uint32_t* out_anchor_id,
                                            void* stream);

/* Phases timed by the workspace's optional phase timer. */
typedef enum {
  FARM_PHASE_NORMALIZE = 0, /* query vector normalisation (and quantisation) */
  FARM_PHASE_GEMM = 1,      /* similarity GEMM */
  FARM_PHASE_PAIR = 2,      /* relational pass (relation terms + composite) */
  FARM_PHASE_TOPK = 3,      /* TopK selection */
  FARM_PHASE_RESCORE = 4,   /* candidate relation terms (one kernel) */
  FARM_PHASE_EXPLAIN = 5,   /* ScoredCandidate breakdown of the winners */
  FARM_PHASE_PROPOSE = 6,   /* semantic anchor sets of the proposal method */
  FARM_PHASE_FALLBACK = 7,  /* full anchor scans of the terms the proposals could not certify */
  FARM_PHASE_SELECT = 8,    /* candidate composite scores and final TopK */
  FARM_PHASE_COUNT = 9
} farm_phase;

/*
 * Phase timer: when enabled, every scoring call on this workspace brackets each
 * phase with HIP events on its stream (a small serialisation cost).  Read the
 * accumulated milliseconds and launch counts per phase with
 * farm_workspace_timings (synchronises the events; resets when reset != 0).
 *   ms     host [FARM_PHASE_COUNT] out, may be NULL
 *   count  host [FARM_PHASE_COUNT] out, may be NULL
 */
FARM_API farm_status farm_workspace_set_timing(farm_workspace* ws, int32_t enable);
FARM_API farm_status farm_workspace_timings(farm_workspace* ws, double* ms, int64_t* count, int32_t reset);

/* ------------------------------------------------------------------------
 * Learned anchor proposal network.
 *
 * The query-time complexity analysis of the paper (Appendix "Robust
 * Relational Retrieval Formulation") bounds the binding cost by the anchor
 * candidate-set size K_a.  This network proposes, per (target, predicate), the
 * anchors worth evaluating; exhaustive scoring stays the fallback and the reference
 * of exactness (see farm_build_proposals).
 *
 *   x  = [u_o (dp) | u_a (dp) | g(o,a) / 4 m (12) | 0]     dp = d rounded up to 64
 *   h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2), y = W3 h2 + b3 (P = FARM_NUM_PROP_PRED
 *   logits, one per farm_pred), GELU(v) = v/2 (1 + erf(v / sqrt 2))
 *   g  = [c_o - c_a (3), e_o (3), e_a (3), |c_o - c_a|, (c_o - c_a).r,
 *         bottom_o - top_a]
 * FP32 master weights and AdamW moments (beta 0.9 / 0.999, eps 1e-8); GEMMs on
 * BF16 copies with FP32 accumulation.  Weights are row-major:
 * W1 [256][in_dim], b1 [256], W2 [256][256], b2 [256], W3 [P][256], b3 [P];
 * in_dim = 2 dp + 64 (unused input columns hold zero weights).
 * ------------------------------------------------------------------------ */
#define FARM_MLP_HIDDEN 256

typedef struct farm_mlp farm_mlp;

/* d: descriptor width of the memories it will serve; max_batch: pairs per
   call (1..2^22); seed: deterministic initialisation. */
FARM_API farm_status farm_mlp_create(int32_t d, int32_t max_batch, uint64_t seed, farm_mlp** out);
FARM_API farm_status farm_mlp_free(farm_mlp* mlp);
FARM_API farm_status farm_mlp_shape(const farm_mlp* mlp, int32_t* in_dim, int32_t* hidden);
/* host FP32 copies of the master weights / of the last step's gradients
   (synchronising); any pointer may be NULL */
FARM_API farm_status farm_mlp_get_weights(const farm_mlp* mlp, float* W1, float* b1, float* W2, float* b2,
                                          float* W3, float* b3);
FARM_API farm_status farm_mlp_get_grads(const farm_mlp* mlp, float* W1, float* b1, float* W2, float* b2,
                                        float* W3, float* b3);
/* Host copies of the last training step's batch tensors, first nb rows
   (synchronising; any pointer may be NULL): pre-activations Z1, Z2 [nb][256]
   FP32, activations A1, A2 [nb][256] BF16, logits Y [nb][FARM_NUM_PROP_PRED]
   FP32, the back-propagated dZ2 [nb][256] BF16, dA1 = dZ2 W2 [nb][256] FP32
   and dZ1 [nb][256] BF16.  They stay valid until the next step, logits or
   table call of this network; for checking each layer on its own inputs. */
FARM_API farm_status farm_mlp_get_batch(const farm_mlp* mlp, int32_t nb, float* Z1, uint16_t* A1, float* Z2,
                                        uint16_t* A2, float* Y, uint16_t* dZ2, float* dA1, uint16_t* dZ1);
FARM_API farm_status farm_mlp_set_weights(farm_mlp* mlp, const float* W1, const float* b1, const float* W2,
                                          const float* b2, const float* W3, const float* b3);
/* Network inputs of nb pairs (device o_idx, a_idx: object indices into mem)
   as BF16 rows x_out [nb][in_dim] (device). */
FARM_API farm_status farm_mlp_inputs(farm_mlp* mlp, const farm_memory* mem, int32_t nb, const int32_t* o_idx,
                                     const int32_t* a_idx, uint16_t* x_out, void* stream);
/* Logits [nb][FARM_NUM_PROP_PRED] (device) of nb pairs. */
FARM_API farm_status farm_mlp_logits(farm_mlp* mlp, const farm_memory* mem, int32_t nb, const int32_t* o_idx,
                                     const int32_t* a_idx, float* logits, void* stream);
/* One training step on nb labelled pairs (device pred [nb] farm_pred,
   label [nb] in {0,1}): forward, mean BCE-with-logits on the labelled
   predicate, backward; with update != 0 an AdamW step (lr, decoupled
   weight_decay on every parameter).  loss_out: device scalar or NULL.
   Pairs whose predicate has no output (id outside 0..FARM_NUM_PROP_PRED-1)
   add nothing to the loss or the gradients (they still count in nb). */
FARM_API farm_status farm_mlp_step(farm_mlp* mlp, const farm_memory* mem, int32_t nb, const int32_t* o_idx,
                                   const int32_t* a_idx, const int32_t* pred, const float* label, float lr,
                                   float weight_decay, int32_t update, float* loss_out, void* stream);

/*
 * Proposal tables of a memory (method FARM_METHOD_PROPOSAL).  For every
 * object o and predicate p < FARM_NUM_PROP_PRED (one network output per
 * predicate) the M anchors a != o with the largest logit y_p of
 * the network on (o, a), their predicate values P_p(o, a), and the largest
 * P_p(o, a) over the anchors left out.  This is the anchor candidate set K_a
 * of the query-time complexity analysis (Appendix "Robust Relational Retrieval
 * Formulation"), learned and query-independent; the exact maximum over all
 * anchors remains the fallback whenever the tables cannot certify a term.
 *   mem     memory to extend (owned tables replace earlier ones; the memory
 *           must not be in use by another stream during the call)
 *   mlp     network with the memory's descriptor width, same device
 *   M       list length, 1..FARM_MAX_K (clamped to n - 1)
 * Memory: n * M * P * 8 bytes + P n * 4 bytes (P = FARM_NUM_PROP_PRED), plus transient chunk buffers
 * (up to 4 GiB for very large n).  Synchronises `stream`.
 * Errors: INVALID_ARG (null, width/device mismatch, M out of range),
 * UNSUPPORTED (n > 500,000), OOM, HIP.
 */
FARM_API farm_status farm_build_proposals(farm_memory* mem, farm_mlp* mlp, int32_t M, void* stream);

/*
 * The non-learned baseline of the same tables: for every object o and
 * predicate p < FARM_NUM_PROP_PRED the M anchors with the largest predicate
 * value P_p(o, a) (ties by id), their values and the largest value left out --
 * the tightest Pout any list of M can have -- ranked without a network.
 * Same layout, certificate, memory and errors as farm_build_proposals; the
 * results of FARM_METHOD_PROPOSAL do not depend on how the lists were ranked,
 * only how often a term falls back to the full scan.
 */
FARM_API farm_status farm_build_proposals_by_value(farm_memory* mem, int32_t M, void* stream);

/*
 * Logits of the table build's forward pass (the factorised first layer that
 * farm_build_proposals ranks anchors by) for targets t0 .. t0 + tc - 1
 * against every anchor of the memory:
 *   logits   device [FARM_NUM_PROP_PRED][tc][n] FP32 (self pairs -INFINITY)
 * 1 <= tc <= 16, tc * n <= 2^22.  Allocates and frees its temporaries;
 * synchronises `stream`.  Errors: INVALID_ARG, OOM, HIP.
 */
FARM_API farm_status farm_mlp_table_logits(farm_mlp* mlp, const farm_memory* mem, int64_t t0, int32_t tc,
                                           float* logits, void* stream);

/*
 * Copy of the proposal tables (stream-ordered device-to-device copies):
 *   m_out  host out: list length M (0 = no tables; nothing else is written)
 *   idx    device [P][n][M] int32 anchor indices (P = FARM_NUM_PROP_PRED), or NULL
 *   val    device [P][n][M] FP32 predicate values (Near/NextTo/On: log P), or NULL
 *   out    device [P][n] FP32 largest value outside each list, or NULL
 */
FARM_API farm_status farm_get_proposals(const farm_memory* mem, int32_t* m_out, int32_t* idx, float* val, float* out,
                                        void* stream);

/*
 * Which form FARM_METHOD_PROPOSAL uses on this memory for a similarity dtype:
 * *in_lds = 1 when each relation's similarity row is staged in LDS (one block
 * per row, the semantic set selected in the same kernel), 0 when the pass
 * gathers similarities from global memory (rows too large for LDS).
 */
FARM_API farm_status farm_proposal_pass_form(const farm_memory* mem, int32_t dtype, int32_t* in_lds);

/*
 * Candidate-scoring counters of a workspace since the last reset (host [4]):
 * stats[0] = (candidate, relation) terms evaluated by FARM_METHOD_PROPOSAL
 *            (by FARM_METHOD_BOUNDED: terms scanned over all anchors),
 * stats[1] = those that fell back to the scan over all anchors,
 * stats[2], stats[3] = FP32 dot products taken, in the proposal pass and in
 *            the scans over all anchors, for anchors whose reduced-precision
 *            bound could not be resolved.
 * Synchronises `stream`; reset != 0 clears the counters afterwards.
 */
FARM_API farm_status farm_workspace_proposal_stats(farm_workspace* ws, int64_t* stats, int32_t reset, void* stream);

/* ------------------------------------------------------------------------
 * Request loop over resident scenes (serving).
 *
 * The paper answers one query at a time and reports its latency (Appendix on
 * query latency); here many queries against several resident scenes are
 * served together.  The loop is driven by the caller: farm_server_progress
 * reaps finished batches and admits new ones, without blocking.
 *   * continuous batching: a free slot takes the pending requests of one scene
 *     (oldest first, up to max_batch_q queries and max_batch_rel relations);
 *     slots run on their own streams, so batches of different scenes overlap;
 *   * admission: each batch needs a workspace of its scene; idle ones are
 *     reused, new ones are created while the workspaces held stay within
 *     hbm_budget bytes (farm_workspace_estimate), idle workspaces of other
 *     scenes are released to make room, and otherwise the requests wait;
 *   * every request's result equals what it gets alone (rows are scored
 *     independently of the batch they ride in).
 * One server is used from one host thread.  Scenes must outlive the server.
 * ------------------------------------------------------------------------ */
typedef struct farm_server farm_server;

typedef struct {
  int32_t slots;          /* concurrent batches (1..64), one stream each */
  int32_t max_batch_q;    /* queries per batch (>= 1) */
  int32_t max_batch_rel;  /* relations per batch (0..8*max_batch_q) */
  int32_t k;              /* TopK of every request (1..FARM_MAX_K) */
  int32_t dtype;          /* farm_dtype of the similarity GEMM */
  int32_t method;         /* farm_method */
  size_t hbm_budget;      /* bytes of workspaces the server may hold */
} farm_server_config;

/* Errors: INVALID_ARG for a configuration outside the ranges above. */
FARM_API farm_status farm_server_create(const farm_server_config* cfg, farm_server** out);
/* Register a resident scene; all scenes share one descriptor width.  The
   first scene allocates the slots' streams and staging buffers.
   Errors: INVALID_ARG (width/device mismatch), UNSUPPORTED (the scene lacks
   the dtype's copy or, for FARM_METHOD_PROPOSAL, its tables), OOM, HIP. */
FARM_API farm_status farm_server_add_scene(farm_server* sv, const farm_memory* mem, int32_t* scene_out);
/* Queue one request (host arrays, copied): target [d], target class (-1 =
   none), r relations with predicates preds [r] and anchor vectors anchors
   [r][d].  Validates on the host (finite, non-zero, predicates, r <= 8 and
   <= max_batch_rel) so that a bad request never reaches a batch. */
FARM_API farm_status farm_server_submit(farm_server* sv, int32_t scene, int32_t d, const float* target,
                                        int32_t target_cls, int32_t r, const int32_t* preds, const float* anchors,
                                        uint64_t* request_id);
/* Cancel a pending or in-flight request; it completes with status 1 and the
   other requests of its batch are unaffected. */
FARM_API farm_status farm_server_cancel(farm_server* sv, uint64_t request_id);
/* Reap finished batches, admit new ones.  busy_slots / pending: host out or NULL. */
FARM_API farm_status farm_server_progress(farm_server* sv, int32_t* busy_slots, int32_t* pending);
/* Completed requests in completion order, at most max_results (host arrays,
   each may be NULL): request ids, status (0 done, 1 cancelled, 2 failed),
   certified flag, latency from submit to the progress call that saw it
   finish (ns), TopK ids [max_results][k] and scores. */
FARM_API farm_status farm_server_poll(farm_server* sv, int32_t max_results, uint64_t* ids, int32_t* status,
                                      int32_t* certified, int64_t* latency_ns, uint32_t* topk_ids,
                                      float* topk_scores, int32_t* n_out);
/* stats [5]: batches launched, admissions deferred, workspaces released to
   make room, bytes held, workspaces held. */
FARM_API farm_status farm_server_stats(const farm_server* sv, int64_t* stats);
/* Waits for the slots' streams, frees the workspaces and buffers. */
FARM_API farm_status farm_server_free(farm_server* sv);

/*
 * Synchronise `stream` and report whether any scoring call since the last
 * check saw an invalid device input vector (FARM_ERR_INVALID_ARG) -- then
 * clear the flag.
 */
FARM_API farm_status farm_workspace_status(farm_workspace* ws, void* stream);

/* Message for the calling thread's last failure ("" if none). */
FARM_API const char* farm_last_error(void);

/* Library version string. */
FARM_API const char* farm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FARM_H */
