/*
 * farm_oracle.c -- plain, slow, FP64 reference for FARM's query-time
 * relational scoring.  TEST INFRASTRUCTURE ONLY: only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library.  It
 * shares no code, header or constant table with the GPU library.
 *
 * What it computes (paper, Section 2.3 "Executable query specification and
 * compositional retrieval"; Appendix "Robust Relational Retrieval
 * Formulation", soft verification and query-time complexity; Appendix
 * "Retrieval Details", steps 3-5 and the "Why soft, not hard?" paragraph):
 *
 *   sim(i, v)   = max(0, <u_i, v^>), u_i and v^ the L2-normalised descriptor
 *                 and query vector (unary score s_sigma in [0, 1]);
 *   s_sem(i)    = kappa_i * sim(i, q_t), kappa_i = 0.3 when both the parsed
 *                 target class and the object's class are known and differ
 *                 (composite-scoring step: the soft class factor), else 1;
 *   t_r(i)      = max_{j != i} sim(j, q_r) * P_{p_r}(i, j)
 *                 (greedy binding of each anchor of the star-shaped query:
 *                 conditioning on the target separates the anchors, so the
 *                 joint maximum over bindings is the per-relation maximum);
 *   b_r(i)      = the maximising anchor's object id (smallest id on ties);
 *   gbar(i)     = (prod_r t_r(i))^(1/R), 1 when R = 0 (geometric mean of the
 *                 predicate scores);
 *   s(i)        = s_sem(i) * ((1 - w) + w * gbar(i)), w = 0.5;
 *   TopK        = the first min(K, N) objects ordered by (s desc, id asc).
 *
 * Predicates (Appendix "Retrieval Details", predicate evaluation), with
 * D = c_i - c_j the target-minus-anchor box-center offset and sig(u) the
 * logistic function:
 *   NEAR     = exp(-|D|^2 / (2 * 0.5^2))          (Gaussian, sigma = 0.5 m)
 *   ABOVE    = sig(D_z / 0.1),  BELOW = sig(-D_z / 0.1)
 *   RIGHT_OF = sig((D_x r_x + D_y r_y) / 0.1),  LEFT_OF = sig(-(...) / 0.1)
 *   NEXT_TO  = exp(-|D|^2 / (2 * 1.0^2))
 *   IN_FRONT_OF = sig(-(D_x f_x + D_y f_y) / 0.1),  BEHIND = sig(+(...) / 0.1)
 *   ON       = exp(-(D_x^2 + D_y^2) / (2 * 0.5^2)) * exp(-g^2 / (2 * 0.125^2)),
 *              g = (c_i,z - e_i,z / 2) - (c_j,z + e_j,z / 2)
 *   CLOSEST  = 1 / rank,  FARTHEST = 1 / (last rank - rank + 1): the rank of i
 *              among the query's candidates by distance to j (see rank_value)
 *   INSIDE   = prod_k sig((e_j,k / 2 - |D_k|) / 0.1): i's center within j's box
 *   BETWEEN  (ternary, two anchors j1, j2; see between_value) = sig(s / 0.1)
 *              sig((L - s) / 0.1) exp(-h^2 / (2 * 0.5^2)): s the offset of i's
 *              center along the axis from j1 to j2, L = |c_j2 - c_j1|, h its
 *              distance from that axis; 0 when L = 0.  Its anchors range over
 *              candidate sets of 64 (see between_set)
 * where (r_x, r_y) is the scene viewer's right vector, f = (-r_y, r_x) its
 * viewing direction and e the full box extents.
 *
 * With entity Gaussians and stored views (Section "Memory Construction": each
 * entity's 3D Gaussian N(mu, Sigma), mu its center, and its representative
 * posed views; Section "Robust Relational Object Retrieval", implementation
 * paragraph: Hellinger distance for Near; Appendix "Retrieval Details", step
 * 4: the viewpoint-dependent predicates in stored camera views of the target
 * candidate):
 *   NEAR_H   = 1 - H(N_i, N_j), H^2 = 1 - BC, BC the Bhattacharyya
 *              coefficient of the two Gaussians (see hellinger_near)
 *   LEFT_OF_V / RIGHT_OF_V = sig(+-(u_j - u_i) / 0.05), u = x_c / z_c the
 *              horizontal image-plane coordinate of a center in target i's
 *              stored view; IN_FRONT_OF_V / BEHIND_V = sig(+-(z_j - z_i) /
 *              0.1), z the camera-frame depth; 0 unless both centers are in
 *              that view (see view_predicate).
 * The temperatures
 * (0.1 m), the Gaussian's normalisation, the clamp at zero, the viewer
 * convention and On's Gaussian gate and band with their widths are readings
 * where the paper is silent.
 *
 * Everything is computed in double precision from the float inputs, with plain
 * loops in the order of the definition.  OpenMP parallelises only independent
 * loops: over the objects of a query (full scores) or over queries (sampled
 * pairs, bounded TopK).
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_W 0.5
#define ORACLE_CLASS_FACTOR 0.3
#define ORACLE_NEAR_SIGMA 0.5
#define ORACLE_NEXT_TO_SIGMA 1.0
#define ORACLE_TAU 0.1
#define ORACLE_ON_SIGMA_H 0.5
#define ORACLE_ON_SIGMA_V 0.125
#define ORACLE_MAX_REL 8
#define ORACLE_NO_ID 0xFFFFFFFFu

enum { P_NEAR = 0, P_ABOVE = 1, P_BELOW = 2, P_LEFT_OF = 3, P_RIGHT_OF = 4, P_NEXT_TO = 5, P_IN_FRONT_OF = 6,
       P_BEHIND = 7, P_ON = 8, P_CLOSEST = 9, P_FARTHEST = 10, P_INSIDE = 11, P_BETWEEN = 12, P_AND = 13,
       P_NEAR_H = 14, P_LEFT_OF_V = 15, P_RIGHT_OF_V = 16, P_IN_FRONT_OF_V = 17, P_BEHIND_V = 18,
       P_COUNT = 19 };

static double logistic(double u) { return 1.0 / (1.0 + exp(-u)); }

/* Soft predicate P_p(i, j) for target center ci and anchor center cj, full
 * box extents ei and ej (Appendix "Retrieval Details", closed-form
 * evaluators): Near and NextTo are Gaussians of the centroid distance (sigma
 * 0.5 m and 1.0 m); Above/Below a logistic of the vertical offset;
 * LeftOf/RightOf a logistic of the offset along the viewer's right axis r,
 * InFrontOf/Behind of the offset along its viewing direction f = (-r_y, r_x)
 * (in front = nearer the viewer), one viewer frame per scene standing in for
 * the stored camera views; temperature 0.1 m.  On is a gate on the horizontal
 * center distance times a band on the vertical gap between the target's bottom
 * face and the anchor's top face, both Gaussians (sigma 0.5 m and 0.125 m). */
double oracle_predicate(int p, const double* ci, const double* cj, const double* ei, const double* ej,
                        const double* right) {
    double dx = ci[0] - cj[0], dy = ci[1] - cj[1], dz = ci[2] - cj[2];
    double depth = dx * -right[1] + dy * right[0];  /* offset along f */
    switch (p) {
    case P_NEAR: {
        double d2 = dx * dx + dy * dy + dz * dz;
        return exp(-d2 / (2.0 * ORACLE_NEAR_SIGMA * ORACLE_NEAR_SIGMA));
    }
    case P_NEXT_TO: {
        double d2 = dx * dx + dy * dy + dz * dz;
        return exp(-d2 / (2.0 * ORACLE_NEXT_TO_SIGMA * ORACLE_NEXT_TO_SIGMA));
    }
    case P_ABOVE: return logistic(dz / ORACLE_TAU);
    case P_BELOW: return logistic(-dz / ORACLE_TAU);
    case P_RIGHT_OF: return logistic((dx * right[0] + dy * right[1]) / ORACLE_TAU);
    case P_LEFT_OF: return logistic(-(dx * right[0] + dy * right[1]) / ORACLE_TAU);
    case P_IN_FRONT_OF: return logistic(-depth / ORACLE_TAU);
    case P_BEHIND: return logistic(depth / ORACLE_TAU);
    case P_INSIDE: {
        /* a soft containment test: along each axis the target's center lies
         * within the anchor's half extent (logistic of the margin, 0.1 m) */
        double v = 1.0;
        for (int k = 0; k < 3; ++k) v *= logistic((0.5 * ej[k] - fabs(ci[k] - cj[k])) / ORACLE_TAU);
        return v;
    }
    case P_ON: {
        double h2 = dx * dx + dy * dy;
        double gap = (ci[2] - 0.5 * ei[2]) - (cj[2] + 0.5 * ej[2]);  /* bottom of i minus top of j */
        double gate = exp(-h2 / (2.0 * ORACLE_ON_SIGMA_H * ORACLE_ON_SIGMA_H));
        double band = exp(-gap * gap / (2.0 * ORACLE_ON_SIGMA_V * ORACLE_ON_SIGMA_V));
        return gate * band;
    }
    default: return NAN;
    }
}

/* Exported wrapper so tests can pin single predicate values. */
double farm_oracle_predicate(int p, const float* ci, const float* cj, const float* ei, const float* ej,
                             const float* right) {
    double a[3] = {ci[0], ci[1], ci[2]}, b[3] = {cj[0], cj[1], cj[2]}, r[2] = {right[0], right[1]};
    double ea[3] = {ei[0], ei[1], ei[2]}, eb[3] = {ej[0], ej[1], ej[2]};
    return oracle_predicate(p, a, b, ea, eb, r);
}

/* Between(i; j1, j2) (Appendix "Retrieval Details": a predicate of the
 * vocabulary; Appendix "Robust Relational Retrieval Formulation", query-time
 * complexity: a higher-arity predicate coupling the target and two anchors).
 * The paper gives no form; reading: i lies between the anchors when its
 * center projects inside the segment joining their centers -- both margins
 * along the axis positive, each a logistic with the other sigmoids'
 * temperature (0.1 m) -- and lies near that axis -- Near's Gaussian (0.5 m) of
 * the perpendicular distance.  Symmetric in j1, j2; 0 for coincident anchors. */
static double between_value(const double* ci, const double* c1, const double* c2) {
    double u[3], w[3];
    for (int k = 0; k < 3; ++k) { u[k] = c2[k] - c1[k]; w[k] = ci[k] - c1[k]; }
    double L2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (L2 == 0.0) return 0.0;
    double L = sqrt(L2);
    double s = (w[0] * u[0] + w[1] * u[1] + w[2] * u[2]) / L;
    double h2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2] - s * s;
    if (h2 < 0.0) h2 = 0.0;
    return logistic(s / ORACLE_TAU) * logistic((L - s) / ORACLE_TAU) *
           exp(-h2 / (2.0 * ORACLE_NEAR_SIGMA * ORACLE_NEAR_SIGMA));
}

double farm_oracle_between(const float* ci, const float* c1, const float* c2) {
    double a[3] = {ci[0], ci[1], ci[2]}, b[3] = {c1[0], c1[1], c1[2]}, c[3] = {c2[0], c2[1], c2[2]};
    return between_value(a, b, c);
}

/* ------------------------------------------------ Gaussians and stored views */

/* A symmetric 3x3 matrix from its packed upper triangle (xx, xy, xz, yy, yz, zz). */
static void unpack_sym(const double* p6, double m[3][3]) {
    m[0][0] = p6[0]; m[0][1] = p6[1]; m[0][2] = p6[2];
    m[1][0] = p6[1]; m[1][1] = p6[3]; m[1][2] = p6[4];
    m[2][0] = p6[2]; m[2][1] = p6[4]; m[2][2] = p6[5];
}

static double det3(double m[3][3]) {
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
           m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

/* v^T m^-1 v: solve m x = v by Cramer's rule (column k of m replaced by v). */
static double inverse_quadratic_form(double m[3][3], const double* v) {
    double d = det3(m), q = 0.0;
    for (int k = 0; k < 3; ++k) {
        double c[3][3];
        for (int r = 0; r < 3; ++r)
            for (int col = 0; col < 3; ++col) c[r][col] = (col == k) ? v[r] : m[r][col];
        q += v[k] * det3(c) / d;
    }
    return q;
}

/* Near over entity Gaussians (Section "Robust Relational Object Retrieval",
 * implementation paragraph: the Hellinger distance for Near; the Gaussian
 * N(mu, Sigma) of each entity, Section "Memory Construction").  The
 * Bhattacharyya coefficient of N(mu_i, A) and N(mu_j, B) with M = (A + B) / 2
 * is BC = det(A)^(1/4) det(B)^(1/4) / det(M)^(1/2) exp(-(mu_i - mu_j)^T M^-1
 * (mu_i - mu_j) / 8), the squared Hellinger distance H^2 = 1 - BC, and the
 * soft relation -- a membership in [0, 1] that is 1 for identical Gaussians --
 * is 1 - H (a reading: the paper names the distance, not the map). */
static double hellinger_near(const double* ci, const double* cov_i, const double* cj, const double* cov_j) {
    double A[3][3], B[3][3], M[3][3];
    unpack_sym(cov_i, A);
    unpack_sym(cov_j, B);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[r][c] = 0.5 * (A[r][c] + B[r][c]);
    double dmu[3] = {ci[0] - cj[0], ci[1] - cj[1], ci[2] - cj[2]};
    double q = inverse_quadratic_form(M, dmu);
    double bc = pow(det3(A), 0.25) * pow(det3(B), 0.25) / sqrt(det3(M)) * exp(-q / 8.0);
    double h2 = 1.0 - bc;
    if (h2 < 0.0) h2 = 0.0;
    return 1.0 - sqrt(h2);
}

/* A stored view: the camera center p (3) and the rows of the world-to-camera
 * rotation R (9: the camera's right, down and forward axes in world
 * coordinates), so that a point x has camera coordinates R (x - p), depth
 * along the third. */
#define ORACLE_VIEW_TAU_U 0.05   /* temperature of the image-plane offset (normalised coordinates) */
#define ORACLE_VIEW_Z_MIN 0.1    /* a center is in the view when its depth is at least 0.1 m ... */
#define ORACLE_VIEW_HALF_W 1.0   /* ... and it projects within the 90 x 73.7 degree field of view */
#define ORACLE_VIEW_HALF_H 0.75

static void camera_coords(const double* view, const double* x, double* xc) {
    double w[3] = {x[0] - view[0], x[1] - view[1], x[2] - view[2]};
    for (int r = 0; r < 3; ++r) xc[r] = view[3 + 3 * r] * w[0] + view[4 + 3 * r] * w[1] + view[5 + 3 * r] * w[2];
}

static int in_view(const double* xc) {
    return xc[2] >= ORACLE_VIEW_Z_MIN && fabs(xc[0]) <= ORACLE_VIEW_HALF_W * xc[2] &&
           fabs(xc[1]) <= ORACLE_VIEW_HALF_H * xc[2];
}

/* The viewpoint-dependent predicates in a stored camera view of the target
 * candidate i (Appendix "Retrieval Details", step 4): left/right from the
 * anchor-relative horizontal offset of the two objects on the image plane,
 * front/behind from their relative camera-frame depth.  Readings: the view is
 * the target's first stored view; a center stands in for its mask centroid
 * (projected at u = x_c / z_c); the offsets pass through the logistic with
 * temperature 0.05 (image plane) and 0.1 m (depth); an object outside the
 * view (behind the near plane at 0.1 m or outside the field of view) gives 0. */
static double view_predicate(int p, const double* view_i, const double* ci, const double* cj) {
    double a[3], b[3];
    camera_coords(view_i, ci, a);
    camera_coords(view_i, cj, b);
    if (!in_view(a) || !in_view(b)) return 0.0;
    double ua = a[0] / a[2], ub = b[0] / b[2];
    switch (p) {
    case P_LEFT_OF_V: return logistic((ub - ua) / ORACLE_VIEW_TAU_U);
    case P_RIGHT_OF_V: return logistic((ua - ub) / ORACLE_VIEW_TAU_U);
    case P_IN_FRONT_OF_V: return logistic((b[2] - a[2]) / ORACLE_TAU);
    case P_BEHIND_V: return logistic((a[2] - b[2]) / ORACLE_TAU);
    default: return NAN;
    }
}

/* Exported for pins: one value of the predicates above for float inputs
 * (cov: packed 6-vectors of target and anchor; view: the target's view). */
double farm_oracle_hellinger_near(const float* ci, const float* cov_i, const float* cj, const float* cov_j) {
    double a[3] = {ci[0], ci[1], ci[2]}, b[3] = {cj[0], cj[1], cj[2]}, A[6], B[6];
    for (int k = 0; k < 6; ++k) { A[k] = cov_i[k]; B[k] = cov_j[k]; }
    return hellinger_near(a, A, b, B);
}

double farm_oracle_view_predicate(int p, const float* view_i, const float* ci, const float* cj) {
    double v[12], a[3] = {ci[0], ci[1], ci[2]}, b[3] = {cj[0], cj[1], cj[2]};
    for (int k = 0; k < 12; ++k) v[k] = view_i[k];
    return view_predicate(p, v, a, b);
}

/* Entity Gaussians [n][6] and stored views [n][12] of the scene the next
 * scoring calls receive (NULL: the scene has none); the arrays must stay
 * valid until cleared.  Predicates that need them fail (-1) without them. */
static const float* g_cov = NULL;
static const float* g_view = NULL;
static int64_t g_ext_n = -1;

void farm_oracle_set_entity_geometry(int64_t n, const float* cov6, const float* view12) {
    g_ext_n = n;
    g_cov = cov6;
    g_view = view12;
}

static void unit_vector(const float* v, int d, double* out) {
    double ss = 0.0;
    for (int k = 0; k < d; ++k) ss += (double)v[k] * (double)v[k];
    double nrm = sqrt(ss);
    for (int k = 0; k < d; ++k) out[k] = (double)v[k] / nrm;
}

static double clamped_cosine(const double* u, const double* v, int d) {
    double dot = 0.0;
    for (int k = 0; k < d; ++k) dot += u[k] * v[k];
    return dot > 0.0 ? dot : 0.0;
}

typedef struct {
    int64_t n;
    int d;
    double* u;        /* [n][d] normalised descriptors */
    double* c;        /* [n][3] centers */
    double* e;        /* [n][3] full extents */
    const uint32_t* id;
    const int32_t* cls;
    double right[2];
    double* cov;      /* [n][6] packed entity covariances, or NULL */
    double* view;     /* [n][12] stored views, or NULL */
} scene64;

static int scene_init(scene64* s, int64_t n, int d, const float* desc, const float* center,
                      const float* extent, const uint32_t* id, const int32_t* cls, const float* right) {
    s->n = n;
    s->d = d;
    s->cov = NULL;
    s->view = NULL;
    s->u = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)d);
    s->c = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 3);
    s->e = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 3);
    if (!s->u || !s->c || !s->e) return -2;
    for (int64_t i = 0; i < n; ++i) {
        unit_vector(desc + (size_t)i * d, d, s->u + (size_t)i * d);
        for (int k = 0; k < 3; ++k) s->c[i * 3 + k] = center[i * 3 + k];
        for (int k = 0; k < 3; ++k) s->e[i * 3 + k] = extent[i * 3 + k];
    }
    s->id = id;
    s->cls = cls;
    s->right[0] = right[0];
    s->right[1] = right[1];
    if (g_ext_n == n && g_cov) {
        s->cov = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 6);
        if (!s->cov) return -2;
        for (int64_t k = 0; k < n * 6; ++k) s->cov[k] = g_cov[k];
    }
    if (g_ext_n == n && g_view) {
        s->view = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * 12);
        if (!s->view) return -2;
        for (int64_t k = 0; k < n * 12; ++k) s->view[k] = g_view[k];
    }
    return 0;
}

static void scene_free(scene64* s) {
    free(s->u);
    free(s->c);
    free(s->e);
    free(s->cov);
    free(s->view);
}

static int is_view_pred(int p) { return p >= P_LEFT_OF_V && p <= P_BEHIND_V; }

/* P_p(i, j) of every pairwise predicate but the rank ones and Between. */
static double pair_value(const scene64* s, int p, int64_t i, int64_t j) {
    if (p == P_NEAR_H) return hellinger_near(s->c + i * 3, s->cov + i * 6, s->c + j * 3, s->cov + j * 6);
    if (is_view_pred(p)) return view_predicate(p, s->view + i * 12, s->c + i * 3, s->c + j * 3);
    return oracle_predicate(p, s->c + i * 3, s->c + j * 3, s->e + i * 3, s->e + j * 3, s->right);
}

/* Queries that name a Gaussian or view predicate need the scene to carry them. */
static int check_scene_geometry(const scene64* s, int32_t q, const int32_t* rel_off, const int32_t* rel_pred) {
    for (int32_t r = 0; r < rel_off[q]; ++r) {
        if (rel_pred[r] == P_NEAR_H && !s->cov) return -1;
        if (is_view_pred(rel_pred[r]) && !s->view) return -1;
    }
    return 0;
}

/* Per-query state: normalised target, anchor similarities per relation. */
typedef struct {
    int r;                      /* number of relations */
    int32_t tcls;               /* parsed target class (-1: none) */
    int pred[ORACLE_MAX_REL];
    double* sem;                /* [n]  s_sem(i) */
    double* asim;               /* [r][n] sim(j, q_r) */
} query64;

/* Unary scores supplied from outside (farm_oracle_set_similarities): the
 * target rows s_sem [q][n], class factor included, and the relation rows
 * sim(j, q_r) [r_tot][n] of the next scoring calls, in place of the clamped
 * cosines of the query vectors -- for a unary score with another definition
 * (the multi-channel reciprocal-rank fusion of oracle/rrf.py).  NULL: cosines. */
static const double* g_sim_sem = NULL;
static const double* g_sim_asim = NULL;
static int64_t g_sim_n = -1;
static int32_t g_sim_q = -1, g_sim_r = -1;

void farm_oracle_set_similarities(int32_t q, int32_t r_tot, int64_t n, const double* sem, const double* asim) {
    g_sim_q = q;
    g_sim_r = r_tot;
    g_sim_n = n;
    g_sim_sem = sem;
    g_sim_asim = asim;
}

/* query k of the batch (its relations start at row r0) */
static int query_init(query64* qs, const scene64* s, int32_t k, int32_t r0, const float* target, int32_t tcls,
                      int r, const int32_t* pred, const float* anchors) {
    int64_t n = s->n;
    int d = s->d;
    qs->r = r;
    qs->tcls = tcls;
    qs->sem = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    qs->asim = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)(r > 0 ? r : 1));
    double* v = (double*)malloc(sizeof(double) * (size_t)d);
    if (!qs->sem || !qs->asim || !v) { free(v); return -2; }
    if (g_sim_sem && g_sim_n == n && k < g_sim_q && r0 + r <= g_sim_r) {
        for (int64_t i = 0; i < n; ++i) qs->sem[i] = g_sim_sem[(size_t)k * n + i];
        for (int rr = 0; rr < r; ++rr) {
            qs->pred[rr] = pred[rr];
            for (int64_t j = 0; j < n; ++j) qs->asim[(size_t)rr * n + j] = g_sim_asim[(size_t)(r0 + rr) * n + j];
        }
        free(v);
        return 0;
    }
    unit_vector(target, d, v);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double kappa = (tcls >= 0 && s->cls && s->cls[i] >= 0 && s->cls[i] != tcls) ? ORACLE_CLASS_FACTOR : 1.0;
        qs->sem[i] = kappa * clamped_cosine(s->u + (size_t)i * d, v, d);
    }
    for (int rr = 0; rr < r; ++rr) {
        qs->pred[rr] = pred[rr];
        unit_vector(anchors + (size_t)rr * d, d, v);
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j) qs->asim[(size_t)rr * n + j] = clamped_cosine(s->u + (size_t)j * d, v, d);
    }
    free(v);
    return 0;
}

static void query_free(query64* qs) {
    free(qs->sem);
    free(qs->asim);
}

/* Closest / Farthest (Appendix "Retrieval Details": a rank within the
 * candidate set, scored 1 / (|rank - r*| + 1)).  Readings: the candidate set C
 * holds the objects of the query's parsed target class (every object when the
 * query or the scene has no class); for target i and anchor j the rank is one
 * plus the number of other candidates c (c != i, c != j) nearer to j than i,
 * equal distances ordered by object id; r* = 1 for Closest and the last rank,
 * |C minus i and j| + 1, for Farthest.  Distances are the Euclidean distances
 * of the box centers, compared as squared distances in double precision from
 * the double differences of the float centers. */
static double dist2(const double* c, int64_t a, int64_t b) {
    double dx = c[a * 3] - c[b * 3];
    double dy = c[a * 3 + 1] - c[b * 3 + 1];
    double dz = c[a * 3 + 2] - c[b * 3 + 2];
    return dx * dx + dy * dy + dz * dz;
}

/* Threads the parallel loops use (OpenMP's maximum), and a way to set it. */
int farm_oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void farm_oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static int is_rank_pred(int p) { return p == P_CLOSEST || p == P_FARTHEST; }

/* Tie-aware mode of the rank predicates, for checking another implementation
 * that compares distances at a lower precision (a check, not a reading of the
 * paper).  mode 0 (default): the exact rank above.  mode -1 / +1: every
 * candidate whose squared distance to j lies within a relative rank_eps of
 * i's, |d_c - d_i| <= rank_eps (d_c + d_i), may be ordered either way; the
 * value returned is the lowest / highest 1 / (|rank - r*| + 1) over the ranks
 * this allows.  Set per call by farm_oracle_set_rank_tolerance. */
static int g_rank_mode = 0;
static double g_rank_eps = 0.0;

void farm_oracle_set_rank_tolerance(int mode, double eps) {
    g_rank_mode = mode < 0 ? -1 : (mode > 0 ? 1 : 0);
    g_rank_eps = eps > 0.0 ? eps : 0.0;
}

static double rank_value(const scene64* s, int32_t tcls, int p, int64_t i, int64_t j) {
    double dij = dist2(s->c, i, j);
    int64_t nearer = 0, open = 0, m = 0;
    for (int64_t c = 0; c < s->n; ++c) {
        if (c == i || c == j) continue;
        if (tcls >= 0 && s->cls && s->cls[c] != tcls) continue;
        ++m;
        double dc = dist2(s->c, c, j);
        if (g_rank_mode != 0 && fabs(dc - dij) <= g_rank_eps * (dc + dij)) { ++open; continue; }
        if (dc < dij || (dc == dij && s->id[c] < s->id[i])) ++nearer;
    }
    int64_t rstar = p == P_CLOSEST ? 1 : m + 1;
    int64_t lo = nearer + 1, hi = nearer + 1 + open;  /* the ranks i can take */
    int64_t dlo = lo > rstar ? lo - rstar : rstar - lo;
    int64_t dhi = hi > rstar ? hi - rstar : rstar - hi;
    int64_t off;
    if (g_rank_mode < 0) off = dlo > dhi ? dlo : dhi;                       /* farthest from r* */
    else if (g_rank_mode > 0) off = (lo <= rstar && rstar <= hi) ? 0 : (dlo < dhi ? dlo : dhi);
    else off = dlo;                                                           /* open = 0: lo = hi */
    return 1.0 / (double)(off + 1);
}

/* Between's candidate sets.  Bucket elimination of a factor over two anchor
 * variables costs K^2 per target for candidate sets of K anchors (Appendix
 * "Robust Relational Retrieval Formulation", query-time complexity: the cost
 * grows with the candidate-set size); reading: each of Between's anchor
 * variables ranges over the ORACLE_BETWEEN_K anchors of largest similarity to
 * its description (ties by the smaller id) -- the paper's per-anchor
 * candidate sets K_a -- where the binary relations take every anchor.
 * set[k] = object indices, returns the set's size (min(K, n)).
 * Tie-aware mode (a check of another implementation's similarity rounding,
 * see farm_oracle_set_between_tolerance): mode -1 keeps only the members
 * whose similarity exceeds the K-th largest by more than eps (surely in any
 * set computed within eps), mode +1 adds every anchor within eps of it. */
#define ORACLE_BETWEEN_K 64
static int g_btw_mode = 0;
static double g_btw_eps = 0.0;

void farm_oracle_set_between_tolerance(int mode, double eps) {
    g_btw_mode = mode < 0 ? -1 : (mode > 0 ? 1 : 0);
    g_btw_eps = eps > 0.0 ? eps : 0.0;
}

static int64_t between_set(const scene64* s, const double* a, int64_t* set) {
    int64_t k = s->n < ORACLE_BETWEEN_K ? s->n : ORACLE_BETWEEN_K;
    unsigned char* taken = (unsigned char*)calloc((size_t)(s->n > 0 ? s->n : 1), 1);
    if (!taken) return 0;
    double kth = 0.0;
    for (int64_t r = 0; r < k; ++r) {  /* selection by repeated scans */
        int64_t best = -1;
        for (int64_t j = 0; j < s->n; ++j) {
            if (taken[j]) continue;
            if (best < 0 || a[j] > a[best] || (a[j] == a[best] && s->id[j] < s->id[best])) best = j;
        }
        taken[best] = 1;
        kth = a[best];
    }
    int64_t m = 0;
    for (int64_t j = 0; j < s->n; ++j) {
        int in = taken[j];
        if (g_btw_mode < 0 && in && !(a[j] > kth + g_btw_eps)) in = k == s->n;  /* all anchors: surely in */
        if (g_btw_mode > 0 && !in && a[j] >= kth - g_btw_eps) in = 1;
        if (in) set[m++] = j;
    }
    free(taken);
    return m;
}

/* Between's term: max over j1 in the first set, j2 in the second, j1 != j2,
 * both != i, of sim(j1, q_rr) sim(j2, q_rr+1) Between(i; j1, j2) (the two
 * relation slots rr, rr + 1 hold the two anchor descriptions); ties by the
 * smaller (id(j1), id(j2)); no binding (NO_ID) when the term is 0. */
static void between_term(const scene64* s, const query64* qs, int rr, int64_t i, double* t, uint32_t* b1,
                         uint32_t* b2) {
    const double* a1 = qs->asim + (size_t)rr * s->n;
    const double* a2 = qs->asim + (size_t)(rr + 1) * s->n;
    int64_t* set1 = (int64_t*)malloc(sizeof(int64_t) * (size_t)(s->n > 0 ? s->n : 1));
    int64_t* set2 = (int64_t*)malloc(sizeof(int64_t) * (size_t)(s->n > 0 ? s->n : 1));
    double best = 0.0;
    uint32_t id1 = ORACLE_NO_ID, id2 = ORACLE_NO_ID;
    int64_t m1 = set1 ? between_set(s, a1, set1) : 0, m2 = set2 ? between_set(s, a2, set2) : 0;
    for (int64_t u = 0; u < m1; ++u) {
        const int64_t j1 = set1[u];
        if (j1 == i) continue;
        for (int64_t w = 0; w < m2; ++w) {
            const int64_t j2 = set2[w];
            if (j2 == i || j2 == j1) continue;
            double v = a1[j1] * a2[j2] * between_value(s->c + i * 3, s->c + j1 * 3, s->c + j2 * 3);
            if (v <= 0.0) continue;
            if (v > best || (v == best && (s->id[j1] < id1 || (s->id[j1] == id1 && s->id[j2] < id2)))) {
                best = v;
                id1 = s->id[j1];
                id2 = s->id[j2];
            }
        }
    }
    free(set1);
    free(set2);
    *t = best;
    *b1 = id1;
    if (b2) *b2 = id2;
}

/* t_r(i) and b_r(i): exhaustive maximum over anchors j != i. */
static void relation_term(const scene64* s, const query64* qs, int rr, int64_t i, double* t, uint32_t* b) {
    if (qs->pred[rr] == P_BETWEEN) { between_term(s, qs, rr, i, t, b, NULL); return; }
    double best = -1.0;
    uint32_t best_id = ORACLE_NO_ID;
    const double* a = qs->asim + (size_t)rr * s->n;
    const int p = qs->pred[rr];
    for (int64_t j = 0; j < s->n; ++j) {
        if (j == i) continue;
        double v = a[j] * (is_rank_pred(p) ? rank_value(s, qs->tcls, p, i, j) : pair_value(s, p, i, j));
        if (v > best || (v == best && s->id[j] < best_id)) {
            best = v;
            best_id = s->id[j];
        }
    }
    if (best < 0.0) best = 0.0; /* N = 1: no anchor exists */
    *t = best;
    *b = best_id;
}

/* Every slot's term and binding of object i.  A Between invocation spans two
 * slots: both report its term, the first binds j1 and the second j2. */
static void query_terms(const scene64* s, const query64* qs, int64_t i, double* t, uint32_t* b) {
    for (int rr = 0; rr < qs->r; ++rr) {
        if (qs->pred[rr] == P_BETWEEN) {
            between_term(s, qs, rr, i, &t[rr], &b[rr], &b[rr + 1]);
            t[rr + 1] = t[rr];
            ++rr;
        } else {
            relation_term(s, qs, rr, i, &t[rr], &b[rr]);
        }
    }
}

/* The composite over the query's predicate invocations: geometric mean of the
 * terms (a Between invocation's two slots count once). */
static double composite(double sem, int r, const double* t, const int* pred) {
    double gbar = 1.0;
    double prod = 1.0;
    int cnt = 0;
    for (int rr = 0; rr < r; ++rr) {
        if (pred[rr] == P_AND) continue;
        prod *= t[rr];
        ++cnt;
    }
    if (cnt > 0) gbar = pow(prod, 1.0 / (double)cnt);
    return sem * ((1.0 - ORACLE_W) + ORACLE_W * gbar);
}

static int check_query_meta(int32_t q, const int32_t* rel_off, const int32_t* rel_pred) {
    if (rel_off[0] != 0) return -1;
    for (int32_t k = 0; k < q; ++k) {
        int r = rel_off[k + 1] - rel_off[k];
        if (r < 0 || r > ORACLE_MAX_REL) return -1;
        for (int rr = rel_off[k]; rr < rel_off[k + 1]; ++rr) {
            if (rel_pred[rr] < 0 || rel_pred[rr] >= P_COUNT) return -1;
            /* Between's second anchor follows it in the same query, and only there */
            if (rel_pred[rr] == P_BETWEEN && (rr + 1 >= rel_off[k + 1] || rel_pred[rr + 1] != P_AND)) return -1;
            if (rel_pred[rr] == P_AND && (rr == rel_off[k] || rel_pred[rr - 1] != P_BETWEEN)) return -1;
        }
    }
    return 0;
}

/*
 * Full scores for every (query, object).
 *   scores[q][n]          composite scores
 *   sem[q][n]             s_sem (may be NULL)
 *   rel_terms[r_tot][n]   t_r (may be NULL)
 *   rel_anchor_id[r_tot][n] b_r (may be NULL)
 * Returns 0, -1 on invalid metadata, -2 on allocation failure.
 */
int farm_oracle_score(int64_t n, int d, const float* desc, const float* center, const float* extent,
                      const uint32_t* id, const int32_t* cls, const float* right, int32_t q, const float* target,
                      const int32_t* target_cls, const int32_t* rel_off, const int32_t* rel_pred,
                      const float* rel_anchor, double* scores, double* sem, double* rel_terms,
                      uint32_t* rel_anchor_id) {
    if (check_query_meta(q, rel_off, rel_pred)) return -1;
    scene64 s;
    if (scene_init(&s, n, d, desc, center, extent, id, cls, right)) { scene_free(&s); return -2; }
    if (check_scene_geometry(&s, q, rel_off, rel_pred)) { scene_free(&s); return -1; }
    int err = 0;
    /* queries one after another; the objects of a query (and its similarity
     * rows) in parallel, so that every thread works whatever the query count */
    for (int32_t k = 0; k < q && !err; ++k) {
        query64 qs;
        int r = rel_off[k + 1] - rel_off[k];
        int r0 = rel_off[k];
        if (query_init(&qs, &s, k, r0, target + (size_t)k * d, target_cls ? target_cls[k] : -1, r,
                       rel_pred + r0, rel_anchor + (size_t)r0 * d)) {
            query_free(&qs);
            err = -2;
            continue;
        }
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            double t[ORACLE_MAX_REL];
            uint32_t b[ORACLE_MAX_REL];
            query_terms(&s, &qs, i, t, b);
            for (int rr = 0; rr < r; ++rr) {
                if (rel_terms) rel_terms[(size_t)(r0 + rr) * n + i] = t[rr];
                if (rel_anchor_id) rel_anchor_id[(size_t)(r0 + rr) * n + i] = b[rr];
            }
            scores[(size_t)k * n + i] = composite(qs.sem[i], r, t, qs.pred);
            if (sem) sem[(size_t)k * n + i] = qs.sem[i];
        }
        query_free(&qs);
    }
    scene_free(&s);
    return err;
}

/*
 * Scores of selected (query, object) pairs only: out[m] for pair m =
 * (qsel[m], osel[m]); each costs O(R * N) after the query's similarities.
 * rel_terms/rel_anchor_id, when not NULL, are [m][8] (unused slots = 0 / NO_ID).
 */
int farm_oracle_score_pairs(int64_t n, int d, const float* desc, const float* center, const float* extent,
                            const uint32_t* id, const int32_t* cls, const float* right, int32_t q, const float* target,
                            const int32_t* target_cls, const int32_t* rel_off, const int32_t* rel_pred,
                            const float* rel_anchor, int64_t m, const int32_t* qsel, const int64_t* osel,
                            double* out, double* out_sem, double* rel_terms, uint32_t* rel_anchor_id) {
    if (check_query_meta(q, rel_off, rel_pred)) return -1;
    for (int64_t p = 0; p < m; ++p)
        if (qsel[p] < 0 || qsel[p] >= q || osel[p] < 0 || osel[p] >= n) return -1;
    scene64 s;
    if (scene_init(&s, n, d, desc, center, extent, id, cls, right)) { scene_free(&s); return -2; }
    if (check_scene_geometry(&s, q, rel_off, rel_pred)) { scene_free(&s); return -1; }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t k = 0; k < q; ++k) {
        int64_t cnt = 0;
        for (int64_t p = 0; p < m; ++p) cnt += (qsel[p] == k);
        if (!cnt) continue;
        query64 qs;
        int r = rel_off[k + 1] - rel_off[k];
        int r0 = rel_off[k];
        if (query_init(&qs, &s, k, r0, target + (size_t)k * d, target_cls ? target_cls[k] : -1, r,
                       rel_pred + r0, rel_anchor + (size_t)r0 * d)) {
            query_free(&qs);
#pragma omp atomic write
            err = -2;
            continue;
        }
        for (int64_t p = 0; p < m; ++p) {
            if (qsel[p] != k) continue;
            int64_t i = osel[p];
            double t[ORACLE_MAX_REL];
            uint32_t b[ORACLE_MAX_REL];
            for (int rr = 0; rr < ORACLE_MAX_REL; ++rr) { t[rr] = 0.0; b[rr] = ORACLE_NO_ID; }
            query_terms(&s, &qs, i, t, b);
            for (int rr = 0; rr < ORACLE_MAX_REL; ++rr) {
                if (rel_terms) rel_terms[p * ORACLE_MAX_REL + rr] = t[rr];
                if (rel_anchor_id) rel_anchor_id[p * ORACLE_MAX_REL + rr] = b[rr];
            }
            out[p] = composite(qs.sem[i], r, t, qs.pred);
            if (out_sem) out_sem[p] = qs.sem[i];
        }
        query_free(&qs);
    }
    scene_free(&s);
    return err;
}

/* TopK of one score row: first min(k, n) indices by (score desc, id asc). */
static int topk_cmp_scores_desc(const double* sc, const uint32_t* id, int64_t a, int64_t b) {
    if (sc[a] > sc[b]) return -1;
    if (sc[a] < sc[b]) return 1;
    return (id[a] < id[b]) ? -1 : (id[a] > id[b]);
}

int farm_oracle_topk(int64_t n, const double* scores, const uint32_t* id, int32_t k, int64_t* out_idx) {
    /* Selection by repeated scans: plain and obviously correct. */
    int64_t kk = k < n ? k : n;
    unsigned char* taken = (unsigned char*)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!taken) return -2;
    for (int64_t r = 0; r < kk; ++r) {
        int64_t best = -1;
        for (int64_t i = 0; i < n; ++i) {
            if (taken[i]) continue;
            if (best < 0 || topk_cmp_scores_desc(scores, id, i, best) < 0) best = i;
        }
        taken[best] = 1;
        out_idx[r] = best;
    }
    for (int64_t r = kk; r < k; ++r) out_idx[r] = -1;
    free(taken);
    return 0;
}

/*
 * Exact TopK of large queries without scoring every object.  The soft blend
 * bounds every score: (1 - w) s_sem(i) <= s(i) <= s_sem(i) (the spatial factor
 * stays in [1 - w, 1]; "Why soft, not hard?" paragraph).  Let L be the K-th
 * largest lower bound (1 - w) s_sem.  K objects score at least L, so an object
 * with s_sem(i) < L scores strictly below them and cannot enter the TopK.
 * Only objects with s_sem(i) >= L are scored, exhaustively over anchors.
 *   out_idx[q][k] object indices (-1 padding), out_score[q][k],
 *   n_scored[q]   how many objects were scored exactly (may be NULL).
 */
int farm_oracle_topk_bounded(int64_t n, int d, const float* desc, const float* center, const float* extent,
                             const uint32_t* id, const int32_t* cls, const float* right, int32_t q, const float* target,
                             const int32_t* target_cls, const int32_t* rel_off, const int32_t* rel_pred,
                             const float* rel_anchor, int32_t k, int64_t* out_idx, double* out_score,
                             double* out_terms, uint32_t* out_anchor_id, int64_t* n_scored) {
    if (check_query_meta(q, rel_off, rel_pred) || k < 1) return -1;
    scene64 s;
    if (scene_init(&s, n, d, desc, center, extent, id, cls, right)) { scene_free(&s); return -2; }
    if (check_scene_geometry(&s, q, rel_off, rel_pred)) { scene_free(&s); return -1; }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t qq = 0; qq < q; ++qq) {
        query64 qs;
        int r = rel_off[qq + 1] - rel_off[qq];
        int r0 = rel_off[qq];
        double* full = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double* lower = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        int64_t* sel = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
        if (!full || !lower || !sel ||
            query_init(&qs, &s, qq, r0, target + (size_t)qq * d, target_cls ? target_cls[qq] : -1, r,
                       rel_pred + r0, rel_anchor + (size_t)r0 * d)) {
            free(full); free(lower); free(sel);
#pragma omp atomic write
            err = -2;
            continue;
        }
        /* K-th largest lower bound. */
        for (int64_t i = 0; i < n; ++i) lower[i] = (1.0 - ORACLE_W) * qs.sem[i];
        double L = -1.0;
        if (n > 0) {
            int64_t kk = k < n ? k : n;
            /* plain partial selection of the kk-th largest value */
            double* tmp = (double*)malloc(sizeof(double) * (size_t)n);
            memcpy(tmp, lower, sizeof(double) * (size_t)n);
            for (int64_t rr = 0; rr < kk; ++rr) {
                int64_t bi = rr;
                for (int64_t i = rr + 1; i < n; ++i) if (tmp[i] > tmp[bi]) bi = i;
                double x = tmp[rr]; tmp[rr] = tmp[bi]; tmp[bi] = x;
            }
            L = tmp[kk - 1];
            free(tmp);
        }
        int64_t cnt = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (qs.sem[i] >= L) {
                double t[ORACLE_MAX_REL];
                uint32_t b[ORACLE_MAX_REL];
                query_terms(&s, &qs, i, t, b);
                full[i] = composite(qs.sem[i], r, t, qs.pred);
                ++cnt;
            } else {
                full[i] = -INFINITY; /* provably outside the TopK */
            }
        }
        if (n_scored) n_scored[qq] = cnt;
        farm_oracle_topk(n, full, s.id, k, sel);
        for (int32_t rr = 0; rr < k; ++rr) {
            out_idx[(size_t)qq * k + rr] = sel[rr];
            out_score[(size_t)qq * k + rr] = sel[rr] >= 0 ? full[sel[rr]] : -INFINITY;
            double tv[ORACLE_MAX_REL];
            uint32_t bv[ORACLE_MAX_REL];
            for (int e = 0; e < ORACLE_MAX_REL; ++e) { tv[e] = 0.0; bv[e] = ORACLE_NO_ID; }
            if (sel[rr] >= 0) query_terms(&s, &qs, sel[rr], tv, bv);
            for (int e = 0; e < ORACLE_MAX_REL; ++e) {
                if (out_terms) out_terms[((size_t)qq * k + rr) * ORACLE_MAX_REL + e] = tv[e];
                if (out_anchor_id) out_anchor_id[((size_t)qq * k + rr) * ORACLE_MAX_REL + e] = bv[e];
            }
        }
        free(full); free(lower); free(sel);
        query_free(&qs);
    }
    scene_free(&s);
    return err;
}

/*
 * Value of one binding: sim(j, q_r) * P_p(i, j) in FP64 -- used to check that
 * an anchor chosen by another implementation attains the relation term.
 */
double farm_oracle_binding_value(int64_t n, int d, const float* desc, const float* center, const float* extent,
                                 const uint32_t* id, const int32_t* cls, const float* right, int32_t tcls,
                                 int p, const float* anchor, int64_t i, int64_t j) {
    if (i < 0 || j < 0 || i >= n || j >= n || p < 0 || p >= P_COUNT) return NAN;
    double* u = (double*)malloc(sizeof(double) * (size_t)d);
    double* v = (double*)malloc(sizeof(double) * (size_t)d);
    if (!u || !v) { free(u); free(v); return NAN; }
    unit_vector(desc + (size_t)j * d, d, u);
    unit_vector(anchor, d, v);
    double a = clamped_cosine(u, v, d);
    double ci[3] = {center[i * 3], center[i * 3 + 1], center[i * 3 + 2]};
    double cj[3] = {center[j * 3], center[j * 3 + 1], center[j * 3 + 2]};
    double ei[3] = {extent[i * 3], extent[i * 3 + 1], extent[i * 3 + 2]};
    double ej[3] = {extent[j * 3], extent[j * 3 + 1], extent[j * 3 + 2]};
    double r[2] = {right[0], right[1]};
    double val;
    if (is_rank_pred(p)) {
        scene64 s0;
        memset(&s0, 0, sizeof(s0));
        s0.n = n;
        s0.c = (double*)malloc(sizeof(double) * (size_t)n * 3);
        if (!s0.c) { free(u); free(v); return NAN; }
        for (int64_t k = 0; k < n * 3; ++k) s0.c[k] = center[k];
        s0.id = id;
        s0.cls = cls;
        val = a * rank_value(&s0, tcls, p, i, j);
        free(s0.c);
    } else if (p == P_NEAR_H || is_view_pred(p)) {
        /* the entity geometry of the scene (farm_oracle_set_entity_geometry) */
        if (g_ext_n != n || (p == P_NEAR_H && !g_cov) || (p != P_NEAR_H && !g_view)) {
            val = NAN;
        } else if (p == P_NEAR_H) {
            double A[6], B[6];
            for (int k = 0; k < 6; ++k) { A[k] = g_cov[i * 6 + k]; B[k] = g_cov[j * 6 + k]; }
            val = a * hellinger_near(ci, A, cj, B);
        } else {
            double w[12];
            for (int k = 0; k < 12; ++k) w[k] = g_view[i * 12 + k];
            val = a * view_predicate(p, w, ci, cj);
        }
    } else {
        val = a * oracle_predicate(p, ci, cj, ei, ej, r);
    }
    free(u);
    free(v);
    return val;
}

/* Value of one Between binding: sim(j1, v1) sim(j2, v2) Between(i; j1, j2). */
double farm_oracle_between_binding_value(int64_t n, int d, const float* desc, const float* center,
                                         const float* anchor1, const float* anchor2, int64_t i, int64_t j1,
                                         int64_t j2) {
    if (i < 0 || j1 < 0 || j2 < 0 || i >= n || j1 >= n || j2 >= n) return NAN;
    double* u = (double*)malloc(sizeof(double) * (size_t)d);
    double* v = (double*)malloc(sizeof(double) * (size_t)d);
    if (!u || !v) { free(u); free(v); return NAN; }
    unit_vector(desc + (size_t)j1 * d, d, u);
    unit_vector(anchor1, d, v);
    double a1 = clamped_cosine(u, v, d);
    unit_vector(desc + (size_t)j2 * d, d, u);
    unit_vector(anchor2, d, v);
    double a2 = clamped_cosine(u, v, d);
    free(u);
    free(v);
    double ci[3], c1[3], c2[3];
    for (int k = 0; k < 3; ++k) { ci[k] = center[i * 3 + k]; c1[k] = center[j1 * 3 + k]; c2[k] = center[j2 * 3 + k]; }
    return a1 * a2 * between_value(ci, c1, c2);
}

/* ------------------------------------------------------------------------
 * Learned anchor proposal network (test infrastructure for the GPU kernels).
 * Not a construct of the paper: the anchor-candidate sets K_a of the
 * query-time complexity analysis are produced here by a small network that
 * ranks (target, anchor) pairs per predicate.
 *
 *   x  = [u_o ; u_a ; g(o, a)]                (2d + 12 inputs)
 *   h1 = GELU(W1 x + b1),  h2 = GELU(W2 h1 + b2),  y = W3 h2 + b3   (9 logits)
 *   GELU(v) = v/2 (1 + erf(v / sqrt 2))
 *   loss = mean_s BCEwithLogits(y_s[p_s], label_s)
 *        = mean_s [ max(y,0) - y*label + log(1 + exp(-|y|)) ]
 *
 * g(o, a) = [c_o - c_a (3), e_o (3), e_a (3), |c_o - c_a|, (c_o - c_a).r,
 *            (z_o - e_o,z/2) - (z_a + e_a,z/2)]   (bottom of o minus top of a)
 * Weights are row-major: W1 [h][in], W2 [h][h], W3 [9][h] (one output per predicate).
 * ------------------------------------------------------------------------ */
#define ORACLE_NPRED 9
#define ORACLE_NGEO 12

static double gelu(double v) { return 0.5 * v * (1.0 + erf(v / sqrt(2.0))); }
static double gelu_grad(double v) {
    return 0.5 * (1.0 + erf(v / sqrt(2.0))) + v * exp(-0.5 * v * v) / sqrt(2.0 * M_PI);
}

void farm_oracle_pair_features(const float* center, const float* extent, const float* right, int64_t o, int64_t a,
                               double* g) {
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = (double)center[o * 3 + k] - (double)center[a * 3 + k];
    for (int k = 0; k < 3; ++k) g[k] = d[k];
    for (int k = 0; k < 3; ++k) g[3 + k] = extent[o * 3 + k];
    for (int k = 0; k < 3; ++k) g[6 + k] = extent[a * 3 + k];
    g[9] = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    g[10] = d[0] * (double)right[0] + d[1] * (double)right[1];
    g[11] = ((double)center[o * 3 + 2] - 0.5 * (double)extent[o * 3 + 2]) -
            ((double)center[a * 3 + 2] + 0.5 * (double)extent[a * 3 + 2]);
}

/*
 * Loss and gradients over nsamp samples with inputs X [nsamp][in], predicate
 * p_s and binary label_s.  Gradient outputs may be NULL; logits [nsamp][9]
 * may be NULL.  Plain backpropagation, one sample at a time.
 */
int farm_oracle_mlp(int in, int h, const double* W1, const double* b1, const double* W2, const double* b2,
                    const double* W3, const double* b3, int64_t nsamp, const double* X, const int32_t* pred,
                    const double* label, double* loss, double* gW1, double* gb1, double* gW2, double* gb2,
                    double* gW3, double* gb3, double* logits) {
    double* z1 = (double*)malloc(sizeof(double) * h);
    double* a1 = (double*)malloc(sizeof(double) * h);
    double* z2 = (double*)malloc(sizeof(double) * h);
    double* a2 = (double*)malloc(sizeof(double) * h);
    double* d2 = (double*)malloc(sizeof(double) * h);
    double* d1 = (double*)malloc(sizeof(double) * h);
    if (!z1 || !a1 || !z2 || !a2 || !d2 || !d1) { free(z1); free(a1); free(z2); free(a2); free(d2); free(d1); return -2; }
    if (gW1) memset(gW1, 0, sizeof(double) * (size_t)h * in);
    if (gb1) memset(gb1, 0, sizeof(double) * h);
    if (gW2) memset(gW2, 0, sizeof(double) * (size_t)h * h);
    if (gb2) memset(gb2, 0, sizeof(double) * h);
    if (gW3) memset(gW3, 0, sizeof(double) * ORACLE_NPRED * h);
    if (gb3) memset(gb3, 0, sizeof(double) * ORACLE_NPRED);
    double total = 0.0;
    for (int64_t s = 0; s < nsamp; ++s) {
        const double* x = X + s * in;
        for (int j = 0; j < h; ++j) {
            double acc = b1[j];
            for (int k = 0; k < in; ++k) acc += W1[(size_t)j * in + k] * x[k];
            z1[j] = acc;
            a1[j] = gelu(acc);
        }
        for (int j = 0; j < h; ++j) {
            double acc = b2[j];
            for (int k = 0; k < h; ++k) acc += W2[(size_t)j * h + k] * a1[k];
            z2[j] = acc;
            a2[j] = gelu(acc);
        }
        double y[ORACLE_NPRED];
        for (int c = 0; c < ORACLE_NPRED; ++c) {
            double acc = b3[c];
            for (int k = 0; k < h; ++k) acc += W3[(size_t)c * h + k] * a2[k];
            y[c] = acc;
            if (logits) logits[s * ORACLE_NPRED + c] = acc;
        }
        const int p = pred[s];
        const double t = label[s], v = y[p];
        total += (v > 0 ? v : 0.0) - v * t + log1p(exp(-fabs(v)));
        if (!gW1 && !gb1 && !gW2 && !gb2 && !gW3 && !gb3) continue;
        /* d loss / d y[p] = sigmoid(y[p]) - label, divided by nsamp (mean) */
        const double dy = (1.0 / (1.0 + exp(-v)) - t) / (double)nsamp;
        for (int k = 0; k < h; ++k) {
            if (gW3) gW3[(size_t)p * h + k] += dy * a2[k];
            d2[k] = dy * W3[(size_t)p * h + k] * gelu_grad(z2[k]);
        }
        if (gb3) gb3[p] += dy;
        for (int j = 0; j < h; ++j) {
            if (gb2) gb2[j] += d2[j];
            if (gW2) for (int k = 0; k < h; ++k) gW2[(size_t)j * h + k] += d2[j] * a1[k];
        }
        for (int k = 0; k < h; ++k) {
            double acc = 0.0;
            for (int j = 0; j < h; ++j) acc += W2[(size_t)j * h + k] * d2[j];
            d1[k] = acc * gelu_grad(z1[k]);
        }
        for (int j = 0; j < h; ++j) {
            if (gb1) gb1[j] += d1[j];
            if (gW1) for (int k = 0; k < in; ++k) gW1[(size_t)j * in + k] += d1[j] * x[k];
        }
    }
    if (loss) *loss = total / (double)(nsamp > 0 ? nsamp : 1);
    free(z1); free(a1); free(z2); free(a2); free(d2); free(d1);
    return 0;
}
