// scan_math.h -- predicates evaluated by a per-anchor scan: Closest /
// Farthest, a rank within the query's candidate set (Appendix "Retrieval
// Details", predicate evaluation: score 1 / (|rank - r*| + 1)), and Inside, a
// soft containment test (per axis a logistic, 0.1 m, of the margin between
// the anchor's half extent and the target's center offset; the product over
// the three axes).  Neither fits the pair kernels' anchor records: the rank
// depends on the candidate set, Inside on the anchor's extents.
//
// The candidate set C holds the objects of the query's parsed target class
// (every object when the query or the memory has no classes).  For target o
// and anchor a, rank = 1 + the number of candidates c (c != o, c != a) nearer
// to a than o, equal distances ordered by object id; r* = 1 for Closest and
// the last rank, m + 1 with m = |C minus o and a|, for Farthest.  The rank is
// an integer decided by distance comparisons, so it is decided in one fixed
// FP32 order: ((dx*dx + dy*dy) + dz*dz) of FP32 center differences, without
// contraction.
//
// The term t = max_{a != o} sim(a) * P(o, a) of every scanned predicate is
// taken by one wave (or split over a block's waves): anchors
// whose similarity (or its upper bound) is below the best value so far are
// skipped, since P <= 1; for the others Inside is one evaluation and the
// rank a wave-wide count over the candidates.  With a class, the candidates
// are a contiguous range of the memory's class order (found by binary search
// once per term), so an anchor costs O(|C|); without one, O(N).
#pragma once

#include <math.h>

#include "farm_internal.h"

namespace farm {

__device__ inline bool is_rank(int p) { return p == FARM_CLOSEST || p == FARM_FARTHEST; }
// Predicates over the entity Gaussians / stored views (FP64, O(1) per anchor).
__device__ inline bool is_entity_geo(int p) { return p >= FARM_NEAR_HELLINGER && p <= FARM_BEHIND_VIEW; }
// O(1) per anchor: Inside and the entity-geometry predicates.
__device__ inline bool is_local(int p) { return p == FARM_INSIDE || is_entity_geo(p); }
// Between and its second-anchor slot are scanned too (between_term_wave): the
// pairwise kernels and the proposal lists leave them alone.
__device__ inline bool is_scanned(int p) {
  return is_rank(p) || is_local(p) || p == FARM_BETWEEN || p == FARM_AND;
}

struct ScanCtx {
  const float *x, *y, *z;
  const float* ext;  // [3][n] full extents (Inside)
  const uint32_t* ids;
  const int32_t* cls;         // object classes, or null
  const int32_t* cls_order;   // objects in class order (null without classes)
  const int32_t* cls_sorted;  // their classes, ascending
  int32_t tc;                 // the query's parsed target class (-1: none)
  int64_t n;
  int p;                      // a scanned predicate other than Between
  int64_t lo = 0, hi = -1;    // the class's range in cls_order (hi < 0: every object is a candidate)
  EntityGeo eg{};             // Gaussians and stored views (entity-geometry predicates)
};

// The candidates' range in the class order: [lower_bound, upper_bound) of tc.
__device__ inline void rank_range(ScanCtx& k) {
  if (!is_rank(k.p) || k.tc < 0 || k.cls == nullptr || k.cls_order == nullptr) return;
  int64_t a = 0, b = k.n;
  while (a < b) {
    const int64_t mid = (a + b) >> 1;
    if (k.cls_sorted[mid] < k.tc) a = mid + 1; else b = mid;
  }
  int64_t c = a, d = k.n;
  while (c < d) {
    const int64_t mid = (c + d) >> 1;
    if (k.cls_sorted[mid] <= k.tc) c = mid + 1; else d = mid;
  }
  k.lo = a;
  k.hi = c;
}

__device__ inline float rank_d2(float ax, float ay, float az, float bx, float by, float bz) {
#pragma clang fp contract(off)
  const float dx = ax - bx, dy = ay - by, dz = az - bz;
  float s = dx * dx;
  s = s + dy * dy;
  s = s + dz * dz;
  return s;
}

__device__ inline float wave_max_scan(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

__device__ inline int wave_sum_i(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// P(o, a) by one wave (every lane returns the same value).
__device__ inline float rank_pred_wave(const ScanCtx& k, int64_t o, int64_t a, int lane) {
  const float ax = k.x[a], ay = k.y[a], az = k.z[a];
  const float doa = rank_d2(k.x[o], k.y[o], k.z[o], ax, ay, az);
  const uint32_t ido = k.ids[o];
  int nearer = 0, m = 0;
  auto count = [&](int64_t c) {
    if (c == o || c == a) return;
    ++m;
    const float dc = rank_d2(k.x[c], k.y[c], k.z[c], ax, ay, az);
    nearer += (dc < doa || (dc == doa && k.ids[c] < ido)) ? 1 : 0;
  };
  if (k.hi >= 0) {
    for (int64_t e = k.lo + lane; e < k.hi; e += 64) count(k.cls_order[e]);
  } else {
    const bool filter = k.tc >= 0 && k.cls != nullptr;
    for (int64_t c = lane; c < k.n; c += 64)
      if (!filter || k.cls[c] == k.tc) count(c);
  }
  nearer = wave_sum_i(nearer);
  m = wave_sum_i(m);
  const int rank = nearer + 1;
  const int rstar = k.p == FARM_CLOSEST ? 1 : m + 1;
  const int off = rank > rstar ? rank - rstar : rstar - rank;
  return 1.0f / (float)(off + 1);
}

// t and the binding anchor's id for target o by one wave.  hi_of(a): an upper
// bound of sim(a) (lane-local); exact_of(a): sim(a), called by the whole wave
// with a uniform a (it may be a wave-wide dot product).  Optionally the
// relation's semantic set (sidx, sn: the anchors of largest similarity) goes
// first; when the best value then exceeds out_bound, a bound on the
// similarity of every other anchor, no other anchor can reach it (P <= 1) and
// the scan ends there.  best is -1 when no anchor exists (n = 1); the caller
// clamps.
// The two phases of a term, each over a share of its anchors: part w of
// parts takes semantic-set entries w, w + parts, ... and anchor chunks of 64
// starting at 64 w with stride 64 parts (several waves of a block can split
// one term and merge (best, id) afterwards).  best/bid carry the running
// maximum in and out; k must have its range set (rank_range).
// Inside(o, a): every lane computes the same value.
__device__ inline float inside_value(const ScanCtx& k, int64_t o, int64_t a) {
  const float d[3] = {k.x[o] - k.x[a], k.y[o] - k.y[a], k.z[o] - k.z[a]};
  float v = 1.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float u = (0.5f * k.ext[c * k.n + a] - fabsf(d[c])) * 10.0f;  // margin / 0.1 m
    v *= 1.0f / (1.0f + expf(-u));
  }
  return v;
}

// Near over the entity Gaussians in FP64: 1 - H, H^2 = 1 - BC, written as
// H^2 = -expm1(-D) with the Bhattacharyya distance D = q / 8 + log det M / 2 -
// (log det A + log det B) / 4, M = (A + B) / 2 and q = d^T M^-1 d through the
// adjugate of M (d the center offset; the FP32 centers are exact in FP64).
__device__ inline float hellinger_near_value(const ScanCtx& k, int64_t o, int64_t a) {
  const float* C = k.eg.cov;
  const int64_t n = k.n;
  const double m00 = 0.5 * ((double)C[o] + (double)C[a]);
  const double m01 = 0.5 * ((double)C[n + o] + (double)C[n + a]);
  const double m02 = 0.5 * ((double)C[2 * n + o] + (double)C[2 * n + a]);
  const double m11 = 0.5 * ((double)C[3 * n + o] + (double)C[3 * n + a]);
  const double m12 = 0.5 * ((double)C[4 * n + o] + (double)C[4 * n + a]);
  const double m22 = 0.5 * ((double)C[5 * n + o] + (double)C[5 * n + a]);
  const double c00 = m11 * m22 - m12 * m12, c01 = m02 * m12 - m01 * m22, c02 = m01 * m12 - m02 * m11;
  const double c11 = m00 * m22 - m02 * m02, c12 = m01 * m02 - m00 * m12, c22 = m00 * m11 - m01 * m01;
  const double det = m00 * c00 + m01 * c01 + m02 * c02;
  const double dx = (double)k.x[o] - (double)k.x[a], dy = (double)k.y[o] - (double)k.y[a],
               dz = (double)k.z[o] - (double)k.z[a];
  const double qf = (c00 * dx * dx + c11 * dy * dy + c22 * dz * dz + 2.0 * (c01 * dx * dy + c02 * dx * dz + c12 * dy * dz)) / det;
  const double db = 0.125 * qf + 0.5 * log(det) - 0.25 * (k.eg.cov_ld[o] + k.eg.cov_ld[a]);
  double h2 = -expm1(-db);
  if (h2 < 0.0) h2 = 0.0;
  return (float)(1.0 - sqrt(h2));
}

// The stored-view predicates in target o's view, FP64: camera coordinates
// R (c - p) of both centers; 0 unless both lie in the view (depth >= 0.1 m,
// |x| <= depth, |y| <= 0.75 depth); then a logistic of the image-plane
// offset x / z (temperature 0.05) or of the depth offset (0.1 m).
__device__ inline float view_value(const ScanCtx& k, int64_t o, int64_t a) {
  const float* V = k.eg.view;
  const int64_t n = k.n;
  double v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = V[c * n + o];
  auto cam = [&](int64_t i, double& xc, double& yc, double& zc) {
    const double w0 = (double)k.x[i] - v[0], w1 = (double)k.y[i] - v[1], w2 = (double)k.z[i] - v[2];
    xc = v[3] * w0 + v[4] * w1 + v[5] * w2;
    yc = v[6] * w0 + v[7] * w1 + v[8] * w2;
    zc = v[9] * w0 + v[10] * w1 + v[11] * w2;
  };
  double xo, yo, zo, xa, ya, za;
  cam(o, xo, yo, zo);
  cam(a, xa, ya, za);
  auto in_view = [](double x, double y, double z) { return z >= 0.1 && fabs(x) <= z && fabs(y) <= 0.75 * z; };
  if (!in_view(xo, yo, zo) || !in_view(xa, ya, za)) return 0.0f;
  double arg;
  switch (k.p) {
    case FARM_LEFT_OF_VIEW: arg = (xa / za - xo / zo) * 20.0; break;
    case FARM_RIGHT_OF_VIEW: arg = (xo / zo - xa / za) * 20.0; break;
    case FARM_IN_FRONT_OF_VIEW: arg = (za - zo) * 10.0; break;
    default: arg = (zo - za) * 10.0; break;  // FARM_BEHIND_VIEW
  }
  return (float)(1.0 / (1.0 + exp(-arg)));
}

// P(o, a) of the O(1) predicates (every lane computes the same value).  The
// scans are instantiated twice: GEO for the entity-geometry predicates (FP64,
// many registers) and !GEO for the others, so that the FP64 code does not
// weigh on the register budget of the rank, Inside and Between scans.
template <bool GEO>
__device__ inline float local_value(const ScanCtx& k, int64_t o, int64_t a) {
  if constexpr (GEO) {
    if (k.p == FARM_NEAR_HELLINGER) return hellinger_near_value(k, o, a);
    return view_value(k, o, a);
  } else {
    return inside_value(k, o, a);
  }
}

template <bool GEO>
__device__ inline float scan_pred_wave(const ScanCtx& k, int64_t o, int64_t a, int lane) {
  if constexpr (GEO) return local_value<true>(k, o, a);
  else return is_local(k.p) ? local_value<false>(k, o, a) : rank_pred_wave(k, o, a, lane);
}

template <bool GEO, class ExactOf>
__device__ inline void scan_visit(const ScanCtx& k, int64_t o, int64_t aa, int lane, ExactOf& exact_of, float& best,
                                  uint32_t& bid) {
  const float s = exact_of(aa);
  if (s < best) return;
  const float v = s * scan_pred_wave<GEO>(k, o, aa, lane);
  const uint32_t ida = k.ids[aa];
  if (v > best || (v == best && ida < bid)) {
    best = v;
    bid = ida;
  }
}

template <bool GEO, class ExactOf>
__device__ void scan_set_part(const ScanCtx& k, int64_t o, int lane, ExactOf exact_of, const int32_t* sidx, int sn,
                              int w, int parts, float& best, uint32_t& bid) {
  for (int e = w; e < sn; e += parts) {
    const int64_t aa = __builtin_amdgcn_readfirstlane(sidx[e]);
    if (aa != o) scan_visit<GEO>(k, o, aa, lane, exact_of, best, bid);
  }
}

template <bool GEO, class LoOf, class HiOf, class ExactOf>
__device__ void scan_anchor_part(const ScanCtx& k, int64_t o, int lane, LoOf lo_of, HiOf hi_of, ExactOf exact_of, int w,
                                 int parts, float& best, uint32_t& bid) {
  if (GEO || is_local(k.p)) {
    // P costs O(1): each lane bounds its anchor's value by sim_lo * P and
    // sim_hi * P (products round monotonically, so they bound the exact s * P);
    // the largest lower bound L prunes every anchor whose upper bound is below it
    float L = best;
    for (int64_t a0 = (int64_t)64 * w; a0 < k.n; a0 += (int64_t)64 * parts) {
      const int64_t a = a0 + lane;
      if (a < k.n && a != o) L = fmaxf(L, lo_of(a) * local_value<GEO>(k, o, a));
    }
    L = wave_max_scan(L);
    for (int64_t a0 = (int64_t)64 * w; a0 < k.n; a0 += (int64_t)64 * parts) {
      const int64_t a = a0 + lane;
      const bool valid = a < k.n && a != o;
      const float pv = valid ? local_value<GEO>(k, o, a) : 0.f;
      const float hb = valid ? hi_of(a) * pv : -INFINITY;
      uint64_t mask = __ballot(hb >= best && hb >= L);
      while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        if (__shfl(hb, src) < best) continue;
        const int64_t aa = a0 + src;
        const float v = exact_of(aa) * __shfl(pv, src);
        const uint32_t ida = k.ids[aa];
        if (v > best || (v == best && ida < bid)) {
          best = v;
          bid = ida;
        }
      }
    }
    return;
  }
  for (int64_t a0 = (int64_t)64 * w; a0 < k.n; a0 += (int64_t)64 * parts) {
    const int64_t a = a0 + lane;
    const float h = (a < k.n && a != o) ? hi_of(a) : -INFINITY;
    uint64_t mask = __ballot(h >= best);
    while (mask) {
      const int src = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      if (__shfl(h, src) < best) continue;  // the best grew meanwhile
      scan_visit<GEO>(k, o, a0 + src, lane, exact_of, best, bid);
    }
  }
}

template <bool GEO, class LoOf, class HiOf, class ExactOf>
__device__ void scan_term_wave(ScanCtx k, int64_t o, int lane, LoOf lo_of, HiOf hi_of, ExactOf exact_of, float& out_best,
                               uint32_t& out_bid, const int32_t* sidx = nullptr, int sn = 0,
                               float out_bound = INFINITY) {
  rank_range(k);
  float best = -1.0f;
  uint32_t bid = FARM_NO_ID;
  scan_set_part<GEO>(k, o, lane, exact_of, sidx, sn, 0, 1, best, bid);
  if (!(sn > 0 && best > out_bound)) scan_anchor_part<GEO>(k, o, lane, lo_of, hi_of, exact_of, 0, 1, best, bid);
  out_best = best;
  out_bid = bid;
}

// ---------------------------------------------------------------- Between
// Between(o; a1, a2) = sig(s1 / tau) sig(s2 / tau) exp(-h^2 / (2 sigma^2)),
// tau = 0.1 m, sigma = 0.5 m: s1 = (c_o - c_a1) . u and s2 = (c_a2 - c_o) . u
// are the two margins along the unit axis u from a1 to a2 (each formed from
// its own anchor, so that it is accurate relative to that offset), h the
// distance of c_o from the axis, from the cross product with the offset to
// the nearer anchor.  0 when the anchors coincide.
__device__ inline float between_p(float ox, float oy, float oz, float x1, float y1, float z1, float x2, float y2,
                                  float z2) {
  float ux = x2 - x1, uy = y2 - y1, uz = z2 - z1;
  const float l2 = ux * ux + uy * uy + uz * uz;
  if (l2 == 0.f) return 0.f;
  const float inv = 1.0f / sqrtf(l2);
  ux *= inv;
  uy *= inv;
  uz *= inv;
  const float w1x = ox - x1, w1y = oy - y1, w1z = oz - z1;
  const float w2x = x2 - ox, w2y = y2 - oy, w2z = z2 - oz;
  const float s1 = w1x * ux + w1y * uy + w1z * uz;
  const float s2 = w2x * ux + w2y * uy + w2z * uz;
  const bool near1 = fabsf(s1) <= fabsf(s2);
  const float wx = near1 ? w1x : -w2x, wy = near1 ? w1y : -w2y, wz = near1 ? w1z : -w2z;
  const float cx = wy * uz - wz * uy, cy = wz * ux - wx * uz, cz = wx * uy - wy * ux;
  const float h2 = cx * cx + cy * cy + cz * cz;
  // logistic(v / 0.1) = 1 / (1 + 2^(-v * 10 log2 e)); Gaussian exp(-h^2 / 0.5) = 2^(-2 log2(e) h^2)
  constexpr float kS = 14.426950408889634f;  // 10 log2(e)
  constexpr float kG = 2.8853900817779268f;  // 2 log2(e)
  const float g1 = 1.0f / (1.0f + exp2f(-s1 * kS));
  const float g2 = 1.0f / (1.0f + exp2f(-s2 * kS));
  return g1 * g2 * exp2f(-h2 * kG);
}

// (value, id1, id2) ordering of Between bindings: larger value, then the
// smaller id pair.
__device__ inline bool between_better(float v, uint32_t i1, uint32_t i2, float bv, uint32_t b1, uint32_t b2) {
  return v > bv || (v == bv && (i1 < b1 || (i1 == b1 && i2 < b2)));
}

__device__ inline void between_wave_best(float& v, uint32_t& i1, uint32_t& i2) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float ov = __shfl_xor(v, off);
    const uint32_t o1 = __shfl_xor(i1, off), o2 = __shfl_xor(i2, off);
    if (between_better(ov, o1, o2, v, i1, i2)) {
      v = ov;
      i1 = o1;
      i2 = o2;
    }
  }
}

// Between's term for target o by one wave: the maximum over a1 in the first
// candidate set and a2 in the second (a1 != a2, both != o) of
// (sim1(a1) sim2(a2)) Between(o; a1, a2), ties by the smaller id pair; the
// candidate sets are the 64 anchors of largest similarity of each slot
// (k_between_sets) with their exact similarities.  t = 0 and no binding
// (FARM_NO_ID) when no pair has a positive value.
__device__ inline void between_term_wave(const float* __restrict__ x, const float* __restrict__ y,
                                         const float* __restrict__ z, const uint32_t* __restrict__ ids, int64_t o,
                                         int lane, const int32_t* __restrict__ s1, const float* __restrict__ e1,
                                         int n1, const int32_t* __restrict__ s2, const float* __restrict__ e2, int n2,
                                         float& out_t, uint32_t& out_b1, uint32_t& out_b2) {
  const float ox = x[o], oy = y[o], oz = z[o];
  float best = 0.f;
  uint32_t b1 = FARM_NO_ID, b2 = FARM_NO_ID;
  const int pairs = n1 * n2;
  for (int idx = lane; idx < pairs; idx += 64) {
    const int m1 = idx / n2, m2 = idx - m1 * n2;
    const int64_t a1 = s1[m1], a2 = s2[m2];
    if (a1 == o || a2 == o || a1 == a2) continue;
    const float v = (e1[m1] * e2[m2]) * between_p(ox, oy, oz, x[a1], y[a1], z[a1], x[a2], y[a2], z[a2]);
    if (v <= 0.f) continue;
    const uint32_t i1 = ids[a1], i2 = ids[a2];
    if (between_better(v, i1, i2, best, b1, b2)) {
      best = v;
      b1 = i1;
      b2 = i2;
    }
  }
  between_wave_best(best, b1, b2);
  out_t = best;
  out_b1 = best > 0.f ? b1 : FARM_NO_ID;
  out_b2 = best > 0.f ? b2 : FARM_NO_ID;
}

// Between's candidate sets as the term kernels see them: per relation slot
// row r, kBetweenSet entries of idx / sim and the count.
constexpr int kBetweenSet = kBetweenSetSize;
struct BetweenView {
  const int32_t* idx = nullptr;  // [R][kBetweenSet]
  const float* sim = nullptr;    // [R][kBetweenSet]
  const int32_t* cnt = nullptr;  // [R]
};

// The term of the Between invocation whose first slot is relation row r.
__device__ inline void between_term_row(const BetweenView& bv, const float* x, const float* y, const float* z,
                                        const uint32_t* ids, int r, int64_t o, int lane, float& t, uint32_t& b1,
                                        uint32_t& b2) {
  between_term_wave(x, y, z, ids, o, lane, bv.idx + (int64_t)r * kBetweenSet, bv.sim + (int64_t)r * kBetweenSet,
                    bv.cnt[r], bv.idx + (int64_t)(r + 1) * kBetweenSet, bv.sim + (int64_t)(r + 1) * kBetweenSet,
                    bv.cnt[r + 1], t, b1, b2);
}

}  // namespace farm
