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
__device__ inline bool is_scanned(int p) { return is_rank(p) || p == FARM_INSIDE; }

struct ScanCtx {
  const float *x, *y, *z;
  const float* ext;  // [3][n] full extents (Inside)
  const uint32_t* ids;
  const int32_t* cls;         // object classes, or null
  const int32_t* cls_order;   // objects in class order (null without classes)
  const int32_t* cls_sorted;  // their classes, ascending
  int32_t tc;                 // the query's parsed target class (-1: none)
  int64_t n;
  int p;                      // FARM_CLOSEST, FARM_FARTHEST or FARM_INSIDE
  int64_t lo = 0, hi = -1;    // the class's range in cls_order (hi < 0: every object is a candidate)
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

__device__ inline float scan_pred_wave(const ScanCtx& k, int64_t o, int64_t a, int lane) {
  return k.p == FARM_INSIDE ? inside_value(k, o, a) : rank_pred_wave(k, o, a, lane);
}

template <class ExactOf>
__device__ inline void scan_visit(const ScanCtx& k, int64_t o, int64_t aa, int lane, ExactOf& exact_of, float& best,
                                  uint32_t& bid) {
  const float s = exact_of(aa);
  if (s < best) return;
  const float v = s * scan_pred_wave(k, o, aa, lane);
  const uint32_t ida = k.ids[aa];
  if (v > best || (v == best && ida < bid)) {
    best = v;
    bid = ida;
  }
}

template <class ExactOf>
__device__ void scan_set_part(const ScanCtx& k, int64_t o, int lane, ExactOf exact_of, const int32_t* sidx, int sn,
                              int w, int parts, float& best, uint32_t& bid) {
  for (int e = w; e < sn; e += parts) {
    const int64_t aa = __builtin_amdgcn_readfirstlane(sidx[e]);
    if (aa != o) scan_visit(k, o, aa, lane, exact_of, best, bid);
  }
}

template <class LoOf, class HiOf, class ExactOf>
__device__ void scan_anchor_part(const ScanCtx& k, int64_t o, int lane, LoOf lo_of, HiOf hi_of, ExactOf exact_of, int w,
                                 int parts, float& best, uint32_t& bid) {
  if (k.p == FARM_INSIDE) {
    // P costs O(1): each lane bounds its anchor's value by sim_lo * P and
    // sim_hi * P (products round monotonically, so they bound the exact s * P);
    // the largest lower bound L prunes every anchor whose upper bound is below it
    float L = best;
    for (int64_t a0 = (int64_t)64 * w; a0 < k.n; a0 += (int64_t)64 * parts) {
      const int64_t a = a0 + lane;
      if (a < k.n && a != o) L = fmaxf(L, lo_of(a) * inside_value(k, o, a));
    }
    L = wave_max_scan(L);
    for (int64_t a0 = (int64_t)64 * w; a0 < k.n; a0 += (int64_t)64 * parts) {
      const int64_t a = a0 + lane;
      const bool valid = a < k.n && a != o;
      const float pv = valid ? inside_value(k, o, a) : 0.f;
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
      scan_visit(k, o, a0 + src, lane, exact_of, best, bid);
    }
  }
}

template <class LoOf, class HiOf, class ExactOf>
__device__ void scan_term_wave(ScanCtx k, int64_t o, int lane, LoOf lo_of, HiOf hi_of, ExactOf exact_of, float& out_best,
                               uint32_t& out_bid, const int32_t* sidx = nullptr, int sn = 0,
                               float out_bound = INFINITY) {
  rank_range(k);
  float best = -1.0f;
  uint32_t bid = FARM_NO_ID;
  scan_set_part(k, o, lane, exact_of, sidx, sn, 0, 1, best, bid);
  if (!(sn > 0 && best > out_bound)) scan_anchor_part(k, o, lane, lo_of, hi_of, exact_of, 0, 1, best, bid);
  out_best = best;
  out_bid = bid;
}

}  // namespace farm
