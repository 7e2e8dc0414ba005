// rescore.hip -- FP32 rescoring of TopK candidates and the final selection.
//
// Reduced-precision form: the similarity GEMM runs in BF16 or FP8 e4m3 and the
// relational pass scores every object from those similarities (an estimate
// s~) and bounds its score from above (s_hi >= s, from proven similarity error
// bounds); the top C = rescore_mult * K objects by s~ are rescored here in
// FP32 and the TopK is taken among them.  The returned set is the exact TopK
// ("certified") whenever the K-th rescored score exceeds the largest s_hi of
// any object outside the candidates.
//
// Rescoring one candidate o: one wave per (candidate, relation) term, then
// one wave per candidate for the composite.
//   s_sem:  the FP32 GEMM's value, or an FP32 dot of the normalised target and
//           descriptor rows when the GEMM ran in reduced precision;
//   t_r:    with a similarity bound |a~_j - a_j| <= delta_j, the best value is
//           at least L = max_j (a~_j - delta_j)+ * P(o, j); only anchors with
//           min(1, a~_j + delta_j) * P(o, j) >= L can reach it, so only those
//           get an FP32 dot product (the wave iterates over the ballot of
//           survivors).  Without a bound (FP32 similarities) the maximum is
//           taken directly.
// With anchor proposals the maximum is first taken over the target's learned
// anchor list and the relation's semantic set only (the same bound-and-survive
// rule for reduced precision).  Every other anchor j has a similarity at most
// tau (the largest one outside the semantic set, plus the error bound) and a
// predicate value at most Pout(o, p) (the largest outside the list), so its
// value is at most tau * Pout (log domain for Near).  A subset maximum strictly
// above that is the exact term and binding; otherwise the anchors are scanned
// in full (the fallback).
// The per-pair arithmetic is the shared pair_math.h, so a rescored term equals
// what the FP32 relational pass computes from the same similarity.
#include <math.h>

#include "farm_internal.h"
#include "pair_math.h"
#include "scan_math.h"
#include "sort_util.h"

namespace farm {
namespace {

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// FP32 dot product of two zero-padded rows (ldk a multiple of 128) by one wave.
// Lane l accumulates elements 2l, 2l+1 of every 128-element slab, in slab
// order; the loads of four slabs are issued before their FMAs so that one
// memory round trip covers four slabs (the arithmetic order is unchanged).
__device__ inline float wave_dot(const float* __restrict__ a, const float* __restrict__ b, int32_t ldk, int lane) {
  float acc = 0.f;
  int k = 2 * lane;
  for (; k + 128 < ldk; k += 2 * 128) {
    float2 x[2], y[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      x[u] = *reinterpret_cast<const float2*>(a + k + 128 * u);
      y[u] = *reinterpret_cast<const float2*>(b + k + 128 * u);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      acc = fmaf(x[u].x, y[u].x, acc);
      acc = fmaf(x[u].y, y[u].y, acc);
    }
  }
  for (; k < ldk; k += 128) {
    const float2 x = *reinterpret_cast<const float2*>(a + k);
    const float2 y = *reinterpret_cast<const float2*>(b + k);
    acc = fmaf(x.x, y.x, acc);
    acc = fmaf(x.y, y.y, acc);
  }
  return wave_sum(acc);
}

// wave_dot with SL slabs of `b` loaded before their FMAs (one memory round
// trip per SL slabs; `a` is read at the FMA, e.g. from LDS).  Same per-lane
// order and reduction tree as wave_dot, so the values are bit-identical.
template <int SL>
__device__ inline float wave_dot_deep(const float* __restrict__ a, const float* __restrict__ b, int32_t ldk,
                                      int lane) {
  float acc = 0.f;
  for (int base = 0; base < ldk; base += SL * 128) {
    float2 y[SL];
#pragma unroll
    for (int u = 0; u < SL; ++u)
      if (base + 128 * u < ldk) y[u] = *reinterpret_cast<const float2*>(b + base + 128 * u + 2 * lane);
#pragma unroll
    for (int u = 0; u < SL; ++u)
      if (base + 128 * u < ldk) {
        const float2 x = *reinterpret_cast<const float2*>(a + base + 128 * u + 2 * lane);
        acc = fmaf(x.x, y[u].x, acc);
        acc = fmaf(x.y, y[u].y, acc);
      }
  }
  return wave_sum(acc);
}

// NN dot products against the same row `a`, interleaved for memory-level
// parallelism; each one with exactly wave_dot's arithmetic (same per-lane
// order, same reduction tree), so the values are bit-identical.  SLABS slabs
// of loads are issued ahead of their FMAs (more registers, fewer round trips).
template <int NN, int SLABS = 1>
__device__ inline void wave_dots(const float* __restrict__ a, const float* const (&b)[NN], int32_t ldk, int lane,
                                 float (&out)[NN]) {
  float acc[NN];
#pragma unroll
  for (int u = 0; u < NN; ++u) acc[u] = 0.f;
  int k = 2 * lane;
  if constexpr (SLABS > 1) {
    for (; k + (SLABS - 1) * 128 < ldk; k += SLABS * 128) {
      float2 x[SLABS], y[SLABS][NN];
#pragma unroll
      for (int s = 0; s < SLABS; ++s) {
        x[s] = *reinterpret_cast<const float2*>(a + k + 128 * s);
#pragma unroll
        for (int u = 0; u < NN; ++u) y[s][u] = *reinterpret_cast<const float2*>(b[u] + k + 128 * s);
      }
#pragma unroll
      for (int s = 0; s < SLABS; ++s)
#pragma unroll
        for (int u = 0; u < NN; ++u) {
          acc[u] = fmaf(x[s].x, y[s][u].x, acc[u]);
          acc[u] = fmaf(x[s].y, y[s][u].y, acc[u]);
        }
    }
  }
  for (; k < ldk; k += 128) {
    const float2 x = *reinterpret_cast<const float2*>(a + k);
#pragma unroll
    for (int u = 0; u < NN; ++u) {
      const float2 y = *reinterpret_cast<const float2*>(b[u] + k);
      acc[u] = fmaf(x.x, y.x, acc[u]);
      acc[u] = fmaf(x.y, y.y, acc[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < NN; ++u) out[u] = wave_sum(acc[u]);
}

__device__ inline bool better(float v, uint32_t id, float bv, uint32_t bid) {
  return v > bv || (v == bv && id < bid);
}

// max with the smallest-id tie-break; the id is read only when v reaches best
__device__ inline void take_max(float v, int64_t j, const uint32_t* __restrict__ ids, float& best, uint32_t& bid) {
  if (v >= best && v != -INFINITY) {
    const uint32_t idj = ids[j];
    if (v > best || idj < bid) {
      best = v;
      bid = idj;
    }
  }
}

// max with the smallest-id tie-break that remembers the anchor's index; the
// ids are read only to break exact ties (resolve with the index at the end)
__device__ inline void take_max_j(float v, int64_t j, const uint32_t* __restrict__ ids, float& best, int64_t& bj) {
  if (v > best) {
    best = v;
    bj = j;
  } else if (v == best && bj >= 0 && j != bj && ids[j] < ids[bj]) {
    bj = j;
  }
}
__device__ inline void take_max_j32(float v, int32_t j, const uint32_t* __restrict__ ids, float& best,
                                    int32_t& bj) {
  if (v > best) {
    best = v;
    bj = j;
  } else if (v == best && bj >= 0 && j != bj && ids[j] < ids[bj]) {
    bj = j;
  }
}

// Wave-wide arg-max with the smallest-id tie-break; every lane gets the result.
__device__ inline void wave_argmax(float& best, uint32_t& bid) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float v = __shfl_xor(best, off);
    const uint32_t id = (uint32_t)__shfl_xor((int)bid, off);
    if (better(v, id, best, bid)) {
      best = v;
      bid = id;
    }
  }
}

__device__ inline float wave_max_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

// Geometry of the memory, passed by value.  z is the targets' vertical
// coordinate and za the anchors' (the same array except for On).
struct Geo {
  const float *x, *y, *z, *za, *hhi, *hlo;  // hhi/hlo: [2][n], lateral then depth pairs
  const uint32_t* ids;
  const float* vz;     // [2][n]: 4 * bottom face, 4 * top face (On)
  const int32_t* cls;  // object classes or null (the candidate set of Closest/Farthest)
  const int32_t *cls_order, *cls_sorted;  // objects in class order, their classes
  const float* ext;    // [3][n] full extents (Inside)
  EntityGeo eg;        // Gaussians and stored views (entity-geometry predicates)
};

// The coordinates predicate p uses: InFrontOf/Behind take the depth pair
// (entries n..2n-1) where the other Left/Right-family predicates take the
// lateral one; On takes the target's bottom and the anchor's top face.
__device__ inline Geo geo_for(const Geo& g, int p, int64_t n) {
  Geo r = g;
  if (is_depth(p)) {
    r.hhi += n;
    r.hlo += n;
  }
  const ZPair zp = z_for(p, g.z, g.vz, n);
  r.z = zp.tgt;
  r.za = zp.anc;
  return r;
}

// Learned anchor lists exist for predicates 0..FARM_NUM_PROP_PRED-1 only.
__device__ inline bool has_lists(int p) { return p < FARM_NUM_PROP_PRED; }

// Anchors of one term: the list of the target (lidx/lval, M entries) and the
// relation's semantic set (sidx, sn entries); M == 0 means none.
struct Subset {
  const int32_t* lidx;
  const float* lval;
  int M;
  const int32_t* sidx;
  int sn;
  const float* ssim;  // exact similarities of the semantic set (reduced precision), or null
  float cert;         // bound on the value of every anchor outside the subset (family domain)
  const float4* sgeo = nullptr;  // the set's anchor coordinates (geo_of layout), or null: read from Geo
};

// An anchor's coordinates as its family uses them: Near (x, y, z), Above/Below
// (z), Left/Right (h hi, h lo).
template <int FAM>
__device__ inline float4 geo_of(int64_t j, const Geo& g) {
  if (FAM == kFamNear) return make_float4(g.x[j], g.y[j], g.za[j], 0.f);
  if (FAM == kFamVert) return make_float4(g.za[j], 0.f, 0.f, 0.f);
  return make_float4(g.hhi[j], g.hlo[j], 0.f, 0.f);
}
// anchor record (as anchor_record_pre) from such coordinates
template <int FAM>
__device__ inline float4 record_of(float a, float la, const float4& c) {
  if (FAM == kFamNear) return make_float4(la, c.x, c.y, c.z);
  if (FAM == kFamVert) return make_float4(a, c.x, 0.f, 0.f);
  return make_float4(a, c.x, c.y, 0.f);
}

// The exact maximum over every anchor of one relation term of target o, by
// one wave.  Returns the family-domain maximum (log for Near) and its anchor id.
// With reduced precision, members of the relation's semantic set (sidx, sn;
// exact similarities ssim, may be null) start the maximum at their exact
// values and never need a dot product of their own.
template <int FAM>
__device__ void full_term(const float* __restrict__ arow, const float* __restrict__ qrow,
                          const float* __restrict__ dn, int32_t ldk, int64_t n, int64_t o, float c, bool bounded,
                          float qn, float qe, const float* __restrict__ o_err, const Geo& g, int lane,
                          const int32_t* __restrict__ sidx, int sn, const float* __restrict__ ssim,
                          float& out_best, uint32_t& out_bid, uint32_t& dots) {
  const Tgt t = load_target(FAM, o, g.x, g.y, g.z, g.hhi, g.hlo);
  float best = value_floor<FAM>();
  uint32_t bid = FARM_NO_ID;
  // lane e < sn holds semantic-set member e (for the membership ballot below)
  int64_t my_member = -1;
  if (bounded && ssim && lane < sn) {
    my_member = sidx[lane];
    if (my_member != o) {
      const float a = ssim[lane];
      take_max(pair_value<FAM>(t, anchor_record(FAM, a, my_member, g.x, g.y, g.za, g.hhi, g.hlo), c), my_member,
               g.ids, best, bid);
    }
  }
  if (!bounded) {
    // FP32 similarities: the maximum directly, with the relational pass's arithmetic
    for (int64_t j = lane; j < n; j += 64) {
      if (j == o) continue;
      const float v = pair_value<FAM>(t, anchor_record(FAM, arow[j], j, g.x, g.y, g.za, g.hhi, g.hlo), c);
      take_max(v, j, g.ids, best, bid);
    }
  } else {
    float lo = best;  // exact values of the semantic-set members are lower bounds too
    for (int64_t j = lane; j < n; j += 64) {
      if (j == o) continue;
      const float a = fmaxf(0.f, arow[j] - fmaf(qn, o_err[j], qe));
      lo = fmaxf(lo, pair_value<FAM>(t, anchor_record(FAM, a, j, g.x, g.y, g.za, g.hhi, g.hlo), c));
    }
    lo = wave_max_f(lo);
    const float L = lo - (fabsf(lo) * 1e-6f + 1e-30f);  // slack for rounding of the bounded values
    for (int64_t base = 0; base < n; base += 64) {
      const int64_t j = base + lane;
      bool f = false;
      if (j < n && j != o) {
        const float a = fminf(1.0f, arow[j] + fmaf(qn, o_err[j], qe));
        f = pair_value<FAM>(t, anchor_record(FAM, a, j, g.x, g.y, g.za, g.hhi, g.hlo), c) >= L;
      }
      uint64_t mask = __ballot(f);
      while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const int64_t j2 = base + src;
        if (__ballot(my_member == j2)) continue;  // a semantic-set member: its exact value is in already
        const float a = fmaxf(0.f, wave_dot(qrow, dn + j2 * ldk, ldk, lane));
        ++dots;
        take_max(pair_value<FAM>(t, anchor_record(FAM, a, j2, g.x, g.y, g.za, g.hhi, g.hlo), c), j2, g.ids, best,
                 bid);
      }
    }
  }
  wave_argmax(best, bid);
  out_best = best;
  out_bid = bid;
}

// The maximum over the subset (the target's list and the relation's semantic
// set) by one wave; true when it certifies the term (strictly above the bound
// on every other anchor).
// Similarity row of the proposal pass: FP32 values (global memory or LDS), or
// BF16 roundings of a reduced-precision GEMM's values staged in LDS, whose
// rounding is folded into the bounds.  BF16 keeps 8 significant bits, so
// round to nearest even moves x by at most 2^-8 |x|: the staged b satisfies
// b (1 - 2^-8) <= x (1 - 2^-16) and x <= b (1 + 2^-8 + 2^-15).  The margin
// m = 2^-8 + 2^-14 therefore gives b (1 - m) <= x <= b (1 + m) with room for
// the FP32 rounding of the products (2^-24 relative).
struct RowF32 {
  const float* p;
  __device__ float get(int64_t j) const { return p[j]; }
  __device__ float lo(int64_t j, float d) const { return fmaxf(0.f, p[j] - d); }
  __device__ float hi(int64_t j, float d) const { return fminf(1.0f, p[j] + d); }
};
constexpr float kBf16Margin = 1.0f / 256.0f + 1.0f / 16384.0f;
__device__ inline float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
struct RowBF16 {
  const uint16_t* p;
  __device__ float get(int64_t j) const { return bf16_value(p[j]); }
  __device__ float lo(int64_t j, float d) const { return fmaxf(0.f, bf16_value(p[j]) * (1.0f - kBf16Margin) - d); }
  __device__ float hi(int64_t j, float d) const { return fminf(1.0f, bf16_value(p[j]) * (1.0f + kBf16Margin) + d); }
};

// subset_term for lists of at most 256 entries, a multiple of 4: each lane
// holds list entries 4l..4l+3 (one 16-byte load of ids, one of cached
// predicate values) and semantic-set member l, all loaded before the first
// use, so one memory round trip serves the whole subset.  Same values, bounds
// and survivor rule as the general form.
constexpr int kRegEntries = 4;
static_assert(kSemMax <= 64, "one semantic-set member per lane");
struct RegList {
  int4 j;    // anchor ids of list entries 4l..4l+3 (-1: none)
  float4 p;  // their cached predicate values
};
__device__ inline RegList load_reg_list(const int32_t* __restrict__ lidx, const float* __restrict__ lval, int M,
                                        int lane) {
  RegList l{make_int4(-1, -1, -1, -1), make_float4(0.f, 0.f, 0.f, 0.f)};
  const int e0 = kRegEntries * lane;
  if (e0 < M) {
    l.j = *reinterpret_cast<const int4*>(lidx + e0);
    l.p = *reinterpret_cast<const float4*>(lval + e0);
  }
  return l;
}

// Survivor queue of the proposal pass (LDS): instead of taking each survivor's
// FP32 dot product inside its term, a wave appends the survivors that can
// still be the maximum to the block's queue, and after all terms the block's
// waves take the queued dot products four at a time (one memory round trip
// serves four) and fold them into the terms' maxima.
constexpr int kDeferCap = 512;  // survivor queue entries per block
__shared__ int32_t dq_n;                  // entries reserved so far
__shared__ uint16_t dq_tag[kDeferCap];    // (term << 8) | list entry index (terms < 256, lists <= 256 entries)
__shared__ int32_t dq_anchor[kDeferCap];  // anchor index of the entry; -1 for a slot left unused

// 64-bit key whose unsigned order is (value, then smaller id): the value's
// IEEE bits mapped monotonically onto unsigned integers, then the inverted id.
// Key 0 stands for "no anchor yet" (below every real key).
__device__ inline uint64_t value_key(float v, uint32_t id) {
  const uint32_t u = __float_as_uint(v);
  const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return ((uint64_t)ord << 32) | (uint64_t)(0xFFFFFFFFu - id);
}
__device__ inline float key_value(uint64_t key) {
  const uint32_t ord = (uint32_t)(key >> 32);
  return __uint_as_float((ord & 0x80000000u) ? (ord & 0x7FFFFFFFu) : ~ord);
}
__device__ inline uint32_t key_id(uint64_t key) { return 0xFFFFFFFFu - (uint32_t)key; }

// Result codes of subset_term_reg: kTermOpen (not certified: the fallback
// scans it), kTermDone (certified), kTermQueued (survivors queued; the set's
// value so far returned).
enum { kTermOpen = 0, kTermDone = 1, kTermQueued = 2 };

template <int FAM, class Row, int SL = 2, bool DEFER = false>
__device__ int subset_term_reg(Row arow, const float* __restrict__ qrow, const float* __restrict__ dn,
                                int32_t ldk, int64_t o, float c, bool bounded, float qn, float qe,
                                const float* __restrict__ o_err, float qd_uniform, const Geo& g, const Subset& sub,
                                const Tgt& t, const RegList& lst, int lane, float& out_best, uint32_t& out_bid,
                                uint32_t& dots, int defer_term = -1) {
  const int4 j4 = lst.j;
  int code = kTermOpen;
  bool full = false;
  const float4 p4 = lst.p;
  const int32_t jl[kRegEntries] = {j4.x, j4.y, j4.z, j4.w};
  const float pl[kRegEntries] = {p4.x, p4.y, p4.z, p4.w};
  // list value from a similarity: cached predicate value times it (log domain for Near)
  auto list_value = [&](float a, float p) { return FAM == kFamNear ? near_log(a) + p : a * p; };
  auto delta = [&](int64_t j) { return o_err ? fmaf(qn, o_err[j], qe) : qd_uniform; };
  float best = value_floor<FAM>();
  int32_t bj = -1;  // anchor index of best
  // semantic-set member of this lane: exact similarity (carried, or the FP32 row)
  // (the member's data are re-read per term, not held across a caller's loop
  // of terms: an opaque copy of the lane index keeps them from being hoisted)
  int sl = lane;
  asm volatile("" : "+v"(sl));
  if (sl < sub.sn) {
    const int32_t js = sub.sidx[sl];
    if (js != o) {
      const float a = bounded ? sub.ssim[sl] : arow.get(js);
      const float4 cs = sub.sgeo ? sub.sgeo[sl] : geo_of<FAM>(js, g);
      best = pair_value<FAM>(t, record_of<FAM>(a, FAM == kFamNear ? near_log(a) : 0.f, cs), c);
      bj = js;
    }
  }
  if (!bounded) {
#pragma unroll
    for (int k = 0; k < kRegEntries; ++k) {
      const int64_t j = jl[k];
      if (j < 0 || j == o) continue;
      take_max_j32(list_value(arow.get(j), pl[k]), (int32_t)j, g.ids, best, bj);
    }
  } else {
    float lo = best;
#pragma unroll
    for (int k = 0; k < kRegEntries; ++k) {
      const int64_t j = jl[k];
      if (j < 0 || j == o) continue;
      lo = fmaxf(lo, list_value(arow.lo(j, delta(j)), pl[k]));
    }
    lo = wave_max_f(lo);
    const float L = lo - (fabsf(lo) * 1e-6f + 1e-30f);  // slack for rounding of the bounded values
    uint32_t surv = 0;  // entries of this lane whose upper bound reaches L
#pragma unroll
    for (int k = 0; k < kRegEntries; ++k) {
      const int64_t j = jl[k];
      if (j < 0 || j == o) continue;
      surv |= (list_value(arow.hi(j, delta(j)), pl[k]) >= L ? 1u : 0u) << k;
    }
    float B = wave_max_f(best);
    if constexpr (DEFER) {
      // queue the survivors whose upper bound reaches the best exact value so
      // far (a queued entry is evaluated like one taken here, so the maximum
      // and its anchor are the same); with the queue full the term is left
      // uncertified (the fallback scans it in full)
      const float Bs = B - (fabsf(B) * 1e-6f + 1e-30f);
      uint32_t keep = 0;
#pragma unroll
      for (int k = 0; k < kRegEntries; ++k)
        if ((surv >> k) & 1u) {
          const int64_t j = jl[k];
          keep |= (list_value(arow.hi(j, delta(j)), pl[k]) >= Bs ? 1u : 0u) << k;
        }
      const int mine = __popc(keep);
      int incl = mine;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
      }
      const int total = __shfl(incl, 63);
      if (total > 0) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&dq_n, total);
        base = __shfl(base, 0);
        if (base + total <= kDeferCap) {
          int pos = base + incl - mine;
#pragma unroll
          for (int k = 0; k < kRegEntries; ++k)
            if ((keep >> k) & 1u) {
              dq_tag[pos] = (uint16_t)((defer_term << 8) | (kRegEntries * lane + k));
              dq_anchor[pos] = jl[k];
              ++pos;
            }
          code = kTermQueued;
        } else {
          for (int i = base + lane; i < base + total && i < kDeferCap; i += 64) dq_anchor[i] = -1;
          best = value_floor<FAM>();
          bj = -1;
          full = true;
        }
      }
      surv = 0;
    }
    // survivors: the entry is re-read (one uniform load) so that nothing of
    // the register-held list stays live across the dot products
#pragma unroll
    for (int k = 0; k < kRegEntries; ++k) {
      uint64_t mask = __ballot((surv >> k) & 1u);
      while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const int e2 = kRegEntries * src + k;
        const int32_t j2 = sub.lidx[e2];
        const float p2 = sub.lval[e2];
        if (list_value(arow.hi(j2, delta(j2)), p2) < B - (fabsf(B) * 1e-6f + 1e-30f)) continue;
        const float a = fmaxf(0.f, wave_dot_deep<SL>(qrow, dn + (int64_t)j2 * ldk, ldk, lane));
        ++dots;
        const float v = list_value(a, p2);
        take_max_j32(v, j2, g.ids, best, bj);
        B = fmaxf(B, v);
      }
    }
  }
  uint32_t bid = bj >= 0 ? g.ids[bj] : FARM_NO_ID;
  wave_argmax(best, bid);
  out_best = best;
  out_bid = bid;
  if (DEFER && (full || code == kTermQueued)) return code;
  return best > sub.cert ? kTermDone : kTermOpen;
}

template <int FAM, class Row>
__device__ bool subset_term_gen(Row arow, const float* __restrict__ qrow, const float* __restrict__ dn,
                                int32_t ldk, int64_t o, float c, bool bounded, float qn, float qe,
                                const float* __restrict__ o_err, float qd_uniform, const Geo& g, const Subset& sub,
                                int lane, float& out_best, uint32_t& out_bid, uint32_t& dots) {
  const Tgt t = load_target(FAM, o, g.x, g.y, g.z, g.hhi, g.hlo);
  float best = value_floor<FAM>();
  int64_t bj = -1;
  const int tot = sub.M + sub.sn;
  auto anchor_of = [&](int e) -> int64_t { return e < sub.M ? sub.lidx[e] : sub.sidx[e - sub.M]; };
  // list entries carry the cached predicate value; semantic-set entries are evaluated
  auto entry = [&](int e, int64_t j, float a, float la) -> float {
    if (e < sub.M) return FAM == kFamNear ? la + sub.lval[e] : a * sub.lval[e];
    return pair_value<FAM>(t, anchor_record_pre(FAM, a, la, j, g.x, g.y, g.za, g.hhi, g.hlo), c);
  };
  // similarity error bound of anchor j (per anchor, or one bound for all)
  auto delta = [&](int64_t j) { return o_err ? fmaf(qn, o_err[j], qe) : qd_uniform; };
  if (!bounded) {
    for (int e = lane; e < tot; e += 64) {
      const int64_t j = anchor_of(e);
      if (j == o) continue;
      const float a = arow.get(j);
      take_max_j(entry(e, j, a, FAM == kFamNear ? near_log(a) : 0.f), j, g.ids, best, bj);
    }
  } else {
    // semantic-set members carry their exact similarity: exact values at once
    for (int e = sub.M + lane; e < tot; e += 64) {
      const int64_t j = anchor_of(e);
      if (j == o) continue;
      const float a = sub.ssim[e - sub.M];
      take_max_j(entry(e, j, a, FAM == kFamNear ? near_log(a) : 0.f), j, g.ids, best, bj);
    }
    // list entries: lower and upper bounds from the reduced-precision
    // similarity, a~ -+ delta; only entries whose upper bound reaches the best
    // lower bound L (the semantic set's exact values included) can be the
    // maximum, and each of those needs an FP32 dot product.
    auto value_at = [&](int e, int64_t j, float a) { return entry(e, j, a, FAM == kFamNear ? near_log(a) : 0.f); };
    auto upper = [&](int e, int64_t j) { return value_at(e, j, arow.hi(j, delta(j))); };
    float lo = best;
    for (int e = lane; e < sub.M; e += 64) {
      const int64_t j = anchor_of(e);
      if (j == o) continue;
      lo = fmaxf(lo, value_at(e, j, arow.lo(j, delta(j))));
    }
    lo = wave_max_f(lo);
    const float L = lo - (fabsf(lo) * 1e-6f + 1e-30f);  // slack for rounding of the bounded values
    // survivors in index order; each exact value raises B, and a survivor
    // whose upper bound has fallen below B (beyond the rounding slack, so ties
    // are still resolved exactly) is skipped without its dot product
    float B = wave_max_f(best);
    for (int base = 0; base < sub.M; base += 64) {
      const int e = base + lane;
      float u = -INFINITY;
      bool f = false;
      if (e < sub.M) {
        const int64_t j = anchor_of(e);
        if (j != o) {
          u = upper(e, j);
          f = u >= L;
        }
      }
      uint64_t mask = __ballot(f);
      while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const float us = __shfl(u, src);
        if (us < B - (fabsf(B) * 1e-6f + 1e-30f)) continue;
        const int e2 = base + src;
        const int64_t j2 = anchor_of(e2);
        const float a = fmaxf(0.f, wave_dot(qrow, dn + j2 * ldk, ldk, lane));
        ++dots;
        const float v = value_at(e2, j2, a);
        take_max_j(v, j2, g.ids, best, bj);
        B = fmaxf(B, v);
      }
    }
  }
  uint32_t bid = bj >= 0 ? g.ids[bj] : FARM_NO_ID;
  wave_argmax(best, bid);
  out_best = best;
  out_bid = bid;
  return best > sub.cert;
}

// Lists of at most 256 entries (a multiple of 4) take the register form.
__device__ inline bool reg_list(int M) { return (M & (kRegEntries - 1)) == 0 && M <= 64 * kRegEntries; }

template <int FAM, class Row = RowF32>
__device__ bool subset_term(Row arow, const float* __restrict__ qrow, const float* __restrict__ dn,
                            int32_t ldk, int64_t o, float c, bool bounded, float qn, float qe,
                            const float* __restrict__ o_err, float qd_uniform, const Geo& g, const Subset& sub,
                            int lane, float& out_best, uint32_t& out_bid, uint32_t& dots) {
  if (reg_list(sub.M))
    return subset_term_reg<FAM>(arow, qrow, dn, ldk, o, c, bounded, qn, qe, o_err, qd_uniform, g, sub,
                                load_target(FAM, o, g.x, g.y, g.z, g.hhi, g.hlo),
                                load_reg_list(sub.lidx, sub.lval, sub.M, lane), lane, out_best, out_bid, dots);
  return subset_term_gen<FAM>(arow, qrow, dn, ldk, o, c, bounded, qn, qe, o_err, qd_uniform, g, sub, lane, out_best,
                              out_bid, dots);
}

// The form fixed at compile time (one form per kernel keeps its register count down).
template <bool REG, int FAM, class Row, int SL = 2, bool DEFER = false>
__device__ inline int subset_term_sel(Row arow, const float* __restrict__ qrow, const float* __restrict__ dn,
                                       int32_t ldk, int64_t o, float c, bool bounded, float qn, float qe,
                                       const float* __restrict__ o_err, float qd_uniform, const Geo& g,
                                       const Subset& sub, const Tgt& t, const RegList& lst, int lane,
                                       float& out_best, uint32_t& out_bid, uint32_t& dots,
                                       int defer_term = -1) {
  if constexpr (REG)
    return subset_term_reg<FAM, Row, SL, DEFER>(arow, qrow, dn, ldk, o, c, bounded, qn, qe, o_err, qd_uniform, g,
                                                sub, t, lst, lane, out_best, out_bid, dots, defer_term);
  else
    return (int)subset_term_gen<FAM>(arow, qrow, dn, ldk, o, c, bounded, qn, qe, o_err, qd_uniform, g, sub, lane,
                                out_best, out_bid, dots);
}

// Proposal subset of term (candidate o, relation r) and the bound on every
// anchor outside it.
__device__ inline Subset make_subset(const PropView& pv, int r, int p, int64_t o, int64_t n, bool bounded, float qnr,
                                     float qer, float err_max) {
  Subset sub;
  const int64_t off = ((int64_t)p * n + o) * pv.m;
  sub.lidx = pv.idx + off;
  sub.lval = pv.val + off;
  sub.M = pv.m;
  sub.sidx = pv.sem_idx + (int64_t)r * kSemMax;
  sub.sn = pv.sem_cnt[r];
  sub.ssim = pv.sem_sim ? pv.sem_sim + (int64_t)r * kSemMax : nullptr;
  const float pout = pv.out[(int64_t)p * n + o];
  // every anchor outside the subset has similarity <= a_hi and predicate value <= pout
  const float a_hi = bounded ? pv.sem_tau[r] + fmaf(qnr, err_max, qer) : pv.sem_tau[r];
  if (family_of(p) == kFamNear) {
    const float b = near_log(a_hi) + pout;
    sub.cert = b + fabsf(b) * 1e-6f;  // covers the rounding of the logarithm
  } else {
    sub.cert = a_hi * pout;
  }
  return sub;
}

constexpr int kTermWaves = 4;    // waves per block
constexpr int kTermBlocksX = 8;  // blocks per query: 32 waves sweep a query's terms

enum { kTermsFull = 0, kTermsSubset = 1, kTermsFallback = 2 };

// Term of a scanned predicate (Closest, Farthest, Inside) of target o by one
// wave (scan_math.h).  Reduced
// precision: an anchor whose upper bound (BF16/FP8 value + error bound)
// reaches the best value so far gets its exact FP32 similarity (wave dot).
// With the relation's semantic set (sidx, sn) and tau, the largest similarity
// outside it (plus the error bound for reduced precision), the set goes first
// and ends the scan when it certifies the term.
template <bool GEO>
__device__ inline void scan_term(const Geo& g, int32_t tc, int p, const float* __restrict__ arow,
                                 const float* __restrict__ qrow, const float* __restrict__ dn, int32_t ldk, int64_t n,
                                 int64_t o, bool bounded, float qnr, float qer, const float* __restrict__ o_err,
                                 int lane, float& best, uint32_t& bid, uint32_t& dots,
                                 const int32_t* __restrict__ sidx = nullptr, int sn = 0, float tau = INFINITY) {
  ScanCtx k{g.x, g.y, g.z, g.ext, g.ids, g.cls, g.cls_order, g.cls_sorted, tc, n, p};
  k.eg = g.eg;
  if (!bounded) {
    scan_term_wave<GEO>(
        k, o, lane, [&](int64_t a) { return arow[a]; }, [&](int64_t a) { return arow[a]; },
        [&](int64_t a) { return arow[a]; }, best, bid, sidx, sn, tau);
  } else {
    scan_term_wave<GEO>(
        k, o, lane, [&](int64_t a) { return fmaxf(0.f, arow[a] - fmaf(qnr, o_err[a], qer)); },
        [&](int64_t a) { return arow[a] + fmaf(qnr, o_err[a], qer); },
        [&](int64_t a) {
          ++dots;
          return fmaxf(0.f, wave_dot(qrow, dn + a * ldk, ldk, lane));
        },
        best, bid, sidx, sn, tau);
  }
}

// One wave per (candidate, relation) term.  Writes the family-domain maximum
// (Near: log of the term; others: the term) into rs_terms and the bound
// anchor into rs_anchor; k_rescore_combine turns them into scores.
//   kTermsFull:     every term over all anchors;
//   kTermsSubset:   every term over its proposal subset; a term the subset
//                   cannot certify is marked NaN;
//   kTermsFallback: the NaN-marked terms over all anchors (a wave tests 64
//                   terms with one ballot).
template <int MODE, bool BOUNDED>
__global__ __launch_bounds__(64 * kTermWaves) void k_rescore_terms(
    const float* __restrict__ sim, int64_t ld_s, int32_t q, MetaView meta, SimBound bound,
    const float* __restrict__ qn, const float* __restrict__ dn, int32_t ldk, const int32_t* __restrict__ cand,
    const int32_t* __restrict__ cand_count, int32_t C, Geo g, int64_t n,
    float* __restrict__ rs_terms, uint32_t* __restrict__ rs_anchor, PropView pv) {
  const int lane = threadIdx.x & 63;
  const int32_t qq = blockIdx.y;
  const int r0 = meta.rel_off[qq], R = meta.rel_off[qq + 1] - r0;
  if (R == 0) return;
  const int32_t cnt = cand_count ? (cand_count[qq] < C ? cand_count[qq] : C) : C;
  const int64_t terms = (int64_t)cnt * R;
  const int wave = blockIdx.x * kTermWaves + (threadIdx.x >> 6);
  const int stride = kTermBlocksX * kTermWaves;
  constexpr bool bounded = BOUNDED;  // reduced-precision similarities with an error bound
  const float err_max = bounded ? *bound.o_err_max : 0.f;
  unsigned long long checked = 0, fell = 0;
  uint32_t dots = 0;
  auto term_args = [&](int64_t tix, int64_t& slot, int& e, int64_t& o) {
    const int32_t cc = (int32_t)(tix / R);
    e = (int)(tix % R);
    slot = (int64_t)qq * C + cc;
    o = cand[slot];
  };
  auto full = [&](int64_t slot, int e, int64_t o) {
    const int r = r0 + e;
    if (is_scanned(meta.rel_pred[r])) return;  // k_scan_terms takes these
    const int32_t* sidx = pv.sem_idx ? pv.sem_idx + (int64_t)r * kSemMax : nullptr;
    const int sn = pv.sem_idx ? pv.sem_cnt[r] : 0;
    const float* ssim = pv.sem_sim ? pv.sem_sim + (int64_t)r * kSemMax : nullptr;
    const int p = meta.rel_pred[r];
    const float c = sigmoid_scale(p);
    const Geo gp = geo_for(g, p, n);
    const float* arow = sim + (int64_t)(q + r) * ld_s;
    const float* qrow = qn + (int64_t)(q + r) * ldk;
    const float qnr = bounded ? bound.q_nrm[q + r] : 0.f;
    const float qer = bounded ? bound.q_err[q + r] + bound.acc : 0.f;
    float best;
    uint32_t bid;
    switch (family_of(p)) {
      case kFamNear:
        full_term<kFamNear>(arow, qrow, dn, ldk, n, o, c, bounded, qnr, qer, bound.o_err, gp, lane, sidx, sn, ssim,
                             best, bid, dots);
        break;
      case kFamVert:
        full_term<kFamVert>(arow, qrow, dn, ldk, n, o, c, bounded, qnr, qer, bound.o_err, gp, lane, sidx, sn, ssim,
                             best, bid, dots);
        break;
      default:
        full_term<kFamLat>(arow, qrow, dn, ldk, n, o, c, bounded, qnr, qer, bound.o_err, gp, lane, sidx, sn, ssim,
                             best, bid, dots);
        break;
    }
    if (lane == 0) {
      rs_terms[slot * kMaxRel + e] = best;
      rs_anchor[slot * kMaxRel + e] = bid;
    }
  };
  if (MODE == kTermsFallback) {
    for (int64_t base = (int64_t)wave * 64; base < terms; base += (int64_t)stride * 64) {
      const int64_t tix = base + lane;
      bool marked = false;
      if (tix < terms) {
        int64_t slot, o;
        int e;
        term_args(tix, slot, e, o);
        marked = o >= 0 && isnan(rs_terms[slot * kMaxRel + e]);
      }
      uint64_t mask = __ballot(marked);
      while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        int64_t slot, o;
        int e;
        term_args(base + src, slot, e, o);
        full(slot, e, o);
      }
    }
  } else {
    for (int64_t tix = wave; tix < terms; tix += stride) {
      int64_t slot, o;
      int e;
      term_args(tix, slot, e, o);
      if (o < 0) continue;
      if (MODE == kTermsFull) {
        full(slot, e, o);
        checked += meta.rel_pred[r0 + e] != FARM_AND;
        continue;
      }
      const int r = r0 + e;
      const int p = meta.rel_pred[r];
      if (p == FARM_AND) continue;  // written with the Between slot before it
      const float c = sigmoid_scale(p);
      const Geo gp = geo_for(g, p, n);
      const float* arow = sim + (int64_t)(q + r) * ld_s;
      const float* qrow = qn + (int64_t)(q + r) * ldk;
      const float qnr = bounded ? bound.q_nrm[q + r] : 0.f;
      const float qer = bounded ? bound.q_err[q + r] + bound.acc : 0.f;
      float best = 0.f;
      uint32_t bid = FARM_NO_ID;
      bool ok = false;  // a predicate without lists is left to the fallback
      if (has_lists(p)) {
      const Subset sub = make_subset(pv, r, p, o, n, bounded, qnr, qer, err_max);
      switch (family_of(p)) {
        case kFamNear:
          ok = subset_term<kFamNear>(RowF32{arow}, qrow, dn, ldk, o, c, bounded, qnr, qer, bound.o_err, 0.f, gp, sub, lane, best,
                                     bid, dots);
          break;
        case kFamVert:
          ok = subset_term<kFamVert>(RowF32{arow}, qrow, dn, ldk, o, c, bounded, qnr, qer, bound.o_err, 0.f, gp, sub, lane, best,
                                     bid, dots);
          break;
        default:
          ok = subset_term<kFamLat>(RowF32{arow}, qrow, dn, ldk, o, c, bounded, qnr, qer, bound.o_err, 0.f, gp, sub, lane, best,
                                    bid, dots);
          break;
      }
      }
      if (lane == 0) {
        rs_terms[slot * kMaxRel + e] = ok ? best : NAN;  // NaN: scanned in full by the fallback pass
        rs_anchor[slot * kMaxRel + e] = bid;
        if (!ok && pv.fb_list) {
          const uint32_t pos = atomicAdd(pv.fb_count, 1u);
          if (pos < pv.fb_cap) pv.fb_list[pos] = ((unsigned long long)qq << 32) | (unsigned long long)tix;
        }
      }
      checked += 1;
      fell += ok ? 0 : 1;
    }
  }
  if (pv.stats && lane == 0 && (checked || dots)) {
    if (checked) atomicAdd(&pv.stats[0], checked);
    if (fell) atomicAdd(&pv.stats[1], fell);
    if (dots) atomicAdd(&pv.stats[MODE == kTermsSubset ? 2 : 3], (unsigned long long)dots);
  }
}

// Terms of the scanned predicates (Closest, Farthest, Inside), one wave per
// term: every such term of the candidates (SWEEP = false: the bound-pruned
// method), or those still unresolved (NaN) after the listed fallback (SWEEP =
// true).  A kernel of its own keeps k_rescore_terms' register budget.
template <bool BOUNDED, bool SWEEP, bool GEO>
__global__ __launch_bounds__(64 * kTermWaves) void k_scan_terms(
    const float* __restrict__ sim, int64_t ld_s, int32_t q, MetaView meta, SimBound bound,
    const float* __restrict__ qn, const float* __restrict__ dn, int32_t ldk, const int32_t* __restrict__ cand,
    const int32_t* __restrict__ cand_count, int32_t C, Geo g, int64_t n,
    float* __restrict__ rs_terms, uint32_t* __restrict__ rs_anchor, PropView pv) {
  const int lane = threadIdx.x & 63;
  const int32_t qq = blockIdx.y;
  const int r0 = meta.rel_off[qq], R = meta.rel_off[qq + 1] - r0;
  if (R == 0) return;
  const int32_t cnt = cand_count ? (cand_count[qq] < C ? cand_count[qq] : C) : C;
  const int64_t terms = (int64_t)cnt * R;
  const int wave = blockIdx.x * kTermWaves + (threadIdx.x >> 6);
  const int stride = kTermBlocksX * kTermWaves;
  const float err_max = BOUNDED ? *bound.o_err_max : 0.f;
  uint32_t dots = 0;
  for (int64_t tix = wave; tix < terms; tix += stride) {
    const int e = (int)(tix % R);
    const int r = r0 + e;
    const int p = meta.rel_pred[r];
    if (!is_scanned(p) || p == FARM_AND) continue;  // a Between's second slot: written with its first
    if (is_entity_geo(p) != GEO) continue;           // the other instance takes it
    const int64_t slot = (int64_t)qq * C + tix / R;
    const int64_t o = cand[slot];
    if (o < 0) continue;
    if (SWEEP && !isnan(rs_terms[slot * kMaxRel + e])) continue;
    if (!GEO && p == FARM_BETWEEN) {
      float t;
      uint32_t b1, b2;
      between_term_row(BetweenView{pv.btw_idx, pv.btw_sim, pv.btw_cnt}, g.x, g.y, g.z, g.ids, r, o, lane, t, b1, b2);
      if (lane == 0) {
        rs_terms[slot * kMaxRel + e] = t;
        rs_terms[slot * kMaxRel + e + 1] = t;
        rs_anchor[slot * kMaxRel + e] = b1;
        rs_anchor[slot * kMaxRel + e + 1] = b2;
      }
      continue;
    }
    const float* arow = sim + (int64_t)(q + r) * ld_s;
    const float* qrow = qn + (int64_t)(q + r) * ldk;
    const float qnr = BOUNDED ? bound.q_nrm[q + r] : 0.f;
    const float qer = BOUNDED ? bound.q_err[q + r] + bound.acc : 0.f;
    // with a semantic set (proposal fallback) the set goes first and may certify the term
    const int32_t* sidx = pv.sem_idx ? pv.sem_idx + (int64_t)r * kSemMax : nullptr;
    const int sn = pv.sem_idx ? pv.sem_cnt[r] : 0;
    const float tau = sidx ? pv.sem_tau[r] + (BOUNDED ? fmaf(qnr, err_max, qer) : 0.f) : INFINITY;
    float best;
    uint32_t bid;
    scan_term<GEO>(geo_for(g, p, n), meta.tcls[qq], p, arow, qrow, dn, ldk, n, o, BOUNDED, qnr, qer, bound.o_err,
                   lane, best, bid, dots, sidx, sn, tau);
    if (lane == 0) {
      rs_terms[slot * kMaxRel + e] = best;
      rs_anchor[slot * kMaxRel + e] = bid;
    }
  }
  if (pv.stats && lane == 0 && dots) atomicAdd(&pv.stats[3], (unsigned long long)dots);
}

// Proposal pass with the relation's similarity row staged in LDS: one block
// per relation row serves every candidate of its query, so the list entries'
// similarity gathers hit LDS instead of L2.  The block also selects the
// relation's semantic set from the staged row (threshold gamma * max with
// gamma in 1/2, 3/4, 7/8, ... until at most kSemMax anchors exceed it; the
// largest similarity outside bounds the rest), takes the members' exact FP32
// similarities for reduced precision, and publishes the set for the fallback
// scans.  List bounds use the largest descriptor error (no per-anchor
// gather); the exact values are unchanged.
constexpr int kLdsThreads = 512;
constexpr int kLdsWaves = kLdsThreads / 64;

__device__ inline float block_max_lds(float v, float* red) {
  v = wave_max_f(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float m = red[0];
  for (int i = 1; i < kLdsWaves; ++i) m = fmaxf(m, red[i]);
  return m;
}

constexpr int kStageLoads = 8;  // row staging: float4 loads per thread in flight
constexpr int kLdsDotSlabs = 4;  // FP32 dots: descriptor slabs (128 floats) per memory round trip

// Dynamic LDS of the proposal pass: the staged row (BF16 or FP32, padded to a
// multiple of 4 elements).
__host__ __device__ inline size_t subset_row_bytes(int64_t n, bool bounded) {
  return (size_t)((n + 3) & ~(int64_t)3) * (bounded ? sizeof(uint16_t) : sizeof(float));
}
constexpr int kCandLds = 256;   // candidates whose id, coordinates and outside bound are staged in LDS
static_assert(kCandLds <= 256, "a queued survivor's term index takes 8 bits");

template <bool BOUNDED, bool REG, bool QUEUE>
__global__ __launch_bounds__(kLdsThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_rescore_subset_lds(
    const float* __restrict__ sim, int64_t ld_s, int32_t q, MetaView meta, SimBound bound,
    const float* __restrict__ qn, const float* __restrict__ dn, int32_t ldk, const int32_t* __restrict__ cand,
    const int32_t* __restrict__ cand_count, int32_t C, Geo g, int64_t n, float* __restrict__ rs_terms,
    uint32_t* __restrict__ rs_anchor, PropView pv) {
  // FP32 row (exact similarities) or, for a reduced-precision GEMM whose values
  // only feed bounds, its BF16 rounding (half the LDS, more blocks per CU)
  extern __shared__ float srow[];
  uint16_t* srow16 = reinterpret_cast<uint16_t*>(srow);
  auto staged = [&](int64_t j) { return BOUNDED ? bf16_value(srow16[j]) : srow[j]; };
  __shared__ float red[kLdsWaves];
  __shared__ int32_t set_idx[kSemMax];
  __shared__ float set_sim[kSemMax];
  __shared__ float4 set_geo[kSemMax];
  __shared__ int32_t c_id[kCandLds];
  __shared__ float4 c_geo[kCandLds];
  __shared__ float c_pout[kCandLds];
  __shared__ int32_t set_n;
  __shared__ unsigned long long wave_cnt[kLdsWaves][3];
  // survivor queue and the queued terms' running maxima (reduced precision, register lists)
  constexpr bool kDefer = BOUNDED && REG && QUEUE;
  __shared__ unsigned long long t_key[kDefer ? kCandLds : 1];
  __shared__ uint32_t t_def[kDefer ? kCandLds / 32 : 1];
  __shared__ uint32_t fell_def;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t r = blockIdx.x;
  const int32_t qq = meta.rel_query[r];
  const int r0 = meta.rel_off[qq], R = meta.rel_off[qq + 1] - r0;
  const int e = r - r0;
  const float* arow = sim + (int64_t)(q + r) * ld_s;
  // Reduced precision without the survivor queue (FP8): the relation's query
  // row is staged in LDS after the similarity row, since every survivor's dot
  // product reads it
  constexpr bool kQrowLds = BOUNDED && !kDefer;
  float* q_lds = reinterpret_cast<float*>(reinterpret_cast<char*>(srow) + subset_row_bytes(n, BOUNDED));
  if (kQrowLds) {
    const float* qsrc = qn + (int64_t)(q + r) * ldk;
    for (int i = threadIdx.x; i < ldk; i += kLdsThreads) q_lds[i] = qsrc[i];
  }
  // stage the row (rows start 256-byte aligned)
  const int64_t n4 = n >> 2;
  const float4* a4 = reinterpret_cast<const float4*>(arow);
  float4* s4 = reinterpret_cast<float4*>(srow);
  float mx = 0.f;
  // kStageLoads loads per thread in flight before the first use
  for (int64_t base = threadIdx.x; base < n4; base += kStageLoads * kLdsThreads) {
    float4 v[kStageLoads];
#pragma unroll
    for (int u = 0; u < kStageLoads; ++u) {
      const int64_t i = base + (int64_t)u * kLdsThreads;
      v[u] = i < n4 ? a4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < kStageLoads; ++u) {
      const int64_t i = base + (int64_t)u * kLdsThreads;
      if (i >= n4) break;
      if (BOUNDED) {
        ushort4 h;
        h.x = bf16_rne(v[u].x);
        h.y = bf16_rne(v[u].y);
        h.z = bf16_rne(v[u].z);
        h.w = bf16_rne(v[u].w);
        reinterpret_cast<ushort4*>(srow16)[i] = h;
      } else {
        s4[i] = v[u];
      }
      mx = fmaxf(fmaxf(mx, fmaxf(v[u].x, v[u].y)), fmaxf(v[u].z, v[u].w));
    }
  }
  for (int64_t j = (n4 << 2) + threadIdx.x; j < n; j += kLdsThreads) {
    if (BOUNDED) srow16[j] = bf16_rne(arow[j]);
    else srow[j] = arow[j];
    mx = fmaxf(mx, arow[j]);
  }
  if (kDefer) {
    if (threadIdx.x == 0) {
      dq_n = 0;
      fell_def = 0;
    }
    if ((int)threadIdx.x < kCandLds / 32) t_def[threadIdx.x] = 0;
  }
  const float amax = block_max_lds(mx, red);  // synchronises: the row is staged
  // semantic set: the threshold is tau_k = amax - amax / 2^k for the smallest
  // k in 1..kSemLevels with at most kSemMax similarities above it (kSemLevels
  // if there is none), the thresholds formed by the float operations of
  // repeated halving.  One pass over the row: tau_k is non-decreasing in k, so
  // each similarity above tau_1 finds the largest k with v > tau_k by binary
  // search and is counted in a histogram over k; the count above tau_k is the
  // histogram's suffix sum from k.
  constexpr int kSemLevels = 31;
  __shared__ float tau_tab[kSemLevels + 1];
  __shared__ int32_t lvl_hist[kSemLevels + 1];
  if ((int)threadIdx.x <= kSemLevels) {
    float gap = 0.5f * amax, t = 0.5f * amax;
    for (int k = 1; k < (int)threadIdx.x; ++k) {
      gap *= 0.5f;
      t = amax - gap;
    }
    tau_tab[threadIdx.x] = t;  // entry 0 is unused
    lvl_hist[threadIdx.x] = 0;
  }
  __syncthreads();
  const float tau1 = tau_tab[1];
  for (int64_t j = threadIdx.x; j < n; j += kLdsThreads) {
    const float v = staged(j);
    if (!(v > tau1)) continue;
    int lo = 1, hi = kSemLevels;  // v > tau_tab[lo]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (v > tau_tab[mid]) lo = mid;
      else hi = mid - 1;
    }
    atomicAdd(&lvl_hist[lo], 1);
  }
  __syncthreads();
  int ks = kSemLevels;
  {
    int32_t above = 0;
    for (int k = kSemLevels; k >= 1; --k) {
      above += lvl_hist[k];
      if (above > kSemMax) break;
      ks = k;
    }
  }
  const float tau = tau_tab[ks];
  if (threadIdx.x == 0) set_n = 0;
  __syncthreads();
  float out = 0.f;
  for (int64_t j = threadIdx.x; j < n; j += kLdsThreads) {
    const float v = staged(j);
    bool member = false;
    if (v > tau) {
      const int32_t pos = atomicAdd(&set_n, 1);
      if (pos < kSemMax) {
        set_idx[pos] = (int32_t)j;
        member = true;
      }
    }
    if (!member) out = fmaxf(out, v);
  }
  // largest similarity outside the set (a staged BF16 value bounds its source within the margin)
  const float tau_out = block_max_lds(out, red) * (BOUNDED ? 1.0f + kBf16Margin : 1.0f);  // synchronises
  const int sn = set_n < kSemMax ? set_n : kSemMax;
  const float* qrow = kQrowLds ? q_lds : qn + (int64_t)(q + r) * ldk;
  const int p = meta.rel_pred[r];
  const int fam = family_of(p);
  const Geo gp = geo_for(g, p, n);
  const bool tab = has_lists(p);  // without lists every term goes to the fallback
  const bool second = p == FARM_AND;  // a Between's second slot: its terms are written with the first
  const int32_t cnt = cand_count ? (cand_count[qq] < C ? cand_count[qq] : C) : C;
  // the set's anchor coordinates and the first kCandLds candidates (id, own
  // coordinates, bound on the predicate outside the list), read once for all
  // of the relation's terms
  auto coords = [&](int64_t j, const Geo& gg) {
    return fam == kFamNear ? geo_of<kFamNear>(j, gg) : fam == kFamVert ? geo_of<kFamVert>(j, gg)
                                                       : geo_of<kFamLat>(j, gg);
  };
  // candidates are targets: their vertical coordinate is z, not the anchors' za
  // (they differ for On: bottom and top faces); same layout as load_target
  Geo gt = gp;
  gt.za = gp.z;
  if ((int)threadIdx.x < sn) set_geo[threadIdx.x] = coords(set_idx[threadIdx.x], gp);
  for (int32_t i = threadIdx.x; i < cnt && i < kCandLds; i += kLdsThreads) {
    const int32_t o = cand[(int64_t)qq * C + i];
    c_id[i] = o;
    if (o >= 0) {
      c_geo[i] = coords(o, gt);
      c_pout[i] = tab ? pv.out[(int64_t)p * n + o] : 0.f;
    }
  }
  uint32_t dots = 0;  // FP32 dot products of this wave
  if (BOUNDED) {
    // four members per wave at a time (members past the set repeat the last one and are dropped)
    for (int m0 = 4 * wave; m0 < sn; m0 += 4 * kLdsWaves) {
      const float* rows[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) rows[u] = dn + (int64_t)set_idx[m0 + u < sn ? m0 + u : sn - 1] * ldk;
      float d[4];
      wave_dots<4, 3>(qrow, rows, ldk, lane, d);
      if (lane == 0)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (m0 + u < sn) set_sim[m0 + u] = fmaxf(0.f, d[u]);
      dots += (uint32_t)(sn - m0 < 4 ? sn - m0 : 4);  // counted with the wave's other dot products
    }
  }
  __syncthreads();
  // publish the set for the fallback scans
  if ((int)threadIdx.x < sn) {
    pv.sem_idx_out[(int64_t)r * kSemMax + threadIdx.x] = set_idx[threadIdx.x];
    if (BOUNDED) pv.sem_sim_out[(int64_t)r * kSemMax + threadIdx.x] = set_sim[threadIdx.x];
  }
  if (threadIdx.x == 0) {
    pv.sem_cnt_out[r] = sn;
    pv.sem_tau_out[r] = tau_out;
  }
  const float c = sigmoid_scale(p);
  const float qnr = BOUNDED ? bound.q_nrm[q + r] : 0.f;
  const float qer = BOUNDED ? bound.q_err[q + r] + bound.acc : 0.f;
  const float err_max = BOUNDED ? *bound.o_err_max : 0.f;
  const float qd = BOUNDED ? fmaf(qnr, err_max, qer) : 0.f;
  unsigned long long checked = 0, fell = 0;
  // this wave's terms are candidates wave, wave + kLdsWaves, ...
  // (wave-uniform values are moved to scalar registers: fewer vector registers)
  auto uni = [](float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); };
  // with the survivor queue the loop takes the first kCandLds candidates (the
  // queued terms' results have LDS slots); the rest follow after the queue
  const int32_t cnt1 = kDefer && cnt > kCandLds ? kCandLds : cnt;
  auto o_of = [&](int32_t cc) -> int64_t {
    if (cc >= cnt1) return -1;
    return __builtin_amdgcn_readfirstlane(cc < kCandLds ? c_id[cc] : cand[(int64_t)qq * C + cc]);
  };
  // register form: the next term's list ids are loaded while the current
  // term is evaluated (its predicate values at the start of its turn)
  auto ids_of = [&](int64_t o) {
    int4 j = make_int4(-1, -1, -1, -1);
    // the lane's offset is formed anew per call (opaque copy): hoisted out of
    // the terms loop, its 64-bit address would be held, or spilled, across it
    int l4 = kRegEntries * lane;
    asm volatile("" : "+v"(l4));
    if (l4 < pv.m) j = *reinterpret_cast<const int4*>(pv.idx + ((int64_t)p * n + o) * pv.m + l4);
    return j;
  };
  int64_t o_nx = o_of(wave);
  int4 j_nx = make_int4(-1, -1, -1, -1);
  if (REG && tab && o_nx >= 0) j_nx = ids_of(o_nx);
  for (int32_t cc = second ? cnt1 : wave; cc < cnt1; cc += kLdsWaves) {
    const int64_t slot = (int64_t)qq * C + cc;
    const int64_t o = REG ? o_nx : o_of(cc);
    RegList lst{j_nx, make_float4(0.f, 0.f, 0.f, 0.f)};
    if (REG && tab && o >= 0 && kRegEntries * lane < pv.m)
      lst.p = *reinterpret_cast<const float4*>(pv.val + ((int64_t)p * n + o) * pv.m + kRegEntries * lane);
    if (REG) {
      o_nx = o_of(cc + kLdsWaves);
      if (tab && o_nx >= 0) j_nx = ids_of(o_nx);
    }
    if (o < 0) continue;
    Tgt t;
    float pout;
    if (cc < kCandLds) {
      const float4 tc = c_geo[cc];
      t = Tgt{uni(tc.x), uni(tc.y), uni(tc.z)};
      pout = uni(c_pout[cc]);
    } else {
      t = load_target(fam, o, gp.x, gp.y, gp.z, gp.hhi, gp.hlo);
      pout = tab ? pv.out[(int64_t)p * n + o] : 0.f;
    }
    Subset sub;
    const int64_t off = ((int64_t)p * n + o) * pv.m;
    sub.lidx = pv.idx + off;
    sub.lval = pv.val + off;
    sub.M = pv.m;
    sub.sidx = set_idx;
    sub.sn = sn;
    sub.ssim = BOUNDED ? set_sim : nullptr;
    sub.sgeo = set_geo;
    const float a_hi = BOUNDED ? tau_out + qd : tau_out;
    if (family_of(p) == kFamNear) {
      const float b = near_log(a_hi) + pout;
      sub.cert = b + fabsf(b) * 1e-6f;  // covers the rounding of the logarithm
    } else {
      sub.cert = a_hi * pout;
    }
    float best = 0.f;
    uint32_t bid = FARM_NO_ID;
    int code = kTermOpen;
    const int dterm = kDefer ? (int)cc : -1;
    if (tab) switch (family_of(p)) {
      case kFamNear:
        if constexpr (BOUNDED)
          code = subset_term_sel<REG, kFamNear, RowBF16, kLdsDotSlabs, kDefer>(RowBF16{srow16}, qrow, dn, ldk, o, c, true, qnr, qer, nullptr, qd, gp, sub, t, lst, lane,
                                     best, bid, dots, dterm);
        else
          code = subset_term_sel<REG, kFamNear, RowF32, kLdsDotSlabs>(RowF32{srow}, qrow, dn, ldk, o, c, false, qnr, qer, nullptr, qd, gp, sub, t, lst, lane,
                                     best, bid, dots);
        break;
      case kFamVert:
        if constexpr (BOUNDED)
          code = subset_term_sel<REG, kFamVert, RowBF16, kLdsDotSlabs, kDefer>(RowBF16{srow16}, qrow, dn, ldk, o, c, true, qnr, qer, nullptr, qd, gp, sub, t, lst, lane,
                                     best, bid, dots, dterm);
        else
          code = subset_term_sel<REG, kFamVert, RowF32, kLdsDotSlabs>(RowF32{srow}, qrow, dn, ldk, o, c, false, qnr, qer, nullptr, qd, gp, sub, t, lst, lane,
                                     best, bid, dots);
        break;
      default:
        if constexpr (BOUNDED)
          code = subset_term_sel<REG, kFamLat, RowBF16, kLdsDotSlabs, kDefer>(RowBF16{srow16}, qrow, dn, ldk, o, c, true, qnr, qer, nullptr, qd, gp, sub, t, lst, lane,
                                     best, bid, dots, dterm);
        else
          code = subset_term_sel<REG, kFamLat, RowF32, kLdsDotSlabs>(RowF32{srow}, qrow, dn, ldk, o, c, false, qnr, qer, nullptr, qd, gp, sub, t, lst, lane,
                                     best, bid, dots);
        break;
    }
    checked += 1;
    const bool ok = code == kTermDone;
    if (kDefer && code == kTermQueued) {
      // the set's exact values so far; the queued survivors follow after the loop
      if (lane == 0) {
        t_key[cc] = bid == FARM_NO_ID ? 0ull : value_key(best, bid);
        atomicOr(&t_def[cc >> 5], 1u << (cc & 31));
      }
      continue;
    }
    if (lane == 0) {
      rs_terms[slot * kMaxRel + e] = ok ? best : NAN;  // NaN: scanned in full by the fallback pass
      rs_anchor[slot * kMaxRel + e] = bid;
      if (!ok && pv.fb_list) {
        const uint32_t pos = atomicAdd(pv.fb_count, 1u);
        if (pos < pv.fb_cap)
          pv.fb_list[pos] = ((unsigned long long)qq << 32) | (unsigned long long)((int64_t)cc * R + e);
      }
    }
    fell += ok ? 0 : 1;
  }
  if constexpr (kDefer) {
    // the queued survivors' FP32 dot products, four per wave at a time, folded
    // into their terms' maxima (value, then smaller id, as in the term loop)
    __syncthreads();
    const int nq = dq_n < kDeferCap ? dq_n : kDeferCap;
    const float floor_v = fam == kFamNear ? -INFINITY : -1.0f;
    for (int b0 = 4 * wave; b0 < nq; b0 += 4 * kLdsWaves) {
      int32_t aj[4];
      const float* rows[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = b0 + u;
        aj[u] = i < nq ? dq_anchor[i] : -1;
        rows[u] = dn + (int64_t)(aj[u] >= 0 ? aj[u] : 0) * ldk;
      }
      float d[4];
      wave_dots<4, 3>(qrow, rows, ldk, lane, d);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (aj[u] < 0) continue;
        ++dots;
        if (lane == 0) {
          const uint32_t tg = dq_tag[b0 + u];
          const int term = (int)(tg >> 8), e2 = (int)(tg & 0xFFu);
          const int32_t j2 = aj[u];
          const float p2 = pv.val[((int64_t)p * n + c_id[term]) * pv.m + e2];
          const float a = fmaxf(0.f, d[u]);
          const float v = fam == kFamNear ? near_log(a) + p2 : a * p2;
          // an entry at the floor value binds only where the set already did (as in the term loop)
          if (v > floor_v || t_key[term] != 0ull) atomicMax(&t_key[term], value_key(v, gp.ids[j2]));
        }
      }
    }
    __syncthreads();
    // the queued terms' results: certificate, outputs, fallback worklist
    const int nt = cnt < kCandLds ? cnt : kCandLds;
    const float a_hi = tau_out + qd;
    for (int cc = threadIdx.x; cc < nt; cc += kLdsThreads) {
      if (!((t_def[cc >> 5] >> (cc & 31)) & 1u)) continue;
      const unsigned long long key = t_key[cc];
      const float best = key ? key_value(key) : floor_v;
      const uint32_t bid = key ? key_id(key) : FARM_NO_ID;
      const float pout = c_pout[cc];
      float cert;
      if (fam == kFamNear) {
        const float b = near_log(a_hi) + pout;
        cert = b + fabsf(b) * 1e-6f;
      } else {
        cert = a_hi * pout;
      }
      const bool ok = best > cert;
      const int64_t slot = (int64_t)qq * C + cc;
      rs_terms[slot * kMaxRel + e] = ok ? best : NAN;
      rs_anchor[slot * kMaxRel + e] = bid;
      if (!ok) {
        if (pv.fb_list) {
          const uint32_t pos = atomicAdd(pv.fb_count, 1u);
          if (pos < pv.fb_cap)
            pv.fb_list[pos] = ((unsigned long long)qq << 32) | (unsigned long long)((int64_t)cc * R + e);
        }
        atomicAdd(&fell_def, 1u);
      }
    }
    // candidates past the first kCandLds: each term with its survivors' dot products taken in place
    for (int32_t cc = second ? cnt : kCandLds + wave; cc < cnt; cc += kLdsWaves) {
      const int64_t o = __builtin_amdgcn_readfirstlane(cand[(int64_t)qq * C + cc]);
      if (o < 0) continue;
      const int64_t slot = (int64_t)qq * C + cc;
      const Tgt t = load_target(fam, o, gp.x, gp.y, gp.z, gp.hhi, gp.hlo);
      const float pout = tab ? pv.out[(int64_t)p * n + o] : 0.f;
      Subset sub;
      const int64_t off = ((int64_t)p * n + o) * pv.m;
      sub.lidx = pv.idx + off;
      sub.lval = pv.val + off;
      sub.M = pv.m;
      sub.sidx = set_idx;
      sub.sn = sn;
      sub.ssim = set_sim;
      sub.sgeo = set_geo;
      if (fam == kFamNear) {
        const float b = near_log(a_hi) + pout;
        sub.cert = b + fabsf(b) * 1e-6f;
      } else {
        sub.cert = a_hi * pout;
      }
      float best = 0.f;
      uint32_t bid = FARM_NO_ID;
      bool ok = false;
      if (tab) {
        const RegList lst = load_reg_list(sub.lidx, sub.lval, sub.M, lane);
        switch (fam) {
          case kFamNear:
            ok = subset_term_sel<REG, kFamNear, RowBF16, kLdsDotSlabs>(RowBF16{srow16}, qrow, dn, ldk, o, c, true, qnr,
                                                                        qer, nullptr, qd, gp, sub, t, lst, lane, best,
                                                                        bid, dots);
            break;
          case kFamVert:
            ok = subset_term_sel<REG, kFamVert, RowBF16, kLdsDotSlabs>(RowBF16{srow16}, qrow, dn, ldk, o, c, true, qnr,
                                                                        qer, nullptr, qd, gp, sub, t, lst, lane, best,
                                                                        bid, dots);
            break;
          default:
            ok = subset_term_sel<REG, kFamLat, RowBF16, kLdsDotSlabs>(RowBF16{srow16}, qrow, dn, ldk, o, c, true, qnr,
                                                                       qer, nullptr, qd, gp, sub, t, lst, lane, best,
                                                                       bid, dots);
            break;
        }
      }
      if (lane == 0) {
        rs_terms[slot * kMaxRel + e] = ok ? best : NAN;
        rs_anchor[slot * kMaxRel + e] = bid;
        if (!ok && pv.fb_list) {
          const uint32_t pos = atomicAdd(pv.fb_count, 1u);
          if (pos < pv.fb_cap)
            pv.fb_list[pos] = ((unsigned long long)qq << 32) | (unsigned long long)((int64_t)cc * R + e);
        }
      }
      checked += 1;
      fell += ok ? 0 : 1;
    }
  }
  // counters: summed over the block's waves, then one atomic each per block
  __syncthreads();
  if (lane == 0) {
    wave_cnt[wave][0] = checked;
    wave_cnt[wave][1] = fell;
    wave_cnt[wave][2] = dots;
  }
  __syncthreads();
  if (pv.stats && threadIdx.x < 3) {
    unsigned long long t = 0;
    for (int i = 0; i < kLdsWaves; ++i) t += wave_cnt[i][threadIdx.x];
    if (kDefer && threadIdx.x == 1) t += fell_def;
    if (t) atomicAdd(&pv.stats[threadIdx.x], t);
  }
}

constexpr int kFbThreads = 512;

// Block-wide arg-max (smallest id on ties) of per-thread (best, bid).
__device__ inline void block_argmax(float& best, uint32_t& bid, float* sv, uint32_t* sid) {
  wave_argmax(best, bid);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sv[w] = best;
    sid[w] = bid;
  }
  __syncthreads();
  best = sv[0];
  bid = sid[0];
  for (int i = 1; i < kFbThreads / 64; ++i)
    if (better(sv[i], sid[i], best, bid)) {
      best = sv[i];
      bid = sid[i];
    }
}

// Smallest BF16 value >= f (round toward +inf; f finite or -inf).
__device__ inline uint16_t bf16_ceil(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)(f >= 0.f ? (u + 0xFFFFu) >> 16 : u >> 16);
}

constexpr int kFbLoads = 4;       // anchors per thread whose loads are in flight together
constexpr int kFbLds = 20480;     // anchors whose upper values are kept in LDS (40 KB)

// The exact maximum over every anchor of one term by a whole block (the
// block-wide form of full_term, same per-pair arithmetic and survivors rule).
// Loads are issued kFbLoads anchors at a time.  Reduced precision: the first
// pass takes the lower values and keeps each anchor's upper value, rounded up
// to BF16, in LDS (the first kFbLds anchors; the rest are recomputed), and the
// survivors are the anchors whose kept upper value reaches the best lower one.
template <int FAM, bool BOUNDED>
__device__ void full_term_block(const float* __restrict__ arow, const float* __restrict__ qrow,
                                const float* __restrict__ dn, int32_t ldk, int64_t n, int64_t o, float c, float qn,
                                float qe, const float* __restrict__ o_err, const Geo& g,
                                const int32_t* __restrict__ sidx, int sn, const float* __restrict__ ssim, float* sv,
                                uint32_t* sid, uint16_t* hup, float& out_best, uint32_t& out_bid, uint32_t& dots) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const Tgt t = load_target(FAM, o, g.x, g.y, g.z, g.hhi, g.hlo);
  float best = value_floor<FAM>();
  uint32_t bid = FARM_NO_ID;
  int64_t my_member = -1;  // lane e < sn of every wave holds semantic-set member e
  if (BOUNDED && ssim && lane < sn) {
    my_member = sidx[lane];
    if (w == 0 && my_member != o) {
      const float a = ssim[lane];
      take_max(pair_value<FAM>(t, anchor_record(FAM, a, my_member, g.x, g.y, g.za, g.hhi, g.hlo), c), my_member,
               g.ids, best, bid);
    }
  }
  auto value = [&](float a, const float4& cj) {
    return pair_value<FAM>(t, record_of<FAM>(a, FAM == kFamNear ? near_log(a) : 0.f, cj), c);
  };
  if (!BOUNDED) {
    for (int64_t b0 = tid; b0 < n; b0 += (int64_t)kFbThreads * kFbLoads) {
      float av[kFbLoads];
      float4 cv[kFbLoads];
#pragma unroll
      for (int u = 0; u < kFbLoads; ++u) {
        const int64_t j = b0 + (int64_t)u * kFbThreads;
        const int64_t jj = j < n ? j : n - 1;
        av[u] = arow[jj];
        cv[u] = geo_of<FAM>(jj, g);
      }
#pragma unroll
      for (int u = 0; u < kFbLoads; ++u) {
        const int64_t j = b0 + (int64_t)u * kFbThreads;
        if (j < n && j != o) take_max(value(av[u], cv[u]), j, g.ids, best, bid);
      }
    }
  } else {
    float lo = best;
    // lower and upper values of anchor j from its loaded similarity, error and coordinates
    auto bounds = [&](int64_t j, float a, float e, const float4& cj, float& vlo, float& vhi) {
      const float d = fmaf(qn, e, qe);
      vlo = value(fmaxf(0.f, a - d), cj);
      vhi = value(fminf(1.0f, a + d), cj);
    };
    for (int64_t b0 = tid; b0 < n; b0 += (int64_t)kFbThreads * kFbLoads) {
      float av[kFbLoads], ev[kFbLoads];
      float4 cv[kFbLoads];
#pragma unroll
      for (int u = 0; u < kFbLoads; ++u) {
        const int64_t j = b0 + (int64_t)u * kFbThreads;
        const int64_t jj = j < n ? j : n - 1;
        av[u] = arow[jj];
        ev[u] = o_err[jj];
        cv[u] = geo_of<FAM>(jj, g);
      }
#pragma unroll
      for (int u = 0; u < kFbLoads; ++u) {
        const int64_t j = b0 + (int64_t)u * kFbThreads;
        if (j >= n) break;
        float vlo = -INFINITY, vhi = -INFINITY;
        if (j != o) bounds(j, av[u], ev[u], cv[u], vlo, vhi);
        lo = fmaxf(lo, vlo);
        if (j < kFbLds) hup[j] = bf16_ceil(vhi);
      }
    }
    lo = wave_max_f(lo);
    __syncthreads();  // also publishes the kept upper values
    if (lane == 0) sv[w] = lo;
    __syncthreads();
    for (int i = 0; i < kFbThreads / 64; ++i) lo = fmaxf(lo, sv[i]);
    const float L = lo - (fabsf(lo) * 1e-6f + 1e-30f);  // slack for rounding of the bounded values
    // each wave resolves the survivors of its own 64-anchor chunks
    for (int64_t base = (int64_t)w * 64; base < n; base += kFbThreads) {
      const int64_t j = base + lane;
      bool f = false;
      if (j < n && j != o) {
        if (j < kFbLds) {
          f = __uint_as_float((uint32_t)hup[j] << 16) >= L;
        } else {
          float vlo, vhi;
          bounds(j, arow[j], o_err[j], geo_of<FAM>(j, g), vlo, vhi);
          f = vhi >= L;
        }
      }
      uint64_t mask = __ballot(f);
      while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const int64_t j2 = base + src;
        if (__ballot(my_member == j2)) continue;  // a semantic-set member: its exact value is in already
        const float a = fmaxf(0.f, wave_dot(qrow, dn + j2 * ldk, ldk, lane));
        ++dots;
        take_max(pair_value<FAM>(t, anchor_record(FAM, a, j2, g.x, g.y, g.za, g.hhi, g.hlo), c), j2, g.ids, best,
                 bid);
      }
    }
  }
  block_argmax(best, bid, sv, sid);
  out_best = best;
  out_bid = bid;
}

// Term of a scanned predicate of target o by a whole fallback block: its waves
// split the semantic set and then (unless the set certifies the term) the
// anchor scan, merging (best, id) through LDS after each phase.
template <bool BOUNDED, bool GEO>
__device__ void scan_term_block(const Geo& g, int32_t tc, int p, const float* __restrict__ arow,
                                const float* __restrict__ qrow, const float* __restrict__ dn, int32_t ldk, int64_t n,
                                int64_t o, float qnr, float qer, const float* __restrict__ o_err,
                                const int32_t* __restrict__ sidx, int sn, float tau, float* sv, uint32_t* sid,
                                float& out_best, uint32_t& out_bid, uint32_t& dots) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int parts = kFbThreads / 64;
  ScanCtx k{g.x, g.y, g.z, g.ext, g.ids, g.cls, g.cls_order, g.cls_sorted, tc, n, p};
  k.eg = g.eg;
  rank_range(k);
  auto hi_of = [&](int64_t a) { return BOUNDED ? arow[a] + fmaf(qnr, o_err[a], qer) : arow[a]; };
  auto lo_of = [&](int64_t a) { return BOUNDED ? fmaxf(0.f, arow[a] - fmaf(qnr, o_err[a], qer)) : arow[a]; };
  auto exact_of = [&](int64_t a) {
    if (!BOUNDED) return arow[a];
    ++dots;
    return fmaxf(0.f, wave_dot(qrow, dn + a * ldk, ldk, lane));
  };
  float best = -1.0f;
  uint32_t bid = FARM_NO_ID;
  auto merge = [&]() {
    __syncthreads();
    if (lane == 0) {
      sv[w] = best;
      sid[w] = bid;
    }
    __syncthreads();
    for (int u = 0; u < parts; ++u) {
      const float v = sv[u];
      const uint32_t id = sid[u];
      if (v > best || (v == best && id < bid)) {
        best = v;
        bid = id;
      }
    }
  };
  scan_set_part<GEO>(k, o, lane, exact_of, sidx, sn, w, parts, best, bid);
  merge();
  if (!(sn > 0 && best > tau)) {
    scan_anchor_part<GEO>(k, o, lane, lo_of, hi_of, exact_of, w, parts, best, bid);
    merge();
  }
  out_best = best;
  out_bid = bid;
}

// One block per listed uncertified term (grid-stride over the worklist).
template <bool BOUNDED>
__global__ __launch_bounds__(kFbThreads) void k_rescore_fallback(
    const float* __restrict__ sim, int64_t ld_s, int32_t q, MetaView meta, SimBound bound,
    const float* __restrict__ qn, const float* __restrict__ dn, int32_t ldk, const int32_t* __restrict__ cand,
    int32_t C, Geo g, int64_t n, float* __restrict__ rs_terms, uint32_t* __restrict__ rs_anchor, PropView pv) {
  __shared__ float sv[kFbThreads / 64];
  __shared__ uint32_t sid[kFbThreads / 64];
  __shared__ uint16_t hup[BOUNDED ? kFbLds : 1];
  const uint32_t listed = *pv.fb_count;
  const int64_t count = listed < pv.fb_cap ? (int64_t)listed : pv.fb_cap;
  uint32_t dots = 0;
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
    const unsigned long long item = pv.fb_list[i];
    const int32_t qq = (int32_t)(item >> 32);
    const int64_t tix = (int64_t)(item & 0xFFFFFFFFull);
    const int r0 = meta.rel_off[qq], R = meta.rel_off[qq + 1] - r0;
    const int32_t cc = (int32_t)(tix / R);
    const int e = (int)(tix % R);
    const int64_t slot = (int64_t)qq * C + cc;
    const int64_t o = cand[slot];
    const int r = r0 + e;
    const int p = meta.rel_pred[r];
    if (is_scanned(p)) continue;  // k_scan_fallback takes these (block-uniform skip)
    const float c = sigmoid_scale(p);
    const Geo gp = geo_for(g, p, n);
    const float* arow = sim + (int64_t)(q + r) * ld_s;
    const float* qrow = qn + (int64_t)(q + r) * ldk;
    const float qnr = BOUNDED ? bound.q_nrm[q + r] : 0.f;
    const float qer = BOUNDED ? bound.q_err[q + r] + bound.acc : 0.f;
    const int32_t* sidx = pv.sem_idx + (int64_t)r * kSemMax;
    const int sn = pv.sem_cnt[r];
    const float* ssim = pv.sem_sim ? pv.sem_sim + (int64_t)r * kSemMax : nullptr;
    float best = 0.f;
    uint32_t bid = FARM_NO_ID;
    switch (family_of(p)) {
      case kFamNear:
        full_term_block<kFamNear, BOUNDED>(arow, qrow, dn, ldk, n, o, c, qnr, qer, bound.o_err, gp, sidx, sn, ssim, sv,
                                           sid, hup, best, bid, dots);
        break;
      case kFamVert:
        full_term_block<kFamVert, BOUNDED>(arow, qrow, dn, ldk, n, o, c, qnr, qer, bound.o_err, gp, sidx, sn, ssim, sv,
                                           sid, hup, best, bid, dots);
        break;
      default:
        full_term_block<kFamLat, BOUNDED>(arow, qrow, dn, ldk, n, o, c, qnr, qer, bound.o_err, gp, sidx, sn, ssim, sv,
                                          sid, hup, best, bid, dots);
        break;
    }
    if (threadIdx.x == 0) {
      rs_terms[slot * kMaxRel + e] = best;
      rs_anchor[slot * kMaxRel + e] = bid;
    }
    __syncthreads();
  }
  if (pv.stats && (threadIdx.x & 63) == 0 && dots) atomicAdd(&pv.stats[3], (unsigned long long)dots);
}

// The worklist's terms of scanned predicates (Closest, Farthest, Inside): the
// block's waves split each term (scan_term_block).  A kernel of its own so
// that the pairwise fallback keeps its register budget.
template <bool BOUNDED, bool GEO>
__global__ __launch_bounds__(kFbThreads) void k_scan_fallback(
    const float* __restrict__ sim, int64_t ld_s, int32_t q, MetaView meta, SimBound bound,
    const float* __restrict__ qn, const float* __restrict__ dn, int32_t ldk, const int32_t* __restrict__ cand,
    int32_t C, Geo g, int64_t n, float* __restrict__ rs_terms, uint32_t* __restrict__ rs_anchor, PropView pv) {
  __shared__ float sv[kFbThreads / 64];
  __shared__ uint32_t sid[kFbThreads / 64];
  const uint32_t listed = *pv.fb_count;
  const int64_t count = listed < pv.fb_cap ? (int64_t)listed : pv.fb_cap;
  uint32_t dots = 0;
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
    const unsigned long long item = pv.fb_list[i];
    const int32_t qq = (int32_t)(item >> 32);
    const int64_t tix = (int64_t)(item & 0xFFFFFFFFull);
    const int r0 = meta.rel_off[qq], R = meta.rel_off[qq + 1] - r0;
    const int32_t cc = (int32_t)(tix / R);
    const int e = (int)(tix % R);
    const int r = r0 + e;
    const int p = meta.rel_pred[r];
    if (!is_scanned(p) || p == FARM_AND) continue;  // block-uniform
    if (is_entity_geo(p) != GEO) continue;           // the other instance takes it
    const int64_t slot = (int64_t)qq * C + cc;
    const int64_t o = cand[slot];
    if (!GEO && p == FARM_BETWEEN) {  // one wave takes the invocation's term (both slots)
      if (threadIdx.x < 64) {
        float t;
        uint32_t b1, b2;
        between_term_row(BetweenView{pv.btw_idx, pv.btw_sim, pv.btw_cnt}, g.x, g.y, g.z, g.ids, r, o,
                         (int)threadIdx.x, t, b1, b2);
        if (threadIdx.x == 0) {
          rs_terms[slot * kMaxRel + e] = t;
          rs_terms[slot * kMaxRel + e + 1] = t;
          rs_anchor[slot * kMaxRel + e] = b1;
          rs_anchor[slot * kMaxRel + e + 1] = b2;
        }
      }
      __syncthreads();
      continue;
    }
    const float* arow = sim + (int64_t)(q + r) * ld_s;
    const float* qrow = qn + (int64_t)(q + r) * ldk;
    const float qnr = BOUNDED ? bound.q_nrm[q + r] : 0.f;
    const float qer = BOUNDED ? bound.q_err[q + r] + bound.acc : 0.f;
    // the semantic set goes first and may certify the term
    const float tau = pv.sem_tau[r] + (BOUNDED ? fmaf(qnr, *bound.o_err_max, qer) : 0.f);
    float best = 0.f;
    uint32_t bid = FARM_NO_ID;
    scan_term_block<BOUNDED, GEO>(geo_for(g, p, n), meta.tcls[qq], p, arow, qrow, dn, ldk, n, o, qnr, qer, bound.o_err,
                             pv.sem_idx + (int64_t)r * kSemMax, pv.sem_cnt[r], tau, sv, sid, best, bid, dots);
    if (threadIdx.x == 0) {
      rs_terms[slot * kMaxRel + e] = best;
      rs_anchor[slot * kMaxRel + e] = bid;
    }
    __syncthreads();
  }
  if (pv.stats && (threadIdx.x & 63) == 0 && dots) atomicAdd(&pv.stats[3], (unsigned long long)dots);
}

// Composite score of every candidate from its family-domain maxima: one wave
// per candidate.  The target similarity is the FP32 GEMM's value, or an FP32
// dot product when the similarity matrix is reduced-precision.  Terms become
// linear; slots past the query's R get 0 and FARM_NO_ID.
__global__ __launch_bounds__(256) void k_rescore_combine(
    const float* __restrict__ sim, int64_t ld_s, int32_t q, MetaView meta, SimBound bound, const float* __restrict__ qn,
    const float* __restrict__ dn, int32_t ldk, const int32_t* __restrict__ cand, const int32_t* __restrict__ cand_count,
    int32_t C, const int32_t* __restrict__ cls, float* __restrict__ rs_score, float* __restrict__ rs_terms,
    uint32_t* __restrict__ rs_anchor) {
  const int lane = threadIdx.x & 63;
  const int32_t qq = blockIdx.y;
  const int32_t cnt = cand_count ? (cand_count[qq] < C ? cand_count[qq] : C) : C;
  const int r0 = meta.rel_off[qq], R = meta.rel_off[qq + 1] - r0;
  const bool bounded = bound.q_nrm != nullptr;
  const int tc = meta.tcls[qq];
  // four candidates per wave: their target dot products interleaved, then one lane each for the composite
  for (int32_t c0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 4; c0 < cnt; c0 += gridDim.x * 16) {
    int64_t o4[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) o4[u] = c0 + u < cnt ? cand[(int64_t)qq * C + c0 + u] : -1;
    float dot4[4] = {0.f, 0.f, 0.f, 0.f};
    if (bounded) {
      const float* rows[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) rows[u] = dn + (o4[u] >= 0 ? o4[u] : 0) * ldk;
      wave_dots<4, 3>(qn + (int64_t)qq * ldk, rows, ldk, lane, dot4);
    }
    if (lane >= 4 || c0 + lane >= cnt) continue;
    float dot = dot4[0];
#pragma unroll
    for (int u = 1; u < 4; ++u)
      if (lane == u) dot = dot4[u];
    const int64_t slot = (int64_t)qq * C + c0 + lane;
    const int64_t o = o4[0] * (lane == 0) + o4[1] * (lane == 1) + o4[2] * (lane == 2) + o4[3] * (lane == 3);
    if (o < 0) {
      rs_score[slot] = -INFINITY;
      for (int e = 0; e < kMaxRel; ++e) {
        rs_terms[slot * kMaxRel + e] = 0.f;
        rs_anchor[slot * kMaxRel + e] = FARM_NO_ID;
      }
      continue;
    }
    float sem;
    if (!bounded) {
      sem = sim[(int64_t)qq * ld_s + o];
    } else {
      const float kappa = (tc >= 0 && cls && cls[o] >= 0 && cls[o] != tc) ? kClassFactor : 1.0f;
      sem = kappa * fmaxf(0.f, dot);
    }
    float lsum = 0.f;
    int inv = 0;  // predicate invocations (a Between's two slots count once)
    for (int e = 0; e < R; ++e) {
      const float v = rs_terms[slot * kMaxRel + e];
      const int p = meta.rel_pred[r0 + e];
      if (family_of(p) == kFamNear) {
        lsum += v;
        rs_terms[slot * kMaxRel + e] = term_of<kFamNear>(v);
      } else {
        const float term = term_of<kFamVert>(v);
        if (p != FARM_AND) lsum += logf(term);
        rs_terms[slot * kMaxRel + e] = term;
      }
      inv += p != FARM_AND;
    }
    const float gm = inv > 0 ? expf(lsum / (float)inv) : 1.0f;
    rs_score[slot] = sem * ((1.0f - kW) + kW * gm);
    for (int e = R; e < kMaxRel; ++e) {
      rs_terms[slot * kMaxRel + e] = 0.f;
      rs_anchor[slot * kMaxRel + e] = FARM_NO_ID;
    }
  }
}

__global__ __launch_bounds__(256) void k_rescore_select(const float* __restrict__ rs_score,
                                                        const int32_t* __restrict__ rs_idx,
                                                        const float* __restrict__ rs_terms,
                                                        const uint32_t* __restrict__ rs_anchor,
                                                        const uint32_t* __restrict__ ids, int32_t C, int32_t k,
                                                        const uint64_t* __restrict__ hi_key,
                                                        const int32_t* __restrict__ hi_idx,
                                                        const int32_t* __restrict__ cand_count, int64_t n,
                                                        uint32_t* __restrict__ out_id, float* __restrict__ out_score,
                                                        float* __restrict__ out_terms,
                                                        uint32_t* __restrict__ out_anchor,
                                                        int32_t* __restrict__ certified) {
  __shared__ uint64_t keys[kSortMax];
  __shared__ int32_t slot[kSortMax];
  __shared__ int32_t first_out;
  const int32_t qq = blockIdx.x;
  // slots at or beyond the query's candidate count hold nothing
  const int32_t used = cand_count ? (cand_count[qq] < C ? cand_count[qq] : C) : C;
  const int P = pow2_at_least(used > 0 ? used : 1);
  for (int e = threadIdx.x; e < P; e += blockDim.x) {
    int32_t o = e < used ? rs_idx[(int64_t)qq * C + e] : -1;
    keys[e] = o >= 0 ? make_key(rs_score[(int64_t)qq * C + e], ids[o]) : 0;
    slot[e] = o >= 0 ? e : -1;
  }
  if (threadIdx.x == 0) first_out = C + 1;
  __syncthreads();
  // position of the best-bounded object that is not a candidate
  if (certified) {
    for (int e = threadIdx.x; e <= C; e += blockDim.x) {
      const int32_t o = hi_idx[(int64_t)qq * (C + 1) + e];
      bool member = false;
      for (int m = 0; m < C && !member; ++m) member = rs_idx[(int64_t)qq * C + m] == o;
      if (!member) atomicMin(&first_out, e);
    }
  }
  bitonic_desc(keys, slot, P);  // synchronises
  for (int e = threadIdx.x; e < k; e += blockDim.x) {
    const int64_t out = (int64_t)qq * k + e;
    const uint64_t kk = e < P ? keys[e] : 0;
    const int32_t sl = e < P ? slot[e] : -1;
    out_id[out] = kk ? key_id(kk) : FARM_NO_ID;
    out_score[out] = kk ? key_score(kk) : -INFINITY;
    for (int r = 0; r < kMaxRel; ++r) {
      if (out_terms) out_terms[out * kMaxRel + r] = sl >= 0 ? rs_terms[((int64_t)qq * C + sl) * kMaxRel + r] : 0.f;
      if (out_anchor)
        out_anchor[out * kMaxRel + r] = sl >= 0 ? rs_anchor[((int64_t)qq * C + sl) * kMaxRel + r] : FARM_NO_ID;
    }
  }
  if (certified && threadIdx.x == 0) {
    int ok;
    const uint64_t bound_key = first_out <= C ? hi_key[(int64_t)qq * (C + 1) + first_out] : 0;
    if (n <= C || bound_key == 0) {
      ok = 1;  // every object was rescored
    } else {
      const uint64_t kth = k - 1 < P ? keys[k - 1] : 0;
      const float sk = kth ? key_score(kth) : -INFINITY;
      ok = (sk - (1e-5f * fabsf(sk) + 4e-6f)) > key_score(bound_key) ? 1 : 0;
    }
    certified[qq] = ok;
  }
}

// One wave per (relation, semantic-set member): max(0, FP32 dot).
__global__ __launch_bounds__(256) void k_semantic_exact(const float* __restrict__ qn, const float* __restrict__ dn,
                                                        int32_t ldk, int32_t q, int32_t R,
                                                        const int32_t* __restrict__ sem_idx,
                                                        const int32_t* __restrict__ sem_cnt,
                                                        float* __restrict__ sem_sim) {
  const int lane = threadIdx.x & 63;
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int32_t r = (int32_t)(w / kSemMax), e = (int32_t)(w % kSemMax);
  if (r >= R || e >= sem_cnt[r]) return;  // whole waves leave
  const int64_t j = sem_idx[(int64_t)r * kSemMax + e];
  const float a = fmaxf(0.f, wave_dot(qn + (int64_t)(q + r) * ldk, dn + j * ldk, ldk, lane));
  if (lane == 0) sem_sim[(int64_t)r * kSemMax + e] = a;
}

__global__ __launch_bounds__(256) void k_max_reduce(const float* __restrict__ v, int64_t n, float* __restrict__ out) {
  __shared__ float red[256];
  float m = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 256) m = fmaxf(m, v[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

// Whether a similarity row of `bytes` can be staged in LDS by the proposal
// pass on `device` (raises the kernel's dynamic LDS limit once as needed).
bool lds_row_fits(int device, size_t bytes, bool bounded) {
  static int limit[64] = {0};
  static size_t granted[2][64] = {{0}};
  if (device < 0 || device >= 64) return false;
  if (limit[device] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) v = -1;
    limit[device] = v > 0 ? v : -1;
  }
  const void* fn[3] = {bounded ? reinterpret_cast<const void*>(&k_rescore_subset_lds<true, false, false>)
                               : reinterpret_cast<const void*>(&k_rescore_subset_lds<false, false, false>),
                       bounded ? reinterpret_cast<const void*>(&k_rescore_subset_lds<true, true, false>)
                               : reinterpret_cast<const void*>(&k_rescore_subset_lds<false, true, false>),
                       bounded ? reinterpret_cast<const void*>(&k_rescore_subset_lds<true, true, true>)
                               : reinterpret_cast<const void*>(&k_rescore_subset_lds<false, true, false>)};
  // the kernels' own (static) LDS comes on top of the row
  static size_t stat[2] = {0, 0};
  size_t& st = stat[bounded ? 1 : 0];
  if (st == 0) {
    for (const void* f : fn) {
      hipFuncAttributes fa;
      if (hipFuncGetAttributes(&fa, f) != hipSuccess) {
        (void)hipGetLastError();
        return false;
      }
      st = fa.sharedSizeBytes > st ? fa.sharedSizeBytes : st;
    }
  }
  if (limit[device] < 0 || bytes + st > (size_t)limit[device]) return false;
  size_t& g = granted[bounded ? 1 : 0][device];
  if (bytes > 65536 && bytes > g) {
    for (const void* f : fn)
      if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;
      }
    g = bytes;
  }
  return true;
}

bool proposal_pass_in_lds(const farm_memory* mem, bool bounded) {
  // the largest dynamic size an instance uses: the row, plus the query row without the queue
  return lds_row_fits(mem->device, subset_row_bytes(mem->n, bounded) + (bounded ? sizeof(float) * (size_t)mem->ldk : 0),
                      bounded);
}

hipError_t launch_rescore_terms(const farm_memory* mem, const farm_workspace* ws, const float* sim, int64_t ld_s,
                                int32_t q, MetaView meta, const SimBound& bound, const int32_t* cand,
                                const int32_t* cand_count, int32_t c, const PropView& prop_in, bool fallback_pass,
                                hipStream_t s) {
  if (q <= 0 || c <= 0) return hipSuccess;
  const Geo g{mem->x, mem->y, mem->z,   mem->z,   mem->hr_hi,     mem->hr_lo,
              mem->id, mem->vz, mem->cls, mem->cls_order, mem->cls_sorted, mem->ext, entity_geo(mem)};
  const dim3 grid(kTermBlocksX, (unsigned)q), block(64 * kTermWaves);
  PropView prop = prop_in;  // with Between's candidate sets
  prop.btw_idx = ws->btw_idx;
  prop.btw_sim = ws->btw_sim;
  prop.btw_cnt = ws->btw_cnt;
#define FARM_TERMS(MODE, B)                                                                                      \
  hipLaunchKernelGGL((k_rescore_terms<MODE, B>), grid, block, 0, s, sim, ld_s, q, meta, bound, ws->qn, mem->dn, \
                     mem->ldk, cand, cand_count, c, g, mem->n, ws->rs_terms, ws->rs_anchor, prop)
  const bool bounded = bound.q_nrm != nullptr;
  const int mode = prop.m > 0 ? (fallback_pass ? kTermsFallback : kTermsSubset) : kTermsFull;
  if (mode == kTermsFull && fallback_pass) return hipSuccess;
  if (mode == kTermsSubset && prop.fb_count) {
    hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(prop.fb_count), 1, 0, s);
    if (e != hipSuccess) return e;
  }
  if (mode == kTermsFallback && prop.fb_list) {
    // listed terms, one block each; then the sweep below finds any the list could not hold
    const unsigned blocks = 2048;
    if (bounded)
      hipLaunchKernelGGL((k_rescore_fallback<true>), dim3(blocks), dim3(kFbThreads), 0, s, sim, ld_s, q, meta, bound,
                         ws->qn, mem->dn, mem->ldk, cand, c, g, mem->n, ws->rs_terms, ws->rs_anchor, prop);
    else
      hipLaunchKernelGGL((k_rescore_fallback<false>), dim3(blocks), dim3(kFbThreads), 0, s, sim, ld_s, q, meta, bound,
                         ws->qn, mem->dn, mem->ldk, cand, c, g, mem->n, ws->rs_terms, ws->rs_anchor, prop);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // terms of the scanned predicates on the worklist: the entity-geometry ones by an instance of their own
#define FARM_SCANFB(B, GEO)                                                                                       \
  hipLaunchKernelGGL((k_scan_fallback<B, GEO>), dim3(blocks), dim3(kFbThreads), 0, s, sim, ld_s, q, meta, bound, \
                     ws->qn, mem->dn, mem->ldk, cand, c, g, mem->n, ws->rs_terms, ws->rs_anchor, prop)
    if (meta.scan_n > meta.geo_n) {
      if (bounded) FARM_SCANFB(true, false);
      else FARM_SCANFB(false, false);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (meta.geo_n > 0) {
      if (bounded) FARM_SCANFB(true, true);
      else FARM_SCANFB(false, true);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
#undef FARM_SCANFB
  }
  if (mode == kTermsSubset) {
    const size_t lds = subset_row_bytes(mem->n, bounded);
    const size_t lds_q = lds + (bounded ? sizeof(float) * (size_t)mem->ldk : 0);  // + the query row (no queue)
    if (prop.in_lds) {
      const int32_t R = prop.rel_total;
      if (R <= 0) return hipSuccess;
#define FARM_LDS(B, REG, QUEUE, BYTES)                                                                          \
  hipLaunchKernelGGL((k_rescore_subset_lds<B, REG, QUEUE>), dim3((unsigned)R), dim3(kLdsThreads), BYTES, s, sim, ld_s, q, \
                     meta, bound, ws->qn, mem->dn, mem->ldk, cand, cand_count, c, g, mem->n, ws->rs_terms,        \
                     ws->rs_anchor, prop)
      const bool reg = (prop.m & (kRegEntries - 1)) == 0 && prop.m <= 64 * kRegEntries;
      if (bounded) {
        if (reg && prop.queue) FARM_LDS(true, true, true, lds);
        else if (reg) FARM_LDS(true, true, false, lds_q);
        else FARM_LDS(true, false, false, lds_q);
      } else {
        if (reg) FARM_LDS(false, true, false, lds);
        else FARM_LDS(false, false, false, lds);
      }
#undef FARM_LDS
      return hipGetLastError();
    }
  }
  if (bounded) {
    if (mode == kTermsSubset) FARM_TERMS(kTermsSubset, true);
    else if (mode == kTermsFallback) FARM_TERMS(kTermsFallback, true);
    else FARM_TERMS(kTermsFull, true);
  } else {
    if (mode == kTermsSubset) FARM_TERMS(kTermsSubset, false);
    else if (mode == kTermsFallback) FARM_TERMS(kTermsFallback, false);
    else FARM_TERMS(kTermsFull, false);
  }
#undef FARM_TERMS
  if (meta.scan_n > 0 && mode != kTermsSubset) {  // the scanned predicates' terms
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
#define FARM_SCAN(B, SW, GEO)                                                                                    \
  hipLaunchKernelGGL((k_scan_terms<B, SW, GEO>), grid, block, 0, s, sim, ld_s, q, meta, bound, ws->qn, mem->dn,  \
                     mem->ldk, cand, cand_count, c, g, mem->n, ws->rs_terms, ws->rs_anchor, prop)
    const bool sweep = mode == kTermsFallback;
    for (int geo = 0; geo < 2; ++geo) {
      if (geo ? meta.geo_n == 0 : meta.scan_n == meta.geo_n) continue;
      if (bounded) {
        if (sweep) { if (geo) FARM_SCAN(true, true, true); else FARM_SCAN(true, true, false); }
        else { if (geo) FARM_SCAN(true, false, true); else FARM_SCAN(true, false, false); }
      } else {
        if (sweep) { if (geo) FARM_SCAN(false, true, true); else FARM_SCAN(false, true, false); }
        else { if (geo) FARM_SCAN(false, false, true); else FARM_SCAN(false, false, false); }
      }
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
#undef FARM_SCAN
  }
  return hipGetLastError();
}

hipError_t launch_rescore_combine(const farm_memory* mem, const farm_workspace* ws, const float* sim, int64_t ld_s,
                                  int32_t q, MetaView meta, const SimBound& bound, const int32_t* cand,
                                  const int32_t* cand_count, int32_t c, hipStream_t s) {
  if (q <= 0 || c <= 0) return hipSuccess;
  // two blocks (32 candidates per sweep) per query: more blocks than that mostly find no work, and
  // dispatching them costs more than the loop they save
  const unsigned gx = (unsigned)((c + 15) / 16 < 2 ? (c + 15) / 16 : 2);
  hipLaunchKernelGGL(k_rescore_combine, dim3(gx, (unsigned)q), dim3(256), 0, s, sim, ld_s, q, meta, bound, ws->qn,
                     mem->dn, mem->ldk, cand, cand_count, c, mem->cls, ws->rs_score, ws->rs_terms, ws->rs_anchor);
  return hipGetLastError();
}

hipError_t launch_rescore_select(const farm_workspace* ws, int32_t q, int32_t c, int32_t k, const uint64_t* hi_key,
                                 const int32_t* hi_idx, const int32_t* cand_count, int64_t n, uint32_t* out_id,
                                 float* out_score, float* out_terms, uint32_t* out_anchor_id, int32_t* certified,
                                 hipStream_t s) {
  if (q <= 0) return hipSuccess;
  if (c > kSortMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rescore_select, dim3((unsigned)q), dim3(256), 0, s, ws->rs_score, ws->rs_idx, ws->rs_terms,
                     ws->rs_anchor, ws->mem->id, c, k, hi_key, hi_idx, cand_count, n, out_id, out_score, out_terms,
                     out_anchor_id, certified);
  return hipGetLastError();
}

hipError_t launch_semantic_exact(const farm_memory* mem, const farm_workspace* ws, int32_t q, int32_t R,
                                 hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const int64_t waves = (int64_t)R * kSemMax;
  hipLaunchKernelGGL(k_semantic_exact, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, ws->qn, mem->dn, mem->ldk, q,
                     R, ws->sem_idx, ws->sem_cnt, ws->sem_sim);
  return hipGetLastError();
}

namespace {
// Exact FP32 similarities max(0, q . d) of the relation rows of Between
// invocations (FARM_BETWEEN / FARM_AND), in place in the similarity matrix,
// with the rescoring kernels' dot product: Between's candidate sets and
// values are taken on exact similarities whatever the GEMM's dtype.  One wave
// per (row, anchor), four waves per block; blocks of other rows leave at once.
__global__ __launch_bounds__(256) void k_exact_rows(const float* __restrict__ qn, const float* __restrict__ dn,
                                                    int32_t ldk, float* __restrict__ sim, int64_t ld_s, int32_t q,
                                                    MetaView meta, int64_t n) {
  const int r = blockIdx.y;
  const int p = meta.rel_pred[r];
  if (p != FARM_BETWEEN && p != FARM_AND) return;
  const int lane = threadIdx.x & 63;
  const float* qrow = qn + (int64_t)(q + r) * ldk;
  for (int64_t a = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); a < n; a += (int64_t)gridDim.x * 4) {
    const float v = fmaxf(0.f, wave_dot(qrow, dn + a * ldk, ldk, lane));
    if (lane == 0) sim[(int64_t)(q + r) * ld_s + a] = v;
  }
}
}  // namespace

hipError_t launch_exact_rows(const farm_memory* mem, const float* qn, float* sim, int64_t ld_s, int32_t q,
                             MetaView meta, int32_t R, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const int64_t blocks = (mem->n + 3) / 4;
  hipLaunchKernelGGL(k_exact_rows, dim3((unsigned)(blocks < 1024 ? blocks : 1024), (unsigned)R), dim3(256), 0, s, qn,
                     mem->dn, mem->ldk, sim, ld_s, q, meta, mem->n);
  return hipGetLastError();
}

hipError_t launch_max_reduce(const float* v, int64_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, v, n, out);
  return hipGetLastError();
}

}  // namespace farm
