// pair_math.h -- per-(target, anchor) arithmetic shared by the relational
// pass, the ScoredCandidate breakdown and FP32 rescoring, so that all of them
// produce identical values for identical inputs.
//
// Forms (algebraically equal to the definitions of the soft predicates):
//   Near/NextTo: log(a_j) + c |c_i - c_j|^2 with c = -1/(2 sigma^2) (-2 for
//                Near, -1/2 for NextTo) is compared in the log domain (no
//                transcendental per pair); t = exp(max).
//   On:          the same form: the gate's and the band's exponents add up to
//                c (dx^2 + dy^2 + (4 g)^2) with c = -1/(2 * 0.5^2) = -2 and g
//                the gap between the target's bottom and the anchor's top,
//                since the band's width 0.125 m is a quarter of the gate's; the
//                vertical coordinate is 4 * bottom for the target and 4 * top
//                for the anchor instead of the center.
// Every Near-family coefficient is a power of two, so c * d2 is exact and a
// cached c * d2 plus log(a) rounds as fmaf(c, d2, log a) does.
//   Above/Below: P = 1 / (1 + 2^(dz * c)), c = -+(1/tau) log2(e), dz = z_i - z_j.
//   Left/Right:  the same sigmoid of the lateral offset dh = h_i - h_j, with h
//                kept as an unevaluated float pair hi + lo; InFrontOf/Behind
//                the same with the offset along the viewing direction (the
//                "lateral" coordinate pair of those predicates is the depth).
// Offsets are differences of coordinates before any scaling, so argument
// errors are relative to the offset, not to the distance from the origin.
#pragma once

#include <math.h>

#include "farm_internal.h"

namespace farm {

enum Family { kFamNear = 0, kFamVert = 1, kFamLat = 2 };

// (1/tau) * log2(e) with tau = 0.1 m
constexpr float kInvTauLog2e = 14.426950408889634f;

__device__ inline int family_of(int p) {
  return (p == FARM_NEAR || p == FARM_NEXT_TO || p == FARM_ON) ? kFamNear
         : (p == FARM_ABOVE || p == FARM_BELOW)                ? kFamVert
                                                               : kFamLat;
}

// Predicates of the Left/Right family measured along the viewing direction
// (their coordinate pair is the depth, not the lateral offset).
__device__ inline bool is_depth(int p) { return p == FARM_IN_FRONT_OF || p == FARM_BEHIND; }

// Per-predicate constant of pair_value: for the sigmoid families the exponent
// scale c with P = 1 / (1 + 2^(offset * c)); for Near/NextTo the log-domain
// coefficient -1/(2 sigma^2) of the squared distance.
__device__ inline float sigmoid_scale(int p) {
  if (p == FARM_NEAR) return -2.0f;     // sigma 0.5 m
  if (p == FARM_NEXT_TO) return -0.5f;  // sigma 1.0 m
  if (p == FARM_ON) return -2.0f;       // gate sigma 0.5 m (band 0.125 m through the scaled coordinate)
  return (p == FARM_ABOVE || p == FARM_RIGHT_OF || p == FARM_BEHIND) ? -kInvTauLog2e : kInvTauLog2e;
}

__device__ inline float rcp_approx(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ inline float exp2_approx(float v) { return __builtin_amdgcn_exp2f(v); }

// The vertical coordinates of the Near family for predicate p: the target's
// and the anchor's.  On compares the target's bottom face with the anchor's
// top face (vz: [2][n], both scaled by 4); the others the box centers.
struct ZPair {
  const float* tgt;
  const float* anc;
};
__device__ inline ZPair z_for(int p, const float* z, const float* vz, int64_t n) {
  return p == FARM_ON ? ZPair{vz, vz + n} : ZPair{z, z};
}

// Per-target coordinates, family-specific.
struct Tgt {
  float u0, u1, u2;
};

__device__ inline Tgt load_target(int fam, int64_t i, const float* x, const float* y, const float* z,
                                  const float* hhi, const float* hlo) {
  Tgt t{0.f, 0.f, 0.f};
  if (fam == kFamNear) {
    t.u0 = x[i]; t.u1 = y[i]; t.u2 = z[i];
  } else if (fam == kFamVert) {
    t.u0 = z[i];
  } else {
    t.u0 = hhi[i]; t.u1 = hlo[i];
  }
  return t;
}

// Log of a similarity as the Near family stores it (a = 0 maps to a large
// finite negative number so such anchors still order by distance).
__device__ inline float near_log(float a) { return a > 0.f ? logf(a) : -1.0e30f; }

// Anchor record: (value, coordinates).  Near stores log(a_j).
__device__ inline float4 anchor_record(int fam, float a, int64_t j, const float* x, const float* y, const float* z,
                                       const float* hhi, const float* hlo) {
  // a = 0 maps to a large finite negative log so that such anchors still order by
  // distance (any of them is a valid binding of a zero term).
  if (fam == kFamNear) return make_float4(near_log(a), x[j], y[j], z[j]);
  if (fam == kFamVert) return make_float4(a, z[j], 0.f, 0.f);
  return make_float4(a, hhi[j], hlo[j], 0.f);
}

// Anchor record from a precomputed log similarity (Near) or similarity.
__device__ inline float4 anchor_record_pre(int fam, float a, float la, int64_t j, const float* x, const float* y,
                                           const float* z, const float* hhi, const float* hlo) {
  if (fam == kFamNear) return make_float4(la, x[j], y[j], z[j]);
  if (fam == kFamVert) return make_float4(a, z[j], 0.f, 0.f);
  return make_float4(a, hhi[j], hlo[j], 0.f);
}

// Value of one (target, anchor) pair in the family's comparison domain:
// log domain for Near, linear for the sigmoid families.
template <int FAM>
__device__ inline float pair_value(const Tgt& t, const float4& rec, float c) {
  if (FAM == kFamNear) {
    float dx = t.u0 - rec.y, dy = t.u1 - rec.z, dz = t.u2 - rec.w;
    float d2 = dx * dx;
    d2 = fmaf(dy, dy, d2);
    d2 = fmaf(dz, dz, d2);
    return fmaf(c, d2, rec.x);
  } else if (FAM == kFamVert) {
    float e = exp2_approx((t.u0 - rec.y) * c);
    return rec.x * rcp_approx(1.0f + e);
  } else {
    float dh = (t.u0 - rec.y) + (t.u1 - rec.z);
    float e = exp2_approx(dh * c);
    return rec.x * rcp_approx(1.0f + e);
  }
}

// Initial "best" in the comparison domain (below any attainable value).
template <int FAM>
__device__ inline float value_floor() {
  return FAM == kFamNear ? -INFINITY : -1.0f;
}

// Linear relation term from the family-domain maximum.
template <int FAM>
__device__ inline float term_of(float best) {
  if (FAM == kFamNear) return expf(best);
  return best > 0.f ? best : 0.f;
}


}  // namespace farm
