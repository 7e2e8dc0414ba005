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
// Rescoring one candidate o (one block per (candidate, query)):
//   s_sem:  FP32 dot of the normalised target and descriptor rows (block sum),
//           clamp, class factor;
//   t_r:    with a similarity bound |a~_j - a_j| <= delta_j, the best value is
//           at least L = max_j (a~_j - delta_j)+ * P(o, j); only anchors with
//           min(1, a~_j + delta_j) * P(o, j) >= L can reach it, so only those
//           get an FP32 dot product (one wave per anchor), in windows of 2,048
//           anchors so the survivor list never overflows LDS.  Without a bound
//           (FP32 similarities) the maximum is taken directly.
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
#include "sort_util.h"

namespace farm {
namespace {

constexpr int kRsThreads = 256;
constexpr int kWaves = kRsThreads / 64;
constexpr int kWin = 2048;

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// FP32 dot product of two zero-padded rows (ldk a multiple of 128) by one wave.
__device__ inline float wave_dot(const float* __restrict__ a, const float* __restrict__ b, int32_t ldk, int lane) {
  float acc = 0.f;
  for (int k = 2 * lane; k < ldk; k += 128) {
    float2 x = *reinterpret_cast<const float2*>(a + k);
    float2 y = *reinterpret_cast<const float2*>(b + k);
    acc = fmaf(x.x, y.x, acc);
    acc = fmaf(x.y, y.y, acc);
  }
  return wave_sum(acc);
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

template <int FAM>
__device__ void rescore_relation(const float* __restrict__ arow, const float* __restrict__ lrow,
                                 const float* __restrict__ qrow, const float* __restrict__ dn, int32_t ldk,
                                 int64_t n, int64_t o, float c, bool bounded, float qn, float qe,
                                 const float* __restrict__ o_err, const float* x, const float* y, const float* z,
                                 const float* hhi, const float* hlo, const uint32_t* __restrict__ ids, float* red_v,
                                 uint32_t* red_id, int32_t* surv, int* surv_n, const int32_t* __restrict__ lidx,
                                 const float* __restrict__ lval, int M, const int32_t* __restrict__ sidx, int sn,
                                 float cert, float& out_best, uint32_t& out_bid, bool& fell_back) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Tgt t = load_target(FAM, o, x, y, z, hhi, hlo);
  float best = value_floor<FAM>();
  uint32_t bid = FARM_NO_ID;
  fell_back = false;
  if (M > 0) {
    // value of subset entry e (list entries carry the cached predicate value)
    auto entry = [&](int e, float a, float la) -> float {
      if (e < M) return FAM == kFamNear ? la + lval[e] : a * lval[e];
      return pair_value<FAM>(t, anchor_record_pre(FAM, a, la, e < M ? lidx[e] : sidx[e - M], x, y, z, hhi, hlo), c);
    };
    const int tot = M + sn;
    if (!bounded) {
      for (int e = tid; e < tot; e += kRsThreads) {
        const int64_t j = e < M ? lidx[e] : sidx[e - M];
        if (j == o) continue;
        take_max(entry(e, arow[j], FAM == kFamNear ? lrow[j] : 0.f), j, ids, best, bid);
      }
    } else {
      float lo = value_floor<FAM>();
      for (int e = tid; e < tot; e += kRsThreads) {
        const int64_t j = e < M ? lidx[e] : sidx[e - M];
        if (j == o) continue;
        const float a = fmaxf(0.f, arow[j] - fmaf(qn, o_err[j], qe));
        lo = fmaxf(lo, entry(e, a, FAM == kFamNear ? near_log(a) : 0.f));
      }
      red_v[tid] = lo;
      if (tid == 0) *surv_n = 0;
      __syncthreads();
      for (int w = kRsThreads / 2; w > 0; w >>= 1) {
        if (tid < w) red_v[tid] = fmaxf(red_v[tid], red_v[tid + w]);
        __syncthreads();
      }
      const float L = red_v[0] - (fabsf(red_v[0]) * 1e-6f + 1e-30f);
      __syncthreads();
      for (int e = tid; e < tot; e += kRsThreads) {
        const int64_t j = e < M ? lidx[e] : sidx[e - M];
        if (j == o) continue;
        const float a = fminf(1.0f, arow[j] + fmaf(qn, o_err[j], qe));
        if (entry(e, a, FAM == kFamNear ? near_log(a) : 0.f) >= L) surv[atomicAdd(surv_n, 1)] = e;
      }
      __syncthreads();
      const int cnt = *surv_n;
      for (int s = wave; s < cnt; s += kWaves) {
        const int e = surv[s];
        const int64_t j = e < M ? lidx[e] : sidx[e - M];
        const float a = fmaxf(0.f, wave_dot(qrow, dn + j * ldk, ldk, lane));
        take_max(entry(e, a, FAM == kFamNear ? near_log(a) : 0.f), j, ids, best, bid);
      }
      __syncthreads();
    }
    red_v[tid] = best;
    red_id[tid] = bid;
    __syncthreads();
    for (int w = kRsThreads / 2; w > 0; w >>= 1) {
      if (tid < w && better(red_v[tid + w], red_id[tid + w], red_v[tid], red_id[tid])) {
        red_v[tid] = red_v[tid + w];
        red_id[tid] = red_id[tid + w];
      }
      __syncthreads();
    }
    const float sb = red_v[0];
    const uint32_t sid = red_id[0];
    __syncthreads();
    if (sb > cert) {
      out_best = sb;
      out_bid = sid;
      return;
    }
    fell_back = true;
    best = value_floor<FAM>();
    bid = FARM_NO_ID;
  }
  if (!bounded) {
    // FP32 similarities: the maximum directly, with the relational pass's arithmetic
    for (int64_t j = tid; j < n; j += kRsThreads) {
      if (j == o) continue;
      const float v =
          pair_value<FAM>(t, anchor_record_pre(FAM, arow[j], FAM == kFamNear ? lrow[j] : 0.f, j, x, y, z, hhi, hlo), c);
      take_max(v, j, ids, best, bid);
    }
  } else {
    // lower bound L of the best exact value, in the family's comparison domain
    float lo = value_floor<FAM>();
    for (int64_t j = tid; j < n; j += kRsThreads) {
      if (j == o) continue;
      const float a = fmaxf(0.f, arow[j] - fmaf(qn, o_err[j], qe));
      lo = fmaxf(lo, pair_value<FAM>(t, anchor_record(FAM, a, j, x, y, z, hhi, hlo), c));
    }
    red_v[tid] = lo;
    __syncthreads();
    for (int w = kRsThreads / 2; w > 0; w >>= 1) {
      if (tid < w) red_v[tid] = fmaxf(red_v[tid], red_v[tid + w]);
      __syncthreads();
    }
    const float L = red_v[0] - (fabsf(red_v[0]) * 1e-6f + 1e-30f);  // slack for rounding of the bounded values
    __syncthreads();
    for (int64_t w0 = 0; w0 < n; w0 += kWin) {
      if (tid == 0) *surv_n = 0;
      __syncthreads();
      const int64_t w1 = w0 + kWin < n ? w0 + kWin : n;
      for (int64_t j = w0 + tid; j < w1; j += kRsThreads) {
        if (j == o) continue;
        const float a = fminf(1.0f, arow[j] + fmaf(qn, o_err[j], qe));
        if (pair_value<FAM>(t, anchor_record(FAM, a, j, x, y, z, hhi, hlo), c) >= L)
          surv[atomicAdd(surv_n, 1)] = (int32_t)j;
      }
      __syncthreads();
      const int cnt = *surv_n;
      for (int s = wave; s < cnt; s += kWaves) {
        const int64_t j = surv[s];
        const float a = fmaxf(0.f, wave_dot(qrow, dn + j * ldk, ldk, lane));
        const float v = pair_value<FAM>(t, anchor_record(FAM, a, j, x, y, z, hhi, hlo), c);
        take_max(v, j, ids, best, bid);
      }
      __syncthreads();
    }
  }
  red_v[tid] = best;
  red_id[tid] = bid;
  __syncthreads();
  for (int w = kRsThreads / 2; w > 0; w >>= 1) {
    if (tid < w && better(red_v[tid + w], red_id[tid + w], red_v[tid], red_id[tid])) {
      red_v[tid] = red_v[tid + w];
      red_id[tid] = red_id[tid + w];
    }
    __syncthreads();
  }
  out_best = red_v[0];
  out_bid = red_id[0];
  __syncthreads();
}

__global__ __launch_bounds__(kRsThreads) void k_rescore(
    const float* __restrict__ sim, const float* __restrict__ lsim, int64_t ld_s, int32_t q, MetaView meta,
    SimBound bound, const float* __restrict__ qn, const float* __restrict__ dn, int32_t ldk,
    const int32_t* __restrict__ cand,
    const int32_t* __restrict__ cand_count, int32_t C, const float* __restrict__ x, const float* __restrict__ y,
    const float* __restrict__ z, const float* __restrict__ hhi, const float* __restrict__ hlo,
    const uint32_t* __restrict__ ids, const int32_t* __restrict__ cls, int64_t n, float* __restrict__ rs_score,
    float* __restrict__ rs_terms, uint32_t* __restrict__ rs_anchor, PropView pv) {
  __shared__ float red_v[kRsThreads];
  __shared__ uint32_t red_id[kRsThreads];
  __shared__ int32_t surv[kWin];
  __shared__ int surv_n;
  const int32_t qq = blockIdx.y;
  const int tid = threadIdx.x;
  const int r0 = meta.rel_off[qq], r1 = meta.rel_off[qq + 1], R = r1 - r0;
  const int32_t cnt = cand_count ? cand_count[qq] : C;
  const bool bounded = bound.q_nrm != nullptr;
  const float* qt = qn + (int64_t)qq * ldk;
  const int tc = meta.tcls[qq];
  for (int32_t cc = blockIdx.x; cc < cnt; cc += gridDim.x) {
    const int64_t slot = (int64_t)qq * C + cc;
    const int64_t o = cand[slot];
    if (o < 0) {
      if (tid == 0) rs_score[slot] = -INFINITY;
      if (tid < kMaxRel) {
        rs_terms[slot * kMaxRel + tid] = 0.f;
        rs_anchor[slot * kMaxRel + tid] = FARM_NO_ID;
      }
      continue;
    }
    // target similarity: the FP32 GEMM's value, or an FP32 dot product when the
    // similarity matrix is reduced-precision
    float sem;
    if (!bounded) {
      sem = sim[(int64_t)qq * ld_s + o];
    } else {
      const float* dr = dn + o * ldk;
      float part = 0.f;
      for (int k = tid; k < ldk; k += kRsThreads) part = fmaf(qt[k], dr[k], part);
      red_v[tid] = part;
      __syncthreads();
      for (int w = kRsThreads / 2; w > 0; w >>= 1) {
        if (tid < w) red_v[tid] += red_v[tid + w];
        __syncthreads();
      }
      const float dot = red_v[0];
      __syncthreads();
      const float kappa = (tc >= 0 && cls && cls[o] >= 0 && cls[o] != tc) ? kClassFactor : 1.0f;
      sem = kappa * fmaxf(0.f, dot);
    }
    float lsum = 0.f;
    for (int e = 0; e < R; ++e) {
      const int r = r0 + e;
      const int p = meta.rel_pred[r];
      const float c = sigmoid_scale(p);
      const float* arow = sim + (int64_t)(q + r) * ld_s;
      const float* lrow = lsim + (int64_t)r * ld_s;
      const float* qrow = qn + (int64_t)(q + r) * ldk;
      const float qnr = bounded ? bound.q_nrm[q + r] : 0.f;
      const float qer = bounded ? bound.q_err[q + r] + bound.acc : 0.f;
      float best;
      uint32_t bid;
      float term;
      bool fell_back;
      // proposal subset of this (relation, candidate) and the bound on every anchor outside it
      const int32_t* lidx = nullptr;
      const float* lval = nullptr;
      const int32_t* sidx = nullptr;
      int sn = 0;
      float cert = INFINITY;
      if (pv.m > 0) {
        const int64_t lo_ = ((int64_t)p * n + o) * pv.m;
        lidx = pv.idx + lo_;
        lval = pv.val + lo_;
        sidx = pv.sem_idx + (int64_t)r * kSemMax;
        sn = pv.sem_cnt[r];
        const float pout = pv.out[(int64_t)p * n + o];
        const bool near = family_of(p) == kFamNear;
        if (!bounded) {
          cert = near ? pv.sem_ltau[r] + pout : pv.sem_tau[r] * pout;
        } else {
          const float a_hi = pv.sem_tau[r] + fmaf(qnr, *bound.o_err_max, qer);
          if (near) {
            const float b = near_log(a_hi) + pout;
            cert = b + fabsf(b) * 1e-6f;  // covers the rounding of the logarithm
          } else {
            cert = a_hi * pout;
          }
        }
      }
      switch (family_of(p)) {
        case kFamNear:
          rescore_relation<kFamNear>(arow, lrow, qrow, dn, ldk, n, o, c, bounded, qnr, qer, bound.o_err, x, y, z, hhi,
                                     hlo, ids, red_v, red_id, surv, &surv_n, lidx, lval, pv.m, sidx, sn, cert, best, bid,
                                     fell_back);
          term = term_of<kFamNear>(best);
          lsum += best;
          break;
        case kFamVert:
          rescore_relation<kFamVert>(arow, lrow, qrow, dn, ldk, n, o, c, bounded, qnr, qer, bound.o_err, x, y, z, hhi,
                                     hlo, ids, red_v, red_id, surv, &surv_n, lidx, lval, pv.m, sidx, sn, cert, best, bid,
                                     fell_back);
          term = term_of<kFamVert>(best);
          lsum += logf(term);
          break;
        default:
          rescore_relation<kFamLat>(arow, lrow, qrow, dn, ldk, n, o, c, bounded, qnr, qer, bound.o_err, x, y, z, hhi,
                                    hlo, ids, red_v, red_id, surv, &surv_n, lidx, lval, pv.m, sidx, sn, cert, best, bid,
                                     fell_back);
          term = term_of<kFamLat>(best);
          lsum += logf(term);
          break;
      }
      if (tid == 0) {
        rs_terms[slot * kMaxRel + e] = term;
        rs_anchor[slot * kMaxRel + e] = bid;
        if (pv.stats) {
          atomicAdd(&pv.stats[0], 1ull);
          if (fell_back) atomicAdd(&pv.stats[1], 1ull);
        }
      }
    }
    if (tid == 0) {
      const float g = R > 0 ? expf(lsum / (float)R) : 1.0f;
      rs_score[slot] = sem * ((1.0f - kW) + kW * g);
    }
    if (tid >= R && tid < kMaxRel) {
      rs_terms[slot * kMaxRel + tid] = 0.f;
      rs_anchor[slot * kMaxRel + tid] = FARM_NO_ID;
    }
    __syncthreads();
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

hipError_t launch_rescore(const farm_memory* mem, const farm_workspace* ws, const float* sim, const float* lsim,
                          int64_t ld_s, int32_t q, MetaView meta, const SimBound& bound, const int32_t* cand,
                          const int32_t* cand_count, int32_t c, const PropView& prop, hipStream_t s) {
  if (q <= 0 || c <= 0) return hipSuccess;
  // with a device-side count the candidate slots are swept by a fixed number of blocks per query
  const unsigned gx = cand_count ? (unsigned)(c < 64 ? c : 64) : (unsigned)c;
  hipLaunchKernelGGL(k_rescore, dim3(gx, (unsigned)q), dim3(kRsThreads), 0, s, sim, lsim, ld_s, q, meta, bound, ws->qn,
                     mem->dn, mem->ldk, cand, cand_count, c, mem->x, mem->y, mem->z, mem->hr_hi, mem->hr_lo, mem->id,
                     mem->cls, mem->n, ws->rs_score, ws->rs_terms, ws->rs_anchor, prop);
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

hipError_t launch_max_reduce(const float* v, int64_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, v, n, out);
  return hipGetLastError();
}

}  // namespace farm
