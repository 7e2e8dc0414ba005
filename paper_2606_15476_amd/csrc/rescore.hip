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

template <int FAM>
__device__ void rescore_relation(const float* __restrict__ arow, const float* __restrict__ qrow,
                                 const float* __restrict__ dn, int32_t ldk, int64_t n, int64_t o, float c,
                                 bool bounded, float qn, float qe, const float* __restrict__ o_err,
                                 const float* x, const float* y, const float* z, const float* hhi, const float* hlo,
                                 const uint32_t* __restrict__ ids, float* red_v, uint32_t* red_id, int32_t* surv,
                                 int* surv_n, float& out_best, uint32_t& out_bid) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const Tgt t = load_target(FAM, o, x, y, z, hhi, hlo);
  float best = value_floor<FAM>();
  uint32_t bid = FARM_NO_ID;
  if (!bounded) {
    for (int64_t j = tid; j < n; j += kRsThreads) {
      if (j == o) continue;
      float v = pair_value<FAM>(t, anchor_record(FAM, arow[j], j, x, y, z, hhi, hlo), c);
      if (better(v, ids[j], best, bid) && v != -INFINITY) { best = v; bid = ids[j]; }
    }
  } else {
    // lower bound of the best exact value
    float lo = value_floor<FAM>();
    for (int64_t j = tid; j < n; j += kRsThreads) {
      if (j == o) continue;
      float a = fmaxf(0.f, arow[j] - fmaf(qn, o_err[j], qe));
      lo = fmaxf(lo, pair_value<FAM>(t, anchor_record(FAM, a, j, x, y, z, hhi, hlo), c));
    }
    red_v[tid] = lo;
    __syncthreads();
    for (int w = kRsThreads / 2; w > 0; w >>= 1) {
      if (tid < w) red_v[tid] = fmaxf(red_v[tid], red_v[tid + w]);
      __syncthreads();
    }
    const float L = red_v[0];
    const float Ls = L - (fabsf(L) * 1e-6f + 1e-30f);  // slack for rounding of the bounded values
    __syncthreads();
    for (int64_t w0 = 0; w0 < n; w0 += kWin) {
      if (tid == 0) *surv_n = 0;
      __syncthreads();
      const int64_t w1 = w0 + kWin < n ? w0 + kWin : n;
      for (int64_t j = w0 + tid; j < w1; j += kRsThreads) {
        if (j == o) continue;
        float a = fminf(1.0f, arow[j] + fmaf(qn, o_err[j], qe));
        float v = pair_value<FAM>(t, anchor_record(FAM, a, j, x, y, z, hhi, hlo), c);
        if (v >= Ls) surv[atomicAdd(surv_n, 1)] = (int32_t)j;
      }
      __syncthreads();
      const int cnt = *surv_n;
      for (int s = wave; s < cnt; s += kWaves) {
        const int64_t j = surv[s];
        float a = fmaxf(0.f, wave_dot(qrow, dn + j * ldk, ldk, lane));
        float v = pair_value<FAM>(t, anchor_record(FAM, a, j, x, y, z, hhi, hlo), c);
        if (better(v, ids[j], best, bid) && v != -INFINITY) { best = v; bid = ids[j]; }
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
    const float* __restrict__ sim, int64_t ld_s, int32_t q, MetaView meta, SimBound bound,
    const float* __restrict__ qn, const float* __restrict__ dn, int32_t ldk, const int32_t* __restrict__ cand,
    const int32_t* __restrict__ cand_count, int32_t C, const float* __restrict__ x, const float* __restrict__ y,
    const float* __restrict__ z, const float* __restrict__ hhi, const float* __restrict__ hlo,
    const uint32_t* __restrict__ ids, const int32_t* __restrict__ cls, int64_t n, float* __restrict__ rs_score,
    float* __restrict__ rs_terms, uint32_t* __restrict__ rs_anchor) {
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
      const float* qrow = qn + (int64_t)(q + r) * ldk;
      const float qnr = bounded ? bound.q_nrm[q + r] : 0.f;
      const float qer = bounded ? bound.q_err[q + r] + bound.acc : 0.f;
      float best;
      uint32_t bid;
      float term;
      switch (family_of(p)) {
        case kFamNear:
          rescore_relation<kFamNear>(arow, qrow, dn, ldk, n, o, c, bounded, qnr, qer, bound.o_err, x, y, z, hhi,
                                     hlo, ids, red_v, red_id, surv, &surv_n, best, bid);
          term = term_of<kFamNear>(best);
          lsum += best;
          break;
        case kFamVert:
          rescore_relation<kFamVert>(arow, qrow, dn, ldk, n, o, c, bounded, qnr, qer, bound.o_err, x, y, z, hhi,
                                     hlo, ids, red_v, red_id, surv, &surv_n, best, bid);
          term = term_of<kFamVert>(best);
          lsum += logf(term);
          break;
        default:
          rescore_relation<kFamLat>(arow, qrow, dn, ldk, n, o, c, bounded, qnr, qer, bound.o_err, x, y, z, hhi,
                                    hlo, ids, red_v, red_id, surv, &surv_n, best, bid);
          term = term_of<kFamLat>(best);
          lsum += logf(term);
          break;
      }
      if (tid == 0) {
        rs_terms[slot * kMaxRel + e] = term;
        rs_anchor[slot * kMaxRel + e] = bid;
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
                                                        const int32_t* __restrict__ hi_idx, int64_t n,
                                                        uint32_t* __restrict__ out_id, float* __restrict__ out_score,
                                                        float* __restrict__ out_terms,
                                                        uint32_t* __restrict__ out_anchor,
                                                        int32_t* __restrict__ certified) {
  __shared__ uint64_t keys[kSortMax];
  __shared__ int32_t slot[kSortMax];
  __shared__ int32_t first_out;
  const int32_t qq = blockIdx.x;
  const int P = pow2_at_least(C);
  for (int e = threadIdx.x; e < P; e += blockDim.x) {
    int32_t o = e < C ? rs_idx[(int64_t)qq * C + e] : -1;
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

hipError_t launch_rescore(const farm_memory* mem, const farm_workspace* ws, const float* sim, int64_t ld_s, int32_t q,
                          MetaView meta, const SimBound& bound, const int32_t* cand, const int32_t* cand_count,
                          int32_t c, hipStream_t s) {
  if (q <= 0 || c <= 0) return hipSuccess;
  // with a device-side count the candidate slots are swept by a fixed number of blocks per query
  const unsigned gx = cand_count ? (unsigned)(c < 64 ? c : 64) : (unsigned)c;
  hipLaunchKernelGGL(k_rescore, dim3(gx, (unsigned)q), dim3(kRsThreads), 0, s, sim, ld_s, q, meta, bound, ws->qn,
                     mem->dn, mem->ldk, cand, cand_count, c, mem->x, mem->y, mem->z, mem->hr_hi, mem->hr_lo, mem->id,
                     mem->cls, mem->n, ws->rs_score, ws->rs_terms, ws->rs_anchor);
  return hipGetLastError();
}

hipError_t launch_rescore_select(const farm_workspace* ws, int32_t q, int32_t c, int32_t k, const uint64_t* hi_key,
                                 const int32_t* hi_idx, int64_t n, uint32_t* out_id, float* out_score,
                                 float* out_terms, uint32_t* out_anchor_id, int32_t* certified, hipStream_t s) {
  if (q <= 0) return hipSuccess;
  if (c > kSortMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rescore_select, dim3((unsigned)q), dim3(256), 0, s, ws->rs_score, ws->rs_idx, ws->rs_terms,
                     ws->rs_anchor, ws->mem->id, c, k, hi_key, hi_idx, n, out_id, out_score, out_terms, out_anchor_id,
                     certified);
  return hipGetLastError();
}

hipError_t launch_max_reduce(const float* v, int64_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, v, n, out);
  return hipGetLastError();
}

}  // namespace farm
