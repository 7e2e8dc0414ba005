// proposal.hip -- learned anchor proposals: table build and semantic sets.
//
// The star decomposition costs O(|Phi| K_t K_a) with K_a the anchor candidates
// per relation (Appendix "Robust Relational Retrieval Formulation", query-time
// complexity).  Here the exact pass over all anchors is replaced, for each
// candidate target o and relation r, by the union of
//   * a learned list L(o, p) of M anchors per (target, predicate), ranked by
//     the proposal network's logit for p (query-independent, built once per
//     scene, with the predicate value P(o, a) cached), and
//   * the relation's semantic set S_r: the (at most 64) anchors with the
//     largest similarity to the relation's anchor description, found per query.
// Every anchor outside both has sim <= tau_r (the largest similarity outside
// S_r) and P <= Pout(o, p) (the largest predicate value outside L(o, p),
// computed exactly at build time), so its value is at most tau_r * Pout(o, p);
// the rescoring kernel keeps the subset maximum when it is strictly larger and
// scans all anchors otherwise.
//
// Table build (per chunk of targets, all anchors): the first layer is
// factorised, W1 x = W1o u_o + W1a u_a + W1g g, with U = D W1o^T and V = D W1a^T
// computed once per scene by MFMA GEMMs; per pair h1 = GELU(U_o + V_a + b1 +
// W1g g(o, a)), h2 = GELU(W2 h1 + b2) (MFMA GEMM with the GELU epilogue),
// logits from h2; a TopK per (predicate, target) row keeps the M largest.
#include <math.h>

#include <new>
#include <vector>

#include "farm_internal.h"
#include "pair_math.h"
#include "sort_util.h"

namespace farm {
namespace {

constexpr int kNPred = FARM_NUM_PROP_PRED;  // one list per predicate
constexpr float kGeoScale = 0.25f;

__device__ inline uint16_t bf16r(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float from_bf16r(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ inline float gelu_f(float v) { return 0.5f * v * (1.0f + erff(v * 0.70710678118654752f)); }

__device__ inline float geo_f(int f, int64_t o, int64_t a, const float* x, const float* y, const float* z,
                              const float* ext, int64_t n, float rx, float ry) {
  const float dx = x[o] - x[a], dy = y[o] - y[a], dz = z[o] - z[a];
  float v;
  switch (f) {
    case 0: v = dx; break;
    case 1: v = dy; break;
    case 2: v = dz; break;
    case 3: case 4: case 5: v = ext[(f - 3) * n + o]; break;
    case 6: case 7: case 8: v = ext[(f - 6) * n + a]; break;
    case 9: v = sqrtf(dx * dx + dy * dy + dz * dz); break;
    case 10: v = dx * rx + dy * ry; break;
    default: v = (z[o] - 0.5f * ext[2 * n + o]) - (z[a] + 0.5f * ext[2 * n + a]); break;
  }
  return v * kGeoScale;
}

__global__ void k_rows_to_bf16(const float* __restrict__ src, int64_t count, uint16_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = bf16r(src[i]);
}

// h1 of pair (t, a) for targets o_t = t0 + t: one block per pair, one thread per hidden unit
__global__ void k_hidden1(const float* __restrict__ U, const float* __restrict__ V, const float* __restrict__ b1,
                          const uint16_t* __restrict__ W1b, int32_t ldx, int32_t geo0, int64_t t0, int64_t n,
                          const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
                          const float* __restrict__ ext, float rx, float ry, uint16_t* __restrict__ A1) {
  __shared__ float g[12];
  const int64_t p = blockIdx.x;  // pair row = t * n + a
  const int64_t t = p / n, a = p % n, o = t0 + t;
  if (threadIdx.x < 12) g[threadIdx.x] = from_bf16r(bf16r(geo_f(threadIdx.x, o, a, x, y, z, ext, n, rx, ry)));
  __syncthreads();
  const int k = threadIdx.x;
  float acc = U[o * FARM_MLP_HIDDEN + k] + V[a * FARM_MLP_HIDDEN + k] + b1[k];
  const uint16_t* w = W1b + (int64_t)k * ldx + geo0;
#pragma unroll
  for (int f = 0; f < 12; ++f) acc = fmaf(from_bf16r(w[f]), g[f], acc);
  A1[p * FARM_MLP_HIDDEN + k] = bf16r(gelu_f(acc));
}

// logits in predicate-major rows: L[p][t][a] (self pairs excluded with -inf)
__global__ void k_head_rows(const uint16_t* __restrict__ A2, const float* __restrict__ W3r, const float* __restrict__ b3,
                            int64_t t0, int64_t tc, int64_t n, float* __restrict__ L) {
  const int64_t pr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pr >= tc * n) return;
  const int64_t t = pr / n, a = pr % n;
  float acc[kNPred];
#pragma unroll
  for (int c = 0; c < kNPred; ++c) acc[c] = b3[c];
  const uint16_t* row = A2 + pr * FARM_MLP_HIDDEN;
  for (int k = 0; k < FARM_MLP_HIDDEN; ++k) {
    const float v = from_bf16r(row[k]);
#pragma unroll
    for (int c = 0; c < kNPred; ++c) acc[c] = fmaf(v, W3r[c * FARM_MLP_HIDDEN + k], acc[c]);
  }
  const bool self = (t0 + t) == a;
#pragma unroll
  for (int c = 0; c < kNPred; ++c) L[((int64_t)c * tc + t) * n + a] = self ? -INFINITY : acc[c];
}

// Predicate value of (o, a) for predicate p in the family's comparison domain
// (Near/NextTo/On: log P; others: P), computed with the shared per-pair
// arithmetic (hhi/hlo: the coordinate pair of p's family, lateral or depth;
// zp: the target's and the anchor's vertical coordinates).
__device__ inline float pred_value(int p, int64_t o, int64_t a, const float* x, const float* y, ZPair zp,
                                   const float* hhi, const float* hlo) {
  const int fam = family_of(p);
  const float c = sigmoid_scale(p);
  const Tgt t = load_target(fam, o, x, y, zp.tgt, hhi, hlo);
  const float4 r = anchor_record_pre(fam, 1.0f, 0.0f, a, x, y, zp.anc, hhi, hlo);
  if (fam == kFamNear) return pair_value<kFamNear>(t, r, c);
  if (fam == kFamVert) return pair_value<kFamVert>(t, r, c);
  return pair_value<kFamLat>(t, r, c);
}

// Non-learned ranking: L[p][t][a] = P_p(o_t, a) in the family's comparison
// domain (self pairs -inf), so that a list holds the M anchors of largest
// predicate value and Pout is the (M+1)-th largest.
__global__ void k_value_rows(int64_t t0, int64_t tc, int64_t n, const float* __restrict__ x,
                             const float* __restrict__ y, const float* __restrict__ z, const float* __restrict__ vz,
                             const float* __restrict__ hhi, const float* __restrict__ hlo, float* __restrict__ L) {
  const int p = blockIdx.y;
  const int64_t pr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pr >= tc * n) return;
  const int64_t t = pr / n, a = pr % n, o = t0 + t;
  const int64_t sh = is_depth(p) ? n : 0;
  const ZPair zp = z_for(p, z, vz, n);
  L[((int64_t)p * tc + t) * n + a] = a == o ? -INFINITY : pred_value(p, o, a, x, y, zp, hhi + sh, hlo + sh);
}

// One block per (target t of the chunk, predicate): write the list (entries
// that selection could not fill repeat a real anchor) and Pout.
__global__ __launch_bounds__(256) void k_prop_finalize(const int32_t* __restrict__ top_idx, int32_t M, int64_t t0,
                                                       int64_t tc, int64_t n, const float* __restrict__ x,
                                                       const float* __restrict__ y, const float* __restrict__ z,
                                                       const float* __restrict__ vz,
                                                       const float* __restrict__ hhi, const float* __restrict__ hlo,
                                                       int32_t* __restrict__ prop_idx, float* __restrict__ prop_val,
                                                       float* __restrict__ prop_out) {
  extern __shared__ uint32_t bits[];  // n bits: anchors on the list
  __shared__ float red[256];
  const int p = blockIdx.y;
  const int64_t t = blockIdx.x, o = t0 + t;
  const int64_t words = (n + 31) / 32;
  // InFrontOf/Behind use the depth pair stored after the lateral one
  hhi += is_depth(p) ? n : 0;
  hlo += is_depth(p) ? n : 0;
  const ZPair zp = z_for(p, z, vz, n);  // On: the target's bottom and the anchors' top faces
  for (int64_t w = threadIdx.x; w < words; w += blockDim.x) bits[w] = 0;
  __syncthreads();
  const int32_t* row = top_idx + ((int64_t)p * tc + t) * M;
  const int64_t base = ((int64_t)p * n + o) * M;
  for (int m = threadIdx.x; m < M; m += blockDim.x) {
    int32_t a = row[m];
    if (a < 0 || a >= n || a == o) a = o == 0 ? 1 : 0;
    atomicOr(&bits[a >> 5], 1u << (a & 31));
    prop_idx[base + m] = a;
    prop_val[base + m] = pred_value(p, o, a, x, y, zp, hhi, hlo);
  }
  __syncthreads();
  float best = -INFINITY;
  for (int64_t a = threadIdx.x; a < n; a += blockDim.x) {
    if (a == o || (bits[a >> 5] >> (a & 31)) & 1u) continue;
    best = fmaxf(best, pred_value(p, o, a, x, y, zp, hhi, hlo));
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) prop_out[(int64_t)p * n + o] = red[0];
}

// ---------------------------------------------------------------- query time
// Semantic set of one relation row, one wave per row: tau = gamma * max_a sim
// with gamma in 1/2, 3/4, 7/8, ... until at most kSemMax anchors exceed tau;
// the set is their ordered compaction (ballots; truncated to kSemMax if ties
// at the maximum leave more).  Then the largest similarity of the anchors
// outside the set, which bounds every anchor the set leaves out.
constexpr int kSemWaves = 4;

__device__ inline float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}

__global__ __launch_bounds__(64 * kSemWaves) void k_semantic_sets(const float* __restrict__ sim, int64_t ld_s,
                                                                  int32_t q, int32_t R, int64_t n,
                                                                  int32_t* __restrict__ sem_idx,
                                                                  int32_t* __restrict__ sem_cnt,
                                                                  float* __restrict__ sem_tau) {
  const int lane = threadIdx.x & 63;
  const int32_t r = blockIdx.x * kSemWaves + (threadIdx.x >> 6);
  if (r >= R) return;  // the whole wave leaves; no block barrier follows
  const float* row = sim + (int64_t)(q + r) * ld_s;
  float mx = 0.f;
  for (int64_t j = lane; j < n; j += 64) mx = fmaxf(mx, row[j]);
  const float amax = wave_max(mx);
  const uint64_t below = (1ull << lane) - 1ull;
  // one pass: ordered compaction of the anchors above tau (first kSemMax kept),
  // their count, and the largest similarity of the anchors left out
  float out = 0.f;
  auto compact = [&](float tau) {
    int32_t pos = 0;
    out = 0.f;
    for (int64_t base = 0; base < n; base += 64) {
      const int64_t j = base + lane;
      const bool valid = j < n;
      const float v = valid ? row[j] : 0.f;
      const bool above = valid && v > tau;
      const uint64_t mask = __ballot(above);
      const int32_t my = pos + __popcll(mask & below);
      if (above && my < kSemMax) {
        sem_idx[(int64_t)r * kSemMax + my] = (int32_t)j;
      } else if (valid) {
        out = fmaxf(out, v);
      }
      pos += __popcll(mask);
    }
    return pos;
  };
  auto count_above = [&](float tau) {
    int32_t c = 0;
    for (int64_t base = 0; base < n; base += 64) {
      const int64_t j = base + lane;
      c += __popcll(__ballot(j < n && row[j] > tau));
    }
    return c;
  };
  float tau = 0.5f * amax, gap = 0.5f * amax;
  int32_t total = compact(tau);  // usually final: few anchors reach half the best similarity
  if (total > kSemMax) {
    for (int it = 0; it < 30 && total > kSemMax; ++it) {
      gap *= 0.5f;
      tau = amax - gap;
      total = count_above(tau);
    }
    total = compact(tau);
  }
  out = wave_max(out);
  if (lane == 0) {
    sem_cnt[r] = total < kSemMax ? total : kSemMax;
    sem_tau[r] = out;
  }
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_semantic_sets(const float* sim, int64_t ld_s, int32_t q, int32_t R, int64_t n, int32_t* sem_idx,
                                int32_t* sem_cnt, float* sem_tau, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_semantic_sets, dim3((unsigned)((R + kSemWaves - 1) / kSemWaves)), dim3(64 * kSemWaves), 0, s,
                     sim, ld_s, q, R, n, sem_idx, sem_cnt, sem_tau);
  return hipGetLastError();
}

// The table build's forward pass, shared by farm_build_proposals and
// farm_mlp_table_logits.  First-layer factors U = D W1o^T, V = D W1a^T
// ([n][H] FP32) from the BF16 descriptors dnb.
static hipError_t table_factors(const farm_memory* mem, const farm_mlp* mlp, const uint16_t* dnb, float* U, float* V,
                                hipStream_t s) {
  const int64_t H = FARM_MLP_HIDDEN;
  hipError_t e = launch_gemm_nt_bf16(dnb, mem->ldk, mlp->W1b, mlp->ldx, mem->n, H, mlp->dp, U, H, nullptr, false, s);
  if (e == hipSuccess)
    e = launch_gemm_nt_bf16(dnb, mem->ldk, mlp->W1b + mlp->dp, mlp->ldx, mem->n, H, mlp->dp, V, H, nullptr, false, s);
  return e;
}

// Logits L[p][t][a] of targets t0 .. t0 + tc - 1 against every anchor a (self
// pairs -inf); A1, A2: [tc * n][H] BF16 activation buffers.
static hipError_t table_logits_chunk(const farm_memory* mem, const farm_mlp* mlp, const float* U, const float* V,
                                     int64_t t0, int64_t tc, uint16_t* A1, uint16_t* A2, float* L, hipStream_t s) {
  const int64_t H = FARM_MLP_HIDDEN, n = mem->n, pairs = tc * n;
  hipLaunchKernelGGL(k_hidden1, dim3((unsigned)pairs), dim3((unsigned)H), 0, s, U, V, mlp->b1, mlp->W1b, mlp->ldx,
                     2 * mlp->dp, t0, n, mem->x, mem->y, mem->z, mem->ext, mem->rx, mem->ry, A1);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_gemm_nt_bf16(A1, H, mlp->W2b, H, pairs, H, H, A2, H, mlp->b2, true, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_head_rows, dim3(nblk(pairs)), dim3(256), 0, s, A2, mlp->W3r, mlp->b3, t0, tc, n, L);
  return hipGetLastError();
}

}  // namespace farm

using namespace farm;

// The lists of a memory ranked by the network's logits (mlp != null) or by
// the exact predicate value (mlp == null, the non-learned baseline).
static farm_status build_lists(farm_memory* mem, farm_mlp* mlp, int32_t M, void* stream) {
  try {
    if (!mem) { set_error("null memory"); return FARM_ERR_INVALID_ARG; }
    if (mlp && mlp->device != mem->device) { set_error("network and memory live on different devices"); return FARM_ERR_INVALID_ARG; }
    if (mlp && mlp->d != mem->d) { set_error("network width %d != memory width %d", mlp->d, mem->d); return FARM_ERR_INVALID_ARG; }
    if (M < 1 || M > FARM_MAX_K) { set_error("M = %d outside [1, %d]", M, FARM_MAX_K); return FARM_ERR_INVALID_ARG; }
    const int64_t n = mem->n;
    // the per-target bitmap of listed anchors lives in LDS (n / 8 bytes, at most 62.5 KiB)
    if (n > 500000) { set_error("proposal tables need n <= 500000"); return FARM_ERR_UNSUPPORTED; }
    hipStream_t s = (hipStream_t)stream;
    const int64_t H = FARM_MLP_HIDDEN;
    DeviceGuard guard(mem->device);
    // release an earlier table
    if (hipStreamSynchronize(s) != hipSuccess) { set_error("synchronize failed"); return FARM_ERR_HIP; }
    for (void* p : mem->prop_allocs) (void)hipFree(p);
    mem->prop_allocs.clear();
    mem->prop_m = 0;
    mem->prop_idx = nullptr;
    mem->prop_val = nullptr;
    mem->prop_out = nullptr;
    if (n < 2) return FARM_OK;  // no anchors: terms are zero without any table
    if (M > n - 1) M = (int32_t)(n - 1);
    std::vector<void*> tmp;
    auto alloc = [&](std::vector<void*>& list, size_t bytes, void** p) -> bool {
      if (hipMalloc(p, bytes ? bytes : 1) != hipSuccess) { (void)hipGetLastError(); return false; }
      list.push_back(*p);
      return true;
    };
    auto fail = [&](farm_status st, const char* what) {
      (void)hipStreamSynchronize(s);
      for (void* p : tmp) (void)hipFree(p);
      for (void* p : mem->prop_allocs) (void)hipFree(p);
      mem->prop_allocs.clear();
      set_error("building proposals: %s", what);
      return st;
    };
    int32_t* pidx;
    float *pval, *pout;
    if (!alloc(mem->prop_allocs, sizeof(int32_t) * kNPred * M * n, (void**)&pidx) ||
        !alloc(mem->prop_allocs, sizeof(float) * kNPred * M * n, (void**)&pval) ||
        !alloc(mem->prop_allocs, sizeof(float) * kNPred * n, (void**)&pout))
      return fail(FARM_ERR_OOM, "table allocation");
    // network ranking: BF16 descriptors, U = D W1o^T, V = D W1a^T
    const int64_t ldk = mem->ldk;
    uint16_t* dnb = mem->dn_bf16;
    float *U = nullptr, *V = nullptr;
    hipError_t e;
    if (mlp) {
      if (!dnb && !alloc(tmp, sizeof(uint16_t) * n * ldk, (void**)&dnb)) return fail(FARM_ERR_OOM, "descriptor copy");
      if (!alloc(tmp, sizeof(float) * n * H, (void**)&U) || !alloc(tmp, sizeof(float) * n * H, (void**)&V))
        return fail(FARM_ERR_OOM, "first-layer factors");
      if (!mem->dn_bf16) {
        hipLaunchKernelGGL(k_rows_to_bf16, dim3(nblk(n * ldk)), dim3(256), 0, s, mem->dn, n * ldk, dnb);
        if ((e = hipGetLastError()) != hipSuccess) return fail(FARM_ERR_HIP, "descriptor copy");
      }
      if ((e = table_factors(mem, mlp, dnb, U, V, s))) return fail(FARM_ERR_HIP, "first-layer GEMMs");
    }
    // chunks of targets
    // chunk of targets: at most 16, and at most 2^22 pairs (2 GiB of BF16 activations per buffer)
    int64_t tc_max = ((int64_t)1 << 22) / n;
    tc_max = tc_max < 1 ? 1 : tc_max > 16 ? 16 : tc_max;
    if (tc_max > n) tc_max = n;
    uint16_t *A1 = nullptr, *A2 = nullptr;
    float* L;
    if ((mlp && (!alloc(tmp, sizeof(uint16_t) * tc_max * n * H, (void**)&A1) ||
                 !alloc(tmp, sizeof(uint16_t) * tc_max * n * H, (void**)&A2))) ||
        !alloc(tmp, sizeof(float) * kNPred * tc_max * n, (void**)&L))
      return fail(FARM_ERR_OOM, "chunk buffers");
    // TopK candidate buffers in a scratch workspace
    farm_workspace tw;
    tw.mem = mem;
    tw.cand_cap = topk_candidate_capacity(n, (int32_t)(kNPred * tc_max), M);
    for (int b = 0; b < 2; ++b)
      if (!alloc(tmp, sizeof(uint64_t) * tw.cand_cap, (void**)&tw.cand_key[b]) ||
          !alloc(tmp, sizeof(int32_t) * tw.cand_cap, (void**)&tw.cand_idx[b]))
        return fail(FARM_ERR_OOM, "selection buffers");
    int32_t* top_idx;
    if (!alloc(tmp, sizeof(int32_t) * kNPred * tc_max * M, (void**)&top_idx)) return fail(FARM_ERR_OOM, "lists");
    const size_t bitmap = sizeof(uint32_t) * (size_t)((n + 31) / 32);
    for (int64_t t0 = 0; t0 < n; t0 += tc_max) {
      const int64_t tc = n - t0 < tc_max ? n - t0 : tc_max;
      if (mlp) {
        if ((e = table_logits_chunk(mem, mlp, U, V, t0, tc, A1, A2, L, s))) return fail(FARM_ERR_HIP, "table forward");
      } else {
        hipLaunchKernelGGL(k_value_rows, dim3(nblk(tc * n), kNPred), dim3(256), 0, s, t0, tc, n, mem->x, mem->y, mem->z,
                           mem->vz, mem->hr_hi, mem->hr_lo, L);
        if ((e = hipGetLastError()) != hipSuccess) return fail(FARM_ERR_HIP, "predicate values");
      }
      uint64_t* key;
      int32_t* idx;
      if ((e = launch_topk(mem, &tw, L, n, (int32_t)(kNPred * tc), M, &key, &idx, s)))
        return fail(FARM_ERR_HIP, "list selection");
      if ((e = launch_topk_emit(key, idx, (int32_t)(kNPred * tc), M, nullptr, nullptr, top_idx, s)))
        return fail(FARM_ERR_HIP, "list emit");
      hipLaunchKernelGGL(k_prop_finalize, dim3((unsigned)tc, kNPred), dim3(256), bitmap, s, top_idx, M, t0, tc, n,
                         mem->x, mem->y, mem->z, mem->vz, mem->hr_hi, mem->hr_lo, pidx, pval, pout);
      if ((e = hipGetLastError()) != hipSuccess) return fail(FARM_ERR_HIP, "finalize");
    }
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(FARM_ERR_HIP, "synchronize");
    for (void* p : tmp) (void)hipFree(p);
    mem->prop_idx = pidx;
    mem->prop_val = pval;
    mem->prop_out = pout;
    mem->prop_m = M;
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_build_proposals");
    return FARM_ERR_HIP;
  }
}

extern "C" farm_status farm_build_proposals(farm_memory* mem, farm_mlp* mlp, int32_t M, void* stream) {
  if (!mlp) { set_error("null network"); return FARM_ERR_INVALID_ARG; }
  return build_lists(mem, mlp, M, stream);
}

extern "C" farm_status farm_build_proposals_by_value(farm_memory* mem, int32_t M, void* stream) {
  return build_lists(mem, nullptr, M, stream);
}

extern "C" farm_status farm_get_proposals(const farm_memory* mem, int32_t* m_out, int32_t* idx, float* val, float* out,
                                          void* stream) {
  try {
    if (!mem || !m_out) { set_error("null memory or m_out"); return FARM_ERR_INVALID_ARG; }
    *m_out = mem->prop_m;
    if (mem->prop_m == 0) return FARM_OK;
    DeviceGuard guard(mem->device);
    hipStream_t s = (hipStream_t)stream;
    const size_t entries = (size_t)kNPred * mem->n * mem->prop_m;
    hipError_t e = hipSuccess;
    if (idx && e == hipSuccess)
      e = hipMemcpyAsync(idx, mem->prop_idx, entries * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    if (val && e == hipSuccess) e = hipMemcpyAsync(val, mem->prop_val, entries * sizeof(float), hipMemcpyDeviceToDevice, s);
    if (out && e == hipSuccess)
      e = hipMemcpyAsync(out, mem->prop_out, (size_t)kNPred * mem->n * sizeof(float), hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? FARM_OK : hip_fail(e, "copying proposal tables");
  } catch (...) {
    set_error("unexpected host exception in farm_get_proposals");
    return FARM_ERR_HIP;
  }
}

extern "C" farm_status farm_mlp_table_logits(farm_mlp* mlp, const farm_memory* mem, int64_t t0, int32_t tc,
                                             float* logits, void* stream) {
  try {
    if (!mem || !mlp || !logits) { set_error("null memory, network or output"); return FARM_ERR_INVALID_ARG; }
    if (mlp->device != mem->device || mlp->d != mem->d) { set_error("network and memory do not match"); return FARM_ERR_INVALID_ARG; }
    const int64_t n = mem->n, H = FARM_MLP_HIDDEN;
    if (tc < 1 || tc > 16 || t0 < 0 || t0 + tc > n || (int64_t)tc * n > ((int64_t)1 << 22)) {
      set_error("targets [%lld, %lld) outside the memory or the chunk limits", (long long)t0, (long long)(t0 + tc));
      return FARM_ERR_INVALID_ARG;
    }
    DeviceGuard guard(mem->device);
    hipStream_t s = (hipStream_t)stream;
    std::vector<void*> tmp;
    auto alloc = [&](size_t bytes, void** p) -> bool {
      if (hipMalloc(p, bytes ? bytes : 1) != hipSuccess) { (void)hipGetLastError(); return false; }
      tmp.push_back(*p);
      return true;
    };
    auto done = [&](farm_status st, const char* what) {
      (void)hipStreamSynchronize(s);
      for (void* p : tmp) (void)hipFree(p);
      if (st != FARM_OK) set_error("table logits: %s", what);
      return st;
    };
    uint16_t* dnb = mem->dn_bf16;
    float *U, *V;
    uint16_t *A1, *A2;
    if (!dnb && !alloc(sizeof(uint16_t) * n * mem->ldk, (void**)&dnb)) return done(FARM_ERR_OOM, "descriptor copy");
    if (!alloc(sizeof(float) * n * H, (void**)&U) || !alloc(sizeof(float) * n * H, (void**)&V) ||
        !alloc(sizeof(uint16_t) * tc * n * H, (void**)&A1) || !alloc(sizeof(uint16_t) * tc * n * H, (void**)&A2))
      return done(FARM_ERR_OOM, "buffers");
    hipError_t e = hipSuccess;
    if (!mem->dn_bf16) {
      hipLaunchKernelGGL(k_rows_to_bf16, dim3(nblk(n * mem->ldk)), dim3(256), 0, s, mem->dn, n * mem->ldk, dnb);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = table_factors(mem, mlp, dnb, U, V, s);
    if (e == hipSuccess) e = table_logits_chunk(mem, mlp, U, V, t0, tc, A1, A2, logits, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      done(FARM_OK, "");
      return hip_fail(e, "table logits forward");
    }
    return done(FARM_OK, "");
  } catch (...) {
    set_error("unexpected host exception in farm_mlp_table_logits");
    return FARM_ERR_HIP;
  }
}
