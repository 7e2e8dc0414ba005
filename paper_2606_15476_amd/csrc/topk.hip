// topk.hip -- TopK of score rows with the object-id tie-break.
//
// Order: score descending, then object id ascending (Section 2.3 TopK over
// entities; the id tie-break is a reading).  Each (score, id) pair becomes one
// 64-bit key whose unsigned order is exactly that order:
//   key = ord(score) << 32 | (0xFFFFFFFF - id)
// where ord() maps IEEE floats monotonically onto unsigned integers.  Key 0
// never arises from a real entry (it would need a NaN score), so it pads.
//
// Pass 1 sorts blocks of up to 4096 entries of a row in LDS (bitonic network,
// 256 threads) and keeps each block's best k; merge passes sort groups of
// those candidate lists the same way until one list of k remains.  The network
// is data-oblivious: the cost depends only on the sizes.
#include "farm_internal.h"
#include "sort_util.h"

namespace farm {
namespace {

__global__ __launch_bounds__(256) void k_topk_rows(const float* __restrict__ scores, int64_t ld, int64_t n,
                                                   const uint32_t* __restrict__ ids, int32_t k, int32_t nblk,
                                                   uint64_t* __restrict__ out_key, int32_t* __restrict__ out_idx) {
  __shared__ uint64_t keys[kSortMax];
  __shared__ int32_t idx[kSortMax];
  const int32_t qq = blockIdx.y, blk = blockIdx.x;
  const int64_t base = (int64_t)blk * kSortMax;
  const int cnt = (int)(n - base < kSortMax ? n - base : kSortMax);
  const int P = pow2_at_least(cnt);
  const float* row = scores + (int64_t)qq * ld;
  for (int e = threadIdx.x; e < P; e += blockDim.x) {
    if (e < cnt) {
      int64_t i = base + e;
      keys[e] = make_key(row[i], ids[i]);
      idx[e] = (int32_t)i;
    } else {
      keys[e] = 0;
      idx[e] = -1;
    }
  }
  __syncthreads();
  bitonic_desc(keys, idx, P);
  uint64_t* ok = out_key + ((int64_t)qq * nblk + blk) * k;
  int32_t* oi = out_idx + ((int64_t)qq * nblk + blk) * k;
  for (int e = threadIdx.x; e < k; e += blockDim.x) {
    ok[e] = e < P ? keys[e] : 0;
    oi[e] = e < P ? idx[e] : -1;
  }
}

// Merge groups of `group` candidate lists (each of length k) per row.
__global__ __launch_bounds__(256) void k_topk_merge(const uint64_t* __restrict__ in_key,
                                                    const int32_t* __restrict__ in_idx, int32_t nlist, int32_t k,
                                                    int32_t group, int32_t nout, uint64_t* __restrict__ out_key,
                                                    int32_t* __restrict__ out_idx) {
  __shared__ uint64_t keys[kSortMax];
  __shared__ int32_t idx[kSortMax];
  const int32_t qq = blockIdx.y, g = blockIdx.x;
  const int32_t l0 = g * group;
  const int32_t nl = nlist - l0 < group ? nlist - l0 : group;
  const int cnt = nl * k;
  const int P = pow2_at_least(cnt);
  const uint64_t* ik = in_key + ((int64_t)qq * nlist + l0) * k;
  const int32_t* ii = in_idx + ((int64_t)qq * nlist + l0) * k;
  for (int e = threadIdx.x; e < P; e += blockDim.x) {
    keys[e] = e < cnt ? ik[e] : 0;
    idx[e] = e < cnt ? ii[e] : -1;
  }
  __syncthreads();
  bitonic_desc(keys, idx, P);
  uint64_t* ok = out_key + ((int64_t)qq * nout + g) * k;
  int32_t* oi = out_idx + ((int64_t)qq * nout + g) * k;
  for (int e = threadIdx.x; e < k; e += blockDim.x) {
    ok[e] = keys[e];
    oi[e] = idx[e];
  }
}

__global__ void k_topk_emit(const uint64_t* __restrict__ key, const int32_t* __restrict__ idx, int64_t total,
                            uint32_t* __restrict__ out_id, float* __restrict__ out_score,
                            int32_t* __restrict__ out_index) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  uint64_t kk = key[e];
  bool pad = kk == 0;
  if (out_id) out_id[e] = pad ? FARM_NO_ID : 0xFFFFFFFFu - (uint32_t)(kk & 0xFFFFFFFFu);
  if (out_score) out_score[e] = pad ? -INFINITY : unord_float((uint32_t)(kk >> 32));
  if (out_index) out_index[e] = pad ? -1 : idx[e];
}

}  // namespace

int64_t topk_candidate_capacity(int64_t n, int32_t max_q, int32_t max_k) {
  int64_t nblk = (n + kSortMax - 1) / kSortMax;
  if (nblk < 1) nblk = 1;
  return (int64_t)max_q * nblk * max_k;
}

hipError_t launch_topk(const farm_memory* mem, farm_workspace* ws, const float* scores, int64_t ld_scores,
                       int32_t q, int32_t k, uint64_t** out_key, int32_t** out_idx, hipStream_t s) {
  const int64_t n = mem->n;
  int32_t nblk = (int32_t)((n + kSortMax - 1) / kSortMax);
  if ((int64_t)q * nblk * k > ws->cand_cap) return hipErrorInvalidValue;
  int cur = 0;
  hipLaunchKernelGGL(k_topk_rows, dim3((unsigned)nblk, (unsigned)q), dim3(256), 0, s, scores, ld_scores, n, mem->id,
                     k, nblk, ws->cand_key[cur], ws->cand_idx[cur]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int32_t nlist = nblk;
  const int32_t group = kSortMax / k >= 2 ? kSortMax / k : 2;
  while (nlist > 1) {
    int32_t nout = (nlist + group - 1) / group;
    hipLaunchKernelGGL(k_topk_merge, dim3((unsigned)nout, (unsigned)q), dim3(256), 0, s, ws->cand_key[cur],
                       ws->cand_idx[cur], nlist, k, group, nout, ws->cand_key[cur ^ 1], ws->cand_idx[cur ^ 1]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur ^= 1;
    nlist = nout;
  }
  *out_key = ws->cand_key[cur];
  *out_idx = ws->cand_idx[cur];
  return hipSuccess;
}

hipError_t launch_topk_emit(const uint64_t* key, const int32_t* idx, int32_t q, int32_t k, uint32_t* out_id,
                            float* out_score, int32_t* out_index, hipStream_t s) {
  int64_t total = (int64_t)q * k;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_topk_emit, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, key, idx, total, out_id,
                     out_score, out_index);
  return hipGetLastError();
}

}  // namespace farm
