// topk.hip -- TopK of score rows with the object-id tie-break.
//
// Order: score descending, then object id ascending (Section 2.3 TopK over
// entities; the id tie-break is a reading).  Each (score, id) pair becomes one
// 64-bit key whose unsigned order is exactly that order:
//   key = ord(score) << 32 | (0xFFFFFFFF - id)
// where ord() maps IEEE floats monotonically onto unsigned integers.  Key 0
// never arises from a real entry (it would need a NaN score), so it pads.
//
// One block per row.  A first pass takes the largest key of every chunk of
// consecutive entries (64 entries, more for rows longer than 4096 chunks) and
// sorts those chunk maxima: the k-th largest of them, L, has at least k keys
// at or above it (the maxima of the k best chunks), so no key below L can be
// in the TopK.  A second pass keeps a running list of the best k in LDS and
// adds the keys >= L of each segment of the row (at most 4096 - k entries), a
// bitonic sort of the list and the new keys keeping the best k.  For spread
// scores the keys >= L number little more than k, so the row costs two reads
// and a few small sorts; a row of equal scores degenerates into sorting every
// segment, the cost of a full sort.
#include "farm_internal.h"
#include "sort_util.h"

namespace farm {
namespace {

__device__ inline uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

__global__ __launch_bounds__(256) void k_topk_select(const float* __restrict__ scores, int64_t ld, int64_t n,
                                                     const uint32_t* __restrict__ ids, int32_t k,
                                                     uint64_t* __restrict__ out_key, int32_t* __restrict__ out_idx) {
  __shared__ uint64_t keys[kSortMax];
  __shared__ int32_t idx[kSortMax];
  __shared__ int32_t cnt_s;
  const int32_t qq = blockIdx.x;
  const float* row = scores + (int64_t)qq * ld;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  // 1. the largest key of every chunk; at most kSortMax chunks
  int64_t chunk = 64;
  while ((n + chunk - 1) / chunk > kSortMax) chunk += 64;
  const int nch = (int)((n + chunk - 1) / chunk);
  for (int c = wave; c < nch; c += nwave) {
    uint64_t m = 0;
    const int64_t c0 = (int64_t)c * chunk, c1 = c0 + chunk < n ? c0 + chunk : n;
    for (int64_t i = c0 + lane; i < c1; i += 64) {
      const uint64_t key = make_key(row[i], ids[i]);
      m = key > m ? key : m;
    }
    m = wave_max_u64(m);
    if (lane == 0) {
      keys[c] = m;
      idx[c] = -1;
    }
  }
  int P = pow2_at_least(nch);
  for (int e = nch + threadIdx.x; e < P; e += blockDim.x) {
    keys[e] = 0;
    idx[e] = -1;
  }
  __syncthreads();
  bitonic_desc(keys, idx, P);
  const uint64_t L = nch >= k ? keys[k - 1] : 0;
  __syncthreads();
  // 2. running best k over the keys >= L, one segment at a time
  int have = 0;
  const int64_t seg = kSortMax - k;
  for (int64_t s0 = 0; s0 < n; s0 += seg) {
    if (threadIdx.x == 0) cnt_s = have;
    __syncthreads();
    const int64_t s1 = s0 + seg < n ? s0 + seg : n;
    for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
      const uint64_t key = make_key(row[i], ids[i]);
      if (key >= L) {
        const int p = atomicAdd(&cnt_s, 1);
        keys[p] = key;
        idx[p] = (int32_t)i;
      }
    }
    __syncthreads();
    const int c = cnt_s;
    if (c > have) {  // block-uniform
      P = pow2_at_least(c);
      for (int e = c + threadIdx.x; e < P; e += blockDim.x) {
        keys[e] = 0;
        idx[e] = -1;
      }
      __syncthreads();
      bitonic_desc(keys, idx, P);
      have = c < k ? c : k;
    }
    __syncthreads();
  }
  uint64_t* ok = out_key + (int64_t)qq * k;
  int32_t* oi = out_idx + (int64_t)qq * k;
  for (int e = threadIdx.x; e < k; e += blockDim.x) {
    ok[e] = e < have ? keys[e] : 0;
    oi[e] = e < have ? idx[e] : -1;
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
  (void)n;
  return (int64_t)max_q * max_k;  // one list of k per row
}

hipError_t launch_topk(const farm_memory* mem, farm_workspace* ws, const float* scores, int64_t ld_scores,
                       int32_t q, int32_t k, uint64_t** out_key, int32_t** out_idx, hipStream_t s) {
  if ((int64_t)q * k > ws->cand_cap || k > kSortMax / 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_topk_select, dim3((unsigned)q), dim3(256), 0, s, scores, ld_scores, mem->n, mem->id, k,
                     ws->cand_key[0], ws->cand_idx[0]);
  *out_key = ws->cand_key[0];
  *out_idx = ws->cand_idx[0];
  return hipGetLastError();
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
