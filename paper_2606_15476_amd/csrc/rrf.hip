// rrf.hip -- multi-channel reciprocal-rank fusion of the unary scores
// (Appendix "Retrieval Details", step 3: each query channel ranks the whole
// pool and adds w / (mu + rank), mu = 5).
//
// One block ranks one row of a channel's cosines at a time (grid-stride over
// the rows).  The exact rank of every element -- 1 + the number of elements
// with a larger cosine, or an equal one and a smaller object id -- comes from
// a bucketed counting sort: the row's value range is cut into 8192 buckets by
// a map that is monotone in the value, so every element of an earlier bucket
// ranks before every element of a later one; a histogram and its prefix sum
// give each bucket's first rank, and the elements are scattered into bucket
// order.  Work per row O(n + buckets + sum of the squared bucket sizes):
// linear for cosines spread over their range, quadratic only in the size of
// groups of (nearly) equal values.
//
// Rows of at most kRrfLdsMaxN objects (k_rrf_rank_lds): each thread holds its
// elements in registers for all passes, the bucket-ordered values sit in LDS,
// and each element counts the larger values of its own bucket there; object
// ids are compared (through the scattered element indices, block scratch in
// global memory) only within groups of exactly equal values.  Longer rows
// (k_rrf_rank): the bucket-ordered (value, index) pairs go to block scratch in
// global memory (L2-resident) and a wave per bucket counts, for each of its
// elements, the bucket's elements that precede it (64 elements at a time in
// registers, compared through shuffles).
#include <math.h>

#include <algorithm>

#include "farm_internal.h"

namespace farm {
namespace {

constexpr int kRrfBuckets = 8192;
constexpr int kRrfThreads = 256;
constexpr float kRrfMu = 5.0f;

// Bucket of value v for a row with largest value vmax: non-decreasing as v
// decreases (a rounded difference, a product with a positive factor and a
// truncation are each monotone).
__device__ inline int rrf_bucket(float v, float vmax, float scale) {
  const float t = (vmax - v) * scale;
  return t < (float)(kRrfBuckets - 1) ? (int)t : kRrfBuckets - 1;
}

__global__ __launch_bounds__(kRrfThreads) void k_rrf_rank(const float* __restrict__ cos, int64_t ld, int32_t rows,
                                                          int64_t n, const uint32_t* __restrict__ ids, float w,
                                                          float* __restrict__ out, float* __restrict__ sval,
                                                          int32_t* __restrict__ sidx) {
  __shared__ int32_t start[kRrfBuckets];  // first position of each bucket (after the scan)
  __shared__ int32_t fill[kRrfBuckets];   // elements placed so far, then the bucket sizes
  __shared__ int32_t part[kRrfThreads];
  __shared__ float red_lo[kRrfThreads / 64], red_hi[kRrfThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  float* val = sval + (int64_t)blockIdx.x * n;
  int32_t* idx = sidx + (int64_t)blockIdx.x * n;
  for (int32_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const float* c = cos + (int64_t)row * ld;
    // the row's range
    float lo = INFINITY, hi = -INFINITY;
    for (int64_t j = tid; j < n; j += kRrfThreads) {
      const float v = c[j];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off));
      hi = fmaxf(hi, __shfl_xor(hi, off));
    }
    if (lane == 0) {
      red_lo[wave] = lo;
      red_hi[wave] = hi;
    }
    for (int b = tid; b < kRrfBuckets; b += kRrfThreads) {
      start[b] = 0;
      fill[b] = 0;
    }
    __syncthreads();
    lo = red_lo[0];
    hi = red_hi[0];
#pragma unroll
    for (int u = 1; u < kRrfThreads / 64; ++u) {
      lo = fminf(lo, red_lo[u]);
      hi = fmaxf(hi, red_hi[u]);
    }
    float scale = hi > lo ? (float)(kRrfBuckets - 1) / (hi - lo) : 0.0f;
    if (!(scale < INFINITY)) scale = 0.0f;  // a range too small to divide: one bucket
    // histogram
    for (int64_t j = tid; j < n; j += kRrfThreads) atomicAdd(&start[rrf_bucket(c[j], hi, scale)], 1);
    __syncthreads();
    // exclusive prefix sum over the buckets: per-thread runs of 32, then the run totals
    constexpr int kRun = kRrfBuckets / kRrfThreads;
    int sum = 0;
#pragma unroll 4
    for (int e = 0; e < kRun; ++e) {
      const int v = start[tid * kRun + e];
      start[tid * kRun + e] = sum;
      sum += v;
    }
    part[tid] = sum;
    __syncthreads();
    if (tid == 0) {
      int acc = 0;
      for (int t = 0; t < kRrfThreads; ++t) {
        const int v = part[t];
        part[t] = acc;
        acc += v;
      }
    }
    __syncthreads();
    {
      const int add = part[tid];
#pragma unroll 4
      for (int e = 0; e < kRun; ++e) start[tid * kRun + e] += add;
    }
    __syncthreads();
    // scatter into bucket order
    for (int64_t j = tid; j < n; j += kRrfThreads) {
      const float v = c[j];
      const int b = rrf_bucket(v, hi, scale);
      const int p = start[b] + atomicAdd(&fill[b], 1);
      val[p] = v;
      idx[p] = (int32_t)j;
    }
    __syncthreads();
    // exact rank: the elements of earlier buckets, plus those of the own bucket that precede.
    // One wave per bucket: 64 of its elements at a time in registers, each compared with every
    // element of the bucket through shuffles.
    for (int b = wave; b < kRrfBuckets; b += kRrfThreads / 64) {
      const int s0 = start[b], nb = fill[b];
      for (int c0 = 0; c0 < nb; c0 += 64) {
        const bool mine = c0 + lane < nb;
        const float v = mine ? val[s0 + c0 + lane] : 0.0f;
        const int32_t i = mine ? idx[s0 + c0 + lane] : 0;
        const uint32_t id = mine ? ids[i] : 0u;
        int before = 0;
        for (int c1 = 0; c1 < nb; c1 += 64) {
          const bool theirs = c1 + lane < nb;
          const float u = theirs ? val[s0 + c1 + lane] : 0.0f;
          const uint32_t uid = theirs ? ids[idx[s0 + c1 + lane]] : 0u;
          const int cnt = nb - c1 < 64 ? nb - c1 : 64;
          for (int t = 0; t < cnt; ++t) {
            const float ut = __shfl(u, t);
            const uint32_t it = __shfl(uid, t);
            before += (ut > v || (ut == v && it < id)) ? 1 : 0;
          }
        }
        if (mine) out[(int64_t)row * ld + i] += w / (kRrfMu + (float)(s0 + before + 1));
      }
    }
    __syncthreads();  // the next row reuses the tables and the scratch
  }
}

// LDS form: rows of at most kRrfLdsMaxN objects.  1024 threads, kRrfPer
// elements per thread in registers (element j = tid + k * 1024).
constexpr int kRrfLdsThreads = 1024;
constexpr int kRrfLdsWaves = kRrfLdsThreads / 64;
constexpr int kRrfPer = 24;
constexpr size_t kRrfLdsStatic = sizeof(int32_t) * (2 * kRrfBuckets + 1) + sizeof(int32_t) * kRrfLdsWaves + 64;
constexpr size_t kRrfLdsTotal = 160 * 1024;  // LDS of one gfx950 workgroup
constexpr int64_t kRrfLdsMaxN = std::min<int64_t>((int64_t)kRrfLdsThreads * kRrfPer,
                                                  (int64_t)((kRrfLdsTotal - kRrfLdsStatic) / sizeof(float)));

__global__ __launch_bounds__(kRrfLdsThreads) void k_rrf_rank_lds(const float* __restrict__ cos, int64_t ld,
                                                                 int32_t rows, int64_t n,
                                                                 const uint32_t* __restrict__ ids, float w,
                                                                 float* __restrict__ out,
                                                                 int32_t* __restrict__ sidx) {
  extern __shared__ float sval[];          // the row's values in bucket order
  __shared__ int32_t start[kRrfBuckets + 1];  // first position of each bucket; start[kRrfBuckets] = n
  __shared__ int32_t fill[kRrfBuckets];       // scatter cursors
  __shared__ int32_t wsum[kRrfLdsWaves];
  __shared__ float red_lo[kRrfLdsWaves], red_hi[kRrfLdsWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int32_t* idx = sidx + (int64_t)blockIdx.x * n;
  for (int32_t row = blockIdx.x; row < rows; row += gridDim.x) {
    const float* c = cos + (int64_t)row * ld;
    float v[kRrfPer];
    float lo = INFINITY, hi = -INFINITY;
#pragma unroll
    for (int k = 0; k < kRrfPer; ++k) {
      const int64_t j = tid + (int64_t)k * kRrfLdsThreads;
      v[k] = j < n ? c[j] : 0.0f;
      if (j < n) {
        lo = fminf(lo, v[k]);
        hi = fmaxf(hi, v[k]);
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lo = fminf(lo, __shfl_xor(lo, off));
      hi = fmaxf(hi, __shfl_xor(hi, off));
    }
    if (lane == 0) {
      red_lo[wave] = lo;
      red_hi[wave] = hi;
    }
    for (int b = tid; b < kRrfBuckets; b += kRrfLdsThreads) {
      start[b] = 0;
      fill[b] = 0;
    }
    __syncthreads();
    lo = red_lo[0];
    hi = red_hi[0];
#pragma unroll
    for (int u = 1; u < kRrfLdsWaves; ++u) {
      lo = fminf(lo, red_lo[u]);
      hi = fmaxf(hi, red_hi[u]);
    }
    float scale = hi > lo ? (float)(kRrfBuckets - 1) / (hi - lo) : 0.0f;
    if (!(scale < INFINITY)) scale = 0.0f;  // a range too small to divide: one bucket
    // histogram
#pragma unroll
    for (int k = 0; k < kRrfPer; ++k)
      if (tid + (int64_t)k * kRrfLdsThreads < n) atomicAdd(&start[rrf_bucket(v[k], hi, scale)], 1);
    __syncthreads();
    // exclusive prefix sum: runs of kRun buckets per thread, a wave scan of
    // the run totals, then the wave totals
    constexpr int kRun = kRrfBuckets / kRrfLdsThreads;
    int run[kRun];
    int sum = 0;
#pragma unroll
    for (int e = 0; e < kRun; ++e) {
      run[e] = start[tid * kRun + e];
      sum += run[e];
    }
    int incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int base = incl - sum;
    for (int u = 0; u < wave; ++u) base += wsum[u];
#pragma unroll
    for (int e = 0; e < kRun; ++e) {
      start[tid * kRun + e] = base;
      base += run[e];
    }
    if (tid == kRrfLdsThreads - 1) start[kRrfBuckets] = base;  // = n
    __syncthreads();
    // scatter into bucket order (values in LDS, element indices in scratch)
#pragma unroll
    for (int k = 0; k < kRrfPer; ++k) {
      const int64_t j = tid + (int64_t)k * kRrfLdsThreads;
      if (j < n) {
        const int b = rrf_bucket(v[k], hi, scale);
        const int p = start[b] + atomicAdd(&fill[b], 1);
        sval[p] = v[k];
        idx[p] = (int32_t)j;
      }
    }
    __syncthreads();
    // exact rank: the elements of earlier buckets, the larger values of the
    // own bucket, and equal values with a smaller id (the value is read again,
    // from L2: held in registers through this loop it would spill)
#pragma unroll 1
    for (int64_t j = tid; j < n; j += kRrfLdsThreads) {
      const float x = c[j];
      const int b = rrf_bucket(x, hi, scale);
      const int s0 = start[b], s1 = start[b + 1];
      int gt = 0, eq = 0;
      for (int e = s0; e < s1; ++e) {
        const float u = sval[e];
        gt += u > x ? 1 : 0;
        eq += u == x ? 1 : 0;
      }
      if (eq > 1) {  // equal values besides this one: order by id
        const uint32_t id = ids[j];
        for (int e = s0; e < s1; ++e)
          if (sval[e] == x) {
            const int32_t i2 = idx[e];
            gt += (i2 != (int32_t)j && ids[i2] < id) ? 1 : 0;
          }
      }
      out[(int64_t)row * ld + j] += w / (kRrfMu + (float)(s0 + gt + 1));
    }
    __syncthreads();  // the next row reuses the tables
  }
}

__global__ void k_rrf_finish(float* __restrict__ out, int64_t ld, int32_t q, int32_t rows, int64_t n,
                             const int32_t* __restrict__ tcls, const int32_t* __restrict__ cls, float inv_norm) {
  const int32_t row = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows || j >= n) return;
  float f = inv_norm;
  if (row < q && cls) {
    const int32_t tc = tcls[row], oc = cls[j];
    if (tc >= 0 && oc >= 0 && tc != oc) f *= kClassFactor;
  }
  out[(int64_t)row * ld + j] *= f;
}

}  // namespace

hipError_t launch_rrf_rank(const float* cos, int64_t ld, int32_t rows, int64_t n, const uint32_t* ids, float w,
                           float* out, float* val, int32_t* idx, int32_t blocks, hipStream_t s) {
  if (rows <= 0 || n <= 0) return hipSuccess;
  const int32_t g = rows < blocks ? rows : blocks;
  if (n <= kRrfLdsMaxN) {
    const size_t bytes = sizeof(float) * (size_t)n;
    if (bytes > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rrf_rank_lds),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_rrf_rank_lds, dim3((unsigned)g), dim3(kRrfLdsThreads), bytes, s, cos, ld, rows, n, ids, w,
                       out, idx);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_rrf_rank, dim3((unsigned)g), dim3(kRrfThreads), 0, s, cos, ld, rows, n, ids, w, out, val, idx);
  return hipGetLastError();
}

hipError_t launch_rrf_finish(float* out, int64_t ld, int32_t q, int32_t rows, int64_t n, const int32_t* tcls,
                             const int32_t* cls, float inv_norm, hipStream_t s) {
  if (rows <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rrf_finish, dim3((unsigned)((n + 255) / 256), (unsigned)rows), dim3(256), 0, s, out, ld, q,
                     rows, n, tcls, cls, inv_norm);
  return hipGetLastError();
}

}  // namespace farm
