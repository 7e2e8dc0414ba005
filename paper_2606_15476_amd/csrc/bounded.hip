// bounded.hip -- exact TopK without scoring every object.
//
// The soft blend keeps the spatial factor in [1 - w, 1] (Appendix "Retrieval
// Details", "Why soft, not hard?"), so every object's score lies between
// (1 - w) s_sem and s_sem.  Let L be the K-th largest lower bound
// (1 - w) s_sem_lo over all objects: K objects score at least L, so an object
// whose upper bound s_sem_hi is below L scores strictly below them and cannot
// enter the TopK.  Only the remaining candidates are scored (rescore.hip);
// the TopK among them is the exact TopK.  With FP32 similarities
// s_sem_lo = s_sem_hi = s_sem; with BF16/FP8 similarities they are the
// estimate minus/plus its proven error bound.
//
// One block per query: L is found from per-thread sorted top-16 lists and K
// rounds of a block arg-max (K <= 16), or by a 4-round radix select on the
// IEEE bits of the non-negative lower bounds (larger K), and the candidates
// are compacted (an LDS counter for K <= 16, an ordered block scan
// otherwise).  If more than `cap` objects survive, the list keeps the `cap`
// largest upper bounds (a second radix select) and the query is marked
// uncertified.
#include <math.h>

#include "farm_internal.h"

namespace farm {
namespace {

constexpr int kThreads = 256;

struct SemBounds {
  float lo, hi;
};

__device__ inline SemBounds sem_bounds(const float* srow, int64_t i, int tc, const int32_t* cls, const SimBound& b,
                                       int32_t qq) {
  const float s = srow[i];
  if (!b.q_nrm) return {s, s};
  const float kappa = (tc >= 0 && cls && cls[i] >= 0 && cls[i] != tc) ? kClassFactor : 1.0f;
  const float d = kappa * fmaf(b.q_nrm[qq], b.o_err[i], b.q_err[qq] + b.acc);
  return {fmaxf(0.f, s - d), fminf(kappa, s + d)};
}

// K-th largest key among the values produced by `key(i)` (non-negative floats
// as IEEE bits, or 0 for excluded entries).  All threads return the result.
template <int NT = kThreads, class KeyFn>
__device__ uint32_t radix_select_kth(int64_t n, int64_t k, KeyFn key, uint32_t* hist, uint32_t* shared_word) {
  uint32_t prefix = 0, mask = 0;
  int64_t remaining = k;
  for (int shift = 24; shift >= 0; shift -= 8) {
    for (int b = threadIdx.x; b < 256; b += NT) hist[b] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += NT) {
      const uint32_t u = key(i);
      if ((u & mask) == prefix) atomicAdd(&hist[(u >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t acc = 0;
      int bin = 255;
      for (; bin > 0; --bin) {
        if (acc + (int64_t)hist[bin] >= remaining) break;
        acc += hist[bin];
      }
      remaining -= acc;
      shared_word[0] = (uint32_t)bin;
      shared_word[1] = (uint32_t)remaining;
    }
    __syncthreads();
    prefix |= shared_word[0] << shift;
    mask |= 0xFFu << shift;
    remaining = shared_word[1];
    __syncthreads();
  }
  return prefix;
}

// K-th largest of the values lo(i), K <= kSmallK: each thread keeps its own
// sorted top-kSmallK in registers (which must contain its share of the global
// top K), then K rounds of a block arg-max pop the heads.
constexpr int kSmallK = 16;

template <class LoFn>
__device__ float kth_largest_small(int64_t n, int k, LoFn lo, float* red_v, int* red_t) {
  float top[kSmallK];
#pragma unroll
  for (int e = 0; e < kSmallK; ++e) top[e] = -INFINITY;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) {
    const float v = lo(i);
    if (v > top[kSmallK - 1]) {
#pragma unroll
      for (int e = kSmallK - 1; e > 0; --e) top[e] = v > top[e - 1] ? top[e - 1] : fmaxf(v, top[e]);
      top[0] = fmaxf(top[0], v);
    }
  }
  float kth = -INFINITY;
  for (int round = 0; round < k; ++round) {
    red_v[threadIdx.x] = top[0];
    red_t[threadIdx.x] = threadIdx.x;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        const float a = red_v[threadIdx.x], b = red_v[threadIdx.x + w];
        if (b > a || (b == a && red_t[threadIdx.x + w] < red_t[threadIdx.x])) {
          red_v[threadIdx.x] = b;
          red_t[threadIdx.x] = red_t[threadIdx.x + w];
        }
      }
      __syncthreads();
    }
    kth = red_v[0];
    if ((int)threadIdx.x == red_t[0]) {
#pragma unroll
      for (int e = 0; e < kSmallK - 1; ++e) top[e] = top[e + 1];
      top[kSmallK - 1] = -INFINITY;
    }
    __syncthreads();
  }
  return kth;
}

__global__ __launch_bounds__(kThreads) void k_bound_candidates(const float* __restrict__ sim, int64_t ld_s, int64_t n,
                                                               MetaView meta, SimBound bound,
                                                               const int32_t* __restrict__ cls, int32_t k,
                                                               int32_t cap, int32_t* __restrict__ cand,
                                                               int32_t* __restrict__ count,
                                                               int32_t* __restrict__ certified) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t word[2];
  __shared__ int32_t scan[kThreads];
  __shared__ float red_v[kThreads];
  const int32_t qq = blockIdx.x;
  const float* srow = sim + (int64_t)qq * ld_s;
  const int tc = meta.tcls[qq];
  // L: K-th largest lower bound (1 - w) s_sem_lo
  float L = -INFINITY;
  if (n > k) {
    if (k <= kSmallK) {
      auto lo_val = [&](int64_t i) { return (1.0f - kW) * sem_bounds(srow, i, tc, cls, bound, qq).lo; };
      L = kth_largest_small(n, k, lo_val, red_v, scan);
    } else {
      auto lo_key = [&](int64_t i) {
        return __float_as_uint((1.0f - kW) * sem_bounds(srow, i, tc, cls, bound, qq).lo);
      };
      L = __uint_as_float(radix_select_kth(n, k, lo_key, hist, word));
    }
  }
  // candidates: s_sem_hi >= L
  const int64_t chunk = (n + kThreads - 1) / kThreads;
  const int64_t i0 = threadIdx.x * chunk, i1 = i0 + chunk < n ? i0 + chunk : n;
  auto pass = [&](float thresh, bool write) {
    int32_t c = 0;
    for (int64_t i = i0; i < i1; ++i) c += sem_bounds(srow, i, tc, cls, bound, qq).hi >= thresh;
    scan[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {  // inclusive Hillis-Steele scan
      int32_t v = threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
      __syncthreads();
      scan[threadIdx.x] += v;
      __syncthreads();
    }
    const int32_t total = scan[kThreads - 1];
    if (write) {
      int32_t pos = scan[threadIdx.x] - c;
      for (int64_t i = i0; i < i1 && pos < cap; ++i)
        if (sem_bounds(srow, i, tc, cls, bound, qq).hi >= thresh) cand[(int64_t)qq * cap + pos++] = (int32_t)i;
    }
    __syncthreads();
    return total;
  };
  int32_t total = pass(L, false);
  bool exact = true;
  float thresh = L;
  if (total > cap) {
    // keep the cap largest upper bounds (ties at the threshold may exceed cap: truncated in index order)
    auto hi_key = [&](int64_t i) {
      const float h = sem_bounds(srow, i, tc, cls, bound, qq).hi;
      return h >= L ? __float_as_uint(h) : 0u;
    };
    thresh = fmaxf(L, __uint_as_float(radix_select_kth(n, cap, hi_key, hist, word)));
    exact = false;
  }
  total = pass(thresh, true);
  total = total < cap ? total : cap;
  for (int32_t c = total + threadIdx.x; c < cap; c += kThreads) cand[(int64_t)qq * cap + c] = -1;
  if (threadIdx.x == 0) {
    count[qq] = total;
    if (certified) certified[qq] = exact ? 1 : 0;
  }
}


// Block-per-query form for K <= kSmallK: four waves share a query's row (more
// loads in flight than one wave), per-thread sorted top-K lists and K rounds
// of a block arg-max give L, and the candidates are compacted through an LDS
// counter (one atomic per wave and 64 objects; their order is immaterial, the
// final selection sorts by score and id).  More than `cap` candidates: the
// `cap` largest upper bounds are kept (radix select) and the query is marked
// uncertified.
__global__ __launch_bounds__(kThreads) void k_bound_candidates_block(
    const float* __restrict__ sim, int64_t ld_s, int64_t n, MetaView meta, SimBound bound,
    const int32_t* __restrict__ cls, int32_t k, int32_t cap, int32_t* __restrict__ cand, int32_t* __restrict__ count,
    int32_t* __restrict__ certified) {
  __shared__ uint32_t hist[256];
  __shared__ uint32_t word[2];
  __shared__ float wv[kThreads / 64];
  __shared__ int32_t wt[kThreads / 64];
  __shared__ int32_t filled;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int32_t qq = blockIdx.x;
  const float* srow = sim + (int64_t)qq * ld_s;
  const int tc = meta.tcls[qq];
  float L = -INFINITY;
  if (n > k) {
    float top[kSmallK];
#pragma unroll
    for (int e = 0; e < kSmallK; ++e) top[e] = -INFINITY;
    for (int64_t i = tid; i < n; i += kThreads) {
      const float v = (1.0f - kW) * sem_bounds(srow, i, tc, cls, bound, qq).lo;
      if (v > top[kSmallK - 1]) {
#pragma unroll
        for (int e = kSmallK - 1; e > 0; --e) top[e] = v > top[e - 1] ? top[e - 1] : fmaxf(v, top[e]);
        top[0] = fmaxf(top[0], v);
      }
    }
    for (int round = 0; round < k; ++round) {
      // largest head in each wave (lowest lane on ties), then across the waves (lowest thread)
      float m = top[0];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
      const uint64_t holders = __ballot(top[0] == m);
      if (lane == 0) {
        wv[w] = m;
        wt[w] = w * 64 + __ffsll((unsigned long long)holders) - 1;
      }
      __syncthreads();
      float bm = wv[0];
      int bt = wt[0];
      for (int i = 1; i < kThreads / 64; ++i)
        if (wv[i] > bm) {
          bm = wv[i];
          bt = wt[i];
        }
      if (tid == bt) {
#pragma unroll
        for (int e = 0; e < kSmallK - 1; ++e) top[e] = top[e + 1];
        top[kSmallK - 1] = -INFINITY;
      }
      L = bm;
      __syncthreads();
    }
  }
  const uint64_t below = (1ull << lane) - 1ull;
  auto compact = [&](float thresh) {
    if (tid == 0) filled = 0;
    __syncthreads();
    for (int64_t base = (int64_t)w * 64; base < n; base += kThreads) {
      const int64_t i = base + lane;
      const bool f = i < n && sem_bounds(srow, i, tc, cls, bound, qq).hi >= thresh;
      const uint64_t mask = __ballot(f);
      if (!mask) continue;
      int32_t first = 0;
      if (lane == 0) first = atomicAdd(&filled, (int32_t)__popcll(mask));
      first = __shfl(first, 0);
      if (f) {
        const int32_t pos = first + __popcll(mask & below);
        if (pos < cap) cand[(int64_t)qq * cap + pos] = (int32_t)i;
      }
    }
    __syncthreads();
    return filled;
  };
  int32_t total = compact(L);
  bool exact = true;
  if (total > cap) {
    auto hi_key = [&](int64_t i) {
      const float h = sem_bounds(srow, i, tc, cls, bound, qq).hi;
      return h >= L ? __float_as_uint(h) : 0u;
    };
    const float thresh = fmaxf(L, __uint_as_float(radix_select_kth(n, cap, hi_key, hist, word)));
    total = compact(thresh);
    exact = false;
  }
  if (tid == 0) {
    count[qq] = total < cap ? total : cap;
    if (certified) certified[qq] = exact ? 1 : 0;
  }
}

// Block-per-query form for K <= kSmallK that reads the row once: the first
// pass keeps each thread's two largest lower bounds (16-byte loads, kCandLoads
// per thread in flight) and every upper bound, rounded up to BF16, in LDS; the
// compaction tests the LDS copy and confirms an object with its exact upper
// bound only where the rounded one reaches the threshold.  The threshold is the
// K-th largest of the threads' kept values: they belong to distinct objects,
// so it never exceeds the K-th largest lower bound over all objects and the
// pruning stays exact; it falls below that only when three of the K largest
// share a thread, which admits a few more candidates.  Same certificate and
// overflow rule as k_bound_candidates_block.
constexpr int kCandThreads = 512;
constexpr int kCandLoads = 4;
constexpr int kCandKeep = 2;
constexpr int kPreCap = 2048;  // objects listed by the LDS test before their exact bounds are read

__device__ inline uint16_t bf16_round_up(float f) {  // f >= 0: the smallest BF16 value >= f
  return (uint16_t)((__float_as_uint(f) + 0xFFFFu) >> 16);
}

__global__ __launch_bounds__(kCandThreads) void k_bound_candidates_lds(
    const float* __restrict__ sim, int64_t ld_s, int64_t n, MetaView meta, SimBound bound,
    const int32_t* __restrict__ cls, int32_t k, int32_t cap, int32_t* __restrict__ cand, int32_t* __restrict__ count,
    int32_t* __restrict__ certified) {
  extern __shared__ uint16_t hup[];  // upper bounds, rounded up to BF16
  __shared__ uint32_t hist[256];
  __shared__ uint32_t word[2];
  __shared__ float wv[kCandThreads / 64];
  __shared__ int32_t wt[kCandThreads / 64];
  __shared__ int32_t filled;
  __shared__ int32_t pre[kPreCap];  // objects whose rounded upper bound reaches the threshold
  __shared__ int32_t pre_n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int32_t qq = blockIdx.x;
  const float* srow = sim + (int64_t)qq * ld_s;
  const int tc = meta.tcls[qq];
  const bool bnd = bound.q_nrm != nullptr;
  const float qn = bnd ? bound.q_nrm[qq] : 0.f;
  const float qe = bnd ? bound.q_err[qq] + bound.acc : 0.f;
  float top[kCandKeep];
#pragma unroll
  for (int e = 0; e < kCandKeep; ++e) top[e] = -INFINITY;
  // lower bound into the kept pair, upper bound into LDS (sem_bounds' arithmetic)
  auto visit = [&](int64_t i, float sv, int32_t cv, float ev) {
    float lo = sv, hi = sv;
    if (bnd) {
      const float kappa = (tc >= 0 && cv >= 0 && cv != tc) ? kClassFactor : 1.0f;
      const float d = kappa * fmaf(qn, ev, qe);
      lo = fmaxf(0.f, sv - d);
      hi = fminf(kappa, sv + d);
    }
    hup[i] = bf16_round_up(hi);
    const float v = (1.0f - kW) * lo;
    top[1] = fmaxf(top[1], fminf(v, top[0]));
    top[0] = fmaxf(top[0], v);
  };
  const int64_t n4 = n >> 2;
  const float4* s4 = reinterpret_cast<const float4*>(srow);
  const float4* e4 = reinterpret_cast<const float4*>(bound.o_err);
  const int4* c4 = reinterpret_cast<const int4*>(cls);
  for (int64_t b = tid; b < n4; b += (int64_t)kCandThreads * kCandLoads) {
    float4 sv[kCandLoads], ev[kCandLoads];
    int4 cv[kCandLoads];
#pragma unroll
    for (int u = 0; u < kCandLoads; ++u) {
      const int64_t i = b + (int64_t)u * kCandThreads;
      sv[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      ev[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      cv[u] = make_int4(-1, -1, -1, -1);
      if (i < n4) {
        sv[u] = s4[i];
        if (bnd) {
          ev[u] = e4[i];
          if (cls) cv[u] = c4[i];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kCandLoads; ++u) {
      const int64_t i = b + (int64_t)u * kCandThreads;
      if (i >= n4) break;
      visit(4 * i, sv[u].x, cv[u].x, ev[u].x);
      visit(4 * i + 1, sv[u].y, cv[u].y, ev[u].y);
      visit(4 * i + 2, sv[u].z, cv[u].z, ev[u].z);
      visit(4 * i + 3, sv[u].w, cv[u].w, ev[u].w);
    }
  }
  for (int64_t i = 4 * n4 + tid; i < n; i += kCandThreads)
    visit(i, srow[i], cls ? cls[i] : -1, bnd ? bound.o_err[i] : 0.f);
  float L = -INFINITY;
  if (n > k) {
    for (int round = 0; round < k; ++round) {
      // largest head in each wave (lowest lane on ties), then across the waves (lowest thread)
      float m = top[0];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
      const uint64_t holders = __ballot(top[0] == m);
      if (lane == 0) {
        wv[w] = m;
        wt[w] = w * 64 + __ffsll((unsigned long long)holders) - 1;
      }
      __syncthreads();
      float bm = wv[0];
      int bt = wt[0];
      for (int i = 1; i < kCandThreads / 64; ++i)
        if (wv[i] > bm) {
          bm = wv[i];
          bt = wt[i];
        }
      if (tid == bt) {
        top[0] = top[1];
        top[1] = -INFINITY;
      }
      L = bm;
      __syncthreads();
    }
  }
  const uint64_t below = (1ull << lane) - 1ull;
  // appends the objects of this wave with f set to the candidate list
  auto append = [&](bool f, int64_t i) {
    const uint64_t mask = __ballot(f);
    if (!mask) return;
    int32_t first = 0;
    if (lane == 0) first = atomicAdd(&filled, (int32_t)__popcll(mask));
    first = __shfl(first, 0);
    if (f) {
      const int32_t pos = first + __popcll(mask & below);
      if (pos < cap) cand[(int64_t)qq * cap + pos] = (int32_t)i;
    }
  };
  // Two steps: the LDS test alone lists the objects whose rounded upper bound
  // reaches the threshold, then their exact bounds are read all at once (no
  // load waits behind a candidate store or behind another object's test).
  auto compact = [&](float thresh) {
    if (tid == 0) {
      filled = 0;
      pre_n = 0;
    }
    __syncthreads();  // also publishes the LDS upper bounds
    for (int64_t base = (int64_t)w * 64; base < n; base += kCandThreads) {
      const int64_t i = base + lane;
      const bool f = i < n && __uint_as_float((uint32_t)hup[i] << 16) >= thresh;
      const uint64_t mask = __ballot(f);
      if (!mask) continue;
      int32_t first = 0;
      if (lane == 0) first = atomicAdd(&pre_n, (int32_t)__popcll(mask));
      first = __shfl(first, 0);
      if (f) {
        const int32_t pos = first + __popcll(mask & below);
        if (pos < kPreCap) pre[pos] = (int32_t)i;
      }
    }
    __syncthreads();
    const int32_t np = pre_n;
    if (np <= kPreCap) {
      for (int32_t base = w * 64; base < np; base += kCandThreads) {
        const int32_t t = base + lane;
        const int64_t i = t < np ? pre[t] : 0;
        append(t < np && sem_bounds(srow, i, tc, cls, bound, qq).hi >= thresh, i);
      }
    } else {
      // more than kPreCap: test and confirm in one sweep
      for (int64_t base = (int64_t)w * 64; base < n; base += kCandThreads) {
        const int64_t i = base + lane;
        bool f = i < n && __uint_as_float((uint32_t)hup[i] << 16) >= thresh;
        if (f) f = sem_bounds(srow, i, tc, cls, bound, qq).hi >= thresh;
        append(f, i);
      }
    }
    __syncthreads();
    return filled;
  };
  int32_t total = compact(L);
  bool exact = true;
  if (total > cap) {
    auto hi_key = [&](int64_t i) {
      const float h = sem_bounds(srow, i, tc, cls, bound, qq).hi;
      return h >= L ? __float_as_uint(h) : 0u;
    };
    const float thresh = fmaxf(L, __uint_as_float(radix_select_kth<kCandThreads>(n, cap, hi_key, hist, word)));
    total = compact(thresh);
    exact = false;
  }
  if (tid == 0) {
    count[qq] = total < cap ? total : cap;
    if (certified) certified[qq] = exact ? 1 : 0;
  }
}

// Dynamic LDS of k_bound_candidates_lds for n objects fits on `device`
// (raises the kernel's limit once as needed).
bool cand_lds_fits(int device, size_t bytes) {
  static int limit[64] = {0};
  static size_t granted[64] = {0};
  static size_t stat = 0;
  if (device < 0 || device >= 64) return false;
  if (limit[device] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) v = -1;
    limit[device] = v > 0 ? v : -1;
  }
  const void* fn = reinterpret_cast<const void*>(&k_bound_candidates_lds);
  if (stat == 0) {
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, fn) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    stat = fa.sharedSizeBytes;
  }
  if (limit[device] < 0 || bytes + stat > (size_t)limit[device]) return false;
  if (bytes > 65536 && bytes > granted[device]) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    granted[device] = bytes;
  }
  return true;
}
}  // namespace

hipError_t launch_bound_candidates(const farm_memory* mem, const float* sim, int64_t ld_s, int32_t q, MetaView meta,
                                   const SimBound& bound, int32_t k, int32_t cap, int32_t* cand, int32_t* count,
                                   int32_t* certified, hipStream_t s) {
  if (q <= 0) return hipSuccess;
  const size_t lds = (size_t)round_up(mem->n, 4) * sizeof(uint16_t);
  if (k <= kSmallK && cand_lds_fits(mem->device, lds)) {
    hipLaunchKernelGGL(k_bound_candidates_lds, dim3((unsigned)q), dim3(kCandThreads), lds, s, sim, ld_s, mem->n, meta,
                       bound, mem->cls, k, cap, cand, count, certified);
  } else if (k <= kSmallK) {
    hipLaunchKernelGGL(k_bound_candidates_block, dim3((unsigned)q), dim3(kThreads), 0, s, sim, ld_s, mem->n, meta,
                       bound, mem->cls, k, cap, cand, count, certified);
  } else {
    hipLaunchKernelGGL(k_bound_candidates, dim3((unsigned)q), dim3(kThreads), 0, s, sim, ld_s, mem->n, meta, bound,
                       mem->cls, k, cap, cand, count, certified);
  }
  return hipGetLastError();
}

}  // namespace farm
