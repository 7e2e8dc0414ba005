// pair.hip -- the relational pass: per-relation max over anchors and the
// soft composite.
//
// For query q with relations r = (p_r, q_r) and the clamped similarities
// a_r(j) = sim(j, q_r) (rows of the similarity matrix):
//   t_r(i) = max_{j != i} a_r(j) * P_{p_r}(c_i, c_j)        (greedy star binding,
//            Appendix "Robust Relational Retrieval Formulation", query-time complexity)
//   s(i)   = s_sem(i) * (0.5 + 0.5 * exp(mean_r log t_r(i)))  (geometric-mean blend,
//            Appendix "Retrieval Details", composite-scoring step)
//
// Arithmetic forms used on the GPU (algebraically equal to the definitions):
//   Near:        log(a_j) - 2 |c_i - c_j|^2 is maximised in the log domain,
//                no transcendental per pair; t = exp(max).
//   Above/Below: P = 1 / (1 + 2^(dz * c)), c = -+(1/tau) log2(e), with
//                dz = z_i - z_j; exp2 and reciprocal on the transcendental unit.
//   Left/Right:  the same sigmoid on the lateral offset dh = h_i - h_j, with h
//                kept as an unevaluated float pair hi + lo (see prep.hip).
// All offsets are formed as differences of coordinates before any scaling,
// so the argument error is relative to the offset, not to the distance from
// the origin.  The geometric mean is formed as exp of the mean of logs, which
// neither overflows nor underflows for R <= 8 relations.
//
// Exhaustive kernel: one block per (512 targets, query); each thread owns two
// targets; anchors stream through LDS in chunks of 512 as (value, coordinates)
// float4 records that every lane reads as a broadcast.  Only the chunk that
// overlaps the block's own targets carries the j != i test.
//
// The scanned predicates (scan_math.h) do not fit the anchor records: Closest
// and Farthest depend on the query's candidate set, Inside on the anchor's
// extents.  k_scan_rows computes their terms first (one wave per target) into
// the relation's row of lsim (as log t), and the exhaustive kernel adds that
// row like a Near term.
#include <math.h>

#include "farm_internal.h"
#include "pair_math.h"
#include "scan_math.h"

namespace farm {
namespace {

constexpr int kThreads = 256;
constexpr int kTpt = 2;                      // targets per thread
constexpr int kTile = kThreads * kTpt;       // targets per block
constexpr int kChunk = 512;                  // anchors per LDS chunk

template <int FAM, bool SELF, bool WITH_ARG>
__device__ inline void scan_chunk(const float4* __restrict__ rec, const uint32_t* __restrict__ rid, int cnt,
                                  int64_t j0, const Tgt* t, const int64_t* ti, float c, float* best,
                                  uint32_t* bid) {
  for (int jj = 0; jj < cnt; ++jj) {
    float4 r = rec[jj];
#pragma unroll
    for (int u = 0; u < kTpt; ++u) {
      float v = pair_value<FAM>(t[u], r, c);
      if (SELF && j0 + jj == ti[u]) v = -INFINITY;
      if (WITH_ARG) {
        if (v >= best[u] && v != -INFINITY) {  // ties are rare: read the id only then
          uint32_t idj = rid[jj];
          if (v > best[u] || idj < bid[u]) {
            best[u] = v;
            bid[u] = idj;
          }
        }
      } else {
        best[u] = fmaxf(best[u], v);
      }
    }
  }
}

template <int FAM, bool WITH_ARG>
__device__ void relation_pass(const float* __restrict__ arow, const float* __restrict__ lrow, int64_t n,
                              int64_t tile0, const int64_t* ti,
                              const Tgt* t, float c, const float* x, const float* y, const float* z,
                              const float* hhi, const float* hlo, const uint32_t* ids, float4* rec,
                              uint32_t* rid, float* best, uint32_t* bid) {
#pragma unroll
  for (int u = 0; u < kTpt; ++u) {
    best[u] = value_floor<FAM>();
    bid[u] = FARM_NO_ID;
  }
  const int64_t tile1 = tile0 + kTile;
  for (int64_t c0 = 0; c0 < n; c0 += kChunk) {
    int cnt = (int)(n - c0 < kChunk ? n - c0 : kChunk);
    __syncthreads();
    for (int jj = threadIdx.x; jj < cnt; jj += kThreads) {
      int64_t j = c0 + jj;
      rec[jj] = anchor_record_pre(FAM, arow[j], FAM == kFamNear ? lrow[j] : 0.f, j, x, y, z, hhi, hlo);
      if (WITH_ARG) rid[jj] = ids[j];
    }
    __syncthreads();
    bool overlap = c0 < tile1 && c0 + cnt > tile0;
    if (overlap)
      scan_chunk<FAM, true, WITH_ARG>(rec, rid, cnt, c0, t, ti, c, best, bid);
    else
      scan_chunk<FAM, false, WITH_ARG>(rec, rid, cnt, c0, t, ti, c, best, bid);
  }
}

// Terms of the scanned predicates (Closest, Farthest, Inside) of every target
// for the relation rows listed in meta.scan_rows: one wave per (target, row); lsim's row gets log t, and the
// term and anchor outputs are written here when requested.
constexpr int kScanWaves = 4;

template <bool GEO>
__global__ __launch_bounds__(64 * kScanWaves) void k_scan_rows(
    const float* __restrict__ sim, float* __restrict__ lsim, int64_t ld_s, int32_t q, MetaView meta,
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const float* __restrict__ ext, const uint32_t* __restrict__ ids, const int32_t* __restrict__ cls,
    const int32_t* __restrict__ cls_order, const int32_t* __restrict__ cls_sorted, int64_t n,
    float* __restrict__ rel_terms,
    uint32_t* __restrict__ rel_anchor_id, BetweenView bv, EntityGeo eg) {
  const int lane = threadIdx.x & 63;
  const int64_t o = (int64_t)blockIdx.x * kScanWaves + (threadIdx.x >> 6);
  if (o >= n) return;  // whole waves leave together
  const int r = meta.scan_rows[blockIdx.y];
  const int qq = meta.rel_query[r];
  if (is_entity_geo(meta.rel_pred[r]) != GEO) return;  // the other instance takes this row
  if (!GEO && meta.rel_pred[r] == FARM_BETWEEN) {  // both slots of the invocation: the term and the two anchors
    float t;
    uint32_t b1, b2;
    between_term_row(bv, x, y, z, ids, r, o, lane, t, b1, b2);
    if (lane == 0) {
      lsim[(int64_t)r * ld_s + o] = logf(t);
      if (rel_terms) {
        rel_terms[(int64_t)r * n + o] = t;
        rel_terms[(int64_t)(r + 1) * n + o] = t;
      }
      if (rel_anchor_id) {
        rel_anchor_id[(int64_t)r * n + o] = b1;
        rel_anchor_id[(int64_t)(r + 1) * n + o] = b2;
      }
    }
    return;
  }
  ScanCtx k{x, y, z, ext, ids, cls, cls_order, cls_sorted, meta.tcls[qq], n, meta.rel_pred[r]};
  k.eg = eg;
  const float* arow = sim + (int64_t)(q + r) * ld_s;
  float best;
  uint32_t bid;
  auto sim_of = [&](int64_t a) { return arow[a]; };  // lower bound, upper bound and value alike
  scan_term_wave<GEO>(k, o, lane, sim_of, sim_of, sim_of, best, bid);
  const float t = best > 0.f ? best : 0.f;
  if (lane == 0) {
    lsim[(int64_t)r * ld_s + o] = logf(t);
    if (rel_terms) rel_terms[(int64_t)r * n + o] = t;
    if (rel_anchor_id) rel_anchor_id[(int64_t)r * n + o] = bid;
  }
}

template <bool WITH_ARG>
__global__ __launch_bounds__(kThreads) void k_pair_exhaustive(
    const float* __restrict__ sim, const float* __restrict__ lsim, int64_t ld_s, int32_t q, MetaView meta,
    SimBound bound, const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ z,
    const float* __restrict__ vz, const float* __restrict__ hhi, const float* __restrict__ hlo,
    const uint32_t* __restrict__ ids, const int32_t* __restrict__ cls, int64_t n, float* __restrict__ scores,
    int64_t ld_out,
    float* __restrict__ rel_terms, uint32_t* __restrict__ rel_anchor_id, float* __restrict__ scores_hi) {
  __shared__ float4 rec[kChunk];
  __shared__ uint32_t rid[WITH_ARG ? kChunk : 1];
  const int32_t qq = blockIdx.y;
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
  int64_t ti[kTpt];
#pragma unroll
  for (int u = 0; u < kTpt; ++u) {
    int64_t i = tile0 + threadIdx.x + u * kThreads;
    ti[u] = i < n ? i : n - 1;  // out-of-range lanes shadow the last target and do not store
  }
  const int r0 = meta.rel_off[qq], r1 = meta.rel_off[qq + 1];
  float lsum[kTpt], lsum_hi[kTpt];
#pragma unroll
  for (int u = 0; u < kTpt; ++u) lsum[u] = lsum_hi[u] = 0.f;
  const bool bounded = bound.q_nrm != nullptr;
  const float err_max = bounded ? *bound.o_err_max : 0.f;

  int R = 0;  // predicate invocations (a Between's second slot is not one)
  for (int r = r0; r < r1; ++r) {
    const int p = meta.rel_pred[r];
    if (p == FARM_AND) continue;  // its term is the Between slot's before it
    ++R;
    const int fam = family_of(p);
    const float c = sigmoid_scale(p);
    const float* arow = sim + (int64_t)(q + r) * ld_s;
    const float* lrow = lsim + (int64_t)r * ld_s;
    // largest similarity error of this relation row (upper-bound output only)
    const float dmax = bounded ? fmaf(bound.q_nrm[q + r], err_max, bound.q_err[q + r] + bound.acc) : 0.f;
    if (is_scanned(p)) {  // log t from k_scan_rows, which also wrote the term and anchor outputs
#pragma unroll
      for (int u = 0; u < kTpt; ++u) {
        const float l = lrow[ti[u]];
        lsum[u] += l;
        if (bounded) lsum_hi[u] += logf(fminf(1.0f, expf(l) * (1.0f + 1e-6f) + dmax));
      }
      continue;
    }
    // InFrontOf/Behind measure along the viewing direction: the depth pair follows the lateral one
    const float* rhi = hhi + (is_depth(p) ? n : 0);
    const float* rlo = hlo + (is_depth(p) ? n : 0);
    const ZPair zp = z_for(p, z, vz, n);  // On: the target's bottom and the anchors' top faces
    Tgt t[kTpt];
#pragma unroll
    for (int u = 0; u < kTpt; ++u) t[u] = load_target(fam, ti[u], x, y, zp.tgt, rhi, rlo);
    float best[kTpt];
    uint32_t bid[kTpt];
    float term[kTpt];
    if (fam == kFamNear) {
      relation_pass<kFamNear, WITH_ARG>(arow, lrow, n, tile0, ti, t, c, x, y, zp.anc, rhi, rlo, ids, rec, rid, best,
                                        bid);
#pragma unroll
      for (int u = 0; u < kTpt; ++u) {
        term[u] = term_of<kFamNear>(best[u]);
        lsum[u] += best[u];  // already log t
      }
    } else {
      if (fam == kFamVert)
        relation_pass<kFamVert, WITH_ARG>(arow, lrow, n, tile0, ti, t, c, x, y, z, rhi, rlo, ids, rec, rid, best, bid);
      else
        relation_pass<kFamLat, WITH_ARG>(arow, lrow, n, tile0, ti, t, c, x, y, z, rhi, rlo, ids, rec, rid, best, bid);
#pragma unroll
      for (int u = 0; u < kTpt; ++u) {
        term[u] = term_of<kFamVert>(best[u]);
        lsum[u] += logf(term[u]);
      }
    }
    if (bounded) {
#pragma unroll
      for (int u = 0; u < kTpt; ++u) lsum_hi[u] += logf(fminf(1.0f, term[u] + dmax));
    }
#pragma unroll
    for (int u = 0; u < kTpt; ++u) {
      int64_t i = tile0 + threadIdx.x + u * kThreads;
      if (i < n) {
        if (rel_terms) rel_terms[(int64_t)r * n + i] = term[u];
        if (WITH_ARG && rel_anchor_id) rel_anchor_id[(int64_t)r * n + i] = bid[u];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kTpt; ++u) {
    int64_t i = tile0 + threadIdx.x + u * kThreads;
    if (i < n) {
      const float sem = sim[(int64_t)qq * ld_s + i];
      const float g = R > 0 ? expf(lsum[u] / (float)R) : 1.0f;
      scores[(int64_t)qq * ld_out + i] = sem * ((1.0f - kW) + kW * g);
      if (bounded) {  // s_hi: upper bounds of kappa * sim(i, q_t) and of every term
        const int tc = meta.tcls[qq];
        const float kappa = (tc >= 0 && cls && cls[i] >= 0 && cls[i] != tc) ? kClassFactor : 1.0f;
        const float sem_hi =
            fminf(kappa, sem + kappa * fmaf(bound.q_nrm[qq], bound.o_err[i], bound.q_err[qq] + bound.acc));
        const float g_hi = R > 0 ? expf(lsum_hi[u] / (float)R) : 1.0f;
        scores_hi[(int64_t)qq * ld_out + i] = sem_hi * ((1.0f - kW) + kW * g_hi) * (1.0f + 1e-6f);
      }
    }
  }
}

// ---------------------------------------------------------------- explain
// One block per (query, rank): recompute every relation's term and bound
// anchor for the selected object with the same per-pair arithmetic as the
// pass above (identical values), reducing (value, id) across the block.
template <int FAM>
__device__ void explain_relation(const float* __restrict__ arow, int64_t n, int64_t i, float c, const float* x,
                                 const float* y, ZPair zp, const float* hhi, const float* hlo,
                                 const uint32_t* ids, float* red_v, uint32_t* red_id, float& out_t,
                                 uint32_t& out_b) {
  Tgt t = load_target(FAM, i, x, y, zp.tgt, hhi, hlo);
  float best = value_floor<FAM>();
  uint32_t bid = FARM_NO_ID;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    if (j == i) continue;
    float4 r = anchor_record(FAM, arow[j], j, x, y, zp.anc, hhi, hlo);
    float v = pair_value<FAM>(t, r, c);
    if (v >= best && v != -INFINITY) {
      uint32_t idj = ids[j];
      if (v > best || idj < bid) {
        best = v;
        bid = idj;
      }
    }
  }
  red_v[threadIdx.x] = best;
  red_id[threadIdx.x] = bid;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      float v2 = red_v[threadIdx.x + w];
      uint32_t b2 = red_id[threadIdx.x + w];
      float v1 = red_v[threadIdx.x];
      uint32_t b1 = red_id[threadIdx.x];
      if (v2 > v1 || (v2 == v1 && b2 < b1)) {
        red_v[threadIdx.x] = v2;
        red_id[threadIdx.x] = b2;
      }
    }
    __syncthreads();
  }
  out_t = term_of<FAM>(red_v[0]);
  out_b = red_id[0];
  __syncthreads();
}

template <bool GEO>
__global__ __launch_bounds__(256) void k_explain(const float* __restrict__ sim, int64_t ld_s, int32_t q,
                                                 MetaView meta, const int32_t* __restrict__ idx, int32_t k,
                                                 const float* __restrict__ x, const float* __restrict__ y,
                                                 const float* __restrict__ z, const float* __restrict__ vz,
                                                 const float* __restrict__ hhi,
                                                 const float* __restrict__ hlo, const uint32_t* __restrict__ ids,
                                                 const float* __restrict__ ext, const int32_t* __restrict__ cls,
                                                 const int32_t* __restrict__ cls_order,
                                                 const int32_t* __restrict__ cls_sorted,
                                                 int64_t n, float* __restrict__ out_terms,
                                                 uint32_t* __restrict__ out_anchor_id, BetweenView bv, EntityGeo eg) {
  __shared__ float red_v[256];
  __shared__ uint32_t red_id[256];
  const int32_t qq = blockIdx.y, kk = blockIdx.x;
  const int64_t slot = (int64_t)qq * k + kk;
  const int32_t i = idx[slot];
  const int r0 = meta.rel_off[qq], r1 = meta.rel_off[qq + 1];
  for (int e = 0; e < kMaxRel; ++e) {
    float tv = 0.f;
    uint32_t b = FARM_NO_ID;
    // the entity-geometry slots belong to the GEO instance (launched after this one), the rest to the other
    const bool geo_slot = e < r1 - r0 && is_entity_geo(meta.rel_pred[r0 + e]);
    if (geo_slot != GEO) continue;
    if (i >= 0 && e < r1 - r0) {
      const int r = r0 + e;
      const int p = meta.rel_pred[r];
      const float* arow = sim + (int64_t)(q + r) * ld_s;
      const float c = sigmoid_scale(p);
      const float* rhi = hhi + (is_depth(p) ? n : 0);  // depth pair of InFrontOf/Behind
      const float* rlo = hlo + (is_depth(p) ? n : 0);
      const ZPair zp = z_for(p, z, vz, n);  // On: bottom/top faces
      if (GEO) {
        ScanCtx rk{x, y, z, ext, ids, cls, cls_order, cls_sorted, meta.tcls[qq], n, p};
        rk.eg = eg;
        float bv;
        auto sim_of = [&](int64_t a) { return arow[a]; };
        scan_term_wave<true>(rk, i, (int)(threadIdx.x & 63), sim_of, sim_of, sim_of, bv, b);
        tv = bv > 0.f ? bv : 0.f;
      } else if (p == FARM_BETWEEN || p == FARM_AND) {
        // the invocation's term from its first slot; the first slot binds a1, the second a2
        const int rb = p == FARM_BETWEEN ? r : r - 1;
        float bt;
        uint32_t b1, b2;
        between_term_row(bv, x, y, z, ids, rb, i, (int)(threadIdx.x & 63), bt, b1, b2);
        tv = bt;
        b = p == FARM_BETWEEN ? b1 : b2;
      } else if (is_scanned(p)) {
        // every wave takes the same term (identical arithmetic); thread 0 stores it
        ScanCtx rk{x, y, z, ext, ids, cls, cls_order, cls_sorted, meta.tcls[qq], n, p};
        rk.eg = eg;
        float bv;
        auto sim_of = [&](int64_t a) { return arow[a]; };
        scan_term_wave<false>(rk, i, (int)(threadIdx.x & 63), sim_of, sim_of, sim_of, bv, b);
        tv = bv > 0.f ? bv : 0.f;
      } else if (!GEO)
      switch (family_of(p)) {
        case kFamNear: explain_relation<kFamNear>(arow, n, i, c, x, y, zp, rhi, rlo, ids, red_v, red_id, tv, b); break;
        case kFamVert: explain_relation<kFamVert>(arow, n, i, c, x, y, zp, rhi, rlo, ids, red_v, red_id, tv, b); break;
        default: explain_relation<kFamLat>(arow, n, i, c, x, y, zp, rhi, rlo, ids, red_v, red_id, tv, b); break;
      }
    }
    if (threadIdx.x == 0) {
      if (out_terms) out_terms[slot * kMaxRel + e] = tv;
      if (out_anchor_id) out_anchor_id[slot * kMaxRel + e] = b;
    }
  }
}

// Between's candidate sets: for every relation row of a Between invocation,
// the kBetweenSet anchors of largest similarity (ties by the smaller id) and
// their similarities, by repeated block-wide selection of the next anchor in
// (similarity desc, id asc) order -- one 256-thread block per row.
__global__ __launch_bounds__(256) void k_between_sets(const float* __restrict__ sim, int64_t ld_s, int32_t q,
                                                      MetaView meta, const uint32_t* __restrict__ ids, int64_t n,
                                                      int32_t* __restrict__ bidx, float* __restrict__ bsim,
                                                      int32_t* __restrict__ bcnt) {
  __shared__ float rv[256];
  __shared__ uint32_t rid[256];
  __shared__ int32_t rj[256];
  const int r = blockIdx.x;
  const int p = meta.rel_pred[r];
  if (p != FARM_BETWEEN && p != FARM_AND) return;
  const float* row = sim + (int64_t)(q + r) * ld_s;
  const int k = (int)(n < kBetweenSet ? n : kBetweenSet);
  float pv = INFINITY;
  uint32_t pid = 0;
  for (int round = 0; round < k; ++round) {
    float bv = -INFINITY;
    uint32_t bi = FARM_NO_ID;
    int32_t bj = -1;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
      const float v = row[j];
      const uint32_t id = ids[j];
      const bool after = v < pv || (v == pv && id > pid);  // comes after the last one taken
      if (after && (v > bv || (v == bv && id < bi))) {
        bv = v;
        bi = id;
        bj = (int32_t)j;
      }
    }
    rv[threadIdx.x] = bv;
    rid[threadIdx.x] = bi;
    rj[threadIdx.x] = bj;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        const float v2 = rv[threadIdx.x + w];
        const uint32_t i2 = rid[threadIdx.x + w];
        if (v2 > rv[threadIdx.x] || (v2 == rv[threadIdx.x] && i2 < rid[threadIdx.x])) {
          rv[threadIdx.x] = v2;
          rid[threadIdx.x] = i2;
          rj[threadIdx.x] = rj[threadIdx.x + w];
        }
      }
      __syncthreads();
    }
    pv = rv[0];
    pid = rid[0];
    if (threadIdx.x == 0) {
      bidx[(int64_t)r * kBetweenSet + round] = rj[0];
      bsim[(int64_t)r * kBetweenSet + round] = pv;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) bcnt[r] = k;
}

__global__ void k_log_rows(const float* __restrict__ sim, int64_t ld_s, int64_t rows, int64_t n,
                           float* __restrict__ lsim) {
  const int64_t r = blockIdx.y;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
    lsim[r * ld_s + j] = near_log(sim[r * ld_s + j]);
}

}  // namespace

hipError_t launch_between_sets(const farm_memory* mem, const float* sim, int64_t ld_s, int32_t q, MetaView meta,
                               int32_t R, int32_t* bidx, float* bsim, int32_t* bcnt, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_between_sets, dim3((unsigned)R), dim3(256), 0, s, sim, ld_s, q, meta, mem->id, mem->n, bidx,
                     bsim, bcnt);
  return hipGetLastError();
}

hipError_t launch_log_rows(const float* sim, int64_t ld_s, int64_t rows, int64_t n, float* lsim, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const unsigned gx = (unsigned)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64);
  hipLaunchKernelGGL(k_log_rows, dim3(gx, (unsigned)rows), dim3(256), 0, s, sim, ld_s, rows, n, lsim);
  return hipGetLastError();
}

hipError_t launch_pair_exhaustive(const farm_memory* mem, const farm_workspace* ws, const float* sim, const float* lsim,
                                  int64_t ld_s, int32_t q, MetaView meta, const SimBound& bound, float* scores,
                                  int64_t ld_out, float* rel_terms, uint32_t* rel_anchor_id, float* scores_hi,
                                  hipStream_t s) {
  if (q <= 0) return hipSuccess;
  int64_t n = mem->n;
  if (meta.scan_n > 0) {
    const BetweenView bv{ws->btw_idx, ws->btw_sim, ws->btw_cnt};
    // two instances: the entity-geometry rows (FP64) and the others; each skips the other's rows
    const dim3 grid((unsigned)((n + kScanWaves - 1) / kScanWaves), (unsigned)meta.scan_n);
    if (meta.scan_n > meta.geo_n) {
      hipLaunchKernelGGL(k_scan_rows<false>, grid, dim3(64 * kScanWaves), 0, s, sim, const_cast<float*>(lsim), ld_s, q,
                         meta, mem->x, mem->y, mem->z, mem->ext, mem->id, mem->cls, mem->cls_order, mem->cls_sorted,
                         n, rel_terms, rel_anchor_id, bv, entity_geo(mem));
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (meta.geo_n > 0) {
      hipLaunchKernelGGL(k_scan_rows<true>, grid, dim3(64 * kScanWaves), 0, s, sim, const_cast<float*>(lsim), ld_s, q,
                         meta, mem->x, mem->y, mem->z, mem->ext, mem->id, mem->cls, mem->cls_order, mem->cls_sorted,
                         n, rel_terms, rel_anchor_id, bv, entity_geo(mem));
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  dim3 grid((unsigned)((n + kTile - 1) / kTile), (unsigned)q);
  if (rel_anchor_id)
    hipLaunchKernelGGL(k_pair_exhaustive<true>, grid, dim3(kThreads), 0, s, sim, lsim, ld_s, q, meta, bound, mem->x,
                       mem->y, mem->z, mem->vz, mem->hr_hi, mem->hr_lo, mem->id, mem->cls, n, scores, ld_out,
                       rel_terms, rel_anchor_id, scores_hi);
  else
    hipLaunchKernelGGL(k_pair_exhaustive<false>, grid, dim3(kThreads), 0, s, sim, lsim, ld_s, q, meta, bound, mem->x,
                       mem->y, mem->z, mem->vz, mem->hr_hi, mem->hr_lo, mem->id, mem->cls, n, scores, ld_out,
                       rel_terms, rel_anchor_id, scores_hi);
  return hipGetLastError();
}

hipError_t launch_explain(const farm_memory* mem, const farm_workspace* ws, const float* sim, int64_t ld_s, int32_t q,
                          MetaView meta, const int32_t* idx, int32_t k, float* out_terms, uint32_t* out_anchor_id,
                          hipStream_t s) {
  if (q <= 0 || k <= 0 || (!out_terms && !out_anchor_id)) return hipSuccess;
  dim3 grid((unsigned)k, (unsigned)q);
  const BetweenView bv{ws->btw_idx, ws->btw_sim, ws->btw_cnt};
  hipLaunchKernelGGL(k_explain<false>, grid, dim3(256), 0, s, sim, ld_s, q, meta, idx, k, mem->x, mem->y, mem->z,
                     mem->vz, mem->hr_hi, mem->hr_lo, mem->id, mem->ext, mem->cls, mem->cls_order, mem->cls_sorted,
                     mem->n, out_terms, out_anchor_id, bv, entity_geo(mem));
  if (meta.geo_n > 0) {  // the entity-geometry slots
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_explain<true>, grid, dim3(256), 0, s, sim, ld_s, q, meta, idx, k, mem->x, mem->y, mem->z,
                       mem->vz, mem->hr_hi, mem->hr_lo, mem->id, mem->ext, mem->cls, mem->cls_order, mem->cls_sorted,
                       mem->n, out_terms, out_anchor_id, bv, entity_geo(mem));
  }
  return hipGetLastError();
}

}  // namespace farm
