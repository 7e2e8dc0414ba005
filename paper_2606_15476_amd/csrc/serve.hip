// serve.hip -- request loop over resident scenes: continuous batching,
// admission by an HBM budget, one stream per slot.
//
// A request is one parsed query (target vector, class, R relations) against
// one resident scene; its answer is the scene's TopK (farm_query_topk).  The
// loop is driven by the caller (farm_server_progress): it reaps the slots
// whose batch has finished on the device, then admits new batches into free
// slots.  A batch holds pending requests of one scene in arrival order, up to
// the slot's query and relation capacity.  Its workspace comes from a pool:
// an idle workspace of that scene is reused, otherwise a new one is created
// when the pool's bytes (farm_workspace_estimate) stay within the budget,
// otherwise idle workspaces of other scenes are released first; if nothing
// fits the batch waits (the requests stay pending -- deferral, never failure).
// Batches of different scenes run concurrently on the slots' streams.
//
// Every request's result is independent of the batch it rides in: each query
// row is normalised, quantised and scored on its own, and the similarity
// GEMM's accumulation order for a row does not depend on the other rows.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <new>
#include <unordered_map>
#include <vector>

#include "farm_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t id = 0;
  int32_t scene = 0;
  int32_t target_cls = -1;
  std::vector<float> target;     // [d]
  std::vector<int32_t> preds;    // [R]
  std::vector<float> anchors;    // [R][d]
  int64_t submit_ns = 0;
  bool cancelled = false;
};

struct Done {
  uint64_t id;
  int32_t status;  // 0 ok, 1 cancelled
  int32_t certified;
  int64_t submit_ns, done_ns;
  std::vector<uint32_t> ids;
  std::vector<float> scores;
};

struct PooledWs {
  farm_workspace* ws = nullptr;
  int32_t scene = -1;
  size_t bytes = 0;
  bool busy = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  int pool_index = -1;
  int32_t scene = -1;
  std::vector<Request> batch;
  // pinned host staging
  float* h_target = nullptr;     // [max_q][d]
  float* h_anchor = nullptr;     // [max_rel][d]
  uint32_t* h_ids = nullptr;     // [max_q][k]
  float* h_scores = nullptr;     // [max_q][k]
  int32_t* h_cert = nullptr;     // [max_q]
  // device buffers
  float* d_target = nullptr;
  float* d_anchor = nullptr;
  uint32_t* d_ids = nullptr;
  float* d_scores = nullptr;
  int32_t* d_cert = nullptr;
  // host metadata of the batch
  std::vector<int32_t> cls, rel_off, rel_pred;
};

}  // namespace

struct farm_server {
  farm_server_config cfg{};
  int device = 0;
  int32_t d = 0;
  std::vector<const farm_memory*> scenes;
  std::deque<Request> pending;
  std::vector<Slot> slots;
  std::vector<PooledWs> pool;
  size_t pool_bytes = 0;
  std::deque<Done> done;
  uint64_t next_id = 1;
  std::unordered_map<uint64_t, int> in_flight;  // request id -> slot
  int64_t batches = 0, deferrals = 0, evictions = 0;
};

using namespace farm;

namespace {

void release_slot_buffers(Slot& s) {
  if (s.h_target) (void)hipHostFree(s.h_target);
  if (s.h_anchor) (void)hipHostFree(s.h_anchor);
  if (s.h_ids) (void)hipHostFree(s.h_ids);
  if (s.h_scores) (void)hipHostFree(s.h_scores);
  if (s.h_cert) (void)hipHostFree(s.h_cert);
  for (void* p : {(void*)s.d_target, (void*)s.d_anchor, (void*)s.d_ids, (void*)s.d_scores, (void*)s.d_cert})
    if (p) (void)hipFree(p);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot{};
}

farm_status alloc_slot(Slot& s, const farm_server_config& c, int32_t d) {
  const size_t q = (size_t)c.max_batch_q, r = (size_t)(c.max_batch_rel > 0 ? c.max_batch_rel : 1), k = (size_t)c.k;
  hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_target, q * d * sizeof(float), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_anchor, r * d * sizeof(float), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_ids, q * k * sizeof(uint32_t), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_scores, q * k * sizeof(float), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_cert, q * sizeof(int32_t), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void**)&s.d_target, q * d * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&s.d_anchor, r * d * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&s.d_ids, q * k * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc((void**)&s.d_scores, q * k * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&s.d_cert, q * sizeof(int32_t));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_slot_buffers(s);
    set_error("allocating a serving slot failed");
    return e == hipErrorOutOfMemory ? FARM_ERR_OOM : FARM_ERR_HIP;
  }
  return FARM_OK;
}

// A workspace of `scene` for one batch: reuse, create within the budget, or
// release idle ones of other scenes.  -1 = defer.  Pool entries keep their
// index for life (slots refer to them); a released entry is reused.
int acquire_workspace(farm_server* sv, int32_t scene) {
  for (size_t i = 0; i < sv->pool.size(); ++i)
    if (sv->pool[i].ws && !sv->pool[i].busy && sv->pool[i].scene == scene) return (int)i;
  size_t need = 0;
  const int32_t rel = sv->cfg.max_batch_rel;
  if (farm_workspace_estimate(sv->scenes[scene], sv->cfg.max_batch_q, rel, sv->cfg.k, &need) != FARM_OK) return -1;
  if (need > sv->cfg.hbm_budget) return -1;
  while (sv->pool_bytes + need > sv->cfg.hbm_budget) {
    int victim = -1;
    for (size_t i = 0; i < sv->pool.size(); ++i)
      if (sv->pool[i].ws && !sv->pool[i].busy) { victim = (int)i; break; }
    if (victim < 0) return -1;
    (void)farm_workspace_free(sv->pool[victim].ws);
    sv->pool_bytes -= sv->pool[victim].bytes;
    sv->pool[victim] = PooledWs{};
    ++sv->evictions;
  }
  farm_workspace* ws = nullptr;
  if (farm_workspace_create(sv->scenes[scene], sv->cfg.max_batch_q, rel, sv->cfg.k, &ws) != FARM_OK) return -1;
  int slot = -1;
  for (size_t i = 0; i < sv->pool.size() && slot < 0; ++i)
    if (!sv->pool[i].ws) slot = (int)i;
  if (slot < 0) {
    sv->pool.emplace_back();
    slot = (int)sv->pool.size() - 1;
  }
  sv->pool[slot].ws = ws;
  sv->pool[slot].scene = scene;
  sv->pool[slot].bytes = need;
  sv->pool[slot].busy = false;
  sv->pool_bytes += need;
  return slot;
}

// Launch the next batch into slot `si`.  Returns 1 when launched, 0 when nothing to do or deferred.
int launch_batch(farm_server* sv, int si, farm_status* err) {
  *err = FARM_OK;
  while (!sv->pending.empty() && sv->pending.front().cancelled) {
    const Request& r = sv->pending.front();
    sv->done.push_back(Done{r.id, 1, 0, r.submit_ns, now_ns(), {}, {}});
    sv->pending.pop_front();
  }
  if (sv->pending.empty()) return 0;
  // the scene of the oldest pending request that can get a workspace now
  int32_t scene = -1;
  int pi = -1;
  std::vector<int32_t> tried;
  for (const Request& r : sv->pending) {
    if (r.cancelled || std::find(tried.begin(), tried.end(), r.scene) != tried.end()) continue;
    tried.push_back(r.scene);
    pi = acquire_workspace(sv, r.scene);
    if (pi >= 0) {
      scene = r.scene;
      break;
    }
  }
  if (pi < 0) {
    ++sv->deferrals;
    return 0;
  }
  Slot& s = sv->slots[si];
  s.batch.clear();
  s.cls.clear();
  s.rel_off.assign(1, 0);
  s.rel_pred.clear();
  const int32_t d = sv->d;
  int32_t rel = 0;
  for (auto it = sv->pending.begin(); it != sv->pending.end() && (int32_t)s.batch.size() < sv->cfg.max_batch_q;) {
    if (it->scene != scene || it->cancelled) { ++it; continue; }
    const int32_t R = (int32_t)it->preds.size();
    if (rel + R > sv->cfg.max_batch_rel) break;  // keep arrival order within the scene
    const size_t qi = s.batch.size();
    memcpy(s.h_target + qi * d, it->target.data(), sizeof(float) * d);
    if (R) memcpy(s.h_anchor + (size_t)rel * d, it->anchors.data(), sizeof(float) * (size_t)R * d);
    s.cls.push_back(it->target_cls);
    for (int32_t p : it->preds) s.rel_pred.push_back(p);
    rel += R;
    s.rel_off.push_back(rel);
    s.batch.push_back(std::move(*it));
    it = sv->pending.erase(it);
  }
  const int32_t q = (int32_t)s.batch.size();
  PooledWs& pw = sv->pool[pi];
  pw.busy = true;
  s.pool_index = pi;
  s.scene = scene;
  s.busy = true;
  for (const Request& r : s.batch) sv->in_flight[r.id] = si;
  const farm_memory* mem = sv->scenes[scene];
  auto fail = [&](farm_status st) {
    *err = st;
    (void)hipStreamSynchronize(s.stream);
    return 1;
  };
  if (hipMemcpyAsync(s.d_target, s.h_target, sizeof(float) * q * d, hipMemcpyHostToDevice, s.stream) != hipSuccess)
    return fail(FARM_ERR_HIP);
  if (rel && hipMemcpyAsync(s.d_anchor, s.h_anchor, sizeof(float) * (size_t)rel * d, hipMemcpyHostToDevice,
                            s.stream) != hipSuccess)
    return fail(FARM_ERR_HIP);
  farm_score_opts o{};
  o.dtype = sv->cfg.dtype;
  o.method = sv->cfg.method;
  o.rescore_mult = 4;
  o.certified = s.d_cert;
  farm_status st = farm_query_topk(mem, pw.ws, q, d, s.d_target, s.cls.data(), s.rel_off.data(), s.rel_pred.data(),
                                   rel ? s.d_anchor : nullptr, &o, sv->cfg.k, s.d_ids, s.d_scores, nullptr, nullptr,
                                   s.stream);
  if (st != FARM_OK) return fail(st);
  const size_t k = (size_t)sv->cfg.k;
  if (hipMemcpyAsync(s.h_ids, s.d_ids, sizeof(uint32_t) * q * k, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
      hipMemcpyAsync(s.h_scores, s.d_scores, sizeof(float) * q * k, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
      hipMemcpyAsync(s.h_cert, s.d_cert, sizeof(int32_t) * q, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
      hipEventRecord(s.done, s.stream) != hipSuccess)
    return fail(FARM_ERR_HIP);
  ++sv->batches;
  return 1;
}

void finish_slot(farm_server* sv, Slot& s, int32_t status_all) {
  const int64_t t = now_ns();
  const size_t k = (size_t)sv->cfg.k;
  for (size_t qi = 0; qi < s.batch.size(); ++qi) {
    Request& r = s.batch[qi];
    sv->in_flight.erase(r.id);
    Done dn{r.id, r.cancelled ? 1 : status_all, 0, r.submit_ns, t, {}, {}};
    if (dn.status == 0) {
      dn.certified = s.h_cert[qi];
      dn.ids.assign(s.h_ids + qi * k, s.h_ids + (qi + 1) * k);
      dn.scores.assign(s.h_scores + qi * k, s.h_scores + (qi + 1) * k);
    }
    sv->done.push_back(std::move(dn));
  }
  s.batch.clear();
  if (s.pool_index >= 0) sv->pool[s.pool_index].busy = false;
  s.pool_index = -1;
  s.busy = false;
}

}  // namespace

extern "C" {

farm_status farm_server_create(const farm_server_config* cfg, farm_server** out) {
  try {
    if (!cfg || !out) { set_error("null config or out"); return FARM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (cfg->slots < 1 || cfg->slots > 64 || cfg->max_batch_q < 1 || cfg->max_batch_rel < 0 ||
        cfg->max_batch_rel > (int64_t)cfg->max_batch_q * FARM_MAX_REL || cfg->k < 1 || cfg->k > FARM_MAX_K) {
      set_error("invalid server configuration");
      return FARM_ERR_INVALID_ARG;
    }
    auto* sv = new (std::nothrow) farm_server();
    if (!sv) { set_error("host allocation failed"); return FARM_ERR_OOM; }
    sv->cfg = *cfg;
    if (hipGetDevice(&sv->device) != hipSuccess) { delete sv; set_error("no device"); return FARM_ERR_HIP; }
    *out = sv;
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_server_create");
    return FARM_ERR_OOM;
  }
}

farm_status farm_server_add_scene(farm_server* sv, const farm_memory* mem, int32_t* scene_out) {
  try {
    if (!sv || !mem || !scene_out) { set_error("null argument"); return FARM_ERR_INVALID_ARG; }
    if (mem->device != sv->device) { set_error("scene lives on another device"); return FARM_ERR_INVALID_ARG; }
    if (sv->d && mem->d != sv->d) { set_error("scene width %d differs from the server's %d", mem->d, sv->d); return FARM_ERR_INVALID_ARG; }
    if ((sv->cfg.dtype == FARM_BF16 && !mem->dn_bf16) || (sv->cfg.dtype == FARM_FP8_E4M3 && !mem->dn_fp8)) {
      set_error("scene lacks the server dtype's descriptor copy");
      return FARM_ERR_UNSUPPORTED;
    }
    if (sv->cfg.method == FARM_METHOD_PROPOSAL && mem->prop_m == 0 && mem->n >= 2) {
      set_error("scene has no proposal tables");
      return FARM_ERR_UNSUPPORTED;
    }
    DeviceGuard g(sv->device);
    if (sv->slots.empty()) {
      sv->d = mem->d;
      sv->slots.resize(sv->cfg.slots);
      for (Slot& s : sv->slots) {
        farm_status st = alloc_slot(s, sv->cfg, sv->d);
        if (st != FARM_OK) {
          for (Slot& t : sv->slots) release_slot_buffers(t);
          sv->slots.clear();
          sv->d = 0;
          return st;
        }
      }
    }
    sv->scenes.push_back(mem);
    mem->users.fetch_add(1, std::memory_order_acq_rel);
    *scene_out = (int32_t)sv->scenes.size() - 1;
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_server_add_scene");
    return FARM_ERR_OOM;
  }
}

farm_status farm_server_submit(farm_server* sv, int32_t scene, int32_t d, const float* target, int32_t target_cls,
                               int32_t r, const int32_t* preds, const float* anchors, uint64_t* request_id) {
  try {
    if (!sv || !target || !request_id || (r > 0 && (!preds || !anchors))) {
      set_error("null argument");
      return FARM_ERR_INVALID_ARG;
    }
    if (scene < 0 || scene >= (int32_t)sv->scenes.size()) { set_error("unknown scene %d", scene); return FARM_ERR_INVALID_ARG; }
    if (d != sv->d) { set_error("request width %d != %d", d, sv->d); return FARM_ERR_INVALID_ARG; }
    if (r < 0 || r > FARM_MAX_REL || r > sv->cfg.max_batch_rel) { set_error("R = %d out of range", r); return FARM_ERR_INVALID_ARG; }
    double n2 = 0.0;
    for (int32_t i = 0; i < d; ++i) {
      if (!std::isfinite(target[i])) { set_error("non-finite target"); return FARM_ERR_INVALID_ARG; }
      n2 += (double)target[i] * target[i];
    }
    if (n2 == 0.0) { set_error("zero-norm target"); return FARM_ERR_INVALID_ARG; }
    for (int32_t e = 0; e < r; ++e) {
      if (preds[e] < 0 || preds[e] >= FARM_NUM_PRED) { set_error("bad predicate %d", preds[e]); return FARM_ERR_INVALID_ARG; }
      if ((preds[e] == FARM_BETWEEN && (e + 1 >= r || preds[e + 1] != FARM_AND)) ||
          (preds[e] == FARM_AND && (e == 0 || preds[e - 1] != FARM_BETWEEN))) {
        set_error("FARM_BETWEEN must be followed by FARM_AND (relation %d)", e);
        return FARM_ERR_INVALID_ARG;
      }
      const farm_memory* m = sv->scenes[scene];
      if ((preds[e] == FARM_NEAR_HELLINGER && !m->cov) ||
          (preds[e] >= FARM_LEFT_OF_VIEW && preds[e] <= FARM_BEHIND_VIEW && !m->view)) {
        set_error("predicate %d needs the scene's entity Gaussians / stored views (relation %d)", preds[e], e);
        return FARM_ERR_UNSUPPORTED;
      }
      double a2 = 0.0;
      for (int32_t i = 0; i < d; ++i) {
        const float v = anchors[(size_t)e * d + i];
        if (!std::isfinite(v)) { set_error("non-finite anchor"); return FARM_ERR_INVALID_ARG; }
        a2 += (double)v * v;
      }
      if (a2 == 0.0) { set_error("zero-norm anchor"); return FARM_ERR_INVALID_ARG; }
    }
    Request q;
    q.id = sv->next_id++;
    q.scene = scene;
    q.target_cls = target_cls;
    q.target.assign(target, target + d);
    q.preds.assign(preds, preds + r);
    if (r) q.anchors.assign(anchors, anchors + (size_t)r * d);
    q.submit_ns = now_ns();
    *request_id = q.id;
    sv->pending.push_back(std::move(q));
    return FARM_OK;
  } catch (...) {
    set_error("unexpected host exception in farm_server_submit");
    return FARM_ERR_OOM;
  }
}

farm_status farm_server_cancel(farm_server* sv, uint64_t id) {
  if (!sv) { set_error("null server"); return FARM_ERR_INVALID_ARG; }
  for (Request& r : sv->pending)
    if (r.id == id) { r.cancelled = true; return FARM_OK; }
  auto it = sv->in_flight.find(id);
  if (it != sv->in_flight.end()) {
    for (Request& r : sv->slots[it->second].batch)
      if (r.id == id) r.cancelled = true;
    return FARM_OK;
  }
  set_error("request %llu is not pending or in flight", (unsigned long long)id);
  return FARM_ERR_INVALID_ARG;
}

farm_status farm_server_progress(farm_server* sv, int32_t* busy_slots, int32_t* pending) {
  try {
    if (!sv) { set_error("null server"); return FARM_ERR_INVALID_ARG; }
    DeviceGuard g(sv->device);
    farm_status first_err = FARM_OK;
    for (Slot& s : sv->slots) {
      if (!s.busy) continue;
      const hipError_t e = hipEventQuery(s.done);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) {
        (void)hipGetLastError();
        finish_slot(sv, s, 2);
        if (first_err == FARM_OK) first_err = hip_fail(e, "serving batch");
        continue;
      }
      finish_slot(sv, s, 0);
    }
    for (size_t i = 0; i < sv->slots.size(); ++i) {
      if (sv->slots[i].busy) continue;
      farm_status err;
      const int launched = launch_batch(sv, (int)i, &err);
      if (err != FARM_OK) {
        finish_slot(sv, sv->slots[i], 2);
        if (first_err == FARM_OK) first_err = err;
        continue;
      }
      if (!launched) break;  // nothing admissible now
    }
    if (busy_slots) {
      int32_t b = 0;
      for (const Slot& s : sv->slots) b += s.busy;
      *busy_slots = b;
    }
    if (pending) *pending = (int32_t)sv->pending.size();
    return first_err;
  } catch (...) {
    set_error("unexpected host exception in farm_server_progress");
    return FARM_ERR_HIP;
  }
}

farm_status farm_server_poll(farm_server* sv, int32_t max_results, uint64_t* ids, int32_t* status, int32_t* certified,
                             int64_t* latency_ns, uint32_t* topk_ids, float* topk_scores, int32_t* n_out) {
  if (!sv || !n_out || max_results < 0) { set_error("null argument"); return FARM_ERR_INVALID_ARG; }
  const size_t k = (size_t)sv->cfg.k;
  int32_t n = 0;
  while (n < max_results && !sv->done.empty()) {
    Done& dn = sv->done.front();
    if (ids) ids[n] = dn.id;
    if (status) status[n] = dn.status;
    if (certified) certified[n] = dn.certified;
    if (latency_ns) latency_ns[n] = dn.done_ns - dn.submit_ns;
    for (size_t j = 0; j < k; ++j) {
      if (topk_ids) topk_ids[(size_t)n * k + j] = dn.status == 0 ? dn.ids[j] : FARM_NO_ID;
      if (topk_scores) topk_scores[(size_t)n * k + j] = dn.status == 0 ? dn.scores[j] : -INFINITY;
    }
    sv->done.pop_front();
    ++n;
  }
  *n_out = n;
  return FARM_OK;
}

farm_status farm_server_stats(const farm_server* sv, int64_t* stats) {
  if (!sv || !stats) { set_error("null argument"); return FARM_ERR_INVALID_ARG; }
  stats[0] = sv->batches;
  stats[1] = sv->deferrals;
  stats[2] = sv->evictions;
  stats[3] = (int64_t)sv->pool_bytes;
  int64_t live = 0;
  for (const PooledWs& p : sv->pool) live += p.ws != nullptr;
  stats[4] = live;
  return FARM_OK;
}

farm_status farm_server_free(farm_server* sv) {
  if (!sv) return FARM_OK;
  DeviceGuard g(sv->device);
  for (Slot& s : sv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    release_slot_buffers(s);
  }
  for (PooledWs& p : sv->pool)
    if (p.ws) (void)farm_workspace_free(p.ws);
  for (const farm_memory* m : sv->scenes) m->users.fetch_sub(1, std::memory_order_acq_rel);
  delete sv;
  return FARM_OK;
}

}  // extern "C"
