// serve.hip - request loop over the per-source query with continuous
// batching: a queue of requests, `slots` workers, each with its own HIP
// stream and device scratch, forming batches from whatever is queued when
// they become free (host code plus one setup kernel).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lp_common.h"

namespace lp {
lp_status run_query(lp_graph* g, Workspace& w, const int32_t* sources, int64_t nq, int m, int64_t L,
                    int32_t kq, float s_th, int32_t* out_c, float* out_score, int32_t* out_count,
                    hipStream_t st);
void release_workspace(Workspace& w);
void clear_error();
const char* last_error_text();

// Two-hop paths from each vertex (original id order) under a hub limit: the
// sum of the degrees of its neighbours with relabelled id below `hub` (those
// of degree <= L; rows ascend, so they come first): exactly the wedges the
// query's plan counts for it.
__global__ void path_bound_kernel(const uint32_t* __restrict__ off, const uint32_t* __restrict__ adj,
                                  const uint32_t* __restrict__ deg, const uint32_t* __restrict__ rank,
                                  int64_t n, uint32_t hub, unsigned long long* __restrict__ out) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n) return;
  const uint32_t v = rank[o];
  unsigned long long s = 0;
  for (uint32_t e = off[v]; e < off[v + 1] && adj[e] < hub; e++) s += deg[adj[e]];
  out[o] = s;
}
}  // namespace lp

using namespace lp;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  uint64_t id = 0;
  std::vector<int32_t> sources;
  int m = 0;
  int64_t L = 0;
  int32_t kq = 0;
  float s_th = 0;
  int32_t* out_c = nullptr;
  float* out_s = nullptr;
  int32_t* out_n = nullptr;
  uint64_t paths = 0;
  uint64_t bytes = 0;  // device scratch the request needs (see lp_server::need)
  uint32_t hubs = 0;   // sources above the LDS capacity (dense global accumulators)
  Clock::time_point t_submit, t_start, t_done;
  lp_request_info info{};
  std::string error;  // the batch's error text when it failed
  bool done = false;
};

bool same_kind(const Request& a, const Request& b) {
  return a.m == b.m && a.L == b.L && a.kq == b.kq && a.s_th == b.s_th;
}

bool same_shape(const QueryShape& a, const QueryShape& b) {
  return a.m == b.m && a.L == b.L && a.kq == b.kq && a.s_th == b.s_th && a.qcap == b.qcap && a.pcap == b.pcap &&
         a.slabs == b.slabs && a.rounds == b.rounds;
}

uint64_t pow_at_least(uint64_t base, uint64_t x) {
  uint64_t p = 1;
  while (p < x) p *= base;
  return p;
}

uint64_t pow2_at_least(uint64_t x) { return pow_at_least(2, x); }

// results in a replayed batch's pinned output start here (after the status words)
constexpr size_t kReplayResults = 512;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct lp_server {
  lp_graph* g = nullptr;
  lp_server_config cfg{};
  std::vector<uint32_t> degree;  // per original id
  // per hub boundary (relabelled id): each vertex's two-hop paths in
  // original id order, computed on the first request with that boundary
  std::mutex paths_mu;
  std::unordered_map<uint32_t, std::vector<unsigned long long>> paths_at;
  lp_status paths_for(int64_t L, const std::vector<unsigned long long>** out);
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  // Recording a slot's launches must not overlap device allocation by
  // another slot (the runtime refuses allocation while a stream captures):
  // recording holds it exclusively, host-driven batches (which may grow
  // their workspace) hold it shared.
  std::shared_mutex capture_mu;
  std::deque<Request*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_id = 1, next_batch = 1;
  int running = 0;
  bool stop = false;
  // A batch's launches captured as a HIP graph, for one shape (kind of
  // request and capacities); replayed for every later batch that fits it.
  struct Captured {
    QueryShape sh{};
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;  // last batch that replayed it
  };
  static constexpr int kMaxCaptured = 16;
  struct Slot {
    Workspace ws;
    hipStream_t st = nullptr;
    std::vector<int32_t> src, c, n;
    std::vector<float> s;
    std::thread th;
    // replay: pinned inputs / outputs of the device query path, and the
    // captured graphs over this slot's workspace (all stale once a buffer
    // they point into moves, or once the graph's tuning changes)
    HostBuf in, out;
    std::vector<Captured> graphs;
    // candidate capacity per kind of request (measure, hub limit, k_q,
    // threshold): the candidates that pass the per-source floors are far
    // fewer than the path bound, so capacities follow what batches emitted
    struct KindCap {
      int m;
      int64_t L;
      int32_t kq;
      float s_th;
      uint64_t cap;
    };
    std::vector<KindCap> kind_cap;
    uint64_t& cap_of(const QueryShape& sh) {
      for (auto& c : kind_cap)
        if (c.m == sh.m && c.L == sh.L && c.kq == sh.kq && c.s_th == sh.s_th) return c.cap;
      kind_cap.push_back(KindCap{sh.m, sh.L, sh.kq, sh.s_th, 1ull << 18});
      return kind_cap.back().cap;
    }
    lp_tuning tuning_at{};
    uint64_t layout_at = 0;  // workspace digest the graphs were recorded over
    void drop_graphs() {
      for (auto& c : graphs)
        if (c.exec) (void)hipGraphExecDestroy(c.exec);
      graphs.clear();
    }
  };
  std::vector<std::unique_ptr<Slot>> slots;
  unsigned max_slabs = 1;  // dense accumulators one slot's workspace may hold

  void worker(Slot* sl);
  // One batch on the device-count query path as a replayed graph: LP_OK with
  // the results in sl->out, or an error (the caller then runs the batch on
  // the host-driven path).
  lp_status replay(Slot* sl, const QueryShape& sh, uint32_t nq, uint64_t bid);
  // Device scratch of a batch: candidate and sort buffers of 24 bytes per
  // two-hop path (the bound of its candidates), per-source records, counts
  // and outputs, and one dense accumulator of 12 bytes per vertex for each
  // source above the LDS capacity (at most max_slabs at once).
  uint64_t need(uint64_t paths, uint64_t sources, uint32_t hubs, int32_t kq) const {
    const uint64_t slabs = std::min<uint64_t>(hubs, max_slabs);
    return 24 * paths + sources * (4 + 7 * 32 + 8 + 12 * (uint64_t)kq) + slabs * 12 * (uint64_t)g->n;
  }
};

void lp_server::worker(Slot* sl) {
  (void)hipSetDevice(g->device);
  for (;;) {
    std::vector<Request*> batch;
    uint64_t bid = 0;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty(); });
      if (queue.empty()) return;  // stop requested and nothing left
      // the oldest request, then every queued one of the same kind whose
      // sources, paths and device scratch still fit the slot's budget
      Request* r0 = queue.front();
      queue.pop_front();
      batch.push_back(r0);
      uint64_t ns = r0->sources.size(), np = r0->paths;
      uint32_t nh = r0->hubs;
      for (auto it = queue.begin(); it != queue.end();) {
        Request* r = *it;
        if (same_kind(*r, *r0) && ns + r->sources.size() <= (uint64_t)cfg.max_batch_sources &&
            np + r->paths <= (uint64_t)cfg.max_batch_paths &&
            need(np + r->paths, ns + r->sources.size(), nh + r->hubs, r0->kq) <= (uint64_t)cfg.max_batch_bytes) {
          ns += r->sources.size();
          np += r->paths;
          nh += r->hubs;
          batch.push_back(r);
          it = queue.erase(it);
        } else {
          ++it;
        }
      }
      bid = next_batch++;
      running++;
    }
    const Clock::time_point t0 = Clock::now();
    const Request& k = *batch[0];
    size_t total = 0;
    uint64_t bpaths = 0;
    uint32_t bhubs = 0;
    for (auto* r : batch) {
      total += r->sources.size();
      bpaths += r->paths;
      bhubs += r->hubs;
    }
    const uint64_t batch_bytes = need(bpaths, total, bhubs, k.kq);
    sl->src.resize(total);
    size_t pos = 0;
    for (auto* r : batch) {
      std::copy(r->sources.begin(), r->sources.end(), sl->src.begin() + pos);
      pos += r->sources.size();
    }
    sl->c.resize(total * (size_t)k.kq);
    sl->s.resize(total * (size_t)k.kq);
    sl->n.resize(total);
    clear_error();
    lp_status status = LP_OK;
    bool replayed = false;
    uint32_t how = 0;  // lp_request_info.replayed
    std::string replay_error;
    // the replayed shape: capacities in coarse classes (so that later
    // batches of the same kind reuse the recorded graph), within the budget.
    // Sources: powers of 4 from 256; candidates: what this kind emitted so
    // far (never above the path bound); sources above the LDS capacity:
    // powers of 2.
    QueryShape sh{k.m, k.L, k.kq, k.s_th, 0, 0, 0, 0};
    sh.qcap = (uint32_t)std::min<uint64_t>(pow_at_least(4, std::max<uint64_t>(total, 256)), 1ull << 31);
    sh.pcap = std::min(sl->cap_of(sh), pow2_at_least(std::max<uint64_t>(bpaths, 1ull << 16)));
    // sources above the LDS capacity (the admission count bounds them):
    // rounds of `slabs` at a time; none launched when the batch has none
    const uint64_t hubs_cap = bhubs ? pow2_at_least(bhubs) : 0;
    sh.slabs = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(hubs_cap, max_slabs));
    while (sh.slabs > 1 && need(sh.pcap, sh.qcap, sh.slabs, k.kq) > (uint64_t)cfg.max_batch_bytes) sh.slabs >>= 1;
    sh.rounds = (unsigned)((hubs_cap + sh.slabs - 1) / sh.slabs);
    if (!cfg.host_launches && sh.pcap < (1ull << 32) &&
        need(sh.pcap, sh.qcap, sh.slabs, k.kq) <= (uint64_t)cfg.max_batch_bytes) {
      lp_status rs = LP_ERR_DEVICE;
      try {
        rs = replay(sl, sh, (uint32_t)total, bid);
      } catch (...) {
        rs = LP_ERR_DEVICE;
      }
      replayed = rs == LP_OK;
      how = replayed ? 1u : rs == LP_ERR_OUT_OF_MEMORY && last_error_text()[0] == 0 ? 2u : 3u;
      if (!replayed) {
        // run on the host-driven path below; keep why the replay was abandoned
        replay_error = last_error_text();
        clear_error();
      }
    }
    if (!replayed) {
      std::shared_lock<std::shared_mutex> alloc(capture_mu);
      try {
        status = run_query(g, sl->ws, sl->src.data(), (int64_t)total, k.m, k.L, k.kq, k.s_th,
                           sl->c.data(), sl->s.data(), sl->n.data(), sl->st);
      } catch (const std::bad_alloc&) {
        status = LP_ERR_OUT_OF_MEMORY;
      } catch (...) {
        status = LP_ERR_DEVICE;
      }
    }
    // results to each request's buffers (replayed: rows of k_q in the pinned
    // output, scores after qcap * k_q ids, then the counts)
    const char* ho = replayed ? sl->out.as<char>() + kReplayResults : nullptr;
    const size_t qk = (size_t)sh.qcap * (size_t)k.kq;
    pos = 0;
    for (auto* r : batch) {
      const size_t m = r->sources.size();
      if (replayed) {
        std::memcpy(r->out_c, ho + pos * k.kq * 4, m * k.kq * 4);
        std::memcpy(r->out_s, ho + qk * 4 + pos * k.kq * 4, m * k.kq * 4);
        std::memcpy(r->out_n, ho + qk * 8 + pos * 4, m * 4);
      } else if (status == LP_OK) {
        std::copy(sl->c.begin() + pos * k.kq, sl->c.begin() + (pos + m) * k.kq, r->out_c);
        std::copy(sl->s.begin() + pos * k.kq, sl->s.begin() + (pos + m) * k.kq, r->out_s);
        std::copy(sl->n.begin() + pos, sl->n.begin() + pos + m, r->out_n);
      }
      pos += m;
    }
    const Clock::time_point t1 = Clock::now();
    {
      std::lock_guard<std::mutex> lk(mu);
      for (auto* r : batch) {
        r->t_start = t0;
        r->t_done = t1;
        r->info.status = status;
        r->info.batch = bid;
        r->info.batch_requests = (uint32_t)batch.size();
        r->info.replayed = how;
        if (status != LP_OK)
          r->error = std::string(last_error_text()) +
                     (replay_error.empty() ? std::string() : " (replay: " + replay_error + ")");
        r->info.batch_sources = total;
        r->info.batch_bytes = batch_bytes;
        r->info.queue_ms = ms_between(r->t_submit, t0);
        r->info.run_ms = ms_between(t0, t1);
        r->info.total_ms = ms_between(r->t_submit, t1);
        r->done = true;
      }
      running--;
    }
    cv_done.notify_all();
  }
}

lp_status lp_server::paths_for(int64_t L, const std::vector<unsigned long long>** out) {
  const uint32_t hub = hub_start(g, L);
  std::lock_guard<std::mutex> lk(paths_mu);
  auto it = paths_at.find(hub);
  if (it == paths_at.end()) {
    const int64_t n = g->n;
    std::vector<unsigned long long> p((size_t)n, 0);
    if (n > 0) {
      // device allocation: not while a slot records its launches
      std::shared_lock<std::shared_mutex> alloc(capture_mu);
      LP_HIP(hipSetDevice(g->device));
      DevBuf tmp;
      LP_TRY(tmp.ensure((size_t)n * 8));
      hipLaunchKernelGGL(path_bound_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, nullptr, g->off,
                         g->adj, g->deg, g->rank, n, hub, tmp.as<unsigned long long>());
      lp_status st = LP_OK;
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpy(p.data(), tmp.p, (size_t)n * 8, hipMemcpyDeviceToHost);
      if (e != hipSuccess) st = from_hip(e, "path bounds");
      tmp.release();
      if (st != LP_OK) return st;
    }
    it = paths_at.emplace(hub, std::move(p)).first;
  }
  *out = &it->second;
  return LP_OK;
}

lp_status lp_server::replay(Slot* sl, const QueryShape& sh, uint32_t nq, uint64_t bid) {
  // the graph recorded for this shape, if any
  if (std::memcmp(&sl->tuning_at, &g->tuning, sizeof(lp_tuning)) != 0 ||
      query_device_layout(sl->ws) != sl->layout_at) {
    sl->drop_graphs();
    sl->tuning_at = g->tuning;
    sl->layout_at = query_device_layout(sl->ws);
  }
  Captured* cap = nullptr;
  for (auto& c : sl->graphs)
    if (same_shape(c.sh, sh)) cap = &c;
  if (!cap) {
    std::unique_lock<std::shared_mutex> rec(capture_mu);
    // every allocation happens here, before the capture
    bool moved = false;
    LP_TRY(query_device_reserve(g, sl->ws, sh, &moved, sl->st));
    const void* in0 = sl->in.p;
    const void* out0 = sl->out.p;
    LP_TRY(sl->in.ensure(query_device_in_bytes(sh.qcap)));
    LP_TRY(sl->out.ensure(query_device_out_bytes(sh.qcap, sh.kq)));
    if (moved || sl->in.p != in0 || sl->out.p != out0) sl->drop_graphs();
    sl->layout_at = query_device_layout(sl->ws);
    if ((int)sl->graphs.size() >= kMaxCaptured) {
      auto lru = std::min_element(sl->graphs.begin(), sl->graphs.end(),
                                  [](const Captured& a, const Captured& b) { return a.used < b.used; });
      (void)hipGraphExecDestroy(lru->exec);
      sl->graphs.erase(lru);
    }
    LP_HIP(hipStreamBeginCapture(sl->st, hipStreamCaptureModeRelaxed));
    const lp_status es = query_device_enqueue(g, sl->ws, sh, sl->in.p, sl->out.p, sl->st);
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(sl->st, &graph);
    if (es != LP_OK || ee != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      return es != LP_OK ? es : set_error(LP_ERR_DEVICE, "stream capture failed");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess || !exec) {
      (void)hipGetLastError();
      return set_error(LP_ERR_DEVICE, "graph instantiation failed");
    }
    sl->graphs.push_back(Captured{sh, exec, bid});
    cap = &sl->graphs.back();
  }
  cap->used = bid;
  // inputs: the query count, then the sources
  char* hi = sl->in.as<char>();
  std::memcpy(hi, &nq, 4);
  std::memcpy(hi + 64, sl->src.data(), (size_t)nq * 4);
  LP_HIP(hipGraphLaunch(cap->exec, sl->st));
  LP_HIP(hipStreamSynchronize(sl->st));
  uint64_t emitted = 0;
  const lp_status st = query_device_status(sl->out.p, sh, nq, &emitted);
  // later batches of this kind get room for twice what this one emitted
  uint64_t& c = sl->cap_of(sh);
  c = std::max(c, pow2_at_least(2 * emitted));
  return st;
}

extern "C" {

lp_status lp_server_create(lp_graph* g, const lp_server_config* cfg, lp_server** out) {
  clear_error();
  if (!g || !out) return set_error(LP_ERR_INVALID_ARGUMENT, "graph or out is NULL");
  *out = nullptr;
  try {
    std::unique_ptr<lp_server> s(new lp_server());
    s->g = g;
    if (cfg) s->cfg = *cfg;
    if (s->cfg.slots == 0) s->cfg.slots = 2;
    if (s->cfg.max_batch_sources == 0) s->cfg.max_batch_sources = 16384;
    if (s->cfg.max_batch_paths == 0) s->cfg.max_batch_paths = 1ll << 27;
    LP_HIP(hipSetDevice(g->device));
    // every slot's workspace keeps its global accumulators within an eighth of
    // the device memory; the default scratch budget splits that eighth
    s->max_slabs = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>((uint64_t)num_cus(), device_memory() / 8 / ((uint64_t)g->n * 12 + 1)));
    if (s->cfg.max_batch_bytes == 0)
      s->cfg.max_batch_bytes = (int64_t)(device_memory() / 8 / (uint64_t)std::max(1, s->cfg.slots));
    if (s->cfg.slots < 1 || s->cfg.slots > 8 || s->cfg.max_batch_sources < 1 ||
        s->cfg.max_batch_paths < 1 || s->cfg.max_batch_bytes < 1)
      return set_error(LP_ERR_INVALID_ARGUMENT, "server config out of range");
    const int64_t n = g->n;
    if (n > 0) {
      // degrees in original id order (the graph keeps them sorted by new id)
      std::vector<uint32_t> rank((size_t)n);
      LP_HIP(hipMemcpy(rank.data(), g->rank, (size_t)n * 4, hipMemcpyDeviceToHost));
      s->degree.resize((size_t)n);
      for (int64_t o = 0; o < n; o++) s->degree[(size_t)o] = g->host_deg[rank[(size_t)o]];
    }
    for (int i = 0; i < s->cfg.slots; i++) {
      auto sl = std::make_unique<lp_server::Slot>();
      LP_HIP(hipStreamCreateWithFlags(&sl->st, hipStreamNonBlocking));
      s->slots.push_back(std::move(sl));
    }
    for (auto& sl : s->slots) {
      lp_server::Slot* p = sl.get();
      lp_server* sp = s.get();
      sl->th = std::thread([sp, p] { sp->worker(p); });
    }
    *out = s.release();
    return LP_OK;
  } catch (const std::bad_alloc&) {
    return set_error(LP_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return set_error(LP_ERR_DEVICE, "server start failed");
  }
}

lp_status lp_server_destroy(lp_server* s) {
  clear_error();
  if (!s) return set_error(LP_ERR_INVALID_ARGUMENT, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& sl : s->slots)
    if (sl->th.joinable()) sl->th.join();
  (void)hipSetDevice(s->g->device);
  for (auto& sl : s->slots) {
    sl->drop_graphs();
    sl->in.release();
    sl->out.release();
    release_workspace(sl->ws);
    if (sl->st) (void)hipStreamDestroy(sl->st);
  }
  delete s;
  return LP_OK;
}

lp_status lp_server_submit(lp_server* s, const int32_t* sources, int64_t n_sources, lp_measure m,
                           int64_t hub_limit, int32_t k_q, float score_threshold, int32_t* out_c,
                           float* out_score, int32_t* out_count, uint64_t* ticket) {
  clear_error();
  if (!s || !ticket) return set_error(LP_ERR_INVALID_ARGUMENT, "server or ticket is NULL");
  if ((int)m < LP_CN || (int)m > LP_RA) return set_error(LP_ERR_INVALID_ARGUMENT, "measure out of range");
  if (hub_limit < 0) return set_error(LP_ERR_INVALID_ARGUMENT, "hub_limit must be >= 0");
  if (!std::isfinite(score_threshold) || score_threshold < 0.0f)
    return set_error(LP_ERR_INVALID_ARGUMENT, "score_threshold must be finite and >= 0");
  if (k_q <= 0) return set_error(LP_ERR_INVALID_ARGUMENT, "k_q must be > 0");
  if (n_sources <= 0 || n_sources > INT32_MAX)
    return set_error(LP_ERR_INVALID_ARGUMENT, "n_sources must be in [1, 2^31 - 1]");
  if ((uint64_t)n_sources * (uint64_t)k_q >= (1ull << 32))
    return set_error(LP_ERR_INVALID_ARGUMENT, "n_sources * k_q too large");
  if (!sources || !out_c || !out_score || !out_count)
    return set_error(LP_ERR_INVALID_ARGUMENT, "array pointer is NULL");
  try {
    auto r = std::make_unique<Request>();
    r->sources.assign(sources, sources + n_sources);
    // a source's wedges under this hub limit (the plan's count), and whether
    // its table bound (wedges plus degree) exceeds the LDS capacity, so that
    // it takes a dense global accumulator
    for (int32_t v : r->sources)
      if (v < 0 || (int64_t)v >= s->g->n)
        return set_error(LP_ERR_INVALID_ARGUMENT, "source %d outside [0, n)", (int)v);
    const std::vector<unsigned long long>* P = nullptr;
    LP_TRY(s->paths_for(hub_limit, &P));
    const uint64_t cap = s->g->tuning.lds_wedge_cap > 0 ? (uint64_t)s->g->tuning.lds_wedge_cap : 65536;
    uint64_t paths = 0;
    uint32_t hubs = 0;
    for (int32_t v : r->sources) {
      const uint64_t p = (*P)[(size_t)v];
      paths += p;
      hubs += p + s->degree[(size_t)v] > cap ? 1u : 0u;
    }
    r->paths = paths;
    r->hubs = hubs;
    r->bytes = s->need(paths, r->sources.size(), hubs, k_q);
    r->m = (int)m;
    r->L = hub_limit;
    r->kq = k_q;
    r->s_th = score_threshold;
    r->out_c = out_c;
    r->out_s = out_score;
    r->out_n = out_count;
    r->t_submit = Clock::now();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->stop) return set_error(LP_ERR_INVALID_ARGUMENT, "server is stopping");
      r->id = s->next_id++;
      *ticket = r->id;
      s->queue.push_back(r.get());
      s->reqs.emplace(r->id, std::move(r));
    }
    s->cv_work.notify_one();
    return LP_OK;
  } catch (const std::bad_alloc&) {
    return set_error(LP_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

lp_status lp_server_wait(lp_server* s, uint64_t ticket, int64_t timeout_ms, lp_request_info* info) {
  clear_error();
  if (!s) return set_error(LP_ERR_INVALID_ARGUMENT, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(LP_ERR_INVALID_ARGUMENT, "unknown ticket %llu",
                                            (unsigned long long)ticket);
  Request* r = it->second.get();
  auto ready = [&] { return r->done; };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return set_error(LP_ERR_BUSY, "request %llu still running", (unsigned long long)ticket);
  }
  const lp_request_info ri = r->info;
  const std::string err = r->error;
  s->reqs.erase(it);
  if (info) *info = ri;
  if (ri.status != LP_OK)
    return set_error(ri.status, "the batch serving request %llu failed: %s", (unsigned long long)ticket,
                     err.c_str());
  return LP_OK;
}

}  // extern "C"
