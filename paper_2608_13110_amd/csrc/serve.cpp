// Continuous-batching request loop for amplitude requests of mixed shape.
//
// Requests (circuit, bitstring batch, open legs k, storage) arrive through
// tnc_server_submit at any time.  A pool of planner threads turns each
// circuit into a plan (cached by a hash of the circuit, with tile options
// picked per width by the autotuner) and uploads its tables; the dispatcher
// thread admits prepared requests onto free HIP streams as soon as the
// device arena has room for their footprint (tensor workspace, bits,
// output), so requests that arrive while others run start as soon as a
// stream and memory free up, and the work of different requests overlaps on
// the device.
//
// Small requests (boundary bits <= small_bits) run together: the ready
// complex64 requests of one width are taken as a group (up to max_group),
// their launches are recorded, and the k-th launches of all members that use
// the same kernel become one grouped launch (its segments are the members'
// own arguments; kernels.hpp).  A small request whose (plan, k, batches,
// storage) comes back runs as a cached HIP graph: built once, node by node,
// from its launch records (no stream capture), with its own device region,
// and replayed from any stream while idle.  No stream is ever put in capture
// mode, so the server never constrains what other threads do on the device.
// Batches of a plan share only the read-only plan (Sec. 5.2: the batches of
// one circuit differ only in their output bits).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "exec.hpp"
#include "tnc.h"

namespace tnc {

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

// First-fit allocator over [0, size) in 256-byte units, with coalescing.
class Arena {
 public:
  explicit Arena(uint64_t size = 0) { if (size) free_[0] = size; }
  // Returns the offset or UINT64_MAX.
  uint64_t alloc(uint64_t bytes) {
    bytes = (bytes + 255) & ~uint64_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const uint64_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[off + bytes] = len - bytes;
      used_[off] = bytes;
      return off;
    }
    return UINT64_MAX;
  }
  void release(uint64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    uint64_t len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  uint64_t largest() const {
    uint64_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }

 private:
  std::map<uint64_t, uint64_t> free_, used_;
};

struct CircuitKey {
  int32_t n = 0, d = 0;
  std::vector<tnc_c128> one;
  std::vector<tnc_gate2> gates;
  bool operator==(const CircuitKey& o) const {
    return n == o.n && d == o.d && one.size() == o.one.size() && gates.size() == o.gates.size() &&
           std::memcmp(one.data(), o.one.data(), one.size() * sizeof(tnc_c128)) == 0 &&
           std::memcmp(gates.data(), o.gates.data(), gates.size() * sizeof(tnc_gate2)) == 0;
  }
};

struct CachedPlan {
  CircuitKey key;
  tnc_plan_t plan = nullptr;
  int ready = 0;  // 0 building, 1 ready, -1 failed
  int rc = 0;
};

enum ReqState { R_PLANNING = 0, R_READY = 1, R_RUNNING = 2, R_DONE = 3 };

struct Request {
  uint64_t id = 0;
  CircuitKey circuit;
  uint64_t hash = 0;
  std::shared_ptr<CachedPlan> cp;
  int32_t nb = 0, k = 0, storage = 0;
  std::vector<uint8_t> bits;
  tnc_c128* out = nullptr;
  uint64_t ws_bytes = 0, footprint = 0;
  int h = 0;
  int n_launches = 0;  // launches of one batch group (bounds its segment table)
  int state = R_PLANNING;
  int rc = 0;
  std::string err;  // what failed, for tnc_last_error of the waiting thread
  int bypassed = 0;
  bool small = false;
  int mode = 0;  // how it ran: 0 plain, 1 graph replay, 2 in a group of several
  int64_t t_submit = 0, t_ready = 0, t_admit = 0, t_done = 0;
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  uint64_t off = 0;  // its own arena block: workspace, bits, output
  bool busy = false;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  std::vector<std::shared_ptr<Request>> reqs;  // one request, or the members of a group
  std::vector<size_t> out_at;                  // per member: first amplitude in h_out
  uint64_t off = UINT64_MAX;                   // arena block (plain request or group)
  GraphEntry* graph = nullptr;                 // or the cached graph it replays
  unsigned char* h_in = nullptr;               // pinned staging: segment tables and bits
  tnc_c128* h_out = nullptr;                   // pinned staging: amplitudes
  size_t cap_in = 0, cap_out = 0;
};

struct GraphKey {
  tnc_plan_t plan;
  int k, nb, storage;
  bool operator<(const GraphKey& o) const {
    return std::tie(plan, k, nb, storage) < std::tie(o.plan, o.k, o.nb, o.storage);
  }
};

uint64_t up256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

}  // namespace

struct ServerImpl {
  tnc_server_options opt{};
  int device = 0;
  char* arena_base = nullptr;
  uint64_t arena_bytes = 0, graph_bytes = 0, graph_budget = 0;
  Arena arena;
  std::vector<Slot> slots;
  std::map<int, tnc_options> tuning;  // boundary bits -> tile options

  std::mutex mu;
  std::condition_variable cv_plan, cv_dispatch, cv_done;
  std::deque<std::shared_ptr<Request>> to_plan, ready;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs;
  std::unordered_multimap<uint64_t, std::shared_ptr<CachedPlan>> plans;
  std::map<GraphKey, std::unique_ptr<GraphEntry>> graphs;
  std::map<GraphKey, int> seen;  // small requests met per key (a graph is built on the second)
  uint64_t next_id = 1;
  bool stop = false;
  std::vector<std::thread> planners;
  std::thread dispatcher;

  // statistics
  uint64_t n_done = 0, n_graph_launch = 0, n_graph_build = 0, n_graph_failed = 0, n_plain = 0, n_groups = 0,
           n_grouped_reqs = 0, n_grouped_launches = 0, plan_hits = 0, plan_misses = 0;
  int64_t first_submit = 0, last_done = 0;
  std::vector<double> lat_ms;
  int max_inflight = 0;

  tnc_options options_for(int h) const {
    tnc_options o{};
    auto it = tuning.find(h);
    if (it != tuning.end()) o = it->second;
    return o;
  }

  void planner_loop();
  void dispatcher_loop();
  int run_plain(Slot& s, Request& r);
  int run_graph(Slot& s, Request& r, GraphEntry* g);
  int run_group(Slot& s);
  bool admit(Slot& s, std::deque<std::shared_ptr<Request>>::iterator it);
  bool holding(const Request& r, int64_t now) const;
  void finish(Slot& s, bool ok);
};

namespace {

int ceil_half(int d) { return (d + 1) / 2; }

bool ensure_pinned(Slot& s, size_t in_bytes, size_t outs) {
  if (in_bytes > s.cap_in) {
    if (s.h_in) (void)hipHostFree(s.h_in);
    s.h_in = nullptr;
    s.cap_in = 0;
    if (hipHostMalloc((void**)&s.h_in, in_bytes) == hipSuccess) s.cap_in = in_bytes;
  }
  if (outs > s.cap_out) {
    if (s.h_out) (void)hipHostFree(s.h_out);
    s.h_out = nullptr;
    s.cap_out = 0;
    if (hipHostMalloc((void**)&s.h_out, outs * sizeof(tnc_c128)) == hipSuccess) s.cap_out = outs;
  }
  return s.cap_in >= in_bytes && s.cap_out >= outs;
}

int fail_req(Request& r, int code, const std::string& what, hipError_t e) {
  r.err = "serving: " + what + (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : std::string()) +
          (code != TNC_OK && e == hipSuccess ? std::string(": ") + tnc_last_error() : std::string());
  return code;
}

// Device layout of one request inside its block: workspace, bits, output.
struct ReqLayout {
  uint64_t ws = 0, bits = 0, out = 0, total = 0;
};

ReqLayout req_layout(const Request& r) {
  ReqLayout L;
  L.ws = 0;
  L.bits = up256(r.ws_bytes);
  L.out = L.bits + up256((uint64_t)r.nb * r.circuit.n);
  L.total = L.out + up256(((uint64_t)r.nb << r.k) * sizeof(tnc_c128));
  return L;
}

}  // namespace

void ServerImpl::planner_loop() {
  (void)hipSetDevice(device);
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_plan.wait(lk, [&] { return stop || !to_plan.empty(); });
      if (stop && to_plan.empty()) return;
      r = to_plan.front();
      to_plan.pop_front();
    }
    // find or build the plan (one builder per circuit; others wait)
    std::shared_ptr<CachedPlan> cp;
    bool build = false;
    {
      std::unique_lock<std::mutex> lk(mu);
      auto range = plans.equal_range(r->hash);
      for (auto it = range.first; it != range.second; ++it)
        if (it->second->key == r->circuit) cp = it->second;
      if (!cp) {
        cp = std::make_shared<CachedPlan>();
        cp->key = r->circuit;
        plans.emplace(r->hash, cp);
        build = true;
        ++plan_misses;
      } else {
        ++plan_hits;
      }
    }
    int rc = 0;
    if (build) {
      tnc_plan_t p = nullptr;
      tnc_options o;
      {
        std::lock_guard<std::mutex> lk(mu);
        o = options_for(ceil_half(r->circuit.d));
      }
      rc = tnc_plan(r->circuit.n, r->circuit.d, r->circuit.one.data(), (int32_t)r->circuit.gates.size(),
                    r->circuit.gates.data(), &o, &p);
      std::lock_guard<std::mutex> lk(mu);
      cp->plan = p;
      cp->rc = rc;
      cp->ready = rc ? -1 : 1;
      cv_done.notify_all();
    } else {
      std::unique_lock<std::mutex> lk(mu);
      cv_done.wait(lk, [&] { return cp->ready != 0; });
      rc = cp->rc;
    }
    tnc_info info{};
    uint64_t ws = 0;
    if (!rc) rc = tnc_plan_info(cp->plan, r->k, &info);
    if (!rc) rc = tnc_prepare(cp->plan, r->k);
    if (!rc) rc = tnc_workspace_bytes(cp->plan, r->k, r->nb, r->storage, &ws);
    const std::string perr = rc ? std::string("serving: planning: ") + tnc_last_error() : std::string();
    std::lock_guard<std::mutex> lk(mu);
    r->err = perr;
    r->cp = cp;
    r->rc = rc;
    r->h = info.boundary_bits;
    r->ws_bytes = ws;
    r->n_launches = 2 + info.n_passes + info.n_late_launches;
    r->footprint = req_layout(*r).total;
    r->small = opt.small_bits > 0 && r->h <= opt.small_bits;
    r->t_ready = now_ns();
    if (rc) {
      r->state = R_DONE;
      r->t_done = r->t_ready;
      cv_done.notify_all();
    } else {
      r->state = R_READY;
      ready.push_back(r);
      cv_dispatch.notify_one();
    }
  }
}

// A request on its own, from the arena block at s.off.
int ServerImpl::run_plain(Slot& s, Request& r) {
  const ReqLayout L = req_layout(r);
  const size_t nbits = (size_t)r.nb * r.circuit.n, nout = (size_t)r.nb << r.k;
  if (!ensure_pinned(s, nbits, nout)) return fail_req(r, TNC_E_NOMEM, "pinned staging allocation", hipSuccess);
  char* base = arena_base + s.off;
  uint8_t* d_bits = reinterpret_cast<uint8_t*>(base + L.bits);
  tnc_c128* d_out = reinterpret_cast<tnc_c128*>(base + L.out);
  std::memcpy(s.h_in, r.bits.data(), nbits);
  hipError_t e = hipMemcpyAsync(d_bits, s.h_in, nbits, hipMemcpyHostToDevice, s.stream);
  if (e != hipSuccess) return fail_req(r, TNC_E_DEVICE, "bits upload", e);
  const int rc = tnc_amplitudes(r.cp->plan, r.nb, d_bits, r.k, r.storage, d_out, base + L.ws, r.ws_bytes, s.stream);
  if (rc) return fail_req(r, rc, "launch sequence", hipSuccess);
  e = hipMemcpyAsync(s.h_out, d_out, nout * sizeof(tnc_c128), hipMemcpyDeviceToHost, s.stream);
  if (e != hipSuccess) return fail_req(r, TNC_E_DEVICE, "result download", e);
  s.out_at.assign(1, 0);
  ++n_plain;
  return TNC_OK;
}

// A small request through its cached graph (built on first use from the
// launch records of its own region, node after node, without capture).
int ServerImpl::run_graph(Slot& s, Request& r, GraphEntry* g) {
  const ReqLayout L = req_layout(r);
  const size_t nbits = (size_t)r.nb * r.circuit.n, nout = (size_t)r.nb << r.k;
  if (!ensure_pinned(s, nbits, nout)) return fail_req(r, TNC_E_NOMEM, "pinned staging allocation", hipSuccess);
  char* base = arena_base + g->off;
  uint8_t* d_bits = reinterpret_cast<uint8_t*>(base + L.bits);
  tnc_c128* d_out = reinterpret_cast<tnc_c128*>(base + L.out);
  if (!g->exec) {
    std::vector<Launch> ls;
    int rc = record_amplitudes(r.cp->plan, r.nb, d_bits, r.k, r.storage, d_out, base + L.ws, r.ws_bytes, &ls);
    if (rc) return fail_req(r, rc, "launch records", hipSuccess);
    hipGraph_t graph = nullptr;
    hipError_t e = hipGraphCreate(&graph, 0);
    hipGraphNode_t prev = nullptr;
    for (size_t i = 0; e == hipSuccess && i < ls.size(); ++i) {
      hipGraphNode_t node = nullptr;
      e = graph_add(ls[i], graph, &node, prev ? &prev : nullptr, prev ? 1 : 0);
      prev = node;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g->exec = nullptr;
      ++n_graph_failed;
      return fail_req(r, TNC_E_DEVICE, "graph build", e);
    }
    ++n_graph_build;
  }
  std::memcpy(s.h_in, r.bits.data(), nbits);
  hipError_t e = hipMemcpyAsync(d_bits, s.h_in, nbits, hipMemcpyHostToDevice, s.stream);
  if (e != hipSuccess) return fail_req(r, TNC_E_DEVICE, "bits upload", e);
  e = hipGraphLaunch(g->exec, s.stream);
  if (e != hipSuccess) return fail_req(r, TNC_E_DEVICE, "graph launch", e);
  e = hipMemcpyAsync(s.h_out, d_out, nout * sizeof(tnc_c128), hipMemcpyDeviceToHost, s.stream);
  if (e != hipSuccess) return fail_req(r, TNC_E_DEVICE, "result download", e);
  s.out_at.assign(1, 0);
  ++n_graph_launch;
  return TNC_OK;
}

// The members of s.reqs (small complex64 requests of one width) together,
// from the arena block at s.off laid out as [segment tables | bits of every
// member | outputs of every member | workspaces].  Launch i of every member
// that uses the same kernel as the others' launch i runs in one grouped
// launch; the segment tables and the bits go up in one copy, the outputs
// come back in one copy.
int ServerImpl::run_group(Slot& s) {
  const size_t m = s.reqs.size();
  Request& r0 = *s.reqs[0];
  uint64_t seg_bytes = 0, bits_bytes = 0, out_amps = 0, ws_total = 0;
  for (auto& rp : s.reqs) {
    seg_bytes += (uint64_t)rp->n_launches * (kSegHeader + kMaxArgBytes);
    bits_bytes += up256((uint64_t)rp->nb * rp->circuit.n);
    out_amps += (uint64_t)rp->nb << rp->k;
    ws_total += up256(rp->ws_bytes);
  }
  seg_bytes = up256(seg_bytes);
  if (!ensure_pinned(s, seg_bytes + bits_bytes, out_amps))
    return fail_req(r0, TNC_E_NOMEM, "pinned staging allocation", hipSuccess);
  char* base = arena_base + s.off;
  const uint64_t out_base = seg_bytes + bits_bytes;
  uint64_t ws_at = up256(out_base + out_amps * sizeof(tnc_c128));
  uint64_t bits_at = seg_bytes, amp_at = 0;
  std::vector<std::vector<Launch>> ls(m);
  s.out_at.assign(m, 0);
  size_t longest = 0;
  for (size_t i = 0; i < m; ++i) {
    Request& r = *s.reqs[i];
    const size_t nbits = (size_t)r.nb * r.circuit.n;
    std::memcpy(s.h_in + bits_at, r.bits.data(), nbits);
    s.out_at[i] = amp_at;
    int rc = record_amplitudes(r.cp->plan, r.nb, reinterpret_cast<uint8_t*>(base + bits_at), r.k, r.storage,
                               reinterpret_cast<tnc_c128*>(base + out_base) + amp_at, base + ws_at, r.ws_bytes, &ls[i]);
    if (rc) return fail_req(r0, rc, "launch records", hipSuccess);
    bits_at += up256(nbits);
    amp_at += (uint64_t)r.nb << r.k;
    ws_at += up256(r.ws_bytes);
    longest = std::max(longest, ls[i].size());
  }
  // step j: the j-th launch of every member, in buckets of one kernel
  struct Item {
    std::vector<const Launch*> members;
    uint64_t seg_off;
  };
  std::vector<Item> items;
  uint64_t seg_at = 0;
  for (size_t j = 0; j < longest; ++j) {
    const size_t first = items.size();
    for (size_t i = 0; i < m; ++i) {
      if (j >= ls[i].size()) continue;
      const Launch* L = &ls[i][j];
      size_t b = first;
      while (b < items.size() && !groupable(*items[b].members[0], *L)) ++b;
      if (b == items.size()) items.push_back(Item{{}, 0});
      items[b].members.push_back(L);
    }
    for (size_t b = first; b < items.size(); ++b) {
      Item& it = items[b];
      if (it.members.size() < 2) continue;
      const uint64_t need = (uint64_t)it.members.size() * it.members[0]->seg_stride;
      if (seg_at + need > seg_bytes) return fail_req(r0, TNC_E_NOMEM, "group segment tables", hipSuccess);
      it.seg_off = seg_at;
      write_segments(it.members.data(), (int)it.members.size(), s.h_in + seg_at);
      seg_at = up256(seg_at + need);
    }
  }
  hipError_t e = hipMemcpyAsync(base, s.h_in, seg_bytes + bits_bytes, hipMemcpyHostToDevice, s.stream);
  if (e != hipSuccess) return fail_req(r0, TNC_E_DEVICE, "segment and bits upload", e);
  for (const Item& it : items) {
    if (it.members.size() == 1) {
      std::vector<Launch> one(1, *it.members[0]);
      const int rc = issue_recorded(one, s.stream);
      if (rc) return fail_req(r0, rc, "launch", hipSuccess);
      continue;
    }
    e = issue_grouped(it.members.data(), (int)it.members.size(), base + it.seg_off, s.stream);
    if (e != hipSuccess) return fail_req(r0, TNC_E_DEVICE, "grouped launch", e);
    ++n_grouped_launches;
  }
  e = hipMemcpyAsync(s.h_out, base + out_base, out_amps * sizeof(tnc_c128), hipMemcpyDeviceToHost, s.stream);
  if (e != hipSuccess) return fail_req(r0, TNC_E_DEVICE, "result download", e);
  if (m > 1) {
    ++n_groups;
    n_grouped_reqs += m;
  } else {
    ++n_plain;
  }
  (void)ws_total;
  return TNC_OK;
}

void ServerImpl::finish(Slot& s, bool ok) {
  for (size_t i = 0; i < s.reqs.size(); ++i) {
    Request& r = *s.reqs[i];
    if (ok && r.rc == TNC_OK && r.out && i < s.out_at.size())
      std::memcpy(r.out, s.h_out + s.out_at[i], ((size_t)r.nb << r.k) * sizeof(tnc_c128));
    r.t_done = now_ns();
    r.state = R_DONE;
    ++n_done;
    last_done = r.t_done;
    lat_ms.push_back((r.t_done - r.t_submit) * 1e-6);
  }
  if (s.graph) {
    s.graph->busy = false;
    s.graph = nullptr;
  }
  if (s.off != UINT64_MAX) arena.release(s.off);
  s.off = UINT64_MAX;
  s.reqs.clear();
  s.out_at.clear();
}

// Admits the ready request at `it` (and, for a small complex64 request, the
// other ready small complex64 requests of its width) onto slot s.  Returns
// false, changing nothing, when its memory does not fit now.
bool ServerImpl::admit(Slot& s, std::deque<std::shared_ptr<Request>>::iterator it) {
  std::shared_ptr<Request> r = *it;
  s.graph = nullptr;
  s.off = UINT64_MAX;
  int mode = 0;
  if (r->small) {
    const GraphKey key{r->cp->plan, r->k, r->nb, r->storage};
    auto g = graphs.find(key);
    if (g != graphs.end() && !g->second->busy) {
      s.graph = g->second.get();
      mode = 1;
    } else if (g == graphs.end() && seen[key] >= 1 && graphs.size() < (size_t)opt.max_graphs &&
               graph_bytes + up256(r->footprint) <= graph_budget) {
      const uint64_t off = arena.alloc(r->footprint);
      if (off != UINT64_MAX) {
        auto e = std::make_unique<GraphEntry>();
        e->off = off;
        graph_bytes += up256(r->footprint);
        s.graph = e.get();
        graphs.emplace(key, std::move(e));
        mode = 1;
      }
    }
    ++seen[key];
  }
  std::vector<std::shared_ptr<Request>> members{r};
  if (mode == 0 && r->small && r->storage == TNC_STORE_C64 && opt.max_group > 1) {
    for (auto jt = ready.begin(); jt != ready.end() && (int)members.size() < opt.max_group; ++jt) {
      if (jt == it) continue;
      const Request& q = **jt;
      if (q.small && q.storage == TNC_STORE_C64 && q.h == r->h) {
        const GraphKey qk{q.cp->plan, q.k, q.nb, q.storage};
        if (graphs.count(qk)) continue;  // it has a graph of its own
        members.push_back(*jt);
      }
    }
    // the group's block; shed members until it fits
    while (!members.empty()) {
      uint64_t bytes = 0, seg = 0;
      for (auto& mp : members) {
        bytes += mp->footprint;
        seg += (uint64_t)mp->n_launches * (kSegHeader + kMaxArgBytes);
      }
      const uint64_t off = arena.alloc(bytes + up256(seg) + 256);
      if (off != UINT64_MAX) {
        s.off = off;
        break;
      }
      members.pop_back();
    }
    if (s.off == UINT64_MAX) return false;
    mode = members.size() > 1 ? 2 : 0;
  } else if (mode == 0) {
    s.off = arena.alloc(r->footprint);
    if (s.off == UINT64_MAX) return false;
  }
  if (mode == 1) s.graph->busy = true;
  // take the members off the ready queue (r last: `it` stays valid until then)
  for (size_t i = 1; i < members.size(); ++i) ready.erase(std::find(ready.begin(), ready.end(), members[i]));
  ready.erase(std::find(ready.begin(), ready.end(), r));
  s.reqs = members;
  const int64_t t = now_ns();
  for (auto& mp : members) {
    mp->state = R_RUNNING;
    mp->t_admit = t;
    mp->mode = mode;
  }
  int rc;
  if (mode == 1) rc = run_graph(s, *r, s.graph);
  else if (mode == 2) rc = run_group(s);
  else if (r->small && r->storage == TNC_STORE_C64 && s.off != UINT64_MAX && members.size() == 1 &&
           opt.max_group > 1)
    rc = run_group(s);  // a group of one: the same block layout
  else rc = run_plain(s, *r);
  if (rc == TNC_OK) rc = hipEventRecord(s.done, s.stream) == hipSuccess ? TNC_OK : TNC_E_DEVICE;
  if (rc) {
    for (auto& mp : members) {
      mp->rc = rc;
      if (mp->err.empty()) mp->err = r->err.empty() ? std::string("serving: launch failed") : r->err;
    }
    finish(s, false);
    cv_done.notify_all();
  }
  return true;
}

// A small complex64 request waits (up to group_window_us after it became
// ready) for more ready requests of its width, until max_group are there.
bool ServerImpl::holding(const Request& r, int64_t now) const {
  if (!r.small || r.storage != TNC_STORE_C64 || opt.max_group < 2 || opt.group_window_us <= 0) return false;
  if (now - r.t_ready >= (int64_t)opt.group_window_us * 1000) return false;
  int same = 0;
  for (const auto& q : ready)
    if (q->small && q->storage == TNC_STORE_C64 && q->h == r.h) ++same;
  return same < opt.max_group;
}

void ServerImpl::dispatcher_loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool progressed = false;
    // completions
    int inflight = 0;
    for (Slot& s : slots) {
      if (s.reqs.empty()) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) {
        inflight += (int)s.reqs.size();
        continue;
      }
      if (q != hipSuccess)
        for (auto& rp : s.reqs) {
          rp->rc = TNC_E_DEVICE;
          rp->err = std::string("serving: request execution: ") + hipGetErrorString(q);
        }
      finish(s, q == hipSuccess);
      progressed = true;
    }
    if (progressed) cv_done.notify_all();
    // admissions: oldest first; a request that does not fit lets younger
    // ones pass at most 16 times, then the queue waits for it
    bool held = false;
    const int64_t now = now_ns();
    for (size_t si = 0; si < slots.size() && !ready.empty(); ++si) {
      Slot& s = slots[si];
      if (!s.reqs.empty()) continue;
      for (auto it = ready.begin(); it != ready.end(); ++it) {
        Request& r = **it;
        if (holding(r, now)) {
          held = true;
          continue;
        }
        if (!admit(s, it)) {
          if (++r.bypassed > 16) break;
          continue;
        }
        inflight += (int)s.reqs.size();
        progressed = true;
        break;
      }
    }
    max_inflight = std::max(max_inflight, inflight);
    if (stop && ready.empty() && to_plan.empty() && inflight == 0) {
      bool planning = false;
      for (auto& kv : reqs)
        if (kv.second->state == R_PLANNING) planning = true;
      if (!planning) return;
    }
    if (!progressed) cv_dispatch.wait_for(lk, std::chrono::microseconds(inflight ? 20 : held ? 100 : 2000));
  }
}

}  // namespace tnc

using namespace tnc;

struct tnc_server_s {
  std::unique_ptr<ServerImpl> impl;
};

extern "C" {

int tnc_server_create(const tnc_server_options* opt, tnc_server_t* out) {
  if (!out) return TNC_E_INVALID;
  *out = nullptr;
  auto S = std::make_unique<ServerImpl>();
  if (opt) S->opt = *opt;
  tnc_server_options& o = S->opt;
  if (o.n_streams <= 0) o.n_streams = 4;
  if (o.n_planners <= 0) o.n_planners = 4;
  if (o.max_graphs <= 0) o.max_graphs = 256;
  if (o.max_group <= 0) o.max_group = 16;
  if (o.group_window_us < 0 || o.group_window_us > 10000000) return TNC_E_INVALID;
  if (o.small_bits < 0 || o.small_bits > 24 || o.n_streams > 16 || o.n_planners > 16 || o.max_group > 256 ||
      o.arena_bytes == 0)
    return TNC_E_INVALID;
  if (hipGetDevice(&S->device) != hipSuccess) return TNC_E_DEVICE;
  // cached graphs keep their regions: at most a quarter of the arena
  if (hipMalloc((void**)&S->arena_base, o.arena_bytes) != hipSuccess) return TNC_E_NOMEM;
  S->arena_bytes = o.arena_bytes;
  S->graph_budget = o.arena_bytes / 4;
  S->arena = Arena(o.arena_bytes);
  S->slots.resize(o.n_streams);
  for (int i = 0; i < o.n_streams; ++i) {
    Slot& s = S->slots[i];
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
      return TNC_E_DEVICE;
  }
  ServerImpl* raw = S.get();
  for (int i = 0; i < o.n_planners; ++i) S->planners.emplace_back([raw] { raw->planner_loop(); });
  S->dispatcher = std::thread([raw] { raw->dispatcher_loop(); });
  *out = new tnc_server_s{std::move(S)};
  return TNC_OK;
}

int tnc_server_set_tuning(tnc_server_t sv, int32_t boundary_bits, const tnc_options* o) {
  if (!sv || !o || boundary_bits < 1 || boundary_bits > 40) return TNC_E_INVALID;
  std::lock_guard<std::mutex> lk(sv->impl->mu);
  sv->impl->tuning[boundary_bits] = *o;
  return TNC_OK;
}

int tnc_server_submit(tnc_server_t sv, int32_t n, int32_t d, const tnc_c128* one_qubit, int32_t n_gate2,
                      const tnc_gate2* gates, int32_t n_batches, const uint8_t* bits, int32_t k, int32_t storage,
                      tnc_c128* out, uint64_t* id) {
  if (!sv || !one_qubit || (n_gate2 > 0 && !gates) || n_gate2 < 0 || n < 2 || d < 2 || n_batches < 1 ||
      !bits || !out || !id || k < 0 || (int64_t)n * (d + 1) > (1 << 24))
    return TNC_E_INVALID;
  ServerImpl& S = *sv->impl;
  auto r = std::make_shared<Request>();
  r->circuit.n = n;
  r->circuit.d = d;
  r->circuit.one.assign(one_qubit, one_qubit + (size_t)(d + 1) * n * 4);
  r->circuit.gates.assign(gates, gates + n_gate2);
  for (tnc_gate2& g : r->circuit.gates) {
    g.reserved = 0;
    if (g.kind == TNC_GATE_CZ) std::memset(g.m, 0, sizeof(g.m));
  }
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, &n, sizeof(n));
  h = fnv1a(h, &d, sizeof(d));
  h = fnv1a(h, r->circuit.one.data(), r->circuit.one.size() * sizeof(tnc_c128));
  h = fnv1a(h, r->circuit.gates.data(), r->circuit.gates.size() * sizeof(tnc_gate2));
  r->hash = h;
  r->nb = n_batches;
  r->k = k;
  r->storage = storage;
  r->bits.assign(bits, bits + (size_t)n_batches * n);
  r->out = out;
  r->t_submit = now_ns();
  std::lock_guard<std::mutex> lk(S.mu);
  if (S.stop) return TNC_E_INVALID;
  r->id = S.next_id++;
  if (!S.first_submit) S.first_submit = r->t_submit;
  S.reqs[r->id] = r;
  S.to_plan.push_back(r);
  S.cv_plan.notify_one();
  *id = r->id;
  return TNC_OK;
}

int tnc_server_wait(tnc_server_t sv, uint64_t id, tnc_request_stats* st) {
  if (!sv) return TNC_E_INVALID;
  ServerImpl& S = *sv->impl;
  std::unique_lock<std::mutex> lk(S.mu);
  auto it = S.reqs.find(id);
  if (it == S.reqs.end()) return TNC_E_INVALID;
  std::shared_ptr<Request> r = it->second;
  S.cv_done.wait(lk, [&] { return r->state == R_DONE; });
  if (st) {
    st->queue_ms = (r->t_admit ? r->t_admit - r->t_submit : 0) * 1e-6;
    st->plan_ms = (r->t_ready - r->t_submit) * 1e-6;
    st->run_ms = (r->t_admit ? r->t_done - r->t_admit : 0) * 1e-6;
    st->total_ms = (r->t_done - r->t_submit) * 1e-6;
    st->boundary_bits = r->h;
    st->mode = r->mode;
  }
  const int rc = r->rc;
  if (rc) set_error_message(rc, r->err);
  S.reqs.erase(it);
  return rc;
}

int tnc_server_summary(tnc_server_t sv, tnc_server_stats* st) {
  if (!sv || !st) return TNC_E_INVALID;
  ServerImpl& S = *sv->impl;
  std::lock_guard<std::mutex> lk(S.mu);
  std::memset(st, 0, sizeof(*st));
  st->completed = (int64_t)S.n_done;
  st->graph_launches = (int64_t)S.n_graph_launch;
  st->graph_builds = (int64_t)S.n_graph_build;
  st->graph_failures = (int64_t)S.n_graph_failed;
  st->groups = (int64_t)S.n_groups;
  st->grouped_requests = (int64_t)S.n_grouped_reqs;
  st->grouped_launches = (int64_t)S.n_grouped_launches;
  st->plain_launches = (int64_t)S.n_plain;
  st->plan_cache_hits = (int64_t)S.plan_hits;
  st->plan_cache_misses = (int64_t)S.plan_misses;
  st->max_inflight = S.max_inflight;
  std::vector<double> l = S.lat_ms;
  std::sort(l.begin(), l.end());
  if (!l.empty()) {
    auto q = [&](double f) { return l[std::min(l.size() - 1, (size_t)(f * (l.size() - 1) + 0.5))]; };
    st->latency_ms_p50 = q(0.5);
    st->latency_ms_p99 = q(0.99);
    st->latency_ms_max = l.back();
  }
  if (S.last_done > S.first_submit) st->elapsed_s = (S.last_done - S.first_submit) * 1e-9;
  return TNC_OK;
}

int tnc_debug_arena_check(uint64_t seed, int32_t n_ops) {
  // random first-fit allocations and releases against an explicit model:
  // no two live blocks overlap, every block lies inside the arena, and
  // after releasing everything the free space is one block again
  if (n_ops < 0) return TNC_E_INVALID;
  const uint64_t size = 1ull << 24;
  Arena ar(size);
  std::map<uint64_t, uint64_t> live;  // offset -> bytes
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
  auto rnd = [&]() {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return x;
  };
  for (int i = 0; i < n_ops; ++i) {
    if (live.empty() || rnd() % 3 != 0) {
      const uint64_t bytes = 1 + rnd() % (size / 16);
      const uint64_t off = ar.alloc(bytes);
      if (off == UINT64_MAX) continue;
      const uint64_t len = (bytes + 255) & ~uint64_t(255);
      if (off % 256 != 0 || off + len > size) return set_error_message(TNC_E_INVALID, "block outside the arena");
      auto nx = live.lower_bound(off);
      if (nx != live.end() && nx->first < off + len) return set_error_message(TNC_E_INVALID, "overlap");
      if (nx != live.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second > off) return set_error_message(TNC_E_INVALID, "overlap");
      }
      live[off] = len;
    } else {
      auto it = live.begin();
      std::advance(it, (long)(rnd() % live.size()));
      ar.release(it->first);
      live.erase(it);
    }
  }
  for (auto& kv : live) ar.release(kv.first);
  if (ar.largest() != size) return set_error_message(TNC_E_INVALID, "free space not coalesced");
  return TNC_OK;
}

void tnc_server_destroy(tnc_server_t sv) {
  if (!sv) return;
  ServerImpl& S = *sv->impl;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stop = true;
  }
  S.cv_plan.notify_all();
  S.cv_dispatch.notify_all();
  for (std::thread& t : S.planners) t.join();
  S.dispatcher.join();
  for (auto& g : S.graphs)
    if (g.second->exec) (void)hipGraphExecDestroy(g.second->exec);
  for (Slot& s : S.slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.h_in) (void)hipHostFree(s.h_in);
    if (s.h_out) (void)hipHostFree(s.h_out);
  }
  for (auto& kv : S.plans)
    if (kv.second->plan) tnc_release(kv.second->plan);
  if (S.arena_base) (void)hipFree(S.arena_base);
  delete sv;
}

}  // extern "C"
