// Request loop of libgfpfft: continuous batching of polynomial products
// (section 3.3, Alg. Fast Convolution) over a fixed workspace budget.
//
// Structure: one queue of submitted requests (FIFO) and `slots` worker
// threads.  Each worker owns a HIP stream, events and an equal share of the
// workspace.  A free worker takes the requests waiting at the head of the
// queue while their combined workspace fits its share (the same chunk rule as
// gfp_polymul_batched) and enqueues one gfp_polymul_batched call per (field,
// transform size) class, smallest size first, with an event after each; it
// marks each class done as soon as its event completes, so the small requests
// of a mixed batch do not wait for its large ones.  Workers run
// independently, so a batch that arrives while another is on the device is
// launched at once on another stream and the two overlap.  With an express
// slot configured, the last worker only takes requests of small transform
// size (the earliest ones waiting, wherever they are in the queue), so those
// never queue behind large ones.
//
// Graphs: a chunk of C requests of one class is one launch sequence that
// depends on the requests only through the pad / unpad copy descriptors.
// Each slot keeps a descriptor table in device memory, and per
// (field, size, C) the sequence captured once with its copies reading that
// table; a chunk then costs one host-to-device copy of 3C descriptors (from
// pinned staging, a distinct region per chunk of the batch, since the copies
// run later on the stream) and one graph launch.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/gfp.h"
#include "gfp_internal.hpp"

namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct Request {
  gfp_request q;
  uint64_t n = 0;    // transform size
  uint64_t per = 0;  // workspace bytes of this request alone
  uint64_t cap = 1;  // requests of its size per workspace chunk
  bool done = false;
  gfp_result res{};
};

struct Slot {
  hipStream_t stream = nullptr;
  std::vector<hipEvent_t> events;  // one per class of a batch, created on demand
  uint64_t* ws = nullptr;          // chunk workspace (after the descriptor table)
  gfpk::CopyDesc* table = nullptr;  // device descriptor table, 3 max_batch entries
  gfpk::CopyDesc* stage = nullptr;  // pinned host staging, 6 max_batch entries
  std::map<std::tuple<const gfp_field*, uint64_t, uint64_t>, hipGraphExec_t> graphs;  // (field, n, C)
  std::set<std::tuple<const gfp_field*, uint64_t, uint64_t>> seen;                    // chunk shapes met so far
  uint64_t captures = 0, graph_launches = 0;
  bool express = false;  // takes only requests with n <= express_n
  std::thread thread;
};

// Captured chunk graphs kept per slot; beyond this the slot drops them all
// (between batches, when its stream is idle) and captures again.
constexpr size_t kMaxSlotGraphs = 256;

// Requests of one (field, transform size) class within a batch.
struct Class {
  const gfp_field* field;
  uint64_t n;
  std::vector<uint64_t> tickets;
  std::vector<gfp_polymul_desc> descs;
};

}  // namespace

struct gfp_server {
  gfp_server_config cfg{};
  uint64_t slot_bytes = 0;
  uint64_t express_n = 0;  // 0: no express slot
  void* ws_base = nullptr;
  void* table_base = nullptr;  // the slots' descriptor tables
  std::vector<Slot> slots;

  std::mutex mu;
  std::condition_variable cv_work;  // queue or stop changed
  std::condition_variable cv_done;  // a request finished
  std::deque<uint64_t> queue;       // tickets not yet admitted, arrival order
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_ticket = 1;
  uint64_t next_batch = 1;
  uint64_t unfinished = 0;  // submitted and not done
  uint32_t in_flight = 0;   // batches on the device
  bool stopping = false;
  gfp_server_stats st{};
};

namespace {

// Workspace a batch needs: per (field, size) class, min(count, cap) requests'
// worth (its chunks run one after another), and the classes run one after
// another too, so the maximum over classes.
struct Need {
  std::map<std::pair<const gfp_field*, uint64_t>, uint64_t> count;
  uint64_t bytes = 0;
  uint64_t with(const Request& r) const {
    auto it = count.find({r.q.field, r.n});
    const uint64_t c = (it == count.end() ? 0 : it->second) + 1;
    return std::max(bytes, std::min(c, r.cap) * r.per);
  }
  void add(const Request& r) {
    bytes = with(r);
    ++count[{r.q.field, r.n}];
  }
};

void finish(gfp_server* s, const std::vector<uint64_t>& tickets, int status, uint64_t t_done) {
  for (uint64_t t : tickets) {
    Request& r = s->reqs[t];
    r.res.status = status;
    r.res.t_done_ns = t_done;
    r.done = true;
  }
  s->unfinished -= tickets.size();
  s->st.completed += tickets.size();
}

// One class of a batch through the slot's chunk graphs: chunks of at most
// cap requests (the rule of gfp_polymul_batched).  Where a chunk's work is
// small (C n <= kPadElems), C is rounded up to a power of two (at most
// max_batch, within the slot's workspace) so that few distinct graphs serve
// all batch sizes; larger chunks keep their exact C, since padding them
// would cost real work.  A (field, size, C) is captured the second time it
// occurs; the first time its chunk runs eagerly, so that shapes seen once
// cost no capture.
constexpr uint64_t kPadElems = 1ull << 17;

int run_class_graphed(gfp_server* s, Slot& sl, const Class& c, size_t& staged) {
  const uint64_t per = gfpk::polymul_chunk_bytes(c.field, c.n, 1);
  const uint64_t cnt = c.descs.size();
  const uint64_t cap = std::min<uint64_t>(cnt, gfpk::chunk_cap(per));
  for (uint64_t i = 0; i < cnt; i += cap) {
    const uint64_t C = std::min<uint64_t>(cap, cnt - i);
    uint64_t Cb = 1;
    while (Cb < C) Cb <<= 1;
    if (Cb * c.n > kPadElems || Cb > s->cfg.max_batch || gfpk::polymul_chunk_bytes(c.field, c.n, Cb) > s->slot_bytes)
      Cb = C;
    const auto key = std::make_tuple(c.field, c.n, Cb);
    auto it = sl.graphs.find(key);
    if (it == sl.graphs.end() && sl.seen.insert(key).second) {
      // first occurrence: eager launches, no capture
      const int rc = gfp_polymul_batched(c.field, (uint32_t)C, c.descs.data() + i, sl.ws, s->slot_bytes, 0, sl.stream);
      if (rc != GFP_OK) return rc;
      continue;
    }
    if (staged + 3 * Cb > 6ull * s->cfg.max_batch) return GFP_EINVAL;  // cannot happen: Cb <= 2C
    gfpk::CopyDesc* h = sl.stage + staged;
    for (uint64_t j = 0; j < Cb; ++j) {
      if (j < C) {
        const gfp_polymul_desc& d = c.descs[i + j];
        h[j] = gfpk::CopyDesc{d.a, nullptr, d.la, d.ld_a};
        h[Cb + j] = gfpk::CopyDesc{d.b, nullptr, d.lb, d.ld_b};
        h[2 * Cb + j] = gfpk::CopyDesc{nullptr, d.c, d.la + d.lb - 1, d.ld_c};
      } else {  // padding entries: zero operands, nothing written back
        h[j] = h[Cb + j] = h[2 * Cb + j] = gfpk::CopyDesc{nullptr, nullptr, 0, 0};
      }
    }
    staged += 3 * Cb;
    if (it == sl.graphs.end()) {
      hipGraphExec_t ex = nullptr;
      int rc = gfpk::capture_polymul_chunk(c.field, c.n, Cb, sl.ws, sl.table, sl.stream, &ex);
      if (rc != GFP_OK) return rc;
      it = sl.graphs.emplace(key, ex).first;
      ++sl.captures;
    }
    ++sl.graph_launches;
    if (hipMemcpyAsync(sl.table, h, 3 * Cb * sizeof(gfpk::CopyDesc), hipMemcpyHostToDevice, sl.stream) != hipSuccess)
      return GFP_EDEVICE;
    if (hipGraphLaunch(it->second, sl.stream) != hipSuccess) return GFP_EDEVICE;
  }
  return GFP_OK;
}

// Enqueue the batch's classes on the slot's stream (smallest transform size
// first), each followed by an event, then wait for the events in order and
// mark each class done when its event completes.  Enqueueing runs without
// the lock on private copies of the requests.
void run_batch(gfp_server* s, Slot& sl, std::vector<Class>& classes, const std::vector<void*>& ready) {
  std::sort(classes.begin(), classes.end(), [](const Class& x, const Class& y) { return x.n < y.n; });
  std::vector<int> rc(classes.size(), GFP_OK);
  size_t enq = 0;  // classes with an event recorded after them
  int err = GFP_OK;
  for (void* ev : ready) {
    if (hipStreamWaitEvent(sl.stream, (hipEvent_t)ev, 0) != hipSuccess) err = GFP_EDEVICE;
  }
  if (sl.graphs.size() > kMaxSlotGraphs) {
    // the stream is idle between batches, so no graph is still running
    for (auto& g : sl.graphs) (void)hipGraphExecDestroy(g.second);
    sl.graphs.clear();
    sl.seen.clear();
  }
  const bool graphs = !(s->cfg.flags & GFP_SERVER_EAGER);
  size_t staged = 0;  // host staging entries used by this batch
  for (size_t i = 0; i < classes.size(); ++i) {
    if (err == GFP_OK) {
      Class& c = classes[i];
      err = graphs ? run_class_graphed(s, sl, c, staged)
                   : gfp_polymul_batched(c.field, (uint32_t)c.descs.size(), c.descs.data(), sl.ws, s->slot_bytes, 0,
                                         sl.stream);
    }
    rc[i] = err;
    while (sl.events.size() <= i) {
      hipEvent_t e = nullptr;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) break;
      sl.events.push_back(e);
    }
    // an event is recorded even after an error, so the stream has drained
    // before the requests go back to the caller
    if (sl.events.size() > i && hipEventRecord(sl.events[i], sl.stream) == hipSuccess) {
      enq = i + 1;
    } else {
      if (err == GFP_OK) err = GFP_EDEVICE;
      rc[i] = err;
      break;
    }
  }
  if (enq < classes.size()) {  // no event for the rest: wait for the whole stream
    if (hipStreamSynchronize(sl.stream) != hipSuccess && err == GFP_OK) err = GFP_EDEVICE;
  }
  for (size_t i = 0; i < classes.size(); ++i) {
    int st = i < enq ? rc[i] : err;
    if (i < enq && hipEventSynchronize(sl.events[i]) != hipSuccess && st == GFP_OK) st = GFP_EDEVICE;
    if (i >= enq && st == GFP_OK) st = GFP_EDEVICE;
    const uint64_t t_done = now_ns();
    std::lock_guard<std::mutex> lk(s->mu);
    finish(s, classes[i].tickets, st, t_done);
    s->cv_done.notify_all();
  }
}

void worker(gfp_server* s, size_t idx) {
  Slot& sl = s->slots[idx];
  (void)hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // an express slot only wakes for work it can take
    auto eligible = [&]() -> bool {
      if (!sl.express) return !s->queue.empty();
      for (uint64_t t : s->queue)
        if (s->reqs[t].n <= s->express_n) return true;
      return false;
    };
    s->cv_work.wait(lk, [&] { return s->stopping || eligible(); });
    if (!eligible()) {
      if (s->stopping) return;
      continue;
    }
    if (s->cfg.max_wait_us && !s->stopping && s->queue.size() < s->cfg.max_batch) {
      // wait for more requests, up to max_wait_us after the oldest one arrived
      const uint64_t deadline = s->reqs[s->queue.front()].res.t_submit_ns + 1000ull * s->cfg.max_wait_us;
      while (!s->stopping && !s->queue.empty() && s->queue.size() < s->cfg.max_batch) {
        const uint64_t t = now_ns();
        if (t >= deadline) break;
        s->cv_work.wait_for(lk, std::chrono::nanoseconds(deadline - t));
      }
      if (!eligible()) continue;  // another slot took them
    }
    // admission in arrival order while the workspace fits: from the head of
    // the queue (stopping at the first request that does not fit), or for
    // the express slot the small requests wherever they are
    Need need;
    std::vector<uint64_t> tickets;
    std::vector<Class> classes;
    std::vector<void*> ready;
    const uint64_t t_admit = now_ns();
    for (auto it = s->queue.begin(); it != s->queue.end() && tickets.size() < s->cfg.max_batch;) {
      Request& r = s->reqs[*it];
      if (sl.express && r.n > s->express_n) {
        ++it;
        continue;
      }
      if (need.with(r) > s->slot_bytes) break;
      need.add(r);
      r.res.t_admit_ns = t_admit;
      tickets.push_back(*it);
      auto c = std::find_if(classes.begin(), classes.end(),
                            [&](const Class& x) { return x.field == r.q.field && x.n == r.n; });
      if (c == classes.end()) {
        classes.push_back(Class{r.q.field, r.n, {}, {}});
        c = classes.end() - 1;
      }
      c->tickets.push_back(*it);
      c->descs.push_back(gfp_polymul_desc{r.q.a, r.q.la, r.q.ld_a, r.q.b, r.q.lb, r.q.ld_b, r.q.c, r.q.ld_c});
      if (r.q.ready_event) ready.push_back(r.q.ready_event);
      it = s->queue.erase(it);
    }
    const uint64_t bid = s->next_batch++;
    if (s->in_flight > 0) ++s->st.overlapped_batches;
    ++s->in_flight;
    ++s->st.batches;
    s->st.max_batch_size = std::max<uint64_t>(s->st.max_batch_size, tickets.size());
    s->st.max_batch_workspace = std::max(s->st.max_batch_workspace, need.bytes);
    const uint64_t t_launch = now_ns();
    for (uint64_t t : tickets) {
      Request& r = s->reqs[t];
      r.res.batch_id = bid;
      r.res.batch_size = (uint32_t)tickets.size();
      r.res.t_launch_ns = t_launch;
    }
    if (!s->queue.empty()) s->cv_work.notify_all();  // let other free slots take the rest
    lk.unlock();

    const uint64_t cap0 = sl.captures, gl0 = sl.graph_launches;
    run_batch(s, sl, classes, ready);

    lk.lock();
    --s->in_flight;
    s->st.graph_captures += sl.captures - cap0;
    s->st.graph_launches += sl.graph_launches - gl0;
  }
}

bool valid_request(const gfp_request* q) {
  if (!q || !q->field || !q->a || !q->b || !q->c || q->la == 0 || q->lb == 0) return false;
  if (q->ld_a < q->la || q->ld_b < q->lb || q->ld_c < q->la + q->lb - 1) return false;
  return true;
}

void release(gfp_server* s) {
  for (auto& sl : s->slots) {
    for (auto& g : sl.graphs) (void)hipGraphExecDestroy(g.second);
    for (hipEvent_t e : sl.events) (void)hipEventDestroy(e);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.stage) (void)hipHostFree(sl.stage);
  }
  if (s->ws_base) (void)hipFree(s->ws_base);
  if (s->table_base) (void)hipFree(s->table_base);
  delete s;
}

}  // namespace

extern "C" {

int gfp_server_create(const gfp_server_config* cfg, gfp_server** out) {
  if (!out) return GFP_EINVAL;
  *out = nullptr;
  if (!cfg) return GFP_EINVAL;
  gfp_server_config c = *cfg;
  if (c.slots == 0) c.slots = 2;
  if (c.max_batch == 0) c.max_batch = 256;
  if (c.max_pending == 0) c.max_pending = 65536;
  if (c.slots > 64 || c.express_log2n > 40 || (c.express_log2n && c.slots < 2)) return GFP_EINVAL;
  if (c.max_batch > 65535 || (c.flags & ~(uint32_t)GFP_SERVER_EAGER)) return GFP_EINVAL;
  // slot shares are multiples of 256 bytes; the descriptor tables are
  // allocated beside the workspace
  const uint64_t slot_bytes = (c.workspace_bytes / c.slots) & ~255ull;
  const uint64_t table_bytes = (3ull * c.max_batch * sizeof(gfpk::CopyDesc) + 255) & ~255ull;
  if (slot_bytes == 0) return GFP_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return GFP_EDEVICE;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return GFP_EDEVICE;
  if (c.device < 0) c.device = prev;
  if (c.device >= ndev) return GFP_EINVAL;

  gfp_server* s = new (std::nothrow) gfp_server();
  if (!s) return GFP_ENOMEM;
  s->cfg = c;
  s->slot_bytes = slot_bytes;
  s->st.slot_bytes = slot_bytes;
  int rc = GFP_OK;
  if (hipSetDevice(c.device) != hipSuccess) rc = GFP_EDEVICE;
  if (rc == GFP_OK && hipMalloc(&s->ws_base, slot_bytes * c.slots) != hipSuccess) {
    s->ws_base = nullptr;
    rc = GFP_ENOMEM;
  }
  if (rc == GFP_OK && hipMalloc(&s->table_base, table_bytes * c.slots) != hipSuccess) {
    s->table_base = nullptr;
    rc = GFP_ENOMEM;
  }
  s->express_n = c.express_log2n ? (1ull << c.express_log2n) : 0;
  s->slots.resize(c.slots);
  for (uint32_t i = 0; rc == GFP_OK && i < c.slots; ++i) {
    Slot& sl = s->slots[i];
    sl.table = (gfpk::CopyDesc*)((char*)s->table_base + i * table_bytes);
    sl.ws = (uint64_t*)((char*)s->ws_base + i * slot_bytes);
    sl.express = c.express_log2n && i + 1 == c.slots;
    if (hipHostMalloc((void**)&sl.stage, 6ull * c.max_batch * sizeof(gfpk::CopyDesc), hipHostMallocDefault) !=
        hipSuccess) {
      sl.stage = nullptr;
      rc = GFP_ENOMEM;
      break;
    }
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
      sl.stream = nullptr;
      rc = GFP_EDEVICE;
    }
  }
  (void)hipSetDevice(prev);
  if (rc != GFP_OK) {
    release(s);
    return rc;
  }
  for (uint32_t i = 0; i < c.slots; ++i) s->slots[i].thread = std::thread(worker, s, (size_t)i);
  *out = s;
  return GFP_OK;
}

int gfp_server_submit(gfp_server* s, const gfp_request* req, uint64_t* ticket) {
  if (!s || !ticket || !valid_request(req)) return GFP_EINVAL;
  Request r;
  r.q = *req;
  int rc = gfp_polymul_size(req->field, req->la, req->lb, &r.n);
  if (rc == GFP_OK) rc = gfp_polymul_workspace_size(req->field, req->la, req->lb, &r.per);
  if (rc != GFP_OK) return rc;
  r.cap = gfpk::chunk_cap(r.per);
  if (r.per > s->slot_bytes) return GFP_ENOMEM;
  // tables of a size not seen before are built here, on the caller's
  // thread, so that no worker stalls on them while its peers wait
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return GFP_EDEVICE;
  if (prev != s->cfg.device && hipSetDevice(s->cfg.device) != hipSuccess) return GFP_EDEVICE;
  rc = gfpk::prepare_tables(req->field, r.n);
  if (prev != s->cfg.device) (void)hipSetDevice(prev);
  if (rc != GFP_OK) return rc;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return GFP_ECANCELED;
  if (s->queue.size() >= s->cfg.max_pending) {
    ++s->st.rejected;
    return GFP_EAGAIN;
  }
  const uint64_t t = s->next_ticket++;
  r.res.t_submit_ns = now_ns();
  s->reqs.emplace(t, r);
  s->queue.push_back(t);
  ++s->unfinished;
  ++s->st.submitted;
  *ticket = t;
  s->cv_work.notify_all();  // an express slot may not be able to take it
  return GFP_OK;
}

int gfp_server_poll(gfp_server* s, uint64_t ticket, gfp_result* out) {
  if (!s || !out) return GFP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return GFP_EINVAL;
  if (!it->second.done) return GFP_EPENDING;
  *out = it->second.res;
  s->reqs.erase(it);
  return GFP_OK;
}

int gfp_server_wait(gfp_server* s, uint64_t ticket, int64_t timeout_us, gfp_result* out) {
  if (!s || !out) return GFP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->reqs.find(ticket) == s->reqs.end()) return GFP_EINVAL;
  // look the ticket up again after every wake-up: another thread may have
  // polled it meanwhile
  auto ready = [&] {
    auto it = s->reqs.find(ticket);
    return it == s->reqs.end() || it->second.done;
  };
  if (timeout_us < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return GFP_EPENDING;
  }
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return GFP_EINVAL;
  *out = it->second.res;
  s->reqs.erase(it);
  return GFP_OK;
}

int gfp_server_drain(gfp_server* s) {
  if (!s) return GFP_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->unfinished == 0; });
  return GFP_OK;
}

int gfp_server_get_stats(gfp_server* s, gfp_server_stats* out) {
  if (!s || !out) return GFP_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  return GFP_OK;
}

int gfp_server_destroy(gfp_server* s) {
  if (!s) return GFP_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    std::vector<uint64_t> cancelled(s->queue.begin(), s->queue.end());
    s->queue.clear();
    finish(s, cancelled, GFP_ECANCELED, now_ns());
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  for (auto& sl : s->slots)
    if (sl.thread.joinable()) sl.thread.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(s->cfg.device);
  release(s);
  (void)hipSetDevice(prev);
  return GFP_OK;
}

}  // extern "C"
