// Request server: continuous batching of dot / matrix-vector / matrix products
// over several fields on one GPU.
//
// One scheduling thread owns the device side.  Each pass it
//   1. retires launches whose completion event has fired (their requests are
//      done: footprint and slots are released),
//   2. admits waiting requests in arrival order while an in-flight slot and
//      enough of the HBM budget are free (a request that does not fit blocks
//      the ones behind it, so admission never reorders arrivals); optionally
//      a request estimated to take longer than exclusive_ns runs alone,
//   3. launches everything admitted: the dot requests of one field are fused
//      into one batched launch (descriptors staged through pinned memory,
//      results scattered back to each request's output), matrix-vector and
//      matrix products are launched one by one, each on a lane chosen by
//      its estimated device time (below).
// Lanes (three or more streams): every matrix product goes to stream 0
// (bound by the matrix cores, and a large one takes whole CUs: two products
// never share the chip, and a product never holds up streaming work queued
// behind it in another stream); a streaming request (matrix-vector product,
// fused dot batch) estimated to take at least short_ns goes to stream 1, a
// shorter one to the least-loaded of the remaining streams.  A HIP stream
// runs its launches in order, so a short request never waits behind a long
// one.  The server keeps matrix products admitted but unlaunched until
// fewer than matrix_depth (default 2) are outstanding on stream 0, and
// then releases the one with the shortest estimated time, or the oldest once
// it has waited longer than four times its own estimate (at least 2 ms), so
// that small products do not queue behind large ones and none waits
// forever.
// Requests that arrive while others run are therefore taken into the next
// launch as soon as capacity frees up.  In "plain" mode every request is one
// launch on one stream in arrival order: the baseline that serving is
// compared against.  In "fake device" mode nothing touches the GPU and each
// launch completes after a simulated time, so the scheduling logic can be
// exercised without a device.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fdot_internal.h"

fdot_status_t fd_launch_scatter(const void* src, void* const* dst, size_t count,
                                uint32_t elem_bytes, hipStream_t s);

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  fdot_request_t r;
  uint64_t fp = 0;
  fdot_timing_t t;
  bool done = false;
};

// Pinned staging for one batched dot launch: descriptors, destination
// pointers and the batch's results, mirrored on the device.
struct Slot {
  void* host = nullptr;
  void* dev = nullptr;
  bool busy = false;
};

struct Launch {
  std::vector<uint64_t> tickets;
  hipEvent_t ev = nullptr;
  int slot = -1;
  int stream = 0;     // index of the stream it was issued on
  uint64_t est = 0;   // estimated device time, counted in that stream's load
  uint64_t fake_done = 0;
  int32_t status = FDOT_OK;
  bool matrix = false;  // a matrix product counted in matrix_out
};

// Device bytes a request holds while admitted: its operands and result, plus
// the scratch the library takes for it (transposed or digit-split operands
// and the residue sum of a matrix product, copies of x for a matrix-vector
// product); an upper bound, used against the HBM budget.
uint64_t footprint_of(const fdot_request_t& r) {
  if (r.footprint) return r.footprint;
  const uint64_t e = r.field->info.elem_bytes;
  switch (r.op) {
    case FDOT_OP_DOT: return (2 * r.n + 1) * e;
    case FDOT_OP_GEMV: return (r.m * r.n + r.n + r.m) * e + 16 * (r.n * e + 272);
    case FDOT_OP_GEMM: {
      const uint64_t kp = (r.k + 127) / 128 * 128;
      return (r.m * r.k + r.k * r.n + r.m * r.n) * e + 4 * (r.m + r.n) * kp + 4 * r.m * r.n + 4096;
    }
  }
  return 0;
}

// Simulated device time of a request (fake-device mode only).
// Estimated device time of a request: streaming forms at HBM speed, matrix
// products at the rate of the path they take (int8 cores for centred int8
// residues; D^2 int8 digit products, D = 1..4 by the size of p, for the
// other residues up to 4278124237; the vector-ALU kernel beyond).  Used to
// pick the least-loaded stream, for the exclusive rule and for the simulated
// device; only its order of magnitude matters.
uint64_t est_ns(const fdot_request_t& r) {
  const fdot_field_info_t& I = r.field->info;
  const double e = (double)I.elem_bytes;
  double s = 5e-6;
  switch (r.op) {
    case FDOT_OP_DOT: s += 2.0 * r.n * e / 5e12; break;
    case FDOT_OP_GEMV: s += (double)r.m * r.n * e / 5e12; break;
    case FDOT_OP_GEMM: {
      const double ops = 2.0 * r.m * r.n * r.k;
      const uint64_t h = (I.p - 1) / 2;
      if (I.rep == FDOT_REP_CENTRED_I8) {
        s += ops / 1.5e15;
      } else if (I.rep != FDOT_REP_ZECH_U16 && I.p <= 4278124237ull) {
        const double d = h <= 127 ? 1 : h <= 32639 ? 2 : h <= 8355711 ? 3 : 4;
        s += d * d * (10e-6 + ops / 1.6e15);
      } else {
        s += ops / 1e13;
      }
      break;
    }
  }
  return (uint64_t)(s * 1e9);
}
uint64_t fake_ns(const fdot_request_t& r) { return est_ns(r); }

}  // namespace

struct fdot_server_s {
  fdot_server_cfg_t cfg;
  int device = 0;
  std::mutex mu;
  std::condition_variable wake;     // submit -> scheduler
  std::condition_variable progress; // scheduler -> drain / replay
  std::thread thread;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::unordered_map<uint64_t, Req> reqs;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> admitted;
  std::vector<Launch> inflight;
  bool heavy_inflight = false;  // an exclusive request is admitted or running
  std::vector<uint64_t> held;   // admitted matrix products not yet launched (matrix_depth)
  uint32_t matrix_out = 0;      // matrix-product launches outstanding on stream 0
  uint64_t used_fp = 0;
  uint32_t n_admitted = 0;  // admitted and not yet done
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> free_events;
  std::vector<Slot> slots;
  size_t slot_bytes = 0;
  uint32_t rr = 0;
  std::vector<uint64_t> load;  // per stream: estimated ns of work issued and not done
  fdot_server_stats_t st;

  // The stream of a launch whose estimated device time is est (the lanes of
  // the header comment).  Fewer than three streams: matrix products on
  // stream 0, the rest on the least-loaded other one.  Plain: the one stream.
  int pick_stream(const fdot_request_t& r, uint64_t est) {
    if (cfg.plain || streams.size() == 1) return 0;
    if (r.op == FDOT_OP_GEMM) return 0;
    int first = 1;
    if (streams.size() >= 3) {
      if (est >= cfg.short_ns) return 1;
      first = 2;
    }
    const int span = (int)streams.size() - first;
    int best = first + (int)(rr++ % (uint32_t)span);
    for (int i = first; i < (int)streams.size(); ++i)
      if (load[i] < load[best]) best = i;
    return best;
  }

  hipEvent_t get_event() {
    if (!free_events.empty()) {
      hipEvent_t e = free_events.back();
      free_events.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }

  int get_slot() {
    for (size_t i = 0; i < slots.size(); ++i)
      if (!slots[i].busy) {
        slots[i].busy = true;
        return (int)i;
      }
    if (slots.size() >= 64) return -1;
    Slot sl;
    if (hipHostMalloc(&sl.host, slot_bytes, hipHostMallocDefault) != hipSuccess) return -1;
    if (hipMalloc(&sl.dev, slot_bytes) != hipSuccess) {
      hipHostFree(sl.host);
      return -1;
    }
    sl.busy = true;
    slots.push_back(sl);
    return (int)slots.size() - 1;
  }

  // Launch one request by itself.
  fdot_status_t launch_one(Req& q, hipStream_t s) {
    const fdot_request_t& r = q.r;
    if (r.ready && hipStreamWaitEvent(s, (hipEvent_t)r.ready, 0) != hipSuccess)
      return FDOT_E_DEVICE;
    switch (r.op) {
      case FDOT_OP_DOT: {
        Workspace* w = nullptr;
        fdot_status_t stt = fd_workspace_get(s, 1, &w);
        if (stt != FDOT_OK) return stt;
        return fd_launch_dot(r.field, FDOT_ALGO_AUTO, r.a, r.b, r.n, r.out, w, s);
      }
      case FDOT_OP_GEMV: return fd_launch_gemv(r.field, r.m, r.n, r.a, r.n, r.b, r.out, s);
      case FDOT_OP_GEMM:
        return fd_launch_gemm(r.field, r.m, r.n, r.k, r.a, r.k, r.b, r.n, r.out, r.n, s);
    }
    return FDOT_E_INVALID_ARG;
  }

  void finish_launch(Launch& L, uint64_t now) {
    for (uint64_t tk : L.tickets) {
      Req& q = reqs[tk];
      if (!cfg.plain && est_ns(q.r) > cfg.exclusive_ns) heavy_inflight = false;
      q.done = true;
      q.t.done_ns = now;
      q.t.status = L.status;
      used_fp -= q.fp;
      --n_admitted;
      ++st.completed;
    }
    if (L.ev) free_events.push_back(L.ev);
    if (L.slot >= 0) slots[L.slot].busy = false;
    load[L.stream] -= L.est;
    if (L.matrix) --matrix_out;
  }

  void issue(std::vector<uint64_t> tickets, int si, uint64_t est, fdot_status_t stt, int slot) {
    hipStream_t s = streams[si];
    Launch L;
    L.matrix = !cfg.plain && tickets.size() == 1 && reqs[tickets[0]].r.op == FDOT_OP_GEMM;
    if (L.matrix) ++matrix_out;
    L.tickets = std::move(tickets);
    L.slot = slot;
    L.stream = si;
    L.est = est;
    L.status = stt;
    const uint64_t now = now_ns();
    uint64_t dur = 0;
    for (uint64_t tk : L.tickets) {
      Req& q = reqs[tk];
      q.t.launch_ns = now;
      q.t.batch_size = (uint32_t)L.tickets.size();
      q.t.stream = (uint32_t)si;
      dur = std::max(dur, fake_ns(q.r));
    }
    ++st.launches;
    if (cfg.fake_device) {
      L.fake_done = now + dur;
    } else if (stt == FDOT_OK) {
      L.ev = get_event();
      if (!L.ev || hipEventRecord(L.ev, s) != hipSuccess) {
        if (L.ev) free_events.push_back(L.ev);
        L.ev = nullptr;
        L.status = FDOT_E_DEVICE;
      }
    }
    inflight.push_back(std::move(L));
  }

  // Launch everything admitted (lock held).
  void launch_admitted() {
    std::vector<uint64_t> todo;
    todo.swap(admitted);
    if (cfg.plain || cfg.fake_device) {
      if (cfg.plain) {
        for (uint64_t tk : todo) {
          const uint64_t est = est_ns(reqs[tk].r);
          const int si = pick_stream(reqs[tk].r, est);
          load[si] += est;
          const fdot_status_t stt = cfg.fake_device ? FDOT_OK : launch_one(reqs[tk], streams[si]);
          issue({tk}, si, est, stt, -1);
        }
        return;
      }
    }
    // Group dot requests by field; others go one by one.
    std::map<fdot_field_t, std::vector<uint64_t>> dots;
    for (uint64_t tk : todo) {
      Req& q = reqs[tk];
      if (q.r.op == FDOT_OP_DOT) {
        dots[q.r.field].push_back(tk);
      } else if (q.r.op == FDOT_OP_GEMM) {
        held.push_back(tk);
      } else {
        const uint64_t est = est_ns(q.r);
        const int si = pick_stream(q.r, est);
        load[si] += est;
        const fdot_status_t stt = cfg.fake_device ? FDOT_OK : launch_one(q, streams[si]);
        issue({tk}, si, est, stt, -1);
      }
    }
    for (auto& kv : dots) {
      std::vector<uint64_t>& v = kv.second;
      for (size_t b = 0; b < v.size(); b += cfg.max_batch) {
        const size_t e = std::min(v.size(), b + (size_t)cfg.max_batch);
        std::vector<uint64_t> group(v.begin() + b, v.begin() + e);
        uint64_t est = 0;
        for (uint64_t tk : group) est += est_ns(reqs[tk].r);
        const int si = pick_stream(reqs[group[0]].r, est);
        hipStream_t s = streams[si];
        load[si] += est;
        if (cfg.fake_device) {
          issue(group, si, est, FDOT_OK, -1);
          continue;
        }
        if (group.size() == 1) {
          issue(group, si, est, launch_one(reqs[group[0]], s), -1);
          continue;
        }
        const int slot = get_slot();
        if (slot < 0) {  // no staging buffer free: launch these one by one
          for (uint64_t tk : group) issue({tk}, si, est_ns(reqs[tk].r), launch_one(reqs[tk], s), -1);
          continue;
        }
        const size_t n = group.size();
        char* h = (char*)slots[slot].host;
        char* d = (char*)slots[slot].dev;
        fdot_desc_t* hd = (fdot_desc_t*)h;
        void** hdst = (void**)(h + n * sizeof(fdot_desc_t));
        for (size_t i = 0; i < n; ++i) {
          const fdot_request_t& r = reqs[group[i]].r;
          hd[i].x = r.a;
          hd[i].y = r.b;
          hd[i].n = r.n;
          hdst[i] = r.out;
        }
        const size_t bytes = n * (sizeof(fdot_desc_t) + sizeof(void*));
        fdot_status_t stt = FDOT_OK;
        Workspace* w = nullptr;
        for (uint64_t tk : group) {
          const fdot_request_t& r = reqs[tk].r;
          if (r.ready && hipStreamWaitEvent(s, (hipEvent_t)r.ready, 0) != hipSuccess)
            stt = FDOT_E_DEVICE;
        }
        if (stt == FDOT_OK && hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
          stt = FDOT_E_DEVICE;
        if (stt == FDOT_OK) stt = fd_workspace_get(s, n, &w);
        void* results = d + bytes;
        if (stt == FDOT_OK)
          stt = fd_launch_many(kv.first, FDOT_ALGO_AUTO, n, (const fdot_desc_t*)d, results, w, s);
        if (stt == FDOT_OK)
          stt = fd_launch_scatter(results, (void* const*)(d + n * sizeof(fdot_desc_t)), n,
                                  kv.first->info.elem_bytes, s);
        issue(group, si, est, stt, slot);
      }
    }
  }

  // Launch held matrix products while fewer than matrix_depth are
  // outstanding: the shortest estimate first, the oldest once it has waited
  // more than max(2 ms, 4 x its estimate).  Returns whether any launched.
  bool release_held() {
    bool any = false;
    const uint64_t now = now_ns();
    while (!held.empty() && matrix_out < cfg.matrix_depth) {
      size_t pick = 0;
      for (size_t i = 1; i < held.size(); ++i)
        if (est_ns(reqs[held[i]].r) < est_ns(reqs[held[pick]].r)) pick = i;
      size_t oldest = 0;
      for (size_t i = 1; i < held.size(); ++i)
        if (reqs[held[i]].t.admit_ns < reqs[held[oldest]].t.admit_ns) oldest = i;
      const Req& o = reqs[held[oldest]];
      const uint64_t patience = std::max<uint64_t>(2000000, 4 * est_ns(o.r));
      if (now - o.t.admit_ns > patience) pick = oldest;
      const uint64_t tk = held[pick];
      held.erase(held.begin() + (ptrdiff_t)pick);
      Req& q = reqs[tk];
      const uint64_t est = est_ns(q.r);
      load[0] += est;
      const fdot_status_t stt = cfg.fake_device ? FDOT_OK : launch_one(q, streams[0]);
      issue({tk}, 0, est, stt, -1);
      any = true;
    }
    return any;
  }

  void run() {
    if (!cfg.fake_device) hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      bool moved = false;
      const uint64_t now = now_ns();
      for (size_t i = 0; i < inflight.size();) {
        Launch& L = inflight[i];
        bool fin;
        if (cfg.fake_device) {
          fin = now >= L.fake_done;
        } else if (!L.ev) {
          fin = true;  // the launch failed; its requests complete with the error
        } else {
          const hipError_t q = hipEventQuery(L.ev);
          fin = q != hipErrorNotReady;
          if (fin && q != hipSuccess) L.status = FDOT_E_DEVICE;
        }
        if (fin) {
          finish_launch(L, now);
          inflight[i] = std::move(inflight.back());
          inflight.pop_back();
          moved = true;
        } else {
          ++i;
        }
      }
      while (!pending.empty() && n_admitted < cfg.max_inflight && !heavy_inflight) {
        Req& q = reqs[pending.front()];
        if (used_fp + q.fp > cfg.hbm_budget) break;
        if (!cfg.plain && est_ns(q.r) > cfg.exclusive_ns) {
          // runs alone: wait until nothing is admitted or in flight
          if (n_admitted > 0) break;
          heavy_inflight = true;
        }
        used_fp += q.fp;
        ++n_admitted;
        q.t.admit_ns = now_ns();
        admitted.push_back(pending.front());
        pending.pop_front();
        moved = true;
      }
      st.peak_footprint = std::max(st.peak_footprint, used_fp);
      st.peak_inflight = std::max(st.peak_inflight, n_admitted);
      if (!admitted.empty()) {
        launch_admitted();
        moved = true;
      }
      if (!held.empty() && release_held()) moved = true;
      if (moved) progress.notify_all();
      if (stop && pending.empty() && admitted.empty() && held.empty() && inflight.empty()) break;
      if (!moved) {
        if (inflight.empty())
          wake.wait_for(lk, std::chrono::milliseconds(1));
        else {  // poll completions closely while work is on the device
          lk.unlock();
          std::this_thread::yield();
          lk.lock();
        }
      }
    }
    progress.notify_all();
  }
};

extern "C" {

fdot_status_t fdot_server_create(const fdot_server_cfg_t* cfg, fdot_server_t* out) {
  if (!out) return FDOT_E_INVALID_ARG;
  *out = nullptr;
  fdot_server_cfg_t c;
  memset(&c, 0, sizeof c);
  c.hbm_budget = 64ull << 30;
  c.max_inflight = 256;
  c.max_queue = 4096;
  c.streams = 4;
  c.max_batch = 4096;
  if (cfg) {
    if (cfg->hbm_budget) c.hbm_budget = cfg->hbm_budget;
    if (cfg->max_inflight) c.max_inflight = cfg->max_inflight;
    if (cfg->max_queue) c.max_queue = cfg->max_queue;
    if (cfg->streams) c.streams = cfg->streams;
    if (cfg->max_batch) c.max_batch = cfg->max_batch;
    c.fake_device = cfg->fake_device;
    c.plain = cfg->plain;
    c.exclusive_ns = cfg->exclusive_ns;
    c.short_ns = cfg->short_ns;
    c.matrix_depth = cfg->matrix_depth;
  }
  if (c.matrix_depth == 0) c.matrix_depth = 2;
  if (c.exclusive_ns == 0) c.exclusive_ns = ~0ull;  // off
  if (c.short_ns == 0) c.short_ns = 100000;
  if (c.streams > 64) return FDOT_E_INVALID_ARG;
  fdot_server_s* s = new (std::nothrow) fdot_server_s;
  if (!s) return FDOT_E_NOMEM;
  s->cfg = c;
  memset(&s->st, 0, sizeof s->st);
  s->slot_bytes = (size_t)c.max_batch * (sizeof(fdot_desc_t) + sizeof(void*) + 8) + 64;
  if (!c.fake_device) {
    if (hipGetDevice(&s->device) != hipSuccess) {
      delete s;
      return FDOT_E_DEVICE;
    }
    const uint32_t ns = c.plain ? 1 : c.streams;
    for (uint32_t i = 0; i < ns; ++i) {
      hipStream_t st = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        for (hipStream_t x : s->streams) hipStreamDestroy(x);
        delete s;
        return FDOT_E_DEVICE;
      }
      s->streams.push_back(st);
    }
  } else {
    s->streams.assign(c.plain ? 1 : c.streams, nullptr);
  }
  s->load.assign(s->streams.size(), 0);
  if (!c.fake_device) {
    // pinned descriptor slots for the first batches, so that the measured
    // stream does not pay for pinned allocations
    std::vector<int> pre;
    for (uint32_t i = 0; i < std::min<uint32_t>(64, 2 * (uint32_t)s->streams.size()); ++i) {
      const int k = s->get_slot();
      if (k < 0) break;
      pre.push_back(k);
    }
    for (int k : pre) s->slots[k].busy = false;
  }
  s->thread = std::thread([s] { s->run(); });
  *out = s;
  return FDOT_OK;
}

fdot_status_t fdot_server_submit(fdot_server_t s, const fdot_request_t* req, uint64_t* ticket) {
  if (!s || !req || !ticket || !req->field) return FDOT_E_INVALID_ARG;
  const fdot_request_t& r = *req;
  if (r.op < FDOT_OP_DOT || r.op > FDOT_OP_GEMM || !r.out) return FDOT_E_INVALID_ARG;
  if (r.field->degree > 1) return FDOT_E_UNSUPPORTED;  // extension fields: not served
  if (r.op == FDOT_OP_DOT && r.n && (!r.a || !r.b)) return FDOT_E_INVALID_ARG;
  if (r.op == FDOT_OP_GEMV && (r.m == 0 || (r.n && (!r.a || !r.b)))) return FDOT_E_INVALID_ARG;
  if (r.op == FDOT_OP_GEMM && (r.m == 0 || r.n == 0 || (r.k && (!r.a || !r.b))))
    return FDOT_E_INVALID_ARG;
  const uint64_t fp = footprint_of(r);
  std::lock_guard<std::mutex> g(s->mu);
  if (fp > s->cfg.hbm_budget) {
    ++s->st.rejected;
    return FDOT_E_NOMEM;
  }
  if (s->pending.size() >= s->cfg.max_queue) return FDOT_E_BUSY;
  const uint64_t tk = s->next_ticket++;
  Req& q = s->reqs[tk];
  q.r = r;
  q.fp = fp;
  memset(&q.t, 0, sizeof q.t);
  q.t.submit_ns = now_ns();
  s->pending.push_back(tk);
  ++s->st.submitted;
  *ticket = tk;
  s->wake.notify_one();
  return FDOT_OK;
}

fdot_status_t fdot_server_poll(fdot_server_t s, uint64_t ticket, int* done, fdot_timing_t* t) {
  if (!s || !done) return FDOT_E_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return FDOT_E_NOT_FOUND;
  *done = it->second.done ? 1 : 0;
  if (t) *t = it->second.t;
  return FDOT_OK;
}

fdot_status_t fdot_server_drain(fdot_server_t s, uint64_t timeout_ms) {
  if (!s) return FDOT_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
  while (s->st.completed < s->st.submitted) {
    if (s->progress.wait_until(lk, until) == std::cv_status::timeout &&
        s->st.completed < s->st.submitted)
      return FDOT_E_BUSY;
  }
  return FDOT_OK;
}

fdot_status_t fdot_server_replay(fdot_server_t s, const fdot_request_t* reqs,
                                 const double* arrival_s, size_t count, fdot_timing_t* timings) {
  if (!s || (count && (!reqs || !arrival_s || !timings))) return FDOT_E_INVALID_ARG;
  std::vector<uint64_t> tickets(count, 0);
  const auto t0 = std::chrono::steady_clock::now();
  const uint64_t t0_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
                             t0.time_since_epoch()).count();
  for (size_t i = 0; i < count; ++i) {
    const auto due = t0 + std::chrono::nanoseconds((int64_t)(arrival_s[i] * 1e9));
    // sleep until shortly before the arrival, then spin to it
    const auto early = due - std::chrono::microseconds(200);
    if (std::chrono::steady_clock::now() < early) std::this_thread::sleep_until(early);
    while (std::chrono::steady_clock::now() < due) std::this_thread::yield();
    for (;;) {
      const fdot_status_t st = fdot_server_submit(s, &reqs[i], &tickets[i]);
      if (st == FDOT_OK) break;
      if (st != FDOT_E_BUSY) return st;
      std::this_thread::sleep_for(std::chrono::microseconds(50));  // queue full: back-pressure
    }
  }
  fdot_status_t st = fdot_server_drain(s, 600000);
  if (st != FDOT_OK) return st;
  std::lock_guard<std::mutex> g(s->mu);
  for (size_t i = 0; i < count; ++i) {
    // latency counts from the scheduled arrival: a submit that had to wait
    // (for the lock or for queue space) is waiting time of the request
    timings[i] = s->reqs[tickets[i]].t;
    timings[i].submit_ns = std::min(timings[i].submit_ns, t0_ns + (uint64_t)(arrival_s[i] * 1e9));
  }
  return FDOT_OK;
}

fdot_status_t fdot_server_stats(fdot_server_t s, fdot_server_stats_t* out) {
  if (!s || !out) return FDOT_E_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->st;
  return FDOT_OK;
}

fdot_status_t fdot_server_destroy(fdot_server_t s) {
  if (!s) return FDOT_E_INVALID_ARG;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->wake.notify_all();
  }
  s->thread.join();
  if (!s->cfg.fake_device) {
    for (hipStream_t x : s->streams) {
      fd_workspace_release(x);
      fd_scratch_release(x);
      hipStreamSynchronize(x);
      hipStreamDestroy(x);
    }
    for (hipEvent_t e : s->free_events) hipEventDestroy(e);
    for (Slot& sl : s->slots) {
      hipHostFree(sl.host);
      hipFree(sl.dev);
    }
  }
  delete s;
  return FDOT_OK;
}

}  // extern "C"
