// HE Mul serving loop with continuous batching.
//
// Requests (ring, level, operands, output) are queued on submission with a
// host timestamp.  he_server_progress() is non-blocking: it retires batches
// whose completion event has fired (recording each request's latency and
// returning its workspace), then, for every ring with spare in-flight
// capacity, admits queued requests in arrival order while their workspace
// fits the ring's arena (HBM footprint) and launches them as one batched HE
// Mul on that ring's stream.  Requests arriving while earlier batches run
// join the next batch; batches of different rings run concurrently on their
// own streams.  While a ring has a batch in flight, a batch that is not full
// may be held back for a bounded time so that arrivals coalesce.  All device
// memory (context tables, evaluation keys, arenas) belongs to the caller; the
// server only carves the arenas.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <deque>
#include <memory>
#include <string>
#include <vector>

#include "../../include/he_mi355x.h"

void he_set_last_error(const char* msg);  // defined with the library's other entry points

namespace {

using clk = std::chrono::steady_clock;

struct Request {
  uint64_t id;
  uint32_t level;
  const uint64_t *ct1, *ct2;
  uint64_t* out;
  clk::time_point arrival;
  size_t ws_bytes;
};

struct InFlight {
  he_batch* batch = nullptr;
  hipEvent_t done = nullptr;
  size_t arena_off = 0, arena_bytes = 0;
  uint32_t slot = 0;  // descriptor slot
  std::vector<Request> reqs;
};

struct Ring {
  he_ctx* ctx = nullptr;
  const uint64_t* evk = nullptr;
  hipStream_t stream = nullptr;
  uint8_t* arena = nullptr;  // workspace ring buffer (after the descriptor slots)
  size_t arena_size = 0;
  size_t footprint = 0;      // tables + evk + whole arena
  uint8_t* desc = nullptr;   // max_inflight descriptor slots at the head of the caller's arena
  size_t desc_slot = 0;
  uint32_t next_slot = 0;
  std::deque<Request> queue;
  std::deque<InFlight> inflight;
};

struct Done {
  uint64_t id;
  double latency_s;
};

}  // namespace

struct he_server {
  he_server_cfg cfg{};
  std::vector<Ring> rings;
  std::vector<Done> done;
  std::string err;
  uint64_t batches = 0, requests_done = 0;
};

namespace {

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// The live workspace blocks of a ring are exactly its in-flight batches, in
// allocation order, and they are released in that order (one stream), so
// the arena is a ring buffer: the largest block that fits right now starts
// after the newest block, or at 0 when the tail of the arena is too short.
size_t arena_fit(const Ring& r, size_t& off) {
  if (r.inflight.empty()) {
    off = 0;
    return r.arena_size;
  }
  const InFlight& first = r.inflight.front();
  const InFlight& last = r.inflight.back();
  const size_t end = last.arena_off + last.arena_bytes;
  if (last.arena_off >= first.arena_off) {  // not wrapped
    const size_t tail_room = r.arena_size - end, head_room = first.arena_off;
    if (tail_room >= head_room) {
      off = end;
      return tail_room;
    }
    off = 0;
    return head_room;
  }
  off = end;  // wrapped: free space lies between the newest and the oldest block
  return first.arena_off - end;
}

he_status set_err(he_server* s, he_status st, const char* msg) {
  s->err = msg;
  he_set_last_error(msg);
  return st;
}

}  // namespace

extern "C" {

he_status he_server_create(const he_server_cfg* cfg, he_server** out) {
  if (!cfg || !out || cfg->max_batch == 0 || cfg->max_inflight == 0) return HE_EINVAL;
  he_server* s = new he_server;
  s->cfg = *cfg;
  *out = s;
  return HE_OK;
}

size_t he_server_arena_min_bytes(const he_server_cfg* cfg) {
  if (!cfg || cfg->max_batch == 0 || cfg->max_inflight == 0) return 0;
  return he_batch_desc_bytes(cfg->max_batch) * cfg->max_inflight;
}

he_status he_server_add_ring(he_server* s, he_ctx* ctx, const uint64_t* d_evk, void* d_arena, size_t arena_bytes,
                             uint32_t* ring_id) {
  if (!s) return HE_EINVAL;
  if (!ctx || !d_evk || !d_arena || !ring_id) return set_err(s, HE_EINVAL, "null pointer");
  if (he_ctx_word_bytes(ctx) != 8) return set_err(s, HE_EUNSUPPORTED, "serving takes 64-bit-word contexts");
  const size_t desc = he_server_arena_min_bytes(&s->cfg);
  if (arena_bytes <= desc) return set_err(s, HE_ENOMEM, "arena smaller than the descriptor slots");
  const size_t footprint = he_ctx_table_bytes(ctx) + he_evk_bytes(ctx) + arena_bytes;
  size_t total = footprint;
  for (auto& r : s->rings) total += r.footprint;
  if (total > s->cfg.hbm_budget)
    return set_err(s, HE_ENOMEM, "context tables, evaluation keys and arenas exceed the HBM budget");
  Ring r;
  r.ctx = ctx;
  r.evk = d_evk;
  r.footprint = footprint;
  r.desc_slot = he_batch_desc_bytes(s->cfg.max_batch);
  r.desc = (uint8_t*)d_arena;
  r.arena = (uint8_t*)d_arena + desc;
  r.arena_size = arena_bytes - desc;
  if (hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking) != hipSuccess)
    return set_err(s, HE_EDEVICE, "stream creation failed");
  s->rings.push_back(std::move(r));
  *ring_id = (uint32_t)s->rings.size() - 1;
  return HE_OK;
}

he_status he_server_submit(he_server* s, uint32_t ring, uint64_t id, uint32_t level, const uint64_t* d_ct1,
                           const uint64_t* d_ct2, uint64_t* d_out) {
  if (!s) return HE_EINVAL;
  if (ring >= s->rings.size() || !d_ct1 || !d_ct2 || !d_out) return set_err(s, HE_EINVAL, "bad ring or null pointer");
  Ring& r = s->rings[ring];
  he_batch_item it{level, d_ct1, d_ct2, nullptr, d_out};
  const size_t ws = he_batch_workspace_bytes(r.ctx, &it, 1);
  if (ws == 0 || level < 2) return set_err(s, HE_ELEVEL, "level out of range");
  if (round256(ws) > r.arena_size) return set_err(s, HE_ENOMEM, "request larger than its ring arena");
  if (s->cfg.max_queue && r.queue.size() >= s->cfg.max_queue)
    return set_err(s, HE_EBUSY, "the ring's request queue is full");
  r.queue.push_back(Request{id, level, d_ct1, d_ct2, d_out, clk::now(), ws});
  return HE_OK;
}

he_status he_server_progress(he_server* s, uint32_t* launched) {
  if (!s) return HE_EINVAL;
  uint32_t nl = 0;
  for (auto& r : s->rings) {
    // retire finished batches (in stream order)
    while (!r.inflight.empty()) {
      InFlight& f = r.inflight.front();
      const hipError_t q = hipEventQuery(f.done);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return set_err(s, HE_EDEVICE, hipGetErrorString(q));
      const auto now = clk::now();
      for (auto& rq : f.reqs) {
        s->done.push_back(Done{rq.id, std::chrono::duration<double>(now - rq.arrival).count()});
        ++s->requests_done;
      }
      he_batch_destroy(f.batch);
      (void)hipEventDestroy(f.done);
      r.inflight.pop_front();  // releases its arena block
    }
    // admit and launch
    while (!r.queue.empty() && r.inflight.size() < s->cfg.max_inflight) {
      size_t off = 0;
      const size_t room = arena_fit(r, off);
      std::vector<Request> take;
      size_t bytes = 0;
      for (const auto& rq : r.queue) {  // arrival order; stop at the first that does not fit
        if (take.size() >= s->cfg.max_batch) break;
        const size_t nb = bytes + round256(rq.ws_bytes);
        if (nb > room) break;
        take.push_back(rq);
        bytes = nb;
      }
      if (take.empty()) break;  // wait for a retirement to free workspace
      // coalescing: with a batch of this ring already running, a batch that
      // is not full waits until its oldest request has waited hold_us
      if (!r.inflight.empty() && take.size() < s->cfg.max_batch && s->cfg.hold_us &&
          std::chrono::duration<double>(clk::now() - take.front().arrival).count() * 1e6 < s->cfg.hold_us)
        break;
      std::vector<he_batch_item> items;
      for (auto& rq : take) items.push_back(he_batch_item{rq.level, rq.ct1, rq.ct2, nullptr, rq.out});
      InFlight f;
      // descriptor slots are reused in launch order; with at most
      // max_inflight batches in flight the slot being reused has retired
      f.slot = r.next_slot;
      r.next_slot = (r.next_slot + 1) % s->cfg.max_inflight;
      he_status st = he_batch_create_async(r.ctx, items.data(), (uint32_t)items.size(), r.arena + off, bytes,
                                           r.desc + (size_t)f.slot * r.desc_slot, r.desc_slot, r.stream, &f.batch);
      if (st != HE_OK) return set_err(s, st, he_last_error());
      st = he_mul_batch(r.ctx, f.batch, r.evk, 0, r.stream);
      if (st != HE_OK || hipEventCreateWithFlags(&f.done, hipEventDisableTiming) != hipSuccess ||
          hipEventRecord(f.done, r.stream) != hipSuccess) {
        he_batch_destroy(f.batch);
        return set_err(s, st != HE_OK ? st : HE_EDEVICE, "batch launch failed");
      }
      f.arena_off = off;
      f.arena_bytes = bytes;
      f.reqs = std::move(take);
      for (size_t k = 0; k < f.reqs.size(); ++k) r.queue.pop_front();
      r.inflight.push_back(std::move(f));
      ++s->batches;
      ++nl;
    }
  }
  if (launched) *launched = nl;
  return HE_OK;
}

he_status he_server_poll(he_server* s, uint64_t* ids, double* latency_s, uint32_t max, uint32_t* n) {
  if (!s || !n || (max && (!ids || !latency_s))) return HE_EINVAL;
  const uint32_t k = (uint32_t)std::min<size_t>(max, s->done.size());
  for (uint32_t i = 0; i < k; ++i) {
    ids[i] = s->done[i].id;
    latency_s[i] = s->done[i].latency_s;
  }
  s->done.erase(s->done.begin(), s->done.begin() + k);
  *n = k;
  return HE_OK;
}

he_status he_server_stats(const he_server* s, uint64_t* queued, uint64_t* inflight, uint64_t* batches,
                          uint64_t* completed) {
  if (!s) return HE_EINVAL;
  uint64_t q = 0, f = 0;
  for (auto& r : s->rings) {
    q += r.queue.size();
    for (auto& b : r.inflight) f += b.reqs.size();
  }
  if (queued) *queued = q;
  if (inflight) *inflight = f;
  if (batches) *batches = s->batches;
  if (completed) *completed = s->requests_done;
  return HE_OK;
}

void he_server_destroy(he_server* s) {
  if (!s) return;
  for (auto& r : s->rings) {
    (void)hipStreamSynchronize(r.stream);
    for (auto& f : r.inflight) {
      he_batch_destroy(f.batch);
      (void)hipEventDestroy(f.done);
    }
    (void)hipStreamDestroy(r.stream);
  }
  delete s;
}

}  // extern "C"
