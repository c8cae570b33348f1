// dbq_ctx: workspace pool, pinned staging, kernel timing.
#include "ctx.h"

#include <algorithm>

namespace dbq {

void* ws_get(dbq_ctx* c, size_t bytes) {
  bytes = (bytes + 255) & ~size_t(255);
  int best = -1;
  for (size_t i = 0; i < c->pool.size(); ++i) {
    const auto& b = c->pool[i];
    if (!b.busy && b.bytes >= bytes && (best < 0 || b.bytes < c->pool[best].bytes)) best = int(i);
  }
  if (best >= 0) {
    c->pool[best].busy = true;
    return c->pool[best].p;
  }
  void* p = nullptr;
  const size_t alloc = std::max(bytes, size_t(1) << 20);
  hipError_t e = hipMalloc(&p, alloc);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // release idle buffers and retry once
    DBQ_HIP(hipStreamSynchronize(c->stream));
    for (auto it = c->pool.begin(); it != c->pool.end();) {
      if (!it->busy) {
        (void)hipFree(it->p);
        it = c->pool.erase(it);
      } else {
        ++it;
      }
    }
    e = hipMalloc(&p, alloc);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(DBQ_ENOMEM, "device allocation of " + std::to_string(alloc) + " bytes failed");
    }
  }
  c->pool.push_back({p, alloc, true});
  return p;
}

void ws_release(dbq_ctx* c, void* p) {
  for (auto& b : c->pool)
    if (b.p == p) b.busy = false;
}

void* pinned_get(dbq_ctx* c, size_t bytes) {
  if (c->pinned_bytes < bytes) {
    if (c->pinned) DBQ_HIP(hipHostFree(c->pinned));
    c->pinned = nullptr;
    const size_t alloc = std::max(bytes, size_t(1) << 16);
    DBQ_HIP(hipHostMalloc(&c->pinned, alloc, hipHostMallocDefault));
    c->pinned_bytes = alloc;
  }
  return c->pinned;
}

WsScope::WsScope(dbq_ctx* ctx) : c(ctx), mark(0) {}
WsScope::~WsScope() {
  for (size_t i = 0; i < taken.size(); ++i) ws_release(c, reinterpret_cast<void*>(taken[i]));
}
void* WsScope::take(size_t bytes) {
  void* p = ws_get(c, bytes);
  taken.push_back(reinterpret_cast<size_t>(p));
  return p;
}

void timer_begin(dbq_ctx* c, int kind, hipEvent_t* ev_out) {
  *ev_out = nullptr;
  if (!c->timing) return;
  auto& t = c->timers[kind];
  if ((t.calls++ % c->timing_sample) != 0) return;
  hipEvent_t e;
  if (!t.spare.empty()) {
    e = t.spare.back();
    t.spare.pop_back();
  } else {
    DBQ_HIP(hipEventCreate(&e));
  }
  DBQ_HIP(hipEventRecord(e, c->stream));
  *ev_out = e;
}

void timer_end(dbq_ctx* c, int kind, hipEvent_t ev_begin, double bytes) {
  if (!c->timing || !ev_begin) return;
  auto& t = c->timers[kind];
  hipEvent_t e;
  if (!t.spare.empty()) {
    e = t.spare.back();
    t.spare.pop_back();
  } else {
    DBQ_HIP(hipEventCreate(&e));
  }
  DBQ_HIP(hipEventRecord(e, c->stream));
  if (c->cap_timers) {
    // inside a capture: the pair is recorded by every replay of the graph
    c->cap_timers->push_back({kind, ev_begin, e, bytes});
    return;
  }
  t.ev.push_back({ev_begin, e});
  t.bytes += bytes;
  t.n += 1;
}

void graph_timers_add(dbq_ctx* c, const std::vector<dbq_ctx::GraphTimer>& g) {
  for (const auto& gt : g) {
    DBQ_HIP(hipEventSynchronize(gt.end));
    float ms = 0;
    DBQ_HIP(hipEventElapsedTime(&ms, gt.begin, gt.end));
    auto& t = c->timers[gt.kind];
    t.ms += ms;
    t.n += 1;
    t.bytes += gt.bytes;
  }
}

void graph_timers_release(dbq_ctx* c, std::vector<dbq_ctx::GraphTimer>& g) {
  for (const auto& gt : g) {
    c->timers[gt.kind].spare.push_back(gt.begin);
    c->timers[gt.kind].spare.push_back(gt.end);
  }
  g.clear();
}

void timer_collect(dbq_ctx* c) {
  for (auto& t : c->timers) {
    for (auto& pr : t.ev) {
      DBQ_HIP(hipEventSynchronize(pr.second));
      float ms = 0;
      DBQ_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
      t.ms += ms;
      t.spare.push_back(pr.first);
      t.spare.push_back(pr.second);
    }
    t.ev.clear();
  }
  if (c->acct) {
    unsigned long long v[3];
    DBQ_HIP(hipMemcpyAsync(v, c->acct, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    DBQ_HIP(hipStreamSynchronize(c->stream));
    for (int k = 0; k < 3; ++k) {
      c->timers[k].bytes += double(v[k] - c->acct_seen[k]);
      c->acct_seen[k] = v[k];
    }
  }
}

}  // namespace dbq
