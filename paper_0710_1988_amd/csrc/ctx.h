// Library context: stream, workspace pool, pinned staging buffer, kernel timing.
#pragma once

#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "common.h"

struct dbq_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;

  // ---- workspace pool: device buffers kept across calls, handed out per call
  struct Buf {
    void* p;
    size_t bytes;
    bool busy;
  };
  std::vector<Buf> pool;

  // ---- this device's copy of the allocation-free apply's static scratch array (its device
  //      address, looked up at dbq_create; null until then)
  void* scratch = nullptr;

  // ---- pinned host staging for scalar readbacks
  void* pinned = nullptr;
  size_t pinned_bytes = 0;

  // ---- timing of kernel launches: kind 0 = Dslash FP64, 1 = Dslash FP32, 2 = the FP32
  //      BiCGStab x/r update with its inner products (the XR step)
  bool timing = false;
  int timing_sample = 1;  // every timing_sample-th launch of a class is timed
  struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;  // recorded, not yet read
    std::vector<hipEvent_t> spare;
    double ms = 0;
    int64_t n = 0;
    double bytes = 0;
    int64_t calls = 0;  // launches seen; every TIMING_SAMPLE-th one is timed
  } timers[3];


  // ---- device accumulators for the algorithmic bytes of gated launches (timing only):
  //      [kind] bytes so far (kinds 0-2), [8 + 8 * kind + lattice] set while a Dslash launch has
  //      counted the lattice's links.  acct_seen = the values already added to the timers.
  unsigned long long* acct = nullptr;
  unsigned long long acct_seen[3] = {0, 0, 0};

  // ---- graph capture of the solver's inner iteration blocks: a private stream to capture on
  //      (the caller's stream may be the null stream, which cannot be captured) and, while a
  //      capture is open, the timed launch pairs recorded into the graph instead of the timers
  hipStream_t cap_stream = nullptr;
  struct GraphTimer {
    int kind;
    hipEvent_t begin, end;
    double bytes;  // host-counted algorithmic bytes (0 when the device counts them)
  };
  std::vector<GraphTimer>* cap_timers = nullptr;
  // odd-site scratch of the reduced operator's first half step, owned by a solve that captures
  // its iterations (a graph replays the pointers it was captured with); null: taken per launch
  void* schur_tmp = nullptr;
  size_t schur_tmp_bytes = 0;

  // ---- Dslash launch shape chosen by timing, keyed by (kind, V, nrhs): rhs per thread (0: LDS
  //      tile kernel), rhs groups per site sweep (rhs per block for tiles), tile order
  std::map<std::tuple<int, int, int>, std::tuple<int, int, int>> ds_tune;
};

namespace dbq {

void* ws_get(dbq_ctx* c, size_t bytes);
void ws_release(dbq_ctx* c, void* p);
void* pinned_get(dbq_ctx* c, size_t bytes);

// RAII: everything taken from the pool inside a scope is returned at its end
struct WsScope {
  dbq_ctx* c;
  size_t mark;
  WsScope(const WsScope&) = delete;
  WsScope& operator=(const WsScope&) = delete;
  explicit WsScope(dbq_ctx* ctx);
  ~WsScope();
  template <typename T>
  T* get(size_t count) {
    return reinterpret_cast<T*>(take(count * sizeof(T)));
  }
  void* take(size_t bytes);
  std::vector<size_t> taken;
};

// Timing brackets around one launch; every c->timing_sample-th launch of a class is timed (each
// pair of events adds a few microseconds to the stream).  ev_out is null for a launch that is
// not sampled (timer_end then ignores it).
void timer_begin(dbq_ctx* c, int kind, hipEvent_t* ev_out);
void timer_end(dbq_ctx* c, int kind, hipEvent_t ev_begin, double bytes);
void timer_collect(dbq_ctx* c);
// after a replay of a graph has completed: add the durations of the launches timed inside it
void graph_timers_add(dbq_ctx* c, const std::vector<dbq_ctx::GraphTimer>& g);
// return a graph's timing events to the spare lists
void graph_timers_release(dbq_ctx* c, std::vector<dbq_ctx::GraphTimer>& g);

}  // namespace dbq
