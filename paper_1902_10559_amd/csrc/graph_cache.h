// A cache of instantiated HIP graphs shared by the iterative solvers.
//
// A solve looks its graph up (or captures and instantiates it), launches it
// any number of times, then releases it, which records an event after its
// last launch.  An entry in use (between lookup and release) is never
// evicted, so another thread cannot destroy a graph that a solve is about to
// launch; an idle entry is evicted least recently used first, and only after
// its last launch has completed, so an asynchronous solve's graph is never
// destroyed while it still runs.
#pragma once

#include <map>
#include <mutex>

#include "device.h"
#include "internal.h"

namespace ss {

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  uint64_t last_use = 0;
  int users = 0;
};

template <class Key>
class GraphCache {
 public:
  explicit GraphCache(size_t cap) : cap_(cap) {}

  // Finds or builds the graph for `key` on `device` and marks it in use.
  // `capture(stream)` enqueues the work to capture on the given stream.
  template <class Capture>
  ss_status acquire(const Key& key, int device, Capture&& capture, GraphEntry** out) {
    std::lock_guard<std::mutex> lock(mu_);
    auto it = execs_.find(key);
    if (it != execs_.end()) {
      it->second.users += 1;
      it->second.last_use = ++uses_;
      *out = &it->second;
      return SS_OK;
    }
    evict_idle();
    hipStream_t cs;
    auto sit = capture_streams_.find(device);
    if (sit == capture_streams_.end()) {
      SS_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      capture_streams_[device] = cs;
    } else {
      cs = sit->second;
    }
    SS_HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    capture(cs);
    hipGraph_t graph;
    const hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (ce != hipSuccess) return fail(SS_E_HIP, "graph capture failed: %s", hipGetErrorString(ce));
    hipGraphExec_t exec;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(SS_E_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
    hipEvent_t done;
    const hipError_t ee = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (ee != hipSuccess) {
      (void)hipGraphExecDestroy(exec);
      return fail(SS_E_HIP, "graph event creation failed: %s", hipGetErrorString(ee));
    }
    GraphEntry& e = execs_[key];
    e.exec = exec;
    e.done = done;
    e.users = 1;
    e.last_use = ++uses_;
    *out = &e;
    return SS_OK;
  }

  // Destroys an entry that this caller acquired and never launched (its
  // capture did not complete as intended).
  void drop(const Key& key) {
    std::lock_guard<std::mutex> lock(mu_);
    auto it = execs_.find(key);
    if (it == execs_.end()) return;
    (void)hipEventDestroy(it->second.done);
    (void)hipGraphExecDestroy(it->second.exec);
    execs_.erase(it);
  }

  // Ends a solve's use of its graph; `st` is the stream it was launched on.
  void release(GraphEntry* e, hipStream_t st) {
    std::lock_guard<std::mutex> lock(mu_);
    (void)hipEventRecord(e->done, st);
    e->users -= 1;
  }

 private:
  // Drops idle entries, least recently used first, until there is room for
  // one more (if every entry is in use the cache grows past its cap).
  void evict_idle() {
    while (execs_.size() >= cap_) {
      auto victim = execs_.end();
      for (auto it = execs_.begin(); it != execs_.end(); ++it)
        if (it->second.users == 0 && (victim == execs_.end() || it->second.last_use < victim->second.last_use))
          victim = it;
      if (victim == execs_.end()) return;
      (void)hipEventSynchronize(victim->second.done);
      (void)hipEventDestroy(victim->second.done);
      (void)hipGraphExecDestroy(victim->second.exec);
      execs_.erase(victim);
    }
  }

  std::mutex mu_;
  std::map<Key, GraphEntry> execs_;
  std::map<int, hipStream_t> capture_streams_;
  uint64_t uses_ = 0;
  size_t cap_;
};

}  // namespace ss
