// Host-side resumable tasks for the TT algorithms.
//
// An algorithm that must read device results on the host (a truncation rank,
// a residual, k) is written as a coroutine: at each such point it copies the
// values into pinned host memory and suspends with `co_await Sync{slot, s}`,
// which records an event on its stream.  A driver resumes it once the event
// has completed.  The blocking driver waits on the event; the batched driver
// polls the events of many independent problems from one host thread and
// resumes whichever is ready, so their device work overlaps on several
// streams without host threads.
#pragma once

#include <coroutine>
#include <exception>

#include "common.h"

namespace ttnt {

// A lazily started task; awaiting it runs it as a child of the awaiter.
struct Co {
  struct promise_type {
    std::coroutine_handle<> cont;
    std::exception_ptr exc;
    Co get_return_object() {
      return Co{std::coroutine_handle<promise_type>::from_promise(*this)};
    }
    std::suspend_always initial_suspend() noexcept { return {}; }
    struct Final {
      bool await_ready() noexcept { return false; }
      std::coroutine_handle<> await_suspend(std::coroutine_handle<promise_type> h) noexcept {
        std::coroutine_handle<> c = h.promise().cont;
        return c ? c : std::noop_coroutine();
      }
      void await_resume() noexcept {}
    };
    Final final_suspend() noexcept { return {}; }
    void return_void() {}
    void unhandled_exception() { exc = std::current_exception(); }
  };

  std::coroutine_handle<promise_type> h;

  explicit Co(std::coroutine_handle<promise_type> x) : h(x) {}
  Co(Co&& o) noexcept : h(o.h) { o.h = {}; }
  Co(const Co&) = delete;
  Co& operator=(const Co&) = delete;
  ~Co() {
    if (h) h.destroy();
  }

  bool done() const { return h.done(); }
  bool await_ready() const noexcept { return false; }
  std::coroutine_handle<> await_suspend(std::coroutine_handle<> parent) noexcept {
    h.promise().cont = parent;
    return h;
  }
  void await_resume() {
    if (h.promise().exc) std::rethrow_exception(h.promise().exc);
  }
};

// Where a suspended task waits: the event to poll and the coroutine to resume.
struct SyncSlot {
  hipEvent_t ev = nullptr;
  std::coroutine_handle<> resume;
};

// Suspends the awaiting task until the work issued so far on `s` is done.
struct Sync {
  SyncSlot* slot;
  hipStream_t s;
  bool await_ready() const noexcept { return false; }
  void await_suspend(std::coroutine_handle<> h) {
    TT_HIP(hipEventRecord(slot->ev, s));
    slot->resume = h;
  }
  void await_resume() const noexcept {}
};

// Starts `task` (or continues it) and returns when it has finished or is
// suspended at a Sync; true when finished.  Rethrows the task's exception.
inline bool resume_task(Co& task, SyncSlot& slot) {
  std::coroutine_handle<> r = slot.resume ? slot.resume : std::coroutine_handle<>(task.h);
  slot.resume = nullptr;
  r.resume();
  if (task.h.done()) {
    if (task.h.promise().exc) std::rethrow_exception(task.h.promise().exc);
    return true;
  }
  TT_REQUIRE(slot.resume, "task suspended outside a device synchronization");
  return false;
}

// Runs `task` to completion on the calling thread.
inline void run_blocking(Co& task, SyncSlot& slot) {
  slot.resume = nullptr;
  while (!resume_task(task, slot)) TT_HIP(hipEventSynchronize(slot.ev));
}

}  // namespace ttnt
