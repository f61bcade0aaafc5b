// Task executor for independent chains of TT operations: a fixed set of worker threads,
// each owning a HIP stream (non-blocking, default priority) and a device arena.  A task
// receives its worker's context, enqueues work on that stream, and the worker synchronises
// the stream before the task counts as done, so results are visible to every stream once
// run() returns.
#pragma once
#include <condition_variable>
#include <deque>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"

namespace ttfv {

class Pool {
 public:
  using Task = std::function<void(Ctx &)>;

  Pool(int nworkers, size_t arena_bytes, int device) {
    for (int i = 0; i < nworkers; ++i) {
      auto c = std::make_unique<Ctx>();
      HIP_CHECK(hipSetDevice(device));
      HIP_CHECK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->arena.init(arena_bytes);
      c->prepare();
      ctx_.push_back(std::move(c));
    }
    for (int i = 0; i < nworkers; ++i)
      threads_.emplace_back([this, i, device]() { loop(i, device); });
  }

  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto &t : threads_) t.join();
    for (auto &c : ctx_) {
      hipStream_t st = c->stream;
      c.reset();                       // frees the context's buffers while its stream exists
      if (st) (void)hipStreamDestroy(st);
    }
  }

  int size() const { return (int)ctx_.size(); }
  Ctx &ctx(int i) { return *ctx_[i]; }

  // Run all tasks and wait; the first exception raised by a task is rethrown here.  Several
  // threads may call run() at once (an ensemble of solvers shares one pool); each call waits
  // only for its own tasks.
  void run(std::vector<Task> tasks) {
    if (tasks.empty()) return;
    Group g;
    g.pending = (int)tasks.size();
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (auto &t : tasks) q_.push_back({std::move(t), &g});
    }
    cv_.notify_all();
    std::unique_lock<std::mutex> lk(mu_);
    g.cv.wait(lk, [&g] { return g.pending == 0; });
    if (g.err) std::rethrow_exception(g.err);
  }

  void set_sketch(int width, int power_iters) {
    for (auto &c : ctx_) {
      c->sketch_width = width;
      c->power_iters = power_iters;
    }
  }

 private:
  struct Group {
    int pending = 0;
    std::exception_ptr err;
    std::condition_variable cv;
  };

  void loop(int i, int device) {
    (void)hipSetDevice(device);
    for (;;) {
      std::pair<Task, Group *> item;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [this] { return stop_ || !q_.empty(); });
        if (stop_ && q_.empty()) return;
        item = std::move(q_.front());
        q_.pop_front();
      }
      std::exception_ptr e = nullptr;
      try {
        Scope sc(ctx_[i]->arena);
        item.first(*ctx_[i]);
        ctx_[i]->sync();
      } catch (...) {
        e = std::current_exception();
        (void)hipStreamSynchronize(ctx_[i]->stream);
      }
      std::lock_guard<std::mutex> lk(mu_);
      Group *g = item.second;
      if (e && !g->err) g->err = e;
      if (--g->pending == 0) g->cv.notify_all();
    }
  }

  std::vector<std::unique_ptr<Ctx>> ctx_;
  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::pair<Task, Group *>> q_;
  bool stop_ = false;
};

}  // namespace ttfv
