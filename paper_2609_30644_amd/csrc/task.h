// A planning instance as a coroutine: its synchronisation points suspend it
// instead of blocking a thread, so that one host thread can drive many
// instances whose device work is merged (batched and served planning), while
// a plain plan runs straight through.
#pragma once

#include <coroutine>
#include <exception>
#include <utility>

#include <hip/hip_runtime.h>

namespace mrpop {

// Result-carrying coroutine, started by the first resume().  Awaiting a Task
// from another coroutine runs it and continues the awaiting one when it ends.
template <class T>
class Task {
 public:
  struct promise_type {
    T value{};
    std::coroutine_handle<> cont;
    Task get_return_object() { return Task(std::coroutine_handle<promise_type>::from_promise(*this)); }
    std::suspend_always initial_suspend() noexcept { return {}; }
    struct Final {
      bool await_ready() noexcept { return false; }
      std::coroutine_handle<> await_suspend(std::coroutine_handle<promise_type> h) noexcept {
        const std::coroutine_handle<> c = h.promise().cont;
        return c ? c : std::noop_coroutine();
      }
      void await_resume() noexcept {}
    };
    Final final_suspend() noexcept { return {}; }
    void return_value(T v) { value = std::move(v); }
    void unhandled_exception() { std::terminate(); }
  };

  Task() = default;
  explicit Task(std::coroutine_handle<promise_type> h) : h_(h) {}
  Task(Task &&o) noexcept : h_(std::exchange(o.h_, {})) {}
  Task &operator=(Task &&o) noexcept {
    if (this != &o) {
      if (h_) h_.destroy();
      h_ = std::exchange(o.h_, {});
    }
    return *this;
  }
  Task(const Task &) = delete;
  Task &operator=(const Task &) = delete;
  ~Task() {
    if (h_) h_.destroy();
  }

  std::coroutine_handle<> handle() const { return h_; }
  bool done() const { return h_ && h_.done(); }
  const T &result() const { return h_.promise().value; }

  // awaited by another coroutine
  bool await_ready() const noexcept { return false; }
  std::coroutine_handle<> await_suspend(std::coroutine_handle<> c) noexcept {
    h_.promise().cont = c;
    return h_;
  }
  T await_resume() { return h_.promise().value; }

 private:
  std::coroutine_handle<promise_type> h_;
};

}  // namespace mrpop
