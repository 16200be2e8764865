// Fork-join helper used by the host preparation (dynamic chunked scheduling).
#pragma once

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

namespace peers {

template <class Fn>
void parallel_for(int64_t n, int threads, Fn&& fn) {
  if (n <= 0) return;
  if (threads <= 1 || n == 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  int nt = (int)std::min<int64_t>(threads, n);
  std::atomic<int64_t> next{0};
  auto body = [&]() {
    for (;;) {
      int64_t i = next.fetch_add(1, std::memory_order_relaxed);
      if (i >= n) break;
      fn(i);
    }
  };
  std::vector<std::thread> pool;
  pool.reserve(nt - 1);
  for (int t = 1; t < nt; ++t) pool.emplace_back(body);
  body();
  for (auto& th : pool) th.join();
}

}  // namespace peers
