// Minimal host thread pool: parallel_for over [0, n) with dynamic scheduling.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace skelfmm {

inline int host_threads(int requested) {
    if (requested > 0) return requested;
    unsigned hc = std::thread::hardware_concurrency();
    return hc ? static_cast<int>(std::min(hc, 64u)) : 1;
}

// fn(i) for every i in [0, n); items are handed out `chunk` at a time.
// The first exception thrown by any worker is rethrown on the caller.
template <class Fn>
void parallel_for(int64_t n, int threads, Fn&& fn, int64_t chunk = 1) {
    if (n <= 0) return;
    threads = std::max(1, std::min<int>(threads, static_cast<int>((n + chunk - 1) / chunk)));
    if (threads == 1) {
        for (int64_t i = 0; i < n; ++i) fn(i);
        return;
    }
    std::atomic<int64_t> next{0};
    std::exception_ptr err;
    std::mutex mu;
    auto worker = [&]() {
        try {
            for (;;) {
                int64_t b = next.fetch_add(chunk);
                if (b >= n) break;
                int64_t e = std::min(n, b + chunk);
                for (int64_t i = b; i < e; ++i) fn(i);
            }
        } catch (...) {
            std::lock_guard<std::mutex> g(mu);
            if (!err) err = std::current_exception();
            next.store(n);
        }
    };
    std::vector<std::thread> pool;
    pool.reserve(threads - 1);
    for (int t = 1; t < threads; ++t) pool.emplace_back(worker);
    worker();
    for (auto& t : pool) t.join();
    if (err) std::rethrow_exception(err);
}

}  // namespace skelfmm
