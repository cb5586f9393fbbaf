// parallel.hpp -- host threads for the planner's loops (no GPU code).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace bltc {

// Host threads a planning loop may use (at most 16: the planner runs beside
// the process's other work).
inline int64_t planner_threads()
{
    const unsigned hw = std::thread::hardware_concurrency();
    return std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 1, 16));
}

// f(i) for i in [0, n), indices handed out `grain` at a time; serial below
// `serial_below` items.  An exception thrown by f (say std::bad_alloc) stops
// the hand-out and is rethrown to the caller once every thread has joined.
template <class F>
void parallel_for(int64_t n, F&& f, int64_t grain = 16, int64_t serial_below = 64)
{
    const int64_t nthr = std::min<int64_t>(planner_threads(), (n + grain - 1) / grain);
    if (n < serial_below || nthr <= 1) {
        for (int64_t i = 0; i < n; ++i)
            f(i);
        return;
    }
    std::vector<std::thread> th;
    std::atomic<int64_t> next{0};
    std::mutex err_mu;
    std::exception_ptr err;
    for (int64_t t = 0; t < nthr; ++t)
        th.emplace_back([&]() {
            try {
                for (;;) {
                    int64_t i = next.fetch_add(grain);
                    if (i >= n)
                        break;
                    const int64_t e = std::min<int64_t>(n, i + grain);
                    for (; i < e; ++i)
                        f(i);
                }
            } catch (...) {
                next = n;   // no more work for anyone
                std::lock_guard<std::mutex> lock(err_mu);
                if (!err)
                    err = std::current_exception();
            }
        });
    for (auto& t : th)
        t.join();
    if (err)
        std::rethrow_exception(err);
}

// the same for a few heavy items: one index at a time, threads from 2 items on
template <class F>
void parallel_each(int64_t n, F&& f)
{
    parallel_for(n, f, 1, 2);
}

// std::sort on host threads: pieces sorted in parallel, then merged pairwise.
// With a strict total order (no equivalent elements) the result is the one
// std::sort gives.
template <class It, class Cmp>
void parallel_sort(It first, It last, Cmp cmp)
{
    const int64_t n = last - first;
    const int64_t nthr = planner_threads();
    if (n < (int64_t(1) << 16) || nthr == 1) {
        std::sort(first, last, cmp);
        return;
    }
    int64_t parts = 1;
    while (parts < nthr)
        parts *= 2;
    std::vector<int64_t> cut(static_cast<size_t>(parts) + 1);
    for (int64_t i = 0; i <= parts; ++i)
        cut[i] = n * i / parts;
    parallel_each(parts, [&](int64_t i) { std::sort(first + cut[i], first + cut[i + 1], cmp); });
    for (int64_t w = 1; w < parts; w *= 2)
        parallel_each(parts / (2 * w), [&](int64_t k) {
            std::inplace_merge(first + cut[2 * w * k], first + cut[2 * w * k + w],
                               first + cut[2 * w * k + 2 * w], cmp);
        });
}

}  // namespace bltc
