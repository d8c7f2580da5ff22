// Host worker threads for the index builds (ba_create, the FSAI and network
// index structures).  Every helper writes results at positions fixed by the
// input alone, so the structures do not depend on the thread count or on
// the order in which the threads run.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace ba {

// BA_THREADS from the environment, else the hardware threads, at most 16
inline int host_threads() {
    static const int n = [] {
        if (const char* s = std::getenv("BA_THREADS")) {
            const int v = std::atoi(s);
            if (v > 0) return v;
        }
        const int hw = (int)std::thread::hardware_concurrency();
        return std::max(1, std::min(hw, 16));
    }();
    return n;
}

// Runs f(begin, end, thread) over [0, n) in pieces of `grain` taken in turn by
// the workers (thread < host_threads()); the first exception is rethrown.
template <typename F>
void parallel_for(int64_t n, int64_t grain, F&& f) {
    if (n <= 0) return;
    grain = std::max<int64_t>(1, grain);
    const int nt = (int)std::min<int64_t>(host_threads(), (n + grain - 1) / grain);
    if (nt <= 1) {
        f((int64_t)0, n, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    std::exception_ptr err;
    std::mutex mu;
    auto work = [&](int t) {
        try {
            for (;;) {
                const int64_t b = next.fetch_add(grain);
                if (b >= n) break;
                f(b, std::min(n, b + grain), t);
            }
        } catch (...) {
            std::lock_guard<std::mutex> g(mu);
            if (!err) err = std::current_exception();
            next.store(n);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
    work(0);
    for (auto& x : th) x.join();
    if (err) std::rethrow_exception(err);
}

// Stable counting sort of [0, n) by key(i) in [0, n_keys) (a negative key
// drops i): out[ptr[key] ..] lists the i of each key in ascending order; ptr
// has n_keys + 1 entries.  Threads take contiguous ranges of i and count per
// key first, with n_keys counters each (meant for key ranges up to a few
// million).
template <typename K, typename O>
void counting_sort(int64_t n, int32_t n_keys, K&& key, std::vector<int64_t>& ptr, std::vector<O>& out) {
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / (1 << 16)));
    const int64_t step = (n + nt - 1) / nt;
    std::vector<std::vector<int64_t>> cnt(nt, std::vector<int64_t>((size_t)n_keys, 0));
    parallel_for(nt, 1, [&](int64_t t0, int64_t t1, int) {
        for (int64_t t = t0; t < t1; ++t)
            for (int64_t i = t * step; i < std::min(n, (t + 1) * step); ++i) {
                const int32_t k = key(i);
                if (k >= 0) cnt[t][k]++;
            }
    });
    ptr.assign((size_t)n_keys + 1, 0);
    for (int32_t k = 0; k < n_keys; ++k) {
        int64_t s = ptr[k];
        for (int t = 0; t < nt; ++t) {
            const int64_t c = cnt[t][k];
            cnt[t][k] = s;   // the thread's first slot for key k
            s += c;
        }
        ptr[k + 1] = s;
    }
    out.resize((size_t)ptr[n_keys]);
    parallel_for(nt, 1, [&](int64_t t0, int64_t t1, int) {
        for (int64_t t = t0; t < t1; ++t)
            for (int64_t i = t * step; i < std::min(n, (t + 1) * step); ++i) {
                const int32_t k = key(i);
                if (k >= 0) out[cnt[t][k]++] = (O)i;
            }
    });
}

}  // namespace ba
