// Checks of the host build's thread helpers (host_par.hpp), built with g++
// by tests/test_host_par.py: prints, for a seeded input, a counting sort's
// pointer array and order, the first index of a predicate, and a parallel
// sum written at fixed positions, so that the test can compare runs with
// different thread counts and against a plain Python reference.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2307_08383_amd/csrc/host_par.hpp"

int main(int argc, char** argv) {
    const int64_t n = argc > 1 ? std::atoll(argv[1]) : 100000;
    const int32_t n_keys = argc > 2 ? std::atoi(argv[2]) : 97;
    // seeded keys (xorshift), some negative (dropped)
    std::vector<int32_t> key(n);
    uint64_t x = 88172645463325252ull;
    for (int64_t i = 0; i < n; ++i) {
        x ^= x << 13; x ^= x >> 7; x ^= x << 17;
        key[i] = (int32_t)(x % (uint64_t)(n_keys + 3)) - 3;   // -3..n_keys-1
    }
    std::vector<int64_t> ptr;
    std::vector<int32_t> out;
    ba::counting_sort(n, n_keys, [&](int64_t i) { return key[i]; }, ptr, out);
    // per-index work written at fixed positions
    std::vector<int64_t> sq(n);
    ba::parallel_for(n, 1000, [&](int64_t a, int64_t b, int) {
        for (int64_t i = a; i < b; ++i) sq[i] = (int64_t)key[i] * key[i] + i;
    });
    int64_t s = 0;
    for (int64_t i = 0; i < n; ++i) s += sq[i];
    std::printf("threads %d\n", ba::host_threads());
    std::printf("ptr");
    for (int32_t k = 0; k <= n_keys; ++k) std::printf(" %lld", (long long)ptr[k]);
    std::printf("\nout");
    for (size_t i = 0; i < out.size(); ++i) std::printf(" %d", out[i]);
    std::printf("\nsum %lld\n", (long long)s);
    // an exception thrown in a worker reaches the caller
    bool caught = false;
    try {
        ba::parallel_for(n, 100, [&](int64_t a, int64_t b, int) {
            if (a <= n / 2 && n / 2 < b) throw 7;   // the piece holding index n / 2
        });
    } catch (int v) {
        caught = v == 7;
    }
    std::printf("caught %d\n", caught ? 1 : 0);
    return 0;
}
