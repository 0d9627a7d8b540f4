// Host-only harness for the library's host worker pool
// (paper_1805_08995_amd/csrc/cashash_pool.h), built with AddressSanitizer and
// UndefinedBehaviorSanitizer, and with ThreadSanitizer: repeated fork-join
// runs of random sizes (including empty and single-task runs) must visit
// every task exactly once, and split copies of random sizes and offsets must
// equal memcpy.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_1805_08995_amd/csrc/cashash_pool.h"

int main() {
    std::mt19937_64 rng(777);
    int failures = 0;
    for (int threads : {1, 2, 5, 8}) {
        cashash::WorkPool pool(threads);
        for (int trial = 0; trial < 300; ++trial) {
            const int64_t n = (int64_t)(rng() % 300);
            std::vector<std::atomic<int>> hits((size_t)n);
            for (auto& h : hits) h.store(0);
            pool.run(n, [&](int64_t i) { hits[(size_t)i].fetch_add(1); });
            for (int64_t i = 0; i < n; ++i)
                if (hits[(size_t)i].load() != 1) {
                    std::fprintf(stderr, "threads %d trial %d: task %lld ran %d times\n", threads, trial,
                                 (long long)i, hits[(size_t)i].load());
                    failures++;
                }
        }
        for (int trial = 0; trial < 60; ++trial) {
            const size_t bytes = (size_t)(rng() % (3u << 20));
            const size_t off = (size_t)(rng() % 64);
            std::vector<uint8_t> src(bytes + off), dst(bytes + off + 64, 0xAB), ref(bytes + off + 64, 0xAB);
            for (auto& b : src) b = (uint8_t)rng();
            cashash::parallel_copy(pool, dst.data() + off, src.data() + off, bytes, (size_t)(1 + rng() % 300000));
            if (bytes) std::memcpy(ref.data() + off, src.data() + off, bytes);
            if (dst != ref) {
                std::fprintf(stderr, "threads %d: copy of %zu bytes at %zu differs\n", threads, bytes, off);
                failures++;
            }
        }
    }
    if (failures) return 1;
    std::printf("pool harness ok\n");
    return 0;
}
