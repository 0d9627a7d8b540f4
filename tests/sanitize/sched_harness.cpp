// Host-only harness for the block scheduler of host-memory matching
// (paper_1805_08995_amd/csrc/cashash_sched.h), built with AddressSanitizer
// and UndefinedBehaviorSanitizer: random image sizes, pair lists (self
// pairs, repeats, unused images) and slot sizes, checking that every pair is
// visited exactly once, in a step of its own block pair, in the scheduler's
// block-pair order, with at most three blocks resident.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_1805_08995_amd/csrc/cashash_sched.h"

int main() {
    std::mt19937_64 rng(12345);
    int failures = 0;
    auto check = [&](bool ok, const char* what, int trial) {
        if (!ok) {
            std::fprintf(stderr, "trial %d: %s\n", trial, what);
            failures++;
        }
    };
    for (int trial = 0; trial < 400; ++trial) {
        const int n_img = (int)(rng() % 40);
        std::vector<int64_t> bytes(n_img);
        for (auto& b : bytes) b = 1 + (int64_t)(rng() % 1000);
        const int64_t n_pairs = n_img ? (int64_t)(rng() % 200) : 0;
        std::vector<int32_t> pairs(2 * n_pairs);
        for (auto& v : pairs) v = (int32_t)(rng() % (uint64_t)n_img);
        const int64_t slot = 1 + (int64_t)(rng() % 4000);
        cashash::Schedule s;
        const int r = cashash::plan_schedule(n_img, bytes.data(), n_pairs, pairs.data(), slot, s);
        bool too_big = false;
        for (int64_t p = 0; p < n_pairs; ++p)
            for (int k = 0; k < 2; ++k) too_big |= bytes[pairs[2 * p + k]] > slot;
        if (too_big) {
            check(r == -1, "an image above the slot size must be refused", trial);
            continue;
        }
        check(r == 0, "plan_schedule failed", trial);
        std::vector<int> seen(n_pairs, 0);
        for (int64_t p : s.order) {
            check(p >= 0 && p < n_pairs, "order holds a pair index out of range", trial);
            if (p >= 0 && p < n_pairs) seen[p]++;
        }
        for (int64_t p = 0; p < n_pairs; ++p) check(seen[p] == 1, "a pair not visited exactly once", trial);
        const int nb = (int)s.block_first.size() - 1;
        for (int b = 0; b < nb; ++b) {
            int64_t fill = 0;
            for (int i = s.block_first[b]; i < s.block_first[b + 1]; ++i) fill += bytes[s.block_images[i]];
            check(fill <= slot, "a block above the slot size", trial);
        }
        std::vector<int32_t> resident;
        for (size_t k = 0; k < s.steps.size(); ++k) {
            const cashash::SchedStep& st = s.steps[k];
            check(st.bi <= st.bk && st.bk < nb && st.pair_begin < st.pair_end, "bad step", trial);
            if (k > 0) {
                const cashash::SchedStep& pv = s.steps[k - 1];
                const int64_t a = (int64_t)pv.bi * 1000000 + (pv.bk == pv.bi ? 999999 : pv.bk);
                const int64_t b = (int64_t)st.bi * 1000000 + (st.bk == st.bi ? 999999 : st.bk);
                check(a < b, "steps out of the block-pair order", trial);
            }
            for (int64_t i = st.pair_begin; i < st.pair_end; ++i) {
                const int64_t p = s.order[i];
                int32_t x = s.block_of[pairs[2 * p]], y = s.block_of[pairs[2 * p + 1]];
                if (x > y) std::swap(x, y);
                check(x == st.bi && y == st.bk, "a pair in a step of other blocks", trial);
            }
            for (int32_t blk : {st.bi, st.bk})
                if (std::find(resident.begin(), resident.end(), blk) == resident.end()) {
                    if (resident.size() >= 3)
                        for (size_t q = 0; q < resident.size(); ++q)
                            if (resident[q] != st.bi && resident[q] != st.bk) {
                                resident.erase(resident.begin() + (int64_t)q);
                                break;
                            }
                    resident.push_back(blk);
                }
            check(resident.size() <= 3, "more than three blocks resident", trial);
        }
    }
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("scheduler harness ok\n");
    return 0;
}
