// Block scheduler for host-memory mode ("Three-Level Data Scheduling
// Strategy", matching subsection).  Images used by the pair list are packed,
// in index order, into blocks whose device footprint fits one slot.  Block
// pairs are visited in the paper's load order: block i stays resident while
// every later block k is matched against it, then block i is matched within
// itself, then block i + 1 takes its place.  At most three blocks are
// resident: the two being matched and the one being prefetched.
// Pure host code: no HIP calls.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

namespace cashash {

struct SchedStep {
    int32_t bi, bk;                // block pair (bi <= bk); bi == bk matches inside one block
    int64_t pair_begin, pair_end;  // range in Schedule::order
};

struct Schedule {
    std::vector<int32_t> block_of;     // image -> block, -1 if the image is unused
    std::vector<int32_t> block_first;  // block b holds block_images[block_first[b] .. block_first[b+1])
    std::vector<int32_t> block_images;
    std::vector<int64_t> order;        // pair indices in visiting order
    std::vector<SchedStep> steps;
    int64_t block_loads = 0;           // blocks brought to the device, 3 resident slots
    int64_t image_loads = 0;
};

// Returns 0, or -1 if an image alone exceeds slot_bytes, or -2 for bad input.
inline int plan_schedule(int32_t n_images, const int64_t* img_bytes, int64_t n_pairs, const int32_t* pairs,
                         int64_t slot_bytes, Schedule& s) {
    s = Schedule();
    if (n_images < 0 || n_pairs < 0 || slot_bytes <= 0) return -2;
    std::vector<char> used(n_images, 0);
    for (int64_t p = 0; p < n_pairs; ++p) {
        const int32_t q = pairs[2 * p], t = pairs[2 * p + 1];
        if (q < 0 || t < 0 || q >= n_images || t >= n_images) return -2;
        used[q] = used[t] = 1;
    }
    s.block_of.assign(n_images, -1);
    s.block_first.push_back(0);
    int64_t fill = 0;
    for (int32_t m = 0; m < n_images; ++m) {
        if (!used[m]) continue;
        if (img_bytes[m] > slot_bytes) return -1;
        if (fill + img_bytes[m] > slot_bytes && fill > 0) {
            s.block_first.push_back((int32_t)s.block_images.size());
            fill = 0;
        }
        s.block_of[m] = (int32_t)s.block_first.size() - 1;
        s.block_images.push_back(m);
        fill += img_bytes[m];
    }
    s.block_first.push_back((int32_t)s.block_images.size());
    const int32_t M = (int32_t)s.block_first.size() - 1;
    if (s.block_images.empty()) {
        s.block_first.assign(1, 0);
        return 0;
    }
    // bucket the pairs by unordered block pair, stable in pair order
    auto key = [&](int64_t p) {
        int32_t a = s.block_of[pairs[2 * p]], b = s.block_of[pairs[2 * p + 1]];
        if (a > b) std::swap(a, b);
        return (int64_t)a * M + b;
    };
    std::vector<int64_t> cnt((size_t)M * M + 1, 0);
    for (int64_t p = 0; p < n_pairs; ++p) cnt[key(p) + 1]++;
    for (size_t i = 1; i < cnt.size(); ++i) cnt[i] += cnt[i - 1];
    std::vector<int64_t> byblock(n_pairs);
    std::vector<int64_t> fillp(cnt.begin(), cnt.end() - 1);
    for (int64_t p = 0; p < n_pairs; ++p) byblock[fillp[key(p)]++] = p;
    // visiting order: (i, i+1), ..., (i, M-1), then (i, i)
    std::vector<int32_t> res;  // resident blocks, most recent last
    auto visit = [&](int32_t a, int32_t b) {
        const int64_t k = (int64_t)a * M + b;
        if (cnt[k + 1] == cnt[k]) return;
        SchedStep st{a, b, (int64_t)s.order.size(), 0};
        for (int64_t i = cnt[k]; i < cnt[k + 1]; ++i) s.order.push_back(byblock[i]);
        st.pair_end = (int64_t)s.order.size();
        s.steps.push_back(st);
        for (int32_t blk : {a, b}) {
            if (std::find(res.begin(), res.end(), blk) != res.end()) continue;
            if (res.size() >= 3) {
                // evict the oldest block that this step does not use
                for (size_t r = 0; r < res.size(); ++r)
                    if (res[r] != a && res[r] != b) {
                        res.erase(res.begin() + (int64_t)r);
                        break;
                    }
            }
            res.push_back(blk);
            s.block_loads++;
            s.image_loads += s.block_first[blk + 1] - s.block_first[blk];
        }
    };
    for (int32_t i = 0; i < M; ++i) {
        for (int32_t k = i + 1; k < M; ++k) visit(i, k);
        visit(i, i);
    }
    return 0;
}

}  // namespace cashash
