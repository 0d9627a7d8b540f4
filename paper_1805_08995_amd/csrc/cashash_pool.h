// Fork-join pool of host threads for the library's bulk host copies: the
// staging of caller inputs into pinned memory and the scatter of results
// back into the caller's arrays in host-memory mode.  A single memcpy thread
// moves a few GB/s, well below what PCIe moves, so large copies are split
// over the workers and the calling thread.
// Pure host code: no HIP calls.
#pragma once
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace cashash {

class WorkPool {
  public:
    // n_threads - 1 workers; the caller of run() is the last thread
    explicit WorkPool(int n_threads) {
        const int w = std::max(0, n_threads - 1);
        for (int i = 0; i < w; ++i) workers_.emplace_back([this] { work(); });
    }
    ~WorkPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : workers_) t.join();
    }
    WorkPool(const WorkPool&) = delete;
    WorkPool& operator=(const WorkPool&) = delete;

    int threads() const { return (int)workers_.size() + 1; }

    // f(i) for every i in [0, n), spread over the threads; returns when all
    // are done.  Calls from one thread at a time.
    void run(int64_t n, const std::function<void(int64_t)>& f) {
        if (n <= 0) return;
        if (workers_.empty() || n == 1) {
            for (int64_t i = 0; i < n; ++i) f(i);
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            job_ = &f;
            n_ = n;
            next_.store(0);
            active_ = (int)workers_.size();
            ++gen_;
        }
        cv_.notify_all();
        drain(f, n);
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [this] { return active_ == 0; });
        job_ = nullptr;
    }

  private:
    void drain(const std::function<void(int64_t)>& f, int64_t n) {
        for (int64_t i = next_.fetch_add(1); i < n; i = next_.fetch_add(1)) f(i);
    }
    void work() {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int64_t)>* f;
            int64_t n;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                f = job_;
                n = n_;
            }
            drain(*f, n);
            {
                std::lock_guard<std::mutex> lk(mu_);
                if (--active_ == 0) done_cv_.notify_one();
            }
        }
    }

    std::vector<std::thread> workers_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int64_t)>* job_ = nullptr;
    int64_t n_ = 0;
    std::atomic<int64_t> next_{0};
    int active_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

// memcpy of `bytes` split into pieces of at least `grain` bytes over the pool.
inline void parallel_copy(WorkPool& pool, void* dst, const void* src, size_t bytes, size_t grain = (size_t)1 << 20) {
    const int64_t pieces = std::max<int64_t>(1, std::min<int64_t>((int64_t)(bytes / std::max<size_t>(grain, 1)),
                                                                  4 * (int64_t)pool.threads()));
    if (pieces == 1) {
        if (bytes) std::memcpy(dst, src, bytes);
        return;
    }
    const size_t step = (bytes + (size_t)pieces - 1) / (size_t)pieces;
    pool.run(pieces, [&](int64_t i) {
        const size_t lo = (size_t)i * step;
        if (lo >= bytes) return;
        const size_t n = std::min(step, bytes - lo);
        std::memcpy(static_cast<uint8_t*>(dst) + lo, static_cast<const uint8_t*>(src) + lo, n);
    });
}

}  // namespace cashash
