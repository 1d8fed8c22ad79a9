// Persistent worker threads for the library's host-side parallel loops
// (graph validation and index build, the plans of a batch).  Host code only,
// no HIP types, so it builds and is tested on the CPU.
//
// Spawning threads per call cost more than the loops themselves for batches
// of a few thousand patterns; these workers are started once and parked on a
// condition variable between jobs.  One job runs at a time (callers from
// several threads take turns); the caller works on the job too.  A job's
// function must not start another job (it would wait on itself).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

class HostWorkers {
public:
    using Fn = std::function<void(int64_t, int64_t)>;

    explicit HostWorkers(unsigned threads = 0) : want_(threads) {}
    HostWorkers(const HostWorkers &) = delete;
    HostWorkers &operator=(const HostWorkers &) = delete;
    ~HostWorkers()
    {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
            gen_++;
        }
        cv_.notify_all();
        for (auto &t : threads_) t.join();
    }

    // fn(a, b) for the blocks [a, b) of `grain` indices of [0, n).
    void run(int64_t n, int64_t grain, const Fn &fn)
    {
        if (n <= 0) return;
        grain = std::max<int64_t>(grain, 1);
        std::lock_guard<std::mutex> job(job_mu_);
        start();
        {
            std::lock_guard<std::mutex> lk(mu_);
            fn_ = &fn;
            n_ = n;
            grain_ = grain;
            next_.store(0);
            busy_ = (int)threads_.size();
            gen_++;
        }
        cv_.notify_all();
        drain(fn, n, grain);
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return busy_ == 0; });
        fn_ = nullptr;
    }

    size_t threads() const { return threads_.size(); }

private:
    void start()
    {
        if (started_) return;
        started_ = true;
        unsigned hw = want_ ? want_ : std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        for (unsigned t = 1; t < hw; t++) threads_.emplace_back([this] { loop(); });
    }

    void drain(const Fn &fn, int64_t n, int64_t grain)
    {
        for (;;) {
            const int64_t a = next_.fetch_add(grain);
            if (a >= n) return;
            fn(a, std::min(n, a + grain));
        }
    }

    void loop()
    {
        uint64_t seen = 0;
        std::unique_lock<std::mutex> lk(mu_);
        for (;;) {
            cv_.wait(lk, [&] { return gen_ != seen; });
            seen = gen_;
            if (stop_) return;
            const Fn *fn = fn_;
            const int64_t n = n_, grain = grain_;
            lk.unlock();
            drain(*fn, n, grain);
            lk.lock();
            if (--busy_ == 0) done_cv_.notify_all();
        }
    }

    unsigned want_;
    bool started_ = false;
    std::mutex job_mu_, mu_;
    std::condition_variable cv_, done_cv_;
    std::vector<std::thread> threads_;
    const Fn *fn_ = nullptr;
    int64_t n_ = 0, grain_ = 1;
    std::atomic<int64_t> next_{0};
    int busy_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};
