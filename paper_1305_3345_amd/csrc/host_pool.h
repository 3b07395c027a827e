// host_pool.h -- a fixed set of host threads that run one parallel loop at a
// time, for planning large single-call batches (validation and unit records
// written straight into the pinned staging buffer).  The caller's thread
// takes part; run() returns when every index is done.  One pool belongs to
// one context, which is used by one host thread at a time.
#pragma once

#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace aesgpu {

class HostPool {
  public:
    explicit HostPool(int workers) {
        for (int i = 0; i < workers; i++)
            th_.emplace_back([this] { loop(); });
    }
    ~HostPool() {
        {
            std::lock_guard<std::mutex> lk(m_);
            quit_ = true;
        }
        cv_.notify_all();
        for (std::thread &t : th_)
            t.join();
    }
    HostPool(const HostPool &) = delete;
    HostPool &operator=(const HostPool &) = delete;

    // Threads that take part in run(): the workers and the caller.
    int threads() const { return (int)th_.size() + 1; }

    // Calls f(i) for every i in [0, n) on the workers and the calling thread.
    void run(int n, const std::function<void(int)> &f) {
        {
            std::lock_guard<std::mutex> lk(m_);
            f_ = &f;
            n_ = n;
            next_.store(0, std::memory_order_relaxed);
            busy_ = (int)th_.size();
            gen_++;
        }
        cv_.notify_all();
        for (int i; (i = next_.fetch_add(1, std::memory_order_relaxed)) < n;)
            f(i);
        std::unique_lock<std::mutex> lk(m_);
        done_cv_.wait(lk, [this] { return busy_ == 0; });
        f_ = nullptr;
    }

  private:
    void loop() {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int)> *f;
            int n;
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return quit_ || gen_ != seen; });
                if (quit_)
                    return;
                seen = gen_;
                f = f_;
                n = n_;
            }
            for (int i; (i = next_.fetch_add(1, std::memory_order_relaxed)) < n;)
                (*f)(i);
            std::lock_guard<std::mutex> lk(m_);
            if (--busy_ == 0)
                done_cv_.notify_one();
        }
    }

    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)> *f_ = nullptr;
    int n_ = 0;
    std::atomic<int> next_{0};
    int busy_ = 0;
    uint64_t gen_ = 0;
    bool quit_ = false;
};

}  // namespace aesgpu
