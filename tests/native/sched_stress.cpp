// Stress of the serving scheduler under AddressSanitizer/UBSan (host only):
// concurrent submitters, random cancellations, polling until every ticket
// is resolved, then destruction with work in flight.
#include <atomic>
#include <cstdio>
#include <memory>
#include <random>
#include <thread>
#include <vector>

#include "scheduler.h"

using namespace xrdvi;

namespace {
class StepExecutor : public Executor {
  public:
    size_t footprint(const Job &j) const override { return (size_t)j.K * 512; }
    int start(Job &j, int, size_t) override { j.steps_done = 0; return 0; }
    int run(const std::vector<Job *> &a, int steps, bool changed) override {
        (void)changed;
        for (Job *j : a) j->steps_done = std::min(j->steps, j->steps_done + steps);
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        return 0;
    }
    int finish(Job &j) override {
        for (int k = 0; k < 4 * j.K; ++k) j.out_loc[k] = (double)j.ticket;
        return 0;
    }
    void release(Job &) override {}
};
}  // namespace

int main() {
    StepExecutor ex;
    auto sched = std::make_unique<Scheduler>(&ex, 64 * 1024, 8, 100000, 3);
    const int per_thread = 150, nthreads = 4;
    std::vector<std::vector<double>> outs(per_thread * nthreads);
    std::vector<uint64_t> tickets(per_thread * nthreads);
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t)
        th.emplace_back([&, t] {
            std::mt19937 rng(t);
            for (int i = 0; i < per_thread; ++i) {
                const int idx = t * per_thread + i;
                auto j = std::make_unique<Job>();
                j->K = 1 + rng() % 20;
                j->N = 10;
                j->steps = 1 + rng() % 30;
                outs[idx].assign(4 * j->K, -1.0);
                j->out_loc = outs[idx].data();
                if (sched->submit(std::move(j), &tickets[idx]) != 0) std::abort();
                if (rng() % 7 == 0) sched->cancel(tickets[idx]);
            }
        });
    for (auto &x : th) x.join();
    int ok = 0, canceled = 0;
    for (size_t i = 0; i < tickets.size(); ++i) {
        JobStatus st{};
        int rc;
        while ((rc = sched->poll(tickets[i], &st)) == 1)
            std::this_thread::sleep_for(std::chrono::microseconds(100));
        if (rc == 0) {
            ++ok;
            for (double v : outs[i])
                if (v != (double)tickets[i]) { std::printf("bad output\n"); return 1; }
        } else if (rc == -6) {
            ++canceled;
        } else {
            std::printf("unexpected state %d\n", rc);
            return 1;
        }
    }
    for (int i = 0; i < 50; ++i) {
        auto j = std::make_unique<Job>();
        j->K = 5; j->N = 10; j->steps = 1000000;
        uint64_t t;
        sched->submit(std::move(j), &t);
    }
    sched.reset();
    std::printf("ok=%d canceled=%d\n", ok, canceled);
    return ok + canceled == per_thread * nthreads ? 0 : 1;
}
