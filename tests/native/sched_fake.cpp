// Test double of the serving executor: exercises the scheduler's queueing,
// memory admission, slot reuse, cancellation, error propagation and time
// stamps on the CPU.  A fake job of K phases and N points occupies
// K * 1024 + N * 16 arena bytes; every run() advances all resident jobs by
// steps_per_run steps; outputs encode the ticket so routing can be checked.
#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <memory>
#include <thread>

#include "scheduler.h"

using namespace xrdvi;

namespace {

class FakeExecutor : public Executor {
  public:
    explicit FakeExecutor(int sleep_us) : sleep_us_(sleep_us) {}
    size_t footprint(const Job &j) const override {
        return (size_t)j.K * 1024 + (size_t)j.N * 16;
    }
    int start(Job &j, int slot, size_t) override {
        if (j.seed == 13) return -3;          // simulated upload failure
        j.steps_done = 0;
        used_slots_ = std::max(used_slots_, slot + 1);
        return 0;
    }
    int run(const std::vector<Job *> &active, int steps, bool changed) override {
        max_active_ = std::max<int>(max_active_, (int)active.size());
        size_t resident = 0;
        for (const Job *j : active) resident += footprint(*j);
        max_resident_ = std::max(max_resident_, resident);
        ++runs_;
        // the resident set as (slot, ticket): any difference from the last
        // run must be announced, or the executor would keep stale work
        // prefixes for a slot now holding another analysis
        std::vector<std::pair<int, uint64_t>> members;
        for (const Job *j : active) members.emplace_back(j->slot, j->ticket);
        std::sort(members.begin(), members.end());
        if (members != last_ && !changed) ++missed_changes_;
        if (changed) ++changed_runs_;
        last_ = members;
        for (Job *j : active) j->steps_done = std::min(j->steps, j->steps_done + steps);
        if (sleep_us_) std::this_thread::sleep_for(std::chrono::microseconds(sleep_us_));
        return 0;
    }
    int finish(Job &j) override {
        for (int k = 0; k < 4 * j.K; ++k)
            if (j.out_loc) j.out_loc[k] = (double)j.ticket * 1000.0 + k;
        for (int n = 0; n < j.steps; ++n)
            if (j.out_trace) j.out_trace[n] = n;
        j.final_elbo = -(double)j.ticket;
        return j.seed == 666 ? -7 : 0;       // simulated non-finite ELBO
    }
    void release(Job &) override {}
    int max_active_ = 0, runs_ = 0, used_slots_ = 0;
    size_t max_resident_ = 0;
    int missed_changes_ = 0, changed_runs_ = 0;
    std::vector<std::pair<int, uint64_t>> last_;

  private:
    int sleep_us_;
};

struct Fake {
    std::unique_ptr<FakeExecutor> ex;
    std::unique_ptr<Scheduler> sched;
};

}  // namespace

extern "C" {

void *fake_create_budget(size_t arena, int max_slots, int max_queue,
                         int steps_per_run, int sleep_us, size_t resident) {
    auto *f = new Fake();
    f->ex = std::make_unique<FakeExecutor>(sleep_us);
    f->sched = std::make_unique<Scheduler>(f->ex.get(), arena, max_slots, max_queue,
                                           steps_per_run, resident);
    return f;
}

void *fake_create(size_t arena, int max_slots, int max_queue, int steps_per_run,
                  int sleep_us) {
    return fake_create_budget(arena, max_slots, max_queue, steps_per_run,
                              sleep_us, 0);
}

size_t fake_max_resident(void *h) {
    return static_cast<Fake *>(h)->ex->max_resident_;
}

int fake_submit(void *h, int K, int N, int steps, uint64_t seed, double *out_loc,
                double *out_trace, uint64_t *ticket) {
    auto *f = static_cast<Fake *>(h);
    auto j = std::make_unique<Job>();
    j->K = K;
    j->N = N;
    j->steps = steps;
    j->seed = seed;
    j->out_loc = out_loc;
    j->out_trace = out_trace;
    return f->sched->submit(std::move(j), ticket);
}

int fake_poll(void *h, uint64_t ticket, double *info) {
    JobStatus st{};
    const int rc = static_cast<Fake *>(h)->sched->poll(ticket, &st);
    info[0] = st.state; info[1] = st.steps_done; info[2] = st.t_arrive;
    info[3] = st.t_admit; info[4] = st.t_done; info[5] = st.final_elbo;
    return rc;
}

int fake_cancel(void *h, uint64_t ticket) {
    return static_cast<Fake *>(h)->sched->cancel(ticket);
}

void fake_stats(void *h, int *max_active, int *runs, int *used_slots) {
    auto *f = static_cast<Fake *>(h);
    *max_active = f->ex->max_active_;
    *runs = f->ex->runs_;
    *used_slots = f->ex->used_slots_;
}

void fake_changes(void *h, int *missed, int *changed_runs) {
    auto *f = static_cast<Fake *>(h);
    *missed = f->ex->missed_changes_;
    *changed_runs = f->ex->changed_runs_;
}

void fake_destroy(void *h) {
    auto *f = static_cast<Fake *>(h);
    f->sched->shutdown();
    delete f;
}

}  // extern "C"
