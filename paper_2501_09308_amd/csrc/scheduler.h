// Continuous-batching scheduler of the serving loop (host only, no HIP).
//
// Requests are queued at submit, admitted in arrival order as soon as a
// slot and enough arena memory are free, advanced together by the
// executor (a batch of optimisation steps over every resident analysis at
// a time), and completed individually: outputs are copied to the caller's
// buffers, then the slot and memory are reused.  Submit, poll and cancel
// are thread-safe; one scheduler thread drives the executor.
#pragma once

#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace xrdvi {

// One analysis request as held by the server: host copies of the problem,
// run parameters, caller-owned output pointers and its life-cycle state.
struct Job {
    uint64_t ticket = 0;
    // problem (Appendix A.1), copied at submit
    int N = 0, K = 0;
    std::vector<double> x, y, bg, pos, inten;
    std::vector<int> off;
    double cutoff = 0.0;
    double lambda_h = 0.0, mu_sd = 0.03, w_shape = 3.0, w_rate = 100.0;
    int D = 4;                   // latent types per phase (5: asymmetric)
    int width_law = 0;           // 1: full width w sec(rho / 2)
    double alpha_mean = 1.0, alpha_sd = 0.2;
    // run
    int S = 1, steps = 1;
    uint64_t seed = 0;
    double lr = 1e-2;
    std::vector<double> init_loc, init_logscale;   // [D K]
    double *out_loc = nullptr, *out_logscale = nullptr, *out_trace = nullptr;
    // life cycle
    int state = 1;               // 1 pending (queued or active), 0 done, <0 error
    bool active = false;
    bool cancel_requested = false;
    int slot = -1;
    size_t arena_off = 0, bytes = 0;
    int steps_done = 0;
    double t_arrive = 0, t_admit = -1, t_done = -1, final_elbo = 0;
};

// First-fit allocator of byte ranges inside a fixed arena (256-byte units).
class ArenaAllocator {
  public:
    explicit ArenaAllocator(size_t bytes);
    bool alloc(size_t bytes, size_t *off);
    void free(size_t off, size_t bytes);
    size_t capacity() const { return cap_; }
    size_t free_bytes() const;

  private:
    size_t cap_;
    std::map<size_t, size_t> free_;   // offset -> size, disjoint, coalesced
};

// The device side of the server.  All calls come from the scheduler thread.
class Executor {
  public:
    virtual ~Executor() = default;
    // Arena bytes a job needs while resident.
    virtual size_t footprint(const Job &j) const = 0;
    // Upload and initialise job j into `slot` at arena offset `off`.
    virtual int start(Job &j, int slot, size_t off) = 0;
    // Advance every job of `active` by up to `steps` optimisation steps and
    // update their steps_done.  `changed` is set whenever the resident set
    // differs from the previous call (a job admitted, finished or dropped;
    // a slot may now hold another job of another shape).  A non-zero
    // return fails all of them.
    virtual int run(const std::vector<Job *> &active, int steps,
                    bool changed) = 0;
    // Copy the results of a finished job to its caller buffers and set
    // final_elbo; a negative return marks the job failed.
    virtual int finish(Job &j) = 0;
    // Forget the job's slot (its memory is returned by the scheduler).
    virtual void release(Job &j) = 0;
};

struct JobStatus {
    int state, steps_done;
    double t_arrive, t_admit, t_done, final_elbo;
};

class Scheduler {
  public:
    // resident_bytes > 0 caps the summed footprint of the resident analyses
    // (one analysis is always admitted when none is resident): on MI355X a
    // batched step over a working set that fits the last-level caches runs
    // faster than one spread over many more analyses.
    Scheduler(Executor *ex, size_t arena_bytes, int max_slots, int max_queue,
              int steps_per_run, size_t resident_bytes = 0);
    ~Scheduler();

    // Codes follow the C ABI: 0 ok, -1 invalid, -2 never fits, -4 busy.
    int submit(std::unique_ptr<Job> job, uint64_t *ticket);
    // 1 pending, 0 done (outputs written), <0 error / cancelled; a terminal
    // state is reported once, then the ticket is forgotten (-5 after that).
    int poll(uint64_t ticket, JobStatus *st);
    int cancel(uint64_t ticket);
    double now() const;
    // Stops admitting and cancels everything not finished.
    void shutdown();

  private:
    void loop();
    void complete(Job *j, int state);
    int take_slot();

    Executor *ex_;
    ArenaAllocator arena_;
    int max_slots_, max_queue_, steps_per_run_;
    size_t resident_limit_ = 0, resident_ = 0;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Job *> queue_;
    std::vector<Job *> active_;
    std::vector<char> slot_used_;
    std::map<uint64_t, std::unique_ptr<Job>> jobs_;
    uint64_t next_ticket_ = 1;
    bool stop_ = false;
    bool changed_ = true;
    std::thread worker_;
    double t0_;
};

}  // namespace xrdvi
