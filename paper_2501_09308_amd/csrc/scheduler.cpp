// Continuous-batching scheduler (host only).  See scheduler.h.
#include "scheduler.h"

#include <algorithm>
#include <chrono>

namespace xrdvi {

namespace {
constexpr int kOk = 0, kPending = 1, kEInval = -1, kENoMem = -2, kEBusy = -4,
              kENoEnt = -5, kECanceled = -6;
constexpr size_t kAlign = 256;

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

double steady_seconds() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

// ---- arena ------------------------------------------------------------------

ArenaAllocator::ArenaAllocator(size_t bytes) : cap_(bytes / kAlign * kAlign) {
    if (cap_ > 0) free_[0] = cap_;
}

bool ArenaAllocator::alloc(size_t bytes, size_t *off) {
    const size_t need = round_up(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= need) {
            *off = it->first;
            const size_t rest = it->second - need;
            const size_t at = it->first + need;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
    }
    return false;
}

void ArenaAllocator::free(size_t off, size_t bytes) {
    size_t size = round_up(std::max<size_t>(bytes, 1));
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + size == next->first) {
        size += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            prev->second += size;
            return;
        }
    }
    free_[off] = size;
}

size_t ArenaAllocator::free_bytes() const {
    size_t s = 0;
    for (auto &kv : free_) s += kv.second;
    return s;
}

// ---- scheduler ------------------------------------------------------------

Scheduler::Scheduler(Executor *ex, size_t arena_bytes, int max_slots,
                     int max_queue, int steps_per_run, size_t resident_bytes)
    : ex_(ex), arena_(arena_bytes), max_slots_(max_slots),
      max_queue_(max_queue), steps_per_run_(steps_per_run),
      resident_limit_(resident_bytes), slot_used_(max_slots, 0),
      t0_(steady_seconds()) {
    worker_ = std::thread([this] { loop(); });
}

Scheduler::~Scheduler() { shutdown(); }

double Scheduler::now() const { return steady_seconds() - t0_; }

void Scheduler::shutdown() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_ && !worker_.joinable()) return;
        stop_ = true;
    }
    cv_.notify_all();
    if (worker_.joinable()) worker_.join();
}

int Scheduler::submit(std::unique_ptr<Job> job, uint64_t *ticket) {
    if (!job || !ticket) return kEInval;
    const size_t bytes = ex_->footprint(*job);
    if (round_up(bytes) > arena_.capacity()) return kENoMem;
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return kEInval;
    if ((int)queue_.size() >= max_queue_) return kEBusy;
    job->ticket = next_ticket_++;
    job->bytes = bytes;
    job->t_arrive = now();
    job->state = kPending;
    *ticket = job->ticket;
    queue_.push_back(job.get());
    jobs_[job->ticket] = std::move(job);
    cv_.notify_all();
    return kOk;
}

int Scheduler::poll(uint64_t ticket, JobStatus *st) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return kENoEnt;
    Job *j = it->second.get();
    if (st) {
        st->state = j->state;
        st->steps_done = j->steps_done;
        st->t_arrive = j->t_arrive;
        st->t_admit = j->t_admit;
        st->t_done = j->t_done;
        st->final_elbo = j->final_elbo;
    }
    const int s = j->state;
    if (s != kPending) jobs_.erase(it);
    return s;
}

int Scheduler::cancel(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return kENoEnt;
    Job *j = it->second.get();
    if (j->state != kPending) return kOk;   // already finished
    auto q = std::find(queue_.begin(), queue_.end(), j);
    if (q != queue_.end()) {
        queue_.erase(q);
        j->state = kECanceled;
        j->t_done = now();
    } else {
        j->cancel_requested = true;         // resident: dropped by the loop
    }
    cv_.notify_all();
    return kOk;
}

int Scheduler::take_slot() {
    for (int i = 0; i < max_slots_; ++i)
        if (!slot_used_[i]) {
            slot_used_[i] = 1;
            return i;
        }
    return -1;
}

// Called with the lock held, after the executor has released the job.
void Scheduler::complete(Job *j, int state) {
    arena_.free(j->arena_off, j->bytes);
    resident_ -= j->bytes;
    if (j->slot >= 0) slot_used_[j->slot] = 0;
    j->slot = -1;
    j->active = false;
    changed_ = true;
    j->state = state;
    j->t_done = now();
    active_.erase(std::remove(active_.begin(), active_.end(), j), active_.end());
}

void Scheduler::loop() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        if (stop_) {
            for (Job *j : std::vector<Job *>(active_)) {
                lk.unlock();
                ex_->release(*j);
                lk.lock();
                complete(j, kECanceled);
            }
            for (Job *j : queue_) {
                j->state = kECanceled;
                j->t_done = now();
            }
            queue_.clear();
            return;
        }
        // drop cancelled residents
        for (Job *j : std::vector<Job *>(active_)) {
            if (!j->cancel_requested) continue;
            lk.unlock();
            ex_->release(*j);
            lk.lock();
            complete(j, kECanceled);
        }
        // admit in arrival order while a slot, arena memory and the
        // resident budget allow
        while (!queue_.empty() && (int)active_.size() < max_slots_) {
            Job *j = queue_.front();
            if (resident_limit_ > 0 && !active_.empty() &&
                resident_ + j->bytes > resident_limit_)
                break;
            size_t off = 0;
            if (!arena_.alloc(j->bytes, &off)) break;
            queue_.pop_front();
            resident_ += j->bytes;
            j->slot = take_slot();
            j->arena_off = off;
            j->t_admit = now();
            j->active = true;
            changed_ = true;
            active_.push_back(j);
            lk.unlock();
            const int rc = ex_->start(*j, j->slot, off);
            lk.lock();
            if (rc != kOk) {
                lk.unlock();
                ex_->release(*j);
                lk.lock();
                complete(j, rc);
            }
        }
        if (active_.empty()) {
            cv_.wait(lk, [this] { return stop_ || !queue_.empty(); });
            continue;
        }
        std::vector<Job *> batch(active_);
        const bool changed = changed_;
        changed_ = false;
        lk.unlock();
        const int rc = ex_->run(batch, steps_per_run_, changed);
        lk.lock();
        for (Job *j : batch) {
            if (rc != kOk) {
                lk.unlock();
                ex_->release(*j);
                lk.lock();
                complete(j, rc);
                continue;
            }
            if (j->cancel_requested || j->steps_done < j->steps) continue;
            lk.unlock();
            const int fr = ex_->finish(*j);
            ex_->release(*j);
            lk.lock();
            complete(j, fr < 0 ? fr : kOk);
        }
    }
}

}  // namespace xrdvi
