// Serving: the GPU executor of the continuous-batching scheduler and the
// serving part of the C ABI (server, submit/poll/cancel, Adam step and the
// one-analysis-at-a-time reference runner).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "batch.h"
#include "scheduler.h"
#include "xrdvi.h"
#include "xrdvi_internal.h"

using namespace xrdvi;

namespace {

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

// Problem description viewing a job's host copies.
xrdvi_problem_desc job_desc(const Job &j) {
    xrdvi_problem_desc d{};
    d.N = j.N;
    d.K = j.K;
    d.x = j.x.data();
    d.y = j.y.data();
    d.bg = j.bg.data();
    d.peak_off = j.off.data();
    d.peak_pos = j.pos.data();
    d.peak_int = j.inten.data();
    d.cutoff = j.cutoff;
    d.prior.lambda_h = j.lambda_h;
    d.prior.mu_sd = j.mu_sd;
    d.prior.w_shape = j.w_shape;
    d.prior.w_rate = j.w_rate;
    d.prior.alpha_mean = j.alpha_mean;
    d.prior.alpha_sd = j.alpha_sd;
    d.asymmetric = j.D == 5;
    d.width_law = j.width_law;
    return d;
}

// Arena layout of one resident analysis.
struct SlotLayout {
    size_t prob, step, state, trace, total;
};

SlotLayout slot_layout(const Job &j) {
    SlotLayout L{};
    const int T = j.off[j.K];
    L.prob = 0;
    L.step = a256(problem_bytes(j.N, j.K, T));
    const StepShape sh{num_tiles(j.N), j.K, T, j.S, j.N, j.D, j.cutoff == 0.0,
                       j.width_law != 0};
    L.state = L.step + a256(step_bytes(sh));
    L.trace = L.state + a256(sizeof(double) * 6 * j.D * (size_t)j.K);
    L.total = L.trace + a256(sizeof(double) * (size_t)j.steps);
    return L;
}

class GpuExecutor : public Executor {
  public:
    GpuExecutor(int device, char *arena, hipStream_t stream, bool use_graph,
                int graph_steps)
        : device_(device), arena_(arena), stream_(stream),
          use_graph_(use_graph), graph_steps_(graph_steps),
          h_tab_(kMaxSlots) {}

    int init() {
        (void)hipSetDevice(device_);
        if (hipMalloc(&d_tab_, sizeof(SlotDev) * kMaxSlots) != hipSuccess ||
            hipMalloc(&d_sch_, sizeof(SchedDev)) != hipSuccess ||
            hipMalloc(&d_steps_, sizeof(int) * kMaxSlots) != hipSuccess)
            return fail(XRDVI_ENOMEM, "server tables: device allocation failed");
        h_sch_ = std::make_unique<SchedDev>();
        std::memset(h_sch_.get(), 0, sizeof(SchedDev));
        if (hipMemcpy(d_sch_, h_sch_.get(), sizeof(SchedDev),
                      hipMemcpyHostToDevice) != hipSuccess)
            return fail(XRDVI_EDEVICE, "server tables: upload failed");
        return XRDVI_OK;
    }

    ~GpuExecutor() override {
        (void)hipSetDevice(device_);
        (void)hipStreamSynchronize(stream_);
        for (int v = 0; v < kClassSets; ++v) {
            if (gexec_[v]) (void)hipGraphExecDestroy(gexec_[v]);
            if (graph_[v]) (void)hipGraphDestroy(graph_[v]);
        }
        if (d_tab_) (void)hipFree(d_tab_);
        if (d_sch_) (void)hipFree(d_sch_);
        if (d_steps_) (void)hipFree(d_steps_);
    }

    size_t footprint(const Job &j) const override { return slot_layout(j).total; }

    int start(Job &j, int slot, size_t off) override {
        (void)hipSetDevice(device_);
        const SlotLayout L = slot_layout(j);
        char *base = arena_ + off;
        SlotDev d{};
        const xrdvi_problem_desc desc = job_desc(j);
        hipError_t e = upload_problem(desc, j.lambda_h, base + L.prob, d.P, nullptr,
                                      stream_);
        if (e != hipSuccess) return dev_fail(e, "upload");
        d.st = carve_step(base + L.step, step_shape(d.P, j.S));
        if (d.P.cutoff == 0.0) d.st.rres = nullptr;   // dense: no residual array
        const size_t D = (size_t)j.D * j.K;
        double *state = (double *)(base + L.state);
        d.loc = state;
        d.logscale = state + D;
        d.m1_loc = state + 2 * D;
        d.m2_loc = state + 3 * D;
        d.m1_ls = state + 4 * D;
        d.m2_ls = state + 5 * D;
        d.trace = (double *)(base + L.trace);
        d.step = d_steps_ + slot;
        d.steps = j.steps;
        d.seed = j.seed;
        d.lr = j.lr;
        e = hipMemcpyAsync(d.loc, j.init_loc.data(), sizeof(double) * D,
                           hipMemcpyHostToDevice, stream_);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d.logscale, j.init_logscale.data(), sizeof(double) * D,
                               hipMemcpyHostToDevice, stream_);
        if (e == hipSuccess)
            e = hipMemsetAsync(d.m1_loc, 0, sizeof(double) * 4 * D, stream_);
        if (e == hipSuccess)
            e = hipMemsetAsync(d.trace, 0, sizeof(double) * (size_t)j.steps, stream_);
        if (e == hipSuccess) e = hipMemsetAsync(d.step, 0, sizeof(int), stream_);
        h_tab_[slot] = d;
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_tab_ + slot, &h_tab_[slot], sizeof(SlotDev),
                               hipMemcpyHostToDevice, stream_);
        if (e == hipSuccess) e = hipStreamSynchronize(stream_);
        if (e != hipSuccess) return dev_fail(e, "start");
        j.steps_done = 0;
        return XRDVI_OK;
    }

    int run(const std::vector<Job *> &active, int steps, bool changed) override {
        (void)hipSetDevice(device_);
        // membership = (slot, ticket): a slot re-used by another analysis
        // changes its shape and therefore its work units
        std::vector<std::pair<int, uint64_t>> members;
        for (const Job *j : active) members.emplace_back(j->slot, j->ticket);
        // analyses with more peaks per point first: their work units are the
        // larger ones, and the persistent grids deal units in this order,
        // so the steps end on small units (then by slot, so the order is a
        // function of the membership)
        std::sort(members.begin(), members.end(), [&](const auto &l, const auto &r) {
            const ProbDev &a = h_tab_[l.first].P, &b = h_tab_[r.first].P;
            const double da = (double)a.T / a.N, db = (double)b.T / b.N;
            return da != db ? da > db : l < r;
        });
        // each variant's kernels run only while an analysis of it is resident
        unsigned classes = 0;
        for (const auto &m : members) classes |= 1u << batch_class(h_tab_[m.first].P);
        hipError_t e = hipSuccess;
        if (changed || members != members_) {
            members_ = members;
            SchedDev &h = *h_sch_;
            h.n = (int)members.size();
            for (int kind = 0; kind < kKinds; ++kind) h.pre[kind][0] = 0;
            for (int i = 0; i < h.n; ++i) {
                const int sl = members[i].first;
                h.slot[i] = sl;
                int units[kKinds];
                batch_units(h_tab_[sl].P, h_tab_[sl].st.S, units);
                for (int kind = 0; kind < kKinds; ++kind)
                    h.pre[kind][i + 1] = h.pre[kind][i] + units[kind];
            }
            e = hipMemcpyAsync(d_sch_, h_sch_.get(), sizeof(SchedDev),
                               hipMemcpyHostToDevice, stream_);
        }
        if (e == hipSuccess) {
            if (use_graph_) {
                if (!gexec_[classes]) e = capture(classes);
                for (int done = 0; e == hipSuccess && done < steps; done += graph_steps_)
                    e = hipGraphLaunch(gexec_[classes], stream_);
            } else {
                for (int i = 0; e == hipSuccess && i < steps; ++i)
                    e = launch_batch_step(d_tab_, d_sch_, stream_, classes);
            }
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_steps_, d_steps_, sizeof(int) * kMaxSlots,
                               hipMemcpyDeviceToHost, stream_);
        if (e == hipSuccess) e = hipStreamSynchronize(stream_);
        if (e != hipSuccess) return dev_fail(e, "batched step");
        for (Job *j : active) j->steps_done = h_steps_[j->slot];
        return XRDVI_OK;
    }

    int finish(Job &j) override {
        (void)hipSetDevice(device_);
        const SlotDev &d = h_tab_[j.slot];
        const size_t D = (size_t)j.D * j.K;
        std::vector<double> trace(j.steps);
        hipError_t e = hipMemcpyAsync(trace.data(), d.trace, sizeof(double) * j.steps,
                                      hipMemcpyDeviceToHost, stream_);
        if (e == hipSuccess && j.out_loc)
            e = hipMemcpyAsync(j.out_loc, d.loc, sizeof(double) * D,
                               hipMemcpyDeviceToHost, stream_);
        if (e == hipSuccess && j.out_logscale)
            e = hipMemcpyAsync(j.out_logscale, d.logscale, sizeof(double) * D,
                               hipMemcpyDeviceToHost, stream_);
        if (e == hipSuccess) e = hipStreamSynchronize(stream_);
        if (e != hipSuccess) return dev_fail(e, "results");
        if (j.out_trace) std::memcpy(j.out_trace, trace.data(), sizeof(double) * j.steps);
        j.final_elbo = trace[j.steps - 1];
        for (double v : trace)
            if (!std::isfinite(v)) return XRDVI_ENONFINITE;
        return XRDVI_OK;
    }

    void release(Job &) override {}

  private:
    int dev_fail(hipError_t e, const char *what) {
        return fail(XRDVI_EDEVICE, std::string("server ") + what + ": " +
                                       hipGetErrorString(e));
    }

    // One graph holding graph_steps_ batched steps; kernels read the slot
    // table and work prefix from fixed device buffers.  One graph per set of
    // resident variant classes, captured when that set first occurs.
    hipError_t capture(unsigned classes) {
        hipError_t e = hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal);
        for (int i = 0; e == hipSuccess && i < graph_steps_; ++i)
            e = launch_batch_step(d_tab_, d_sch_, stream_, classes);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(stream_, &g);
        if (e == hipSuccess) e = e2;
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return e;
        }
        graph_[classes] = g;
        return hipGraphInstantiate(&gexec_[classes], graph_[classes], nullptr, nullptr, 0);
    }

    int device_;
    char *arena_;
    hipStream_t stream_;
    bool use_graph_;
    int graph_steps_;
    std::vector<SlotDev> h_tab_;
    std::unique_ptr<SchedDev> h_sch_;
    SlotDev *d_tab_ = nullptr;
    SchedDev *d_sch_ = nullptr;
    int *d_steps_ = nullptr;
    int h_steps_[kMaxSlots] = {};
    std::vector<std::pair<int, uint64_t>> members_;
    static constexpr int kClassSets = 256;   // subsets of the 8 variant classes
    hipGraph_t graph_[kClassSets] = {};
    hipGraphExec_t gexec_[kClassSets] = {};
};

// Validates a request and builds the job (host copies, default init).
int make_job(const xrdvi_request *r, std::unique_ptr<Job> *out) {
    if (!r) return fail(XRDVI_EINVAL, "request is NULL");
    double lam = 0.0, ymax = 0.0;
    int rc = validate_problem(&r->problem, &lam, &ymax);
    if (rc != XRDVI_OK) return rc;
    if (r->S < 1 || r->S > kMaxSamples) return fail(XRDVI_EINVAL, "S must be in [1, 1024]");
    if (r->steps < 1) return fail(XRDVI_EINVAL, "steps must be >= 1");
    if (!(r->lr >= 0.0) || !std::isfinite(r->lr)) return fail(XRDVI_EINVAL, "lr must be >= 0");
    const xrdvi_problem_desc &p = r->problem;
    auto j = std::make_unique<Job>();
    j->N = p.N;
    j->K = p.K;
    j->x.assign(p.x, p.x + p.N);
    j->y.assign(p.y, p.y + p.N);
    j->bg.assign(p.bg, p.bg + p.N);
    j->off.assign(p.peak_off, p.peak_off + p.K + 1);
    const int T = p.peak_off[p.K];
    j->pos.assign(p.peak_pos, p.peak_pos + T);
    j->inten.assign(p.peak_int, p.peak_int + T);
    j->cutoff = p.cutoff;
    j->lambda_h = lam;
    j->mu_sd = p.prior.mu_sd;
    j->w_shape = p.prior.w_shape;
    j->w_rate = p.prior.w_rate;
    j->D = latent_types(p);
    j->width_law = p.width_law;
    j->alpha_mean = p.prior.alpha_mean;
    j->alpha_sd = p.prior.alpha_sd;
    j->S = r->S;
    j->steps = r->steps;
    j->seed = r->seed;
    j->lr = r->lr > 0.0 ? r->lr : 1e-2;
    const size_t D = (size_t)j->D * p.K;
    if (r->init_loc) j->init_loc.assign(r->init_loc, r->init_loc + D);
    if (r->init_logscale) j->init_logscale.assign(r->init_logscale, r->init_logscale + D);
    // default initialisation: m_h = ln(0.01 / lambda), m_mu = 0,
    // m_w = ln 0.1, m_r = 0, m_alpha = 0, omega = ln 0.1
    if (j->init_loc.empty()) {
        j->init_loc.assign(D, 0.0);
        for (int k = 0; k < p.K; ++k) {
            j->init_loc[k] = std::log(0.01 / lam);
            j->init_loc[2 * p.K + k] = std::log(0.1);
        }
    }
    if (j->init_logscale.empty()) j->init_logscale.assign(D, std::log(0.1));
    j->out_loc = r->out_loc;
    j->out_logscale = r->out_logscale;
    j->out_trace = r->out_elbo_trace;
    *out = std::move(j);
    return XRDVI_OK;
}

}  // namespace

struct xrdvi_server {
    int device = 0;
    hipStream_t stream = nullptr;
    void *arena = nullptr;
    bool own_arena = false;
    std::unique_ptr<GpuExecutor> ex;
    std::unique_ptr<Scheduler> sched;
};

#define API_GUARD_BEGIN try {
#define API_GUARD_END                                                  \
    }                                                                  \
    catch (const std::bad_alloc &) {                                   \
        return fail(XRDVI_ENOMEM, "host allocation failed");           \
    }                                                                  \
    catch (...) {                                                      \
        return fail(XRDVI_EDEVICE, "unexpected internal exception");   \
    }

extern "C" {

int xrdvi_server_create(const xrdvi_server_config *cfg, xrdvi_server **out) {
    API_GUARD_BEGIN
    if (!cfg || !out) return fail(XRDVI_EINVAL, "NULL argument");
    if (cfg->max_slots < 1 || cfg->max_slots > kMaxSlots)
        return fail(XRDVI_EINVAL, "max_slots must be in [1, 512]");
    if (cfg->steps_per_launch < 1) return fail(XRDVI_EINVAL, "steps_per_launch must be >= 1");
    if (cfg->max_queue < 1) return fail(XRDVI_EINVAL, "max_queue must be >= 1");
    if (cfg->arena_bytes < 4096) return fail(XRDVI_EINVAL, "arena_bytes too small");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
        return fail(XRDVI_EINVAL, "device index out of range");
    auto srv = std::make_unique<xrdvi_server>();
    srv->device = cfg->device;
    (void)hipSetDevice(cfg->device);
    if (cfg->arena) {
        srv->arena = cfg->arena;
    } else {
        if (hipMalloc(&srv->arena, cfg->arena_bytes) != hipSuccess)
            return fail(XRDVI_ENOMEM, "arena allocation failed");
        srv->own_arena = true;
    }
    if (hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) != hipSuccess) {
        if (srv->own_arena) (void)hipFree(srv->arena);
        return fail(XRDVI_EDEVICE, "stream creation failed");
    }
    srv->ex = std::make_unique<GpuExecutor>(cfg->device, static_cast<char *>(srv->arena),
                                            srv->stream, cfg->use_graph != 0,
                                            cfg->steps_per_launch);
    int rc = srv->ex->init();
    if (rc != XRDVI_OK) {
        srv->ex.reset();
        (void)hipStreamDestroy(srv->stream);
        if (srv->own_arena) (void)hipFree(srv->arena);
        return rc;
    }
    srv->sched = std::make_unique<Scheduler>(srv->ex.get(), cfg->arena_bytes,
                                             cfg->max_slots, cfg->max_queue,
                                             cfg->steps_per_launch,
                                             cfg->resident_bytes);
    *out = srv.release();
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_server_destroy(xrdvi_server *srv) {
    API_GUARD_BEGIN
    if (!srv) return XRDVI_OK;
    srv->sched->shutdown();
    srv->sched.reset();
    srv->ex.reset();
    (void)hipSetDevice(srv->device);
    (void)hipStreamDestroy(srv->stream);
    if (srv->own_arena) (void)hipFree(srv->arena);
    delete srv;
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_submit(xrdvi_server *srv, const xrdvi_request *req, uint64_t *ticket) {
    API_GUARD_BEGIN
    if (!srv || !ticket) return fail(XRDVI_EINVAL, "NULL argument");
    std::unique_ptr<Job> j;
    int rc = make_job(req, &j);
    if (rc != XRDVI_OK) return rc;
    rc = srv->sched->submit(std::move(j), ticket);
    if (rc == XRDVI_ENOMEM) return fail(rc, "request never fits the server arena");
    if (rc == XRDVI_EBUSY) return fail(rc, "server queue is full");
    if (rc != XRDVI_OK) return fail(rc, "server is shutting down");
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_request_footprint(const xrdvi_request *req, size_t *bytes) {
    API_GUARD_BEGIN
    if (!bytes) return fail(XRDVI_EINVAL, "NULL argument");
    std::unique_ptr<Job> j;
    const int rc = make_job(req, &j);
    if (rc != XRDVI_OK) return rc;
    *bytes = slot_layout(*j).total;
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_poll(xrdvi_server *srv, uint64_t ticket, xrdvi_status *st) {
    API_GUARD_BEGIN
    if (!srv) return fail(XRDVI_EINVAL, "NULL argument");
    JobStatus js{};
    const int rc = srv->sched->poll(ticket, &js);
    if (rc == XRDVI_ENOENT) return fail(rc, "unknown ticket");
    if (st) {
        st->state = js.state;
        st->steps_done = js.steps_done;
        st->t_arrive = js.t_arrive;
        st->t_admit = js.t_admit;
        st->t_done = js.t_done;
        st->final_elbo = js.final_elbo;
    }
    if (rc < 0) set_error(rc == XRDVI_ECANCELED ? "request cancelled"
                                                 : "request failed on the device");
    return rc;
    API_GUARD_END
}

int xrdvi_cancel(xrdvi_server *srv, uint64_t ticket) {
    API_GUARD_BEGIN
    if (!srv) return fail(XRDVI_EINVAL, "NULL argument");
    const int rc = srv->sched->cancel(ticket);
    if (rc == XRDVI_ENOENT) return fail(rc, "unknown ticket");
    return rc;
    API_GUARD_END
}

double xrdvi_server_clock(xrdvi_server *srv) { return srv ? srv->sched->now() : -1.0; }

int xrdvi_adam_step(xrdvi_ctx *ctx, int32_t n, double *theta, double *m1,
                    double *m2, const double *grad, int32_t t, double lr,
                    double beta1, double beta2, double eps, void *stream) {
    API_GUARD_BEGIN
    if (!ctx || !theta || !m1 || !m2 || !grad) return fail(XRDVI_EINVAL, "NULL argument");
    if (n < 0 || t < 1) return fail(XRDVI_EINVAL, "n must be >= 0 and t >= 1");
    if (n == 0) return XRDVI_OK;
    const hipError_t e = launch_adam(n, theta, m1, m2, grad, t, lr, beta1, beta2,
                                     eps, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(XRDVI_EDEVICE, std::string("adam: ") + hipGetErrorString(e));
    return XRDVI_OK;
    API_GUARD_END
}

int xrdvi_plain_run(xrdvi_ctx *ctx, const xrdvi_request *req, xrdvi_status *st,
                    void *stream) {
    API_GUARD_BEGIN
    if (!ctx || !req) return fail(XRDVI_EINVAL, "NULL argument");
    std::unique_ptr<Job> j;
    int rc = make_job(req, &j);
    if (rc != XRDVI_OK) return rc;
    const xrdvi_problem_desc desc = job_desc(*j);
    xrdvi_problem *prob = nullptr;
    xrdvi_tape *tape = nullptr;
    rc = xrdvi_problem_create(ctx, &desc, &prob);
    if (rc == XRDVI_OK) rc = xrdvi_tape_create(ctx, prob, j->S, &tape);
    const size_t D = (size_t)j->D * j->K;
    double *mem = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (rc == XRDVI_OK && hipMalloc(&mem, sizeof(double) * (8 * D + j->steps)) != hipSuccess)
        rc = fail(XRDVI_ENOMEM, "plain run: allocation failed");
    if (rc == XRDVI_OK) {
        double *loc = mem, *ls = mem + D, *gl = mem + 2 * D, *gs = mem + 3 * D,
               *m = mem + 4 * D, *trace = mem + 8 * D;
        hipError_t e = hipMemcpyAsync(loc, j->init_loc.data(), sizeof(double) * D,
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ls, j->init_logscale.data(), sizeof(double) * D,
                               hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(m, 0, sizeof(double) * 4 * D, s);
        if (e != hipSuccess) rc = fail(XRDVI_EDEVICE, "plain run: upload failed");
        for (int n = 0; rc == XRDVI_OK && n < j->steps; ++n) {
            rc = xrdvi_elbo_fwd(ctx, prob, j->S, loc, ls, nullptr, j->seed, n, 1,
                                trace + n, nullptr, tape, stream);
            if (rc == XRDVI_OK) rc = xrdvi_elbo_bwd(ctx, tape, 1.0, nullptr, gl, gs, stream);
            if (rc == XRDVI_OK)
                rc = xrdvi_adam_step(ctx, (int)D, loc, m, m + D, gl, n + 1, j->lr, 0.9,
                                     0.999, 1e-8, stream);
            if (rc == XRDVI_OK)
                rc = xrdvi_adam_step(ctx, (int)D, ls, m + 2 * D, m + 3 * D, gs, n + 1,
                                     j->lr, 0.9, 0.999, 1e-8, stream);
        }
        std::vector<double> tr(j->steps);
        if (rc == XRDVI_OK) {
            e = hipMemcpyAsync(tr.data(), trace, sizeof(double) * j->steps,
                               hipMemcpyDeviceToHost, s);
            if (e == hipSuccess && j->out_loc)
                e = hipMemcpyAsync(j->out_loc, loc, sizeof(double) * D,
                                   hipMemcpyDeviceToHost, s);
            if (e == hipSuccess && j->out_logscale)
                e = hipMemcpyAsync(j->out_logscale, ls, sizeof(double) * D,
                                   hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) rc = fail(XRDVI_EDEVICE, "plain run: download failed");
        }
        if (rc == XRDVI_OK) {
            if (j->out_trace) std::memcpy(j->out_trace, tr.data(), sizeof(double) * j->steps);
            if (st) {
                st->state = XRDVI_OK;
                st->steps_done = j->steps;
                st->final_elbo = tr[j->steps - 1];
                st->t_arrive = st->t_admit = st->t_done = 0.0;
            }
            for (double v : tr)
                if (!std::isfinite(v)) rc = fail(XRDVI_ENONFINITE, "non-finite ELBO");
        }
    }
    if (mem) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(mem);
    }
    if (tape) xrdvi_tape_destroy(tape);
    if (prob) xrdvi_problem_destroy(prob);
    return rc;
    API_GUARD_END
}

}  // extern "C"
