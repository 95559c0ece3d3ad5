// Request server for interior point solves of different sizes on one GPU.
//
// Requests are admitted (first fit in arrival order) while fewer than
// max_active solves are resident and their estimated device footprint stays
// within the budget. Each admitted solve owns a host thread and a stream; its
// plan, iterates and preconditioner stay on the device until it finishes, and
// admission continues as slots and memory free up, so work of different solves
// overlaps on the GPU. With shared launches, the one-vector matvecs that the
// resident solves issue are collected by a combiner thread and run together
// (one launch per matvec stage for up to kMaxJobs solves); stream events order
// each matvec after the producer of its input and before its consumer.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>

#include "plan.hpp"
#include "server.hpp"
#include "solver.hpp"

namespace anv {

thread_local bool t_blocking_waits = false;

void host_wait(hipStream_t st) {
    if (!t_blocking_waits) {
        ANV_HIP(hipStreamSynchronize(st));
        return;
    }
    // one blocking-sync event per thread and device, destroyed when the thread ends
    struct Ev {
        hipEvent_t e = nullptr;
        int dev = -1;
        ~Ev() {
            if (e) (void)hipEventDestroy(e);
        }
    };
    thread_local Ev ev;
    int dev = 0;
    ANV_HIP(hipGetDevice(&dev));
    if (!ev.e || ev.dev != dev) {
        if (ev.e) (void)hipEventDestroy(ev.e);
        ev.e = nullptr;
        ANV_HIP(hipEventCreateWithFlags(&ev.e, hipEventBlockingSync | hipEventDisableTiming));
        ev.dev = dev;
    }
    ANV_HIP(hipEventRecord(ev.e, st));
    ANV_HIP(hipEventSynchronize(ev.e));
}

namespace {

using clk = std::chrono::steady_clock;

// largest per-axis error of a request's trigonometric kernel approximation
// (absolute, the Gaussian's maximum being 1) that the server accepts: the
// matvec accuracy bar
constexpr double kMaxKernelErr = 1e-4;

double ms_between(clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
    int64_t ticket = 0;
    int64_t N = 0;
    int32_t d = 0, P = 0;
    double C = 0;
    std::vector<double> X, labels, sigma;
    std::vector<int32_t> windows;
    anova_opts nfft;
    anova_ipm_opts ipm;
    int64_t footprint = 0;
    clk::time_point t_submit, t_admit;
};

struct Result {
    bool done = false;
    int status = ANOVA_OK;
    std::string error;
    std::vector<double> alpha;
    anova_result res;
};

}  // namespace

// Collects one-vector matvecs from resident solves and runs them in shared launches.
class Combiner {
  public:
    // grouped: matvecs of one plan from several solves go out as one batched
    // call (enqueue_matvec_grouped); otherwise one vector per plan and launch
    Combiner(int device, double gather_us, bool grouped = false)
        : device_(device), gather_us_(gather_us), grouped_(grouped) {
        ANV_HIP(hipSetDevice(device_));
        ANV_HIP(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
        thread_ = std::thread([this] { loop(); });
    }
    ~Combiner() {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_ = true;
        }
        cv_.notify_all();
        thread_.join();
        (void)hipStreamDestroy(stream_);
    }
    void solver_leave(bool& joined) {
        {
            std::lock_guard<std::mutex> g(m_);
            if (joined) --active_;
            joined = false;
        }
        cv_.notify_all();
    }
    // Called from a solver thread: y = K x on `st`, in a shared launch. A solve
    // counts as taking part (the combiner waits for its matvecs) from its
    // first matvec until solver_leave.
    void matvec(Plan& pl, const double* x, double* y, hipStream_t st, hipEvent_t ready, hipEvent_t done,
                bool& joined) {
        Item it{&pl, x, y, ready, done, false, nullptr};
        ANV_HIP(hipEventRecord(ready, st));
        std::unique_lock<std::mutex> lk(m_);
        if (!joined) {
            ++active_;
            joined = true;
        }
        pending_.push_back(&it);
        if (pending_.size() == 1) first_ = clk::now();
        cv_.notify_all();
        cv_.wait(lk, [&] { return it.launched; });
        if (it.err) std::rethrow_exception(it.err);
        lk.unlock();
        ANV_HIP(hipStreamWaitEvent(st, done, 0));
    }
    int64_t launches() const { return launches_.load(); }
    int64_t matvecs() const { return matvecs_.load(); }

  private:
    struct Item {
        Plan* pl;
        const double* x;
        double* y;
        hipEvent_t ready, done;
        bool launched;
        std::exception_ptr err;
    };
    void loop() {
        (void)hipSetDevice(device_);
        std::unique_lock<std::mutex> lk(m_);
        for (;;) {
            cv_.wait(lk, [&] { return stop_ || !pending_.empty(); });
            if (pending_.empty()) {
                if (stop_) return;
                continue;
            }
            // wait for the other resident solves' matvecs, up to gather_us
            const auto deadline = first_ + std::chrono::microseconds(int64_t(gather_us_));
            cv_.wait_until(lk, deadline, [&] { return stop_ || int(pending_.size()) >= active_; });
            std::vector<Item*> batch(pending_.begin(), pending_.end());
            pending_.clear();
            lk.unlock();
            std::exception_ptr err;
            try {
                std::vector<Plan*> plans;
                std::vector<const double*> xs;
                std::vector<double*> ys;
                for (Item* it : batch) {
                    ANV_HIP(hipStreamWaitEvent(stream_, it->ready, 0));
                    plans.push_back(it->pl);
                    xs.push_back(it->x);
                    ys.push_back(it->y);
                }
                if (grouped_)
                    enqueue_matvec_grouped(plans.data(), xs.data(), ys.data(), int(plans.size()), stream_);
                else
                    enqueue_matvec_multi(plans.data(), xs.data(), ys.data(), int(plans.size()), stream_);
                for (Item* it : batch) ANV_HIP(hipEventRecord(it->done, stream_));
                launches_ += 1;
                matvecs_ += int64_t(batch.size());
            } catch (...) {
                err = std::current_exception();
            }
            lk.lock();
            for (Item* it : batch) {
                it->err = err;
                it->launched = true;
            }
            cv_.notify_all();
        }
    }
    int device_;
    double gather_us_;
    bool grouped_;
    hipStream_t stream_ = nullptr;
    std::mutex m_;
    std::condition_variable cv_;
    std::deque<Item*> pending_;
    clk::time_point first_;
    int active_ = 0;
    bool stop_ = false;
    std::atomic<int64_t> launches_{0}, matvecs_{0};
    std::thread thread_;
};

struct Server::Impl {
    anova_server_opts opts;
    int device = 0;
    std::unique_ptr<Combiner> comb;
    std::mutex m;
    std::condition_variable cv;
    std::list<std::unique_ptr<Request>> queue;
    std::map<int64_t, Result> results;
    std::map<int64_t, std::thread> workers;  // by ticket
    std::vector<int64_t> finished;           // tickets whose worker has returned (joined by the scheduler)
    int active = 0;
    int64_t used = 0;
    int64_t next_ticket = 1;
    bool stop = false;
    std::thread scheduler;

    void run_scheduler() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(m);
        for (;;) {
            cv.wait(lk, [&] { return stop || !finished.empty() || (!queue.empty() && active < opts.max_active); });
            reap_finished(lk);
            if (stop && queue.empty()) return;
            if (queue.empty()) continue;  // woken only to join finished workers
            // first fit in arrival order
            bool admitted = false;
            for (auto it = queue.begin(); it != queue.end() && active < opts.max_active; ++it) {
                if (used + (*it)->footprint > opts.hbm_budget && active > 0) continue;
                std::unique_ptr<Request> r = std::move(*it);
                queue.erase(it);
                r->t_admit = clk::now();
                used += r->footprint;
                ++active;
                Request* raw = r.release();
                const int64_t tk = raw->ticket;
                workers.emplace(tk, std::thread([this, raw] { run_request(std::unique_ptr<Request>(raw)); }));
                admitted = true;
                break;
            }
            if (!admitted) cv.wait(lk);  // nothing fits: wait for a solve to finish
        }
    }

    // joins the threads of requests that have finished (called with m held;
    // the joins wait at most for the threads' last few instructions)
    void reap_finished(std::unique_lock<std::mutex>& lk) {
        std::vector<std::thread> done;
        for (int64_t tk : finished) {
            auto it = workers.find(tk);
            if (it == workers.end()) continue;
            done.push_back(std::move(it->second));
            workers.erase(it);
        }
        finished.clear();
        lk.unlock();
        for (auto& t : done) t.join();
        lk.lock();
    }

    void run_request(std::unique_ptr<Request> r) {
        BlockingWaits blocking;
        Result out;
        std::vector<double> alpha_h(size_t(r->N), 0.0);
        anova_ipm_stats st{};
        double lambda = 0.0;
        int status = ANOVA_OK;
        std::string err;
        hipStream_t stream = nullptr;
        hipEvent_t ev_ready = nullptr, ev_done = nullptr;
        bool joined = false;
        // device state of the request; released only after its stream has
        // drained (also when the solve ends in an error)
        DevBuf<double> Xd, yd, ad;
        std::unique_ptr<Plan> pl;
        try {
            ANV_HIP(hipSetDevice(device));
            ANV_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
            ANV_HIP(hipEventCreateWithFlags(&ev_ready, hipEventDisableTiming));
            ANV_HIP(hipEventCreateWithFlags(&ev_done, hipEventDisableTiming));
            Xd.alloc(r->X.size());
            yd.alloc(size_t(r->N));
            ad.alloc(size_t(r->N));
            ANV_HIP(hipMemcpyAsync(Xd.p, r->X.data(), r->X.size() * sizeof(double), hipMemcpyHostToDevice, stream));
            ANV_HIP(hipMemcpyAsync(yd.p, r->labels.data(), r->labels.size() * sizeof(double),
                                   hipMemcpyHostToDevice, stream));
            pl.reset(create_plan(Xd.p, r->N, r->d, r->d, r->windows.data(), r->P, r->sigma.data(), nullptr, &r->nfft,
                                 stream));
            // the plan's kernel approximation must meet the matvec accuracy the
            // solve relies on (data outside the scale the bandwidth resolves
            // would otherwise be solved with a far worse kernel)
            if (!(pl->max_kerr <= kMaxKernelErr))
                throw Error(ANOVA_INVALID_ARG, "kernel approximation error " + std::to_string(pl->max_kerr) +
                                                   " exceeds " + std::to_string(kMaxKernelErr) +
                                                   ": scale the features or raise the bandwidth");
            Plan* plp = pl.get();
            MatvecHook hook = [this, plp, ev_ready, ev_done, &joined](const double* x, double* y, hipStream_t s) {
                comb->matvec(*plp, x, y, s, ev_ready, ev_done, joined);
            };
            status = ipm_solve(*pl, yd.p, r->C, r->ipm, ad.p, &lambda, &st, stream, nullptr, comb ? &hook : nullptr);
            if (comb) comb->solver_leave(joined);
            ANV_HIP(hipMemcpyAsync(alpha_h.data(), ad.p, alpha_h.size() * sizeof(double), hipMemcpyDeviceToHost,
                                   stream));
            ANV_HIP(hipStreamSynchronize(stream));
        } catch (const Error& e) {
            status = e.code;
            err = e.what();
        } catch (const std::exception& e) {
            status = ANOVA_HIP_ERROR;
            err = e.what();
        }
        if (comb) comb->solver_leave(joined);
        if (stream) (void)hipStreamSynchronize(stream);
        pl.reset();
        Xd.release();
        yd.release();
        ad.release();
        if (stream) (void)hipStreamDestroy(stream);
        if (ev_ready) (void)hipEventDestroy(ev_ready);
        if (ev_done) (void)hipEventDestroy(ev_done);
        const auto t_end = clk::now();
        out.done = true;
        out.status = status;
        out.error = err;
        out.alpha = std::move(alpha_h);
        std::memset(&out.res, 0, sizeof(out.res));
        out.res.status = status;
        out.res.footprint = r->footprint;
        out.res.queue_ms = ms_between(r->t_submit, r->t_admit);
        out.res.run_ms = ms_between(r->t_admit, t_end);
        out.res.latency_ms = ms_between(r->t_submit, t_end);
        out.res.lambda = lambda;
        out.res.stats = st;
        {
            std::lock_guard<std::mutex> g(m);
            results[r->ticket] = std::move(out);
            used -= r->footprint;
            --active;
            finished.push_back(r->ticket);
        }
        cv.notify_all();
    }
};

int64_t request_footprint(int64_t N, int32_t d, int32_t P, const anova_opts& nfft, const anova_ipm_opts& ipm) {
    const int W = 2 * nfft.cutoff_m;
    const int eb = nfft.precision == ANOVA_PREC_FP64 ? 8 : 4;
    const int64_t E = 24 + W;  // occupied extent per axis for data scaled into the box
    const int64_t pw = N * P;
    int64_t b = N * d * 8 + 2 * N * 8;                              // X, labels, alpha
    b += pw * (24 + 12 + 3 * W * eb + 16 + 8 * eb);                  // plan per point-window
    b += int64_t(P) * E * E * E * (W * W + 4) * eb;                  // grids and fold target
    b += 18 * (N + 1) * 8;                                           // IPM vectors
    const int64_t k = (ipm.precond == ANOVA_PRECOND_PCHOL || ipm.precond == ANOVA_PRECOND_NYSTROM ||
                       ipm.precond == ANOVA_PRECOND_RPCHOL || ipm.precond == ANOVA_PRECOND_RFF) ? ipm.rank : 0;
    b += (ipm.precond == ANOVA_PRECOND_NYSTROM ? 4 : 2) * N * k * 8;  // factor and its build
    if (ipm.factor_fp32) b += N * k * 4;                             // FP32 copy for the products
    b += 260 * k * k * 8;                                            // capacitance partial sums
    if (ipm.krylov == ANOVA_KRYLOV_GMRES)                            // Arnoldi basis and P^{-1} v
        b += (int64_t(std::min(ipm.max_kry, 100)) + 2) * ((N + 1 + 31) / 32 * 32) * 8;
    return b + b / 4;                                                // margin
}

Server::Server(const anova_server_opts& o, int device) : impl_(new Impl) {
    impl_->opts = o;
    impl_->device = device;
    ANV_HIP(hipSetDevice(device));
    if (impl_->opts.hbm_budget <= 0) {
        size_t fr = 0, tot = 0;
        ANV_HIP(hipMemGetInfo(&fr, &tot));
        impl_->opts.hbm_budget = int64_t(double(fr) * 0.8);
    }
    if (o.share_launches) impl_->comb.reset(new Combiner(device, o.gather_us));
    impl_->scheduler = std::thread([this] { impl_->run_scheduler(); });
}

Server::~Server() {
    {
        std::lock_guard<std::mutex> g(impl_->m);
        impl_->stop = true;
    }
    impl_->cv.notify_all();
    impl_->scheduler.join();
    for (auto& t : impl_->workers) t.second.join();
    impl_->comb.reset();
}

int64_t Server::submit(const anova_request& q) {
    ANV_CHECK(q.X && q.labels && q.windows && q.sigma, "NULL request field");
    ANV_CHECK(q.N >= 2 && q.d >= 1 && q.P >= 1, "bad request sizes");
    ANV_CHECK(std::isfinite(q.C) && q.C > 0.0, "C must be > 0");
    auto r = std::make_unique<Request>();
    r->t_submit = clk::now();
    r->N = q.N;
    r->d = q.d;
    r->P = q.P;
    r->C = q.C;
    r->X.assign(q.X, q.X + q.N * q.d);
    r->labels.assign(q.labels, q.labels + q.N);
    r->windows.assign(q.windows, q.windows + 3 * q.P);
    r->sigma.assign(q.sigma, q.sigma + q.P);
    if (q.nfft) {
        ANV_CHECK(q.nfft->version == ANOVA_OPTS_VERSION, "anova_opts.version mismatch");
        r->nfft = *q.nfft;
    } else {
        anova_opts_default(&r->nfft);
    }
    if (q.ipm) {
        ANV_CHECK(q.ipm->version == ANOVA_IPM_OPTS_VERSION, "anova_ipm_opts.version mismatch");
        r->ipm = *q.ipm;
    } else {
        anova_ipm_opts_default(&r->ipm);
    }
    r->footprint = request_footprint(r->N, r->d, r->P, r->nfft, r->ipm);
    int64_t t;
    {
        std::lock_guard<std::mutex> g(impl_->m);
        ANV_CHECK(!impl_->stop, "server is shutting down");
        t = impl_->next_ticket++;
        r->ticket = t;
        impl_->results[t];  // reserve: done = false
        impl_->queue.push_back(std::move(r));
    }
    impl_->cv.notify_all();
    return t;
}

int Server::wait(int64_t ticket, double* alpha, anova_result* res) {
    std::unique_lock<std::mutex> lk(impl_->m);
    auto it = impl_->results.find(ticket);
    ANV_CHECK(it != impl_->results.end(), "unknown or already collected ticket");
    // a second waiter on the same ticket finds the entry gone once the first
    // has collected it, and reports that instead of waiting for ever
    impl_->cv.wait(lk, [&] {
        auto f = impl_->results.find(ticket);
        return f == impl_->results.end() || f->second.done;
    });
    it = impl_->results.find(ticket);
    ANV_CHECK(it != impl_->results.end(), "ticket collected by another waiter");
    Result r = std::move(it->second);
    impl_->results.erase(it);
    lk.unlock();
    if (alpha) std::memcpy(alpha, r.alpha.data(), r.alpha.size() * sizeof(double));
    if (res) *res = r.res;
    if (!r.error.empty()) throw Error(r.status, r.error);
    return r.status;
}

void Server::counters(int64_t* launches, int64_t* matvecs) const {
    *launches = impl_->comb ? impl_->comb->launches() : 0;
    *matvecs = impl_->comb ? impl_->comb->matvecs() : 0;
}

void grid_solve(const GridProblem* probs, int nprob, const anova_ipm_opts& o, int max_active, double gather_us,
                int device, int64_t* launches, int64_t* matvecs) {
    ANV_CHECK(probs && nprob >= 1, "no problems");
    ANV_CHECK(max_active >= 1 && max_active <= 256, "max_active must be in [1, 256]");
    ANV_CHECK(std::isfinite(gather_us) && gather_us >= 0.0, "gather_us must be >= 0");
    struct Task {
        int p, c;
    };
    std::vector<Task> tasks;
    for (int p = 0; p < nprob; ++p) {
        const GridProblem& g = probs[p];
        ANV_CHECK(g.plan && g.labels && g.C && g.alpha && g.lambda && g.stats, "NULL problem field");
        ANV_CHECK(g.nC >= 1, "every problem needs at least one C");
        for (int c = 0; c < g.nC; ++c) ANV_CHECK(std::isfinite(g.C[c]) && g.C[c] > 0.0, "C must be > 0");
        for (int q = 0; q < p; ++q) ANV_CHECK(probs[q].plan != g.plan, "a plan may appear in one problem only");
        for (int c = 0; c < g.nC; ++c) tasks.push_back({p, c});
    }
    struct ProbState {
        std::once_flag once;
        LowRankFactor f;
        int status = ANOVA_OK;
        std::string err;
        std::atomic<int> left{0};
    };
    std::vector<std::unique_ptr<ProbState>> ps;
    for (int p = 0; p < nprob; ++p) {
        ps.emplace_back(new ProbState);
        ps.back()->left = probs[p].nC;
    }
    ANV_HIP(hipSetDevice(device));
    Combiner comb(device, gather_us, true);
    std::atomic<size_t> next{0};
    auto worker = [&] {
        BlockingWaits blocking;
        hipStream_t stream = nullptr;
        hipEvent_t ready = nullptr, done = nullptr;
        bool ok = hipSetDevice(device) == hipSuccess &&
                  hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&ready, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess;
        for (;;) {
            const size_t t = next++;
            if (t >= tasks.size()) break;
            const GridProblem& g = probs[tasks[t].p];
            ProbState& P = *ps[tasks[t].p];
            const int c = tasks[t].c;
            anova_ipm_stats st{};
            double lam = 0.0;
            int status = ANOVA_HIP_ERROR;
            if (ok) {
                try {
                    // the first solve of a problem builds the factor its C values share
                    std::call_once(P.once, [&] {
                        try {
                            build_low_rank(*g.plan, o, P.f, stream);
                        } catch (const Error& e) {
                            P.status = e.code;
                            P.err = e.what();
                        }
                    });
                    if (P.status != ANOVA_OK) throw Error(P.status, P.err);
                    bool joined = false;
                    MatvecHook hook = [&](const double* x, double* y, hipStream_t s) {
                        comb.matvec(*g.plan, x, y, s, ready, done, joined);
                    };
                    try {
                        status = ipm_solve(*g.plan, g.labels, g.C[c], o, g.alpha + int64_t(c) * g.plan->N, &lam, &st,
                                           stream, &P.f, &hook);
                    } catch (...) {
                        comb.solver_leave(joined);
                        throw;
                    }
                    comb.solver_leave(joined);
                } catch (const Error& e) {
                    status = e.code;
                } catch (const std::exception&) {
                    status = ANOVA_HIP_ERROR;
                }
            }
            st.status = status;
            g.lambda[c] = lam;
            g.stats[c] = st;
            if (--P.left == 0) {  // the problem's last solve has finished
                P.f.Z.release();
                P.f.Z32.release();
            }
        }
        if (stream) {
            (void)hipStreamSynchronize(stream);
            (void)hipStreamDestroy(stream);
        }
        if (ready) (void)hipEventDestroy(ready);
        if (done) (void)hipEventDestroy(done);
    };
    std::vector<std::thread> pool;
    const int nthreads = int(std::min<size_t>(size_t(max_active), tasks.size()));
    for (int i = 0; i < nthreads; ++i) pool.emplace_back(worker);
    for (auto& th : pool) th.join();
    if (launches) *launches = comb.launches();
    if (matvecs) *matvecs = comb.matvecs();
}

}  // namespace anv
