// extern "C" entry points: argument checks, exception-to-status translation
// and the thread-local error message.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "plan.hpp"
#include "server.hpp"
#include "solver.hpp"
#include "tune.hpp"
#include "windows.hpp"

namespace anv {
static thread_local std::string g_last_error;
void set_last_error(const std::string& m) { g_last_error = m; }
}  // namespace anv

using anv::Error;

template <class F>
static int guarded(F&& f) {
    try {
        anv::set_last_error("");
        return f();
    } catch (const Error& e) {
        anv::set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        anv::set_last_error("host allocation failed");
        return ANOVA_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        anv::set_last_error(e.what());
        return ANOVA_HIP_ERROR;
    }
}

struct anova_plan_s {
    std::unique_ptr<anv::Plan> p;
};

struct anova_server_s {
    std::unique_ptr<anv::Server> s;
};

extern "C" {

int anova_opts_default(anova_opts* o) {
    if (!o) return ANOVA_INVALID_ARG;
    std::memset(o, 0, sizeof(*o));
    o->version = ANOVA_OPTS_VERSION;
    o->n_bw = 32;
    o->oversample = 2;
    o->cutoff_m = 4;
    o->eps_b = 0.25;
    o->reg_p = 0;
    o->precision = ANOVA_PREC_FP64;
    o->seg_points = 0;
    o->batch_min_rhs = 0;
    return ANOVA_OK;
}

int anova_plan_create(const double* X, int64_t N, int32_t d, int64_t ldx, const int32_t* windows,
                      int32_t P, const double* sigma, const double* eta, const anova_opts* opts,
                      void* stream, anova_plan_t* out) {
    return guarded([&] {
        ANV_CHECK(out != nullptr, "NULL output handle");
        *out = nullptr;
        auto h = std::make_unique<anova_plan_s>();
        h->p.reset(anv::create_plan(X, N, d, ldx, windows, P, sigma, eta, opts,
                                    static_cast<hipStream_t>(stream)));
        *out = h.release();
        return ANOVA_OK;
    });
}

int anova_matvec(anova_plan_t plan, const double* x, int32_t R, int64_t ldx_, double* y, int64_t ldy,
                 void* stream) {
    return guarded([&] {
        ANV_CHECK(plan && plan->p, "NULL plan");
        ANV_CHECK(x && y, "NULL vector");
        ANV_CHECK(R >= 1, "R < 1");
        ANV_CHECK(ldx_ >= plan->p->N && ldy >= plan->p->N, "leading dimension < N");
        anv::enqueue_matvec(*plan->p, x, R, ldx_, y, ldy, static_cast<hipStream_t>(stream));
        return ANOVA_OK;
    });
}

int anova_matvec_noalloc(anova_plan_t plan, const double* x, int32_t R, int64_t ldx_, double* y, int64_t ldy,
                         void* stream) {
    return guarded([&] {
        ANV_CHECK(plan && plan->p, "NULL plan");
        ANV_CHECK(x && y, "NULL vector");
        ANV_CHECK(R >= 1, "R < 1");
        ANV_CHECK(ldx_ >= plan->p->N && ldy >= plan->p->N, "leading dimension < N");
        anv::enqueue_matvec_noalloc(*plan->p, x, R, ldx_, y, ldy, static_cast<hipStream_t>(stream));
        return ANOVA_OK;
    });
}

int anova_kaiser_bessel(const anova_opts* opts, const double* u, int32_t nu, double* phi, double* phi_hat) {
    return guarded([&] {
        anova_opts o;
        anova_opts_default(&o);
        if (opts) o = *opts;
        ANV_CHECK(o.version == ANOVA_OPTS_VERSION, "anova_opts.version mismatch");
        ANV_CHECK(o.n_bw >= 4 && o.n_bw % 2 == 0 && o.oversample >= 2 && o.cutoff_m >= 1, "bad options");
        ANV_CHECK(nu >= 0 && (nu == 0 || (u && phi)), "NULL argument");
        const int n = o.oversample * o.n_bw, m = o.cutoff_m;
        const double b = M_PI * (2.0 - double(o.n_bw) / n);
        for (int32_t i = 0; i < nu; ++i) {
            ANV_CHECK(std::fabs(u[i]) <= double(m), "|u| > m");
            phi[i] = anv::kb_window(u[i], m, b);
        }
        if (phi_hat)
            for (int k = 0; k <= n / 2; ++k) phi_hat[k] = anv::kb_hat(k, n, m, b);
        return ANOVA_OK;
    });
}

int anova_axis_coefficients(double lo, double hi, double sigma, const anova_opts* opts, double* bk, double* circ,
                            double* axis, int32_t* reg_p) {
    return guarded([&] {
        anova_opts o;
        anova_opts_default(&o);
        if (opts) o = *opts;
        ANV_CHECK(o.version == ANOVA_OPTS_VERSION, "anova_opts.version mismatch");
        ANV_CHECK(o.n_bw >= 4 && o.n_bw % 2 == 0 && o.oversample >= 2 && o.cutoff_m >= 1, "bad options");
        ANV_CHECK(o.eps_b > 0.0 && o.eps_b < 0.5, "eps_b must be in (0, 1/2)");
        ANV_CHECK(std::isfinite(lo) && std::isfinite(hi) && lo <= hi, "need finite lo <= hi");
        ANV_CHECK(std::isfinite(sigma) && sigma > 0.0, "sigma must be > 0");
        anv::NfftParams prm;
        prm.n_bw = o.n_bw;
        prm.n_os = o.oversample * o.n_bw;
        prm.m = o.cutoff_m;
        prm.eps_b = o.eps_b;
        prm.reg_p = o.reg_p;
        const anv::AxisCoef ax = anv::build_axis(lo, hi, sigma, prm);
        if (bk) std::copy(ax.bk.begin(), ax.bk.end(), bk);
        if (circ) std::copy(ax.circ.begin(), ax.circ.end(), circ);
        if (axis) {
            axis[0] = ax.center;
            axis[1] = ax.scale;
            axis[2] = ax.sigma_a;
            axis[3] = ax.kerr;
        }
        if (reg_p) *reg_p = ax.reg_p;
        return ANOVA_OK;
    });
}

int anova_plan_destroy(anova_plan_t plan) {
    return guarded([&] {
        if (plan) {
            (void)hipDeviceSynchronize();
            delete plan;
        }
        return ANOVA_OK;
    });
}

int anova_plan_info(anova_plan_t plan, anova_plan_info_t* info) {
    return guarded([&] {
        ANV_CHECK(plan && plan->p && info, "NULL argument");
        const anv::Plan& p = *plan->p;
        std::memset(info, 0, sizeof(*info));
        info->n_points = p.N;
        info->n_windows = p.P;
        info->n_segments = int32_t(p.segs_h.size());
        info->cutoff_m = p.prm.m;
        info->precision = p.precision;
        info->eps_b = p.prm.eps_b;
        info->max_kernel_err = p.max_kerr;
        info->grid_cells = p.grid_total;
        info->device_bytes = p.device_bytes();
        return ANOVA_OK;
    });
}

int anova_profile_begin(anova_plan_t plan) {
    return guarded([&] {
        ANV_CHECK(plan && plan->p, "NULL plan");
        anv::profile_begin(*plan->p);
        return ANOVA_OK;
    });
}

int anova_profile_end(anova_plan_t plan, double* stage_ms, int32_t nstage, int32_t* passes) {
    return guarded([&] {
        ANV_CHECK(plan && plan->p, "NULL plan");
        ANV_CHECK(stage_ms && nstage >= 0, "NULL stage_ms");
        int n = anv::profile_end(*plan->p, stage_ms, nstage);
        if (passes) *passes = n;
        return ANOVA_OK;
    });
}

int anova_ipm_opts_default(anova_ipm_opts* o) {
    if (!o) return ANOVA_INVALID_ARG;
    std::memset(o, 0, sizeof(*o));
    o->version = ANOVA_IPM_OPTS_VERSION;
    o->factor_fp32 = 1;
    o->max_ip = 100;
    o->max_kry = 100;
    o->precond = ANOVA_PRECOND_PCHOL;
    o->tol = 1e-6;
    o->tol_inf = 1e-1;
    o->tol_kry = 1e-3;
    o->sigma_bar = 0.6;
    o->gamma0 = 0.99995;
    o->mu0 = 1.0;
    o->rank = 200;
    o->err_tol = 1e-5;
    o->seed = 0;
    o->graphs = 1;
    return ANOVA_OK;
}

int svm_ipm_solve(anova_plan_t plan, const double* labels, double C, const anova_ipm_opts* opts,
                  double* alpha, double* lambda, anova_ipm_stats* stats, void* stream) {
    return guarded([&] {
        ANV_CHECK(plan && plan->p, "NULL plan");
        anova_ipm_opts o;
        anova_ipm_opts_default(&o);
        if (opts) {
            ANV_CHECK(opts->version == ANOVA_IPM_OPTS_VERSION, "anova_ipm_opts.version mismatch");
            o = *opts;
        }
        return anv::ipm_solve(*plan->p, labels, C, o, alpha, lambda, stats,
                              static_cast<hipStream_t>(stream));
    });
}

int anova_pivoted_cholesky(anova_plan_t plan, int32_t rank, double err_tol, double* L, int64_t ldl,
                           int64_t* piv, int32_t* rank_used, void* stream) {
    return guarded([&] {
        ANV_CHECK(plan && plan->p, "NULL plan");
        ANV_CHECK(L && piv && rank_used, "NULL output");
        ANV_CHECK(rank >= 1 && rank <= plan->p->N, "rank must be in [1, N]");
        ANV_CHECK(ldl >= plan->p->N, "ldl < N");
        ANV_CHECK(err_tol >= 0.0, "err_tol < 0");
        *rank_used = anv::pivoted_cholesky(*plan->p, rank, err_tol, L, ldl, piv,
                                           static_cast<hipStream_t>(stream));
        return ANOVA_OK;
    });
}

int anova_rp_cholesky(anova_plan_t plan, int32_t rank, double err_tol, const double* uniforms, double* L,
                      int64_t ldl, int64_t* piv, int32_t* rank_used, void* stream) {
    return guarded([&] {
        ANV_CHECK(plan && plan->p, "NULL plan");
        ANV_CHECK(L && piv && rank_used && uniforms, "NULL argument");
        ANV_CHECK(rank >= 1 && rank <= plan->p->N, "rank must be in [1, N]");
        ANV_CHECK(ldl >= plan->p->N, "ldl < N");
        ANV_CHECK(err_tol >= 0.0, "err_tol < 0");
        for (int32_t j = 0; j < rank; ++j)
            ANV_CHECK(uniforms[j] >= 0.0 && uniforms[j] < 1.0, "uniforms must lie in [0, 1)");
        *rank_used = anv::pivoted_cholesky(*plan->p, rank, err_tol, L, ldl, piv, static_cast<hipStream_t>(stream),
                                           uniforms);
        return ANOVA_OK;
    });
}

int anova_rff_factor(anova_plan_t plan, int32_t k, const double* w, const double* b, double* Z, int64_t ldz,
                     void* stream) {
    return guarded([&] {
        ANV_CHECK(plan && plan->p, "NULL plan");
        ANV_CHECK(w && b && Z, "NULL argument");
        for (int64_t i = 0; i < int64_t(k) * 3; ++i) ANV_CHECK(std::isfinite(w[i]), "w must be finite");
        for (int32_t j = 0; j < k; ++j) ANV_CHECK(std::isfinite(b[j]), "b must be finite");
        anv::rff_factor(*plan->p, k, w, b, Z, ldz, static_cast<hipStream_t>(stream));
        return ANOVA_OK;
    });
}

int anova_nystrom(anova_plan_t plan, const double* G, int32_t k, int64_t ldg, double* Zt, int64_t ldz,
                  void* stream) {
    return guarded([&] {
        ANV_CHECK(plan && plan->p, "NULL plan");
        ANV_CHECK(G && Zt, "NULL pointer");
        ANV_CHECK(k >= 1 && k <= plan->p->N, "k must be in [1, N]");
        ANV_CHECK(ldg >= plan->p->N && ldz >= plan->p->N, "leading dimension < N");
        anv::nystrom_factor(*plan->p, G, k, ldg, Zt, ldz, static_cast<hipStream_t>(stream));
        return ANOVA_OK;
    });
}

int anova_lowrank_apply(int64_t N, int32_t k, const double* Z, int64_t ldz, const double* theta, const double* y,
                        const double* r, int32_t fp32_products, double* out, void* stream) {
    return guarded([&] {
        ANV_CHECK(fp32_products == 0 || fp32_products == 1, "fp32_products must be 0 or 1");
        anv::lowrank_apply(N, k, Z, ldz, theta, y, r, fp32_products != 0, out, static_cast<hipStream_t>(stream));
        return ANOVA_OK;
    });
}

int anova_server_opts_default(anova_server_opts* o) {
    if (!o) return ANOVA_INVALID_ARG;
    std::memset(o, 0, sizeof(*o));
    o->version = ANOVA_SERVER_OPTS_VERSION;
    o->max_active = 8;
    o->hbm_budget = 0;
    o->share_launches = 1;
    o->gather_us = 200.0;
    return ANOVA_OK;
}

int anova_server_create(const anova_server_opts* opts, int32_t device, anova_server_t* out) {
    return guarded([&] {
        ANV_CHECK(out != nullptr, "NULL output handle");
        *out = nullptr;
        anova_server_opts o;
        anova_server_opts_default(&o);
        if (opts) {
            ANV_CHECK(opts->version == ANOVA_SERVER_OPTS_VERSION, "anova_server_opts.version mismatch");
            o = *opts;
        }
        ANV_CHECK(o.max_active >= 1 && o.max_active <= 64, "max_active must be in [1, 64]");
        ANV_CHECK(o.gather_us >= 0.0 && o.gather_us <= 1e6, "gather_us must be in [0, 1e6]");
        int ndev = 0;
        ANV_HIP(hipGetDeviceCount(&ndev));
        ANV_CHECK(device >= 0 && device < ndev, "no such device");
        auto h = std::make_unique<anova_server_s>();
        h->s.reset(new anv::Server(o, device));
        *out = h.release();
        return ANOVA_OK;
    });
}

int anova_server_submit(anova_server_t s, const anova_request* req, int64_t* ticket) {
    return guarded([&] {
        ANV_CHECK(s && req && ticket, "NULL argument");
        *ticket = s->s->submit(*req);
        return ANOVA_OK;
    });
}

int anova_server_wait(anova_server_t s, int64_t ticket, double* alpha, anova_result* result) {
    return guarded([&] {
        ANV_CHECK(s != nullptr, "NULL server");
        return s->s->wait(ticket, alpha, result);
    });
}

int anova_server_counters(anova_server_t s, int64_t* launches, int64_t* matvecs) {
    return guarded([&] {
        ANV_CHECK(s && launches && matvecs, "NULL argument");
        s->s->counters(launches, matvecs);
        return ANOVA_OK;
    });
}

int anova_server_destroy(anova_server_t s) {
    return guarded([&] {
        delete s;
        return ANOVA_OK;
    });
}

int anova_request_footprint(int64_t N, int32_t d, int32_t P, const anova_opts* nfft, const anova_ipm_opts* ipm,
                            int64_t* bytes) {
    return guarded([&] {
        ANV_CHECK(bytes != nullptr, "NULL output");
        ANV_CHECK(N >= 1 && d >= 1 && P >= 1, "bad sizes");
        anova_opts o;
        anova_opts_default(&o);
        if (nfft) o = *nfft;
        anova_ipm_opts io;
        anova_ipm_opts_default(&io);
        if (ipm) io = *ipm;
        *bytes = anv::request_footprint(N, d, P, o, io);
        return ANOVA_OK;
    });
}

int anova_grid_solve(const anova_grid_problem* problems, int32_t n_problems, const anova_ipm_opts* opts,
                     int32_t max_active, double gather_us, int64_t* launches, int64_t* matvecs) {
    return guarded([&] {
        ANV_CHECK(problems && n_problems >= 1, "no problems");
        anova_ipm_opts o;
        anova_ipm_opts_default(&o);
        if (opts) {
            ANV_CHECK(opts->version == ANOVA_IPM_OPTS_VERSION, "anova_ipm_opts.version mismatch");
            o = *opts;
        }
        std::vector<anv::GridProblem> g(static_cast<size_t>(n_problems));
        for (int32_t i = 0; i < n_problems; ++i) {
            const anova_grid_problem& q = problems[i];
            ANV_CHECK(q.plan && q.plan->p, "NULL plan");
            g[i] = anv::GridProblem{q.plan->p.get(), q.labels, q.n_c, q.C, q.alpha, q.lambda, q.stats};
        }
        int device = 0;
        ANV_HIP(hipGetDevice(&device));
        anv::grid_solve(g.data(), n_problems, o, max_active, gather_us, device, launches, matvecs);
        return ANOVA_OK;
    });
}

int anova_decision_function(const double* X, int64_t N, int64_t ldx, const double* Xnew, int64_t M,
                            int64_t ldn, int32_t d, const int32_t* windows, int32_t P, const double* sigma,
                            const double* eta, const anova_opts* opts, const double* labels,
                            const double* alpha, double lambda, double* f, void* stream) {
    return guarded([&] {
        anv::decision_function(X, N, ldx, Xnew, M, ldn, d, windows, P, sigma, eta, opts, labels, alpha, lambda, f,
                               static_cast<hipStream_t>(stream));
        return ANOVA_OK;
    });
}

int anova_tune_opts_default(anova_tune_opts* t) {
    if (!t) return ANOVA_INVALID_ARG;
    std::memset(t, 0, sizeof(*t));
    t->version = ANOVA_TUNE_OPTS_VERSION;
    t->rhs = 1;
    t->target_rel_err = 1e-4;
    t->precisions = 3;
    t->reps = 3;
    t->seed = 0;
    return ANOVA_OK;
}

int anova_autotune(const double* X, int64_t N, int32_t d, int64_t ldx, const int32_t* windows, int32_t P,
                   const double* sigma, const double* eta, const anova_tune_opts* t, void* stream,
                   anova_opts* best, anova_tune_candidate* cands, int32_t max_cands, int32_t* n_cands) {
    return guarded([&] {
        ANV_CHECK(best != nullptr, "NULL output");
        ANV_CHECK(cands == nullptr || max_cands >= 0, "max_cands < 0");
        anova_tune_opts o;
        anova_tune_opts_default(&o);
        if (t) {
            ANV_CHECK(t->version == ANOVA_TUNE_OPTS_VERSION, "anova_tune_opts.version mismatch");
            o = *t;
        }
        anv::autotune(X, N, d, ldx, windows, P, sigma, eta, o, static_cast<hipStream_t>(stream), best, cands,
                      max_cands, n_cands);
        return ANOVA_OK;
    });
}

int anova_mi_windows(const double* X, int64_t N, int32_t d, int64_t ldx, const double* labels, int32_t bins,
                     int32_t P, int32_t* windows, double* mi, void* stream) {
    return guarded([&] {
        anv::mi_windows(X, N, d, ldx, labels, bins, P, windows, mi, static_cast<hipStream_t>(stream));
        return ANOVA_OK;
    });
}

const char* anova_last_error(void) { return anv::g_last_error.c_str(); }

}  // extern "C"
