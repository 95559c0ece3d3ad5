// Request server for interior point solves (continuous batching on one GPU).
#pragma once
#include <memory>

#include "common.hpp"

namespace anv {

class Server {
  public:
    Server(const anova_server_opts& o, int device);
    ~Server();
    int64_t submit(const anova_request& q);
    // blocks until the ticket's solve has finished; returns its status
    int wait(int64_t ticket, double* alpha, anova_result* res);
    void counters(int64_t* launches, int64_t* matvecs) const;
    struct Impl;

  private:
    std::unique_ptr<Impl> impl_;
};

struct Plan;

// One problem of a hyperparameter grid: a plan (data and kernel widths) with
// its labels and several values of C.
struct GridProblem {
    Plan* plan;
    const double* labels;     // N of the plan, device
    int nC;
    const double* C;          // host, nC
    double* alpha;            // device, N x nC column-major
    double* lambda;           // host, nC
    anova_ipm_stats* stats;   // host, nC; stats[c].status is the solve's status
};

// Runs every (problem, C) solve, up to max_active at once on their own
// streams; the solves of one problem share its low-rank factor, and matvecs
// of concurrent solves share launches (same-plan vectors batched). Returns
// when all have finished; per-solve failures are reported in the stats.
void grid_solve(const GridProblem* probs, int nprob, const anova_ipm_opts& o, int max_active, double gather_us,
                int device, int64_t* launches, int64_t* matvecs);

int64_t request_footprint(int64_t N, int32_t d, int32_t P, const anova_opts& nfft, const anova_ipm_opts& ipm);

}  // namespace anv
