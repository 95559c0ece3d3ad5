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

int64_t request_footprint(int64_t N, int32_t d, int32_t P, const anova_opts& nfft, const anova_ipm_opts& ipm);

}  // namespace anv
