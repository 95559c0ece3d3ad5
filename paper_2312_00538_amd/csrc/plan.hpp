// The fast-summation plan: everything that depends only on (X, windows, sigma).
#pragma once
#include <array>
#include <functional>
#include <memory>

#include "common.hpp"

namespace anv {

struct Plan {
    int64_t N = 0;
    int32_t d = 0, P = 0;
    int32_t W = 8;              // taps per axis = 2m
    NfftParams prm;
    int32_t precision = ANOVA_PREC_FP64;
    int32_t seg_points = 768;   // work-item length for 3-feature windows
    int32_t seg_points_lane = 128;  // work-item length for 1- and 2-feature windows (set by the plan)
    std::vector<int32_t> win;   // P x 3 as given
    std::vector<double> sigma, eta;
    std::vector<std::array<int32_t, 3>> slot_feat;  // feature per slot, -1 = dummy
    std::vector<std::array<AxisCoef, 3>> axes;
    std::vector<WinDev> wins_h;
    DevBuf<WinDev> wins_d;

    // per (window, sorted position): point index, base z cell, Kaiser-Bessel weights
    DevBuf<int32_t> perm;       // [P*N] sorted position -> point
    DevBuf<int32_t> pos;        // [P*N] point -> sorted position
    DevBuf<int32_t> zq;         // [P*N]
    DevBuf<double> wts64;       // [P*N][3][W]
    DevBuf<float> wts32;        // same, mixed precision

    std::vector<Segment> segs_h;
    DevBuf<Segment> segs;
    DevBuf<int2> fold;          // per (window, column, layer): covering segment range
    DevBuf<int64_t> sbase;      // per segment: slab offset - z0 * lanes
    // wavefront tables: for windows with 3, 2, 1 features, the work items each
    // wavefront handles (64/W per wave for 3 features, 64 otherwise; -1 = none)
    DevBuf<int32_t> wave_items;
    // per 3-feature work item: start of each of its layers relative to its first point
    // (z1 - z0 + 2 entries), at lstart[lstart_off[item]]
    DevBuf<int32_t> lstart, lstart_off;
    // per work item: 1 if it is the only item of its column (3-feature windows write
    // such items straight into the fold's target-major buffer)
    DevBuf<uint8_t> alone;
    // fold entries (window, column, layer) that need the slab reduction, and per
    // column the layers holding data in the target-major buffer (x > y = none)
    DevBuf<int64_t> flist;
    int64_t nflist = 0;
    int64_t nflist3 = 0;        // entries [0, nflist3) belong to 3-feature windows
    DevBuf<int2> crange;
    int64_t wave_off[4] = {0, 0, 0, 0};
    int32_t nwave[4] = {0, 0, 0, 0};
    int64_t fold_total = 0;
    DevBuf<double> tmat;        // Toeplitz matrices, row-major E x E per (window, slot)
    int64_t tmat_total = 0;
    int64_t grid_total = 0;     // occupied cells summed over windows
    int64_t grid_max = 0;       // largest window grid
    int32_t emax[3] = {1, 1, 1}; // largest occupied extent per slot over windows
    int64_t slab_total = 0;
    int64_t tgt_total = 0;      // fold target-major buffer: cells x footprint positions

    // original windowed coordinates [N][P][3] (exact kernel columns)
    DevBuf<double> xw;

    // matvec scratch
    DevBuf<double> vs, fs;      // [P*N]
    DevBuf<double> g64, h64, c64a, c64b;  // grids [grid_total]
    DevBuf<float> g32, h32, c32a, c32b;
    DevBuf<double> slab64;
    DevBuf<float> slab32;

    // batched path (16 right-hand sides per pass; FP32 elements for mixed
    // precision, FP64 for FP64 plans), allocated on first use: inputs [N][16]
    // (point order), slabs, fold targets, grids and gathered values, each with
    // the 16 right-hand sides innermost (storage in doubles, either element type)
    int32_t batch_min_rhs = 2;
    bool b_ready = false;
    int32_t b_rsplit = 2;       // grid-step blocks per slice (right-hand sides split for LDS)
    DevBuf<double> xtb, fsb, slabb, tgtb, g1b, hb;
    DevBuf<int32_t> b_items;    // work items of 2-feature then 1-feature windows
    DevBuf<int32_t> b_queue;    // work-queue counters of the matrix-core spread and gather
    int32_t b_grid[2] = {1, 1}; // their persistent grid sizes
    int32_t nb_items2 = 0, nb_items1 = 0;

    // stage timing (measurement hook)
    bool profiling = false;
    std::vector<hipEvent_t> events;
    size_t events_used = 0;
    void record_stage_event(hipStream_t st);

    double max_kerr = 0.0;
    ~Plan();
    int64_t device_bytes() const;
};

// One plan's share of a matvec launch that may serve several plans at once
// (pointers to the plan's arrays and scratch, the caller's vectors, sizes).
constexpr int kMaxJobs = 8;
struct MvJob {
    const double* x;
    double* y;
    const int32_t* perm;
    const int32_t* pos;
    const int32_t* zq;
    const void* wts;
    const Segment* segs;
    const int32_t* lstart;
    const int32_t* lstart_off;
    const WinDev* wins;
    const uint8_t* alone;
    const int32_t* wave_items;
    const int64_t* flist;
    const int2* fold;
    const int64_t* sbase;
    const int2* crange;
    const double* tmat;
    double* vs;
    double* fs;
    void* slab;
    void* g;
    void* h;
    void* ca;
    int64_t N;
    int64_t nflist;
    int64_t nflist3;
    int64_t wave_off[4];
    int32_t nwave[4];
    int32_t P;
    int32_t emax[3];
};
// Passed to every kernel by value: the jobs and, per kernel, the first block
// of each job.
struct MvLaunch {
    MvJob job[kMaxJobs];
    int32_t njobs;
    int32_t off[kMaxJobs + 1];
};
static_assert(sizeof(MvLaunch) < 4000, "kernel argument block");

Plan* create_plan(const double* X, int64_t N, int32_t d, int64_t ldx, const int32_t* windows,
                  int32_t P, const double* sigma, const double* eta, const anova_opts* opts,
                  hipStream_t stream);

// y[:, r] = K x[:, r] for r < R (device pointers, column-major with leading dims).
void enqueue_matvec(Plan& pl, const double* x, int R, int64_t ldx, double* y, int64_t ldy,
                    hipStream_t stream);

// y[:, r] = K x[:, r] one vector at a time, with every scratch array of the
// pass placed in a static per-device array of kNoAllocScratchBytes instead of
// the plan's buffers: no device memory is allocated. Plans whose one-vector
// scratch (noalloc_scratch_bytes) exceeds the maximum are rejected
// (ANOVA_INVALID_ARG). All calls on a device share its array, so calls that
// overlap on one device race.
constexpr size_t kNoAllocScratchBytes = size_t(ANOVA_NOALLOC_SCRATCH_BYTES);
size_t noalloc_scratch_bytes(const Plan& pl);
void enqueue_matvec_noalloc(Plan& pl, const double* x, int R, int64_t ldx, double* y, int64_t ldy,
                            hipStream_t stream);

// The 16-wide batched kernels (matvec_batched.hip): used by enqueue_matvec for
// R >= batch_min_rhs when batched_supported(pl).
bool batched_supported(const Plan& pl);
void enqueue_matvec_batched(Plan& pl, const double* x, int R, int64_t ldx, double* y, int64_t ldy,
                            hipStream_t stream);
// frees the batched path's buffers (and the FP32 weights of an FP64 plan)
void release_batched_buffers(Plan& pl);

// y_i = K_i x_i for n (plan, vector) pairs, one vector per plan: the plans'
// stages share launches (grouped by cutoff and precision, up to kMaxJobs plans).
void enqueue_matvec_multi(Plan* const* plans, const double* const* x, double* const* y, int n,
                          hipStream_t stream);
// batched matvec of R vectors given by column pointers (N doubles each)
void enqueue_matvec_batched_cols(Plan& pl, const double* const* x, double* const* y, int R, hipStream_t stream);
// y_i = K_i x_i for n (plan, vector) pairs in which a plan may repeat: the
// vectors of a plan that the batched path supports go through it together
// (any number, also one, so that a vector's result does not depend on the
// others in the call); the rest as in enqueue_matvec_multi.
void enqueue_matvec_grouped(Plan* const* plans, const double* const* x, double* const* y, int n,
                            hipStream_t stream);

void profile_begin(Plan& pl);
int profile_end(Plan& pl, double* stage_ms, int nstage);  // returns passes measured

}  // namespace anv
