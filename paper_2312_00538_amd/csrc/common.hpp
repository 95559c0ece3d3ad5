// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/anova_nfft.h"

namespace anv {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define ANV_HIP(x)                                                                       \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess)                                                            \
            throw ::anv::Error(e_ == hipErrorOutOfMemory ? ANOVA_OUT_OF_MEMORY           \
                                                         : ANOVA_HIP_ERROR,              \
                               std::string(#x) + ": " + hipGetErrorString(e_));          \
    } while (0)

#define ANV_CHECK(cond, msg)                                                             \
    do {                                                                                 \
        if (!(cond)) throw ::anv::Error(ANOVA_INVALID_ARG, (msg));                       \
    } while (0)

void set_last_error(const std::string& m);

// Host waits of the solver. By default a wait spins (lowest latency, right for
// one solve at a time); a thread that runs one of many concurrent solves turns
// on blocking waits (BlockingWaits), which sleep until the GPU signals, so
// that dozens of waiting threads leave the host cores to the threads that
// launch work.
extern thread_local bool t_blocking_waits;
void host_wait(hipStream_t st);
struct BlockingWaits {
    bool prev;
    BlockingWaits() : prev(t_blocking_waits) { t_blocking_waits = true; }
    ~BlockingWaits() { t_blocking_waits = prev; }
};

// Device allocation owned by a plan or a solver; freed in the destructor.
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) count = 1;
        ANV_HIP(hipMalloc(&p, count * sizeof(T)));
        n = count;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// ---------------------------------------------------------------- coefficients
// One axis of one window: the affine map onto the torus box, the width of the
// 1D Gaussian in torus units, and the first column of the real symmetric
// circulant that the grid step applies along this axis.
struct AxisCoef {
    double lo = 0, hi = 0;        // data range of the feature
    double center = 0, scale = 1; // u = (x - center) * scale, |u| <= (1/2 - eps_b)/2
    double sigma_a = 1;           // sigma * scale
    int reg_p = 0;                // smoothness of the regularisation used
    double kerr = 0;              // max |trig interpolant - Gaussian| on the box
    std::vector<double> circ;     // circ[delta], delta = 0..n_os-1
    std::vector<double> bk;       // b_k, k = -n_bw/2 .. n_bw/2 - 1 (index k + n_bw/2)
};

struct NfftParams {
    int n_bw = 32, n_os = 64, m = 4;
    double eps_b = 0.25;
    int reg_p = 0;
};

// Builds the axis coefficients (host, FP64). Defined in coeffs.cpp.
AxisCoef build_axis(double lo, double hi, double sigma, const NfftParams& prm);

// Normalised Kaiser-Bessel window phi(u)/phi(0) at offset u (grid cells), |u| <= m.
double kb_window(double u, int m, double b);
// Its Fourier transform divided by phi(0), at integer frequency k for FFT length n.
double kb_hat(int k, int n, int m, double b);

// ---------------------------------------------------------------- plan
constexpr int kMaxW = 8;  // 2m for the supported cutoffs m <= 4
// layers a work item spans at most (its z1 - z0 + 1): its z1 - z0 + 2 layer
// starts then fit one per lane of a wavefront
constexpr int kItemLayers = 62;

// elements per point record of Kaiser-Bessel weights (x, y, z taps), padded to
// a multiple of 16 bytes so records can be moved in 16-byte pieces
__host__ __device__ constexpr int rec_stride(int W, int elem_bytes) {
    return ((3 * W * elem_bytes + 15) / 16) * 16 / elem_bytes;
}

struct WinDev {          // per-window geometry read by the kernels
    int32_t E[3];        // occupied grid extent per slot (x, y, z); 1 for a dummy slot
    int32_t nb[3];       // number of base cells per slot = E - Wslot + 1
    int32_t Wslot[3];    // taps per slot: W, or 1 for a dummy slot
    int32_t lanes;       // Wslot[0] * Wslot[1]
    int64_t grid_off;    // offset of this window's grid in the grid buffers
    int64_t fold_off;    // offset of this window's fold index
    int64_t t_off[3];    // offsets of the Toeplitz matrices (E x E, row-major)
    int64_t tgt_off;     // offset of this window in the fold's target-major buffer
    int64_t col_off;     // index of this window's first column in per-column tables
    double eta;
    int32_t pad;
};

struct Segment {         // one spreading/gathering work item (one wavefront)
    int32_t win, col, start, count, z0, z1;
    int64_t off;         // slab offset (elements)
};
static_assert(sizeof(Segment) == 32, "segment layout");

}  // namespace anv
