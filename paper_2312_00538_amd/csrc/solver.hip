// Low-rank kernel factors (Section 4), the preconditioned Krylov solve of the
// Newton system (Sections 2 and 5) and the interior point method (Algorithm 1).
//
// All solver arithmetic is FP64 on the device. Reductions are deterministic:
// every block folds its part in a fixed tree order and a single block then adds
// the block partials in block order, so a solve is bitwise reproducible.
// The host drives the iterations and reads back a few scalars per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>

#include "solver.hpp"

namespace anv {

namespace {

constexpr int kT = 256;        // threads per block of the vector kernels
constexpr int kRedBlocks = 512; // blocks of the partial-sum reductions
inline unsigned nblk(int64_t n, int t = kT) { return unsigned(std::max<int64_t>(1, (n + t - 1) / t)); }

// ------------------------------------------------------------------ reductions
template <int NS>
__device__ void block_sums(double (&v)[NS], double* __restrict__ out) {
    __shared__ double sh[NS][kT];
#pragma unroll
    for (int q = 0; q < NS; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < NS; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NS; ++q) out[blockIdx.x * NS + q] = sh[q][0];
    }
}

// fold block partials [nb][ns]: out[q] = sum_b part[b][q], one wavefront per q;
// lane j adds blocks j, j + 64, ... in order, then a fixed xor tree adds the lanes
__global__ void k_fold_partials(const double* __restrict__ part, int nb, int ns, double* __restrict__ out) {
    const int q = blockIdx.x, j = threadIdx.x;
    double s = 0.0;
#pragma unroll 8
    for (int b = j; b < nb; b += 64) s += part[b * ns + q];  // unrolled: the loads go out together
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (j == 0) out[q] = s;
}

// up to 4 dot products sum_i a_q[i] * b_q[i] over [0, n)
struct DotArgs {
    const double* a[4];
    const double* b[4];
};
template <int NS>
__global__ void k_dots(DotArgs d, int64_t n, double* __restrict__ part) {
    double v[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) v[q] = 0.0;
    for (int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT) {
#pragma unroll
        for (int q = 0; q < NS; ++q) v[q] += d.a[q][i] * d.b[q][i];
    }
    block_sums<NS>(v, part);
}

// ------------------------------------------------------------------ kernel columns
// col[i] = sum_l eta_l exp(-sum_a (x_ia - x_pa)^2 / sigma_l^2) - sum_{j<r} L_ij L_pj,
// L[:, r] = col / sqrt(col_p), d -= L[:, r]^2. (Column form of Algorithm 2.)
__global__ void k_pchol_column(const double* __restrict__ xw, int64_t N, int32_t P,
                               const double* __restrict__ inv_s2, const double* __restrict__ eta,
                               int64_t p, int r, double* __restrict__ L, double* __restrict__ dres,
                               double pivval) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i >= N) return;
    const double* xi = xw + i * P * 3;
    const double* xp = xw + p * P * 3;
    double kv = 0.0;
    for (int l = 0; l < P; ++l) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double df = xi[3 * l + a] - xp[3 * l + a];
            s += df * df;
        }
        kv += eta[l] * exp(-s * inv_s2[l]);
    }
    for (int j = 0; j < r; ++j) kv -= L[j * N + i] * L[j * N + p];
    double lv = kv / sqrt(pivval);
    L[int64_t(r) * N + i] = lv;
    double dn = dres[i] - lv * lv;
    dres[i] = (i == p) ? 0.0 : dn;
}

// Randomly pivoted Cholesky (Section 4 names it beside the greedy rule): the
// pivot is drawn with probability proportional to the residual diagonal. With
// C_i = sum_{t <= i} max(d_t, 0) and a uniform u in [0, 1), the pivot is the
// smallest i with C_i > u C_{N-1}. Block b sums [b chunk, (b + 1) chunk).
__global__ void k_block_sums(const double* __restrict__ d, int64_t n, int64_t chunk, double* __restrict__ psum) {
    __shared__ double ss[kT];
    const int64_t i0 = int64_t(blockIdx.x) * chunk, i1 = std::min<int64_t>(n, i0 + chunk);
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kT) s += fmax(d[i], 0.0);
    ss[threadIdx.x] = s;
    __syncthreads();
    for (int k = kT / 2; k > 0; k >>= 1) {
        if (int(threadIdx.x) < k) ss[threadIdx.x] += ss[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) psum[blockIdx.x] = ss[0];
}

// one thread: out = {d[pivot], pivot, total}; the block whose range holds the
// crossing is found from the block sums, then its elements are walked in order
__global__ void k_sample_pivot(const double* __restrict__ d, int64_t n, int64_t chunk,
                               const double* __restrict__ psum, int nb, double u, double* __restrict__ out) {
    double total = 0.0;
    for (int b = 0; b < nb; ++b) total += psum[b];
    const double target = u * total;
    double acc = 0.0;
    int b = 0;
    while (b + 1 < nb && acc + psum[b] <= target) acc += psum[b++];
    int64_t i = int64_t(b) * chunk, pick = -1, last = -1;
    const int64_t i1 = std::min<int64_t>(n, i + chunk);
    for (; i < i1; ++i) {
        const double v = fmax(d[i], 0.0);
        if (v > 0.0) last = i;
        acc += v;
        if (acc > target && v > 0.0) {
            pick = i;
            break;
        }
    }
    if (pick < 0) pick = last >= 0 ? last : 0;  // rounding at the end of the range
    out[0] = d[pick];
    out[1] = double(pick);
    out[2] = total;
}

// Random Fourier features (Section 4, with Bochner's theorem for the Gaussian of
// each window): column j of Z^T (N x k, column-major) belongs to window fwin[j]
// and is fscale[j] cos(w_j^T x^{W} + b_j), w_j given per coordinate slot.
__global__ void k_rff(const double* __restrict__ xw, int64_t N, int32_t P, const int32_t* __restrict__ fwin,
                      const double* __restrict__ fw, const double* __restrict__ fb,
                      const double* __restrict__ fscale, double* __restrict__ Z) {
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= N) return;
    const double* x = xw + (i * P + fwin[j]) * 3;
    const double t = fb[j] + fw[3 * j] * x[0] + fw[3 * j + 1] * x[1] + fw[3 * j + 2] * x[2];
    Z[int64_t(j) * N + i] = fscale[j] * cos(t);
}

// residual diagonal of the pivot: K_pp - sum_j L_pj^2 (one thread)
__global__ void k_pivot_value(const double* __restrict__ L, int64_t N, int64_t p, int r, double kpp,
                              double* __restrict__ out) {
    double v = kpp;
    for (int j = 0; j < r; ++j) v -= L[j * N + p] * L[j * N + p];
    out[0] = v;
}

// block partials of (max value, its lowest index, sum) of d
__global__ void k_argmax_sum(const double* __restrict__ d, int64_t n, double* __restrict__ pval,
                             int64_t* __restrict__ pidx, double* __restrict__ psum) {
    __shared__ double sv[kT], ss[kT];
    __shared__ int64_t si[kT];
    double best = -INFINITY, sum = 0.0;
    int64_t bi = INT64_MAX;
    for (int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT) {
        double v = d[i];
        sum += v;
        if (v > best) {  // indices increase along the stride, so '>' keeps the lowest
            best = v;
            bi = i;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    ss[threadIdx.x] = sum;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            double v2 = sv[threadIdx.x + s];
            int64_t i2 = si[threadIdx.x + s];
            if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
                sv[threadIdx.x] = v2;
                si[threadIdx.x] = i2;
            }
            ss[threadIdx.x] += ss[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pval[blockIdx.x] = sv[0];
        pidx[blockIdx.x] = si[0];
        psum[blockIdx.x] = ss[0];
    }
}

// out = {largest value (ties: smallest index), its index, sum of the block
// sums}: lane j takes blocks j, j + 64, ... in order, then a fixed xor tree
// combines the lanes (the argmax does not depend on the order; the sum's order
// is fixed)
__global__ void k_argmax_final(const double* __restrict__ pval, const int64_t* __restrict__ pidx,
                               const double* __restrict__ psum, int nb, double* __restrict__ out) {
    double best = -INFINITY, sum = 0.0;
    int64_t bi = INT64_MAX;
#pragma unroll 4
    for (int b = threadIdx.x; b < nb; b += 64) {
        const double v = pval[b];
        const int64_t i = pidx[b];
        if (v > best || (v == best && i < bi)) {
            best = v;
            bi = i;
        }
        sum += psum[b];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double v = __shfl_xor(best, o, 64);
        const int64_t i = __shfl_xor(bi, o, 64);
        if (v > best || (v == best && i < bi)) {
            best = v;
            bi = i;
        }
        sum += __shfl_xor(sum, o, 64);
    }
    if (threadIdx.x == 0) {
        out[0] = best;
        out[1] = double(bi);
        out[2] = sum;
    }
}

__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < n) x[i] = v;
}

// ------------------------------------------------------------------ low-rank products
// part[c] = sum_{i in chunk c} A_i B_i^T / theta_i (k x k; theta NULL = 1): one block per
// 16 x 16 output tile and row chunk; the chunk partials are folded in order.
constexpr int kSy = 16;
__global__ void k_gram_partial(const double* __restrict__ Z, const double* __restrict__ Zb, int64_t N, int k,
                               const double* __restrict__ theta, int64_t chunk,
                               double* __restrict__ part) {
    // block: (tile a, tile b, chunk c); threads 16 x 16
    const int ta = blockIdx.x, tb = blockIdx.y, c = blockIdx.z;
    const int ia = ta * kSy + threadIdx.x / kSy, ib = tb * kSy + threadIdx.x % kSy;
    __shared__ double za[64][kSy], zb[64][kSy], wt[64];
    const int64_t i0 = int64_t(c) * chunk, i1 = std::min<int64_t>(N, i0 + chunk);
    double acc = 0.0;
    for (int64_t ib0 = i0; ib0 < i1; ib0 += 64) {
        for (int e = threadIdx.x; e < 64 * kSy; e += kT) {
            int rr = e / kSy, cc = e % kSy;
            int64_t i = ib0 + rr;
            int ca = ta * kSy + cc, cb = tb * kSy + cc;
            za[rr][cc] = (i < i1 && ca < k) ? Z[int64_t(ca) * N + i] : 0.0;
            zb[rr][cc] = (i < i1 && cb < k) ? Zb[int64_t(cb) * N + i] : 0.0;
        }
        for (int e = threadIdx.x; e < 64; e += kT) {
            int64_t i = ib0 + e;
            wt[e] = (i < i1) ? (theta ? 1.0 / theta[i] : 1.0) : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int rr = 0; rr < 64; ++rr) acc += za[rr][threadIdx.x / kSy] * zb[rr][threadIdx.x % kSy] * wt[rr];
        __syncthreads();
    }
    if (ia < k && ib < k) part[(int64_t(c) * k + ia) * k + ib] = acc;
}

// Weighted Gram matrix on the FP64 matrix cores (v_mfma_f64_16x16x4f64), the
// factor stored in FP64 or as its FP32 copy (read as FP32, multiplied and
// summed in FP64, so that the matrix is exactly the Gram matrix of the stored
// values up to FP64 rounding, as the Woodbury applies that use it assume):
// part[c][a][b] = sum_{i in chunk c} Z_a(i) Z_b(i) / theta_i for a >= b (the
// upper triangle is filled only inside diagonal super-tiles). Block = 4 waves on
// one pair (sa >= sb) of 128-column super-tiles and one row chunk; wave w owns
// tile rows 2w, 2w+1 x all 8 tile columns (16 accumulators of 16 x 16). Rows go
// through LDS in panels of 16 (four k-steps of 4 rows). FP64 16x16x4 operand
// layout: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; element e of
// the result is D[l / 16 + 4 e][l % 16].
constexpr int kST = 128;   // super-tile columns
constexpr int kSP = 16;    // panel rows
template <class ZT>
__global__ __launch_bounds__(256) void k_syrk_mfma(const ZT* __restrict__ Z, int64_t N, int k,
                                                   const double* __restrict__ theta, int64_t chunk,
                                                   double* __restrict__ part) {
    typedef double d4 __attribute__((ext_vector_type(4)));
    __shared__ double pa[kST][kSP + 1], pb[kST][kSP + 1], wt[kSP];
    int sa = 0;
    while ((sa + 1) * (sa + 2) / 2 <= int(blockIdx.x)) ++sa;
    const int sb = int(blockIdx.x) - sa * (sa + 1) / 2;
    const int c = blockIdx.y;
    const int64_t i0 = int64_t(c) * chunk, i1 = std::min<int64_t>(N, i0 + chunk);
    const int t = threadIdx.x, w = t / 64, l = t % 64, lm = l % 16, lg = l / 16;
    d4 acc[2][8];
#pragma unroll
    for (int tr = 0; tr < 2; ++tr)
#pragma unroll
        for (int tc = 0; tc < 8; ++tc) acc[tr][tc] = d4{0.0, 0.0, 0.0, 0.0};
    // the next panel is loaded into registers while the current one is multiplied
    constexpr int PE = kST * kSP / 256;  // panel elements per thread and operand
    double ra[PE], rb[PE], rw = 0.0;
    auto load_panel = [&](int64_t ib0) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < PE; ++q) {
            const int e = t + 256 * q, col = e / kSP, r = e % kSP;
            const int64_t i = ib0 + r;
            const int ga = sa * kST + col, gb = sb * kST + col;
            ra[q] = (ga < k && i < i1) ? double(Z[int64_t(ga) * N + i]) : 0.0;
            rb[q] = (gb < k && i < i1) ? double(Z[int64_t(gb) * N + i]) : 0.0;
        }
        if (t < kSP) {
            const int64_t i = ib0 + t;
            rw = (i < i1) ? (theta ? 1.0 / theta[i] : 1.0) : 0.0;
        }
    };
    // 16 x 16 result blocks: row block rb0 + tr of this wave, column block
    // cb0 + tc. Blocks past k and blocks wholly above the diagonal are never
    // read by the fold, so the wave skips them (the tests are wave-uniform).
    const int nb = (k + 15) / 16;
    const int rb0 = sa * (kST / 16) + 2 * w, cb0 = sb * (kST / 16);
    auto live = [&](int tr, int tc) __attribute__((always_inline)) {
        return rb0 + tr < nb && cb0 + tc < nb && cb0 + tc <= rb0 + tr;
    };
    if (i0 < i1) load_panel(i0);
    for (int64_t ib0 = i0; ib0 < i1; ib0 += kSP) {
#pragma unroll
        for (int q = 0; q < PE; ++q) {
            const int e = t + 256 * q;
            pa[e / kSP][e % kSP] = ra[q];
            pb[e / kSP][e % kSP] = rb[q];
        }
        if (t < kSP) wt[t] = rw;
        __syncthreads();
        if (ib0 + kSP < i1) load_panel(ib0 + kSP);
        if (live(1, 0) || live(0, 0)) {
#pragma unroll
            for (int s4 = 0; s4 < kSP / 4; ++s4) {
                const int r = 4 * s4 + lg;
                double av[2];
#pragma unroll
                for (int tr = 0; tr < 2; ++tr) av[tr] = pa[(2 * w + tr) * 16 + lm][r] * wt[r];
#pragma unroll
                for (int tc = 0; tc < 8; ++tc) {
                    if (!live(1, tc) && !live(0, tc)) continue;
                    const double bv = pb[tc * 16 + lm][r];
#pragma unroll
                    for (int tr = 0; tr < 2; ++tr)
                        if (live(tr, tc))
                            acc[tr][tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[tr], bv, acc[tr][tc], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int tr = 0; tr < 2; ++tr)
#pragma unroll
        for (int tc = 0; tc < 8; ++tc) {
            if (!live(tr, tc)) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ia = sa * kST + (2 * w + tr) * 16 + lg + 4 * e, ib = sb * kST + tc * 16 + lm;
                if (ia < k && ib < k) part[(int64_t(c) * k + ia) * k + ib] = acc[tr][tc][e];
            }
        }
}

// The same partial sums for k <= 256, balanced over the wavefronts: one block
// per row chunk computes every lower 16 x 16 result block over its rows, the
// blocks dealt to its kSyW wavefronts in turn (block q, counted down the block
// columns, to wavefront q % kSyW, slot q / kSyW), so that every wavefront issues
// nearly the same number of matrix-core products. Panels of P rows of Z (all k
// columns) and their weights 1 / theta are staged in LDS, double-buffered; the
// next panel's loads are in flight while the current one is multiplied. P = 32
// for k <= 208 (half the barriers of 16-row panels: 560 -> 503 us at N = 5e5,
// k = 200), 16 above, where 32 rows would spill registers.
constexpr int kSyW = 8;
constexpr int kSyKP = 256 + 1;  // panel row stride in LDS
constexpr int kSyChunk = 32;    // row chunks are whole panels of either height
template <int NS, int P>
__global__ __launch_bounds__(64 * kSyW) void k_syrk_tri(const double* __restrict__ Z, int64_t N, int k,
                                                         const double* __restrict__ theta, int64_t chunk,
                                                         double* __restrict__ part) {
    typedef double d4 __attribute__((ext_vector_type(4)));
    __shared__ double pz[2][P][kSyKP], wt[2][P];
    __shared__ int blk[kSyW * NS];  // block q: I | J << 8 (-1: none)
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int nb = (k + 15) >> 4, nq = nb * (nb + 1) / 2;
    if (t < kSyW * NS) {
        int q = t, J = 0, v = -1;
        if (q < nq) {
            while (q >= nb - J) {
                q -= nb - J;
                ++J;
            }
            v = (J + q) | (J << 8);
        }
        blk[t] = v;
    }
    const int c = blockIdx.x;
    const int64_t i0 = int64_t(c) * chunk, i1 = std::min<int64_t>(N, i0 + chunk);
    constexpr int PE = P * 256 / (64 * kSyW);  // panel elements per thread
    double ra[PE], rw = 0.0;
    auto load_panel = [&](int64_t ib0) __attribute__((always_inline)) {
#pragma unroll
        for (int m = 0; m < PE; ++m) {
            const int e = t + 64 * kSyW * m, col = e / P, r = e % P;
            const int64_t i = ib0 + r;
            ra[m] = (col < k && i < i1) ? Z[int64_t(col) * N + i] : 0.0;
        }
        if (t < P) {
            const int64_t i = ib0 + t;
            rw = (i < i1) ? (theta ? 1.0 / theta[i] : 1.0) : 0.0;
        }
    };
    d4 acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] = d4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();  // the block table
    int cI[NS], cJ[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int v = __builtin_amdgcn_readfirstlane(blk[s * kSyW + w]);
        cI[s] = v < 0 ? -1 : (v & 255);
        cJ[s] = v < 0 ? -1 : (v >> 8);
    }
    if (i0 < i1) load_panel(i0);
    int buf = 0;
    for (int64_t ib0 = i0; ib0 < i1; ib0 += P, buf ^= 1) {
#pragma unroll
        for (int m = 0; m < PE; ++m) {
            const int e = t + 64 * kSyW * m;
            pz[buf][e % P][e / P] = ra[m];
        }
        if (t < P) wt[buf][t] = rw;
        __syncthreads();
        if (ib0 + P < i1) load_panel(ib0 + P);
#pragma unroll
        for (int s4 = 0; s4 < P / 4; ++s4) {
            const int r = 4 * s4 + (l >> 4);
            const double wr = wt[buf][r];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (cI[s] >= 0) {
                    const double a = pz[buf][r][16 * cI[s] + (l & 15)] * wr;
                    const double b = pz[buf][r][16 * cJ[s] + (l & 15)];
                    acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
                }
            }
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (cI[s] < 0) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ia = 16 * cI[s] + (l >> 4) + 4 * e, ib = 16 * cJ[s] + (l & 15);
            if (ia < k && ib < k) part[(int64_t(c) * k + ia) * k + ib] = acc[s][e];
        }
    }
}

// M[a][b] = M[b][a] = diag [a == b] + sum_c part[c][a][b] for a >= b (chunks in
// order); threads run along rows of the lower triangle, so the partial sums are
// read contiguously
__global__ void k_syrk_fold(const double* __restrict__ part, int nchunk, int k, double diag,
                            double* __restrict__ M) {
    const int64_t e = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (e >= int64_t(k) * k) return;
    const int a = int(e / k), b = int(e % k);
    if (b > a) return;
    double s = (a == b) ? diag : 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[int64_t(c) * k * k + e];
    M[e] = s;
    M[int64_t(b) * k + a] = s;
}

// Two-level form of k_syrk_fold for the capacitance matrix: group g of
// gridDim.y adds its run of consecutive chunks (in chunk order) for every
// lower-triangle entry, then k_syrk_fold_fin adds the group sums in group order.
// Spreading the long sums over groups gives their loads gridDim.y times more
// blocks than one thread per entry does.
constexpr int kFoldGroups = 16;
__global__ void k_syrk_fold_grp(const double* __restrict__ part, int nchunk, int k, double* __restrict__ gsum,
                                int full = 0) {
    const int64_t kk = int64_t(k) * k;
    const int64_t e = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (e >= kk || (!full && e % k > e / k)) return;
    const int g = blockIdx.y, ng = gridDim.y;
    const int c0 = int(int64_t(nchunk) * g / ng), c1 = int(int64_t(nchunk) * (g + 1) / ng);
    double s = 0.0;
#pragma unroll 8
    for (int c = c0; c < c1; ++c) s += part[c * kk + e];
    gsum[g * kk + e] = s;
}

// full != 0: every entry of a general k x k sum (no mirroring)
__global__ void k_syrk_fold_fin(const double* __restrict__ gsum, int ng, int k, double diag,
                                double* __restrict__ M, int ldm, int full = 0) {
    const int64_t kk = int64_t(k) * k;
    const int64_t e = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (e >= kk) return;
    const int a = int(e / k), b = int(e % k);
    if (!full && b > a) return;
    double s = (a == b) ? diag : 0.0;
    for (int g = 0; g < ng; ++g) s += gsum[g * kk + e];
    M[int64_t(a) * ldm + b] = s;
    if (!full) M[int64_t(b) * ldm + a] = s;
}

// row chunks of k_syrk_mfma: enough blocks to fill the GPU, partials within 256 MB,
// at least 256 rows per chunk (the fold reads nchunk k x k partials), chunks a
// whole number of panels
void syrk_chunks(int64_t N, int k, int& nchunk, int64_t& chunk) {
    const int ns = (k + kST - 1) / kST, pairs = ns * (ns + 1) / 2;
    int64_t want = std::max<int64_t>(1, (1024 + pairs - 1) / pairs);
    want = std::min<int64_t>(want, std::max<int64_t>(1, (int64_t(256) << 20) / (int64_t(k) * k * 8)));
    want = std::min<int64_t>(want, std::max<int64_t>(1, N / 256));
    chunk = (N + want - 1) / want;
    chunk = (chunk + kSP - 1) / kSP * kSP;
    nchunk = int((N + chunk - 1) / chunk);
}

// row chunks of k_syrk_tri (k <= 256): one block per compute unit, at least
// 256 rows per chunk, partials within 256 MB, chunks a whole number of panels
void syrk_tri_chunks(int64_t N, int k, int& nchunk, int64_t& chunk) {
    int64_t want = 256;
    want = std::min<int64_t>(want, std::max<int64_t>(1, (int64_t(256) << 20) / (int64_t(k) * k * 8)));
    want = std::min<int64_t>(want, std::max<int64_t>(1, N / 256));
    chunk = (N + want - 1) / want;
    chunk = (chunk + kSyChunk - 1) / kSyChunk * kSyChunk;
    nchunk = int((N + chunk - 1) / chunk);
}

// A^T B for two N x k column-major matrices (k <= 208), partial sums per row
// chunk: two blocks of 16 wavefronts per chunk (blockIdx.y) share the nb x nb
// 16 x 16 blocks of the product, dealt evenly over their wavefronts (block
// q = I nb + J to split q % 2, wavefront (q / 2) % 16, slot q / 32), from 16-row
// panels of both matrices in LDS. The Nystrom method's Q^T (K Q).
constexpr int kGrW = 16, kGrSplit = 2, kGrSlots = 6;  // 169 blocks at k = 208
__global__ __launch_bounds__(64 * kGrW) void k_gram_mfma(const double* __restrict__ A, const double* __restrict__ B,
                                                         int64_t N, int k, int64_t chunk, double* __restrict__ part) {
    typedef double d4 __attribute__((ext_vector_type(4)));
    __shared__ double pa[kSP][kSyKP], pb[kSP][kSyKP];
    __shared__ int blk[kGrW * kGrSlots];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int nb = (k + 15) >> 4, nq = nb * nb;
    if (t < kGrW * kGrSlots) {
        const int q = t * kGrSplit + int(blockIdx.y);
        blk[t] = q < nq ? (q / nb) | ((q % nb) << 8) : -1;
    }
    const int c = blockIdx.x;
    const int64_t i0 = int64_t(c) * chunk, i1 = std::min<int64_t>(N, i0 + chunk);
    constexpr int PE = kSP * 256 / (64 * kGrW);  // panel elements per thread and matrix
    double ra[PE], rb[PE];
    auto load_panel = [&](int64_t ib0) __attribute__((always_inline)) {
#pragma unroll
        for (int m = 0; m < PE; ++m) {
            const int e = t + 64 * kGrW * m, col = e / kSP, r = e % kSP;
            const int64_t i = ib0 + r;
            const bool ok = col < k && i < i1;
            ra[m] = ok ? A[int64_t(col) * N + i] : 0.0;
            rb[m] = ok ? B[int64_t(col) * N + i] : 0.0;
        }
    };
    d4 acc[kGrSlots];
#pragma unroll
    for (int s = 0; s < kGrSlots; ++s) acc[s] = d4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();  // the block table
    int cI[kGrSlots], cJ[kGrSlots];
#pragma unroll
    for (int s = 0; s < kGrSlots; ++s) {
        const int v = __builtin_amdgcn_readfirstlane(blk[s * kGrW + w]);
        cI[s] = v < 0 ? -1 : (v & 255);
        cJ[s] = v < 0 ? -1 : (v >> 8);
    }
    if (i0 < i1) load_panel(i0);
    for (int64_t ib0 = i0; ib0 < i1; ib0 += kSP) {
#pragma unroll
        for (int m = 0; m < PE; ++m) {
            const int e = t + 64 * kGrW * m;
            pa[e % kSP][e / kSP] = ra[m];
            pb[e % kSP][e / kSP] = rb[m];
        }
        __syncthreads();
        if (ib0 + kSP < i1) load_panel(ib0 + kSP);
#pragma unroll
        for (int s4 = 0; s4 < kSP / 4; ++s4) {
            const int r = 4 * s4 + (l >> 4);
#pragma unroll
            for (int s = 0; s < kGrSlots; ++s) {
                if (cI[s] >= 0) {
                    const double a = pa[r][16 * cI[s] + (l & 15)];
                    const double b = pb[r][16 * cJ[s] + (l & 15)];
                    acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
                }
            }
        }
        __syncthreads();  // before the panels are overwritten
    }
#pragma unroll
    for (int s = 0; s < kGrSlots; ++s) {
        if (cI[s] < 0) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ia = 16 * cI[s] + (l >> 4) + 4 * e, ib = 16 * cJ[s] + (l & 15);
            if (ia < k && ib < k) part[(int64_t(c) * k + ia) * k + ib] = acc[s][e];
        }
    }
}

// out = Y T for Y: N x k column-major, T: k x kc row-major, out: N x kc
// column-major (kc <= 208): a block of 16 wavefronts takes 256 rows, each
// wavefront 16 rows and all column blocks, on the matrix cores; 16-row pieces of
// T are staged in LDS in turn while Y streams through once.
constexpr int kGmW = 16, kGmCB = 13;  // column blocks of 16: kc <= 208
constexpr int kGmTP = 16 * kGmCB + 4;  // staged row stride of T
__global__ __launch_bounds__(64 * kGmW) void k_gemm_nk_mfma(const double* __restrict__ Y, int64_t N, int k,
                                                            const double* __restrict__ T, int kc,
                                                            double* __restrict__ out) {
    typedef double d4 __attribute__((ext_vector_type(4)));
    __shared__ double tp[16][kGmTP];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int64_t row0 = int64_t(blockIdx.x) * (16 * kGmW) + 16 * w;
    const int64_t ri = row0 + (l & 15);
    d4 acc[kGmCB];
#pragma unroll
    for (int cb = 0; cb < kGmCB; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
    for (int m0 = 0; m0 < k; m0 += 16) {
        for (int e = t; e < 16 * 16 * kGmCB; e += 64 * kGmW) {
            const int mr = e / (16 * kGmCB), j = e % (16 * kGmCB);
            tp[mr][j] = (m0 + mr < k && j < kc) ? T[int64_t(m0 + mr) * kc + j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int mr = 4 * s4 + (l >> 4), m = m0 + mr;
            const double a = (m < k && ri < N) ? Y[int64_t(m) * N + ri] : 0.0;
#pragma unroll
            for (int cb = 0; cb < kGmCB; ++cb) {
                if (16 * cb < kc) {
                    const double b = tp[mr][16 * cb + (l & 15)];
                    acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
                }
            }
        }
        __syncthreads();  // before the next piece of T is staged
    }
#pragma unroll
    for (int cb = 0; cb < kGmCB; ++cb) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t row = row0 + (l >> 4) + 4 * e;
            const int col = 16 * cb + (l & 15);
            if (row < N && col < kc) out[int64_t(col) * N + row] = acc[cb][e];
        }
    }
}

// w_part[s][j] = sum over rows of segment s of Z[j N + i] u[i]: one block per
// (group of kGemvCols columns, segment s), so that the product of long columns
// keeps the GPU busy and each value of u read serves kGemvCols columns
constexpr int kGemvCols = 4;
template <class ZT>
__global__ __launch_bounds__(kT) void k_gemv_t_seg(const ZT* __restrict__ Z, int64_t N, int k,
                                                   const double* __restrict__ u, int64_t seg,
                                                   double* __restrict__ wpart) {
    const int j0 = blockIdx.x * kGemvCols, sgi = blockIdx.y;
    const int nc = min(kGemvCols, k - j0);
    const int64_t r0 = int64_t(sgi) * seg, r1 = std::min<int64_t>(N, r0 + seg);
    double a0[kGemvCols], a1[kGemvCols];
#pragma unroll
    for (int c = 0; c < kGemvCols; ++c) a0[c] = a1[c] = 0.0;
    int64_t i = r0 + threadIdx.x;
    for (; i + kT < r1; i += 2 * kT) {
        const double u0 = u[i], u1 = u[i + kT];
#pragma unroll
        for (int c = 0; c < kGemvCols; ++c) {
            if (c < nc) {
                const ZT* zc = Z + int64_t(j0 + c) * N;
                a0[c] += double(zc[i]) * u0;
                a1[c] += double(zc[i + kT]) * u1;
            }
        }
    }
    if (i < r1) {
        const double u0 = u[i];
#pragma unroll
        for (int c = 0; c < kGemvCols; ++c)
            if (c < nc) a0[c] += double(Z[int64_t(j0 + c) * N + i]) * u0;
    }
    __shared__ double sh[kGemvCols][kT];
#pragma unroll
    for (int c = 0; c < kGemvCols; ++c) sh[c][threadIdx.x] = a0[c] + a1[c];
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int c = 0; c < kGemvCols; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < nc) wpart[int64_t(sgi) * k + j0 + threadIdx.x] = sh[threadIdx.x][0];
}

// The same for the FP32 factor copy with N and the segment length multiples of
// 4: a thread takes 4 consecutive rows at a time, so every factor load moves 16
// bytes per lane (the one-row form moves 4 and reaches less of the HBM rate)
__global__ __launch_bounds__(kT) void k_gemv_t_seg4(const float* __restrict__ Z, int64_t N, int k,
                                                    const double* __restrict__ u, int64_t seg,
                                                    double* __restrict__ wpart) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    typedef double d2v __attribute__((ext_vector_type(2)));
    const int j0 = blockIdx.x * kGemvCols, sgi = blockIdx.y;
    const int nc = min(kGemvCols, k - j0);
    const int64_t r0 = int64_t(sgi) * seg, r1 = std::min<int64_t>(N, r0 + seg);
    double a0[kGemvCols], a1[kGemvCols];
#pragma unroll
    for (int c = 0; c < kGemvCols; ++c) a0[c] = a1[c] = 0.0;
    auto step = [&](int64_t i, double (&a)[kGemvCols]) __attribute__((always_inline)) {
        const d2v ua = *reinterpret_cast<const d2v*>(u + i), ub = *reinterpret_cast<const d2v*>(u + i + 2);
#pragma unroll
        for (int c = 0; c < kGemvCols; ++c) {
            if (c < nc) {
                const f4v z = *reinterpret_cast<const f4v*>(Z + int64_t(j0 + c) * N + i);
                a[c] += double(z[0]) * ua[0];
                a[c] += double(z[1]) * ua[1];
                a[c] += double(z[2]) * ub[0];
                a[c] += double(z[3]) * ub[1];
            }
        }
    };
    int64_t i = r0 + 4 * threadIdx.x;
    for (; i + 4 * kT < r1; i += 8 * kT) {
        step(i, a0);
        step(i + 4 * kT, a1);
    }
    if (i < r1) step(i, a0);
    __shared__ double sh[kGemvCols][kT];
#pragma unroll
    for (int c = 0; c < kGemvCols; ++c) sh[c][threadIdx.x] = a0[c] + a1[c];
    __syncthreads();
    for (int s2 = kT / 2; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) {
#pragma unroll
            for (int c = 0; c < kGemvCols; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + s2];
        }
        __syncthreads();
    }
    if (threadIdx.x < nc) wpart[int64_t(sgi) * k + j0 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_gram_fold(const double* __restrict__ part, int nchunk, int k, double diag,
                            double* __restrict__ M) {
    int64_t e = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (e >= int64_t(k) * k) return;
    double s = (e / k == e % k) ? diag : 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[int64_t(c) * k * k + e];
    M[e] = s;
}

// In-place Cholesky of the k x k SPD matrix M (row-major, lower triangle used),
// one block, right-looking in panels of kCB columns: the first wavefront factors
// the diagonal block in registers (lane r holds row r, shuffles broadcast the
// pivots), all threads solve the panel below it (one row each), then the
// trailing lower triangle is updated in kTT x kTT tiles whose two panel slices
// are staged in LDS. status[0] = 0 ok, 1 = non-positive pivot.
// Launched with kCholT threads (8 x 4 trailing elements per thread).
constexpr int kCB = 16, kTT = 128, kCholT = 512;
// rows i >= j0 + nb of the panel: x L_D^T = m, with L_D in D (reciprocal
// pivots on its diagonal); kept out of line so that its registers are not
// allocated together with the diagonal factorisation's
__device__ __attribute__((noinline)) void chol_panel(double* __restrict__ M, int k, int j0, int nb,
                                                     const double (*D)[kCB + 1]) {
    for (int i = j0 + nb + int(threadIdx.x); i < k; i += kCholT) {
        double x[kCB];
        double* mi = M + int64_t(i) * k + j0;
#pragma unroll
        for (int c = 0; c < kCB; ++c) x[c] = c < nb ? mi[c] : 0.0;  // all loads before any store
#pragma unroll
        for (int c = 0; c < kCB; ++c) {
            if (c < nb) {
                double v = x[c];
#pragma unroll
                for (int q = 0; q < c; ++q) v -= x[q] * D[c][q];
                x[c] = v * D[c][c];
            }
        }
#pragma unroll
        for (int c = 0; c < kCB; ++c)
            if (c < nb) mi[c] = x[c];
    }
}

__global__ __launch_bounds__(kCholT) void k_chol(double* __restrict__ M, int k, int* __restrict__ status) {
    __shared__ double D[kCB][kCB + 1];  // diagonal block, reciprocals on its diagonal
    __shared__ double Pa[kTT][kCB + 1], Pb[kTT][kCB + 1];
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    for (int j0 = 0; j0 < k; j0 += kCB) {
        const int nb = min(kCB, k - j0);
        __syncthreads();  // the previous trailing update is complete
        if (t < 64) {
            double d[kCB];
#pragma unroll
            for (int c = 0; c < kCB; ++c) d[c] = (t < nb && c <= t) ? M[int64_t(j0 + t) * k + j0 + c] : 0.0;
#pragma unroll
            for (int c = 0; c < kCB; ++c) {
                if (c < nb) {
                    double dcc = __shfl(d[c], c, 64);
                    if (!(dcc > 0.0)) {
                        if (t == 0) bad = 1;
                        dcc = 1e-300;
                    }
                    dcc = sqrt(dcc);
                    const double rdc = 1.0 / dcc;
                    if (t == c) d[c] = dcc;
                    else if (t > c) d[c] *= rdc;
#pragma unroll
                    for (int cc = c + 1; cc < kCB; ++cc) {
                        const double lcc = __shfl(d[c], cc, 64);  // L[cc][c], from lane cc
                        if (cc <= t && t < nb) d[cc] -= d[c] * lcc;
                    }
                }
            }
            if (t < nb) {
#pragma unroll
                for (int c = 0; c < kCB; ++c)
                    if (c <= t) {
                        M[int64_t(j0 + t) * k + j0 + c] = d[c];
                        D[t][c] = c == t ? 1.0 / d[c] : d[c];  // reciprocal on the diagonal
                    }
            }
        }
        __syncthreads();
        chol_panel(M, k, j0, nb, D);
        __syncthreads();
        // trailing lower triangle, tile (R, Cc) with Cc <= R
        const int j1 = j0 + nb, m = k - j1, nt = (m + kTT - 1) / kTT;
        const int ty = t / 32, tx = t % 32;
        for (int R = 0; R < nt; ++R)
            for (int Cc = 0; Cc <= R; ++Cc) {
                for (int e = t; e < kTT * kCB; e += kCholT) {
                    const int r = e / kCB, q = e % kCB;
                    const int ia = j1 + R * kTT + r, ib = j1 + Cc * kTT + r;
                    Pa[r][q] = (ia < k && q < nb) ? M[int64_t(ia) * k + j0 + q] : 0.0;
                    Pb[r][q] = (ib < k && q < nb) ? M[int64_t(ib) * k + j0 + q] : 0.0;
                }
                __syncthreads();
                double acc[8][4];
#pragma unroll
                for (int a = 0; a < 8; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 4
                for (int q = 0; q < kCB; ++q) {
                    double pa[8], pb[4];
#pragma unroll
                    for (int a = 0; a < 8; ++a) pa[a] = Pa[ty + 16 * a][q];
#pragma unroll
                    for (int b = 0; b < 4; ++b) pb[b] = Pb[tx + 32 * b][q];
#pragma unroll
                    for (int a = 0; a < 8; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b) acc[a][b] += pa[a] * pb[b];
                }
#pragma unroll
                for (int a = 0; a < 8; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int r = R * kTT + ty + 16 * a, c = Cc * kTT + tx + 32 * b;
                        if (r < m && c <= r) M[int64_t(j1 + r) * k + j1 + c] -= acc[a][b];
                    }
                __syncthreads();  // before the panel slices are staged again
            }
    }
    __syncthreads();
    if (t == 0) status[0] = bad;
}

// t = (L L^T)^{-1} w with L the Cholesky factor in the lower triangle of M and
// w the sum of the nseg partial vectors wpart[g][:] (segments in order); one
// block, panels of kCB. The first wavefront solves each diagonal block in
// registers (forward: lane j holds row j of the block; backward: lane j holds
// column j), all threads then update the remaining entries.
__global__ void k_chol_solve(const double* __restrict__ Lm, int k, const double* __restrict__ wpart, int nseg,
                             double* __restrict__ t) {
    extern __shared__ double sx[];
    const int tid = threadIdx.x;
    for (int i = tid; i < k; i += blockDim.x) {
        double v = 0.0;
#pragma unroll 8
        for (int g = 0; g < nseg; ++g) v += wpart[int64_t(g) * k + i];
        sx[i] = v;
    }
    __syncthreads();
    for (int j0 = 0; j0 < k; j0 += kCB) {  // forward: L z = w
        const int nb = min(kCB, k - j0);
        if (tid < 64) {
            double d[kCB];
#pragma unroll
            for (int c = 0; c < kCB; ++c) d[c] = (tid < nb && c <= tid) ? Lm[int64_t(j0 + tid) * k + j0 + c] : 0.0;
            double b = tid < nb ? sx[j0 + tid] : 0.0;
#pragma unroll
            for (int c = 0; c < kCB; ++c) {
                if (c < nb) {
                    const double xc = __shfl(b, c, 64) / __shfl(d[c], c, 64);
                    if (tid == c) b = xc;
                    else if (tid > c) b -= d[c] * xc;
                }
            }
            if (tid < nb) sx[j0 + tid] = b;
        }
        __syncthreads();
        for (int i = j0 + nb + tid; i < k; i += blockDim.x) {
            const double* lr = Lm + int64_t(i) * k + j0;
            double v = 0.0;
            for (int q = 0; q < nb; ++q) v += lr[q] * sx[j0 + q];
            sx[i] -= v;
        }
        __syncthreads();
    }
    for (int j1 = k; j1 > 0; j1 -= kCB) {  // backward: L^T t = z
        const int j0 = max(0, j1 - kCB), nb = j1 - j0;
        if (tid < 64) {
            double d[kCB];  // column tid of the block: d[q] = L[j0 + q][j0 + tid]
#pragma unroll
            for (int q = 0; q < kCB; ++q) d[q] = (tid < nb && q < nb && q >= tid) ? Lm[int64_t(j0 + q) * k + j0 + tid] : 0.0;
            double b = tid < nb ? sx[j0 + tid] : 0.0;
#pragma unroll
            for (int c = kCB - 1; c >= 0; --c) {
                if (c < nb) {
                    const double xc = __shfl(b, c, 64) / __shfl(d[c], c, 64);
                    if (tid == c) b = xc;
                    else if (tid < c) b -= d[c] * xc;
                }
            }
            if (tid < nb) sx[j0 + tid] = b;
        }
        __syncthreads();
        for (int i = tid; i < j0; i += blockDim.x) {
            double v = 0.0;
            for (int q = 0; q < nb; ++q) v += Lm[int64_t(j0 + q) * k + i] * sx[j0 + q];
            sx[i] -= v;
        }
        __syncthreads();
    }
    for (int i = tid; i < k; i += blockDim.x) t[i] = sx[i];
}

// value of x in lane `lane` (a wave-uniform index), in every lane
__device__ __forceinline__ double lane_bcast(double x, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// Capacitance factor and solves for k <= kRegCholK. k_chol_reg leaves L in
// the lower triangle of M and L^T in its strict upper triangle (M[i][j] =
// L[max(i, j)][min(i, j)]), so that k_chol_solve_b reads only rows of M.
constexpr int kRegCholK = 256;
constexpr int kRegWaves = 8;   // slots per wavefront: 12 up to k = 208 (91 blocks), 17 up to k = 256 (136)

// 1 / sqrt(x) for x > 0 to about one unit in the last place: the hardware
// estimate refined by two Newton steps y <- y (3/2 - x y^2 / 2)
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y *= fma(-h * y, y, 1.5);
    y *= fma(-h * y, y, 1.5);
    return y;
}

// Barrier for LDS hand-offs between the wavefronts of a block: waits for the
// wave's LDS accesses only, so that global loads and stores issued earlier stay
// in flight across it (a __syncthreads would wait for them as well).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" : : : "memory"); }

// In-place Cholesky, one block of kRegWaves wavefronts, blocked by 16 x 16. The
// nb (nb + 1) / 2 lower blocks stay in registers in the FP64 matrix-core result
// layout (lane l, element e: row l / 16 + 4 e, column l % 16); block q, counted
// down the block columns, belongs to wavefront q % kRegWaves, slot q / kRegWaves. The matrix
// is padded to whole blocks with the identity. For block column p: (a) its
// owners copy it to LDS; (b) wavefront 0 factors the diagonal block (lane r
// holds row r, lane reads broadcast the pivots and the finished column's
// entries); (c) one thread per row below it
// solves x L_pp^T = m; (d) the finished column goes to global memory in both
// triangles, and every wavefront subtracts P_I P_J^T from its blocks (I, J),
// J > p, on the matrix cores. The LDS copy is double-buffered: the barriers of
// (a)-(c) of column p + 1 separate (d) of column p - 1 from the reuse of its
// buffer. The barriers wait for LDS traffic only (no wavefront reads what another
// writes to global memory), so (d)'s stores drain while the next column is
// factored. status[0] = 0 ok, 1 = non-positive pivot.
template <int NS>
__global__ __launch_bounds__(64 * kRegWaves) void k_chol_reg(double* __restrict__ M, int k, int ldm,
                                                              int* __restrict__ status) {
    typedef double d4 __attribute__((ext_vector_type(4)));
    __shared__ double pan[2][16][16][17];  // [buffer][block row][row][column]
    __shared__ double rdiag[16];
    __shared__ int blk[kRegWaves * NS];    // block q: I | J << 8 (-1: none)
    __shared__ int bad;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int nb = (k + 15) >> 4, nq = nb * (nb + 1) / 2;
    if (t == 0) bad = 0;
    if (t < kRegWaves * NS) {
        int q = t, J = 0, v = -1;
        if (q < nq) {
            while (q >= nb - J) {
                q -= nb - J;
                ++J;
            }
            v = (J + q) | (J << 8);
        }
        blk[t] = v;
    }
    __syncthreads();
    // block coordinates of slot s of this wavefront (wave-uniform)
    auto coords = [&](int s, int& I, int& J) __attribute__((always_inline)) {
        const int v = __builtin_amdgcn_readfirstlane(blk[s * kRegWaves + w]);
        I = v < 0 ? -1 : (v & 255);
        J = v < 0 ? -1 : (v >> 8);
    };
    d4 acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        int I, J;
        coords(s, I, J);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            double v = 0.0;
            if (I >= 0) {
                const int row = 16 * I + (l >> 4) + 4 * e, col = 16 * J + (l & 15);
                v = (row < k && col < k) ? M[int64_t(row) * ldm + col] : (row == col ? 1.0 : 0.0);
            }
            acc[s][e] = v;
        }
    }
    for (int p = 0; p < nb; ++p) {
        double (*P)[16][17] = pan[p & 1];
        // (a)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            int I, J;
            coords(s, I, J);
            if (J == p)
#pragma unroll
                for (int e = 0; e < 4; ++e) P[I][(l >> 4) + 4 * e][l & 15] = acc[s][e];
        }
        lds_barrier();
        // (b)
        if (w == 0) {
            double d[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) d[c] = (l < 16 && c <= l) ? P[p][l][c] : 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                double dcc = lane_bcast(d[c], c);
                if (!(dcc > 0.0)) {
                    if (l == 0) bad = 1;
                    dcc = 1e-300;
                }
                // 1 / sqrt(pivot) from the hardware estimate and two Newton steps
                // (each doubles the correct bits), the square root as pivot times it:
                // a short dependent chain, where sqrt and a division take two long ones
                const double rdc = rsqrt_nr(dcc);
                if (l == c) d[c] = dcc * rdc;
                else if (l > c) d[c] *= rdc;
#pragma unroll
                for (int cc = c + 1; cc < 16; ++cc) {
                    const double lcc = lane_bcast(d[c], cc);  // L[cc][c], from lane cc
                    if (cc <= l && l < 16) d[cc] -= d[c] * lcc;
                }
            }
            if (l < 16) {
#pragma unroll
                for (int c = 0; c < 16; ++c) P[p][l][c] = c <= l ? d[c] : 0.0;
                rdiag[l] = 1.0 / d[l];
            }
        }
        lds_barrier();
        // (c)
        if (t < (nb - 1 - p) * 16) {
            const int I = p + 1 + (t >> 4), r = t & 15;
            double x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) x[c] = P[I][r][c];
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                double v = x[c];
#pragma unroll
                for (int q = 0; q < c; ++q) v -= x[q] * P[p][c][q];
                x[c] = v * rdiag[c];
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) P[I][r][c] = x[c];
        }
        lds_barrier();
        // (d) the finished column, then the trailing update
        for (int idx = t; idx < (nb - p) * 256; idx += 64 * kRegWaves) {
            const int I = p + (idx >> 8), r = (idx >> 4) & 15, c = idx & 15;
            const int row = 16 * I + r, col = 16 * p + c;
            if (row < k && col < k && (I > p || c <= r)) {
                const double v = P[I][r][c];
                M[int64_t(row) * ldm + col] = v;
                M[int64_t(col) * ldm + row] = v;
            }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            int I, J;
            coords(s, I, J);
            if (J > p) {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4) {
                    const double a = -P[I][l & 15][4 * s4 + (l >> 4)];
                    const double b = P[J][l & 15][4 * s4 + (l >> 4)];
                    acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[s], 0, 0, 0);
                }
            }
        }
    }
    lds_barrier();
    if (t == 0) status[0] = bad;
}


// Inverses of the 16 x 16 diagonal blocks of the capacitance factor L (as
// k_chol_reg leaves it), block J row-major at Dinv + 256 J and transposed at
// Dinv + 256 (nb + J) (nb blocks); rows and columns past k belong to an
// identity block. One wavefront per block: lane c < 16 solves L_JJ x = e_c by
// forward substitution (entries above the diagonal come out as exact zeros).
__global__ __launch_bounds__(64) void k_diag_inv(const double* __restrict__ Lm, int k, int ldm,
                                                 double* __restrict__ Dinv) {
    __shared__ double lb[16][17];
    const int J = int(blockIdx.x), c0 = 16 * J, l = int(threadIdx.x);
    for (int e = l; e < 256; e += 64) {
        const int r = e / 16, i = e % 16;
        lb[r][i] = (c0 + r < k && c0 + i < k) ? Lm[int64_t(c0 + r) * ldm + c0 + i] : (r == i ? 1.0 : 0.0);
    }
    __syncthreads();
    if (l < 16) {
        double x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double v = r == l ? 1.0 : 0.0;
#pragma unroll
            for (int i = 0; i < r; ++i) v -= lb[r][i] * x[i];
            x[r] = v / lb[r][r];
        }
        const int nb = int(gridDim.x);
#pragma unroll
        for (int r = 0; r < 16; ++r) Dinv[256 * J + 16 * r + l] = x[r];
#pragma unroll
        for (int r = 0; r < 16; ++r) Dinv[256 * (nb + J) + 16 * l + r] = x[r];
    }
}

// t = (L L^T)^{-1} w for k <= kRegCholK with the factor as k_chol_reg leaves
// it (L on and below the diagonal of M, L^T above it, row stride ldm, a
// multiple of 16) and the inverses of its diagonal blocks from k_diag_inv; w
// the sum of the nseg partial vectors wpart[g][:] (segments in order). Both
// sweeps go over panels of 16 rows: 16 lanes multiply the panel's part of the
// right-hand side by the inverse of the diagonal block (forward) or by its
// transpose (backward), so no step waits on another; then every thread
// subtracts its own row's product with the panel's 16 solved entries (forward:
// the rows after the panel, reading L left of the diagonal; backward: the rows
// before it, reading row j right of the diagonal, which holds L^T's row j). A
// panel's entries are loaded while the panel before it is solved.
constexpr int kSbT = 256;  // threads; k <= kRegCholK <= kSbT rows, one per thread
static_assert(kRegCholK <= kSbT, "one thread per row of the capacitance matrix");

__global__ __launch_bounds__(kSbT) void k_chol_solve_b(const double* __restrict__ Lm, int k, int ldm,
                                                      const double* __restrict__ Dinv,
                                                      const double* __restrict__ wpart, int nseg,
                                                      double* __restrict__ t) {
    __shared__ double bv[kSbT];  // right-hand side, then the solution
    __shared__ double xs[16];    // a panel's solved entries
    const int tid = int(threadIdx.x);
    const int nb = (k + 15) / 16;
    // panel s of the two sweeps (s < nb forward, then nb .. 2 nb - 1 backward)
    auto panel_col = [&](int s) __attribute__((always_inline)) { return 16 * (s < nb ? s : 2 * nb - 1 - s); };
    // the thread's row's 16 entries of panel s's columns (rows after the panel
    // forward, before it backward), and for threads t < 16 row t (forward) or
    // column t (backward) of the inverse diagonal block. The loads read whole
    // panels of a row (rows are padded to ldm = 16 nb columns; the users drop
    // the padding columns and the rows that do not take part), threads past k
    // reading row 0, so that every load is in bounds and no load has to be
    // waited for before the panel that uses it.
    const double* __restrict__ myrow = Lm + int64_t(tid < k ? tid : 0) * ldm;
    const int dl = tid & 15;
    auto load_panel = [&](int s, double (&lp)[16], double (&dr)[16]) __attribute__((always_inline)) {
        const int c0 = panel_col(s < 2 * nb ? s : 0);
#pragma unroll
        for (int i = 0; i < 16; ++i) lp[i] = myrow[c0 + i];
        // forward: row t of the inverse block, from its transpose; backward:
        // column t; either way lanes read consecutive entries
        const double* db = Dinv + 256 * (c0 / 16 + (s < nb ? nb : 0));
#pragma unroll
        for (int i = 0; i < 16; ++i) dr[i] = db[16 * i + dl];
    };
    auto panel = [&](int s, const double (&lp)[16], const double (&dr)[16], double (&lpn)[16], double (&drn)[16])
                     __attribute__((always_inline)) {
        const bool fwd = s < nb;
        const int c0 = panel_col(s);
        load_panel(s + 1, lpn, drn);
        if (tid < 16) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) acc += dr[i] * bv[c0 + i];
            const bool live = c0 + tid < k;
            if (live) bv[c0 + tid] = acc;
            xs[tid] = live ? acc : 0.0;
        }
        lds_barrier();
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc += (c0 + i < k ? lp[i] : 0.0) * xs[i];
        if (tid < k && (fwd ? tid >= c0 + 16 : tid < c0)) bv[tid] -= acc;
        lds_barrier();
    };
    double lpa[16], dra[16], lpb[16], drb[16];
    load_panel(0, lpa, dra);
    {
        // w: the partial vectors added in segment order, 32 loads issued together
        // (in flight with the first panel's)
        double sum = 0.0;
        for (int g = 0; g < nseg; g += 32) {
            double x[32];
#pragma unroll
            for (int q = 0; q < 32; ++q) x[q] = (tid < k && g + q < nseg) ? wpart[int64_t(g + q) * k + tid] : 0.0;
#pragma unroll
            for (int q = 0; q < 32; ++q) sum += x[q];
        }
        bv[tid] = sum;
    }
    lds_barrier();
#pragma unroll 1
    for (int s = 0; s < 2 * nb; s += 2) {  // 2 nb panels: an even count
        panel(s, lpa, dra, lpb, drb);
        panel(s + 1, lpb, drb, lpa, dra);
    }
    if (tid < k) t[tid] = bv[tid];
}

// ------------------------------------------------------------------ IPM vector kernels
// theta = mu (1/a^2 + 1/(C - a)^2)
__global__ void k_theta(const double* __restrict__ a, int64_t N, double C, double mu,
                        double* __restrict__ th) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i >= N) return;
    double ai = a[i], bi = C - ai;
    th[i] = mu * (1.0 / (ai * ai) + 1.0 / (bi * bi));
}

// u = y * a (the vector the kernel is applied to: K Y a)
// w_i = |1 - y_i (K Y a)_i| * min(a_i, C - a_i): the complementarity that the
// reduced gradient at lambda = 0 would give at the starting point
__global__ void k_compl_scale(const double* __restrict__ y, const double* __restrict__ a,
                              const double* __restrict__ kya, int64_t N, double C, double* __restrict__ w) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    w[i] = fabs(1.0 - y[i] * kya[i]) * fmin(a[i], C - a[i]);
}

__global__ void k_mul(const double* __restrict__ y, const double* __restrict__ a, int64_t N,
                      double* __restrict__ u) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < N) u[i] = y[i] * a[i];
}

// Newton right-hand side: r1 = e - y*kya + lam y + mu/a - mu/(C-a); r[N] = y^T a (host value)
__global__ void k_rhs(const double* __restrict__ y, const double* __restrict__ a,
                      const double* __restrict__ kya, int64_t N, double lam, double mu, double C,
                      double r2, double* __restrict__ r) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < N) r[i] = 1.0 - y[i] * kya[i] + lam * y[i] + mu / a[i] - mu / (C - a[i]);
    if (i == N) r[N] = r2;
}

// IPM statistics after a step: sums of [alpha, (y a) . kya, hinge, xi_lambda^2, y.a]
__global__ void k_ipm_stats(const double* __restrict__ y, const double* __restrict__ a,
                            const double* __restrict__ kya, int64_t N, double lam, double mu, double C,
                            double* __restrict__ part) {
    double v[5] = {0, 0, 0, 0, 0};
    for (int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x; i < N; i += int64_t(gridDim.x) * kT) {
        double yi = y[i], ai = a[i], ki = kya[i];
        v[0] += ai;
        v[1] += yi * ai * ki;
        double m = 1.0 - yi * (ki - lam);
        v[2] += m > 0.0 ? m : 0.0;
        double xl = 1.0 - yi * ki + lam * yi + mu / ai - mu / (C - ai);
        v[3] += xl * xl;
        v[4] += yi * ai;
    }
    block_sums<5>(v, part);
}

// largest step in (0, inf] keeping 0 < a + s da < C: block partial minima
__global__ void k_step_partial(const double* __restrict__ a, const double* __restrict__ da, int64_t N,
                               double C, double* __restrict__ part) {
    __shared__ double sh[kT];
    double m = INFINITY;
    for (int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x; i < N; i += int64_t(gridDim.x) * kT) {
        double d = da[i];
        if (d < 0.0) m = fmin(m, -a[i] / d);
        else if (d > 0.0) m = fmin(m, (C - a[i]) / d);
    }
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_min_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    // lane j takes partials j, j + 64, ...; the minimum does not depend on the order
    double m = INFINITY;
#pragma unroll 8
    for (int b = threadIdx.x; b < nb; b += 64) m = fmin(m, part[b]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
    if (threadIdx.x == 0) out[0] = m;
}

__global__ void k_step(double* __restrict__ a, const double* __restrict__ da, int64_t N, double s) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < N) a[i] += s * da[i];
}

// ------------------------------------------------------------------ Newton operator, MINRES
// p = (A z) * sc - cprev * rprev, with A = [[Y K Y + Theta, -y], [-y^T, 0]] and
// kyz = K (y * z[0:N]) already computed; p[N] gets -y^T z[0:N] * sc - cprev*rprev[N]
// from the host-provided dot value.
// preconditioners with a low-rank factor of K (the others need none)
inline bool low_rank_precond(int p) {
    return p == ANOVA_PRECOND_PCHOL || p == ANOVA_PRECOND_NYSTROM || p == ANOVA_PRECOND_RPCHOL ||
           p == ANOVA_PRECOND_RFF;
}

// uniforms in [0, 1) for randomly pivoted Cholesky: splitmix64 (Steele, Lea and
// Flood 2014) of seed + j, top 53 bits
std::vector<double> pivot_uniforms(uint64_t seed, int n) {
    std::vector<double> u(static_cast<size_t>(n));
    for (int j = 0; j < n; ++j) {
        uint64_t z = seed + uint64_t(j) + 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        u[size_t(j)] = double(z >> 11) * 0x1.0p-53;
    }
    return u;
}

// MINRES iterations whose convergence flag the host reads before queueing the next
constexpr int kEagerChecks = 4;
constexpr int kGmRestart = 100;  // GMRES restart length cap (the basis holds one more column)

// sqrt(a^2 + b^2) from correctly rounded operations only (one fma), so that
// the host loop and the device kernel of MINRES round identically
__host__ __device__ inline double hypot_ieee(double a, double b) {
    a = fabs(a);
    b = fabs(b);
    const double m = a > b ? a : b, n = a > b ? b : a;
    if (m == 0.0) return 0.0;
    const double r = n / m;
    return m * sqrt(fma(r, r, 1.0));
}

// Scalars of one MINRES solve, kept on the device so that an iteration needs
// no host round trip: the three inner products of the iteration, the Lanczos
// and Givens recurrences, and the coefficients of the solution update.
struct KryScal {
    double dot_ytz, dot_a, dot_rz;             // y^T z, z^T p, r^T M^{-1} r
    double beta, beta_prev, beta1, c, s, dbar, eps_next, phibar;
    double rtol, inv_s;                        // relative tolerance; 1 / (y^T A_hat^{-1} y)
    double inv_beta_prev, eps_cur, delta, inv_gam, phi;  // update of this iteration
    int done;                                  // converged: later iterations change nothing
    int active;                                // this iteration updates the solution
    int kit;                                   // iterations that updated the solution
};

// start of a Newton solve: tolerance, preconditioner scalar, Givens state
__global__ void k_kry_start(KryScal* ks, double rtol, double s_last) {
    ks->rtol = rtol;
    ks->inv_s = 1.0 / s_last;
    ks->beta_prev = 0.0;
    ks->c = -1.0;
    ks->s = 0.0;
    ks->dbar = 0.0;
    ks->eps_next = 0.0;
    ks->done = 0;
    ks->active = 0;
    ks->kit = 0;
}

// beta_1 = sqrt(r0^T M^{-1} r0) from dot_rz
__global__ void k_kry_beta1(KryScal* ks) {
    const double b = sqrt(fmax(0.0, ks->dot_rz));
    ks->beta = b;
    ks->beta1 = b;
    ks->phibar = b;
    ks->done = b > 0.0 ? 0 : 1;
}

// p = A (z / beta) - (beta / beta_prev) r_prev, with A z = [Y K Y z + Theta z - y z_N ; -y^T z]
__global__ void k_newton_out(const double* __restrict__ y, const double* __restrict__ th,
                             const double* __restrict__ z, const double* __restrict__ kyz, int64_t N,
                             const KryScal* __restrict__ ks, const double* __restrict__ rprev,
                             double* __restrict__ p) {
    if (ks->done) return;
    const double sc = 1.0 / ks->beta;
    const double cprev = ks->kit > 0 ? ks->beta / ks->beta_prev : 0.0;
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < N) {
        double v = y[i] * kyz[i] + th[i] * z[i] - y[i] * z[N];
        p[i] = v * sc - cprev * rprev[i];
    } else if (i == N) {
        p[N] = -ks->dot_ytz * sc - cprev * rprev[N];
    }
}

// p -= (a / beta) r with a = z^T p / beta
__global__ void k_kry_axpy(double* __restrict__ p, const double* __restrict__ r, int64_t n,
                           const KryScal* __restrict__ ks) {
    if (ks->done) return;
    const double a = ks->dot_a / ks->beta;
    const double sa = -a / ks->beta;
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < n) p[i] += sa * r[i];
}

// Lanczos and Givens recurrences of one iteration (one thread), after the new
// beta's inner product
__global__ void k_kry_scalars(KryScal* ks) {
#pragma clang fp contract(off)  // round as the host loop does (no fused multiply-adds)
    if (ks->done) {
        ks->active = 0;
        return;
    }
    ks->active = 1;
    ks->kit += 1;
    const double a = ks->dot_a / ks->beta;
    const double beta_prev = ks->beta;
    const double beta = sqrt(fmax(0.0, ks->dot_rz));
    const double c = ks->c, s = ks->s, dbar = ks->dbar;
    const double eps_cur = ks->eps_next;
    const double delta = c * dbar + s * a;
    const double gbar = s * dbar - c * a;
    ks->eps_next = s * beta;
    ks->dbar = -c * beta;
    double gam = hypot_ieee(gbar, beta);
    if (gam == 0.0) gam = 1e-300;
    ks->c = gbar / gam;
    ks->s = beta / gam;
    ks->phi = ks->c * ks->phibar;
    ks->phibar = ks->s * ks->phibar;
    ks->beta_prev = beta_prev;
    ks->beta = beta;
    ks->inv_beta_prev = 1.0 / beta_prev;
    ks->eps_cur = eps_cur;
    ks->delta = delta;
    ks->inv_gam = 1.0 / gam;
    ks->done = (!(ks->phibar > ks->rtol * ks->beta1) || !(beta > 0.0)) ? 1 : 0;
}

// d_new = (z / beta_prev - eps d2 - delta d1) / gam; x += phi d_new; rotates d2 <- d1 <- d_new
__global__ void k_minres_update(const double* __restrict__ z, int64_t n, const KryScal* __restrict__ ks,
                                double* __restrict__ d1, double* __restrict__ d2, double* __restrict__ x) {
    if (!ks->active) return;
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i >= n) return;
    double dn = (z[i] * ks->inv_beta_prev - ks->eps_cur * d2[i] - ks->delta * d1[i]) * ks->inv_gam;
    d2[i] = d1[i];
    d1[i] = dn;
    x[i] += ks->phi * dn;
}

// by-value forms of the MINRES kernels, for solves whose host loop keeps the scalars
__global__ void k_newton_out_v(const double* __restrict__ y, const double* __restrict__ th,
                             const double* __restrict__ z, const double* __restrict__ kyz, int64_t N,
                             double sc, double cprev, const double* __restrict__ rprev,
                             double lastv, double* __restrict__ p) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < N) {
        double v = y[i] * kyz[i] + th[i] * z[i] - y[i] * z[N];
        p[i] = v * sc - cprev * rprev[i];
    } else if (i == N) {
        p[N] = lastv * sc - cprev * rprev[N];
    }
}

__global__ void k_axpy(double* __restrict__ x, const double* __restrict__ v, int64_t n, double s) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < n) x[i] += s * v[i];
}

// d_new = (z / beta - e * d2 - dl * d1) / gam; x += phi * d_new; rotates d2 <- d1 <- d_new
__global__ void k_minres_update_v(const double* __restrict__ z, int64_t n, double inv_beta, double e,
                                double dl, double inv_gam, double phi, double* __restrict__ d1,
                                double* __restrict__ d2, double* __restrict__ x) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i >= n) return;
    double dn = (z[i] * inv_beta - e * d2[i] - dl * d1[i]) * inv_gam;
    d2[i] = d1[i];
    d1[i] = dn;
    x[i] += phi * dn;
}

// ---- GMRES (Section 5): the Arnoldi basis V holds up to kGmMaxCols columns of
// length n = N + 1, column c at V + c * ldv
constexpr int kGmMaxCols = 128;
constexpr int kGmRows = 8;  // rows per thread of the basis inner products

// part[b * nc + c] = sum of V_c[i] w[i] over block b's rows (w held in registers)
__global__ __launch_bounds__(kT) void k_gm_dots(const double* __restrict__ V, int64_t ldv, int nc,
                                                const double* __restrict__ w, int64_t n, double* __restrict__ part) {
    const int64_t base = int64_t(blockIdx.x) * (kT * kGmRows) + threadIdx.x;
    double wr[kGmRows];
#pragma unroll
    for (int r = 0; r < kGmRows; ++r) {
        const int64_t i = base + int64_t(r) * kT;
        wr[r] = i < n ? w[i] : 0.0;
    }
    __shared__ double wsum[kT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = 0; c < nc; ++c) {
        const double* v = V + int64_t(c) * ldv;
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < kGmRows; ++r) {
            const int64_t i = base + int64_t(r) * kT;
            if (i < n) s += v[i] * wr[r];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) wsum[wave] = s;
        __syncthreads();
        if (threadIdx.x == 0) part[int64_t(blockIdx.x) * nc + c] = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
        __syncthreads();
    }
}

// w = (keep ? w : 0) - sum_{c < nc} V_c h_c
__global__ void k_gm_sub(const double* __restrict__ V, int64_t ldv, int nc, const double* __restrict__ h, int keep,
                         int64_t n, double* __restrict__ w) {
    __shared__ double hs[kGmMaxCols];
    for (int c = threadIdx.x; c < nc; c += kT) hs[c] = h[c];
    __syncthreads();
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < nc; ++c) s += V[int64_t(c) * ldv + i] * hs[c];
    w[i] = (keep ? w[i] : 0.0) - s;
}

// w = A [z; z_N] for the Newton matrix A = [[Y K Y + Theta, -y], [-y^T, 0]], with
// kyz = K (y o z), ytz = y^T z (device), and z_N the last entry of P^{-1} v:
// -(y^T z) - v_N for the block-triangular P (tri = 1), v_N for P = I (tri = 0)
__global__ void k_gm_op(const double* __restrict__ y, const double* __restrict__ th, const double* __restrict__ z,
                        const double* __restrict__ kyz, int64_t N, const double* __restrict__ ytz,
                        const double* __restrict__ v, int tri, double* __restrict__ w) {
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    const double d = *ytz;
    if (i < N) {
        const double zl = tri ? -d - v[N] : v[N];
        w[i] = y[i] * kyz[i] + th[i] * z[i] - y[i] * zl;
    } else if (i == N) {
        w[N] = -d;
    }
}

// r = b - A x, with kx = K (y o x) and ytx = y^T x (device)
__global__ void k_gm_resid(const double* __restrict__ y, const double* __restrict__ th, const double* __restrict__ x,
                           const double* __restrict__ kx, int64_t N, const double* __restrict__ ytx,
                           const double* __restrict__ b, double* __restrict__ r) {
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < N) r[i] = b[i] - (y[i] * kx[i] + th[i] * x[i] - y[i] * x[N]);
    else if (i == N) r[N] = b[N] + *ytx;
}

// x += P^{-1} u, given z = (P^{-1} u)_{1..N} and ytz = y^T z (device)
__global__ void k_gm_fin(const double* __restrict__ z, const double* __restrict__ ytz, const double* __restrict__ u,
                         int64_t N, int tri, double* __restrict__ x) {
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < N) x[i] += z[i];
    else if (i == N) x[N] += tri ? -*ytz - u[N] : u[N];
}

__global__ void k_scale(double* __restrict__ x, int64_t n, double s) {
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < n) x[i] *= s;
}

// Woodbury apply, first half: u = y * r / theta (written to tmp)
__global__ void k_wb_in(const double* __restrict__ y, const double* __restrict__ th,
                        const double* __restrict__ r, int64_t N, double* __restrict__ u) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < N) u[i] = y[i] * r[i] / th[i];
}

// second half: out = r / theta - (y / theta) * (Z t); out[N] = r[N] / s
template <class ZT>
__global__ void k_wb_out(const double* __restrict__ y, const double* __restrict__ th,
                         const double* __restrict__ r, const ZT* __restrict__ Z, int64_t N, int k,
                         const double* __restrict__ t, const double* __restrict__ inv_s, int has_last,
                         double* __restrict__ out) {
    __shared__ double ts[1024];
    for (int j = threadIdx.x; j < k; j += kT) ts[j] = t[j];
    __syncthreads();
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < N) {
        double zt = 0.0;
        for (int j = 0; j < k; ++j) zt += double(Z[int64_t(j) * N + i]) * ts[j];
        double ti = 1.0 / th[i];
        out[i] = r[i] * ti - y[i] * ti * zt;
    } else if (i == N && has_last) {
        out[N] = r[N] * *inv_s;
    }
}

// b = a rounded to FP32, and a replaced by those rounded values, so that both
// copies hold the same numbers
__global__ void k_narrow(double* __restrict__ a, int64_t n, float* __restrict__ b) {
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < n) {
        const float v = float(a[i]);
        b[i] = v;
        a[i] = double(v);
    }
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
    int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// out = Y T: Y N x k column-major, T k x kc row-major, out N x kc column-major.
// Block: 256 rows x 16 output columns; T's 16-column panel is staged in LDS.
__global__ void k_gemm_nk(const double* __restrict__ Y, int64_t N, int k, const double* __restrict__ T, int kc,
                          double* __restrict__ out) {
    extern __shared__ double tp_raw[];  // k x 16 panel of T
    double (*tp)[16] = reinterpret_cast<double (*)[16]>(tp_raw);
    const int j0 = blockIdx.y * 16;
    for (int e = threadIdx.x; e < k * 16; e += kT) {
        int m = e / 16, jj = e % 16;
        tp[m][jj] = (j0 + jj < kc) ? T[int64_t(m) * kc + j0 + jj] : 0.0;
    }
    __syncthreads();
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i >= N) return;
    double acc[16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) acc[jj] = 0.0;
    for (int m = 0; m < k; ++m) {
        const double y = Y[int64_t(m) * N + i];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) acc[jj] += y * tp[m][jj];
    }
#pragma unroll
    for (int jj = 0; jj < 16; ++jj)
        if (j0 + jj < kc) out[int64_t(j0 + jj) * N + i] = acc[jj];
}

// Gaussian test matrix: Philox4x32-10 (Salmon et al., SC'11) on the counter
// (row, column, 0, 0) with the seed as key, two 32-bit words -> a 53-bit uniform
// in (0, 1), Box-Muller with the next two words.
__device__ inline void philox_round(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
    const uint64_t p0 = uint64_t(0xD2511F53u) * c[0];
    const uint64_t p1 = uint64_t(0xCD9E8D57u) * c[2];
    const uint32_t hi0 = uint32_t(p0 >> 32), lo0 = uint32_t(p0);
    const uint32_t hi1 = uint32_t(p1 >> 32), lo1 = uint32_t(p1);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}
__device__ inline void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        philox_round(c, k0, k1);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}
__global__ void k_gaussian(double* __restrict__ G, int64_t N, int k, uint64_t seed) {
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= N) return;
    uint32_t c[4] = {uint32_t(i), uint32_t(uint64_t(i) >> 32), uint32_t(j), 0u};
    philox4x32_10(c, uint32_t(seed), uint32_t(seed >> 32));
    const double u1 = (double((uint64_t(c[0]) << 21) ^ (c[1] >> 11)) + 0.5) * 0x1.0p-53;
    const double u2 = (double((uint64_t(c[2]) << 21) ^ (c[3] >> 11)) + 0.5) * 0x1.0p-53;
    G[int64_t(j) * N + i] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// fraction of the gap tolerance at which the IPM stops (the rest covers the
// difference between the gap in the fast-summation kernel and in the exact one)
constexpr double kGapMargin = 0.5;
// the barrier parameter is not reduced below the value whose central point has
// this fraction of the gap tolerance as its relative duality gap
constexpr double kMuFloor = 1e-2;

// ------------------------------------------------------------------ host helpers
struct Reducer {
    DevBuf<double> part, out;
    double* host = nullptr;
    Reducer() {
        part.alloc(size_t(kRedBlocks) * 8);
        out.alloc(8);
        ANV_HIP(hipHostMalloc(&host, 8 * sizeof(double)));
    }
    ~Reducer() {
        if (host) (void)hipHostFree(host);
    }
    unsigned blocks(int64_t n) const { return unsigned(std::min<int64_t>(kRedBlocks, nblk(n))); }
    // sums of NS dot products of length n, read back to host (synchronises)
    template <int NS>
    const double* dots(const DotArgs& d, int64_t n, hipStream_t st) {
        unsigned nb = blocks(n);
        hipLaunchKernelGGL(k_dots<NS>, dim3(nb), dim3(kT), 0, st, d, n, part.p);
        hipLaunchKernelGGL(k_fold_partials, dim3(NS), dim3(64), 0, st, part.p, int(nb), NS, out.p);
        ANV_HIP(hipMemcpyAsync(host, out.p, NS * sizeof(double), hipMemcpyDeviceToHost, st));
        host_wait(st);
        return host;
    }
    double dot(const double* a, const double* b, int64_t n, hipStream_t st) {
        DotArgs d{};
        d.a[0] = a;
        d.b[0] = b;
        return dots<1>(d, n, st)[0];
    }
    // a^T b into out (device), no host wait
    void dot_dev(const double* a, const double* b, int64_t n, double* out, hipStream_t st) {
        DotArgs d{};
        d.a[0] = a;
        d.b[0] = b;
        const unsigned nb = blocks(n);
        hipLaunchKernelGGL(k_dots<1>, dim3(nb), dim3(kT), 0, st, d, n, part.p);
        hipLaunchKernelGGL(k_fold_partials, dim3(1), dim3(64), 0, st, part.p, int(nb), 1, out);
    }
};

struct Workspace {
    int64_t N = 0;
    int k = 0;
    int* hstatus = nullptr;               // pinned mirror of status
    Workspace() { ANV_HIP(hipHostMalloc(&hstatus, sizeof(int))); }
    ~Workspace() {
        if (hstatus) (void)hipHostFree(hstatus);
    }
    Workspace(const Workspace&) = delete;
    Workspace& operator=(const Workspace&) = delete;
    const double* Z = nullptr;            // N x k column-major low-rank factor Z^T
    const float* Z32 = nullptr;           // its FP32 copy, when the N x k products run in FP32
    DevBuf<double> M, Mpart, Mgrp, t;     // capacitance (its factor in place), partials, group sums, M^{-1} w
    DevBuf<double> Dinv;                  // inverses of the factor's 16 x 16 diagonal blocks and their transposes
    DevBuf<int> status;
    DevBuf<double> tmp, kyz;              // N
    DevBuf<double> wpart;                 // per-segment partials of Z^T u
    int ldm = 0;                          // leading dimension of M
    int nchunk = 0;
    int64_t chunk = 0;
    int nseg = 1;
    int64_t seg = 1;
};

// kernel matvec of one vector (device pointers, length N)
void kmv(Plan& pl, const MatvecHook* hook, const double* x, double* y, hipStream_t st) {
    if (hook)
        (*hook)(x, y, st);
    else
        enqueue_matvec(pl, x, 1, pl.N, y, pl.N, st);
}

// A_hat^{-1} applied to r (first N entries); out[N] = r[N] * inv_s[0] (device) when has_last
void woodbury_apply(Workspace& ws, const double* y, const double* th, const double* r, const double* inv_s,
                    bool has_last, double* out, hipStream_t st) {
    const int64_t N = ws.N;
    if (ws.k > 0) {
        hipLaunchKernelGGL(k_wb_in, dim3(nblk(N)), dim3(kT), 0, st, y, th, r, N, ws.tmp.p);
        const dim3 g(unsigned((ws.k + kGemvCols - 1) / kGemvCols), unsigned(ws.nseg));
        if (ws.Z32 && N % 4 == 0 && ws.seg % 4 == 0)
            hipLaunchKernelGGL(k_gemv_t_seg4, g, dim3(kT), 0, st, ws.Z32, N, ws.k, ws.tmp.p, ws.seg, ws.wpart.p);
        else if (ws.Z32)
            hipLaunchKernelGGL(k_gemv_t_seg<float>, g, dim3(kT), 0, st, ws.Z32, N, ws.k, ws.tmp.p, ws.seg, ws.wpart.p);
        else
            hipLaunchKernelGGL(k_gemv_t_seg<double>, g, dim3(kT), 0, st, ws.Z, N, ws.k, ws.tmp.p, ws.seg, ws.wpart.p);
        if (ws.k <= kRegCholK)
            hipLaunchKernelGGL(k_chol_solve_b, dim3(1), dim3(kSbT), 0, st, ws.M.p, ws.k, ws.ldm, ws.Dinv.p, ws.wpart.p,
                               ws.nseg, ws.t.p);
        else
            hipLaunchKernelGGL(k_chol_solve, dim3(1), dim3(256), ws.k * sizeof(double), st, ws.M.p, ws.k,
                               ws.wpart.p, ws.nseg, ws.t.p);
    }
    if (ws.Z32)
        hipLaunchKernelGGL(k_wb_out<float>, dim3(nblk(N + 1)), dim3(kT), 0, st, y, th, r, ws.Z32, N, ws.k, ws.t.p,
                           inv_s, has_last ? 1 : 0, out);
    else
        hipLaunchKernelGGL(k_wb_out<double>, dim3(nblk(N + 1)), dim3(kT), 0, st, y, th, r, ws.Z, N, ws.k, ws.t.p,
                           inv_s, has_last ? 1 : 0, out);
}

void refresh_capacitance(Workspace& ws, const double* th, hipStream_t st) {
    if (ws.k == 0) return;
    const int k = ws.k;
    const int ns = (k + kST - 1) / kST;
    // the FP64 factor (holding the FP32 copy's values when there is one): the
    // 128-column panels of the Gram kernel read whole 128-byte rows in FP64
    if (k <= kRegCholK)
        hipLaunchKernelGGL((k <= 208 ? k_syrk_tri<12, 32> : k_syrk_tri<17, 16>), dim3(unsigned(ws.nchunk)), dim3(64 * kSyW), 0,
                           st, ws.Z, ws.N, k, th, ws.chunk, ws.Mpart.p);
    else
        hipLaunchKernelGGL(k_syrk_mfma<double>, dim3(unsigned(ns * (ns + 1) / 2), unsigned(ws.nchunk)), dim3(256), 0,
                           st, ws.Z, ws.N, k, th, ws.chunk, ws.Mpart.p);
    const int ng = std::min(ws.nchunk, kFoldGroups);
    hipLaunchKernelGGL(k_syrk_fold_grp, dim3(nblk(int64_t(k) * k), unsigned(ng)), dim3(kT), 0, st, ws.Mpart.p,
                       ws.nchunk, k, ws.Mgrp.p);
    hipLaunchKernelGGL(k_syrk_fold_fin, dim3(nblk(int64_t(k) * k)), dim3(kT), 0, st, ws.Mgrp.p, ng, k, 1.0, ws.M.p,
                       ws.ldm);
    if (k <= kRegCholK) {
        hipLaunchKernelGGL(k <= 208 ? k_chol_reg<12> : k_chol_reg<17>, dim3(1), dim3(64 * kRegWaves), 0, st, ws.M.p, k,
                           ws.ldm, ws.status.p);
        hipLaunchKernelGGL(k_diag_inv, dim3(unsigned((k + 15) / 16)), dim3(64), 0, st, ws.M.p, k, ws.ldm, ws.Dinv.p);
    } else
        hipLaunchKernelGGL(k_chol, dim3(1), dim3(kCholT), 0, st, ws.M.p, k, ws.status.p);
    // read back through pinned memory: an asynchronous copy into pageable
    // (here: stack) memory is not guaranteed to have landed when the stream's
    // later work completes
    ANV_HIP(hipMemcpyAsync(ws.hstatus, ws.status.p, sizeof(int), hipMemcpyDeviceToHost, st));
    host_wait(st);
    if (*ws.hstatus) throw Error(ANOVA_NUMERICAL, "capacitance matrix is not positive definite");
}

void setup_factor_storage(Workspace& ws, int64_t N, int k) {
    ws.N = N;
    ws.k = k;
    if (k > 0) {
        // rows of the register-resident factor padded to whole 16-column panels
        ws.ldm = k <= kRegCholK ? (k + 15) / 16 * 16 : k;
        ws.M.alloc(size_t(k) * ws.ldm);
        if (k <= kRegCholK) ws.Dinv.alloc(size_t((k + 15) / 16) * 512);
        ws.t.alloc(k);
        ws.status.alloc(1);
        if (k <= kRegCholK)
            syrk_tri_chunks(N, k, ws.nchunk, ws.chunk);
        else
            syrk_chunks(N, k, ws.nchunk, ws.chunk);
        ws.Mpart.alloc(size_t(ws.nchunk) * k * k);
        ws.Mgrp.alloc(size_t(std::min(ws.nchunk, kFoldGroups)) * k * k);
        // segments of Z^T u: about 1024 blocks in all (fewer partial sums for the
        // solve to fold, and still four blocks per compute unit)
        const int64_t ncb = (k + kGemvCols - 1) / kGemvCols;
        ws.nseg = int(std::max<int64_t>(1, std::min<int64_t>((1024 + ncb - 1) / ncb, (N + 4095) / 4096)));
        ws.seg = ((N + ws.nseg - 1) / ws.nseg + 3) / 4 * 4;  // whole groups of 4 rows
        ws.nseg = int((N + ws.seg - 1) / ws.seg);
        ws.wpart.alloc(size_t(ws.nseg) * k);
    }
    ws.tmp.alloc(N + 1);
    ws.kyz.alloc(N + 1);
}

// greedy pivoted Cholesky into a column-major N x ldl buffer; returns rank
// greedy pivoted Cholesky (uniforms == NULL) or randomly pivoted Cholesky with
// one uniform per step (host array of `rank` values in [0, 1))
int pchol_into(Plan& pl, int rank, double err_tol, double* L, int64_t ldl, int64_t* piv, hipStream_t st,
               const double* uniforms = nullptr) {
    const int64_t N = pl.N;
    const int P = pl.P;
    ANV_CHECK(ldl == N, "internal: pivoted Cholesky storage must have ldl == N");
    std::vector<double> inv_s2(P), eta(P);
    double kpp = 0.0;
    for (int l = 0; l < P; ++l) {
        inv_s2[l] = 1.0 / (pl.sigma[l] * pl.sigma[l]);
        eta[l] = pl.eta[l];
        kpp += eta[l];
    }
    ANV_CHECK(kpp > 0.0, "pivoted Cholesky needs a positive kernel diagonal (sum of eta > 0)");
    DevBuf<double> is2, et, dres, pv, ps, fin;
    DevBuf<int64_t> pi;
    is2.alloc(P);
    et.alloc(P);
    ANV_HIP(hipMemcpyAsync(is2.p, inv_s2.data(), P * sizeof(double), hipMemcpyHostToDevice, st));
    ANV_HIP(hipMemcpyAsync(et.p, eta.data(), P * sizeof(double), hipMemcpyHostToDevice, st));
    dres.alloc(N);
    hipLaunchKernelGGL(k_fill, dim3(nblk(N)), dim3(kT), 0, st, dres.p, N, kpp);
    const unsigned nb = unsigned(std::min<int64_t>(kRedBlocks, nblk(N)));
    pv.alloc(nb);
    ps.alloc(nb);
    pi.alloc(nb);
    fin.alloc(4);
    double* hfin = nullptr;
    ANV_HIP(hipHostMalloc(&hfin, 4 * sizeof(double)));
    const double trace0 = kpp * double(N);
    int r = 0;
    try {
        for (; r < rank; ++r) {
            if (uniforms) {
                const int64_t chunk = (N + nb - 1) / nb;
                const unsigned nbs = unsigned((N + chunk - 1) / chunk);
                hipLaunchKernelGGL(k_block_sums, dim3(nbs), dim3(kT), 0, st, dres.p, N, chunk, ps.p);
                hipLaunchKernelGGL(k_sample_pivot, dim3(1), dim3(1), 0, st, dres.p, N, chunk, ps.p, int(nbs),
                                   uniforms[r], fin.p);
            } else {
                hipLaunchKernelGGL(k_argmax_sum, dim3(nb), dim3(kT), 0, st, dres.p, N, pv.p, pi.p, ps.p);
                hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(64), 0, st, pv.p, pi.p, ps.p, int(nb), fin.p);
            }
            ANV_HIP(hipMemcpyAsync(hfin, fin.p, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
            host_wait(st);
            const double best = hfin[0], rest = hfin[2];
            const int64_t p = int64_t(hfin[1]);
            if (!(best > 0.0)) break;
            if (err_tol > 0.0 && rest <= err_tol * trace0) break;
            hipLaunchKernelGGL(k_pivot_value, dim3(1), dim3(1), 0, st, L, N, p, r, kpp, fin.p + 3);
            ANV_HIP(hipMemcpyAsync(hfin + 3, fin.p + 3, sizeof(double), hipMemcpyDeviceToHost, st));
            host_wait(st);
            const double pivval = hfin[3];
            if (!(pivval > 0.0)) break;
            hipLaunchKernelGGL(k_pchol_column, dim3(nblk(N)), dim3(kT), 0, st, pl.xw.p, N, P, is2.p, et.p, p,
                               r, L, dres.p, pivval);
            ANV_HIP(hipGetLastError());
            piv[r] = p;
        }
    } catch (...) {
        (void)hipHostFree(hfin);
        throw;
    }
    (void)hipHostFree(hfin);
    host_wait(st);
    return r;
}

// ---- small dense helpers (host, FP64, k <= 1024)
// lower Cholesky in place (row-major); returns false on a non-positive pivot
bool host_chol(std::vector<double>& A, int k) {
    for (int j = 0; j < k; ++j) {
        double d = A[size_t(j) * k + j];
        for (int m = 0; m < j; ++m) d -= A[size_t(j) * k + m] * A[size_t(j) * k + m];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        A[size_t(j) * k + j] = d;
        for (int i = j + 1; i < k; ++i) {
            double v = A[size_t(i) * k + j];
            for (int m = 0; m < j; ++m) v -= A[size_t(i) * k + m] * A[size_t(j) * k + m];
            A[size_t(i) * k + j] = v / d;
        }
    }
    return true;
}
// T = L^{-T} (row-major k x k upper triangular), L lower from host_chol
std::vector<double> inv_lower_transposed(const std::vector<double>& L, int k) {
    std::vector<double> X(size_t(k) * k, 0.0);  // X = L^{-1}, lower
    for (int c = 0; c < k; ++c) {
        X[size_t(c) * k + c] = 1.0 / L[size_t(c) * k + c];
        for (int i = c + 1; i < k; ++i) {
            double v = 0.0;
            for (int m = c; m < i; ++m) v -= L[size_t(i) * k + m] * X[size_t(m) * k + c];
            X[size_t(i) * k + c] = v / L[size_t(i) * k + i];
        }
    }
    std::vector<double> T(size_t(k) * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) T[size_t(i) * k + j] = X[size_t(j) * k + i];
    return T;
}

// out = Y T (Y: N x k column-major, T: k x kc row-major, out: N x kc column-major)
void gemm_nk(const double* Y, int64_t N, int k, const double* T, int kc, double* out, hipStream_t st) {
    if (k <= 16 * kGmCB && kc <= 16 * kGmCB)
        hipLaunchKernelGGL(k_gemm_nk_mfma, dim3(unsigned((N + 16 * kGmW - 1) / (16 * kGmW))), dim3(64 * kGmW), 0, st, Y,
                           N, k, T, kc, out);
    else
        hipLaunchKernelGGL(k_gemm_nk, dim3(nblk(N), unsigned((kc + 15) / 16)), dim3(kT), k * 16 * sizeof(double), st,
                           Y, N, k, T, kc, out);
}

struct Gram {
    DevBuf<double> part, M, gsum;
    int nchunk = 1, nchunk_s = 1, nchunk_t = 1;
    int64_t chunk = 1, chunk_s = 1, chunk_t = 1;
    void setup(int64_t N, int k) {
        chunk = 8192;
        nchunk = int(std::min<int64_t>(256, (N + chunk - 1) / chunk));
        chunk = (N + nchunk - 1) / nchunk;
        syrk_chunks(N, k, nchunk_s, chunk_s);
        syrk_tri_chunks(N, k, nchunk_t, chunk_t);
        part.alloc(size_t(std::max(std::max(nchunk, nchunk_s), nchunk_t)) * k * k);
        gsum.alloc(size_t(kFoldGroups) * k * k);
        M.alloc(size_t(k) * k);
    }
    // the chunk partials of the balanced kernels, folded in order (full: a
    // general product; else the lower triangle, mirrored)
    void fold_tri(int k, bool full, hipStream_t st) {
        const int ng = std::min(nchunk_t, kFoldGroups);
        hipLaunchKernelGGL(k_syrk_fold_grp, dim3(nblk(int64_t(k) * k), unsigned(ng)), dim3(kT), 0, st, part.p,
                           nchunk_t, k, gsum.p, full ? 1 : 0);
        hipLaunchKernelGGL(k_syrk_fold_fin, dim3(nblk(int64_t(k) * k)), dim3(kT), 0, st, gsum.p, ng, k, 0.0, M.p, k,
                           full ? 1 : 0);
    }
    // host copy of A^T B (k x k, row-major), on the matrix cores for k <= 208
    // (A == B: k <= 256)
    std::vector<double> run(const double* A, const double* B, int64_t N, int k, hipStream_t st) {
        if (A == B && k <= kRegCholK) {
            hipLaunchKernelGGL((k <= 208 ? k_syrk_tri<12, 32> : k_syrk_tri<17, 16>), dim3(unsigned(nchunk_t)), dim3(64 * kSyW), 0,
                               st, A, N, k, (const double*)nullptr, chunk_t, part.p);
            fold_tri(k, false, st);
        } else if (A != B && k <= 208) {
            hipLaunchKernelGGL(k_gram_mfma, dim3(unsigned(nchunk_t), kGrSplit), dim3(64 * kGrW), 0, st, A, B, N, k,
                               chunk_t, part.p);
            fold_tri(k, true, st);
        } else if (A == B) {
            const int ns = (k + kST - 1) / kST;
            hipLaunchKernelGGL(k_syrk_mfma<double>, dim3(unsigned(ns * (ns + 1) / 2), unsigned(nchunk_s)), dim3(256), 0, st, A,
                               N, k, (const double*)nullptr, chunk_s, part.p);
            hipLaunchKernelGGL(k_syrk_fold, dim3(nblk(int64_t(k) * k)), dim3(kT), 0, st, part.p, nchunk_s, k, 0.0,
                               M.p);
        } else {
            const int tiles = (k + kSy - 1) / kSy;
            hipLaunchKernelGGL(k_gram_partial, dim3(tiles, tiles, nchunk), dim3(kT), 0, st, A, B, N, k,
                               (const double*)nullptr, chunk, part.p);
            hipLaunchKernelGGL(k_gram_fold, dim3(nblk(int64_t(k) * k)), dim3(kT), 0, st, part.p, nchunk, k, 0.0,
                               M.p);
        }
        std::vector<double> h(size_t(k) * k);
        ANV_HIP(hipMemcpyAsync(h.data(), M.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        host_wait(st);
        return h;
    }
};

// Q <- orth(Y) in place by shifted Cholesky-QR followed by two Cholesky-QR passes
void orthonormalize(DevBuf<double>& Y, DevBuf<double>& tmp, int64_t N, int k, hipStream_t st) {
    Gram gr;
    gr.setup(N, k);
    DevBuf<double> T;
    T.alloc(size_t(k) * k);
    for (int pass = 0; pass < 3; ++pass) {
        std::vector<double> A = gr.run(Y.p, Y.p, N, k, st);
        double tr = 0.0;
        for (int j = 0; j < k; ++j) tr += A[size_t(j) * k + j];
        ANV_CHECK(std::isfinite(tr), "non-finite Gram matrix in orthonormalisation");
        if (!(tr > 0.0)) throw Error(ANOVA_NUMERICAL, "orthonormalisation: zero matrix");
        // first pass: shift 11 (N k + k(k+1)) u ||Y||_F^2 (shifted Cholesky-QR); later passes
        // shift only if the unshifted factorisation breaks down
        double shift = pass == 0 ? 11.0 * (double(N) * k + double(k) * (k + 1)) * 0x1.0p-53 * tr : 0.0;
        std::vector<double> L;
        for (int attempt = 0; attempt < 8; ++attempt) {
            L = A;
            for (int j = 0; j < k; ++j) L[size_t(j) * k + j] += shift;
            if (host_chol(L, k)) break;
            shift = shift > 0.0 ? shift * 100.0 : 1e-14 * tr;
            if (attempt == 7) throw Error(ANOVA_NUMERICAL, "orthonormalisation: Cholesky-QR broke down");
        }
        std::vector<double> Th = inv_lower_transposed(L, k);
        ANV_HIP(hipMemcpyAsync(T.p, Th.data(), Th.size() * sizeof(double), hipMemcpyHostToDevice, st));
        gemm_nk(Y.p, N, k, T.p, k, tmp.p, st);
        std::swap(Y.p, tmp.p);
    }
    host_wait(st);
}

// Z^T (N x k, column-major, ld N) = (K Q) L^{-T} D^{-1/2} with Q^T K Q = L D L^T (clamped)
void nystrom_core(Plan& pl, DevBuf<double>& Y, int k, double* Zt, hipStream_t st) {
    const int64_t N = pl.N;
    DevBuf<double> tmp;
    tmp.alloc(size_t(N) * k);
    orthonormalize(Y, tmp, N, k, st);                    // Y := Q
    enqueue_matvec(pl, Y.p, k, N, tmp.p, N, st);          // tmp := B = K Q
    Gram gr;
    gr.setup(N, k);
    std::vector<double> Cm = gr.run(Y.p, tmp.p, N, k, st);  // Q^T K Q
    double dmax = 0.0;
    for (int i = 0; i < k; ++i) {
        for (int j = 0; j < i; ++j) {
            double v = 0.5 * (Cm[size_t(i) * k + j] + Cm[size_t(j) * k + i]);
            Cm[size_t(i) * k + j] = Cm[size_t(j) * k + i] = v;
        }
        dmax = std::max(dmax, Cm[size_t(i) * k + i]);
    }
    ANV_CHECK(std::isfinite(dmax), "non-finite Q^T K Q");
    // LDL^T without pivoting; D entries below tau are raised to tau (Section 4).
    // tau sits at the operator's relative accuracy: below it, directions of
    // Q^T K Q are rounding noise of the matvec (FP32 grids: about 1e-7), and
    // raising them to a much smaller value would amplify that noise in Z.
    const double tau = (pl.precision == ANOVA_PREC_FP64 ? 1e-12 : 1e-6) * dmax;
    std::vector<double> L(size_t(k) * k, 0.0), D(k);
    for (int j = 0; j < k; ++j) {
        double dj = Cm[size_t(j) * k + j];
        for (int m = 0; m < j; ++m) dj -= L[size_t(j) * k + m] * L[size_t(j) * k + m] * D[m];
        if (!(dj >= tau)) dj = tau;
        D[j] = dj;
        L[size_t(j) * k + j] = 1.0;
        for (int i = j + 1; i < k; ++i) {
            double v = Cm[size_t(i) * k + j];
            for (int m = 0; m < j; ++m) v -= L[size_t(i) * k + m] * L[size_t(j) * k + m] * D[m];
            L[size_t(i) * k + j] = v / dj;
        }
    }
    std::vector<double> T = inv_lower_transposed(L, k);   // L^{-T}
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) T[size_t(i) * k + j] /= std::sqrt(D[j]);
    DevBuf<double> Td;
    Td.alloc(size_t(k) * k);
    ANV_HIP(hipMemcpyAsync(Td.p, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice, st));
    gemm_nk(tmp.p, N, k, Td.p, k, Zt, st);
    ANV_HIP(hipGetLastError());
    host_wait(st);
}

}  // namespace

void lowrank_apply(int64_t N, int k, const double* Z, int64_t ldz, const double* theta, const double* y,
                   const double* r, bool fp32_products, double* out, hipStream_t st) {
    ANV_CHECK(N >= 1 && k >= 1 && k <= 1024, "need N >= 1 and 1 <= k <= 1024");
    ANV_CHECK(Z && theta && r && out && ldz >= N, "NULL pointer or ldz < N");
    DevBuf<double> zc, yc;
    DevBuf<float> z32;
    zc.alloc(size_t(N) * k);
    ANV_HIP(hipMemcpy2DAsync(zc.p, N * sizeof(double), Z, ldz * sizeof(double), N * sizeof(double), k,
                             hipMemcpyDeviceToDevice, st));
    if (!y) {
        yc.alloc(N);
        hipLaunchKernelGGL(k_fill, dim3(nblk(N)), dim3(kT), 0, st, yc.p, N, 1.0);
        y = yc.p;
    }
    Workspace ws;
    ws.Z = zc.p;
    if (fp32_products) {  // as the solver does: both copies hold the FP32-rounded values
        z32.alloc(size_t(N) * k);
        hipLaunchKernelGGL(k_narrow, dim3(nblk(int64_t(N) * k)), dim3(kT), 0, st, zc.p, int64_t(N) * k, z32.p);
        ws.Z32 = z32.p;
    }
    setup_factor_storage(ws, N, k);
    refresh_capacitance(ws, theta, st);  // synchronises the stream
    woodbury_apply(ws, y, theta, r, nullptr, false, out, st);
    host_wait(st);                       // the buffers above are released on return
}

int pivoted_cholesky(Plan& pl, int rank, double err_tol, double* L, int64_t ldl, int64_t* piv, hipStream_t st,
                     const double* uniforms) {
    if (ldl == pl.N) return pchol_into(pl, rank, err_tol, L, ldl, piv, st, uniforms);
    DevBuf<double> tmp;
    tmp.alloc(size_t(pl.N) * rank);
    int r = pchol_into(pl, rank, err_tol, tmp.p, pl.N, piv, st, uniforms);
    if (r > 0)
        ANV_HIP(hipMemcpy2DAsync(L, ldl * sizeof(double), tmp.p, pl.N * sizeof(double), pl.N * sizeof(double), r,
                                 hipMemcpyDeviceToDevice, st));
    host_wait(st);
    return r;
}

std::vector<int> rff_counts(int k, int P) {
    std::vector<int> c(size_t(P), k / P);
    for (int l = 0; l < k % P; ++l) ++c[size_t(l)];
    return c;
}

void rff_factor(Plan& pl, int k, const double* w, const double* b, double* Z, int64_t ldz, hipStream_t st) {
    const int64_t N = pl.N;
    const int P = pl.P;
    ANV_CHECK(k >= 1 && k <= 65535, "k must be in [1, 65535]");
    ANV_CHECK(ldz >= N, "ldz < N");
    const std::vector<int> cnt = rff_counts(k, P);
    std::vector<int32_t> fwin(size_t(k), 0);
    std::vector<double> fw(static_cast<size_t>(k) * 3, 0.0), fb(static_cast<size_t>(k)), fs(static_cast<size_t>(k));
    int j = 0;
    for (int l = 0; l < P; ++l) {
        int nf = 0;
        for (int a = 0; a < 3; ++a) nf += pl.slot_feat[size_t(l)][size_t(a)] >= 0;
        for (int q = 0; q < cnt[size_t(l)]; ++q, ++j) {
            fwin[size_t(j)] = l;
            for (int a = 0; a < nf; ++a) fw[size_t(j) * 3 + size_t(3 - nf + a)] = w[size_t(j) * 3 + size_t(a)];
            fb[size_t(j)] = b[size_t(j)];
            fs[size_t(j)] = std::sqrt(pl.eta[size_t(l)] * 2.0 / cnt[size_t(l)]);
        }
    }
    DevBuf<int32_t> dwin;
    DevBuf<double> dw, db, ds, Zc;
    dwin.alloc(size_t(k));
    dw.alloc(size_t(k) * 3);
    db.alloc(size_t(k));
    ds.alloc(size_t(k));
    ANV_HIP(hipMemcpyAsync(dwin.p, fwin.data(), fwin.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    ANV_HIP(hipMemcpyAsync(dw.p, fw.data(), fw.size() * sizeof(double), hipMemcpyHostToDevice, st));
    ANV_HIP(hipMemcpyAsync(db.p, fb.data(), fb.size() * sizeof(double), hipMemcpyHostToDevice, st));
    ANV_HIP(hipMemcpyAsync(ds.p, fs.data(), fs.size() * sizeof(double), hipMemcpyHostToDevice, st));
    double* out = Z;
    if (ldz != N) {
        Zc.alloc(size_t(N) * k);
        out = Zc.p;
    }
    hipLaunchKernelGGL(k_rff, dim3(nblk(N), unsigned(k)), dim3(kT), 0, st, pl.xw.p, N, P, dwin.p, dw.p, db.p, ds.p,
                       out);
    ANV_HIP(hipGetLastError());
    if (ldz != N)
        ANV_HIP(hipMemcpy2DAsync(Z, ldz * sizeof(double), out, N * sizeof(double), N * sizeof(double), k,
                                 hipMemcpyDeviceToDevice, st));
    host_wait(st);
}

void nystrom_factor(Plan& pl, const double* G, int k, int64_t ldg, double* Zt, int64_t ldz, hipStream_t st) {
    const int64_t N = pl.N;
    ANV_CHECK(k <= 1024, "k must be <= 1024");
    DevBuf<double> Y, Gc;
    Y.alloc(size_t(N) * k);
    Gc.alloc(size_t(N) * k);
    ANV_HIP(hipMemcpy2DAsync(Gc.p, N * sizeof(double), G, ldg * sizeof(double), N * sizeof(double), k,
                             hipMemcpyDeviceToDevice, st));
    enqueue_matvec(pl, Gc.p, k, N, Y.p, N, st);          // Y = K G
    if (ldz == N) {
        nystrom_core(pl, Y, k, Zt, st);
    } else {
        DevBuf<double> Z;
        Z.alloc(size_t(N) * k);
        nystrom_core(pl, Y, k, Z.p, st);
        ANV_HIP(hipMemcpy2DAsync(Zt, ldz * sizeof(double), Z.p, N * sizeof(double), N * sizeof(double), k,
                                 hipMemcpyDeviceToDevice, st));
        host_wait(st);
    }
}

// ------------------------------------------------------------------ Algorithm 1
void build_low_rank(Plan& pl, const anova_ipm_opts& o, LowRankFactor& f, hipStream_t st) {
    using clk = std::chrono::steady_clock;
    const int64_t N = pl.N;
    ANV_CHECK(o.precond == ANOVA_PRECOND_NONE || o.precond == ANOVA_PRECOND_PCHOL ||
                  o.precond == ANOVA_PRECOND_NYSTROM || o.precond == ANOVA_PRECOND_DIAG ||
                  o.precond == ANOVA_PRECOND_RPCHOL || o.precond == ANOVA_PRECOND_RFF,
              "unknown preconditioner");
    ANV_CHECK(!low_rank_precond(o.precond) || (o.rank >= 1 && o.rank <= std::min<int64_t>(N, 1024)),
              "rank must be in [1, min(N, 1024)]");
    const auto t0 = clk::now();
    f.precond = o.precond;
    f.rank = 0;
    if (o.precond == ANOVA_PRECOND_PCHOL || o.precond == ANOVA_PRECOND_RPCHOL) {
        f.Z.alloc(size_t(N) * o.rank);
        std::vector<int64_t> piv(o.rank);
        std::vector<double> u;
        if (o.precond == ANOVA_PRECOND_RPCHOL) u = pivot_uniforms(o.seed, o.rank);
        f.rank = pchol_into(pl, o.rank, o.err_tol, f.Z.p, N, piv.data(), st, u.empty() ? nullptr : u.data());
    } else if (o.precond == ANOVA_PRECOND_RFF) {
        // draws: w ~ N(0, 2 / sigma_l^2) per window coordinate (Box-Muller on
        // splitmix64 uniforms), b ~ U(0, 2 pi)
        f.rank = o.rank;
        f.Z.alloc(size_t(N) * o.rank);
        const std::vector<int> cnt = rff_counts(o.rank, pl.P);
        const std::vector<double> u = pivot_uniforms(o.seed, 8 * o.rank);
        std::vector<double> w(size_t(o.rank) * 3), b(size_t(o.rank));
        int j = 0;
        for (int l = 0; l < pl.P; ++l)
            for (int q = 0; q < cnt[size_t(l)]; ++q, ++j) {
                const double sw = std::sqrt(2.0) / pl.sigma[size_t(l)];
                const double* uu = u.data() + size_t(8) * j;
                const double r0 = std::sqrt(-2.0 * std::log(1.0 - uu[0])), r1 = std::sqrt(-2.0 * std::log(1.0 - uu[2]));
                w[size_t(j) * 3 + 0] = sw * r0 * std::cos(2.0 * M_PI * uu[1]);
                w[size_t(j) * 3 + 1] = sw * r0 * std::sin(2.0 * M_PI * uu[1]);
                w[size_t(j) * 3 + 2] = sw * r1 * std::cos(2.0 * M_PI * uu[3]);
                b[size_t(j)] = 2.0 * M_PI * uu[4];
            }
        rff_factor(pl, o.rank, w.data(), b.data(), f.Z.p, N, st);
    } else if (o.precond == ANOVA_PRECOND_NYSTROM) {
        f.rank = o.rank;
        f.Z.alloc(size_t(N) * o.rank);
        DevBuf<double> Gd, Y;
        Gd.alloc(size_t(N) * o.rank);
        Y.alloc(size_t(N) * o.rank);
        hipLaunchKernelGGL(k_gaussian, dim3(nblk(N), unsigned(o.rank)), dim3(kT), 0, st, Gd.p, N, o.rank, o.seed);
        enqueue_matvec(pl, Gd.p, o.rank, N, Y.p, N, st);
        nystrom_core(pl, Y, o.rank, f.Z.p, st);
    }
    if (o.factor_fp32 && f.rank > 0) {  // FP32 copy for the Woodbury products; the FP64 factor takes its values
        f.Z32.alloc(size_t(N) * f.rank);
        hipLaunchKernelGGL(k_narrow, dim3(nblk(N * f.rank)), dim3(kT), 0, st, f.Z.p, N * f.rank, f.Z32.p);
        ANV_HIP(hipGetLastError());
    }
    host_wait(st);
    f.t_setup_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
}

int ipm_solve(Plan& pl, const double* labels, double C, const anova_ipm_opts& o, double* alpha,
              double* lambda_out, anova_ipm_stats* stats, hipStream_t st, const LowRankFactor* factor,
              const MatvecHook* hook) {
    using clk = std::chrono::steady_clock;
    const auto t_start = clk::now();
    const int64_t N = pl.N;
    ANV_CHECK(labels && alpha && lambda_out, "NULL argument");
    ANV_CHECK(std::isfinite(C) && C > 0.0, "C must be > 0");
    ANV_CHECK(o.max_ip >= 1 && o.max_kry >= 1, "iteration caps must be >= 1");
    ANV_CHECK(o.sigma_bar > 0.0 && o.sigma_bar < 1.0, "sigma_bar must be in (0, 1)");
    ANV_CHECK(o.gamma0 > 0.0 && o.gamma0 < 1.0, "gamma0 must be in (0, 1)");
    ANV_CHECK(std::isfinite(o.mu0) && o.tol > 0.0 && o.tol_inf > 0.0 && o.tol_kry > 0.0,
              "tolerances must be > 0 and mu0 finite");
    ANV_CHECK(o.mu_rule == 0 || o.mu_rule == 1, "mu_rule must be 0 or 1");
    ANV_CHECK(o.krylov == ANOVA_KRYLOV_MINRES || o.krylov == ANOVA_KRYLOV_GMRES, "krylov must be MINRES or GMRES");
    ANV_CHECK(o.precond == ANOVA_PRECOND_NONE || o.precond == ANOVA_PRECOND_PCHOL ||
                  o.precond == ANOVA_PRECOND_NYSTROM || o.precond == ANOVA_PRECOND_DIAG ||
                  o.precond == ANOVA_PRECOND_RPCHOL || o.precond == ANOVA_PRECOND_RFF,
              "unknown preconditioner");
    ANV_CHECK(!low_rank_precond(o.precond) || (o.rank >= 1 && o.rank <= std::min<int64_t>(N, 1024)),
              "rank must be in [1, min(N, 1024)]");

    // labels: must be +-1 with both classes present
    std::vector<double> yh(N);
    ANV_HIP(hipMemcpyAsync(yh.data(), labels, N * sizeof(double), hipMemcpyDeviceToHost, st));
    host_wait(st);
    double ysum = 0.0;
    int64_t npos = 0;
    for (double v : yh) {
        ANV_CHECK(v == 1.0 || v == -1.0, "labels must be +1 or -1");
        ysum += v;
        npos += v > 0;
    }
    ANV_CHECK(npos > 0 && npos < N, "both classes must be present");

    // Krylov iterations: device scalars, host flags, and (direct path) graphs
    // replayed on a stream of the solve's own
    struct KryRes {
        hipStream_t caller = nullptr, own = nullptr;
        hipEvent_t fev[2] = {nullptr, nullptr};
        int* hflag = nullptr;  // done flags of two iterations, iteration count
        hipGraphExec_t g[6] = {};
        ~KryRes() {
            (void)hipStreamSynchronize(own ? own : caller);
            for (auto& x : g)
                if (x) (void)hipGraphExecDestroy(x);
            if (own) (void)hipStreamDestroy(own);
            for (auto e : fev)
                if (e) (void)hipEventDestroy(e);
            if (hflag) (void)hipHostFree(hflag);
        }
    } kr;
    kr.caller = st;
    const bool use_graphs = o.graphs != 0 && hook == nullptr && !pl.profiling;
    bool warmed = false;
    if (use_graphs) {
        ANV_HIP(hipStreamCreateWithFlags(&kr.own, hipStreamNonBlocking));
        hipEvent_t e = nullptr;
        ANV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        const hipError_t r1 = hipEventRecord(e, st);
        const hipError_t r2 = r1 == hipSuccess ? hipStreamWaitEvent(kr.own, e, 0) : r1;
        (void)hipEventDestroy(e);
        ANV_HIP(r2);
        st = kr.own;
    }
    ANV_HIP(hipHostMalloc(&kr.hflag, 4 * sizeof(int)));
    for (auto& e : kr.fev)
        ANV_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming | (t_blocking_waits ? hipEventBlockingSync : 0)));
    DevBuf<KryScal> ksd;
    ksd.alloc(1);

    Reducer red;
    Workspace ws;
    LowRankFactor own;
    if (factor) {
        ANV_CHECK(factor->precond == o.precond && (!low_rank_precond(o.precond) || factor->Z.n >= size_t(N) * factor->rank),
                  "shared factor does not match the preconditioner options or the plan");
    } else {
        build_low_rank(pl, o, own, st);
        factor = &own;
    }
    const int rank_used = factor->rank;
    ws.Z = factor->Z.p;
    ws.Z32 = (o.factor_fp32 && factor->Z32.n >= size_t(N) * factor->rank) ? factor->Z32.p : nullptr;
    setup_factor_storage(ws, N, low_rank_precond(o.precond) ? rank_used : 0);
    const double t_setup_ms = factor->t_setup_ms;

    // state
    DevBuf<double> ya, kya, th, rhs, sol, xk, rprev, rcur, zcur, zold, pv, d1, d2, ytmp;
    const int64_t n1 = N + 1;
    for (auto* b : {&ya, &kya, &th, &ytmp}) b->alloc(N);
    for (auto* b : {&rhs, &sol, &xk, &rprev, &rcur, &zcur, &zold, &pv, &d1, &d2}) b->alloc(n1);
    // initial point: alpha_i = C(2 + y_i)/4 if sum(y) >= 0 else C(2 - y_i)/4; lambda = 0
    {
        std::vector<double> a0(N);
        for (int64_t i = 0; i < N; ++i) a0[i] = (ysum >= 0.0) ? C * (2.0 + yh[i]) / 4.0 : C * (2.0 - yh[i]) / 4.0;
        ANV_HIP(hipMemcpyAsync(alpha, a0.data(), N * sizeof(double), hipMemcpyHostToDevice, st));
    }
    double lam = 0.0, mu = o.mu0;
    int matvecs = 0;

    // GMRES storage: the Arnoldi basis (mr + 1 columns), P^{-1} v, partial inner
    // products, device scalars and their pinned host mirror
    const bool gmres = o.krylov == ANOVA_KRYLOV_GMRES;
    const int mr = gmres ? std::min(kGmRestart, o.max_kry) : 0;  // restart length
    DevBuf<double> gV, gz, gpart, gd;
    const int64_t gldv = (n1 + 31) / 32 * 32;
    const unsigned gnb = unsigned((n1 + kT * kGmRows - 1) / (kT * kGmRows));
    double* gh = nullptr;
    if (gmres) {
        gV.alloc(size_t(mr + 1) * gldv);
        gz.alloc(N);
        gpart.alloc(size_t(gnb) * (mr + 1));
        gd.alloc(3 * size_t(mr + 1) + 2);
        ANV_HIP(hipHostMalloc(&gh, (3 * size_t(mr + 1) + 2) * sizeof(double)));
    }
    struct GhFree {
        double* p;
        ~GhFree() { if (p) (void)hipHostFree(p); }
    } gh_guard{gh};

    DevBuf<double> spart, sout;
    spart.alloc(size_t(kRedBlocks) * 5);
    sout.alloc(8);
    double* sh = nullptr;
    ANV_HIP(hipHostMalloc(&sh, 8 * sizeof(double)));
    struct HostFree {
        double* p;
        ~HostFree() { if (p) (void)hipHostFree(p); }
    } sh_guard{sh};
    // Declared after every buffer of the solve, so destroyed first: when an
    // exception leaves the solve, the stream's queued kernels and copies (which
    // read and write those buffers) finish before any of them is freed.
    struct SyncOnUnwind {
        hipStream_t s;
        ~SyncOnUnwind() {
            if (std::uncaught_exceptions() > 0) (void)hipStreamSynchronize(s);
        }
    } unwind_guard{st};
    const unsigned rb = red.blocks(N);

    auto eval_stats = [&](double& xa, double& xl, double& D, double& Pr, double& G) {
        hipLaunchKernelGGL(k_mul, dim3(nblk(N)), dim3(kT), 0, st, labels, alpha, N, ya.p);
        kmv(pl, hook, ya.p, kya.p, st);
        ++matvecs;
        hipLaunchKernelGGL(k_ipm_stats, dim3(rb), dim3(kT), 0, st, labels, alpha, kya.p, N, lam, mu, C, spart.p);
        hipLaunchKernelGGL(k_fold_partials, dim3(5), dim3(64), 0, st, spart.p, int(rb), 5, sout.p);
        ANV_HIP(hipMemcpyAsync(sh, sout.p, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
        host_wait(st);
        const double quad = sh[1];
        D = sh[0] - 0.5 * quad;
        Pr = 0.5 * quad + C * sh[2];
        G = (Pr - D) / (1.0 + std::fabs(Pr));
        xl = std::sqrt(sh[3]);
        xa = std::fabs(sh[4]);
    };

    if (!(o.mu0 > 0.0)) {
        // automatic start: the mean complementarity implied by the reduced
        // gradient at the starting point, never below the value 1 of Algorithm 1
        hipLaunchKernelGGL(k_mul, dim3(nblk(N)), dim3(kT), 0, st, labels, alpha, N, ya.p);
        kmv(pl, hook, ya.p, kya.p, st);
        ++matvecs;
        hipLaunchKernelGGL(k_compl_scale, dim3(nblk(N)), dim3(kT), 0, st, labels, alpha, kya.p, N, C, ytmp.p);
        hipLaunchKernelGGL(k_fill, dim3(nblk(N)), dim3(kT), 0, st, th.p, N, 1.0);
        mu = std::max(1.0, red.dot(ytmp.p, th.p, N, st) / double(N));
    }
    double xa0, xl0, D, Pr, G;
    eval_stats(xa0, xl0, D, Pr, G);
    double xa = xa0, xl = xl0;
    ANV_CHECK(xa0 > 0.0 && xl0 > 0.0, "initial infeasibilities vanish");
    int it = 0, kry_total = 0, kry_max = 0;
    int status = ANOVA_NOT_CONVERGED;
    double s_prev = 1.0;
    const double gap_stop = (pl.precision == ANOVA_PREC_FP64 ? kGapMargin : 1.0) * o.tol;
    for (;;) {
        if (!(std::isfinite(mu) && std::isfinite(G) && std::isfinite(xl))) {
            status = ANOVA_NUMERICAL;
            break;
        }
        // the gap is measured with the fast-summation kernel, which differs from
        // the exact one by the matvec error (~1e-7 relative for FP64 plans);
        // stopping at half the tolerance keeps the gap in the exact kernel below
        // it. Mixed-precision plans (matvec error ~5e-7, above the tolerance's
        // reach) stop at the tolerance itself.
        if (mu <= o.tol && xa / xa0 <= o.tol && xl / xl0 <= o.tol_inf && G <= gap_stop) {
            status = ANOVA_OK;
            break;
        }
        if (it >= o.max_ip) break;
        // Section 2: a constant reduction factor, or one that changes every iteration;
        // the default scales the reduction by the previous step length
        mu *= (o.mu_rule == 1) ? o.sigma_bar : 1.0 - (1.0 - o.sigma_bar) * s_prev;
        // never below the mu whose central point has a relative duality gap of
        // kMuFloor * tol (its gap is 2 N mu): a smaller mu changes nothing the stop
        // test can see, and the barrier weights of rows at a bound grow like 1/mu
        mu = std::max(mu, kMuFloor * o.tol * (1.0 + std::fabs(Pr)) / (2.0 * double(N)));
        hipLaunchKernelGGL(k_theta, dim3(nblk(N)), dim3(kT), 0, st, alpha, N, C, mu, th.p);
        const double r2 = red.dot(labels, alpha, N, st);
        hipLaunchKernelGGL(k_rhs, dim3(nblk(n1)), dim3(kT), 0, st, labels, alpha, kya.p, N, lam, mu, C, r2,
                           rhs.p);
        // preconditioner for this iteration: diag(A_hat, s), s = y^T A_hat^{-1} y
        double s_last = 1.0;
        const bool prec = o.precond != ANOVA_PRECOND_NONE;  // diag(A_hat, s); without a factor A_hat = Theta
        if (prec) {
            refresh_capacitance(ws, th.p, st);
            if (!gmres) {
                woodbury_apply(ws, labels, th.p, labels, nullptr, false, ytmp.p, st);
                s_last = red.dot(labels, ytmp.p, N, st);
                if (!(s_last > 0.0)) {
                    status = ANOVA_NUMERICAL;
                    break;
                }
            }
        }
        KryScal* ks = ksd.p;
        const double* inv_s = &ks->inv_s;  // device address
        auto precond = [&](const double* r, double* out) {
            if (prec)
                woodbury_apply(ws, labels, th.p, r, inv_s, true, out, st);
            else
                hipLaunchKernelGGL(k_copy, dim3(nblk(n1)), dim3(kT), 0, st, r, out, n1);
        };
        // ---- preconditioned MINRES on A sol = rhs (Lanczos in the M-inner product + Givens QR).
        // Own matvecs: the recurrence scalars stay on the device, the host learns
        // of convergence after the iteration or, past the first few, one iteration
        // late (an iteration that starts after convergence leaves the solution
        // untouched, so the result is that of a loop that stops at once), and
        // iterations are replayed from graphs.
        const double rtol = std::max(1e-10, std::min(o.tol_kry, 0.1 * G));
        const int kcap = prec ? o.max_kry : std::max<int64_t>(o.max_kry, 2 * n1);
        int kit = 0;
        if (gmres) {
            // ---- GMRES preconditioned from the right with the block-triangular
            // P = [[A_hat, 0], [-y^T, -1]] of Section 5 (P = I without a preconditioner),
            // restarted every mr steps. Arnoldi by classical Gram-Schmidt applied twice
            // (two passes of basis inner products, each one launch), least squares by
            // Givens rotations on the host; |g_{j+1}| is the residual ||rhs - A sol|| of
            // the iterate and is tested against rtol ||rhs||.
            const int64_t hn_at = 2 * int64_t(mr + 1), ytz_at = hn_at + 1, cf_at = hn_at + 2;
            double* const ytz_d = gd.p + ytz_at;
            const int tri = prec ? 1 : 0;
            // first N entries of P^{-1} v, and y^T of them to ytz_d
            auto pinv_head = [&](const double* v) -> const double* {
                const double* z = v;
                if (prec) {
                    woodbury_apply(ws, labels, th.p, v, nullptr, false, gz.p, st);
                    z = gz.p;
                }
                red.dot_dev(labels, z, N, ytz_d, st);
                return z;
            };
            std::vector<double> H(size_t(mr + 1) * mr), cs(mr), sn(mr), g(mr + 1), tv(mr);
            hipLaunchKernelGGL(k_fill, dim3(nblk(n1)), dim3(kT), 0, st, sol.p, n1, 0.0);
            const double beta0 = std::sqrt(std::max(0.0, red.dot(rhs.p, rhs.p, n1, st)));
            double beta = beta0;
            if (beta0 > 0.0) hipLaunchKernelGGL(k_copy, dim3(nblk(n1)), dim3(kT), 0, st, rhs.p, gV.p, n1);
            while (beta > rtol * beta0 && kit < kcap) {
                // one cycle from the residual in the basis' first column
                hipLaunchKernelGGL(k_scale, dim3(nblk(n1)), dim3(kT), 0, st, gV.p, n1, 1.0 / beta);
                std::fill(g.begin(), g.end(), 0.0);
                g[0] = beta;
                int jj = 0;
                double res = beta;
                while (jj < mr && kit < kcap) {
                    const double* vj = gV.p + jj * gldv;
                    double* w = gV.p + (jj + 1) * gldv;
                    const double* z = pinv_head(vj);
                    hipLaunchKernelGGL(k_mul, dim3(nblk(N)), dim3(kT), 0, st, labels, z, N, ws.tmp.p);
                    kmv(pl, hook, ws.tmp.p, ws.kyz.p, st);
                    ++matvecs;
                    hipLaunchKernelGGL(k_gm_op, dim3(nblk(n1)), dim3(kT), 0, st, labels, th.p, z, ws.kyz.p, N, ytz_d,
                                       vj, tri, w);
                    const int nc = jj + 1;
                    for (int pass = 0; pass < 2; ++pass) {
                        double* h = gd.p + pass * int64_t(mr + 1);
                        hipLaunchKernelGGL(k_gm_dots, dim3(gnb), dim3(kT), 0, st, gV.p, gldv, nc, w, n1, gpart.p);
                        hipLaunchKernelGGL(k_fold_partials, dim3(nc), dim3(64), 0, st, gpart.p, int(gnb), nc, h);
                        hipLaunchKernelGGL(k_gm_sub, dim3(nblk(n1)), dim3(kT), 0, st, gV.p, gldv, nc, h, 1, n1, w);
                    }
                    red.dot_dev(w, w, n1, gd.p + hn_at, st);
                    ANV_HIP(hipMemcpyAsync(gh, gd.p, (hn_at + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
                    host_wait(st);
                    double* hc = &H[size_t(jj) * (mr + 1)];
                    for (int i = 0; i < nc; ++i) hc[i] = gh[i] + gh[mr + 1 + i];
                    const double hn = std::sqrt(std::max(0.0, gh[hn_at]));
                    hc[nc] = hn;
                    if (hn > 0.0) hipLaunchKernelGGL(k_scale, dim3(nblk(n1)), dim3(kT), 0, st, w, n1, 1.0 / hn);
                    for (int i = 0; i < jj; ++i) {  // the earlier rotations on the new column
                        const double a = hc[i], b = hc[i + 1];
                        hc[i] = cs[i] * a + sn[i] * b;
                        hc[i + 1] = -sn[i] * a + cs[i] * b;
                    }
                    double rho = hypot_ieee(hc[jj], hc[jj + 1]);
                    if (rho == 0.0) rho = 1e-300;
                    cs[jj] = hc[jj] / rho;
                    sn[jj] = hc[jj + 1] / rho;
                    hc[jj] = rho;
                    hc[jj + 1] = 0.0;
                    g[jj + 1] = -sn[jj] * g[jj];
                    g[jj] = cs[jj] * g[jj];
                    ++jj;
                    ++kit;
                    res = std::fabs(g[jj]);
                    if (!(res > rtol * beta0) || !(hn > 0.0)) break;
                }
                // sol += P^{-1} V t, R t = g by back substitution (coefficients go
                // to the device negated: k_gm_sub subtracts)
                for (int i = jj - 1; i >= 0; --i) {
                    double acc = g[i];
                    for (int c = i + 1; c < jj; ++c) acc -= H[size_t(c) * (mr + 1) + i] * tv[c];
                    tv[i] = acc / H[size_t(i) * (mr + 1) + i];
                    gh[cf_at + i] = -tv[i];
                }
                ANV_HIP(hipMemcpyAsync(gd.p + cf_at, gh + cf_at, jj * sizeof(double), hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_gm_sub, dim3(nblk(n1)), dim3(kT), 0, st, gV.p, gldv, jj, gd.p + cf_at, 0, n1, pv.p);
                const double* zu = pinv_head(pv.p);
                hipLaunchKernelGGL(k_gm_fin, dim3(nblk(n1)), dim3(kT), 0, st, zu, ytz_d, pv.p, N, tri, sol.p);
                if (!(res > rtol * beta0) || kit >= kcap) break;
                // restart from the residual of the iterate
                hipLaunchKernelGGL(k_mul, dim3(nblk(N)), dim3(kT), 0, st, labels, sol.p, N, ws.tmp.p);
                kmv(pl, hook, ws.tmp.p, ws.kyz.p, st);
                ++matvecs;
                red.dot_dev(labels, sol.p, N, ytz_d, st);
                hipLaunchKernelGGL(k_gm_resid, dim3(nblk(n1)), dim3(kT), 0, st, labels, th.p, sol.p, ws.kyz.p, N,
                                   ytz_d, rhs.p, gV.p);
                beta = std::sqrt(std::max(0.0, red.dot(gV.p, gV.p, n1, st)));
            }
            host_wait(st);
        } else {
            hipLaunchKernelGGL(k_kry_start, dim3(1), dim3(1), 0, st, ks, rtol, s_last);
            hipLaunchKernelGGL(k_fill, dim3(nblk(n1)), dim3(kT), 0, st, sol.p, n1, 0.0);
            hipLaunchKernelGGL(k_fill, dim3(nblk(n1)), dim3(kT), 0, st, rprev.p, n1, 0.0);
            hipLaunchKernelGGL(k_fill, dim3(nblk(n1)), dim3(kT), 0, st, d1.p, n1, 0.0);
            hipLaunchKernelGGL(k_fill, dim3(nblk(n1)), dim3(kT), 0, st, d2.p, n1, 0.0);
            hipLaunchKernelGGL(k_copy, dim3(nblk(n1)), dim3(kT), 0, st, rhs.p, rcur.p, n1);
            precond(rcur.p, zcur.p);
            if (hook) {
                // matvecs through a hook (shared launches of a server or grid): the
                // host keeps the scalars and waits for each inner product
                double beta = std::sqrt(std::max(0.0, red.dot(rcur.p, zcur.p, n1, st)));
                const double beta1 = beta;
                double beta_prev = 0.0, c = -1.0, s = 0.0, dbar = 0.0, eps_next = 0.0, phibar = beta1;
                double* rp = rprev.p;
                double* rc = rcur.p;
                double* zc = zcur.p;
                double* zo = zold.p;
                double* pp = pv.p;
                if (beta1 > 0.0) {
                    while (kit < kcap) {
                        ++kit;
                        // p = A (z / beta) - (beta / beta_prev) r_prev
                        hipLaunchKernelGGL(k_mul, dim3(nblk(N)), dim3(kT), 0, st, labels, zc, N, ws.tmp.p);
                        kmv(pl, hook, ws.tmp.p, ws.kyz.p, st);
                        ++matvecs;
                        const double ytz = red.dot(labels, zc, N, st);
                        const double cprev = kit > 1 ? beta / beta_prev : 0.0;
                        hipLaunchKernelGGL(k_newton_out_v, dim3(nblk(n1)), dim3(kT), 0, st, labels, th.p, zc, ws.kyz.p, N,
                                           1.0 / beta, cprev, rp, -ytz, pp);
                        const double a = red.dot(zc, pp, n1, st) / beta;
                        hipLaunchKernelGGL(k_axpy, dim3(nblk(n1)), dim3(kT), 0, st, pp, rc, n1, -a / beta);
                        // rotate r_prev <- r_cur <- p; z_old <- z_cur; z_cur <- M^{-1} r_cur
                        std::swap(rp, rc);
                        std::swap(rc, pp);
                        std::swap(zo, zc);
                        precond(rc, zc);
                        beta_prev = beta;
                        beta = std::sqrt(std::max(0.0, red.dot(rc, zc, n1, st)));
                        const double eps_cur = eps_next;
                        const double delta = c * dbar + s * a;
                        const double gbar = s * dbar - c * a;
                        eps_next = s * beta;
                        dbar = -c * beta;
                        double gam = hypot_ieee(gbar, beta);
                        if (gam == 0.0) gam = 1e-300;
                        c = gbar / gam;
                        s = beta / gam;
                        const double phi = c * phibar;
                        phibar = s * phibar;
                        hipLaunchKernelGGL(k_minres_update_v, dim3(nblk(n1)), dim3(kT), 0, st, zo, n1, 1.0 / beta_prev,
                                           eps_cur, delta, 1.0 / gam, phi, d1.p, d2.p, sol.p);
                        if (!(phibar > rtol * beta1) || !(beta > 0.0)) break;
                    }
                }
            } else {
                red.dot_dev(rcur.p, zcur.p, n1, &ks->dot_rz, st);
                hipLaunchKernelGGL(k_kry_beta1, dim3(1), dim3(1), 0, st, ks);
                // iteration j starts with r_prev, r, p = Rb[j], Rb[j + 1], Rb[j + 2] (mod 3) and
                // z, z_old = Zb[j], Zb[j + 1] (mod 2): the buffers rotate with period 6
                double* const Rb[3] = {rprev.p, rcur.p, pv.p};
                double* const Zb[2] = {zcur.p, zold.p};
                auto iteration = [&](int j) {
                    double* rp = Rb[j % 3];
                    double* rc = Rb[(j + 1) % 3];
                    double* pp = Rb[(j + 2) % 3];
                    double* zc = Zb[j % 2];
                    double* zo = Zb[(j + 1) % 2];
                    // p = A (z / beta) - (beta / beta_prev) r_prev; p -= (z^T p / beta^2) r
                    hipLaunchKernelGGL(k_mul, dim3(nblk(N)), dim3(kT), 0, st, labels, zc, N, ws.tmp.p);
                    red.dot_dev(labels, zc, N, &ks->dot_ytz, st);
                    kmv(pl, hook, ws.tmp.p, ws.kyz.p, st);
                    hipLaunchKernelGGL(k_newton_out, dim3(nblk(n1)), dim3(kT), 0, st, labels, th.p, zc, ws.kyz.p, N, ks, rp,
                                       pp);
                    red.dot_dev(zc, pp, n1, &ks->dot_a, st);
                    hipLaunchKernelGGL(k_kry_axpy, dim3(nblk(n1)), dim3(kT), 0, st, pp, rc, n1, ks);
                    // p becomes the residual r; its preconditioned form goes to z_old's buffer
                    precond(pp, zo);
                    red.dot_dev(pp, zo, n1, &ks->dot_rz, st);
                    hipLaunchKernelGGL(k_kry_scalars, dim3(1), dim3(1), 0, st, ks);
                    hipLaunchKernelGGL(k_minres_update, dim3(nblk(n1)), dim3(kT), 0, st, zc, n1, ks, d1.p, d2.p, sol.p);
                };
                for (int j = 0; j < kcap; ++j) {
                    const int state = j % 6;
                    if (use_graphs && warmed) {
                        if (!kr.g[state]) {
                            // capture once per solve: every kernel argument is fixed for the solve
                            hipGraph_t g = nullptr;
                            ANV_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                            try {
                                iteration(state);
                            } catch (...) {
                                hipGraph_t tmp = nullptr;
                                (void)hipStreamEndCapture(st, &tmp);
                                if (tmp) (void)hipGraphDestroy(tmp);
                                throw;
                            }
                            ANV_HIP(hipStreamEndCapture(st, &g));
                            const hipError_t e = hipGraphInstantiate(&kr.g[state], g, nullptr, nullptr, 0);
                            (void)hipGraphDestroy(g);
                            ANV_HIP(e);
                        }
                        ANV_HIP(hipGraphLaunch(kr.g[state], st));
                    } else {
                        iteration(j);
                        warmed = true;
                    }
                    ++matvecs;
                    // the iteration's done flag, in stream order, to the host
                    ANV_HIP(hipMemcpyAsync(kr.hflag + (j & 1), &ks->done, sizeof(int), hipMemcpyDeviceToHost, st));
                    ANV_HIP(hipEventRecord(kr.fev[j & 1], st));
                    // the first iterations are checked at once (a well-preconditioned
                    // solve takes only a few); later ones one iteration late, so that
                    // the GPU always has the next iteration queued
                    if (j < kEagerChecks) {
                        ANV_HIP(hipEventSynchronize(kr.fev[j & 1]));
                        if (kr.hflag[j & 1]) break;
                    } else {
                        ANV_HIP(hipEventSynchronize(kr.fev[(j - 1) & 1]));
                        if (kr.hflag[(j - 1) & 1]) break;
                    }
                }
                ANV_HIP(hipMemcpyAsync(kr.hflag + 2, &ks->kit, sizeof(int), hipMemcpyDeviceToHost, st));
                host_wait(st);
                kit = kr.hflag[2];
            }
        }
        kry_total += kit;
        kry_max = std::max(kry_max, kit);
        // ---- step to the boundary (Algorithm 1): s = gamma0 * min(1, s_max), same for lambda
        hipLaunchKernelGGL(k_step_partial, dim3(rb), dim3(kT), 0, st, alpha, sol.p, N, C, spart.p);
        hipLaunchKernelGGL(k_min_final, dim3(1), dim3(64), 0, st, spart.p, int(rb), sout.p);
        ANV_HIP(hipMemcpyAsync(sh + 5, sout.p, sizeof(double), hipMemcpyDeviceToHost, st));
        ANV_HIP(hipMemcpyAsync(sh + 6, sol.p + N, sizeof(double), hipMemcpyDeviceToHost, st));
        host_wait(st);
        const double smax_dl[2] = {sh[5], sh[6]};
        const double step = o.gamma0 * std::min(1.0, smax_dl[0]);
        s_prev = step;
        hipLaunchKernelGGL(k_step, dim3(nblk(N)), dim3(kT), 0, st, alpha, sol.p, N, step);
        lam += step * smax_dl[1];
        ++it;
        eval_stats(xa, xl, D, Pr, G);
    }
    host_wait(st);
    *lambda_out = lam;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->ip_iters = it;
        stats->kry_iters_total = kry_total;
        stats->kry_iters_max = kry_max;
        stats->rank_used = rank_used;
        stats->status = status;
        stats->matvecs = matvecs;
        stats->mu = mu;
        stats->rel_gap = G;
        stats->dual_obj = D;
        stats->primal_obj = Pr;
        stats->xi_alpha_rel = xa / xa0;
        stats->xi_lambda_rel = xl / xl0;
        stats->t_setup_ms = t_setup_ms;
        stats->t_solve_ms = std::chrono::duration<double, std::milli>(clk::now() - t_start).count();
    }
    if (status == ANOVA_NUMERICAL) throw Error(ANOVA_NUMERICAL, "IPM produced NaN/Inf or lost positive definiteness");
    if (status == ANOVA_NOT_CONVERGED) set_last_error("IPM iteration cap reached");
    return status;
}

// ------------------------------------------------------------------ decision function
namespace {
// x = [y * alpha ; 0]
__global__ void k_pad_coeffs(const double* __restrict__ y, const double* __restrict__ a, int64_t N, int64_t M,
                             double* __restrict__ x) {
    const int64_t i = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (i < N) x[i] = y[i] * a[i];
    else if (i < N + M) x[i] = 0.0;
}
// f_j = (K x)_{N + j} - lambda
__global__ void k_take_shift(const double* __restrict__ ye, int64_t N, int64_t M, double lam, double* __restrict__ f) {
    const int64_t j = blockIdx.x * int64_t(kT) + threadIdx.x;
    if (j < M) f[j] = ye[N + j] - lam;
}
}  // namespace

void decision_function(const double* X, int64_t N, int64_t ldx, const double* Xnew, int64_t M, int64_t ldn,
                       int32_t d, const int32_t* windows, int32_t P, const double* sigma, const double* eta,
                       const anova_opts* opts, const double* labels, const double* alpha, double lambda, double* f,
                       hipStream_t st) {
    ANV_CHECK(X && Xnew && labels && alpha && f, "NULL argument");
    ANV_CHECK(N >= 1 && M >= 1 && d >= 1, "need N >= 1, M >= 1, d >= 1");
    ANV_CHECK(ldx >= d && ldn >= d, "leading dimension < d");
    ANV_CHECK(std::isfinite(lambda), "lambda must be finite");
    const int64_t T = N + M;
    DevBuf<double> U, xe, ye;
    U.alloc(size_t(T) * d);
    ANV_HIP(hipMemcpy2DAsync(U.p, d * sizeof(double), X, ldx * sizeof(double), d * sizeof(double), N,
                             hipMemcpyDeviceToDevice, st));
    ANV_HIP(hipMemcpy2DAsync(U.p + N * d, d * sizeof(double), Xnew, ldn * sizeof(double), d * sizeof(double), M,
                             hipMemcpyDeviceToDevice, st));
    std::unique_ptr<Plan> pl(create_plan(U.p, T, d, d, windows, P, sigma, eta, opts, st));
    xe.alloc(T);
    ye.alloc(T);
    hipLaunchKernelGGL(k_pad_coeffs, dim3(nblk(T)), dim3(kT), 0, st, labels, alpha, N, M, xe.p);
    enqueue_matvec(*pl, xe.p, 1, T, ye.p, T, st);
    hipLaunchKernelGGL(k_take_shift, dim3(nblk(M)), dim3(kT), 0, st, ye.p, N, M, lambda, f);
    ANV_HIP(hipGetLastError());
    host_wait(st);
}

}  // namespace anv
