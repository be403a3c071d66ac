// pt_resample.hip -- the two optimisers that resample with replacement
// (Sec. III-D.1 WRS, Eq. 4; Sec. III-D.2 REPS, Eqs. 5-6) for gfx950.
//
//   k_weighted_draw   one workgroup per group: window-mean costs, the
//                     temperature (fixed for WRS; REPS: bisection on the
//                     dual's optimality condition), the weights, their
//                     running sum in LDS and one categorical draw per
//                     simulation (Philox counter (j, window, 3, 0))
//   k_gather          snapshot of every simulation's parent (state, params,
//                     warm cache), all simulations in parallel
//   k_apply           copy back from the snapshot, explore every simulation
//                     and clear its running cost
//
// The snapshot makes the copies independent of the order the simulations
// are written in: a parent may itself be replaced in the same call.
#include "pt_internal.h"
#include "pt_io.hpp"

namespace pt {

constexpr int DRAW_THREADS = 1024;
constexpr int DRAW_WAVES = DRAW_THREADS / WAVE;
constexpr int REPS_BISECTIONS = 48;     // log(eta) bracket of width 60 -> 2e-13

// block-wide sums and extrema of doubles (every thread gets the result)
struct DrawLds {
    double red[2][DRAW_WAVES * 2];
    int ired[DRAW_WAVES * 2];
};

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// sums of (a, b) over the block; `phase` alternates the LDS slot so that
// consecutive calls need one barrier each
__device__ __forceinline__ void block_sum2(double &a, double &b, DrawLds &L, int phase)
{
    const int w = threadIdx.x / WAVE;
    a = wave_sum_d(a);
    b = wave_sum_d(b);
    double *r = L.red[phase & 1];
    if (lane_id() == 0) { r[2 * w] = a; r[2 * w + 1] = b; }
    __syncthreads();
    a = 0.0; b = 0.0;
    for (int k = 0; k < DRAW_WAVES; ++k) { a += r[2 * k]; b += r[2 * k + 1]; }
}

__device__ __forceinline__ void block_minmax(double &lo, double &hi, DrawLds &L)
{
    const int w = threadIdx.x / WAVE;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off));
        hi = fmax(hi, __shfl_xor(hi, off));
    }
    __syncthreads();
    if (lane_id() == 0) { L.red[0][2 * w] = lo; L.red[0][2 * w + 1] = hi; }
    __syncthreads();
    for (int k = 0; k < DRAW_WAVES; ++k) { lo = fmin(lo, L.red[0][2 * k]); hi = fmax(hi, L.red[0][2 * k + 1]); }
    __syncthreads();
}

__device__ __forceinline__ void block_isum2(int &a, int &b, DrawLds &L)
{
    const int w = threadIdx.x / WAVE;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b = max(b, __shfl_xor(b, off));
    }
    __syncthreads();
    if (lane_id() == 0) { L.ired[2 * w] = a; L.ired[2 * w + 1] = b; }
    __syncthreads();
    a = 0; int m = -1;
    for (int k = 0; k < DRAW_WAVES; ++k) { a += L.ired[2 * k]; m = max(m, L.ired[2 * k + 1]); }
    b = m;
    __syncthreads();
}

// kind 0: WRS with lambda = hyper; kind 1: REPS with KL bound eps = hyper.
// Reads cost_sum (the window's running sums over n_steps steps), writes
// parent (global index of the drawn simulation), optionally the group's
// weights (they sum to 1 over the group) and REPS's eta* (0: the limit
// eta -> 0+, uniform over the lowest costs; +inf: all finite costs equal,
// or none finite).
__global__ __launch_bounds__(DRAW_THREADS) void k_weighted_draw(int kind, float hyper, const int32_t *__restrict__ group_start,
                                                                const float *__restrict__ cost_sum, int n_steps,
                                                                uint32_t window_idx, uint64_t seed,
                                                                float *__restrict__ weights, float *__restrict__ eta_out,
                                                                int32_t *__restrict__ parent)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ DrawLds L;
    double *cdf = reinterpret_cast<double *>(smem);
    const int g = blockIdx.x;
    const int lo = group_start[g], hi = group_start[g + 1];
    const int n = hi - lo;
    if (n <= 0) return;
    const int ch = (n + DRAW_THREADS - 1) / DRAW_THREADS;
    const int i0 = threadIdx.x * ch;
    const double inv_steps = 1.0 / (double)n_steps;

    // window means of this thread's contiguous chunk, kept in the LDS array
    // that later holds the running sum of the weights (each thread reads its
    // own entries before it overwrites them); NaN and inf are not finite
    // costs (weight 0)
    double cmin = __longlong_as_double(0x7ff0000000000000ll), cmax = -cmin;
    const int i1 = min(i0 + ch, n);
    for (int i = i0; i < i1; ++i) {
        const double ci = (double)cost_sum[lo + i] * inv_steps;
        cdf[i] = ci;
        if (isfinite(ci)) {
            cmin = fmin(cmin, ci);
            cmax = fmax(cmax, ci);
        }
    }
    block_minmax(cmin, cmax, L);
    int nf = 0, nmin = 0;
    for (int i = i0; i < i1; ++i) {
        const double ci = cdf[i];
        if (isfinite(ci)) { ++nf; nmin += ci == cmin ? 1 : 0; }
    }
    {
        int a = nf, b = -1;
        block_isum2(a, b, L);
        nf = a;
        int m = nmin, d = -1;
        block_isum2(m, d, L);
        nmin = m;
    }

    // temperature: weights exp(-lam (c - cmin)) on finite costs, or one of
    // the uniform cases
    enum { WEIGHTED, UNIFORM_ALL, UNIFORM_FINITE, UNIFORM_MIN };
    int mode = WEIGHTED;
    double lam = (double)hyper, eta = 0.0;
    if (nf == 0) {
        mode = UNIFORM_ALL;
        eta = __longlong_as_double(0x7ff0000000000000ll);
    } else if (kind == 1) {
        const double eps = (double)hyper;
        const double spread = cmax - cmin;
        if (spread == 0.0) {
            mode = UNIFORM_FINITE;
            eta = __longlong_as_double(0x7ff0000000000000ll);
        } else if (eps >= log((double)nf / (double)nmin)) {
            mode = UNIFORM_MIN;
            eta = 0.0;
        } else {
            // KL(P_eta || uniform) = log nf - log Z - S1 / (eta Z), with
            // Z = sum exp(-(c - cmin) / eta), S1 = sum (c - cmin) exp(...);
            // it falls as eta grows, and the dual's minimiser is where it
            // equals eps (below spread / eps, where KL <= spread / eta <= eps)
            double thi = log(spread / eps), tlo = thi - 60.0;
            for (int it = 0; it < REPS_BISECTIONS; ++it) {
                const double tm = 0.5 * (tlo + thi);
                const double ie = exp(-tm);
                double z = 0.0, s1 = 0.0;
                for (int i = i0; i < i1; ++i) {
                    const double ci = cdf[i];
                    if (isfinite(ci)) {
                        const double d = ci - cmin;
                        const double x = exp(-d * ie);
                        z += x;
                        s1 += d * x;
                    }
                }
                block_sum2(z, s1, L, it);
                const double kl = log((double)nf) - log(z) - s1 * ie / z;
                if (kl > eps) tlo = tm; else thi = tm;
            }
            eta = exp(0.5 * (tlo + thi));
            lam = 1.0 / eta;
        }
    }

    // weights of the chunk and their running sum (inclusive) through the
    // block: chunk sums scanned over the threads (the weights are formed
    // twice, for the chunk sum and for the running sum)
    auto weight = [&](double ci) -> double {
        if (mode == UNIFORM_ALL) return 1.0;
        if (!isfinite(ci)) return 0.0;
        if (mode == UNIFORM_FINITE) return 1.0;
        if (mode == UNIFORM_MIN) return ci == cmin ? 1.0 : 0.0;
        return exp(-lam * (ci - cmin));
    };
    double tsum = 0.0;
    int last = -1;
    for (int i = i0; i < i1; ++i) {
        const double wi = weight(cdf[i]);
        if (wi > 0.0) last = i;
        tsum += wi;
    }
    // exclusive scan of the thread sums: inclusive within the wave by
    // shuffles, wave totals through LDS
    const int lane = lane_id(), wv = threadIdx.x / WAVE;
    double incl = tsum;
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const double y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    __syncthreads();
    if (lane == WAVE - 1) L.red[0][wv] = incl;
    __syncthreads();
    double base = 0.0, total = 0.0;
    for (int k = 0; k < DRAW_WAVES; ++k) {
        const double t = L.red[0][k];
        if (k < wv) base += t;
        total += t;
    }
    double run = base + (incl - tsum);
    for (int i = i0; i < i1; ++i) {
        const double wi = weight(cdf[i]);
        run += wi;
        cdf[i] = run;
        if (weights) weights[lo + i] = (float)(wi / total);
    }
    {
        int a = 0, b = last;
        block_isum2(a, b, L);
        last = b;
    }
    if (eta_out && threadIdx.x == 0) eta_out[g] = kind == 1 ? (float)eta : 0.f;
    __syncthreads();

    // one draw per simulation: the first index whose running sum exceeds
    // u * total, u = (w0 + 1/2) 2^-32
    const uint32_t key0 = (uint32_t)(seed & 0xffffffffu), key1 = (uint32_t)(seed >> 32);
    for (int i = threadIdx.x; i < n; i += DRAW_THREADS) {
        const int j = lo + i;
        uint32_t r[4];
        philox4x32_10((uint32_t)j, window_idx, 3u, 0u, key0, key1, r);
        const double t = ((double)r[0] + 0.5) * 2.3283064365386963e-10 * total;
        int a = 0, b = n;                    // first index in [a, b) with cdf > t
        while (a < b) {
            const int m = (a + b) >> 1;
            if (cdf[m] > t) b = m; else a = m + 1;
        }
        parent[j] = lo + (a < last ? a : last);
    }
}

// snapshot rows: state (13), params (5) as [18][K], then the warm cache
// [K][C_max][4]
__global__ __launch_bounds__(256) void k_gather(int K, int C_max, const int32_t *__restrict__ parent,
                                                const float *__restrict__ state, const float *__restrict__ params,
                                                const float *__restrict__ warm, float *__restrict__ snap)
{
    const size_t rows = (size_t)18 * K;
    const size_t warm4 = (size_t)K * C_max;
    const size_t total = rows + warm4;
    float4 *sw = reinterpret_cast<float4 *>(snap + rows);
    const float4 *ww = reinterpret_cast<const float4 *>(warm);
    for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (size_t)gridDim.x * blockDim.x) {
        if (x < rows) {
            const int r = (int)(x / K), j = (int)(x - (size_t)r * K);
            const int p = parent[j];
            snap[x] = r < 13 ? state[(size_t)r * K + p] : params[(size_t)(r - 13) * K + p];
        } else {
            const size_t y = x - rows;
            const int j = (int)(y / C_max), c = (int)(y - (size_t)j * C_max);
            sw[y] = ww[(size_t)parent[j] * C_max + c];
        }
    }
}

__global__ __launch_bounds__(256) void k_apply(int K, int C_max, ResampleArgs R, uint32_t window_idx,
                                               const float *__restrict__ snap, float *__restrict__ state,
                                               float *__restrict__ params, float *__restrict__ warm,
                                               float *__restrict__ cost_sum)
{
    const size_t rows = (size_t)18 * K;
    const size_t warm4 = (size_t)K * C_max;
    const size_t total = (size_t)13 * K + warm4 + K;
    const float4 *sw = reinterpret_cast<const float4 *>(snap + rows);
    float4 *ww = reinterpret_cast<float4 *>(warm);
    for (size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (size_t)gridDim.x * blockDim.x) {
        if (x < (size_t)13 * K) {
            state[x] = snap[x];
        } else if (x < (size_t)13 * K + warm4) {
            const size_t y = x - (size_t)13 * K;
            ww[y] = sw[y];
        } else {
            const int j = (int)(x - (size_t)13 * K - warm4);
            float e[5];
            explore(R, (uint32_t)j, window_idx, snap[(size_t)13 * K + j], snap[(size_t)14 * K + j], e);
            for (int c = 0; c < 5; ++c) params[(size_t)c * K + j] = e[c];
            cost_sum[j] = 0.f;
        }
    }
}

}  // namespace pt

using namespace pt;

size_t weighted_draw_lds_bytes(int max_group) { return (size_t)8 * (size_t)max_group; }

hipError_t launch_weighted_resample(const Consts &P, const ResampleArgs &R, int kind, float hyper,
                                    const int32_t *group_start, int max_group, int n_steps, uint32_t window_idx,
                                    float *cost_sum, float *state, float *params, float *warm, float *snap,
                                    int32_t *parent, float *weights, float *eta, hipStream_t s)
{
    hipLaunchKernelGGL(k_weighted_draw, dim3(P.G), dim3(DRAW_THREADS), weighted_draw_lds_bytes(max_group), s, kind,
                       hyper, group_start, cost_sum, n_steps, window_idx, R.seed, weights, eta, parent);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t total = (size_t)18 * P.K + (size_t)P.K * P.C_max;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(256), 0, s, P.K, P.C_max, parent, state, params, warm, snap);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_apply, dim3(blocks), dim3(256), 0, s, P.K, P.C_max, R, window_idx, snap, state, params,
                       warm, cost_sum);
    return hipGetLastError();
}

hipError_t set_draw_lds_limits(size_t bytes)
{
    return set_dynamic_lds_limit(reinterpret_cast<const void *>(k_weighted_draw), bytes);
}
