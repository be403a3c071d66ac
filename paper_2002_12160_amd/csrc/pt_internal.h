// pt_internal.h -- declarations shared by the kernels and the host API of
// libpt (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pt_device.hpp"
#include "pt_step.hpp"

namespace pt {

constexpr int HAND_STRIDE = 20;
constexpr int MAX_LINKS = 62;

struct ResampleArgs {
    float elite_frac, sigma_mu, sigma_m, sigma_f, mu_lo, mu_hi, m_lo, m_hi;
    uint64_t seed;
};

// bytes of LDS per wavefront: candidate (d, key) list, selected keys,
// previous warm keys and impulses, contact staging for the observation
__host__ __device__ constexpr size_t wave_lds_bytes(int max_cand)
{
    return (size_t)8 * max_cand + 4 * 64 + 4 * 64 + 12 * 64 + 16 * 64;
}

}  // namespace pt

hipError_t launch_hand_fk(const float *hand, int L, float dt, const float *u_prev, const float *u, int stride,
                          int nsteps, float *seg_out, hipStream_t s);
hipError_t launch_step(const pt::Consts &P, const pt::Tables &tb, const float *seg, float *state, float *params,
                       float *warm, float *contacts, int64_t *stats, int waves_per_block, hipStream_t s);
hipError_t launch_observe(const pt::Consts &P, const float *contacts, float *obs, hipStream_t s);
hipError_t launch_cost(const pt::Consts &P, const int32_t *group_of, const float *obs, const float *obs_gt,
                       float *cost_sum, hipStream_t s);
hipError_t launch_argmin(int G, const int32_t *group_start, const float *cost, int32_t *best, hipStream_t s);
hipError_t launch_resample(const pt::Consts &P, const pt::ResampleArgs &R, const int32_t *group_start, int max_group,
                           uint32_t window_idx, float *cost_sum, float *state, float *params, float *warm,
                           int32_t *parent, hipStream_t s);
hipError_t launch_reset_queue(int32_t *q, hipStream_t s);
hipError_t launch_window(const pt::Consts &P, const pt::Tables &tb, const float *seg_win, float *state, float *params,
                         float *warm, const float *obs_gt_win, float *cost_sum, float *obs_out,
                         const int32_t *env_order, int32_t *queue, int64_t *stats, int waves_per_block, int blocks,
                         hipStream_t s);
hipError_t window_occupancy(int waves_per_block, int max_cand, bool fp64, int *blocks_per_cu);
hipError_t set_lds_limits(size_t bytes);
