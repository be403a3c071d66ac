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

// refinement step: per-component scales of the gradient step over
// (x(3), q(4), v(3), w(3), m, mu) and the clamp ranges of m and mu
struct RefineArgs {
    float scale[15];
    float m_lo, m_hi, mu_lo, mu_hi;
};

// populations up to this size rank their groups in the last workgroup of the
// cost or window kernel instead of a launch of their own
constexpr int FUSED_ARGMIN_MAX = 4096;

// capacity of a simulation's LDS candidate list (entries of gap + key): a
// step that finds more cuts its list to the C_max lowest when it fills up
// and keeps only candidates below the last kept one, so the LDS per
// simulation stays within ~16-29 KiB whatever S_max and L are
constexpr int CAND_CAP = 1536;

// step statistics (steps, candidates, contacts, dropped) are accumulated in
// STATS_SLOTS slots one 128-byte line apart, a wavefront adding to slot
// (its index mod STATS_SLOTS): the atomics of a launch spread over many
// lines instead of queueing on one; the totals are the slots' sums
constexpr int STATS_SLOTS = 256;
constexpr int STATS_STRIDE = 16;   // int64 per slot

// rows of a window start: x(3) q(4) v(3) w(3) m mu f(3)
constexpr int XI_ROWS = 18;

// elites kept per group of n simulations: max(1, floor(n elite_frac)), at most n
__host__ __device__ inline int elite_count(int n, float elite_frac)
{
    int kb = (int)floorf((float)n * elite_frac);
    return kb < 1 ? 1 : (kb > n ? n : kb);
}

// slots of one group's sort: the next power of two
__host__ __device__ constexpr int sort_slots(int n)
{
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

// threads of a per-group workgroup (sort, resample, elites): one per
// simulation of the largest group, in whole wavefronts, 64 to 1024
constexpr int group_threads(int max_group)
{
    return max_group >= 1024 ? 1024 : (max_group <= 64 ? 64 : (max_group + 63) / 64 * 64);
}

// LDS of one group's sort: costs and indices over sort_slots(max_group)
__host__ __device__ constexpr size_t resample_lds_bytes(int max_group)
{
    return (size_t)8 * (size_t)sort_slots(max_group);
}

// bytes of LDS per wavefront: candidate (d, key) list, selected keys,
// previous warm keys and impulses, contact staging for the observation, the
// step's L hand segment records (L = 0 for the window kernels, which read
// them from HBM)
__host__ __device__ constexpr size_t wave_lds_bytes(int max_cand, int L)
{
    return (size_t)8 * max_cand + 4 * 64 + 4 * 64 + 12 * 64 + 16 * 64 + (size_t)64 * L;
}

// the selected keys, warm-cache lookup and contact stage after the
// candidate list: nothing reads them between the warm start and the end of
// a step's solve, so the solve's sum rows may run on into them
constexpr int WAVE_SPARE_BYTES = 4 * 64 + 4 * 64 + 12 * 64 + 16 * 64;

}  // namespace pt

// Lets kernel f take dynamic LDS up to `bytes` of workgroup LDS less its own
// static LDS.
inline hipError_t set_dynamic_lds_limit(const void *f, size_t bytes)
{
    hipFuncAttributes a;
    hipError_t e = hipFuncGetAttributes(&a, f);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(bytes - a.sharedSizeBytes));
}

hipError_t launch_hand_fk(const float *hand, int L, int D, float dt, const float *u_prev, const float *u,
                          int stride, int nsteps, float *seg_out, hipStream_t s);
// seg_in: the step's segments are already in seg_out (k_hand_fk), for the
// float64 solve; otherwise every wavefront evaluates them
hipError_t launch_step(const pt::Consts &P, const pt::Tables &tb, const float *u_prev, const float *u, float *state,
                       float *params, float *warm, float *contacts, float *cslip, float *seg_out, int64_t *stats,
                       int waves_per_block, bool seg_in, hipStream_t s);
size_t hand_fk_lds_bytes(int L, int D);
hipError_t launch_observe(const pt::Consts &P, const float *contacts, const float *cslip, const float *seg, float *obs,
                          hipStream_t s);
hipError_t launch_cost(const pt::Consts &P, const int32_t *group_of, const int32_t *group_start, const float *obs,
                       const float *obs_gt, float *cost_sum, int32_t *best, int32_t *done, hipStream_t s);
hipError_t launch_argmin(int G, const int32_t *group_start, const float *cost, int32_t *best, hipStream_t s);
hipError_t launch_resample(const pt::Consts &P, const pt::ResampleArgs &R, const int32_t *group_start, int max_group,
                           uint32_t window_idx, float *cost_sum, float *state, float *params, float *warm,
                           int32_t *parent, hipStream_t s);
hipError_t launch_window(const pt::Consts &P, const pt::Tables &tb, const float *seg_win, float *state, float *params,
                         float *warm, const float *obs_gt_win, float *cost_sum, float *obs_out,
                         const int32_t *env_order, int32_t *queue, int64_t *stats, int waves_per_block, int blocks,
                         float *ckpt, const int32_t *group_start, int32_t *best, hipStream_t s);
hipError_t window_occupancy(const pt::Consts &P, int waves_per_block, int *blocks_per_cu);
hipError_t set_lds_limits(size_t bytes);
hipError_t set_grad_lds_limits(size_t bytes);
size_t ckpt_floats(const pt::Consts &P, int n);
hipError_t launch_window_fwd(const pt::Consts &P, const pt::Tables &tb, const float *seg_win, int n, int i0,
                             int count, const int32_t *env, const float *xi, const float *warm0,
                             const float *obs_gt_win, float *cost, float *end_state, float *end_warm, float *ckpt,
                             hipStream_t s, float *resid = nullptr);
hipError_t launch_window_bwd(const pt::Consts &P, const pt::Tables &tb, const float *seg_win, int n, int i0,
                             int count, const int32_t *env, const float *xi, const float *obs_gt_win,
                             const float *ckpt, bool ckpt_by_env, const int32_t *flag, float *grad,
                             hipStream_t s);
hipError_t launch_select_elites(int G, int max_group, float elite_frac, const int32_t *group_start,
                                const float *cost_sum, int32_t *elite_env, hipStream_t s);
hipError_t launch_refine_gather(int n, int K, int C_max, const int32_t *env, const float *state, const float *params,
                                const float *warm, const float *cost_sum, float *xi, float *warm0, float *cost,
                                float *rho, float rho0, hipStream_t s);
hipError_t launch_refine_propose(int n, int i0, int count, const pt::RefineArgs &A, const float *xi,
                                 const float *grad, const float *rho, float *xi_try, hipStream_t s);
hipError_t launch_refine_accept(int n, int i0, int count, int K, int C_max, const int32_t *env, float *cost_cur,
                                const float *cost_try, float *xi, const float *xi_try, float *rho, int32_t *flag,
                                const float *end_state, const float *end_warm, float *state, float *params,
                                float *warm, float *cost_sum, hipStream_t s);
hipError_t launch_weighted_resample(const pt::Consts &P, const pt::ResampleArgs &R, int kind, float hyper,
                                    const int32_t *group_start, int max_group, int n_steps, uint32_t window_idx,
                                    float *cost_sum, float *state, float *params, float *warm, float *snap,
                                    int32_t *parent, float *weights, float *eta, hipStream_t s);
hipError_t set_draw_lds_limits(size_t bytes);

// the PD-controlled hand (pt_pd.hip)
namespace pt {
struct PdConsts;
}
hipError_t set_pd_lds_limits(size_t bytes);
hipError_t launch_step_pd(const pt::Consts &P, const pt::PdConsts &Q, const pt::Tables &tb, const int32_t *pd_tab,
                          const float *u, float *state, float *params, float *warm, float *hstate, float *contacts,
                          int64_t *stats, hipStream_t s);
hipError_t launch_window_pd(const pt::Consts &P, const pt::PdConsts &Q, const pt::Tables &tb, const int32_t *pd_tab,
                            const float *u_win, float *state, float *params, float *warm, float *hstate,
                            const float *obs_gt_win, float *cost_sum, float *obs_out, int64_t *stats, hipStream_t s);
hipError_t launch_observe_pd(const pt::Consts &P, const float *contacts, const float *hstate, float *obs,
                             hipStream_t s);
hipError_t launch_cost_pd(const pt::Consts &P, const pt::PdConsts &Q, const int32_t *group_of, const float *obs,
                          const float *obs_gt, float *cost_sum, hipStream_t s);
hipError_t launch_copy_hand(int K, int rows, const int32_t *parent, float *hstate, hipStream_t s);
