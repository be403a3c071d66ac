// pt_pd.hip -- kernels of the PD-controlled hand (hand_mode 1) for CDNA4
// (gfx950): the per-step path of the kinematic hand with the joint angles
// and rates as per-simulation state.
//
//   k_step_pd      one simulation step per wavefront (links against the
//                  object's sphere set or its distance field): hand kinematics and
//                  mass matrix at the simulation's joint angles, narrow
//                  phase and cap, the (6 + D) contact solve, integration of
//                  object and joints
//   k_window_pd    the batched window: T steps per wavefront with the
//                  observation and step cost of every step (the same bits
//                  as the per-step kernels)
//   k_observe_pd   per-sensor contact force of the last step and the
//                  simulation's joint angles (the observation of Sec. III-A)
//   k_cost_pd      step cost: the force terms plus w_q |q - q_gt|^2
//   k_copy_hand    the resampler's copies of the joint state
#include "pt_io.hpp"
#include "pt_pd.hpp"

namespace pt {

// G: the batch's largest joint group, rounded up to 4 or PD_GMAX (the size
// of the group eliminations)
template <bool SDF, int G>
__global__ __launch_bounds__(WAVE) void k_step_pd(Consts P, PdConsts Q, Tables tb, PdTab T,
                                                  const float *__restrict__ u, float *__restrict__ state,
                                                  float *__restrict__ params, float *__restrict__ warm,
                                                  float *__restrict__ hstate, float *__restrict__ contacts,
                                                  int64_t *__restrict__ stats)
{
    extern __shared__ __align__(16) char smem[];
    const int e = xcd_block(blockIdx.x, gridDim.x);
    if (e >= P.K) return;
    const int lane = lane_id();
    const int D = P.D;
    const size_t K = P.K;
    WaveLds lds = carve_lds(smem, 0, P.max_cand, P.L);
    const PdLds pl = carve_pd(smem + wave_lds_bytes(P.max_cand, P.L), D, lds.sel);
    const int type = tb.env_type[e];
    const int S = tb.n_spheres[type];
    const float *sph = tb.spheres + (size_t)type * P.S_max * 4;
    const float inv[3] = {tb.inv_inertia[3 * type], tb.inv_inertia[3 * type + 1], tb.inv_inertia[3 * type + 2]};
    const float rows = load_body_rows(state, params, P.K, e);
    int wkey;
    float wr[3];
    load_warm(warm, P.C_max, e, wkey, wr);
    // the joint state by position, one joint per lane
    float qv = 0.f, qdv = 0.f;
    int jl = 0;
    if (lane < D) {
        jl = T.jat(lane);
        qv = hstate[(size_t)jl * K + e];
        qdv = hstate[(size_t)(D + jl) * K + e];
    }
    pd_stage_joints(D, pl, qv, qdv);
    Body B;
    body_from_rows(rows, B);
    StepStats st = {0, 0, 0};
    SdfRef sdf;
    if (SDF) {
        sdf.v = tb.sdf + (size_t)type * P.sdf_n * P.sdf_n * P.sdf_n;
        sdf.box = tb.sdf_box + 4 * type;
        sdf.n = P.sdf_n;
        sdf.M = P.link_samples;
    }
    int link;
    float imp[3];
    pd_step<SDF, G>(P, Q, tb, T, u, lds, pl, sph, S, inv, sdf, qv, B, wkey, wr, st, link, imp);
    if (lane < D) {
        const double w = pl.nuh[lane];
        hstate[(size_t)jl * K + e] = (float)((double)qv + (double)P.dt * w);
        hstate[(size_t)(D + jl) * K + e] = (float)w;
    }
    store_body(state, params, P.K, e, B);
    store_warm(warm, P.C_max, e, wkey, wr);
    if (lane < P.C_max)
        *reinterpret_cast<float4 *>(contacts + ((size_t)e * P.C_max + lane) * 4) =
            make_float4(__int_as_float(link), imp[0], imp[1], imp[2]);
    flush_stats(stats, st, 1, e);
}

// Batched window of the PD hand: one wavefront per simulation runs the T
// steps of the window (commands u_win rows 1..T), each with the per-step
// kernel's code, its observation (force rows, then the joint angles) and
// the step cost of k_cost_pd added to the simulation's running sum: the
// same bits as T rounds of k_step_pd, k_observe_pd and k_cost_pd.  State,
// joint state and warm cache stay on chip between the steps.
// obs_gt_win [T][4L + D][G]; obs_out [T][4L + D][K] or NULL.
template <bool SDF, int G>
__global__ __launch_bounds__(WAVE) void k_window_pd(Consts P, PdConsts Q, Tables tb, PdTab T,
                                                    const float *__restrict__ u_win, float *__restrict__ state,
                                                    float *__restrict__ params, float *__restrict__ warm,
                                                    float *__restrict__ hstate, const float *__restrict__ obs_gt_win,
                                                    float *__restrict__ cost_sum, float *__restrict__ obs_out,
                                                    int64_t *__restrict__ stats)
{
    extern __shared__ __align__(16) char smem[];
    const int e = xcd_block(blockIdx.x, gridDim.x);
    if (e >= P.K) return;
    const int lane = lane_id();
    const int D = P.D;
    const size_t K = P.K;
    WaveLds lds = carve_lds(smem, 0, P.max_cand, P.L);
    const PdLds pl = carve_pd(smem + wave_lds_bytes(P.max_cand, P.L), D, lds.sel);
    float *stage = contact_stage(lds);
    // the joint angles by row for the cost (the cap's slots are free by then)
    float *qrow = reinterpret_cast<float *>(lds.sel);
    const int type = tb.env_type[e];
    const int g = tb.group_of[e];
    const int S = tb.n_spheres[type];
    const float *sph = tb.spheres + (size_t)type * P.S_max * 4;
    const float inv[3] = {tb.inv_inertia[3 * type], tb.inv_inertia[3 * type + 1], tb.inv_inertia[3 * type + 2]};
    const float rows = load_body_rows(state, params, P.K, e);
    int wkey;
    float wr[3];
    load_warm(warm, P.C_max, e, wkey, wr);
    float qv = 0.f, qdv = 0.f;
    int jl = 0;
    if (lane < D) {
        jl = T.jat(lane);
        qv = hstate[(size_t)jl * K + e];
        qdv = hstate[(size_t)(D + jl) * K + e];
    }
    Body B;
    body_from_rows(rows, B);
    StepStats st = {0, 0, 0};
    SdfRef sdf;
    if (SDF) {
        sdf.v = tb.sdf + (size_t)type * P.sdf_n * P.sdf_n * P.sdf_n;
        sdf.box = tb.sdf_box + 4 * type;
        sdf.n = P.sdf_n;
        sdf.M = P.link_samples;
    }
    const size_t LG = (size_t)P.L * P.G, LK = (size_t)P.L * K;
    const size_t RG = 4 * LG + (size_t)D * P.G, RK = 4 * LK + (size_t)D * K;
    float cost = cost_sum[e];
    for (int t = 0; t < P.T; ++t) {
        pd_stage_joints(D, pl, qv, qdv);
        int link;
        float imp[3];
        pd_step<SDF, G>(P, Q, tb, T, u_win + (size_t)(t + 1) * D, lds, pl, sph, S, inv, sdf, qv, B, wkey, wr, st,
                        link, imp);
        if (lane < D) {
            const double w = pl.nuh[lane];
            qv = (float)((double)qv + (double)P.dt * w);
            qdv = (float)w;
            qrow[jl] = qv;
        }
        uniform_body(B);
        *reinterpret_cast<float4 *>(stage + 4 * lane) = make_float4(__int_as_float(link), imp[0], imp[1], imp[2]);
        wave_sync();
        const float *gt = obs_gt_win + (size_t)t * RG;
        float *ob = obs_out ? obs_out + (size_t)t * RK : nullptr;
        float o[4];
        float cl = 0.f;
        if (sensor_force(P, stage, o)) {
            float gv[4] = {gt[0 * LG + (size_t)lane * P.G + g], gt[1 * LG + (size_t)lane * P.G + g],
                           gt[2 * LG + (size_t)lane * P.G + g], gt[3 * LG + (size_t)lane * P.G + g]};
            cl = sensor_cost(P, o, gv);
            if (ob) {
#pragma unroll
                for (int j = 0; j < 4; ++j) ob[j * LK + (size_t)lane * K + e] = o[j];
            }
        }
        if (ob && lane < D) ob[4 * LK + (size_t)jl * K + e] = qv;
        // sensors in sensor order, then the joints in row order
        float cs = step_cost_wave(P, cl);
        for (int j = 0; j < D; ++j) cs = pd_joint_cost(cs, Q.w_q, qrow[j], gt[4 * LG + (size_t)j * P.G + g]);
        wave_sync();
        cost += cs;
    }
    if (lane < D) {
        hstate[(size_t)jl * K + e] = qv;
        hstate[(size_t)(D + jl) * K + e] = qdv;
    }
    store_body(state, params, P.K, e, B);
    store_warm(warm, P.C_max, e, wkey, wr);
    if (lane == 0) cost_sum[e] = cost;
    flush_stats(stats, st, P.T, e);
}

// one wavefront per simulation, lanes over sensors, then over joints:
// obs rows [4][L] of force terms followed by the D joint angles
__global__ __launch_bounds__(256) void k_observe_pd(Consts P, const float *__restrict__ contacts,
                                                    const float *__restrict__ hstate, float *__restrict__ obs)
{
    __shared__ __align__(16) float stage[4][WAVE * 4];
    const int wib = threadIdx.x / WAVE;
    const int e = xcd_block(blockIdx.x, gridDim.x) * (blockDim.x / WAVE) + wib;
    if (e >= P.K) return;
    const int lane = lane_id();
    float *sg = stage[wib];
    if (lane < P.C_max)
        *reinterpret_cast<float4 *>(sg + 4 * lane) =
            *reinterpret_cast<const float4 *>(contacts + ((size_t)e * P.C_max + lane) * 4);
    wave_sync();
    const size_t LK = (size_t)P.L * P.K;
    float o[7];
    if (sensor_force(P, sg, o)) {
#pragma unroll
        for (int j = 0; j < 4; ++j) obs[j * LK + (size_t)lane * P.K + e] = o[j];
    }
    for (int j = lane; j < P.D; j += WAVE) obs[4 * LK + (size_t)j * P.K + e] = hstate[(size_t)j * P.K + e];
}

// one thread per simulation: the sensors' terms in sensor order (as k_cost),
// then the joints' w_q (q_j - q_gt_j)^2 in joint order; obs_gt [4L + D][G]
__global__ __launch_bounds__(256) void k_cost_pd(Consts P, PdConsts Q, const int32_t *__restrict__ group_of,
                                                 const float *__restrict__ obs, const float *__restrict__ obs_gt,
                                                 float *cost_sum)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P.K) return;
    const int g = P.G == 1 ? 0 : group_of[e];
    const size_t LK = (size_t)P.L * P.K, LG = (size_t)P.L * P.G;
    float cs = 0.f;
    for (int l = 0; l < P.L; ++l) {
        float o[4], gt[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            o[j] = obs[j * LK + (size_t)l * P.K + e];
            gt[j] = obs_gt[j * LG + (size_t)l * P.G + g];
        }
        cs += sensor_cost(P, o, gt);
    }
    for (int j = 0; j < P.D; ++j)
        cs = pd_joint_cost(cs, Q.w_q, obs[4 * LK + (size_t)j * P.K + e], obs_gt[4 * LG + (size_t)j * P.G + g]);
    cost_sum[e] += cs;
}

// joint state rows of every resampled simulation from its parent (parents
// are elites, which the resampler leaves unchanged: every copy reads rows
// nothing here writes)
__global__ __launch_bounds__(256) void k_copy_hand(int K, int rows, const int32_t *__restrict__ parent,
                                                   float *__restrict__ hstate)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= K) return;
    const int p = parent[e];
    if (p < 0) return;
    for (int r = 0; r < rows; ++r) hstate[(size_t)r * K + e] = hstate[(size_t)r * K + p];
}

}  // namespace pt

using namespace pt;

size_t pd_wave_lds_bytes(int max_cand, int L, int D) { return wave_lds_bytes(max_cand, L) + pd_lds_bytes(D); }

hipError_t set_pd_lds_limits(size_t bytes)
{
    const void *fs[] = {(const void *)k_step_pd<false, 4>,         (const void *)k_step_pd<true, 4>,
                        (const void *)k_step_pd<false, PD_GMAX>,   (const void *)k_step_pd<true, PD_GMAX>,
                        (const void *)k_window_pd<false, 4>,       (const void *)k_window_pd<true, 4>,
                        (const void *)k_window_pd<false, PD_GMAX>, (const void *)k_window_pd<true, PD_GMAX>};
    for (const void *f : fs) {
        hipError_t e = set_dynamic_lds_limit(f, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_step_pd(const Consts &P, const PdConsts &Q, const Tables &tb, const int32_t *pd_tab,
                          const float *u, float *state, float *params, float *warm, float *hstate, float *contacts,
                          int64_t *stats, hipStream_t s)
{
    const PdTab T = {pd_tab, P.D, P.L};
    const size_t lds = pd_wave_lds_bytes(P.max_cand, P.L, P.D);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(P.K), dim3(WAVE), lds, s, P, Q, tb, T, u, state, params, warm, hstate,
                           contacts, stats);
    };
    const bool small = Q.gmax <= 4;
    if (P.collision_mode == 1)
        small ? go(k_step_pd<true, 4>) : go(k_step_pd<true, PD_GMAX>);
    else
        small ? go(k_step_pd<false, 4>) : go(k_step_pd<false, PD_GMAX>);
    return hipGetLastError();
}

hipError_t launch_window_pd(const Consts &P, const PdConsts &Q, const Tables &tb, const int32_t *pd_tab,
                            const float *u_win, float *state, float *params, float *warm, float *hstate,
                            const float *obs_gt_win, float *cost_sum, float *obs_out, int64_t *stats, hipStream_t s)
{
    const PdTab T = {pd_tab, P.D, P.L};
    const size_t lds = pd_wave_lds_bytes(P.max_cand, P.L, P.D);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(P.K), dim3(WAVE), lds, s, P, Q, tb, T, u_win, state, params, warm, hstate,
                           obs_gt_win, cost_sum, obs_out, stats);
    };
    const bool small = Q.gmax <= 4;
    if (P.collision_mode == 1)
        small ? go(k_window_pd<true, 4>) : go(k_window_pd<true, PD_GMAX>);
    else
        small ? go(k_window_pd<false, 4>) : go(k_window_pd<false, PD_GMAX>);
    return hipGetLastError();
}

hipError_t launch_observe_pd(const Consts &P, const float *contacts, const float *hstate, float *obs,
                             hipStream_t s)
{
    const int blocks = (P.K + 3) / 4;
    hipLaunchKernelGGL(k_observe_pd, dim3(blocks), dim3(4 * WAVE), 0, s, P, contacts, hstate, obs);
    return hipGetLastError();
}

hipError_t launch_cost_pd(const Consts &P, const PdConsts &Q, const int32_t *group_of, const float *obs,
                          const float *obs_gt, float *cost_sum, hipStream_t s)
{
    hipLaunchKernelGGL(k_cost_pd, dim3((P.K + 255) / 256), dim3(256), 0, s, P, Q, group_of, obs, obs_gt, cost_sum);
    return hipGetLastError();
}

hipError_t launch_copy_hand(int K, int rows, const int32_t *parent, float *hstate, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_hand, dim3((K + 255) / 256), dim3(256), 0, s, K, rows, parent, hstate);
    return hipGetLastError();
}
