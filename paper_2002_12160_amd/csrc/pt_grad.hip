// pt_grad.hip -- gradients of the window cost and the elite refinement built
// on them.
//
//   k_window_fwd      one wavefront per listed simulation: runs the window
//                     from a given start with the step code of the other
//                     kernels (same bits), the cost and optionally the end
//                     state; with a checkpoint buffer it records, before every
//                     step, the body and after the step's solve the kept
//                     contact keys and their impulses (float64)
//   k_window_bwd      the reverse sweep over those checkpoints: each step's
//                     contacts are rebuilt from the recorded keys (no narrow
//                     phase, no Newton solve), then the step adjoint runs
//                     (implicit differentiation of the contact solve).
//                     Output: the gradient of the window cost with respect
//                     to the start (x, q, v, w, m, mu, f)
//   k_select_elites   per group, the simulations of lowest window cost (the
//                     same ranking the resampler keeps)
//   k_refine_*        gather / scaled gradient step / accept-or-halve
#include "pt_adjoint.hpp"
#include "pt_internal.h"
#include "pt_io.hpp"

namespace pt {

__device__ __forceinline__ void load_start(const float *__restrict__ xi, int n, int i, Body &B)
{
    B.x[0] = xi[0 * (size_t)n + i]; B.x[1] = xi[1 * (size_t)n + i]; B.x[2] = xi[2 * (size_t)n + i];
    B.q[0] = xi[3 * (size_t)n + i]; B.q[1] = xi[4 * (size_t)n + i]; B.q[2] = xi[5 * (size_t)n + i];
    B.q[3] = xi[6 * (size_t)n + i];
    B.v[0] = xi[7 * (size_t)n + i]; B.v[1] = xi[8 * (size_t)n + i]; B.v[2] = xi[9 * (size_t)n + i];
    B.w[0] = xi[10 * (size_t)n + i]; B.w[1] = xi[11 * (size_t)n + i]; B.w[2] = xi[12 * (size_t)n + i];
    B.m = xi[13 * (size_t)n + i]; B.mu = xi[14 * (size_t)n + i];
    B.f[0] = xi[15 * (size_t)n + i]; B.f[1] = xi[16 * (size_t)n + i]; B.f[2] = xi[17 * (size_t)n + i];
}

// xi is [18][n]: x(3) q(4) v(3) w(3) m mu f(3); warm0 is [n][C_max][4]
// One launch covers `count` listed simulations i0 .. i0+count-1 of arrays
// with row stride n; the checkpoint buffer holds `count` simulations.
template <typename SR, bool PT>
__global__ __launch_bounds__(WAVE) void k_window_fwd(Consts P, Tables tb, const float *__restrict__ seg_win, int n,
                                                     int i0, int count,
                                                     const int32_t *__restrict__ env, const float *__restrict__ xi,
                                                     const float *__restrict__ warm0,
                                                     const float *__restrict__ obs_gt_win, float *__restrict__ cost_out,
                                                     float *__restrict__ end_state, float *__restrict__ end_warm,
                                                     float *__restrict__ ckpt, float *__restrict__ resid_out)
{
    extern __shared__ __align__(16) char smem[];
    const int c = blockIdx.x;
    if (c >= count) return;
    const int i = i0 + c;
    const int lane = lane_id();
    const int e = env[i];
    if (e < 0 || e >= P.K) {
        // not a simulation of this batch
        if (lane == 0) cost_out[i] = __int_as_float(0x7fc00000);
        return;
    }
    WaveLds lds = carve_lds(smem, 0, P.max_cand, 0);
    float *stage = contact_stage(lds);
    const int type = tb.env_type[e];
    const int g = tb.group_of[e];
    const int S = tb.n_spheres[type];
    const float *sph = tb.spheres + (size_t)type * P.S_max * 4;
    const float inv[3] = {tb.inv_inertia[3 * type], tb.inv_inertia[3 * type + 1], tb.inv_inertia[3 * type + 2]};
    const size_t LG = (size_t)P.L * P.G;
    const size_t CK = ckpt_step_floats(P.C_max);

    Body B;
    load_start(xi, n, i, B);
    int wkey;
    float wr[3];
    load_warm(warm0, P.C_max, i, wkey, wr);
    StepStats stt = {0, 0, 0};

    // cost summed in the order of the other paths; the largest final merit
    // of the window's contact solves (how far they are from the root the
    // reverse sweep assumes)
    float cost = 0.f, resid = 0.f;
    for (int t = 0; t < P.T; ++t) {
        float *ck = ckpt ? ckpt + ((size_t)c * P.T + t) * CK : nullptr;
        if (ck) save_body(ck, B);
        const float *seg = seg_win + (size_t)t * P.L * SEG_STRIDE;
        StepState<SR> st;
        step_setup<SR>(P, seg, sph, S, inv, B, wkey, wr, lds, stt, st);
        step_solve<SR, PT>(P, st, B.mu, inv, reinterpret_cast<SR *>(lds.cand_d));
        resid = fmaxf(resid, (float)st.psi_end);
        if (ck) save_contact<SR>(ck, P.C_max, st);
        int link;
        float imp[3];
        step_finish<SR>(P, st, inv, B, wkey, wr, link, imp);
        uniform_body(B);
        *reinterpret_cast<float4 *>(stage + 4 * lane) = make_float4(__int_as_float(link), imp[0], imp[1], imp[2]);
        wave_sync();
        float o[4];
        float cl = 0.f;
        if (sensor_force(P, stage, o)) {
            const float *gt = obs_gt_win + (size_t)t * 4 * LG;
            float gv[4] = {gt[0 * LG + (size_t)lane * P.G + g], gt[1 * LG + (size_t)lane * P.G + g],
                           gt[2 * LG + (size_t)lane * P.G + g], gt[3 * LG + (size_t)lane * P.G + g]};
            cl = sensor_cost(P, o, gv);
        }
        wave_sync();
        cost += step_cost_wave(P, cl);
    }
    if (lane == 0) {
        cost_out[i] = cost;
        if (resid_out) resid_out[i] = resid;
        if (end_state) {
            const float v13[13] = {B.x[0], B.x[1], B.x[2], B.q[0], B.q[1], B.q[2], B.q[3],
                                   B.v[0], B.v[1], B.v[2], B.w[0], B.w[1], B.w[2]};
            for (int r = 0; r < 13; ++r) end_state[(size_t)r * n + i] = v13[r];
        }
    }
    if (end_warm) store_warm(end_warm, P.C_max, i, wkey, wr);
}

// reverse sweep over the checkpoints k_window_fwd wrote for the same n, env
// and xi (ckpt_by_env = 0: slot c of the launch), or that the population's
// window wrote (ckpt_by_env = 1: slot env[i]); simulations with flag[i] == 0
// are skipped (flag may be NULL)
template <typename SR>
__global__ __launch_bounds__(WAVE) void k_window_bwd(Consts P, Tables tb, const float *__restrict__ seg_win, int n,
                                                     int i0, int count,
                                                     const int32_t *__restrict__ env, const float *__restrict__ xi,
                                                     const float *__restrict__ obs_gt_win,
                                                     const float *__restrict__ ckpt, int ckpt_by_env,
                                                     const int32_t *__restrict__ flag, float *__restrict__ grad)
{
    extern __shared__ __align__(16) char smem[];
    const int c = blockIdx.x;
    if (c >= count) return;
    const int i = i0 + c;
    if (flag && flag[i] == 0) return;
    const int lane = lane_id();
    const int e = env[i];
    if (e < 0 || e >= P.K) {
        if (lane == 0)
            for (int r = 0; r < XI_ROWS; ++r) grad[(size_t)r * n + i] = 0.f;
        return;
    }
    // the sum rows whole in the list: the adjoint stages data in the words after it
    WaveLds lds = carve_lds(smem, 0, P.max_cand_rows, 0);
    float *stage = contact_stage(lds);
    const int type = tb.env_type[e];
    const int g = tb.group_of[e];
    const float *sph = tb.spheres + (size_t)type * P.S_max * 4;
    const float inv[3] = {tb.inv_inertia[3 * type], tb.inv_inertia[3 * type + 1], tb.inv_inertia[3 * type + 2]};
    const size_t LG = (size_t)P.L * P.G;
    const size_t CK = ckpt_step_floats(P.C_max);
    const float m0 = xi[13 * (size_t)n + i], mu0 = xi[14 * (size_t)n + i];

    BodyBar<SR> bar;
#pragma unroll
    for (int k = 0; k < 3; ++k) bar.x[k] = bar.v[k] = bar.w[k] = SR(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) bar.q[k] = SR(0);
    SR mbar = 0, mubar = 0, fbar[3] = {0, 0, 0};
    for (int t = P.T - 1; t >= 0; --t) {
        const float *ck = ckpt + ((size_t)(ckpt_by_env ? e : c) * P.T + t) * CK;
        Body B;
        load_body_ckpt(ck, B);
        B.m = m0;
        B.mu = mu0;
        SR r[3];
        const int key = load_contact<SR>(ck, P.C_max, r);
        const float *seg = seg_win + (size_t)t * P.L * SEG_STRIDE;
        // the step as the forward sweep left it: same contacts, same impulses
        StepState<SR> st;
        step_pose<SR>(P, inv, B, st);
        contact_setup<SR>(P, seg, sph, B, key, st);
        const int C = __popcll(__ballot(st.act));
        st.C = C;
        st.ncand = C;
        st.span = lane_span(C);
        st.r[0] = r[0]; st.r[1] = r[1]; st.r[2] = r[2];
        body_dv(st, st.r, st.nu);
        st.nu[0] += st.vs[0]; st.nu[1] += st.vs[1]; st.nu[2] += st.vs[2];
        st.nu[3] += st.ws[0]; st.nu[4] += st.ws[1]; st.nu[5] += st.ws[2];
        step_adjoint<SR>(P, seg, sph, inv, B, st, obs_gt_win + (size_t)t * 4 * LG, g, stage, lds.wr,
                         reinterpret_cast<SR *>(lds.cand_d), bar, mbar, mubar, t == 0 ? fbar : nullptr);
    }
    if (lane == 0) {
        const SR gv[XI_ROWS] = {bar.x[0], bar.x[1], bar.x[2], bar.q[0], bar.q[1], bar.q[2], bar.q[3],
                                bar.v[0], bar.v[1], bar.v[2], bar.w[0], bar.w[1], bar.w[2],
                                mbar,     mubar,    fbar[0],  fbar[1],  fbar[2]};
        for (int r = 0; r < XI_ROWS; ++r) grad[(size_t)r * n + i] = (float)gv[r];
    }
}

// one workgroup per group: its elites (lowest (cost, index), NaN ranked as
// +inf; count max(1, floor(n elite_frac))) go to elite_env[offset + rank],
// offset = number of elites of the lower groups
__global__ __launch_bounds__(1024) void k_select_elites(int G, float elite_frac, const int32_t *__restrict__ group_start,
                                                        const float *__restrict__ cost_sum, int32_t *__restrict__ elite_env)
{
    extern __shared__ __align__(16) char smem[];
    const int g = blockIdx.x;
    if (g >= G) return;
    int off = 0;
    for (int h = 0; h < g; ++h) off += elite_count(group_start[h + 1] - group_start[h], elite_frac);
    const int lo = group_start[g], n = group_start[g + 1] - lo;
    const int np2 = sort_slots(n);
    const int kb = elite_count(n, elite_frac);
    float *cs = reinterpret_cast<float *>(smem);
    int *order = reinterpret_cast<int *>(smem + 4 * (size_t)np2);
    sort_group(cost_sum + lo, n, np2, cs, order);
    for (int t = threadIdx.x; t < kb; t += blockDim.x) elite_env[off + t] = lo + order[t];
}

// start of each listed simulation from the window-start snapshot (and, if
// cost_sum is given, its window cost)
__global__ void k_refine_gather(int n, int K, int C_max, const int32_t *__restrict__ env,
                                const float *__restrict__ state, const float *__restrict__ params,
                                const float *__restrict__ warm, const float *__restrict__ cost_sum,
                                float *__restrict__ xi, float *__restrict__ warm0, float *__restrict__ cost,
                                float *__restrict__ rho, float rho0)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int e = env[i];
    if (e < 0 || e >= K) return;
    for (int r = 0; r < 13; ++r) xi[(size_t)r * n + i] = state[(size_t)r * K + e];
    for (int r = 0; r < 5; ++r) xi[(size_t)(13 + r) * n + i] = params[(size_t)r * K + e];
    const float4 *src = reinterpret_cast<const float4 *>(warm + (size_t)e * C_max * WARM_STRIDE);
    float4 *dst = reinterpret_cast<float4 *>(warm0 + (size_t)i * C_max * WARM_STRIDE);
    for (int c = 0; c < C_max; ++c) dst[c] = src[c];
    rho[i] = rho0;
    if (cost_sum) cost[i] = cost_sum[e];
}

// trial start: xi - rho (s o s o g) / |s o g| over (x, q, v, w, m, mu), then
// q renormalised and m, mu clamped; the one-step force is kept (elites
// i0 .. i0+count-1 of arrays with row stride n)
__global__ void k_refine_propose(int n, int i0, int count, RefineArgs A, const float *__restrict__ xi,
                                 const float *__restrict__ grad, const float *__restrict__ rho,
                                 float *__restrict__ xi_try)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= count) return;
    const int i = i0 + c;
    float x[XI_ROWS];
    for (int r = 0; r < XI_ROWS; ++r) x[r] = xi[(size_t)r * n + i];
    float sg2 = 0.f;
    for (int r = 0; r < 15; ++r) {
        float v = A.scale[r] * grad[(size_t)r * n + i];
        sg2 += v * v;
    }
    const float nrm = sqrtf(sg2);
    if (nrm > 0.f && nrm < __int_as_float(0x7f800000)) {
        const float f = rho[i] / nrm;
        for (int r = 0; r < 15; ++r) x[r] -= f * A.scale[r] * A.scale[r] * grad[(size_t)r * n + i];
        const float qn = sqrtf(x[3] * x[3] + x[4] * x[4] + x[5] * x[5] + x[6] * x[6]);
        if (qn > 0.f)
            for (int r = 3; r < 7; ++r) x[r] /= qn;
        x[13] = fminf(fmaxf(x[13], A.m_lo), A.m_hi);
        x[14] = fminf(fmaxf(x[14], A.mu_lo), A.mu_hi);
    }
    for (int r = 0; r < XI_ROWS; ++r) xi_try[(size_t)r * n + i] = x[r];
}

// keep the trial where its replayed window cost is lower (the batch slot then
// takes the replay's end-of-window state, mass, friction and warm cache, and
// its window cost; flag[i] = 1 asks for the gradient at the new start);
// otherwise halve the step (flag[i] = 0); elites i0 .. i0+count-1
__global__ void k_refine_accept(int n, int i0, int count, int K, int C_max, const int32_t *__restrict__ env,
                                float *__restrict__ cost_cur,
                                const float *__restrict__ cost_try, float *__restrict__ xi,
                                const float *__restrict__ xi_try, float *__restrict__ rho, int32_t *__restrict__ flag,
                                const float *__restrict__ end_state, const float *__restrict__ end_warm,
                                float *__restrict__ state, float *__restrict__ params, float *__restrict__ warm,
                                float *__restrict__ cost_sum)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= count) return;
    const int i = i0 + c;
    flag[i] = 0;
    const int e = env[i];
    if (e < 0 || e >= K) return;
    const float ct = cost_try[i];
    if (!(ct < cost_cur[i])) {
        rho[i] *= 0.5f;
        return;
    }
    flag[i] = 1;
    cost_cur[i] = ct;
    for (int r = 0; r < XI_ROWS; ++r) xi[(size_t)r * n + i] = xi_try[(size_t)r * n + i];
    for (int r = 0; r < 13; ++r) state[(size_t)r * K + e] = end_state[(size_t)r * n + i];
    params[0 * (size_t)K + e] = xi_try[13 * (size_t)n + i];
    params[1 * (size_t)K + e] = xi_try[14 * (size_t)n + i];
    params[2 * (size_t)K + e] = 0.f;
    params[3 * (size_t)K + e] = 0.f;
    params[4 * (size_t)K + e] = 0.f;
    const float4 *src = reinterpret_cast<const float4 *>(end_warm + (size_t)i * C_max * WARM_STRIDE);
    float4 *dst = reinterpret_cast<float4 *>(warm + (size_t)e * C_max * WARM_STRIDE);
    for (int c = 0; c < C_max; ++c) dst[c] = src[c];
    cost_sum[e] = ct;
}

}  // namespace pt

using namespace pt;

size_t ckpt_floats(const Consts &P, int n) { return (size_t)n * P.T * ckpt_step_floats(P.C_max); }

hipError_t launch_window_fwd(const Consts &P, const Tables &tb, const float *seg_win, int n, int i0, int count,
                             const int32_t *env, const float *xi, const float *warm0, const float *obs_gt_win,
                             float *cost, float *end_state, float *end_warm, float *ckpt, hipStream_t s,
                             float *resid)
{
    if (count <= 0) return hipSuccess;
    size_t lds = wave_lds_bytes(P.max_cand, 0);
    // paired line-search trials when no step can hold more than 32 contacts
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(count), dim3(WAVE), lds, s, P, tb, seg_win, n, i0, count, env, xi, warm0,
                           obs_gt_win, cost, end_state, end_warm, ckpt, resid);
        return hipGetLastError();
    };
    const bool pt = P.C_max <= 32;
    if (P.solve_fp64) return pt ? go(k_window_fwd<double, true>) : go(k_window_fwd<double, false>);
    return pt ? go(k_window_fwd<float, true>) : go(k_window_fwd<float, false>);
}

hipError_t launch_window_bwd(const Consts &P, const Tables &tb, const float *seg_win, int n, int i0, int count,
                             const int32_t *env, const float *xi, const float *obs_gt_win, const float *ckpt,
                             bool ckpt_by_env, const int32_t *flag, float *grad, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    size_t lds = wave_lds_bytes(P.max_cand_rows, 0);
    const int by_env = ckpt_by_env ? 1 : 0;
    if (P.solve_fp64)
        hipLaunchKernelGGL(k_window_bwd<double>, dim3(count), dim3(WAVE), lds, s, P, tb, seg_win, n, i0, count, env,
                           xi, obs_gt_win, ckpt, by_env, flag, grad);
    else
        hipLaunchKernelGGL(k_window_bwd<float>, dim3(count), dim3(WAVE), lds, s, P, tb, seg_win, n, i0, count, env,
                           xi, obs_gt_win, ckpt, by_env, flag, grad);
    return hipGetLastError();
}

hipError_t launch_select_elites(int G, int max_group, float elite_frac, const int32_t *group_start,
                                const float *cost_sum, int32_t *elite_env, hipStream_t s)
{
    hipLaunchKernelGGL(k_select_elites, dim3(G), dim3(group_threads(max_group)), resample_lds_bytes(max_group), s,
                       G, elite_frac,
                       group_start, cost_sum, elite_env);
    return hipGetLastError();
}

hipError_t launch_refine_gather(int n, int K, int C_max, const int32_t *env, const float *state, const float *params,
                                const float *warm, const float *cost_sum, float *xi, float *warm0, float *cost,
                                float *rho, float rho0, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine_gather, dim3((n + 63) / 64), dim3(64), 0, s, n, K, C_max, env, state, params, warm,
                       cost_sum, xi, warm0, cost, rho, rho0);
    return hipGetLastError();
}

hipError_t launch_refine_propose(int n, int i0, int count, const RefineArgs &A, const float *xi, const float *grad,
                                 const float *rho, float *xi_try, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine_propose, dim3((count + 63) / 64), dim3(64), 0, s, n, i0, count, A, xi, grad, rho,
                       xi_try);
    return hipGetLastError();
}

hipError_t launch_refine_accept(int n, int i0, int count, int K, int C_max, const int32_t *env, float *cost_cur,
                                const float *cost_try, float *xi, const float *xi_try, float *rho, int32_t *flag,
                                const float *end_state, const float *end_warm, float *state, float *params,
                                float *warm, float *cost_sum, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_refine_accept, dim3((count + 63) / 64), dim3(64), 0, s, n, i0, count, K, C_max, env,
                       cost_cur, cost_try, xi, xi_try, rho, flag, end_state, end_warm, state, params, warm, cost_sum);
    return hipGetLastError();
}

hipError_t set_grad_lds_limits(size_t bytes)
{
    const void *fs[] = {reinterpret_cast<const void *>(k_select_elites),
                        reinterpret_cast<const void *>(k_window_fwd<float, false>),
                        reinterpret_cast<const void *>(k_window_fwd<double, false>),
                        reinterpret_cast<const void *>(k_window_fwd<float, true>),
                        reinterpret_cast<const void *>(k_window_fwd<double, true>),
                        reinterpret_cast<const void *>(k_window_bwd<float>),
                        reinterpret_cast<const void *>(k_window_bwd<double>)};
    for (const void *f : fs) {
        hipError_t e = set_dynamic_lds_limit(f, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
