// pt_kernels.hip -- HIP kernels of libpt for CDNA4 (gfx950).
//
//   k_hand_fk      forward kinematics of the kinematic hand, once per step
//                  (shared by every simulation: the same command u_t drives
//                  all of them, Alg. 1)
//   k_step         plain path: one simulation step per wavefront; contacts
//                  written to HBM for the observation kernel
//   k_observe      per-sensor contact force of the last step
//   k_cost         step cost against the observed force, running sum (Eq. 1)
//   k_argmin       per-group argmin of the running cost (Eq. 2)
//   k_resample     population-based resampling with Philox4x32-10 (Sec. III-D.3)
//   k_window       batched path: persistent kernel running T steps with the
//                  observation and cost fused, state kept on chip
#include "pt_internal.h"
#include "pt_io.hpp"

namespace pt {

// ---------------------------------------------------------------------
// hand kinematics (double precision: it runs once per step for the whole
// population, and the link velocities are differences of positions)
// ---------------------------------------------------------------------
// Joint rotation of a link for joint vector u, Rot(axis0, u[j0]) Rot(axis1,
// u[j1]) (identity for a joint index < 0), by a pair of adjacent lanes: lane
// j of the pair (j = 0, 1) evaluates the half-angle rotation of joint j, the
// odd lane's moves to the even one (DPP, quad_perm [1,0,3,2]), which composes
// the two and writes them to qj.  Both lanes of the pair must be active.
__device__ __forceinline__ void fk_joint_pair(const float *__restrict__ h, const float *__restrict__ u, int j,
                                              double *qj)
{
    const int jx = (int)h[1 + j];
    const float *ax = h + 3 + 3 * j;
    double q[4] = {1, 0, 0, 0};
    if (jx >= 0) {
        double s, c;
        sincos(0.5 * (double)u[jx], &s, &c);
        q[0] = c; q[1] = s * ax[0]; q[2] = s * ax[1]; q[3] = s * ax[2];
    }
    double r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = dpp_f<0xb1, 0xf>(q[i]);
    if (j == 0) {
        if ((int)h[2] >= 0) {
            double t[4];
            quat_mul_d(q, r, t);
            for (int i = 0; i < 4; ++i) q[i] = t[i];
        }
        for (int i = 0; i < 4; ++i) qj[i] = q[i];
    }
}

// pose of link l in configuration w from its parent's (already computed):
// origin, orientation and the segment [a, b] along the link's local +x axis
__device__ __forceinline__ void fk_link(const float *__restrict__ h, int parent, const double *qj, double *tq, double *tp,
                        double *seg_a, double *seg_b, int l)
{
    double pq[4] = {1, 0, 0, 0}, pp[3] = {0, 0, 0};
    if (parent >= 0) {
        for (int i = 0; i < 4; ++i) pq[i] = tq[4 * parent + i];
        for (int i = 0; i < 3; ++i) pp[i] = tp[3 * parent + i];
    }
    double Rp[9];
    quat_to_mat_d(pq, Rp);
    double off[3] = {h[9], h[10], h[11]};
    double o[3] = {pp[0] + Rp[0] * off[0] + Rp[1] * off[1] + Rp[2] * off[2],
                   pp[1] + Rp[3] * off[0] + Rp[4] * off[1] + Rp[5] * off[2],
                   pp[2] + Rp[6] * off[0] + Rp[7] * off[1] + Rp[8] * off[2]};
    double qo[4] = {h[12], h[13], h[14], h[15]};
    double q0[4], q[4];
    quat_mul_d(pq, qo, q0);
    quat_mul_d(q0, qj + 4 * l, q);
    double len = h[16];
    // local +x axis of the link frame
    double xa[3] = {1 - 2 * (q[2] * q[2] + q[3] * q[3]), 2 * (q[1] * q[2] + q[0] * q[3]),
                    2 * (q[1] * q[3] - q[0] * q[2])};
    double b[3] = {o[0] + len * xa[0], o[1] + len * xa[1], o[2] + len * xa[2]};
    for (int i = 0; i < 4; ++i) tq[4 * l + i] = q[i];
    for (int i = 0; i < 3; ++i) {
        tp[3 * l + i] = b[i];
        seg_a[3 * l + i] = o[i];
        seg_b[3 * l + i] = b[i];
    }
}

// LDS of one evaluation of the hand kinematics: the link table, the link
// depths, and for both configurations the joint rotations, link frames and
// segment ends (double)
struct FkLds {
    float *hs;
    int *depth;
    float *su;       // [2][Ds] staged joint commands (u_prev, u), Ds = fk_staged_joints(D)
    double *cf;      // per configuration w: cf + 17 L w = [qj 4L | tq 4L | tp 3L | sa 3L | sb 3L]
    int L;
    __device__ double *qj(int w) const { return cf + (size_t)17 * L * w; }
    __device__ double *tq(int w) const { return cf + (size_t)17 * L * w + 4 * L; }
    __device__ double *tp(int w) const { return cf + (size_t)17 * L * w + 8 * L; }
    __device__ double *sa(int w) const { return cf + (size_t)17 * L * w + 11 * L; }
    __device__ double *sb(int w) const { return cf + (size_t)17 * L * w + 14 * L; }
};

// joint commands staged in LDS (every command, read before the link table
// says which ones are used); past 2 MAX_LINKS of them they are read from
// global memory where needed
__host__ __device__ constexpr int fk_staged_joints(int D) { return D <= 2 * MAX_LINKS ? D : 0; }

__host__ __device__ constexpr size_t fk_head_bytes(int L, int D)
{
    return ((size_t)L * (4 * HAND_STRIDE + 4) + (size_t)8 * fk_staged_joints(D) + 7) & ~(size_t)7;
}

__host__ __device__ constexpr size_t fk_lds_bytes(int L, int D) { return fk_head_bytes(L, D) + (size_t)L * 2 * 17 * 8; }

__device__ __forceinline__ FkLds carve_fk(char *p, int L, int D)
{
    FkLds s;
    s.hs = reinterpret_cast<float *>(p);
    s.depth = reinterpret_cast<int *>(s.hs + (size_t)L * HAND_STRIDE);
    s.su = reinterpret_cast<float *>(s.depth + L);
    s.cf = reinterpret_cast<double *>(p + fk_head_bytes(L, D));
    s.L = L;
    return s;
}

// Hand kinematics of one step by nt cooperating threads (tid in [0, nt), nt
// even, a wavefront's lanes in order): the link table staged in LDS, the joint
// rotations (the transcendental part) one thread per (configuration, link,
// joint), the chains composed level by
// level of the link tree (links at one depth in parallel, both
// configurations at once), then the segment record of every link: a,
// b - a, the radius, 1/|b - a|^2 and the end-point velocities
// (FK(u) - FK(u_prev)) / dt.  sync() orders the LDS between the stages.
// Every value is computed by the same code whichever threads run it, so a
// workgroup and a wavefront produce the same bits.
template <typename Sync>
__device__ __forceinline__ void hand_kinematics(const float *__restrict__ hand, int L, int D, float dt,
                                                const float *__restrict__ u_prev, const float *__restrict__ u,
                                                const FkLds &s, float *seg_out, int tid, int nt, Sync sync)
{
    const int Ds = fk_staged_joints(D);
    // the loads in flight together before their LDS writes: the commands,
    // then the link table eight per thread at a time (one round trip to
    // memory for a table of up to 8 nt floats, not one per element)
    float up0 = 0.f, uu0 = 0.f;
    if (tid < Ds) {
        up0 = u_prev[tid];
        uu0 = u[tid];
    }
    const int nh = L * HAND_STRIDE;
    for (int i0 = tid; i0 < nh; i0 += 8 * nt) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = hand[min(i0 + k * nt, nh - 1)];   // in bounds, no branch
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (i0 + k * nt < nh) s.hs[i0 + k * nt] = v[k];
    }
    if (tid < Ds) {
        s.su[tid] = up0;
        s.su[Ds + tid] = uu0;
    }
    for (int i = tid + nt; i < Ds; i += nt) {
        s.su[i] = u_prev[i];
        s.su[Ds + i] = u[i];
    }
    sync();
    for (int l = tid; l < L; l += nt) {
        // parents precede children (checked at batch creation), so the walk ends
        int d = 0, p = (int)s.hs[l * HAND_STRIDE];
        while (p >= 0) {
            ++d;
            p = (int)s.hs[p * HAND_STRIDE];
        }
        s.depth[l] = d;
    }
    // thread pairs (2m, 2m + 1) share an iteration (4 L and nt are even)
    for (int i = tid; i < 4 * L; i += nt) {
        const int w = i / (2 * L), r = i - w * 2 * L, l = r >> 1;
        const float *uw = Ds > 0 ? s.su + w * Ds : (w == 0 ? u_prev : u);
        fk_joint_pair(s.hs + l * HAND_STRIDE, uw, r & 1, s.qj(w) + 4 * l);
    }
    sync();
    int dmax = 0;
    for (int l = 0; l < L; ++l) dmax = max(dmax, s.depth[l]);
    for (int d = 0; d <= dmax; ++d) {
        for (int i = tid; i < 2 * L; i += nt) {
            int w = i / L, l = i - w * L;
            if (s.depth[l] == d)
                fk_link(s.hs + l * HAND_STRIDE, (int)s.hs[l * HAND_STRIDE], s.qj(w), s.tq(w), s.tp(w), s.sa(w),
                        s.sb(w), l);
        }
        sync();
    }
    const double idt = 1.0 / (double)dt;
    for (int l = tid; l < L; l += nt) {
        float *o = seg_out + (size_t)l * SEG_STRIDE;
        float a0[3], ab[3];
        const double *sa0 = s.sa(0), *sb0 = s.sb(0), *sa1 = s.sa(1), *sb1 = s.sb(1);
        for (int i = 0; i < 3; ++i) {
            a0[i] = (float)sa0[3 * l + i];
            ab[i] = (float)(sb0[3 * l + i] - sa0[3 * l + i]);
        }
        float L2 = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2];
        float inv = sqrtf(L2) >= 1e-9f ? 1.f / L2 : 0.f;
        for (int i = 0; i < 3; ++i) {
            o[i] = a0[i];
            o[4 + i] = ab[i];
            o[8 + i] = (float)((sa1[3 * l + i] - sa0[3 * l + i]) * idt);
            o[12 + i] = (float)((sb1[3 * l + i] - sb0[3 * l + i]) * idt);
        }
        o[3] = s.hs[l * HAND_STRIDE + 17];
        o[7] = inv;
        o[11] = 0.f;
        o[15] = 0.f;
    }
}

// grid: one block per step; u_prev/u for step t at u_prev + t*stride
__global__ __launch_bounds__(128) void k_hand_fk(const float *__restrict__ hand, int L, int D, float dt,
                                                 const float *__restrict__ u_prev, const float *__restrict__ u,
                                                 int stride, float *__restrict__ seg_out)
{
    __shared__ __align__(16) char fk[fk_lds_bytes(MAX_LINKS, 2 * MAX_LINKS)];
    const int t = blockIdx.x;
    const FkLds s = carve_fk(fk, L, D);
    hand_kinematics(hand, L, D, dt, u_prev + (size_t)t * stride, u + (size_t)t * stride, s,
                    seg_out + (size_t)t * L * SEG_STRIDE, threadIdx.x, blockDim.x, [] { __syncthreads(); });
}


// ---------------------------------------------------------------------
// plain path
// ---------------------------------------------------------------------
// float64 solves need more registers than a 512-thread block leaves a wave
template <typename SR>
struct StepBounds {
    static constexpr int threads = sizeof(SR) == 8 ? 256 : 512;
};

// EQ3: the observation of Eq. 3 (cost_mode 1) compiled in; the default
// force-only kernels carry none of its registers.  SDF: links against the
// object's distance field (collision_mode 1).  SEGIN: the step's hand
// segments come from k_hand_fk (in seg_out) instead of every wavefront's own
// hand kinematics -- the same bits, one evaluation per step instead of one
// per simulation, for launches that fill the GPU
template <typename SR, bool EQ3, bool SDF = false, bool SEGIN = false>
__global__ __launch_bounds__(StepBounds<SR>::threads) void k_step(Consts P, Tables tb,
                                               const float *__restrict__ u_prev, const float *__restrict__ u,
                                               float *__restrict__ state, float *__restrict__ params,
                                               float *__restrict__ warm, float *__restrict__ contacts,
                                               float *__restrict__ cslip, float *__restrict__ seg_out,
                                               int64_t *__restrict__ stats)
{
    extern __shared__ __align__(16) char smem[];
    // the simulation index is wave-uniform: its per-simulation loads go
    // through scalar registers
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int e = xcd_block(blockIdx.x, gridDim.x) * (blockDim.x / WAVE) + wib;
    if (e >= P.K) return;
    WaveLds lds = carve_lds(smem, wib, P.max_cand, SEGIN ? 0 : P.L);
    const int type = tb.env_type[e];
    const int S = tb.n_spheres[type];
    const float *sph = tb.spheres + (size_t)type * P.S_max * 4;
    const float inv[3] = {tb.inv_inertia[3 * type], tb.inv_inertia[3 * type + 1], tb.inv_inertia[3 * type + 2]};
    const float rows = load_body_rows(state, params, P.K, e);
    int wkey;
    float wr[3];
    load_warm(warm, P.C_max, e, wkey, wr);
    // otherwise every wavefront evaluates the step's hand kinematics itself
    // (the candidate list's LDS as scratch), while its state loads are in
    // flight: no launch of its own on the per-step path, and the same bits
    // as k_hand_fk
    if (!SEGIN)
        hand_kinematics(tb.hand, P.L, P.D, P.dt, u_prev, u,
                        carve_fk(reinterpret_cast<char *>(lds.cand_d), P.L, P.D), lds.seg, lane_id(), WAVE,
                        [] { wave_sync(); });
    Body B;
    body_from_rows(rows, B);
    const float *seg = SEGIN ? seg_out : lds.seg;
    StepStats st = {0, 0, 0};
    int link;
    float imp[3];
    StepState<SR> sst;
    SdfRef sdf;
    if (SDF) {
        sdf.v = tb.sdf + (size_t)type * P.sdf_n * P.sdf_n * P.sdf_n;
        sdf.box = tb.sdf_box + 4 * type;
        sdf.n = P.sdf_n;
        sdf.M = P.link_samples;
    }
    step_setup<SR, SDF>(P, seg, sph, S, inv, B, wkey, wr, lds, st, sst, sdf);
    step_solve<SR, true>(P, sst, B.mu, inv, reinterpret_cast<SR *>(lds.cand_d));
    step_finish<SR>(P, sst, inv, B, wkey, wr, link, imp);
    const int lane = lane_id();
    if (EQ3) {
        // Eq. 3's slip data of every contact, and the step's segments (one
        // wavefront) for the observation kernel
        float rec[SLIP_STRIDE];
        slip_record<SR>(sst, seg, B.w, rec);
        if (lane < P.C_max) {
            float4 *o = reinterpret_cast<float4 *>(cslip + ((size_t)e * P.C_max + lane) * SLIP_STRIDE);
            o[0] = make_float4(rec[0], rec[1], rec[2], rec[3]);
            o[1] = make_float4(rec[4], rec[5], rec[6], rec[7]);
        }
        if (!SEGIN && e == 0)
            for (int i = lane; i < P.L * SEG_STRIDE; i += WAVE) seg_out[i] = seg[i];
    }
    store_body(state, params, P.K, e, B);
    store_warm(warm, P.C_max, e, wkey, wr);
    if (lane < P.C_max)
        *reinterpret_cast<float4 *>(contacts + ((size_t)e * P.C_max + lane) * 4) =
            make_float4(__int_as_float(link), imp[0], imp[1], imp[2]);
    flush_stats(stats, st, 1, e);
}

// one wavefront per simulation, lanes over sensors
// (cost_mode 1: the seven rows of Eq. 3's observation, from the contacts'
// slip records and the step's segments)
__global__ __launch_bounds__(256) void k_observe(Consts P, const float *__restrict__ contacts,
                                                 const float *__restrict__ cslip, const float *__restrict__ seg,
                                                 float *__restrict__ obs)
{
    __shared__ __align__(16) float stage[4][WAVE * 4];
    __shared__ __align__(16) float slip[4][WAVE * SLIP_STRIDE];
    const int wib = threadIdx.x / WAVE;
    const int e = xcd_block(blockIdx.x, gridDim.x) * (blockDim.x / WAVE) + wib;
    if (e >= P.K) return;
    const int lane = lane_id();
    float *sg = stage[wib];
    float *sl = slip[wib];
    const bool eq3 = P.cost_mode == 1;
    if (lane < P.C_max) {
        *reinterpret_cast<float4 *>(sg + 4 * lane) =
            *reinterpret_cast<const float4 *>(contacts + ((size_t)e * P.C_max + lane) * 4);
        if (eq3) {
            const float4 *src = reinterpret_cast<const float4 *>(cslip + ((size_t)e * P.C_max + lane) * SLIP_STRIDE);
            *reinterpret_cast<float4 *>(sl + SLIP_STRIDE * lane) = src[0];
            *reinterpret_cast<float4 *>(sl + SLIP_STRIDE * lane + 4) = src[1];
        }
    }
    wave_sync();
    const size_t LK = (size_t)P.L * P.K;
    float o[7];
    const bool sensor = eq3 ? sensor_obs_eq3(P, sg, sl, seg, o) : sensor_force(P, sg, o);
    if (sensor) {
        const int R = eq3 ? 7 : 4;
#pragma unroll
        for (int j = 0; j < 7; ++j)
            if (j < R) obs[j * LK + (size_t)lane * P.K + e] = o[j];
    }
}


// one thread per simulation, its sensors' terms summed in sensor order (the
// order of step_cost_wave, so the plain and batched paths add the same
// bits); obs_gt is [R][L][G] (the observed batch's own observation layout)
// (R = 4: force rows; R = 7: the rows of Eq. 3)
constexpr int COST_THREADS = 256;
template <int R>
__global__ __launch_bounds__(COST_THREADS) void k_cost(Consts P, const int32_t *__restrict__ group_of,
                                                       const int32_t *__restrict__ group_start,
                                                       const float *__restrict__ obs,
                                                       const float *__restrict__ obs_gt, float *cost_sum,
                                                       int32_t *__restrict__ best, int32_t *done)
{
    const int e = blockIdx.x * COST_THREADS + threadIdx.x;
    __shared__ float csum[COST_THREADS];
    if (e < P.K) {
        const int g = P.G == 1 ? 0 : group_of[e];
        const size_t LK = (size_t)P.L * P.K, LG = (size_t)P.L * P.G;
        constexpr bool eq3 = R == 7;
        const float prev = cost_sum[e];
        float cs = 0.f;
        // CH sensors' loads in flight at a time, then their terms in order
        constexpr int CH = eq3 ? 8 : 16;
        for (int l0 = 0; l0 < P.L; l0 += CH) {
            float o[CH][R], gt[CH][R];
            // the simulation's own rows first: they do not wait for g
#pragma unroll
            for (int c = 0; c < CH; ++c)
#pragma unroll
                for (int j = 0; j < R; ++j)
                    o[c][j] = l0 + c < P.L ? obs[j * LK + (size_t)(l0 + c) * P.K + e] : 0.f;
#pragma unroll
            for (int c = 0; c < CH; ++c)
#pragma unroll
                for (int j = 0; j < R; ++j)
                    gt[c][j] = l0 + c < P.L ? obs_gt[j * LG + (size_t)(l0 + c) * P.G + g] : 0.f;
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (l0 + c < P.L) {
                    if constexpr (eq3) cs += sensor_cost_eq3(P, o[c], gt[c]);
                    else cs += sensor_cost(P, o[c], gt[c]);
                }
        }
        cost_sum[e] = prev + cs;
        csum[threadIdx.x] = prev + cs;
    }
    // with `best`: the workgroup that finishes last ranks every group (Eq. 2);
    // a single workgroup ranks its own sums from LDS, with no counter
    __shared__ float sv[16];
    __shared__ int si[17];
    if (!best) return;
    if (gridDim.x == 1) {
        __syncthreads();
        block_argmin(P.G, group_start, csum, best, sv, si);
    } else if (last_block(done, si + 16)) {
        block_argmin(P.G, group_start, cost_sum, best, sv, si);
        if (threadIdx.x == 0) *done = 0;
    }
}

// one block per group: lowest index of the minimum, NaN ranked as +inf
__global__ void k_argmin(const int32_t *__restrict__ group_start, const float *__restrict__ cost,
                         int32_t *__restrict__ best)
{
    __shared__ float sv[16];
    __shared__ int si[16];
    block_argmin(1, group_start + blockIdx.x, cost, best + blockIdx.x, sv, si);
}

// ---------------------------------------------------------------------
// population-based resampling
// ---------------------------------------------------------------------
// copy item i of a resample (i < nr: simulation kb + i / rows of the sorted
// group, row or slot i % rows) read from its parent / written to the child
__device__ __forceinline__ float state_row_src(const float *state, int K, int kb, const int *par, int nr, int i)
{
    if (i >= nr * 13) return 0.f;
    const int t = kb + i / 13, c = i - (i / 13) * 13;
    return state[(size_t)c * K + par[t]];
}
__device__ __forceinline__ void state_row_dst(float *state, int K, int lo, int kb, const int *order, int nr, int i,
                                              float v)
{
    if (i >= nr * 13) return;
    const int t = kb + i / 13, c = i - (i / 13) * 13;
    state[(size_t)c * K + lo + order[t]] = v;
}
__device__ __forceinline__ float4 warm_slot_src(const float4 *w4, int C, int kb, const int *par, int nr, int i)
{
    if (i >= nr * C) return make_float4(0.f, 0.f, 0.f, 0.f);
    const int t = kb + i / C, c = i - (i / C) * C;
    return w4[(size_t)par[t] * C + c];
}
__device__ __forceinline__ void warm_slot_dst(float4 *w4, int C, int lo, int kb, const int *order, int nr, int i,
                                              float4 v)
{
    if (i >= nr * C) return;
    const int t = kb + i / C, c = i - (i / C) * C;
    w4[(size_t)(lo + order[t]) * C + c] = v;
}

// one block per group; sorts by (cost, index), then copies and perturbs
__global__ __launch_bounds__(1024) void k_resample(Consts P, ResampleArgs R, const int32_t *__restrict__ group_start,
                                                   uint32_t window_idx, float *__restrict__ cost_sum,
                                                   float *__restrict__ state, float *__restrict__ params,
                                                   float *__restrict__ warm, int32_t *__restrict__ parent)
{
    extern __shared__ __align__(16) char smem[];
    const int g = blockIdx.x;
    const int lo = group_start[g], hi = group_start[g + 1];
    const int n = hi - lo;
    const int np2 = sort_slots(n);
    float *cs = reinterpret_cast<float *>(smem);
    int *order = reinterpret_cast<int *>(smem + 4 * (size_t)np2);
    sort_group(cost_sum + lo, n, np2, cs, order);
    const int kb = elite_count(n, R.elite_frac);
    const uint32_t key0 = (uint32_t)(R.seed & 0xffffffffu), key1 = (uint32_t)(R.seed >> 32);
    const int K = P.K;
    // parents by rank (the sorted costs' LDS is free after the sort); the
    // parents are elites, never overwritten, so every copy below is
    // independent of the others
    int *par = reinterpret_cast<int *>(cs);
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const int j = lo + order[t];
        if (t < kb) {
            if (parent) parent[j] = -1;
            continue;
        }
        uint32_t w[4];
        philox4x32_10((uint32_t)j, window_idx, 0u, 0u, key0, key1, w);
        const int prank = (int)(((uint64_t)w[0] * (uint64_t)kb) >> 32);
        const int p = lo + order[prank];
        par[t] = p;
        if (parent) parent[j] = p;
        float e[5];
        explore(R, (uint32_t)j, window_idx, params[0 * (size_t)K + p], params[1 * (size_t)K + p], e);
        for (int c = 0; c < 5; ++c) params[(size_t)c * K + j] = e[c];
    }
    __syncthreads();
    // state rows and warm-cache slots, one (simulation, row or slot) per
    // thread, four of them loaded before any is stored (the copies read only
    // elites, which nothing here writes)
    const int nr = n - kb;
    const int nt = blockDim.x;
    for (int i0 = threadIdx.x; i0 < nr * 13; i0 += 4 * nt) {
        const int i1 = i0 + nt, i2 = i0 + 2 * nt, i3 = i0 + 3 * nt;
        const float v0 = state_row_src(state, K, kb, par, nr, i0);
        const float v1 = state_row_src(state, K, kb, par, nr, i1);
        const float v2 = state_row_src(state, K, kb, par, nr, i2);
        const float v3 = state_row_src(state, K, kb, par, nr, i3);
        state_row_dst(state, K, lo, kb, order, nr, i0, v0);
        state_row_dst(state, K, lo, kb, order, nr, i1, v1);
        state_row_dst(state, K, lo, kb, order, nr, i2, v2);
        state_row_dst(state, K, lo, kb, order, nr, i3, v3);
    }
    float4 *w4 = reinterpret_cast<float4 *>(warm);
    const int C = P.C_max;
    for (int i0 = threadIdx.x; i0 < nr * C; i0 += 4 * nt) {
        const int i1 = i0 + nt, i2 = i0 + 2 * nt, i3 = i0 + 3 * nt;
        const float4 v0 = warm_slot_src(w4, C, kb, par, nr, i0);
        const float4 v1 = warm_slot_src(w4, C, kb, par, nr, i1);
        const float4 v2 = warm_slot_src(w4, C, kb, par, nr, i2);
        const float4 v3 = warm_slot_src(w4, C, kb, par, nr, i3);
        warm_slot_dst(w4, C, lo, kb, order, nr, i0, v0);
        warm_slot_dst(w4, C, lo, kb, order, nr, i1, v1);
        warm_slot_dst(w4, C, lo, kb, order, nr, i2, v2);
        warm_slot_dst(w4, C, lo, kb, order, nr, i3, v3);
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) cost_sum[lo + i] = 0.f;
}

// ---------------------------------------------------------------------
// batched path: persistent kernel over a window of T steps
// ---------------------------------------------------------------------
// (the Eq. 3 kernel for large caps, a few registers over what two
// wavefronts per SIMD leave, is held to two with a small spill: ~12% more
// throughput on the 16384-simulation workload)
// SDF: links against the object's distance field (collision_mode 1)
template <typename SR, bool EQ3, bool PT, bool SDF = false>
__global__ __launch_bounds__(StepBounds<SR>::threads) __attribute__((amdgpu_waves_per_eu(!PT ? 2 : 1))) void
k_window(Consts P, Tables tb, const float *__restrict__ seg_win, float *__restrict__ state,
         float *__restrict__ params, float *__restrict__ warm, const float *__restrict__ obs_gt_win,
         float *__restrict__ cost_sum, float *__restrict__ obs_out, const int32_t *__restrict__ env_order,
         int32_t *queue, int64_t *__restrict__ stats, float *__restrict__ ckpt,
         const int32_t *__restrict__ group_start, int32_t *__restrict__ best)
{
    extern __shared__ __align__(16) char smem[];
    const int wib = threadIdx.x / WAVE;
    const int lane = lane_id();
    WaveLds lds = carve_lds(smem, wib, P.max_cand, 0);
    float *stage = contact_stage(lds);
    StepStats st = {0, 0, 0};
    int64_t done = 0;
    const size_t LK = (size_t)P.L * P.K, LG = (size_t)P.L * P.G;
    for (;;) {
        int slot = 0;
        if (lane == 0) slot = atomicAdd(queue, 1);
        slot = __builtin_amdgcn_readfirstlane(slot);
        if (slot >= P.K) break;
        const int e = env_order[slot];
        const int type = tb.env_type[e];
        const int g = tb.group_of[e];
        const int S = tb.n_spheres[type];
        const float *sph = tb.spheres + (size_t)type * P.S_max * 4;
        const float inv[3] = {tb.inv_inertia[3 * type], tb.inv_inertia[3 * type + 1], tb.inv_inertia[3 * type + 2]};
        SdfRef sdf;
        if (SDF) {
            sdf.v = tb.sdf + (size_t)type * P.sdf_n * P.sdf_n * P.sdf_n;
            sdf.box = tb.sdf_box + 4 * type;
            sdf.n = P.sdf_n;
            sdf.M = P.link_samples;
        }
        Body B;
        load_body(state, params, P.K, e, B);
        int wkey;
        float wr[3];
        load_warm(warm, P.C_max, e, wkey, wr);
        // running sum continued step by step, in the order the plain path adds
        float cost = cost_sum[e];
        for (int t = 0; t < P.T; ++t) {
            int link;
            float imp[3];
            // with a checkpoint buffer: the body before the step and the kept
            // contacts' keys and impulses after its solve, per simulation
            const float *seg = seg_win + (size_t)t * P.L * SEG_STRIDE;
            float *ck = ckpt ? ckpt + ((size_t)e * P.T + t) * ckpt_step_floats(P.C_max) : nullptr;
            if (ck) save_body(ck, B);
            StepState<SR> sst;
            step_setup<SR, SDF>(P, seg, sph, S, inv, B, wkey, wr, lds, st, sst, sdf);
            step_solve<SR, PT>(P, sst, B.mu, inv, reinterpret_cast<SR *>(lds.cand_d));
            if (ck) save_contact<SR>(ck, P.C_max, sst);
            step_finish<SR>(P, sst, inv, B, wkey, wr, link, imp);
            uniform_body(B);
            *reinterpret_cast<float4 *>(stage + 4 * lane) = make_float4(__int_as_float(link), imp[0], imp[1], imp[2]);
            // Eq. 3 (cost_mode 1): the contacts' slip records staged in the
            // candidate list's LDS, free between the solve and the next
            // step's narrow phase
            float *slip = lds.cand_d;
            if constexpr (EQ3) {
                float rec[SLIP_STRIDE];
                slip_record<SR>(sst, seg, B.w, rec);
                *reinterpret_cast<float4 *>(slip + SLIP_STRIDE * lane) = make_float4(rec[0], rec[1], rec[2], rec[3]);
                *reinterpret_cast<float4 *>(slip + SLIP_STRIDE * lane + 4) = make_float4(rec[4], rec[5], rec[6], rec[7]);
            }
            wave_sync();
            float cl = 0.f;
            if constexpr (EQ3) {
                float o[7];
                if (sensor_obs_eq3(P, stage, slip, seg, o)) {
                    const float *gt = obs_gt_win + (size_t)t * 7 * LG;
                    float gv[7];
#pragma unroll
                    for (int j = 0; j < 7; ++j) gv[j] = gt[j * LG + (size_t)lane * P.G + g];
                    cl = sensor_cost_eq3(P, o, gv);
                    if (obs_out) {
                        float *ob = obs_out + (size_t)t * 7 * LK;
#pragma unroll
                        for (int j = 0; j < 7; ++j) ob[j * LK + (size_t)lane * P.K + e] = o[j];
                    }
                }
            } else {
                float o[4];
                if (sensor_force(P, stage, o)) {
                    const float *gt = obs_gt_win + (size_t)t * 4 * LG;
                    float gv[4] = {gt[0 * LG + (size_t)lane * P.G + g], gt[1 * LG + (size_t)lane * P.G + g],
                                   gt[2 * LG + (size_t)lane * P.G + g], gt[3 * LG + (size_t)lane * P.G + g]};
                    cl = sensor_cost(P, o, gv);
                    if (obs_out) {
                        float *ob = obs_out + (size_t)t * 4 * LK;
                        ob[0 * LK + (size_t)lane * P.K + e] = o[0];
                        ob[1 * LK + (size_t)lane * P.K + e] = o[1];
                        ob[2 * LK + (size_t)lane * P.K + e] = o[2];
                        ob[3 * LK + (size_t)lane * P.K + e] = o[3];
                    }
                }
            }
            wave_sync();
            // step cost summed over sensors in sensor order
            cost += step_cost_wave(P, cl);
        }
        store_body(state, params, P.K, e, B);
        store_warm(warm, P.C_max, e, wkey, wr);
        if (lane == 0) cost_sum[e] = cost;
        done += P.T;
    }
    flush_stats(stats, st, done, blockIdx.x * (blockDim.x / WAVE) + wib);
    // the workgroup that finishes last ranks every group (Eq. 2) and puts the
    // work queue back to 0 for the next window
    // (the block's dynamic LDS is free once every wave has left the loop)
    float *sv = reinterpret_cast<float *>(smem);
    int *si = reinterpret_cast<int *>(smem) + 16;
    if (last_block(queue + 1, si + 16)) {
        if (best) block_argmin(P.G, group_start, cost_sum, best, sv, si);
        if (threadIdx.x == 0) { queue[0] = 0; queue[1] = 0; }
    }
}

}  // namespace pt

// ---------------------------------------------------------------------
// launch wrappers (host side)
// ---------------------------------------------------------------------
using namespace pt;

size_t hand_fk_lds_bytes(int L, int D) { return fk_lds_bytes(L, D); }

hipError_t launch_hand_fk(const float *hand, int L, int D, float dt, const float *u_prev, const float *u,
                          int stride, int nsteps, float *seg_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_hand_fk, dim3(nsteps), dim3(128), 0, s, hand, L, D, dt, u_prev, u, stride, seg_out);
    return hipGetLastError();
}

hipError_t launch_step(const Consts &P, const Tables &tb, const float *u_prev, const float *u, float *state,
                       float *params, float *warm, float *contacts, float *cslip, float *seg_out, int64_t *stats,
                       int waves_per_block, bool seg_in, hipStream_t s)
{
    int blocks = (P.K + waves_per_block - 1) / waves_per_block;
    seg_in = seg_in && P.solve_fp64;
    size_t lds = (size_t)waves_per_block * wave_lds_bytes(P.max_cand, seg_in ? 0 : P.L);
    const dim3 grid(blocks), block(WAVE * waves_per_block);
    const bool eq3 = P.cost_mode == 1;
    if (seg_in) {
        if (P.collision_mode == 1)
            hipLaunchKernelGGL((k_step<double, false, true, true>), grid, block, lds, s, P, tb, u_prev, u, state,
                               params, warm, contacts, cslip, seg_out, stats);
        else if (!eq3)
            hipLaunchKernelGGL((k_step<double, false, false, true>), grid, block, lds, s, P, tb, u_prev, u, state,
                               params, warm, contacts, cslip, seg_out, stats);
        else
            hipLaunchKernelGGL((k_step<double, true, false, true>), grid, block, lds, s, P, tb, u_prev, u, state,
                               params, warm, contacts, cslip, seg_out, stats);
    } else if (P.collision_mode == 1)   // float64 solve and force terms only (checked at batch creation)
        hipLaunchKernelGGL((k_step<double, false, true>), grid, block, lds, s, P, tb, u_prev, u, state, params,
                           warm, contacts, cslip, seg_out, stats);
    else if (P.solve_fp64 && !eq3)
        hipLaunchKernelGGL((k_step<double, false>), grid, block, lds, s, P, tb, u_prev, u, state, params, warm,
                           contacts, cslip, seg_out, stats);
    else if (P.solve_fp64)
        hipLaunchKernelGGL((k_step<double, true>), grid, block, lds, s, P, tb, u_prev, u, state, params, warm,
                           contacts, cslip, seg_out, stats);
    else if (!eq3)
        hipLaunchKernelGGL((k_step<float, false>), grid, block, lds, s, P, tb, u_prev, u, state, params, warm,
                           contacts, cslip, seg_out, stats);
    else
        hipLaunchKernelGGL((k_step<float, true>), grid, block, lds, s, P, tb, u_prev, u, state, params, warm,
                           contacts, cslip, seg_out, stats);
    return hipGetLastError();
}

hipError_t launch_observe(const Consts &P, const float *contacts, const float *cslip, const float *seg, float *obs,
                          hipStream_t s)
{
    int blocks = (P.K + 3) / 4;
    hipLaunchKernelGGL(k_observe, dim3(blocks), dim3(256), 0, s, P, contacts, cslip, seg, obs);
    return hipGetLastError();
}

hipError_t launch_cost(const Consts &P, const int32_t *group_of, const int32_t *group_start, const float *obs,
                       const float *obs_gt, float *cost_sum, int32_t *best, int32_t *done, hipStream_t s)
{
    int blocks = (P.K + COST_THREADS - 1) / COST_THREADS;
    if (P.cost_mode == 1)
        hipLaunchKernelGGL(k_cost<7>, dim3(blocks), dim3(COST_THREADS), 0, s, P, group_of, group_start, obs, obs_gt,
                           cost_sum, best, done);
    else
        hipLaunchKernelGGL(k_cost<4>, dim3(blocks), dim3(COST_THREADS), 0, s, P, group_of, group_start, obs, obs_gt,
                           cost_sum, best, done);
    return hipGetLastError();
}

hipError_t launch_argmin(int G, const int32_t *group_start, const float *cost, int32_t *best, hipStream_t s)
{
    hipLaunchKernelGGL(k_argmin, dim3(G), dim3(1024), 0, s, group_start, cost, best);
    return hipGetLastError();
}

hipError_t launch_resample(const Consts &P, const ResampleArgs &R, const int32_t *group_start, int max_group,
                           uint32_t window_idx, float *cost_sum, float *state, float *params, float *warm,
                           int32_t *parent, hipStream_t s)
{
    size_t lds = resample_lds_bytes(max_group);
    hipLaunchKernelGGL(k_resample, dim3(P.G), dim3(group_threads(max_group)), lds, s, P, R, group_start, window_idx,
                       cost_sum, state, params, warm, parent);
    return hipGetLastError();
}

// the window kernel for a batch: solve precision, cost mode, and the paired
// line-search trials when no step can hold more than 32 contacts (C_max <=
// 32: latency-bound populations, where the extra registers cost nothing);
// the distance-field collision with the float64 solve and the force terms
// only (checked at batch creation)
template <typename F>
static hipError_t with_window_kernel(const Consts &P, F f)
{
    const bool eq3 = P.cost_mode == 1, pt = P.C_max <= 32;
    if (P.collision_mode == 1) return pt ? f(k_window<double, false, true, true>) : f(k_window<double, false, false, true>);
    if (P.solve_fp64) {
        if (eq3) return pt ? f(k_window<double, true, true>) : f(k_window<double, true, false>);
        return pt ? f(k_window<double, false, true>) : f(k_window<double, false, false>);
    }
    if (eq3) return pt ? f(k_window<float, true, true>) : f(k_window<float, true, false>);
    return pt ? f(k_window<float, false, true>) : f(k_window<float, false, false>);
}

hipError_t launch_window(const Consts &P, const Tables &tb, const float *seg_win, float *state, float *params,
                         float *warm, const float *obs_gt_win, float *cost_sum, float *obs_out,
                         const int32_t *env_order, int32_t *queue, int64_t *stats, int waves_per_block, int blocks,
                         float *ckpt, const int32_t *group_start, int32_t *best, hipStream_t s)
{
    size_t lds = (size_t)waves_per_block * wave_lds_bytes(P.max_cand, 0);
    const dim3 grid(blocks), block(WAVE * waves_per_block);
    return with_window_kernel(P, [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, block, lds, s, P, tb, seg_win, state, params, warm, obs_gt_win, cost_sum,
                           obs_out, env_order, queue, stats, ckpt, group_start, best);
        return hipGetLastError();
    });
}

hipError_t window_occupancy(const Consts &P, int waves_per_block, int *blocks_per_cu)
{
    size_t lds = (size_t)waves_per_block * wave_lds_bytes(P.max_cand, 0);
    return with_window_kernel(P, [&](auto kern) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, reinterpret_cast<const void *>(kern),
                                                            WAVE * waves_per_block, lds);
    });
}

hipError_t set_lds_limits(size_t bytes)
{
    const void *fs[] = {reinterpret_cast<const void *>(k_window<float, false, false>),
                        reinterpret_cast<const void *>(k_window<double, false, false>),
                        reinterpret_cast<const void *>(k_window<float, true, false>),
                        reinterpret_cast<const void *>(k_window<double, true, false>),
                        reinterpret_cast<const void *>(k_window<float, false, true>),
                        reinterpret_cast<const void *>(k_window<double, false, true>),
                        reinterpret_cast<const void *>(k_window<float, true, true>),
                        reinterpret_cast<const void *>(k_window<double, true, true>),
                        reinterpret_cast<const void *>(k_window<double, false, false, true>),
                        reinterpret_cast<const void *>(k_window<double, false, true, true>),
                        reinterpret_cast<const void *>(k_step<float, false>),
                        reinterpret_cast<const void *>(k_step<double, false>),
                        reinterpret_cast<const void *>(k_step<float, true>),
                        reinterpret_cast<const void *>(k_step<double, true>),
                        reinterpret_cast<const void *>(k_step<double, false, true>),
                        reinterpret_cast<const void *>(k_resample)};
    for (const void *f : fs) {
        hipError_t e = set_dynamic_lds_limit(f, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
