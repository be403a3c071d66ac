// pt_io.hpp -- per-simulation helpers shared by the step, window and
// adjoint kernels: workgroup numbering, LDS carving, state and warm-cache
// I/O, sensor forces and the step cost.
#pragma once

#include "pt_internal.h"
#include "pt_step.hpp"

namespace pt {

// Workgroups are dealt round-robin over the 8 XCDs, each with its own L2.
// Renumber them so that consecutive logical workgroups (hence consecutive
// simulations, whose SoA state shares cache lines) run on the same XCD.
constexpr int N_XCD = 8;
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int xcd = b % N_XCD, idx = b / N_XCD;
    const int per = nb / N_XCD, rem = nb % N_XCD;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

__device__ __forceinline__ WaveLds carve_lds(char *base, int wave_in_block, int max_cand, int L)
{
    char *p = base + (size_t)wave_in_block * wave_lds_bytes(max_cand, L);
    WaveLds w;
    w.cand_d = reinterpret_cast<float *>(p);
    w.cand_k = reinterpret_cast<int *>(p + 4 * (size_t)max_cand);
    w.sel = reinterpret_cast<int *>(p + 8 * (size_t)max_cand);
    w.wkey = w.sel + WAVE;
    w.wr = reinterpret_cast<float *>(w.wkey + WAVE);
    w.seg = w.wr + 3 * WAVE + 4 * WAVE;
    return w;
}

__device__ __forceinline__ float *contact_stage(const WaveLds &w) { return w.wr + 3 * WAVE; }  // [64][4]

__device__ __forceinline__ void load_body(const float *__restrict__ state, const float *__restrict__ params, int K,
                                          int e, Body &B)
{
    B.x[0] = state[0 * K + e]; B.x[1] = state[1 * K + e]; B.x[2] = state[2 * K + e];
    B.q[0] = state[3 * K + e]; B.q[1] = state[4 * K + e]; B.q[2] = state[5 * K + e]; B.q[3] = state[6 * K + e];
    B.v[0] = state[7 * K + e]; B.v[1] = state[8 * K + e]; B.v[2] = state[9 * K + e];
    B.w[0] = state[10 * K + e]; B.w[1] = state[11 * K + e]; B.w[2] = state[12 * K + e];
    B.m = params[0 * K + e]; B.mu = params[1 * K + e];
    B.f[0] = params[2 * K + e]; B.f[1] = params[3 * K + e]; B.f[2] = params[4 * K + e];
}

// The body of simulation e spread over the lanes of a wavefront: lane r < 18
// holds row r of the load_body order (13 state rows, then the 5 parameter
// rows).  One vector load covers the whole body, so it is in flight with the
// step's other first loads instead of 18 scalar loads that register
// pressure would wait for a few at a time; body_from_rows reads it out
// (readlane) where the values are needed.
__device__ __forceinline__ float load_body_rows(const float *__restrict__ state, const float *__restrict__ params,
                                                int K, int e)
{
    const int lane = lane_id();
    float v = 0.f;
    if (lane < 13)
        v = state[(size_t)lane * K + e];
    else if (lane < 18)
        v = params[(size_t)(lane - 13) * K + e];
    return v;
}

__device__ __forceinline__ void body_from_rows(float v, Body &B)
{
    float r[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) r[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
    B.x[0] = r[0]; B.x[1] = r[1]; B.x[2] = r[2];
    B.q[0] = r[3]; B.q[1] = r[4]; B.q[2] = r[5]; B.q[3] = r[6];
    B.v[0] = r[7]; B.v[1] = r[8]; B.v[2] = r[9];
    B.w[0] = r[10]; B.w[1] = r[11]; B.w[2] = r[12];
    B.m = r[13]; B.mu = r[14];
    B.f[0] = r[15]; B.f[1] = r[16]; B.f[2] = r[17];
}

__device__ __forceinline__ void store_body(float *__restrict__ state, float *__restrict__ params, int K, int e,
                                           const Body &B)
{
    if (lane_id() == 0) {
        state[0 * K + e] = B.x[0]; state[1 * K + e] = B.x[1]; state[2 * K + e] = B.x[2];
        state[3 * K + e] = B.q[0]; state[4 * K + e] = B.q[1]; state[5 * K + e] = B.q[2]; state[6 * K + e] = B.q[3];
        state[7 * K + e] = B.v[0]; state[8 * K + e] = B.v[1]; state[9 * K + e] = B.v[2];
        state[10 * K + e] = B.w[0]; state[11 * K + e] = B.w[1]; state[12 * K + e] = B.w[2];
        params[2 * K + e] = B.f[0]; params[3 * K + e] = B.f[1]; params[4 * K + e] = B.f[2];
    }
}

__device__ __forceinline__ void load_warm(const float *__restrict__ warm, int C_max, int e, int &wkey, float *wr)
{
    const int lane = lane_id();
    wkey = -1;
    wr[0] = wr[1] = wr[2] = 0.f;
    if (lane < C_max) {
        float4 w = *reinterpret_cast<const float4 *>(warm + ((size_t)e * C_max + lane) * WARM_STRIDE);
        wkey = __float_as_int(w.x);
        wr[0] = w.y; wr[1] = w.z; wr[2] = w.w;
    }
}

__device__ __forceinline__ void store_warm(float *__restrict__ warm, int C_max, int e, int wkey, const float *wr)
{
    const int lane = lane_id();
    if (lane < C_max)
        *reinterpret_cast<float4 *>(warm + ((size_t)e * C_max + lane) * WARM_STRIDE) =
            make_float4(__int_as_float(wkey), wr[0], wr[1], wr[2]);
}

__device__ __forceinline__ void flush_stats(int64_t *stats, const StepStats &st, int64_t steps, int slot)
{
    if (lane_id() == 0) {
        unsigned long long *p =
            reinterpret_cast<unsigned long long *>(stats + (size_t)(slot & (STATS_SLOTS - 1)) * STATS_STRIDE);
        atomicAdd(p + 0, (unsigned long long)steps);
        atomicAdd(p + 1, (unsigned long long)st.cand);
        atomicAdd(p + 2, (unsigned long long)st.contacts);
        atomicAdd(p + 3, (unsigned long long)st.dropped);
    }
}

// per-sensor force from the contacts staged in LDS ([64][4]: link bits,
// impulse on the object), summed in contact order; lane l < L gets
// (|c_l|, c_hat_l).  Returns false on lanes >= L.
__device__ __forceinline__ bool sensor_force(const Consts &P, const float *stage, float *o)
{
    const int lane = lane_id();
    float f0 = 0.f, f1 = 0.f, f2 = 0.f;
    for (int c = 0; c < P.C_max; ++c) {
        const float4 rec = *reinterpret_cast<const float4 *>(stage + 4 * c);
        if (__float_as_int(rec.x) == lane) {
            f0 += rec.y; f1 += rec.z; f2 += rec.w;
        }
    }
    float idt = 1.f / P.dt;
    f0 = -f0 * idt; f1 = -f1 * idt; f2 = -f2 * idt;
    float mag = sqrtf(f0 * f0 + f1 * f1 + f2 * f2);
    bool on = mag > P.tau_contact;
    float im = on ? 1.f / mag : 0.f;
    o[0] = mag; o[1] = on ? f0 * im : 0.f; o[2] = on ? f1 * im : 0.f; o[3] = on ? f2 * im : 0.f;
    return lane < P.L;
}

__device__ __forceinline__ float sensor_cost(const Consts &P, const float *o, const float *gt)
{
    float dm = o[0] - gt[0];
    float d1 = o[1] - gt[1], d2 = o[2] - gt[2], d3 = o[3] - gt[3];
    return P.w_mag * dm * dm + P.w_dir * (d1 * d1 + d2 * d2 + d3 * d3);
}

// ---------------------------------------------------------------------
// the full cost of Eq. 3 (cost_mode 1): contact state, slip and spin
// ---------------------------------------------------------------------
constexpr int SLIP_STRIDE = 8;   // per-contact slip record, floats

// Slip record of this lane's contact after the step: r_n n (3), r_n,
// r_n s (3), q, with s the relative tangential velocity of the object's
// contact point against the link's (the constraint velocity without the
// compliance term, in world axes) and q = r_n (w_obj - w_link) . n, w_link
// = (b - a) x (vb - va) / |b - a|^2 from the link's segment record and
// w_obj the object's angular velocity after the step.  Zeros for an empty
// slot and for a table contact (not a sensor).
template <typename SR>
__device__ __forceinline__ void slip_record(const StepState<SR> &st, const float *seg, const float *w_obj,
                                            float *out)
{
#pragma unroll
    for (int i = 0; i < SLIP_STRIDE; ++i) out[i] = 0.f;
    if (!st.act || st.link < 0) return;
    SR u[3];
    rel_velocity(st, st.nu, st.r, SR(0), u);
    const SR *F = st.F;
    const float rn = (float)st.r[0];
    const float n[3] = {(float)F[0], (float)F[1], (float)F[2]};
    const float sv[3] = {(float)(u[1] * F[3] + u[2] * F[6]), (float)(u[1] * F[4] + u[2] * F[7]),
                         (float)(u[1] * F[5] + u[2] * F[8])};
    const float *sg = seg + st.link * SEG_STRIDE;
    const float ab[3] = {sg[4], sg[5], sg[6]};
    const float dv[3] = {sg[12] - sg[8], sg[13] - sg[9], sg[14] - sg[10]};
    float wl[3];
    cross3(ab, dv, wl);
    const float il2 = sg[7];
    const float q = rn * ((w_obj[0] - wl[0] * il2) * n[0] + (w_obj[1] - wl[1] * il2) * n[1] +
                          (w_obj[2] - wl[2] * il2) * n[2]);
    out[0] = rn * n[0]; out[1] = rn * n[1]; out[2] = rn * n[2]; out[3] = rn;
    out[4] = rn * sv[0]; out[5] = rn * sv[1]; out[6] = rn * sv[2]; out[7] = q;
}

// Eq. 3 observation of sensor `lane` (lanes < L) from the step's staged
// contacts -- stage [C_max][4] (link, impulse), slip [C_max][8] -- and the
// step's segment records: |c|, c/|c| as sensor_force; with n_bar the
// normalised sum r_n n and s = sum r_n s / sum r_n, d = s in the sensor's
// surface frame (e1 = the link axis projected normal to n_bar, or the
// contact-frame rule if the normal runs along the axis; e2 = n_bar x e1),
// normalised, when |s| > tau_slip, else 0; rot = the sign of
// sum q / |sum r_n n| beyond tau_spin, else 0.  o[7].
__device__ __forceinline__ bool sensor_obs_eq3(const Consts &P, const float *stage, const float *slip,
                                               const float *seg, float *o)
{
    const int lane = lane_id();
    const bool sensor = sensor_force(P, stage, o);
    o[4] = o[5] = o[6] = 0.f;
    if (!sensor) return false;
    float N[3] = {0.f, 0.f, 0.f}, S[3] = {0.f, 0.f, 0.f}, W = 0.f, Q = 0.f;
    for (int c = 0; c < P.C_max; ++c) {
        if (__float_as_int(stage[4 * c]) != lane) continue;
        const float4 a = *reinterpret_cast<const float4 *>(slip + SLIP_STRIDE * c);
        const float4 b = *reinterpret_cast<const float4 *>(slip + SLIP_STRIDE * c + 4);
        N[0] += a.x; N[1] += a.y; N[2] += a.z; W += a.w;
        S[0] += b.x; S[1] += b.y; S[2] += b.z; Q += b.w;
    }
    const float nn = sqrtf(dot3(N, N));
    if (!(W > 0.f) || !(nn > 0.f)) return true;
    const float nb[3] = {N[0] / nn, N[1] / nn, N[2] / nn};
    const float sl[3] = {S[0] / W, S[1] / W, S[2] / W};
    if (sqrtf(dot3(sl, sl)) > P.tau_slip) {
        const float *sg = seg + lane * SEG_STRIDE;
        const float la = sqrtf(sg[4] * sg[4] + sg[5] * sg[5] + sg[6] * sg[6]);
        const float ea[3] = {sg[4] / la, sg[5] / la, sg[6] / la};
        const float an = dot3(ea, nb);
        float e1[3] = {ea[0] - an * nb[0], ea[1] - an * nb[1], ea[2] - an * nb[2]}, e2[3];
        const float n1 = sqrtf(dot3(e1, e1));
        if (n1 < 1e-6f) {
            tangent_frame(nb, e1, e2);
        } else {
            e1[0] /= n1; e1[1] /= n1; e1[2] /= n1;
            cross3(nb, e1, e2);
        }
        const float d1 = dot3(sl, e1), d2 = dot3(sl, e2);
        const float dn = sqrtf(d1 * d1 + d2 * d2);
        if (dn > 0.f) { o[4] = d1 / dn; o[5] = d2 / dn; }
    }
    const float spin = Q / nn;
    o[6] = spin > P.tau_spin ? 1.f : (spin < -P.tau_spin ? -1.f : 0.f);
    return true;
}

// angle between two unit vectors of n components, 2 atan2(|a - b|, |a + b|)
// (no loss of accuracy near 0 or pi)
__device__ __forceinline__ float unit_angle(const float *a, const float *b, int n)
{
    float dm = 0.f, dp = 0.f;
    for (int i = 0; i < n; ++i) {
        dm += (a[i] - b[i]) * (a[i] - b[i]);
        dp += (a[i] + b[i]) * (a[i] + b[i]);
    }
    return 2.f * atan2f(sqrtf(dm), sqrtf(dp));
}

// Eq. 3 cost of one sensor: w4 (1 - alpha) + alpha (w5 |dM| + w6 angle of
// the forces when in contact) + w7 (1 - beta) + beta w8 angle of the slip
// directions when slipping + w9 (1 - gamma) + gamma w10 |r - r_gt| when
// spinning (r = 1 for a positive spin); alpha, beta, gamma the agreement of
// the contact, slip and spin states
__device__ __forceinline__ float sensor_cost_eq3(const Consts &P, const float *o, const float *gt)
{
    const float *w = P.w_eq3;
    const bool in_a = o[0] > P.tau_contact, in_b = gt[0] > P.tau_contact;
    const bool sl_a = o[4] != 0.f || o[5] != 0.f, sl_b = gt[4] != 0.f || gt[5] != 0.f;
    const bool ro_a = o[6] != 0.f, ro_b = gt[6] != 0.f;
    float c = 0.f;
    if (in_a == in_b) {
        c += w[1] * fabsf(o[0] - gt[0]);
        if (in_a) c += w[2] * unit_angle(o + 1, gt + 1, 3);
    } else {
        c += w[0];
    }
    if (sl_a == sl_b) {
        if (sl_a) c += w[4] * unit_angle(o + 4, gt + 4, 2);
    } else {
        c += w[3];
    }
    if (ro_a == ro_b) {
        if (ro_a) c += w[6] * fabsf((o[6] > 0.f ? 1.f : 0.f) - (gt[6] > 0.f ? 1.f : 0.f));
    } else {
        c += w[5];
    }
    return c;
}

// step cost of one simulation from its sensors' terms held one per lane
// (lane l < L), summed in sensor order; shared by the plain and batched paths
__device__ __forceinline__ float step_cost_wave(const Consts &P, float cl)
{
    float cs = 0.f;
    for (int l = 0; l < P.L; ++l) cs += bcast_lane(cl, l);
    return cs;
}

// checkpoint of one step of one simulation: body record x(3) q(4) v(3) w(3)
// f(3) (16 floats), then per contact slot r(3) and key as 4 doubles
constexpr int CK_BODY = 16;
__host__ __device__ constexpr size_t ckpt_step_floats(int C_max) { return CK_BODY + 8 * (size_t)C_max; }

__device__ __forceinline__ void save_body(float *__restrict__ ck, const Body &B)
{
    if (lane_id() == 0) {
        float4 *b4 = reinterpret_cast<float4 *>(ck);
        b4[0] = make_float4(B.x[0], B.x[1], B.x[2], B.q[0]);
        b4[1] = make_float4(B.q[1], B.q[2], B.q[3], B.v[0]);
        b4[2] = make_float4(B.v[1], B.v[2], B.w[0], B.w[1]);
        b4[3] = make_float4(B.w[2], B.f[0], B.f[1], B.f[2]);
    }
}

__device__ __forceinline__ void load_body_ckpt(const float *__restrict__ ck, Body &B)
{
    const float4 *b4 = reinterpret_cast<const float4 *>(ck);
    float4 a = b4[0], b = b4[1], c = b4[2], d = b4[3];
    B.x[0] = a.x; B.x[1] = a.y; B.x[2] = a.z; B.q[0] = a.w;
    B.q[1] = b.x; B.q[2] = b.y; B.q[3] = b.z; B.v[0] = b.w;
    B.v[1] = c.x; B.v[2] = c.y; B.w[0] = c.z; B.w[1] = c.w;
    B.w[2] = d.x; B.f[0] = d.y; B.f[1] = d.z; B.f[2] = d.w;
}

template <typename SR>
__device__ __forceinline__ void save_contact(float *__restrict__ ck, int C_max, const StepState<SR> &st)
{
    const int lane = lane_id();
    if (lane < C_max) {
        double2 *d2 = reinterpret_cast<double2 *>(ck + CK_BODY) + 2 * lane;
        d2[0] = make_double2((double)st.r[0], (double)st.r[1]);
        d2[1] = make_double2((double)st.r[2], (double)(st.act ? st.key : -1));
    }
}

template <typename SR>
__device__ __forceinline__ int load_contact(const float *__restrict__ ck, int C_max, SR *r)
{
    const int lane = lane_id();
    r[0] = r[1] = r[2] = SR(0);
    if (lane >= C_max) return -1;
    const double2 *d2 = reinterpret_cast<const double2 *>(ck + CK_BODY) + 2 * lane;
    double2 a = d2[0], b = d2[1];
    r[0] = (SR)a.x; r[1] = (SR)a.y; r[2] = (SR)b.x;
    return (int)b.y;
}

// One group's simulations in (cost, index) order, NaN ranked as +inf: a
// bitonic sort in LDS over np2 slots (a power of two >= n, padding (+inf,
// index >= n) sorts after every real entry).  All threads of the block take
// part; afterwards ix[0..n) holds the group's local indices in order.
__device__ __forceinline__ void sort_group(const float *__restrict__ cost, int n, int np2, float *cs, int *ix)
{
    for (int i = threadIdx.x; i < np2; i += blockDim.x) {
        const float v = i < n ? cost[i] : __int_as_float(0x7f800000);
        cs[i] = (v != v) ? __int_as_float(0x7f800000) : v;
        ix[i] = i;
    }
    __syncthreads();
    for (int k = 2; k <= np2; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < np2; i += blockDim.x) {
                const int p = i ^ j;
                if (p > i) {
                    const float ci = cs[i], cp = cs[p];
                    const int xi = ix[i], xp = ix[p];
                    // entries are distinct (indices are), so "after" is strict
                    const bool after = ci > cp || (ci == cp && xi > xp);
                    if (after == ((i & k) == 0)) {
                        cs[i] = cp; cs[p] = ci;
                        ix[i] = xp; ix[p] = xi;
                    }
                }
            }
            // a stage with j < WAVE stays inside each wavefront's 64-index
            // blocks (blockDim is a multiple of WAVE, so one wavefront owns
            // a block), where the wavefront's own LDS order suffices; a
            // workgroup barrier only around the stages that cross them
            const int jn = j > 1 ? j >> 1 : k;   // the next stage's j
            if (j >= WAVE || (jn >= WAVE && k < np2)) __syncthreads();
            else wave_sync();
        }
    __syncthreads();
}

// True in every thread of the workgroup that arrives last among the grid's
// workgroups, counted on *done (0 before the launch); that workgroup sees the
// global writes every other one made before its call.  The caller's last
// workgroup puts *done back to 0 for the next launch.  Every thread of every
// workgroup calls it once.  flag: one int of LDS, free for the call.
__device__ __forceinline__ bool last_block(int32_t *done, int *flag)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *flag = atomicAdd(done, 1) == (int)gridDim.x - 1;
    __syncthreads();
    const bool l = *flag != 0;
    if (l) __threadfence();
    return l;
}

// Per-group argmin of cost over [group_start[g], group_start[g + 1]) by one
// workgroup (at most 1024 threads): the lowest index of the minimum with NaN
// ranked as +inf, the group's start for an empty group.  (cost, index) pairs
// are totally ordered, so the result does not depend on the order in which
// the threads combine.  sv, si: 16 entries each of LDS, free for the call.
__device__ __forceinline__ void block_argmin(int G, const int32_t *__restrict__ group_start, const float *cost,
                                             int32_t *__restrict__ best, float *sv, int *si)
{
    const int lane = lane_id(), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    const int nt = blockDim.x;
    for (int g = 0; g < G; ++g) {
        const int lo = group_start[g], hi = group_start[g + 1];
        float bv = __int_as_float(0x7f800000);
        int bi = 0x7fffffff;
        for (int i0 = lo + threadIdx.x; i0 < hi; i0 += 4 * nt) {
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = i0 + k * nt < hi ? cost[i0 + k * nt] : 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = i0 + k * nt;
                const float x = v[k] != v[k] ? __int_as_float(0x7f800000) : v[k];
                if (i < hi && (x < bv || (x == bv && i < bi))) { bv = x; bi = i; }
            }
        }
#pragma unroll
        for (int off = WAVE / 2; off > 0; off >>= 1) {
            const float x = __shfl_xor(bv, off);
            const int i = __shfl_xor(bi, off);
            if (x < bv || (x == bv && i < bi)) { bv = x; bi = i; }
        }
        if (lane == 0) { sv[w] = bv; si[w] = bi; }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int k = 1; k < nw; ++k)
                if (sv[k] < bv || (sv[k] == bv && si[k] < bi)) { bv = sv[k]; bi = si[k]; }
            best[g] = bi == 0x7fffffff ? lo : bi;
        }
        __syncthreads();
    }
}

// Philox4x32 with 10 rounds (Salmon et al., SC'11): per round the words 0
// and 2 are multiplied by the two round multipliers, the high halves are
// mixed with the other two words and the round key, and the key is bumped
// by the two Weyl increments.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t *out)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float &n0, float &n1)
{
    // uniforms (w + 1/2) 2^-32 in (0, 1), formed in double to keep every bit
    double u = ((double)a + 0.5) * 2.3283064365386963e-10;
    double v = ((double)b + 0.5) * 2.3283064365386963e-10;
    float rad = sqrtf(-2.f * (float)log(u));
    float ang = (float)(6.283185307179586 * v);
    n0 = rad * cosf(ang);
    n1 = rad * sinf(ang);
}

// Exploration of simulation j after a copy (Sec. III-D): mu and m get
// Gaussian noise around the source values (clamped to their ranges) and the
// perturbation force is drawn afresh, the normals by Box-Muller from the
// Philox counters (j, window, 1, 0) and (j, window, 2, 0).  out: m, mu, f(3).
__device__ __forceinline__ void explore(const ResampleArgs &R, uint32_t j, uint32_t window_idx, float m_src,
                                        float mu_src, float *out)
{
    const uint32_t key0 = (uint32_t)(R.seed & 0xffffffffu), key1 = (uint32_t)(R.seed >> 32);
    uint32_t w1[4], w2[4];
    philox4x32_10(j, window_idx, 1u, 0u, key0, key1, w1);
    philox4x32_10(j, window_idx, 2u, 0u, key0, key1, w2);
    float n0, n1, n2, n3, n4, n5;
    box_muller(w1[0], w1[1], n0, n1);
    box_muller(w1[2], w1[3], n2, n3);
    box_muller(w2[0], w2[1], n4, n5);
    float mu = mu_src + R.sigma_mu * n0;
    float ms = m_src + R.sigma_m * n1;
    out[1] = fminf(fmaxf(mu, R.mu_lo), R.mu_hi);
    out[0] = fminf(fmaxf(ms, R.m_lo), R.m_hi);
    out[2] = R.sigma_f * n2;
    out[3] = R.sigma_f * n3;
    out[4] = R.sigma_f * n4;
}

}  // namespace pt
