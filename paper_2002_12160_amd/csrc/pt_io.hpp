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

__device__ __forceinline__ void flush_stats(int64_t *stats, const StepStats &st, int64_t steps)
{
    if (lane_id() == 0) {
        atomicAdd((unsigned long long *)&stats[0], (unsigned long long)steps);
        atomicAdd((unsigned long long *)&stats[1], (unsigned long long)st.cand);
        atomicAdd((unsigned long long *)&stats[2], (unsigned long long)st.contacts);
        atomicAdd((unsigned long long *)&stats[3], (unsigned long long)st.dropped);
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
            __syncthreads();
        }
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
