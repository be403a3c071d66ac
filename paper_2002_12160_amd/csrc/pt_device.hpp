// pt_device.hpp -- device-side building blocks of one simulation step on
// CDNA4 (gfx950).  One 64-lane wavefront owns one simulation: lanes run over
// the object's spheres in the narrow phase and over contact slots in the
// contact solve (C_max <= 64, one contact per lane); cross-contact sums are
// butterfly all-reductions, so every lane ends with bit-identical uniform
// values and every branch on them is wave-uniform.
//
// World model (Sec. III-A of the paper leaves the simulator open; this is the
// reading implemented by the library): see include/pt.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pt {

constexpr int WAVE = 64;
constexpr int SEG_STRIDE = 16;  // per-link hand segment record, floats
constexpr int WARM_STRIDE = 4;  // key bits + r(3)

// ---------------------------------------------------------------------
// constants of a batch, passed by value to every kernel
// ---------------------------------------------------------------------
struct Consts {
    int K, G, L, D, S_max, C_max, newton_iters, T, max_cand, solve_fp64;
    int max_cand_rows;         // list entries that hold the solve's sum rows whole (the reverse sweep)
    float dt, gx, gy, gz, margin, erp, compliance, kappa, fb_delta, armijo_sigma;
    float tau_contact, w_mag, w_dir;
    int cost_mode;             // 0: force terms, obs rows 4; 1: Eq. 3, obs rows 7
    float tau_slip, tau_spin, w_eq3[7];
    int collision_mode;        // 0: sphere set; 1: links against the object's distance field
    int link_samples, sdf_n;   // collision_mode 1: samples per link axis, grid nodes per axis
};

struct Tables {
    const float *hand;          // [L][20]
    const float *spheres;       // [n_types][S_max][4]
    const int32_t *n_spheres;   // [n_types]
    const float *inv_inertia;   // [n_types][3]
    const int32_t *env_type;    // [K]
    const int32_t *group_of;    // [K]
    const float *sdf;           // [n_types][sdf_n^3] distance-field nodes (collision_mode 1)
    const float *sdf_box;       // [n_types][4] grid origin and node spacing
};

// uniform per-simulation state held in registers
struct Body {
    float x[3], q[4], v[3], w[3];
    float m, mu, f[3];
};

// per-wave LDS scratch
struct WaveLds {
    float *cand_d;   // [max_cand]
    int *cand_k;     // [max_cand]
    int *sel;        // [64]
    int *wkey;       // [64]
    float *wr;       // [64*3]
    float *seg;      // [L][16] hand segment records of the step (after the [64][4] contact stage)
};

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// number of set bits of mask below this lane
__device__ __forceinline__ int mask_rank(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Cross-lane sums with DPP (data-parallel primitives: VALU lane moves, no LDS
// round trip).  Prefix sums inside each 16-lane row (row_shr 1, 2, 4, 8),
// then row 0's total is added into row 1 and row 2's into row 3
// (row_bcast:15), then lane 31 into rows 2-3 (row_bcast:31); the total ends in
// the last lane of the span and is broadcast with readlane, so every lane gets
// the same bits.  `span` (16, 32 or 64, wave-uniform) is the number of lanes
// that can hold non-zero values.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f(double v)
{
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, true);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// A wave-uniform value (the same bits in every lane) moved to scalar
// registers, where it costs no vector register while it stays live
__device__ __forceinline__ float uniform(float x)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uniform(double x)
{
    long long b = __double_as_longlong(x);
    int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// the body after a step is the same in every lane: keep it in scalar registers
__device__ __forceinline__ void uniform_body(Body &B)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        B.x[i] = uniform(B.x[i]); B.v[i] = uniform(B.v[i]);
        B.w[i] = uniform(B.w[i]); B.f[i] = uniform(B.f[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) B.q[i] = uniform(B.q[i]);
    B.m = uniform(B.m); B.mu = uniform(B.mu);
}

// readlane moves 32-bit integers: reinterpret, never convert
__device__ __forceinline__ float bcast_lane(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double bcast_lane(double v, int lane)
{
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ uint64_t bcast_lane(uint64_t v, int lane)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// A candidate contact (gap d, key k >= 0) as one 64-bit word whose unsigned
// order is the (d, k) order: d's bits made monotone (sign set: all bits
// flipped, else the sign bit set; -0 taken as +0 first) above the key.
__device__ __forceinline__ uint64_t pack_gap_key(float d, int k)
{
    uint32_t u = __float_as_uint(d + 0.f);
    u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
    return ((uint64_t)u << 32) | (uint32_t)k;
}

// One half-wave's values in both halves: lanes i and i + 32 both end with
// what lane i held (from_upper false) or what lane i + 32 held (true).  One
// ds_bpermute per 32-bit word (the LDS crossbar, no LDS memory).
__device__ __forceinline__ uint32_t half_bcast(uint32_t x, bool from_upper)
{
    const int src = from_upper ? (lane_id() | 32) : (lane_id() & 31);
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)x);
}
__device__ __forceinline__ float half_bcast(float x, bool from_upper)
{
    return __uint_as_float(half_bcast(__float_as_uint(x), from_upper));
}
__device__ __forceinline__ double half_bcast(double x, bool from_upper)
{
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = half_bcast((uint32_t)b, from_upper), hi = half_bcast((uint32_t)(b >> 32), from_upper);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sums of one value over the first span <= 32 lanes of each half-wave, by the
// same DPP tree as wave_sum (so each half's sum has the bits wave_sum gives
// for the lower half alone): lo over lanes [0, span), hi over [32, 32 + span)
template <typename T>
__device__ __forceinline__ void half_sums(T v, int span, T &lo, T &hi)
{
    v += dpp_f<0x111, 0xf>(v);  // row_shr:1
    v += dpp_f<0x112, 0xf>(v);  // row_shr:2
    v += dpp_f<0x114, 0xf>(v);  // row_shr:4
    v += dpp_f<0x118, 0xf>(v);  // row_shr:8
    if (span <= 16) {
        lo = bcast_lane(v, 15);
        hi = bcast_lane(v, 47);
        return;
    }
    v += dpp_f<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
    lo = bcast_lane(v, 31);
    hi = bcast_lane(v, 63);
}

template <typename T, int N>
__device__ __forceinline__ void wave_sum(T (&v)[N], int span = 64)
{
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_f<0x111, 0xf>(v[i]);  // row_shr:1
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_f<0x112, 0xf>(v[i]);  // row_shr:2
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_f<0x114, 0xf>(v[i]);  // row_shr:4
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_f<0x118, 0xf>(v[i]);  // row_shr:8
    if (span <= 16) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = bcast_lane(v[i], 15);
        return;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_f<0x142, 0xa>(v[i]);  // row_bcast:15 into rows 1, 3
    if (span <= 32) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = bcast_lane(v[i], 31);
        return;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_f<0x143, 0xc>(v[i]);  // row_bcast:31 into rows 2, 3
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = bcast_lane(v[i], 63);
}

template <typename T>
__device__ __forceinline__ T wave_sum1(T a, int span = 64)
{
    T v[1] = {a};
    wave_sum<T, 1>(v, span);
    return v[0];
}

// span of lanes holding the first n contacts
__device__ __forceinline__ int lane_span(int n) { return n <= 16 ? 16 : (n <= 32 ? 32 : 64); }

// ---------------------------------------------------------------------
// small vector helpers
// ---------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T dot3(const T *a, const T *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <typename T>
__device__ __forceinline__ void cross3(const T *a, const T *b, T *o)
{
    T t0 = a[1] * b[2] - a[2] * b[1];
    T t1 = a[2] * b[0] - a[0] * b[2];
    T t2 = a[0] * b[1] - a[1] * b[0];
    o[0] = t0; o[1] = t1; o[2] = t2;
}

__device__ __forceinline__ void quat_to_mat(const float *q, float *R)
{
    float w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}

__device__ __forceinline__ void quat_mul(const float *a, const float *b, float *o)
{
    float w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    float x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    float y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    float z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

// the same in double precision (hand kinematics)
__device__ __forceinline__ void quat_to_mat_d(const double *q, double *R)
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

__device__ __forceinline__ void quat_mul_d(const double *a, const double *b, double *o)
{
    double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

// ---------------------------------------------------------------------
// narrow phase: signed gap of sphere (c, rho) to link l or to the table
// ---------------------------------------------------------------------
// hand segment record (16 floats): a(3), radius, ab(3), 1/|ab|^2 (0 if
// degenerate), va(3), 0, vb(3), 0  -- positions at the start of the step,
// endpoint velocities over the step.
// gap of sphere (c, rho) to the capsule whose record starts at s
__device__ __forceinline__ float segment_gap(const float *s, const float *c, float rho)
{
    float ca0 = c[0] - s[0], ca1 = c[1] - s[1], ca2 = c[2] - s[2];
    float t = (ca0 * s[4] + ca1 * s[5] + ca2 * s[6]) * s[7];
    t = fminf(fmaxf(t, 0.f), 1.f);
    float d0 = ca0 - t * s[4], d1 = ca1 - t * s[5], d2 = ca2 - t * s[6];
    return sqrtf(d0 * d0 + d1 * d1 + d2 * d2) - rho - s[3];
}

__device__ __forceinline__ float pair_gap(const float *__restrict__ seg, int l, int L, const float *c, float rho)
{
    if (l == L) return c[2] - rho;
    return segment_gap(seg + l * SEG_STRIDE, c, rho);
}

// full contact geometry of a kept pair: gap, normal (link -> object),
// contact point on the object, velocity of the link surface point
__device__ __forceinline__ void pair_contact(const float *__restrict__ seg, int l, int L, const float *c, float rho,
                                            float &d, float *n, float *p, float *vl)
{
    if (l == L) {
        d = c[2] - rho;
        n[0] = 0.f; n[1] = 0.f; n[2] = 1.f;
        p[0] = c[0]; p[1] = c[1]; p[2] = c[2] - rho;
        vl[0] = vl[1] = vl[2] = 0.f;
        return;
    }
    const float *s = seg + l * SEG_STRIDE;
    float ca[3] = {c[0] - s[0], c[1] - s[1], c[2] - s[2]};
    float t = (ca[0] * s[4] + ca[1] * s[5] + ca[2] * s[6]) * s[7];
    t = fminf(fmaxf(t, 0.f), 1.f);
    float del[3] = {ca[0] - t * s[4], ca[1] - t * s[5], ca[2] - t * s[6]};
    float dist = sqrtf(dot3(del, del));
    d = dist - rho - s[3];
    if (dist < 1e-7f) {
        // centre on the axis: any normal perpendicular to the link
        float ab[3] = {s[4], s[5], s[6]}, e[3] = {1.f, 0.f, 0.f}, tt[3];
        cross3(ab, e, tt);
        if (sqrtf(dot3(tt, tt)) <= 1e-12f) {
            e[0] = 0.f; e[1] = 1.f;
            cross3(ab, e, tt);
        }
        if (sqrtf(dot3(tt, tt)) <= 1e-12f) { tt[0] = 0.f; tt[1] = 0.f; tt[2] = 1.f; }
        float inv = 1.f / sqrtf(dot3(tt, tt));
        n[0] = tt[0] * inv; n[1] = tt[1] * inv; n[2] = tt[2] * inv;
    } else {
        float inv = 1.f / dist;
        n[0] = del[0] * inv; n[1] = del[1] * inv; n[2] = del[2] * inv;
    }
    p[0] = c[0] - rho * n[0]; p[1] = c[1] - rho * n[1]; p[2] = c[2] - rho * n[2];
    float u = 1.f - t;
    vl[0] = u * s[8] + t * s[12];
    vl[1] = u * s[9] + t * s[13];
    vl[2] = u * s[10] + t * s[14];
}

// ---------------------------------------------------------------------
// link-object collision against the object's signed distance field
// (collision_mode 1): node values on a regular grid in the object frame,
// interpolated trilinearly
// ---------------------------------------------------------------------
struct SdfRef {
    const float *v = nullptr;    // [n^3] node values of the object's type, x fastest
    const float *box = nullptr;  // grid origin (3) and node spacing
    int n = 0;                   // nodes per axis
    int M = 0;                   // samples per link axis
};

// the field at object-frame point p (outside the grid's box: the value at
// the nearest box point plus the distance to it) and, with g, its gradient
// (that of the interpolant, at the nearest box point)
__device__ __forceinline__ float sdf_eval(const SdfRef &f, const float *p, float *g)
{
    const int n = f.n;
    const float h = f.box[3];
    float out2 = 0.f, fr[3];
    int i0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = f.box[a], hi = lo + (float)(n - 1) * h;
        const float c = fminf(fmaxf(p[a], lo), hi);
        out2 += (p[a] - c) * (p[a] - c);
        const float u = (c - lo) / h;
        const int i = min(max((int)floorf(u), 0), n - 2);
        i0[a] = i;
        fr[a] = u - (float)i;
    }
    const float *b = f.v + ((size_t)i0[2] * n + i0[1]) * n + i0[0];
    const size_t sy = n, sz = (size_t)n * n;
    const float v000 = b[0], v100 = b[1], v010 = b[sy], v110 = b[sy + 1];
    const float v001 = b[sz], v101 = b[sz + 1], v011 = b[sz + sy], v111 = b[sz + sy + 1];
    const float fx = fr[0], fy = fr[1], fz = fr[2], gx = 1.f - fx, gy = 1.f - fy, gz = 1.f - fz;
    const float val = gz * (gy * (gx * v000 + fx * v100) + fy * (gx * v010 + fx * v110)) +
                      fz * (gy * (gx * v001 + fx * v101) + fy * (gx * v011 + fx * v111));
    if (g) {
        const float ih = 1.f / h;
        g[0] = (gz * (gy * (v100 - v000) + fy * (v110 - v010)) + fz * (gy * (v101 - v001) + fy * (v111 - v011))) * ih;
        g[1] = (gz * (gx * (v010 - v000) + fx * (v110 - v100)) + fz * (gx * (v011 - v001) + fx * (v111 - v101))) * ih;
        g[2] = (gy * (gx * (v001 - v000) + fx * (v101 - v100)) + fy * (gx * (v011 - v010) + fx * (v111 - v110))) * ih;
    }
    return val + sqrtf(out2);
}

// the point of sample m of the link whose record starts at s: a + t (b - a),
// t = m / (M - 1) (the middle for one sample)
__device__ __forceinline__ float sdf_sample_t(int m, int M) { return M > 1 ? (float)m / (float)(M - 1) : 0.5f; }

// full contact geometry of sample m of link l against the field (object at
// x, R): gap phi - radius, normal (link -> object) minus the world unit
// gradient, contact point the sample moved by -phi along it, velocity of the
// link at the sample
__device__ __forceinline__ void sdf_contact(const SdfRef &f, const float *__restrict__ seg, int l, int m,
                                            const float *x, const float *R, float &d, float *n, float *p, float *vl,
                                            float &t)
{
    const float *s = seg + l * SEG_STRIDE;
    t = sdf_sample_t(m, f.M);
    const float sp[3] = {s[0] + t * s[4], s[1] + t * s[5], s[2] + t * s[6]};
    const float r[3] = {sp[0] - x[0], sp[1] - x[1], sp[2] - x[2]};
    const float po[3] = {R[0] * r[0] + R[3] * r[1] + R[6] * r[2], R[1] * r[0] + R[4] * r[1] + R[7] * r[2],
                         R[2] * r[0] + R[5] * r[1] + R[8] * r[2]};
    float g[3];
    const float phi = sdf_eval(f, po, g);
    const float gn = sqrtf(dot3(g, g));
    float go[3] = {0.f, 0.f, 1.f};
    if (gn >= 1e-12f) {
        const float ig = 1.f / gn;
        go[0] = g[0] * ig; go[1] = g[1] * ig; go[2] = g[2] * ig;
    }
    const float gw[3] = {R[0] * go[0] + R[1] * go[1] + R[2] * go[2], R[3] * go[0] + R[4] * go[1] + R[5] * go[2],
                         R[6] * go[0] + R[7] * go[1] + R[8] * go[2]};
    d = phi - s[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        n[i] = -gw[i];
        p[i] = sp[i] - phi * gw[i];
    }
    const float u = 1.f - t;
    vl[0] = u * s[8] + t * s[12];
    vl[1] = u * s[9] + t * s[13];
    vl[2] = u * s[10] + t * s[14];
}

// tangent frame: e = axis of the smallest |n_i| (lowest index on ties)
__device__ __forceinline__ void tangent_frame(const float *n, float *t1, float *t2)
{
    int e = 0;
    float an0 = fabsf(n[0]), an1 = fabsf(n[1]), an2 = fabsf(n[2]);
    float best = an0;
    if (an1 < best) { e = 1; best = an1; }
    if (an2 < best) { e = 2; }
    float ev[3] = {e == 0 ? 1.f : 0.f, e == 1 ? 1.f : 0.f, e == 2 ? 1.f : 0.f};
    cross3(n, ev, t1);
    float inv = 1.f / sqrtf(dot3(t1, t1));
    t1[0] *= inv; t1[1] *= inv; t1[2] *= inv;
    cross3(n, t1, t2);
}

// ---------------------------------------------------------------------
// smoothed Fischer-Burmeister function of one contact on the Lorentz cone
// ---------------------------------------------------------------------
// x = kappa (mu r_n, r_t), y = (u_n + mu sqrt(|u_t|^2 + delta^2), mu u_t),
// w = sqrt(x o x + y o y + 2 delta^2 e), Phi = x + y - w.  With the spectral
// values l1,2 = z0 -/+ |zb| of z = x o x + y o y + 2 delta^2 e,
// w0 = (sqrt l1 + sqrt l2) / 2 and wb = zb / (sqrt l1 + sqrt l2), where
// sqrt l1 + sqrt l2 = sqrt(2 z0 + 2 sqrt(det z)) and det z = l1 l2 is written
// as a sum of squares: no difference of nearly equal terms, so the small
// spectral value stays accurate when x and y sit on the cone boundary
// (sliding), and |zb| itself is never needed.
template <typename T>
struct FBOut {
    T phi[3];
    T w0, w1, w2, s, st;   // sqrt(z), det(sqrt z), smoothed |u_t|
    T rw, rs, rst;         // 1 / (2 w0), 1 / s, 1 / st
    T x[3], y[3];
};

// 1/sqrt(x) for x > 0 (the math library's, to about an ulp)
__device__ __forceinline__ double rsqrt_t(double x) { return rsqrt(x); }
__device__ __forceinline__ float rsqrt_t(float x) { return rsqrtf(x); }

// 1/x for a finite, normal, nonzero x: the hardware estimate refined by two
// Newton-Raphson steps y <- y + y (1 - x y), each of which squares the
// relative error, to about an ulp in float64
__device__ __forceinline__ double recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ float recip(float x) { return 1.f / x; }

template <typename T>
__device__ __forceinline__ void fb_value(T mu, T kap, T del, const T *r, const T *u, FBOut<T> &o)
{
    T x0 = kap * mu * r[0], x1 = kap * r[1], x2 = kap * r[2];
    // square roots as x * (1/sqrt(x)): the reciprocals serve the Jacobian
    T q2 = u[1] * u[1] + u[2] * u[2] + del * del;
    T rst = rsqrt_t(q2);
    T st = q2 * rst;
    T y0 = u[0] + mu * st, y1 = mu * u[1], y2 = mu * u[2];
    T A = x0 * x0 + x1 * x1 + x2 * x2;
    T B = y0 * y0 + y1 * y1 + y2 * y2;
    T d2 = del * del;
    T z0 = A + B + T(2) * d2;
    T zb1 = T(2) * (x0 * x1 + y0 * y1), zb2 = T(2) * (x0 * x2 + y0 * y2);
    T dx = x0 * x0 - (x1 * x1 + x2 * x2);
    T dy = y0 * y0 - (y1 * y1 + y2 * y2);
    T c1 = x0 * y1 - y0 * x1, c2 = x0 * y2 - y0 * x2;
    T e = x0 * y0 - (x1 * y1 + x2 * y2);
    T cr = x1 * y2 - x2 * y1;
    T detz = dx * dx + dy * dy + T(2) * (c1 * c1 + c2 * c2) + T(2) * e * e + T(2) * cr * cr +
                 T(4) * d2 * (A + B) + T(4) * d2 * d2;
    T rs = rsqrt_t(detz);
    T sd = detz * rs;                        // sqrt(l1) sqrt(l2)
    T s2 = T(2) * (z0 + sd);
    T inv = rsqrt_t(s2);
    T sum = s2 * inv;                        // sqrt(l1) + sqrt(l2)
    o.w0 = T(0.5) * sum;
    o.rw = inv;
    o.rs = rs;
    o.rst = rst;
    o.w1 = zb1 * inv;
    o.w2 = zb2 * inv;
    o.s = sd;
    o.st = st;
    o.x[0] = x0; o.x[1] = x1; o.x[2] = x2;
    o.y[0] = y0; o.y[1] = y1; o.y[2] = y2;
    o.phi[0] = x0 + y0 - o.w0;
    o.phi[1] = x1 + y1 - o.w1;
    o.phi[2] = x2 + y2 - o.w2;
}

// Jacobian blocks of Phi: dPhi/dr = Dx Sx =: JX, dPhi/du = Dy Sy =: JY with
// Dx = I - Lw^-1 Lx, Dy = I - Lw^-1 Ly (row-major 3x3)
template <typename T>
__device__ __forceinline__ void fb_jacobian(T mu, T kap, const T *u, const FBOut<T> &o, T *JX, T *JY,
                                            T *DXo = nullptr, T *DYo = nullptr)
{
    T w0 = o.w0, w1 = o.w1, w2 = o.w2, s = o.s;
    T k = T(2) * o.rw * o.rs;                // 1 / (w0 s)
    T Li[9] = {k * w0 * w0, -k * w0 * w1, -k * w0 * w2,
                   -k * w0 * w1, k * (s + w1 * w1), k * w1 * w2,
                   -k * w0 * w2, k * w1 * w2, k * (s + w2 * w2)};
    const T *x = o.x, *y = o.y;
    // Li * L_a with L_a = [[a0,a1,a2],[a1,a0,0],[a2,0,a0]]
    T Dx[9], Dy[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T *li = Li + 3 * i;
        T px0 = li[0] * x[0] + li[1] * x[1] + li[2] * x[2];
        T px1 = li[0] * x[1] + li[1] * x[0];
        T px2 = li[0] * x[2] + li[2] * x[0];
        T py0 = li[0] * y[0] + li[1] * y[1] + li[2] * y[2];
        T py1 = li[0] * y[1] + li[1] * y[0];
        T py2 = li[0] * y[2] + li[2] * y[0];
        Dx[3 * i + 0] = (i == 0 ? T(1) : T(0)) - px0;
        Dx[3 * i + 1] = (i == 1 ? T(1) : T(0)) - px1;
        Dx[3 * i + 2] = (i == 2 ? T(1) : T(0)) - px2;
        Dy[3 * i + 0] = (i == 0 ? T(1) : T(0)) - py0;
        Dy[3 * i + 1] = (i == 1 ? T(1) : T(0)) - py1;
        Dy[3 * i + 2] = (i == 2 ? T(1) : T(0)) - py2;
    }
    T th1 = mu * u[1] * o.rst, th2 = mu * u[2] * o.rst;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        JX[3 * i + 0] = Dx[3 * i + 0] * (kap * mu);
        JX[3 * i + 1] = Dx[3 * i + 1] * kap;
        JX[3 * i + 2] = Dx[3 * i + 2] * kap;
        JY[3 * i + 0] = Dy[3 * i + 0];
        JY[3 * i + 1] = Dy[3 * i + 0] * th1 + Dy[3 * i + 1] * mu;
        JY[3 * i + 2] = Dy[3 * i + 0] * th2 + Dy[3 * i + 2] * mu;
    }
    if (DXo) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            DXo[i] = Dx[i];
            DYo[i] = Dy[i];
        }
    }
}

// 3x3 inverse by the adjugate
template <typename T>
__device__ __forceinline__ void inv3(const T *a, T *o)
{
    T c00 = a[4] * a[8] - a[5] * a[7];
    T c01 = a[5] * a[6] - a[3] * a[8];
    T c02 = a[3] * a[7] - a[4] * a[6];
    T det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    T id = recip(det);
    o[0] = c00 * id;
    o[1] = (a[2] * a[7] - a[1] * a[8]) * id;
    o[2] = (a[1] * a[5] - a[2] * a[4]) * id;
    o[3] = c01 * id;
    o[4] = (a[0] * a[8] - a[2] * a[6]) * id;
    o[5] = (a[2] * a[3] - a[0] * a[5]) * id;
    o[6] = c02 * id;
    o[7] = (a[1] * a[6] - a[0] * a[7]) * id;
    o[8] = (a[0] * a[4] - a[1] * a[3]) * id;
}

// 6x6 solve S z = b by 3x3 blocks S = [[A, B], [Cb, D]]:
// z2 = (D - Cb A^-1 B)^-1 (b2 - Cb A^-1 b1), z1 = A^-1 (b1 - B z2), both 3x3
// inverses by the adjugate.  A = m I + the sum of the contacts' world blocks
// (the translational part of M + sum J^T Q J; I + M^-1 sum J^T Q J in the
// inverse-mass form) and its Schur complement (the rotational part) stay
// well away from singular, so no pivoting is done: every lane runs the same
// straight-line code in registers.
template <typename T>
__device__ __forceinline__ void solve6(const T (&S)[36], T (&b)[6])
{
    T A[9], Bm[9], Cb[9], Dm[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            A[3 * i + j] = S[6 * i + j];
            Bm[3 * i + j] = S[6 * i + 3 + j];
            Cb[3 * i + j] = S[6 * (3 + i) + j];
            Dm[3 * i + j] = S[6 * (3 + i) + 3 + j];
        }
    T Ai[9];
    inv3(A, Ai);
    T X[9];   // A^-1 B
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) X[3 * i + j] = Ai[3 * i] * Bm[j] + Ai[3 * i + 1] * Bm[3 + j] + Ai[3 * i + 2] * Bm[6 + j];
    T y1[3] = {Ai[0] * b[0] + Ai[1] * b[1] + Ai[2] * b[2], Ai[3] * b[0] + Ai[4] * b[1] + Ai[5] * b[2],
               Ai[6] * b[0] + Ai[7] * b[1] + Ai[8] * b[2]};
    T Sc[9], r2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Sc[3 * i + j] = Dm[3 * i + j] - (Cb[3 * i] * X[j] + Cb[3 * i + 1] * X[3 + j] + Cb[3 * i + 2] * X[6 + j]);
        r2[i] = b[3 + i] - (Cb[3 * i] * y1[0] + Cb[3 * i + 1] * y1[1] + Cb[3 * i + 2] * y1[2]);
    }
    T Si[9];
    inv3(Sc, Si);
    T z2[3] = {Si[0] * r2[0] + Si[1] * r2[1] + Si[2] * r2[2], Si[3] * r2[0] + Si[4] * r2[1] + Si[5] * r2[2],
               Si[6] * r2[0] + Si[7] * r2[1] + Si[8] * r2[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        b[i] = y1[i] - (X[3 * i] * z2[0] + X[3 * i + 1] * z2[1] + X[3 * i + 2] * z2[2]);
        b[3 + i] = z2[i];
    }
}

// Row stride (elements) of the LDS reduction buffer: rows 16-byte aligned,
// and the 16-byte row writes of eight consecutive lanes on distinct banks
// (44 doubles = 88 dwords, rows 24 banks apart); for doubles the narrowest
// stride that holds the 43 sums folded in two halves of 22, since with caps
// above 16 its 32 rows size the solve's share of a simulation's LDS
template <typename T>
struct RedStride {
    static constexpr int value = sizeof(T) == 8 ? 44 : 68;
};

template <typename T>
__device__ __forceinline__ void store16(T *p, const T *v);
template <>
__device__ __forceinline__ void store16<double>(double *p, const double *v)
{
    *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
}
template <>
__device__ __forceinline__ void store16<float>(float *p, const float *v)
{
    *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
template <typename T>
__device__ __forceinline__ void load16(const T *p, T *v);
template <>
__device__ __forceinline__ void load16<double>(const double *p, double *v)
{
    double2 a = *reinterpret_cast<const double2 *>(p);
    v[0] = a.x; v[1] = a.y;
}
template <>
__device__ __forceinline__ void load16<float>(const float *p, float *v)
{
    float4 a = *reinterpret_cast<const float4 *>(p);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// Two half-wave folds in one: lane l < 32 gets a[l] + a[l + 32], lane
// l >= 32 gets b[l - 32] + b[l] (the lower lane's value first).  The swap of
// a's upper half-wave with b's lower one puts both addends of every lane in
// the two swapped registers, with no LDS round trip.
__device__ __forceinline__ double fold_halves(double a, double b)
{
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ float fold_halves(float a, float b)
{
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

// Sum of v[0..N) over lanes [0, n) through LDS, for wide vectors where DPP
// rounds would cost N instructions each.  Every lane >= n must hold zeros.
// First each pair (v[2k], v[2k+1]) is folded across the half-waves
// (fold_halves), so that row r < 32 holds lane r's and lane r + 32's values
// added: the even-indexed sums in its first H = ceil(N / 2) entries (written
// by lane r), the odd-indexed ones in the next H (written by lane r + 32),
// each half padded to whole 16-byte words.  With n <= 32 there is nothing to
// fold and lane r < n16 writes both halves of row r itself (the same bits the
// fold would give: it would add zeros).  Rows up to n16 = n rounded up to 16
// (at most 32) are written; lane j < N then adds its sum's column over them,
// 32 (or 16) reads in flight into four interleaved partial sums in a fixed
// order, and the N sums land in buf[0..N) in their natural order, where every
// lane can read them (the same bits for every lane).  buf: 16-byte aligned,
// n16 rows of RedStride<T> elements.  The sums stay valid until the next
// write to buf.
template <typename T, int N>
__device__ __forceinline__ void lds_colsum(const T (&v)[N], int n, T *buf)
{
    constexpr int RS = RedStride<T>::value;
    constexpr int PER = 16 / (int)sizeof(T);
    constexpr int H = (N + 1) / 2, HP = (H + PER - 1) / PER * PER;
    static_assert(2 * HP <= RS && N <= 64, "vector too long for the reduction buffer");
    const int lane = lane_id();
    const int n16 = min((n + 15) & ~15, 32);
    if (n > 32) {
        T f[HP];
#pragma unroll
        for (int k = 0; k < H; ++k) f[k] = fold_halves(v[2 * k], 2 * k + 1 < N ? v[2 * k + 1] : T(0));
#pragma unroll
        for (int k = H; k < HP; ++k) f[k] = T(0);
        T *row = buf + (lane & 31) * RS + (lane >> 5) * HP;
#pragma unroll
        for (int j = 0; j < HP; j += PER) store16<T>(row + j, f + j);
    } else if (lane < n16) {
        // nothing to fold: each lane writes both halves of its own row
        T e[HP], o[HP];
#pragma unroll
        for (int k = 0; k < HP; ++k) {
            e[k] = 2 * k < N ? v[2 * k] : T(0);
            o[k] = 2 * k + 1 < N ? v[2 * k + 1] : T(0);
        }
        T *row = buf + lane * RS;
#pragma unroll
        for (int j = 0; j < HP; j += PER) store16<T>(row + j, e + j);
#pragma unroll
        for (int j = 0; j < HP; j += PER) store16<T>(row + HP + j, o + j);
    }
    wave_sync();
    T s4[4] = {T(0), T(0), T(0), T(0)};
    if (lane < N) {
        const T *col = buf + (lane & 1) * HP + (lane >> 1);
        if (n16 == 32) {
            T x[32];
#pragma unroll
            for (int k = 0; k < 32; ++k) x[k] = col[k * RS];
#pragma unroll
            for (int k = 0; k < 32; ++k) s4[k & 3] += x[k];
        } else if (n16 == 16) {
            T x[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) x[k] = col[k * RS];
#pragma unroll
            for (int k = 0; k < 16; ++k) s4[k & 3] += x[k];
        }
    }
    const T s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    wave_sync();
    if (lane < N) buf[lane] = s;
    wave_sync();
}

// lds_colsum with the N sums read back into v in every lane
template <typename T, int N>
__device__ __forceinline__ void lds_sum(T (&v)[N], int n, T *buf)
{
    constexpr int PER = 16 / (int)sizeof(T);
    lds_colsum<T, N>(v, n, buf);
#pragma unroll
    for (int j = 0; j + PER <= N; j += PER) load16<T>(buf + j, v + j);
#pragma unroll
    for (int j = N - N % PER; j < N; ++j) v[j] = buf[j];
    wave_sync();
}

// One contact's contribution to the 6x6 Schur system: with the world-frame
// block Qw (3x3) and vector gw, J_c^T Qw J_c = [[Qw, -Qw rhat], [rhat Qw,
// -rhat Qw rhat]] (row i of Qw rhat is q_i x rho) into acc[0..35] row-major,
// and J_c^T gw = (gw, rho x gw) into acc[36..41].
template <typename SR>
__device__ __forceinline__ void schur_contribution(const SR *Qw, const SR *gw, const SR *rho, SR *acc)
{
    // Y = -Qw rhat: row i is rho x q_i, so no block needs a negation
    SR Y[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) cross3(rho, Qw + 3 * i, Y + 3 * i);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            acc[6 * i + j] = Qw[3 * i + j];
            acc[6 * i + 3 + j] = Y[3 * i + j];
        }
    // bottom blocks: columns rho x (column j of Qw), rho x (column j of Y)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        SR cq[3] = {Qw[j], Qw[3 + j], Qw[6 + j]}, cy[3] = {Y[j], Y[3 + j], Y[6 + j]};
        SR a3[3], b3[3];
        cross3(rho, cq, a3);
        cross3(rho, cy, b3);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            acc[6 * (3 + i) + j] = a3[i];
            acc[6 * (3 + i) + 3 + j] = b3[i];
        }
    }
    SR tg[3];
    cross3(rho, gw, tg);
    acc[36] = gw[0]; acc[37] = gw[1]; acc[38] = gw[2];
    acc[39] = tg[0]; acc[40] = tg[1]; acc[41] = tg[2];
}

// Mass matrix of one body for the 6x6 solve: M = diag(m I, Iw) when every
// principal inertia is finite (Iw = Iinv^-1, inverted in SR so that the two
// agree to SR rounding), else only M^-1 = diag(im I, Iinv) (a body that
// cannot turn about some axis).
// Only the form's own block and scalar are kept: (m, Iw) in the inertia
// form, (1/m, Iinv) otherwise.
template <typename SR>
struct BodyMass {
    bool inertia_form;
    SR sc, blk[9];
};

template <typename SR>
__device__ __forceinline__ void body_mass(float m, const float *Iinv, const float *inv_in, BodyMass<SR> &M)
{
    M.inertia_form = inv_in[0] > 0.f && inv_in[1] > 0.f && inv_in[2] > 0.f;
    SR I9[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) I9[i] = Iinv[i];
    if (M.inertia_form) {
        M.sc = m;
        inv3(I9, M.blk);
    } else {
        M.sc = SR(1) / SR(m);
#pragma unroll
        for (int i = 0; i < 9; ++i) M.blk[i] = I9[i];
    }
    // wave-uniform: held in scalar registers through the Newton loop
    M.sc = uniform(M.sc);
#pragma unroll
    for (int i = 0; i < 9; ++i) M.blk[i] = uniform(M.blk[i]);
}

// Solves (I + M^-1 A6) z = -M^-1 b6 for the summed acc (A6 = acc[0..35],
// b6 = acc[36..41]); with finite inertias as (M + A6) z = -b6, the same z
// without forming M^-1 A6.  Result in z.
template <typename SR>
__device__ __forceinline__ void schur_solve(const SR *acc, const BodyMass<SR> &M, SR (&z)[6])
{
    SR S6[36];
    if (M.inertia_form) {
#pragma unroll
        for (int i = 0; i < 36; ++i) S6[i] = acc[i];
        S6[0] += M.sc; S6[7] += M.sc; S6[14] += M.sc;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) S6[6 * (3 + i) + 3 + j] += M.blk[3 * i + j];
#pragma unroll
        for (int i = 0; i < 6; ++i) z[i] = -acc[36 + i];
    } else {
        const SR im = M.sc;
        const SR *Iinv = M.blk;
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            S6[j] = acc[j] * im + (j == 0 ? SR(1) : SR(0));
            S6[6 + j] = acc[6 + j] * im + (j == 1 ? SR(1) : SR(0));
            S6[12 + j] = acc[12 + j] * im + (j == 2 ? SR(1) : SR(0));
#pragma unroll
            for (int i = 0; i < 3; ++i)
                S6[6 * (3 + i) + j] = Iinv[3 * i] * acc[18 + j] + Iinv[3 * i + 1] * acc[24 + j] +
                                      Iinv[3 * i + 2] * acc[30 + j] + (j == 3 + i ? SR(1) : SR(0));
        }
        z[0] = -acc[36] * im; z[1] = -acc[37] * im; z[2] = -acc[38] * im;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            z[3 + i] = -(Iinv[3 * i] * acc[39] + Iinv[3 * i + 1] * acc[40] + Iinv[3 * i + 2] * acc[41]);
    }
    solve6(S6, z);
}

// ---------------------------------------------------------------------
// per-step statistics kept by each wave
// ---------------------------------------------------------------------
struct StepStats {
    int64_t cand, contacts, dropped;
};

}  // namespace pt
