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
    float dt, gx, gy, gz, margin, erp, compliance, kappa, fb_delta, armijo_sigma;
    float tau_contact, w_mag, w_dir;
};

struct Tables {
    const float *hand;          // [L][20]
    const float *spheres;       // [n_types][S_max][4]
    const int32_t *n_spheres;   // [n_types]
    const float *inv_inertia;   // [n_types][3]
    const int32_t *env_type;    // [K]
    const int32_t *group_of;    // [K]
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

// ---------------------------------------------------------------------
// narrow phase: signed gap of sphere (c, rho) to link l or to the table
// ---------------------------------------------------------------------
// hand segment record (16 floats): a(3), radius, ab(3), 1/|ab|^2 (0 if
// degenerate), va(3), 0, vb(3), 0  -- positions at the start of the step,
// endpoint velocities over the step.
__device__ __forceinline__ float pair_gap(const float *__restrict__ seg, int l, int L, const float *c, float rho)
{
    if (l == L) return c[2] - rho;
    const float *s = seg + l * SEG_STRIDE;
    float ca0 = c[0] - s[0], ca1 = c[1] - s[1], ca2 = c[2] - s[2];
    float t = (ca0 * s[4] + ca1 * s[5] + ca2 * s[6]) * s[7];
    t = fminf(fmaxf(t, 0.f), 1.f);
    float d0 = ca0 - t * s[4], d1 = ca1 - t * s[5], d2 = ca2 - t * s[6];
    return sqrtf(d0 * d0 + d1 * d1 + d2 * d2) - rho - s[3];
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
// w = sqrt(x o x + y o y + 2 delta^2 e), Phi = x + y - w.  The small
// spectral value lambda1 of z = x o x + y o y + 2 delta^2 e is obtained as
// det(z) / lambda2 with det(z) written as a sum of squares, which keeps it
// accurate in float32 when x and y sit on the cone boundary (sliding).
template <typename T>
struct FBOut {
    T phi[3];
    T w0, w1, w2, s, st;   // sqrt(z), det(sqrt z), smoothed |u_t|
    T x[3], y[3];
};

template <typename T>
__device__ __forceinline__ void fb_value(T mu, T kap, T del, const T *r, const T *u, FBOut<T> &o)
{
    T x0 = kap * mu * r[0], x1 = kap * r[1], x2 = kap * r[2];
    T st = sqrt(u[1] * u[1] + u[2] * u[2] + del * del);
    T y0 = u[0] + mu * st, y1 = mu * u[1], y2 = mu * u[2];
    T A = x0 * x0 + x1 * x1 + x2 * x2;
    T B = y0 * y0 + y1 * y1 + y2 * y2;
    T d2 = del * del;
    T z0 = A + B + T(2) * d2;
    T zb1 = T(2) * (x0 * x1 + y0 * y1), zb2 = T(2) * (x0 * x2 + y0 * y2);
    T nz = sqrt(zb1 * zb1 + zb2 * zb2);
    T l2 = z0 + nz;
    T dx = x0 * x0 - (x1 * x1 + x2 * x2);
    T dy = y0 * y0 - (y1 * y1 + y2 * y2);
    T c1 = x0 * y1 - y0 * x1, c2 = x0 * y2 - y0 * x2;
    T e = x0 * y0 - (x1 * y1 + x2 * y2);
    T cr = x1 * y2 - x2 * y1;
    T detz = dx * dx + dy * dy + T(2) * (c1 * c1 + c2 * c2) + T(2) * e * e + T(2) * cr * cr +
                 T(4) * d2 * (A + B) + T(4) * d2 * d2;
    T l1 = detz / l2;
    T s1 = sqrt(l1), s2 = sqrt(l2);
    T inv = T(1) / (s1 + s2);
    o.w0 = T(0.5) * (s1 + s2);
    o.w1 = zb1 * inv;
    o.w2 = zb2 * inv;
    o.s = s1 * s2;
    o.st = st;
    o.x[0] = x0; o.x[1] = x1; o.x[2] = x2;
    o.y[0] = y0; o.y[1] = y1; o.y[2] = y2;
    o.phi[0] = x0 + y0 - o.w0;
    o.phi[1] = x1 + y1 - o.w1;
    o.phi[2] = x2 + y2 - o.w2;
}

template <typename T>
__device__ __forceinline__ T fb_merit(T mu, T kap, T del, const T *r, const T *u)
{
    FBOut<T> o;
    fb_value(mu, kap, del, r, u, o);
    return T(0.5) * (o.phi[0] * o.phi[0] + o.phi[1] * o.phi[1] + o.phi[2] * o.phi[2]);
}

// Jacobian blocks of Phi: dPhi/dr = Dx Sx =: JX, dPhi/du = Dy Sy =: JY with
// Dx = I - Lw^-1 Lx, Dy = I - Lw^-1 Ly (row-major 3x3)
template <typename T>
__device__ __forceinline__ void fb_jacobian(T mu, T kap, const T *u, const FBOut<T> &o, T *JX, T *JY)
{
    T w0 = o.w0, w1 = o.w1, w2 = o.w2, s = o.s;
    T k = T(1) / (w0 * s);
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
    T th1 = mu * u[1] / o.st, th2 = mu * u[2] / o.st;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        JX[3 * i + 0] = Dx[3 * i + 0] * (kap * mu);
        JX[3 * i + 1] = Dx[3 * i + 1] * kap;
        JX[3 * i + 2] = Dx[3 * i + 2] * kap;
        JY[3 * i + 0] = Dy[3 * i + 0];
        JY[3 * i + 1] = Dy[3 * i + 0] * th1 + Dy[3 * i + 1] * mu;
        JY[3 * i + 2] = Dy[3 * i + 0] * th2 + Dy[3 * i + 2] * mu;
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
    T id = T(1) / det;
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

// in-register 6x6 LU with partial pivoting; solves A z = b (A, b destroyed)
template <typename T>
__device__ __forceinline__ void solve6(T (&A)[36], T (&b)[6])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        // pivot search (values are wave-uniform, so is the branch)
        int piv = k;
        T best = fabs(A[6 * k + k]);
#pragma unroll
        for (int i = k + 1; i < 6; ++i) {
            T v = fabs(A[6 * i + k]);
            if (v > best) { best = v; piv = i; }
        }
        // swap rows k and piv with selects (keeps everything in registers)
#pragma unroll
        for (int i = k + 1; i < 6; ++i) {
            bool sw = (piv == i);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                T a = A[6 * k + j], c = A[6 * i + j];
                A[6 * k + j] = sw ? c : a;
                A[6 * i + j] = sw ? a : c;
            }
            T a = b[k], c = b[i];
            b[k] = sw ? c : a;
            b[i] = sw ? a : c;
        }
        T ip = T(1) / A[6 * k + k];
#pragma unroll
        for (int i = k + 1; i < 6; ++i) {
            T f = A[6 * i + k] * ip;
#pragma unroll
            for (int j = k + 1; j < 6; ++j) A[6 * i + j] -= f * A[6 * k + j];
            b[i] -= f * b[k];
        }
    }
#pragma unroll
    for (int k = 5; k >= 0; --k) {
        T s = b[k];
#pragma unroll
        for (int j = k + 1; j < 6; ++j) s -= A[6 * k + j] * b[j];
        b[k] = s / A[6 * k + k];
    }
}

// ---------------------------------------------------------------------
// per-step statistics kept by each wave
// ---------------------------------------------------------------------
struct StepStats {
    int64_t cand, contacts, dropped;
};

// ---------------------------------------------------------------------
// one step of one simulation, executed by one wavefront
// ---------------------------------------------------------------------
// Inputs: body (uniform, in/out), per-lane warm slot (key, r) in/out.
// Output per lane c < C: link (or -1 for the table / empty) and the impulse
// on the object in world coordinates.  Geometry runs in float32; the contact
// solve runs in SR (float or double).
template <typename SR>
__device__ __forceinline__ void env_step(const Consts &P, const float *__restrict__ seg,
                                         const float *__restrict__ sph, int S, const float *inv_in, Body &B,
                                         int &wkey, float *wr, int &out_link, float *out_imp, const WaveLds &lds,
                                         StepStats &stats)
{
    const int lane = lane_id();
    const int L = P.L;
    const float dt = P.dt;

    // 1. pose, rotation, inverse inertia, free velocity
    float qn = rsqrtf(B.q[0] * B.q[0] + B.q[1] * B.q[1] + B.q[2] * B.q[2] + B.q[3] * B.q[3]);
    float q[4] = {B.q[0] * qn, B.q[1] * qn, B.q[2] * qn, B.q[3] * qn};
    float R[9];
    quat_to_mat(q, R);
    const float m = B.m;
    const float im = 1.f / m;
    float ii[3] = {inv_in[0] * im, inv_in[1] * im, inv_in[2] * im};
    float Iinv[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Iinv[3 * i + j] = R[3 * i] * ii[0] * R[3 * j] + R[3 * i + 1] * ii[1] * R[3 * j + 1] +
                              R[3 * i + 2] * ii[2] * R[3 * j + 2];
    float vs[3] = {B.v[0] + dt * (P.gx + B.f[0] * im), B.v[1] + dt * (P.gy + B.f[1] * im),
                   B.v[2] + dt * (P.gz + B.f[2] * im)};
    float ws[3] = {B.w[0], B.w[1], B.w[2]};

    // 2. narrow phase: lanes over spheres, candidates appended to LDS in
    //    (sphere block, link) order by ballot + prefix count
    int ncand = 0;
    for (int kb = 0; kb < S; kb += WAVE) {
        int k = kb + lane;
        bool valid = k < S;
        float s4[4] = {0.f, 0.f, 0.f, 0.f};
        if (valid) {
            const float4 t = *reinterpret_cast<const float4 *>(sph + 4 * k);
            s4[0] = t.x; s4[1] = t.y; s4[2] = t.z; s4[3] = t.w;
        }
        float c[3] = {B.x[0] + R[0] * s4[0] + R[1] * s4[1] + R[2] * s4[2],
                      B.x[1] + R[3] * s4[0] + R[4] * s4[1] + R[5] * s4[2],
                      B.x[2] + R[6] * s4[0] + R[7] * s4[1] + R[8] * s4[2]};
        for (int l = 0; l <= L; ++l) {
            float d = pair_gap(seg, l, L, c, s4[3]);
            bool cand = valid && (d < P.margin);
            uint64_t mask = __ballot(cand);
            if (cand) {
                int pos = ncand + mask_rank(mask);
                lds.cand_d[pos] = d;
                lds.cand_k[pos] = k * (L + 1) + l;
            }
            ncand += __popcll(mask);
        }
    }
    wave_sync();
    const int C = ncand < P.C_max ? ncand : P.C_max;

    // 3. cap: rank of every candidate in (d, key) order; the C_max lowest
    //    land in sel[rank]
    for (int i = lane; i < ncand; i += WAVE) {
        float di = lds.cand_d[i];
        int ki = lds.cand_k[i];
        int rank = 0;
        for (int j = 0; j < ncand; ++j) {
            float dj = lds.cand_d[j];
            int kj = lds.cand_k[j];
            rank += (dj < di || (dj == di && kj < ki)) ? 1 : 0;
        }
        if (rank < P.C_max) lds.sel[rank] = ki;
    }
    // previous warm cache to LDS for the key lookup
    lds.wkey[lane] = wkey;
    lds.wr[3 * lane + 0] = wr[0];
    lds.wr[3 * lane + 1] = wr[1];
    lds.wr[3 * lane + 2] = wr[2];
    wave_sync();

    stats.cand += ncand;
    stats.contacts += C;
    stats.dropped += ncand - C;

    // 4. contact setup, one contact per lane
    const bool act = lane < C;
    int key = act ? lds.sel[lane] : -1;
    SR F[9] = {0, 0, 1, 0, 1, 0, 1, 0, 0};  // rows n, t1, t2
    SR rho[3] = {0, 0, 0};
    SR ucst[3] = {0, 0, 0};
    SR r[3] = {0, 0, 0};
    int link = -1;
    if (act) {
        int k = key / (L + 1);
        int l = key - k * (L + 1);
        const float4 t = *reinterpret_cast<const float4 *>(sph + 4 * k);
        float s4[4] = {t.x, t.y, t.z, t.w};
        float c[3] = {B.x[0] + R[0] * s4[0] + R[1] * s4[1] + R[2] * s4[2],
                      B.x[1] + R[3] * s4[0] + R[4] * s4[1] + R[5] * s4[2],
                      B.x[2] + R[6] * s4[0] + R[7] * s4[1] + R[8] * s4[2]};
        float d, n[3], p[3], vl[3];
        pair_contact(seg, l, L, c, s4[3], d, n, p, vl);
        float t1[3], t2[3];
        tangent_frame(n, t1, t2);
        F[0] = n[0]; F[1] = n[1]; F[2] = n[2];
        F[3] = t1[0]; F[4] = t1[1]; F[5] = t1[2];
        F[6] = t2[0]; F[7] = t2[1]; F[8] = t2[2];
        rho[0] = p[0] - B.x[0]; rho[1] = p[1] - B.x[1]; rho[2] = p[2] - B.x[2];
        float bn = d >= 0.f ? d / dt : P.erp * d / dt;
        ucst[0] = -(n[0] * vl[0] + n[1] * vl[1] + n[2] * vl[2]) + bn;
        ucst[1] = -(t1[0] * vl[0] + t1[1] * vl[1] + t1[2] * vl[2]);
        ucst[2] = -(t2[0] * vl[0] + t2[1] * vl[1] + t2[2] * vl[2]);
        link = l < L ? l : -1;
        // warm start from the previous step's impulse of the same key
        for (int j = 0; j < P.C_max; ++j) {
            if (lds.wkey[j] == key) {
                r[0] = lds.wr[3 * j]; r[1] = lds.wr[3 * j + 1]; r[2] = lds.wr[3 * j + 2];
                break;
            }
        }
    }

    // 5. Newton on the smoothed FB system.  The 3C x 3C Newton matrix
    //    A = blkdiag(JX) + blkdiag(JY) W, W = J M^-1 J^T + eps I, is reduced
    //    to the 6x6 system (I + M^-1 sum_c J_c^T P_c^-1 B_c J_c) dnu =
    //    -M^-1 sum_c J_c^T P_c^-1 Phi_c with P_c = JX_c + eps JY_c,
    //    B_c = JY_c; then dr_c = -P_c^-1 (Phi_c + B_c J_c dnu).
    const SR eps = P.compliance, kap = P.kappa, del = P.fb_delta, mu = B.mu;
    const SR imS = SR(1) / SR(m);
    SR IinvS[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) IinvS[i] = Iinv[i];
    const int span = lane_span(C);
    // M^-1 J^T x summed over contacts, for an impulse x of this lane
    auto body_dv = [&](const SR *x, SR *dn) {
        SR f[3] = {F[0] * x[0] + F[3] * x[1] + F[6] * x[2], F[1] * x[0] + F[4] * x[1] + F[7] * x[2],
                   F[2] * x[0] + F[5] * x[1] + F[8] * x[2]};
        SR tq[3];
        cross3(rho, f, tq);
        SR a6[6] = {f[0], f[1], f[2], tq[0], tq[1], tq[2]};
        wave_sum<SR, 6>(a6, span);
        dn[0] = a6[0] * imS; dn[1] = a6[1] * imS; dn[2] = a6[2] * imS;
        dn[3] = IinvS[0] * a6[3] + IinvS[1] * a6[4] + IinvS[2] * a6[5];
        dn[4] = IinvS[3] * a6[3] + IinvS[4] * a6[4] + IinvS[5] * a6[5];
        dn[5] = IinvS[6] * a6[3] + IinvS[7] * a6[4] + IinvS[8] * a6[5];
    };
    // current body velocity nu = nu* + M^-1 J^T r
    SR nu[6];
    body_dv(r, nu);
    nu[0] += vs[0]; nu[1] += vs[1]; nu[2] += vs[2];
    nu[3] += ws[0]; nu[4] += ws[1]; nu[5] += ws[2];
    if (C > 0) {
        for (int it = 0; it < P.newton_iters; ++it) {
            // relative velocity u = F (v + w x rho) + ucst + eps r
            SR pv[3];
            SR nw3[3] = {nu[3], nu[4], nu[5]};
            cross3(nw3, rho, pv);
            pv[0] += nu[0]; pv[1] += nu[1]; pv[2] += nu[2];
            SR u[3] = {dot3(F, pv) + ucst[0] + eps * r[0], dot3(F + 3, pv) + ucst[1] + eps * r[1],
                       dot3(F + 6, pv) + ucst[2] + eps * r[2]};
            FBOut<SR> fo;
            fb_value(mu, kap, del, r, u, fo);
            SR JX[9], JY[9];
            fb_jacobian(mu, kap, u, fo, JX, JY);
            SR Pm[9], Pi[9], Q[9], g[3];
#pragma unroll
            for (int i = 0; i < 9; ++i) Pm[i] = JX[i] + eps * JY[i];
            inv3(Pm, Pi);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Q[3 * i + j] = Pi[3 * i] * JY[j] + Pi[3 * i + 1] * JY[3 + j] + Pi[3 * i + 2] * JY[6 + j];
                g[i] = Pi[3 * i] * fo.phi[0] + Pi[3 * i + 1] * fo.phi[1] + Pi[3 * i + 2] * fo.phi[2];
            }
            // world-frame blocks: Qw = F^T Q F, gw = F^T g
            SR QF[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    QF[3 * i + j] = Q[3 * i] * F[j] + Q[3 * i + 1] * F[3 + j] + Q[3 * i + 2] * F[6 + j];
            SR acc[43];
            SR Qw[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Qw[3 * i + j] = F[i] * QF[j] + F[3 + i] * QF[3 + j] + F[6 + i] * QF[6 + j];
            SR gw[3] = {F[0] * g[0] + F[3] * g[1] + F[6] * g[2], F[1] * g[0] + F[4] * g[1] + F[7] * g[2],
                        F[2] * g[0] + F[5] * g[1] + F[8] * g[2]};
            // A6 = [[Qw, -Qw rhat], [rhat Qw, -rhat Qw rhat]]; row i of Qw rhat = q_i x rho
            SR X[9];
#pragma unroll
            for (int i = 0; i < 3; ++i) cross3(Qw + 3 * i, rho, X + 3 * i);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    acc[6 * i + j] = Qw[3 * i + j];
                    acc[6 * i + 3 + j] = -X[3 * i + j];
                }
            // bottom blocks: columns rho x (column j of Qw), -(rho x column j of X)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                SR cq[3] = {Qw[j], Qw[3 + j], Qw[6 + j]}, cx[3] = {X[j], X[3 + j], X[6 + j]};
                SR a3[3], b3[3];
                cross3(rho, cq, a3);
                cross3(rho, cx, b3);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    acc[6 * (3 + i) + j] = a3[i];
                    acc[6 * (3 + i) + 3 + j] = -b3[i];
                }
            }
            SR tg[3];
            cross3(rho, gw, tg);
            acc[36] = gw[0]; acc[37] = gw[1]; acc[38] = gw[2];
            acc[39] = tg[0]; acc[40] = tg[1]; acc[41] = tg[2];
            acc[42] = SR(0.5) * (fo.phi[0] * fo.phi[0] + fo.phi[1] * fo.phi[1] + fo.phi[2] * fo.phi[2]);
            if (!act) {
#pragma unroll
                for (int i = 0; i < 43; ++i) acc[i] = SR(0);
            }
            wave_sum<SR, 43>(acc, span);
            const SR psi = acc[42];
            // (I + M^-1 A6) dnu = -M^-1 b6
            SR S6[36], rhs[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                S6[j] = acc[j] * imS + (j == 0 ? SR(1) : SR(0));
                S6[6 + j] = acc[6 + j] * imS + (j == 1 ? SR(1) : SR(0));
                S6[12 + j] = acc[12 + j] * imS + (j == 2 ? SR(1) : SR(0));
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    S6[6 * (3 + i) + j] = IinvS[3 * i] * acc[18 + j] + IinvS[3 * i + 1] * acc[24 + j] +
                                          IinvS[3 * i + 2] * acc[30 + j] + (j == 3 + i ? SR(1) : SR(0));
            }
            rhs[0] = -acc[36] * imS; rhs[1] = -acc[37] * imS; rhs[2] = -acc[38] * imS;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                rhs[3 + i] = -(IinvS[3 * i] * acc[39] + IinvS[3 * i + 1] * acc[40] + IinvS[3 * i + 2] * acc[41]);
            solve6(S6, rhs);
            // dr = -g - Q F (dv + dw x rho)
            SR dp[3];
            SR dw3[3] = {rhs[3], rhs[4], rhs[5]};
            cross3(dw3, rho, dp);
            dp[0] += rhs[0]; dp[1] += rhs[1]; dp[2] += rhs[2];
            SR dr[3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                dr[i] = -g[i] - (QF[3 * i] * dp[0] + QF[3 * i + 1] * dp[1] + QF[3 * i + 2] * dp[2]);
            if (!act) { dr[0] = dr[1] = dr[2] = SR(0); }
            // body-velocity change of the step, M^-1 J^T dr, summed afresh so
            // that the tracked velocity stays consistent with r (the 6x6
            // solution equals it only up to the Schur system's conditioning)
            SR dn[6];
            body_dv(dr, dn);
            // du = W dr = F (dn_v + dn_w x rho) + eps dr
            SR dq[3];
            SR dnw[3] = {dn[3], dn[4], dn[5]};
            cross3(dnw, rho, dq);
            dq[0] += dn[0]; dq[1] += dn[1]; dq[2] += dn[2];
            SR du[3] = {dot3(F, dq) + eps * dr[0], dot3(F + 3, dq) + eps * dr[1], dot3(F + 6, dq) + eps * dr[2]};
            // Armijo backtracking over alpha = 1, 1/2, 1/4, 1/8 (1/8 if none passes)
            SR alpha = SR(0.125);
            SR a = SR(1);
            for (int t = 0; t < 4; ++t, a *= SR(0.5)) {
                SR rt[3] = {r[0] + a * dr[0], r[1] + a * dr[1], r[2] + a * dr[2]};
                SR ut[3] = {u[0] + a * du[0], u[1] + a * du[1], u[2] + a * du[2]};
                SR ptr = act ? fb_merit(mu, kap, del, rt, ut) : SR(0);
                ptr = wave_sum1(ptr, span);
                if (ptr <= (SR(1) - SR(2) * SR(P.armijo_sigma) * a) * psi) { alpha = a; break; }
            }
            r[0] += alpha * dr[0]; r[1] += alpha * dr[1]; r[2] += alpha * dr[2];
#pragma unroll
            for (int i = 0; i < 6; ++i) nu[i] += alpha * dn[i];
        }
    }

    // 6. integrate: nu+ = nu* + M^-1 J^T r (fresh sum), x += dt v+,
    //    q <- normalize(Exp(dt w+) q), angular-momentum-preserving w remap
    SR impS[3] = {F[0] * r[0] + F[3] * r[1] + F[6] * r[2], F[1] * r[0] + F[4] * r[1] + F[7] * r[2],
                  F[2] * r[0] + F[5] * r[1] + F[8] * r[2]};
    if (!act) { impS[0] = impS[1] = impS[2] = SR(0); }
    float vp[3], wp[3];
    {
        SR dv[6];
        body_dv(r, dv);
        vp[0] = (float)(SR(vs[0]) + dv[0]); vp[1] = (float)(SR(vs[1]) + dv[1]); vp[2] = (float)(SR(vs[2]) + dv[2]);
        wp[0] = (float)(SR(ws[0]) + dv[3]); wp[1] = (float)(SR(ws[1]) + dv[4]); wp[2] = (float)(SR(ws[2]) + dv[5]);
    }
    float xn[3] = {B.x[0] + dt * vp[0], B.x[1] + dt * vp[1], B.x[2] + dt * vp[2]};
    float th[3] = {dt * wp[0], dt * wp[1], dt * wp[2]};
    float an = sqrtf(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    float eq[4];
    if (an < 1e-4f) {
        float a2 = an * an;
        float sc = 0.5f - a2 / 48.f;
        eq[0] = 1.f - a2 / 8.f; eq[1] = sc * th[0]; eq[2] = sc * th[1]; eq[3] = sc * th[2];
    } else {
        float sc = sinf(0.5f * an) / an;
        eq[0] = cosf(0.5f * an); eq[1] = sc * th[0]; eq[2] = sc * th[1]; eq[3] = sc * th[2];
    }
    float q2[4];
    quat_mul(eq, q, q2);
    float qi = rsqrtf(q2[0] * q2[0] + q2[1] * q2[1] + q2[2] * q2[2] + q2[3] * q2[3]);
    q2[0] *= qi; q2[1] *= qi; q2[2] *= qi; q2[3] *= qi;
    // h = I_w(q) w+ in body components, carried to the new orientation
    float wb[3] = {R[0] * wp[0] + R[3] * wp[1] + R[6] * wp[2], R[1] * wp[0] + R[4] * wp[1] + R[7] * wp[2],
                   R[2] * wp[0] + R[5] * wp[1] + R[8] * wp[2]};
    float hb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) hb[i] = inv_in[i] > 0.f ? wb[i] * m / inv_in[i] : 0.f;
    float h[3] = {R[0] * hb[0] + R[1] * hb[1] + R[2] * hb[2], R[3] * hb[0] + R[4] * hb[1] + R[5] * hb[2],
                  R[6] * hb[0] + R[7] * hb[1] + R[8] * hb[2]};
    float Rn[9];
    quat_to_mat(q2, Rn);
    float hn[3] = {Rn[0] * h[0] + Rn[3] * h[1] + Rn[6] * h[2], Rn[1] * h[0] + Rn[4] * h[1] + Rn[7] * h[2],
                   Rn[2] * h[0] + Rn[5] * h[1] + Rn[8] * h[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i) hn[i] *= ii[i];
    B.w[0] = Rn[0] * hn[0] + Rn[1] * hn[1] + Rn[2] * hn[2];
    B.w[1] = Rn[3] * hn[0] + Rn[4] * hn[1] + Rn[5] * hn[2];
    B.w[2] = Rn[6] * hn[0] + Rn[7] * hn[1] + Rn[8] * hn[2];
    B.x[0] = xn[0]; B.x[1] = xn[1]; B.x[2] = xn[2];
    B.q[0] = q2[0]; B.q[1] = q2[1]; B.q[2] = q2[2]; B.q[3] = q2[3];
    B.v[0] = vp[0]; B.v[1] = vp[1]; B.v[2] = vp[2];
    B.f[0] = B.f[1] = B.f[2] = 0.f;

    // 7. new warm cache slot and contact output of this lane
    wkey = act ? key : -1;
    wr[0] = act ? (float)r[0] : 0.f;
    wr[1] = act ? (float)r[1] : 0.f;
    wr[2] = act ? (float)r[2] : 0.f;
    out_link = act ? link : -1;
    out_imp[0] = (float)impS[0]; out_imp[1] = (float)impS[1]; out_imp[2] = (float)impS[2];
}

}  // namespace pt
