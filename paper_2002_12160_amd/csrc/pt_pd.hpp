// pt_pd.hpp -- one step of one simulation with the PD-controlled hand
// (hand_mode 1), executed by one wavefront.  Sec. III-A lets the state hold
// the joint angles of articulated bodies and the observation the measured
// joint angles; Sec. IV-A drives the simulated hand by PD gains.
//
// Model (the reading shared with the test oracle): revolute joints whose
// angles and rates (q, qdot) are state of every simulation; every capsule
// link a solid cylinder of the hand's link mass; the hand's gravity
// compensated and its velocity-product terms dropped, so the joint-space
// mass matrix M(q) is its only inertia; the PD law taken implicitly,
//   (M + dt kd I + dt^2 kp I) qdot+ = M qdot + dt kp (u - q) + (contact
//   impulses on the joints),  q+ = q + dt qdot+.
// Contacts couple the object's six velocities and the joint rates in one
// Newton system of size 6 + D per simulation (the kinematic path's solve with
// the hand's columns added).
//
// Structure used here.  The joints fall into independent groups (a finger's
// chain): no link is moved by joints of two groups, so the hand's block of
// the Newton matrix is block diagonal by group and couples only to the
// object's velocities.  Every joint's motion is written as a twist about
// the object's centre x: joint p turns the material point x + rho of the
// links it moves with velocity s_v + s_w x rho, s = (a x (x - o), a) for
// its axis a through o.  Per Newton iteration:
//   1. each contact's 6x6 block [I; rho^] Qw [I, -rho^] and vector
//      (gw, rho x gw) of the kinematic path, summed per link (the contacts
//      ordered by link) and over all contacts;
//   2. the object-hand blocks A_oh[:, p] = -Kbar_p s_p, A_ho[p, :] =
//      -s_p^T Kbar_p and b_h[p] = -s_p . kbar_p, Kbar_p the sum over the
//      links joint p moves; a hand-hand entry is -s_i . A_oh[:, j] when i is
//      above j in a chain, -A_ho[i, :] . s_j when j is above i, zero across
//      branches; X = A_h + that block;
//   3. per group, Y = X_g^-1 [A_ho | b_h] by Gaussian elimination with
//      partial pivoting;
//   4. the object's 6x6 Schur complement (A_oo - A_oh Y_A) z = -(b_o -
//      A_oh Y_b) through the kinematic path's 6x6 solve, then z_h = -Y_b -
//      Y_A z;
//   5. per contact dr = -g - Q F (dz_v + dz_w x rho), dz = z minus the twist
//      of the contact's link under z_h, and the Armijo line search of the
//      kinematic path.
// The hand kinematics and every hand quantity are float64; the contact
// geometry float32, as on the kinematic path.
#pragma once

#include "pt_internal.h"

namespace pt {

constexpr int PD_GMAX = 6;    // joints per group, at most
constexpr int PD_CHAIN = 8;   // joints moving one link, at most
constexpr int PD_MAX_D = 64;  // joints, at most (one lane per joint)
constexpr int PD_YS = 8;      // row stride of the group solutions (7 columns used)

struct PdConsts {
    int groups;        // independent joint groups
    int dmax;          // deepest link of the tree (roots at 0)
    int gmax;          // joints in the largest group
    float kp, kd, link_mass, w_q;
};

// The hand's structure, built on the host at batch creation (int32 table).
// Joints are numbered by position p: the groups' joints contiguous, group
// by group.
struct PdTab {
    const int32_t *t;
    int D, L;
    __device__ int jat(int p) const { return t[p]; }                     // joint at position p
    __device__ int pos(int j) const { return t[D + j]; }                 // position of joint j
    __device__ int gs(int p) const { return t[2 * D + p]; }              // first position of p's group
    __device__ int gn(int p) const { return t[3 * D + p]; }              // size of p's group
    __device__ uint64_t sub(int p) const                                 // links moved by p (bit l)
    {
        return (uint64_t)(uint32_t)t[4 * D + p] | ((uint64_t)(uint32_t)t[5 * D + p] << 32);
    }
    __device__ int depth(int l) const { return t[6 * D + l]; }
    __device__ int chain(int l, int i) const { return t[6 * D + L + l * PD_CHAIN + i]; }   // -1 padded
    __device__ int gfirst(int g) const { return t[6 * D + L + L * PD_CHAIN + g]; }        // [groups + 1]
};

__host__ __device__ constexpr size_t pd_tab_ints(int L, int D, int groups)
{
    return (size_t)6 * D + L + (size_t)L * PD_CHAIN + groups + 1;
}

// per-wave LDS of the PD step (after the kinematic path's WaveLds)
struct PdLds {
    double *S;      // [D][6] joint twists about the object centre (first: origin, axis)
    double *Ah;     // [D][PD_GMAX] rows of A_h's group blocks
    double *pm;     // [D] M qdot + dt kp (u - q)
    double *Aoh;    // [D][6] column p of A_oh
    double *Aho;    // [D][6] row p of A_ho
    double *bh;     // [D]
    double *X;      // [D][PD_GMAX]
    double *Y;      // [D][PD_YS]
    double *zh;     // [D] hand part of the Newton direction (first: q staged)
    double *nuh;    // [D] joint rates (first: qdot staged)
    double *tot;    // [48] sums over all contacts
    double *acc;    // [48] the object's reduced system
    int *rowlink;   // [64] link of each row of the ordered contacts
    int *linkrow;   // [64] first row of each link's run of rows (-1: no contact on the link)
};

// Up to PD_SPARE_D joints the group solve's X and Y live in the wave's cap
// slots, warm-cache lookup and contact stage (sel .. the stage's end, 576
// words), which nothing reads between the warm start and the integration:
// on the real-time hand (D = 20) that keeps the wave under 32 KiB, five
// wavefronts per compute unit instead of four.
constexpr int PD_SPARE_WORDS = 9 * 64;
constexpr int PD_SPARE_D = 4 * PD_SPARE_WORDS / (8 * (PD_GMAX + PD_YS));

__host__ __device__ constexpr size_t pd_lds_bytes(int D)
{
    return (size_t)8 * ((size_t)D * (6 + PD_GMAX + 1 + 6 + 6 + 1 + 1 + 1) + 96) +
           (D <= PD_SPARE_D ? 0 : (size_t)8 * D * (PD_GMAX + PD_YS)) + (size_t)4 * (64 + 64);
}

// LDS of the hand kinematics (in the candidate list, before the narrow
// phase): per link the tip frame's quaternion, the tip, the centre of mass
// and the world inertia
__host__ __device__ constexpr size_t pd_fk_bytes(int L) { return (size_t)8 * 19 * L; }

// p: the PD area after the wave's WaveLds; spare: that WaveLds's sel
__device__ __forceinline__ PdLds carve_pd(char *p, int D, int *spare)
{
    PdLds s;
    double *d = reinterpret_cast<double *>(p);
    s.S = d; d += 6 * D;
    s.Ah = d; d += PD_GMAX * D;
    s.pm = d; d += D;
    s.Aoh = d; d += 6 * D;
    s.Aho = d; d += 6 * D;
    s.bh = d; d += D;
    if (D <= PD_SPARE_D) {
        s.X = reinterpret_cast<double *>(spare);
        s.Y = s.X + PD_GMAX * D;
    } else {
        s.X = d; d += PD_GMAX * D;
        s.Y = d; d += PD_YS * D;
    }
    s.zh = d; d += D;
    s.nuh = d; d += D;
    s.tot = d; d += 48;
    s.acc = d; d += 48;
    int *i = reinterpret_cast<int *>(d);
    s.rowlink = i; i += 64;
    s.linkrow = i;
    return s;
}

// Kinematics of the hand at the joint angles staged in pl.zh (by position),
// link by link down the tree (links of one depth in parallel): per joint its
// world axis and origin into pl.S (origin, axis); per link its tip frame, tip,
// centre of mass and world inertia into fk, and its segment record (float,
// zero end velocities: the hand's motion enters through the joint rates)
// into seg.
__device__ __forceinline__ void pd_fk(const Consts &P, const PdConsts &Q, const PdTab &T,
                                      const float *__restrict__ hand, double *fk, const PdLds &pl, float *seg)
{
    const int L = P.L, lane = lane_id();
    double *tq = fk, *tb = fk + 4 * L, *com = fk + 7 * L, *Iw = fk + 10 * L;
    for (int d = 0; d <= Q.dmax; ++d) {
        for (int l = lane; l < L; l += WAVE) {
            if (T.depth(l) != d) continue;
            const float *h = hand + (size_t)l * HAND_STRIDE;
            const int parent = (int)h[0];
            double pq[4] = {1, 0, 0, 0}, pp[3] = {0, 0, 0};
            if (parent >= 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) pq[i] = tq[4 * parent + i];
#pragma unroll
                for (int i = 0; i < 3; ++i) pp[i] = tb[3 * parent + i];
            }
            double Rp[9];
            quat_to_mat_d(pq, Rp);
            const double off[3] = {h[9], h[10], h[11]};
            double o[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) o[i] = pp[i] + Rp[3 * i] * off[0] + Rp[3 * i + 1] * off[1] + Rp[3 * i + 2] * off[2];
            const double qo[4] = {h[12], h[13], h[14], h[15]};
            double qf[4];
            quat_mul_d(pq, qo, qf);
            for (int k = 0; k < 2; ++k) {
                const int j = (int)h[1 + k];
                if (j < 0) continue;
                const int p = T.pos(j);
                const double ax[3] = {h[3 + 3 * k], h[4 + 3 * k], h[5 + 3 * k]};
                double Rf[9];
                quat_to_mat_d(qf, Rf);
                double *s = pl.S + 6 * p;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    s[i] = o[i];
                    s[3 + i] = Rf[3 * i] * ax[0] + Rf[3 * i + 1] * ax[1] + Rf[3 * i + 2] * ax[2];
                }
                double sn, cs;
                sincos(0.5 * pl.zh[p], &sn, &cs);
                const double qj[4] = {cs, sn * ax[0], sn * ax[1], sn * ax[2]};
                double t[4];
                quat_mul_d(qf, qj, t);
#pragma unroll
                for (int i = 0; i < 4; ++i) qf[i] = t[i];
            }
            double R[9];
            quat_to_mat_d(qf, R);
            const double len = h[16], rad = h[17];
            double b[3], c[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                b[i] = o[i] + len * R[3 * i];
                c[i] = o[i] + 0.5 * len * R[3 * i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) tq[4 * l + i] = qf[i];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                tb[3 * l + i] = b[i];
                com[3 * l + i] = c[i];
            }
            // solid cylinder about its centre: axial m r^2 / 2, transverse m (3 r^2 + len^2) / 12
            const double ml = Q.link_mass;
            const double Ib[3] = {0.5 * ml * rad * rad, ml * (3 * rad * rad + len * len) / 12.0,
                                  ml * (3 * rad * rad + len * len) / 12.0};
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Iw[9 * l + 3 * i + j] =
                        R[3 * i] * Ib[0] * R[3 * j] + R[3 * i + 1] * Ib[1] * R[3 * j + 1] + R[3 * i + 2] * Ib[2] * R[3 * j + 2];
            float *sg = seg + (size_t)l * SEG_STRIDE;
            float a0[3], ab[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                a0[i] = (float)o[i];
                ab[i] = (float)(b[i] - o[i]);
            }
            const float L2 = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2];
            const float inv = sqrtf(L2) >= 1e-9f ? 1.f / L2 : 0.f;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                sg[i] = a0[i];
                sg[4 + i] = ab[i];
            }
            sg[3] = h[17];
            sg[7] = inv;
#pragma unroll
            for (int i = 8; i < 16; ++i) sg[i] = 0.f;
        }
        wave_sync();
    }
}

// The group blocks of A_h = M(q) + (dt kd + dt^2 kp) I and the momentum
// pm = M qdot + dt kp (u - q), one lane per joint (joint rates staged in
// pl.nuh by position).  M_ij sums over the links both joints move:
// m v_i . v_j + a_j . Iw a_i with v_i = a_i x (com - o_i).
__device__ __forceinline__ void pd_mass(const Consts &P, const PdConsts &Q, const PdTab &T, const double *fk,
                                        const PdLds &pl, const float *__restrict__ u, const double q_lane)
{
    const int L = P.L, D = P.D, lane = lane_id();
    const double *com = fk + 7 * L, *Iw = fk + 10 * L;
    const double dt = P.dt, cdiag = dt * (double)Q.kd + dt * dt * (double)Q.kp, ml = Q.link_mass;
    if (lane < D) {
        const int p = lane;
        const int g0 = T.gs(p), n = T.gn(p);
        const uint64_t sp = T.sub(p);
        const double *op = pl.S + 6 * p, *ap = op + 3;
        double mom = 0.0;
        for (int k = 0; k < n; ++k) {
            const int j = g0 + k;
            const double *oj = pl.S + 6 * j, *aj = oj + 3;
            uint64_t in = sp & T.sub(j);
            double m = 0.0;
            while (in) {
                const int l = __builtin_ctzll(in);
                in &= in - 1;
                const double *c = com + 3 * l, *I = Iw + 9 * l;
                const double ri[3] = {c[0] - op[0], c[1] - op[1], c[2] - op[2]};
                const double rj[3] = {c[0] - oj[0], c[1] - oj[1], c[2] - oj[2]};
                double vi[3], vj[3];
                cross3(ap, ri, vi);
                cross3(aj, rj, vj);
                const double Ia[3] = {I[0] * ap[0] + I[1] * ap[1] + I[2] * ap[2],
                                      I[3] * ap[0] + I[4] * ap[1] + I[5] * ap[2],
                                      I[6] * ap[0] + I[7] * ap[1] + I[8] * ap[2]};
                m += ml * dot3(vi, vj) + dot3(aj, Ia);
            }
            pl.Ah[PD_GMAX * p + k] = m + (j == p ? cdiag : 0.0);
            mom += m * pl.nuh[j];
        }
        pl.pm[p] = mom + dt * (double)Q.kp * ((double)u[T.jat(p)] - q_lane);
    }
    wave_sync();
}

// joint origins and axes in pl.S become twists about the object centre x
__device__ __forceinline__ void pd_twists(int D, const float *x, const PdLds &pl)
{
    const int lane = lane_id();
    if (lane < D) {
        double *s = pl.S + 6 * lane;
        const double r[3] = {(double)x[0] - s[0], (double)x[1] - s[1], (double)x[2] - s[2]};
        const double a[3] = {s[3], s[4], s[5]};
        double v[3];
        cross3(a, r, v);
        s[0] = v[0]; s[1] = v[1]; s[2] = v[2];
    }
    wave_sync();
}

// Orders the contacts by (link, lane): pos = this contact's row; ends (bit r)
// marks the rows that close a run of rows with one link, and linkrow the
// first row of each link's run (-1: no contact on the link).
__device__ __forceinline__ void pd_order_contacts(const StepState<double> &st, const PdLds &pl, int &pos,
                                                  uint64_t &ends)
{
    const int lane = lane_id(), C = st.C;
    const int lk = st.act ? st.l : 0x7fffffff;
    int ps = 0;
    for (int c = 0; c < C; ++c) {
        const int o = __builtin_amdgcn_readlane(lk, c);
        ps += (o < lk || (o == lk && c < lane)) ? 1 : 0;
    }
    pos = ps;
    pl.linkrow[lane] = -1;
    if (st.act) pl.rowlink[ps] = lk;
    wave_sync();
    const bool start = lane < C && (lane == 0 || pl.rowlink[lane - 1] != pl.rowlink[lane]);
    const bool end = lane < C && (lane == C - 1 || pl.rowlink[lane + 1] != pl.rowlink[lane]);
    if (start) pl.linkrow[pl.rowlink[lane]] = lane;
    ends = __ballot(end);
    wave_sync();
}

// Sums of N values per contact over each run of rows (one link) and over all
// contacts: an active lane writes its values as row `pos` (the contacts are
// lanes 0 .. C-1) and lanes C .. C16-1 zero rows C .. C16-1 (C16 = C rounded
// up to 16), so that lanes e < N then read the rows sixteen at a time with
// no bounds test and add them in row order (the zeros after the last run
// change nothing), each run's sum overwriting its first row (a lane only
// rewrites its own column of a row it has read) and the total landing in
// tot[e].  The runs' ends (bit r of ends, r < C) are wave-uniform, so the
// scan branches on them in scalar code.  buf: 16-byte aligned rows of
// RedStride<double> doubles, at least C16 of them.
template <int N>
__device__ __forceinline__ void pd_segsum(const double (&v)[N], bool act, int pos, int C, uint64_t ends,
                                          double *buf, double *tot)
{
    constexpr int RS = RedStride<double>::value;
    static_assert(N <= RS, "row too long");
    const int lane = lane_id();
    const int C16 = (C + 15) & ~15;
    if (act) {
        double *row = buf + pos * RS;
#pragma unroll
        for (int j = 0; j + 2 <= N; j += 2) store16<double>(row + j, v + j);
        if (N % 2) row[N - 1] = v[N - 1];
    } else if (lane >= C && lane < C16) {
        double *row = buf + lane * RS;
        const double z[2] = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j + 2 <= N; j += 2) store16<double>(row + j, z);
        if (N % 2) row[N - 1] = 0.0;
    }
    wave_sync();
    if (lane < N) {
        double t = 0.0, a = 0.0;
        int start = 0;
        for (int r0 = 0; r0 < C; r0 += 16) {
            double x[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) x[k] = buf[(r0 + k) * RS + lane];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int r = r0 + k;
                a += x[k];
                if ((ends >> r) & 1ull) {
                    buf[start * RS + lane] = a;
                    t += a;
                    a = 0.0;
                    start = r + 1;
                }
            }
        }
        tot[lane] = t;
    }
    wave_sync();
}

// X_g y = b for every group g and right-hand side c (one lane per pair):
// b's entry at position p is B1[p ld1 + c] for c < n1 and B2[p] for c == n1
// (when B2 is given); y goes to Y[p ldy + c].  Gaussian elimination with
// partial pivoting on the block padded to G (the batch's largest group,
// at most PD_GMAX; rows of X at stride PD_GMAX) with the identity.
template <int G>
__device__ __forceinline__ void pd_group_solve(const PdTab &T, int groups, const double *X, const double *B1, int ld1,
                                               int n1, const double *B2, double *Y, int ldy)
{
    const int ncol = n1 + (B2 ? 1 : 0);
    for (int t = lane_id(); t < groups * ncol; t += WAVE) {
        const int g = t / ncol, c = t - g * ncol;
        const int g0 = T.gfirst(g), n = T.gfirst(g + 1) - g0;
        double a[G][G], y[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
#pragma unroll
            for (int k = 0; k < G; ++k)
                a[i][k] = (i < n && k < n) ? X[PD_GMAX * (g0 + i) + k] : (i == k ? 1.0 : 0.0);
            y[i] = i < n ? (c < n1 ? B1[(size_t)(g0 + i) * ld1 + c] : B2[g0 + i]) : 0.0;
        }
#pragma unroll
        for (int k = 0; k < G; ++k) {
#pragma unroll
            for (int i = k + 1; i < G; ++i) {
                const bool sw = fabs(a[i][k]) > fabs(a[k][k]);
#pragma unroll
                for (int m = k; m < G; ++m) {
                    const double hi = a[i][m], lo = a[k][m];
                    a[k][m] = sw ? hi : lo;
                    a[i][m] = sw ? lo : hi;
                }
                const double yi = y[i], yk = y[k];
                y[k] = sw ? yi : yk;
                y[i] = sw ? yk : yi;
            }
            const double inv = 1.0 / a[k][k];
#pragma unroll
            for (int i = k + 1; i < G; ++i) {
                const double f = a[i][k] * inv;
#pragma unroll
                for (int m = k + 1; m < G; ++m) a[i][m] -= f * a[k][m];
                y[i] -= f * y[k];
            }
        }
#pragma unroll
        for (int k = G - 1; k >= 0; --k) {
            double s = y[k];
#pragma unroll
            for (int m = k + 1; m < G; ++m) s -= a[k][m] * y[m];
            y[k] = s / a[k][k];
        }
#pragma unroll
        for (int i = 0; i < G; ++i)
            if (i < n) Y[(size_t)(g0 + i) * ldy + c] = y[i];
    }
}

// twist of link l (l == L: the table, none) under joint rates w: the sum of
// s_p w_p over the joints moving it
__device__ __forceinline__ void pd_link_twist(const PdTab &T, int l, int L, const double *S, const double *w,
                                              double *tw)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) tw[k] = 0.0;
    if (l < 0 || l >= L) return;
    for (int i = 0; i < PD_CHAIN; ++i) {
        const int p = T.chain(l, i);
        if (p < 0) break;
        const double wp = w[p];
#pragma unroll
        for (int k = 0; k < 6; ++k) tw[k] += S[6 * p + k] * wp;
    }
}

// Joint rates for the impulses st.r: A_h qdot = pm + (joint impulse of the
// contacts), the joint impulse -s_p . (sum of the wrenches (f, rho x f)
// about x on the links p moves), f the impulse on the object.  To pl.nuh.
template <int G>
__device__ __forceinline__ void pd_hand_rates(const Consts &P, const PdConsts &Q, const PdTab &T,
                                              const StepState<double> &st, int pos, uint64_t ends, double *red,
                                              const PdLds &pl)
{
    constexpr int RS = RedStride<double>::value;
    const int lane = lane_id(), D = P.D;
    double w6[6] = {0, 0, 0, 0, 0, 0};
    if (st.act) {
        const double *F = st.F, *r = st.r;
        const double f[3] = {F[0] * r[0] + F[3] * r[1] + F[6] * r[2], F[1] * r[0] + F[4] * r[1] + F[7] * r[2],
                             F[2] * r[0] + F[5] * r[1] + F[8] * r[2]};
        double t[3];
        cross3(st.rho, f, t);
        w6[0] = f[0]; w6[1] = f[1]; w6[2] = f[2];
        w6[3] = t[0]; w6[4] = t[1]; w6[5] = t[2];
    }
    pd_segsum<6>(w6, st.act, pos, st.C, ends, red, pl.tot);
    if (lane < D) {
        const double *sp = pl.S + 6 * lane;
        double tau = 0.0;
        for (uint64_t sb = T.sub(lane); sb; sb &= sb - 1) {
            const int r0 = pl.linkrow[__builtin_ctzll(sb)];
            if (r0 >= 0) {
                const double *row = red + r0 * RS;
#pragma unroll
                for (int k = 0; k < 6; ++k) tau -= sp[k] * row[k];
            }
        }
        pl.zh[lane] = pl.pm[lane] + tau;
    }
    wave_sync();
    pd_group_solve<G>(T, Q.groups, pl.Ah, pl.zh, 1, 1, nullptr, pl.nuh, 1);
    wave_sync();
}

// The contact solve of a PD step (the kinematic path's Newton method over
// the generalised velocity (v, w, qdot)); leaves st.r, st.nu (object) and
// pl.nuh (joint rates) for the final impulses.
template <int G>
__device__ __forceinline__ void step_solve_pd(const Consts &P, const PdConsts &Q, const PdTab &T,
                                              StepState<double> &st, float mu_f, const float *inv_in, double *red,
                                              const PdLds &pl, int pos, uint64_t ends)
{
    using SR = double;
    constexpr int RS = RedStride<double>::value;
    const SR eps = P.compliance, kap = P.kappa, del = P.fb_delta, mu = mu_f;
    const int lane = lane_id(), L = P.L, D = P.D;
    BodyMass<SR> Mb;
    body_mass<SR>(st.m, st.Iinv, inv_in, Mb);
    const bool act = st.act;
    SR *r = st.r;
    const SR *F = st.F, *rho = st.rho;
    SR nu[6];
    body_dv(st, r, nu);
    nu[0] += st.vs[0]; nu[1] += st.vs[1]; nu[2] += st.vs[2];
    nu[3] += st.ws[0]; nu[4] += st.ws[1]; nu[5] += st.ws[2];
    pd_hand_rates<G>(P, Q, T, st, pos, ends, red, pl);
    st.psi_end = st.C > 0 && P.newton_iters == 0 ? SR(-1) : SR(0);
    if (st.C > 0) {
        SR u[3];
        {
            SR tw[6], ne[6];
            pd_link_twist(T, st.l, L, pl.S, pl.nuh, tw);
#pragma unroll
            for (int k = 0; k < 6; ++k) ne[k] = nu[k] - tw[k];
            rel_velocity(st, ne, r, eps, u);
        }
        FBOut<SR> fo;
        fb_value(mu, kap, del, r, u, fo);
        for (int it = 0; it < P.newton_iters; ++it) {
            SR JX[9], JY[9];
            fb_jacobian(mu, kap, u, fo, JX, JY);
            SR Pm[9], Pi[9], Qc[9], g[3];
#pragma unroll
            for (int i = 0; i < 9; ++i) Pm[i] = JX[i] + eps * JY[i];
            inv3(Pm, Pi);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Qc[3 * i + j] = Pi[3 * i] * JY[j] + Pi[3 * i + 1] * JY[3 + j] + Pi[3 * i + 2] * JY[6 + j];
                g[i] = Pi[3 * i] * fo.phi[0] + Pi[3 * i + 1] * fo.phi[1] + Pi[3 * i + 2] * fo.phi[2];
            }
            SR QF[9], Qw[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    QF[3 * i + j] = Qc[3 * i] * F[j] + Qc[3 * i + 1] * F[3 + j] + Qc[3 * i + 2] * F[6 + j];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Qw[3 * i + j] = F[i] * QF[j] + F[3 + i] * QF[3 + j] + F[6 + i] * QF[6 + j];
            const SR gw[3] = {F[0] * g[0] + F[3] * g[1] + F[6] * g[2], F[1] * g[0] + F[4] * g[1] + F[7] * g[2],
                              F[2] * g[0] + F[5] * g[1] + F[8] * g[2]};
            SR acc[43];
            schur_contribution(Qw, gw, rho, acc);
            acc[42] = SR(0.5) * (fo.phi[0] * fo.phi[0] + fo.phi[1] * fo.phi[1] + fo.phi[2] * fo.phi[2]);
            // 1. per-link and total sums
            pd_segsum<43>(acc, act, pos, st.C, ends, red, pl.tot);
            const SR psi = pl.tot[42];
            // 2. object-hand blocks
            for (int t = lane; t < 6 * D; t += WAVE) {
                const int p = t / 6, k = t - 6 * (t / 6);
                const SR *sp = pl.S + 6 * p;
                SR aoh = 0, aho = 0, bh = 0;
                for (uint64_t sb = T.sub(p); sb; sb &= sb - 1) {
                    const int r0 = pl.linkrow[__builtin_ctzll(sb)];
                    if (r0 >= 0) {
                        const SR *K = red + r0 * RS;
#pragma unroll
                        for (int m = 0; m < 6; ++m) {
                            aoh -= K[6 * k + m] * sp[m];
                            aho -= sp[m] * K[6 * m + k];
                        }
                        if (k == 0) {
#pragma unroll
                            for (int m = 0; m < 6; ++m) bh -= sp[m] * K[36 + m];
                        }
                    }
                }
                pl.Aoh[6 * p + k] = aoh;
                pl.Aho[6 * p + k] = aho;
                if (k == 0) pl.bh[p] = bh;
            }
            wave_sync();
            for (int t = lane; t < PD_GMAX * D; t += WAVE) {
                const int p = t / PD_GMAX, k = t - PD_GMAX * (t / PD_GMAX);
                if (k < T.gn(p)) {
                    const int j = T.gs(p) + k;
                    const uint64_t si = T.sub(p), sj = T.sub(j), in = si & sj;
                    SR h = 0;
                    if (in != 0) {
                        const SR *a = in == sj ? pl.S + 6 * p : pl.Aho + 6 * p;
                        const SR *b = in == sj ? pl.Aoh + 6 * j : pl.S + 6 * j;
#pragma unroll
                        for (int m = 0; m < 6; ++m) h -= a[m] * b[m];
                    }
                    pl.X[PD_GMAX * p + k] = pl.Ah[PD_GMAX * p + k] + h;
                }
            }
            wave_sync();
            // 3. Y = X^-1 [A_ho | b_h] per group
            pd_group_solve<G>(T, Q.groups, pl.X, pl.Aho, 6, 6, pl.bh, pl.Y, PD_YS);
            wave_sync();
            // 4. the object's reduced 6x6 system and its solve
            if (lane < 42) {
                SR s = pl.tot[lane];
                const int rr = lane < 36 ? lane / 6 : lane - 36, cc = lane < 36 ? lane - 6 * (lane / 6) : 6;
                for (int p = 0; p < D; ++p) s -= pl.Aoh[6 * p + rr] * pl.Y[PD_YS * p + cc];
                pl.acc[lane] = s;
            }
            wave_sync();
            SR z[6];
            schur_solve(pl.acc, Mb, z);
            if (lane < D) {
                SR zh = -pl.Y[PD_YS * lane + 6];
#pragma unroll
                for (int c = 0; c < 6; ++c) zh -= pl.Y[PD_YS * lane + c] * z[c];
                pl.zh[lane] = zh;
            }
            wave_sync();
            // 5. impulse direction, velocity change, line search
            SR dz[6];
            {
                SR tw[6];
                pd_link_twist(T, st.l, L, pl.S, pl.zh, tw);
#pragma unroll
                for (int k = 0; k < 6; ++k) dz[k] = z[k] - tw[k];
            }
            SR dp[3];
            {
                const SR dw3[3] = {dz[3], dz[4], dz[5]};
                cross3(dw3, rho, dp);
                dp[0] += dz[0]; dp[1] += dz[1]; dp[2] += dz[2];
            }
            SR dr[3], du[3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                dr[i] = act ? -g[i] - (QF[3 * i] * dp[0] + QF[3 * i + 1] * dp[1] + QF[3 * i + 2] * dp[2]) : SR(0);
            du[0] = dot3(F, dp) + eps * dr[0];
            du[1] = dot3(F + 3, dp) + eps * dr[1];
            du[2] = dot3(F + 6, dp) + eps * dr[2];
            // Armijo backtracking over alpha = 1, 1/2, 1/4, 1/8 (1/8 if none
            // passes); the last trial evaluated is the one taken
            SR a = SR(1);
            SR rt[3], ut[3];
            FBOut<SR> ft;
            for (int tr = 0; tr < 4; ++tr, a *= SR(0.5)) {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    rt[i] = r[i] + a * dr[i];
                    ut[i] = u[i] + a * du[i];
                }
                fb_value(mu, kap, del, rt, ut, ft);
                SR ptr = act ? SR(0.5) * (ft.phi[0] * ft.phi[0] + ft.phi[1] * ft.phi[1] + ft.phi[2] * ft.phi[2])
                             : SR(0);
                ptr = wave_sum1(ptr, st.span);
                st.psi_end = ptr;
                if (ptr <= (SR(1) - SR(2) * SR(P.armijo_sigma) * a) * psi) break;
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                r[i] = rt[i];
                u[i] = ut[i];
            }
            fo = ft;
        }
    }
    // fresh sums for the final impulses
    body_dv(st, r, st.nu);
    st.nu[0] += st.vs[0]; st.nu[1] += st.vs[1]; st.nu[2] += st.vs[2];
    st.nu[3] += st.ws[0]; st.nu[4] += st.ws[1]; st.nu[5] += st.ws[2];
    pd_hand_rates<G>(P, Q, T, st, pos, ends, red, pl);
}

// The joint state of a step staged by position (lane p: the joint at
// position p), twist rows cleared (a joint that moves no link keeps zeros).
__device__ __forceinline__ void pd_stage_joints(int D, const PdLds &pl, float q, float qd)
{
    const int lane = lane_id();
    if (lane < D) {
        pl.zh[lane] = q;
        pl.nuh[lane] = qd;
#pragma unroll
        for (int k = 0; k < 6; ++k) pl.S[6 * lane + k] = 0.0;
    }
    wave_sync();
}

// One step of one simulation with the PD hand, the joint state staged by
// pd_stage_joints (q_lane: this lane's joint angle): kinematics and mass
// matrix at the joint angles, narrow phase and cap, the (6 + D) contact
// solve and the object's integration.  The joint rates leave in pl.nuh;
// link and imp are this lane's kept contact (as step_finish gives them).
template <bool SDF, int G>
__device__ __forceinline__ void pd_step(const Consts &P, const PdConsts &Q, const Tables &tb, const PdTab &T,
                                        const float *__restrict__ u, const WaveLds &lds, const PdLds &pl,
                                        const float *__restrict__ sph, int S, const float *inv, const SdfRef &sdf,
                                        float q_lane, Body &B, int &wkey, float *wr, StepStats &stats, int &link,
                                        float *imp)
{
    double *fk = reinterpret_cast<double *>(lds.cand_d);
    pd_fk(P, Q, T, tb.hand, fk, pl, lds.seg);
    pd_mass(P, Q, T, fk, pl, u, (double)q_lane);
    pd_twists(P.D, B.x, pl);
    StepState<double> sst;
    step_setup<double, SDF>(P, lds.seg, sph, S, inv, B, wkey, wr, lds, stats, sst, sdf);
    int pos;
    uint64_t ends;
    pd_order_contacts(sst, pl, pos, ends);
    step_solve_pd<G>(P, Q, T, sst, B.mu, inv, reinterpret_cast<double *>(lds.cand_d), pl, pos, ends);
    step_finish<double>(P, sst, inv, B, wkey, wr, link, imp);
}

// The joint-angle term of the step cost (Eq. 3's w_1 term), added to the
// running sum cs: w_q (q - q_gt)^2.
__device__ __forceinline__ float pd_joint_cost(float cs, float w_q, float q, float q_gt)
{
    const float d = q - q_gt;
    return cs + w_q * d * d;
}

}  // namespace pt
