// pt_adjoint.hpp -- hand-written adjoint of one simulation step (one
// wavefront per simulation), for gradients of a window's cost with respect to
// the window-start pose, twist, mass and friction.
//
// The contact impulses r are the solution of Phi(r; u, mu) = 0 with
// u = W r + u_free (the smoothed Fischer-Burmeister system); the adjoint
// treats the computed r as that solution and differentiates it implicitly:
// with A = dPhi/dr (the Newton matrix) it solves A^T lambda = r_bar through
// the transposed 6x6 Schur system, then u_free_bar = -JY^T lambda,
// W_bar = u_free_bar r^T and mu_bar = -lambda . dPhi/dmu.  Contact sets, the
// contact cap and the tangent-frame axis choice are held fixed (the gradient
// of the piecewise-smooth step on its current piece).
#pragma once

#include "pt_step.hpp"

namespace pt {

template <typename SR>
struct BodyBar {
    SR x[3], q[4], v[3], w[3];
};

// Rotation-matrix adjoint: qbar += dR(q)/dq^T [Rbar] (R row-major as quat_to_mat)
template <typename SR>
__device__ __forceinline__ void quat_to_mat_adj(const SR *q, const SR *Rb, SR *qb)
{
    SR w = q[0], x = q[1], y = q[2], z = q[3];
    qb[0] += SR(2) * (-z * Rb[1] + y * Rb[2] + z * Rb[3] - x * Rb[5] - y * Rb[6] + x * Rb[7]);
    qb[1] += SR(2) * (y * Rb[1] + z * Rb[2] + y * Rb[3] - SR(2) * x * Rb[4] - w * Rb[5] + z * Rb[6] + w * Rb[7] -
                      SR(2) * x * Rb[8]);
    qb[2] += SR(2) * (-SR(2) * y * Rb[0] + x * Rb[1] + w * Rb[2] + x * Rb[3] + z * Rb[5] - w * Rb[6] + z * Rb[7] -
                      SR(2) * y * Rb[8]);
    qb[3] += SR(2) * (-SR(2) * z * Rb[0] - w * Rb[1] + x * Rb[2] + w * Rb[3] - SR(2) * z * Rb[4] + y * Rb[5] +
                      x * Rb[6] + y * Rb[7]);
}

template <typename SR>
__device__ __forceinline__ void quat_to_mat_s(const SR *q, SR *R)
{
    SR w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = SR(1) - SR(2) * (y * y + z * z); R[1] = SR(2) * (x * y - w * z); R[2] = SR(2) * (x * z + w * y);
    R[3] = SR(2) * (x * y + w * z); R[4] = SR(1) - SR(2) * (x * x + z * z); R[5] = SR(2) * (y * z - w * x);
    R[6] = SR(2) * (x * z - w * y); R[7] = SR(2) * (y * z + w * x); R[8] = SR(1) - SR(2) * (x * x + y * y);
}

template <typename SR>
__device__ __forceinline__ void quat_mul_s(const SR *a, const SR *b, SR *o)
{
    o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

// adjoint of o = a (x) b (Hamilton): abar += ..., bbar += ...
template <typename SR>
__device__ __forceinline__ void quat_mul_adj(const SR *a, const SR *b, const SR *ob, SR *ab, SR *bb)
{
    ab[0] += ob[0] * b[0] + ob[1] * b[1] + ob[2] * b[2] + ob[3] * b[3];
    ab[1] += -ob[0] * b[1] + ob[1] * b[0] - ob[2] * b[3] + ob[3] * b[2];
    ab[2] += -ob[0] * b[2] + ob[1] * b[3] + ob[2] * b[0] - ob[3] * b[1];
    ab[3] += -ob[0] * b[3] - ob[1] * b[2] + ob[2] * b[1] + ob[3] * b[0];
    bb[0] += ob[0] * a[0] + ob[1] * a[1] + ob[2] * a[2] + ob[3] * a[3];
    bb[1] += -ob[0] * a[1] + ob[1] * a[0] + ob[2] * a[3] - ob[3] * a[2];
    bb[2] += -ob[0] * a[2] - ob[1] * a[3] + ob[2] * a[0] + ob[3] * a[1];
    bb[3] += -ob[0] * a[3] + ob[1] * a[2] - ob[2] * a[1] + ob[3] * a[0];
}

// M (symmetric 3x3) = R diag(dg) R^T;  adjoint given Mb: Rb += (Mb + Mb^T) R diag(dg),
// dgb_i = (R^T Mb R)_ii
template <typename SR>
__device__ __forceinline__ void rdr_adj(const SR *R, const SR *dg, const SR *Mb, SR *Rb, SR *dgb)
{
    SR S[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S[3 * i + j] = Mb[3 * i + j] + Mb[3 * j + i];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Rb[3 * i + j] += (S[3 * i] * R[j] + S[3 * i + 1] * R[3 + j] + S[3 * i + 2] * R[6 + j]) * dg[j];
    if (dgb) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            SR s = 0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) s += R[3 * i + k] * Mb[3 * i + j] * R[3 * j + k];
            dgb[k] += s;
        }
    }
}

// Adjoint of one step.  `st` holds the recomputed forward step (after
// step_setup and step_solve) for pre-step body B; gt is this step's observed
// sensor record ([4][L][G], group g); stage and stage2 are LDS scratch of
// 64 x 4 and 64 x 3 floats, red the LDS of the cross-contact sums.  bar: in = adjoint of the post-step state, out =
// adjoint of the pre-step state (x, q as stored, v, w); mbar and mubar
// accumulate; fbar (optional) receives the adjoint of the one-step external
// force.
template <typename SR>
__device__ void step_adjoint(const Consts &P, const float *__restrict__ seg, const float *__restrict__ sph,
                             const float *inv_in, const Body &B, const StepState<SR> &st,
                             const float *__restrict__ gt, int g, float *stage, float *stage2, SR *red,
                             BodyBar<SR> &bar, SR &mbar, SR &mubar, SR *fbar)
{
    const int lane = lane_id();
    const int L = P.L;
    const SR dt = P.dt;
    wave_sync();
    const SR eps = P.compliance, kap = P.kappa, del = P.fb_delta, mu = B.mu;
    const SR m = st.m, im = SR(1) / m;
    const bool act = st.act;
    const int span = st.span;
    const SR *F = st.F, *rho = st.rho, *r = st.r, *nu = st.nu;
    SR Iinv[9], R[9], q[4];
#pragma unroll
    for (int i = 0; i < 9; ++i) { Iinv[i] = st.Iinv[i]; R[i] = st.R[i]; }
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = st.q[i];
    SR Rbar[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    SR qbar[4] = {0, 0, 0, 0};

    // ---- (A) integration adjoint ------------------------------------
    SR wp[3] = {nu[3], nu[4], nu[5]};
    SR th[3] = {dt * wp[0], dt * wp[1], dt * wp[2]};
    SR an = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    SR eq[4];
    SR sc, cc = 0;
    const bool small = an < SR(1e-4);
    if (small) {
        SR a2 = an * an;
        sc = SR(0.5) - a2 / SR(48);
        eq[0] = SR(1) - a2 / SR(8);
    } else {
        sc = sin(SR(0.5) * an) / an;
        cc = cos(SR(0.5) * an);
        eq[0] = cc;
    }
    eq[1] = sc * th[0]; eq[2] = sc * th[1]; eq[3] = sc * th[2];
    SR qe2[4];
    quat_mul_s(eq, q, qe2);
    SR nq = sqrt(qe2[0] * qe2[0] + qe2[1] * qe2[1] + qe2[2] * qe2[2] + qe2[3] * qe2[3]);
    SR q2[4] = {qe2[0] / nq, qe2[1] / nq, qe2[2] / nq, qe2[3] / nq};
    SR Rn[9];
    quat_to_mat_s(q2, Rn);
    SR Dm[3], Di[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Dm[i] = inv_in[i] > 0.f ? m / SR(inv_in[i]) : SR(0);
        Di[i] = SR(inv_in[i]) / m;
    }
    // I0 = R Dm R^T, In = Rn Di Rn^T
    SR I0[9], In[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            I0[3 * i + j] = R[3 * i] * Dm[0] * R[3 * j] + R[3 * i + 1] * Dm[1] * R[3 * j + 1] + R[3 * i + 2] * Dm[2] * R[3 * j + 2];
            In[3 * i + j] = Rn[3 * i] * Di[0] * Rn[3 * j] + Rn[3 * i + 1] * Di[1] * Rn[3 * j + 1] +
                            Rn[3 * i + 2] * Di[2] * Rn[3 * j + 2];
        }
    SR h[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) h[i] = I0[3 * i] * wp[0] + I0[3 * i + 1] * wp[1] + I0[3 * i + 2] * wp[2];
    SR xbar[3] = {bar.x[0], bar.x[1], bar.x[2]};
    SR vpbar[3] = {bar.v[0] + dt * bar.x[0], bar.v[1] + dt * bar.x[1], bar.v[2] + dt * bar.x[2]};
    SR hbar[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) hbar[i] = In[3 * i] * bar.w[0] + In[3 * i + 1] * bar.w[1] + In[3 * i + 2] * bar.w[2];
    SR Inb[9], I0b[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Inb[3 * i + j] = bar.w[i] * h[j];
            I0b[3 * i + j] = hbar[i] * wp[j];
        }
    SR wpbar[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) wpbar[i] = I0[3 * i] * hbar[0] + I0[3 * i + 1] * hbar[1] + I0[3 * i + 2] * hbar[2];
    SR Rnbar[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    rdr_adj(Rn, Di, Inb, Rnbar, (SR *)nullptr);
    rdr_adj(R, Dm, I0b, Rbar, (SR *)nullptr);
    SR q2bar[4] = {bar.q[0], bar.q[1], bar.q[2], bar.q[3]};
    quat_to_mat_adj(q2, Rnbar, q2bar);
    SR dq2 = q2[0] * q2bar[0] + q2[1] * q2bar[1] + q2[2] * q2bar[2] + q2[3] * q2bar[3];
    SR qe2bar[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) qe2bar[i] = (q2bar[i] - q2[i] * dq2) / nq;
    SR eqbar[4] = {0, 0, 0, 0};
    quat_mul_adj(eq, q, qe2bar, eqbar, qbar);
    SR thbar[3];
    {
        SR tdot = th[0] * eqbar[1] + th[1] * eqbar[2] + th[2] * eqbar[3];
        if (small) {
            SR a2 = an * an;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                thbar[i] = -th[i] / SR(4) * eqbar[0] + (SR(0.5) - a2 / SR(48)) * eqbar[1 + i] - th[i] * tdot / SR(24);
        } else {
            SR dsda = (SR(0.5) * cc - sc) / an;   // d(sin(a/2)/a)/da
#pragma unroll
            for (int i = 0; i < 3; ++i)
                thbar[i] = -SR(0.5) * sc * th[i] * eqbar[0] + sc * eqbar[1 + i] + th[i] * (dsda / an) * tdot;
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) wpbar[i] += dt * thbar[i];

    // ---- (B) observation / cost adjoint ------------------------------
    SR imp[3] = {F[0] * r[0] + F[3] * r[1] + F[6] * r[2], F[1] * r[0] + F[4] * r[1] + F[7] * r[2],
                 F[2] * r[0] + F[5] * r[1] + F[8] * r[2]};
    if (!act) { imp[0] = imp[1] = imp[2] = SR(0); }
    *reinterpret_cast<float4 *>(stage + 4 * lane) =
        make_float4(__int_as_float(act ? st.link : -1), (float)imp[0], (float)imp[1], (float)imp[2]);
    wave_sync();
    {
        SR f0 = 0, f1 = 0, f2 = 0;
        for (int c = 0; c < P.C_max; ++c) {
            const float4 rec = *reinterpret_cast<const float4 *>(stage + 4 * c);
            if (__float_as_int(rec.x) == lane) { f0 += rec.y; f1 += rec.z; f2 += rec.w; }
        }
        SR idt = SR(1) / dt;
        f0 = -f0 * idt; f1 = -f1 * idt; f2 = -f2 * idt;
        SR mag = sqrt(f0 * f0 + f1 * f1 + f2 * f2);
        SR cb[3] = {0, 0, 0};
        if (lane < L && mag > SR(0)) {
            const size_t LG = (size_t)L * P.G;
            SR g0 = gt[0 * LG + (size_t)lane * P.G + g];
            SR gd[3] = {gt[1 * LG + (size_t)lane * P.G + g], gt[2 * LG + (size_t)lane * P.G + g],
                        gt[3 * LG + (size_t)lane * P.G + g]};
            SR magb = SR(2) * SR(P.w_mag) * (mag - g0);
            SR ch[3] = {f0 / mag, f1 / mag, f2 / mag};
#pragma unroll
            for (int i = 0; i < 3; ++i) cb[i] = magb * ch[i];
            if (mag > SR(P.tau_contact)) {
                SR db[3] = {SR(2) * SR(P.w_dir) * (ch[0] - gd[0]), SR(2) * SR(P.w_dir) * (ch[1] - gd[1]),
                            SR(2) * SR(P.w_dir) * (ch[2] - gd[2])};
                SR cd = ch[0] * db[0] + ch[1] * db[1] + ch[2] * db[2];
#pragma unroll
                for (int i = 0; i < 3; ++i) cb[i] += (db[i] - ch[i] * cd) / mag;
            }
        }
        stage2[3 * lane + 0] = (float)cb[0];
        stage2[3 * lane + 1] = (float)cb[1];
        stage2[3 * lane + 2] = (float)cb[2];
    }
    wave_sync();
    SR impbar[3] = {0, 0, 0};
    if (act && st.link >= 0) {
        SR idt = SR(1) / dt;
        impbar[0] = -SR(stage2[3 * st.link + 0]) * idt;
        impbar[1] = -SR(stage2[3 * st.link + 1]) * idt;
        impbar[2] = -SR(stage2[3 * st.link + 2]) * idt;
    }
    // imp = F^T r  ->  rbar = F impbar, Fbar_ij += r_i impbar_j
    SR rbar[3], Fbar[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        rbar[i] = F[3 * i] * impbar[0] + F[3 * i + 1] * impbar[1] + F[3 * i + 2] * impbar[2];
#pragma unroll
        for (int j = 0; j < 3; ++j) Fbar[3 * i + j] = r[i] * impbar[j];
    }

    // ---- (C) velocity adjoint into r: rbar += J M^-1 nubar_down -------
    {
        SR a[3] = {vpbar[0] * im, vpbar[1] * im, vpbar[2] * im};
        SR b[3] = {Iinv[0] * wpbar[0] + Iinv[1] * wpbar[1] + Iinv[2] * wpbar[2],
                   Iinv[3] * wpbar[0] + Iinv[4] * wpbar[1] + Iinv[5] * wpbar[2],
                   Iinv[6] * wpbar[0] + Iinv[7] * wpbar[1] + Iinv[8] * wpbar[2]};
        SR pv[3];
        cross3(b, rho, pv);
        pv[0] += a[0]; pv[1] += a[1]; pv[2] += a[2];
        rbar[0] += dot3(F, pv); rbar[1] += dot3(F + 3, pv); rbar[2] += dot3(F + 6, pv);
    }
    if (!act) { rbar[0] = rbar[1] = rbar[2] = SR(0); }

    // ---- (D) transposed Schur solve: A^T lambda = rbar -----------------
    SR u[3];
    rel_velocity(st, nu, r, eps, u);
    FBOut<SR> fo;
    fb_value(mu, kap, del, r, u, fo);
    SR JX[9], JY[9], DX[9], DY[9];
    fb_jacobian(mu, kap, u, fo, JX, JY, DX, DY);
    SR Pm[9], Pi[9], Q[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Pm[i] = JX[i] + eps * JY[i];
    inv3(Pm, Pi);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Q[3 * i + j] = Pi[3 * i] * JY[j] + Pi[3 * i + 1] * JY[3 + j] + Pi[3 * i + 2] * JY[6 + j];
    SR QwT[9];   // (F^T Q F)^T = F^T Q^T F
    {
        SR QF[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                QF[3 * i + j] = Q[3 * i] * F[j] + Q[3 * i + 1] * F[3 + j] + Q[3 * i + 2] * F[6 + j];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                QwT[3 * j + i] = F[i] * QF[j] + F[3 + i] * QF[3 + j] + F[6 + i] * QF[6 + j];
    }
    SR gtl[3];   // Q^T rbar
#pragma unroll
    for (int i = 0; i < 3; ++i) gtl[i] = Q[i] * rbar[0] + Q[3 + i] * rbar[1] + Q[6 + i] * rbar[2];
    SR gw[3] = {F[0] * gtl[0] + F[3] * gtl[1] + F[6] * gtl[2], F[1] * gtl[0] + F[4] * gtl[1] + F[7] * gtl[2],
                F[2] * gtl[0] + F[5] * gtl[1] + F[8] * gtl[2]};
    SR zeta[6];
    {
        SR acc[42];
        schur_contribution(QwT, gw, rho, acc);
        if (!act) {
#pragma unroll
            for (int i = 0; i < 42; ++i) acc[i] = SR(0);
        }
        if (st.C > 0) lds_sum<SR, 42>(acc, st.C, red);
        SR z[6];
        BodyMass<SR> Mb;
        body_mass<SR>(st.m, st.Iinv, inv_in, Mb);
        schur_solve(acc, Mb, z);
#pragma unroll
        for (int i = 0; i < 6; ++i) zeta[i] = st.C > 0 ? -z[i] : SR(0);
    }
    SR lam[3];
    {
        SR pz[3];
        SR zw[3] = {zeta[3], zeta[4], zeta[5]};
        cross3(zw, rho, pz);
        pz[0] += zeta[0]; pz[1] += zeta[1]; pz[2] += zeta[2];
        SR t3[3] = {rbar[0] - dot3(F, pz), rbar[1] - dot3(F + 3, pz), rbar[2] - dot3(F + 6, pz)};
#pragma unroll
        for (int i = 0; i < 3; ++i) lam[i] = Pi[i] * t3[0] + Pi[3 + i] * t3[1] + Pi[6 + i] * t3[2];
    }
    if (!act) { lam[0] = lam[1] = lam[2] = SR(0); }

    // ---- (E) parameter adjoints at fixed r -----------------------------
    SR ub[3];   // -JY^T lambda
#pragma unroll
    for (int i = 0; i < 3; ++i) ub[i] = -(JY[i] * lam[0] + JY[3 + i] * lam[1] + JY[6 + i] * lam[2]);
    SR mub_c = 0;
    {
        // dPhi/dmu = Dx (kappa r_n, 0, 0) + Dy (st, u_t1, u_t2)
        SR xm = kap * r[0];
        SR ph[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) ph[i] = DX[3 * i] * xm + DY[3 * i] * fo.st + DY[3 * i + 1] * u[1] + DY[3 * i + 2] * u[2];
        mub_c = -(lam[0] * ph[0] + lam[1] * ph[1] + lam[2] * ph[2]);
    }
    if (!act) { ub[0] = ub[1] = ub[2] = SR(0); mub_c = SR(0); }
    // sums over contacts: J^T ub (6), J^T r (6)
    SR nuall[6], sumf[3], sumt[3];
    {
        SR fu[3] = {F[0] * ub[0] + F[3] * ub[1] + F[6] * ub[2], F[1] * ub[0] + F[4] * ub[1] + F[7] * ub[2],
                    F[2] * ub[0] + F[5] * ub[1] + F[8] * ub[2]};
        SR tu[3], ti[3];
        cross3(rho, fu, tu);
        cross3(rho, imp, ti);
        SR a12[12] = {fu[0], fu[1], fu[2], tu[0], tu[1], tu[2], imp[0], imp[1], imp[2], ti[0], ti[1], ti[2]};
        if (!act) {
#pragma unroll
            for (int i = 0; i < 12; ++i) a12[i] = SR(0);
        }
        wave_sum<SR, 12>(a12, span);
        nuall[0] = vpbar[0] + a12[0]; nuall[1] = vpbar[1] + a12[1]; nuall[2] = vpbar[2] + a12[2];
        nuall[3] = wpbar[0] + a12[3]; nuall[4] = wpbar[1] + a12[4]; nuall[5] = wpbar[2] + a12[5];
        sumf[0] = a12[6]; sumf[1] = a12[7]; sumf[2] = a12[8];
        sumt[0] = a12[9]; sumt[1] = a12[10]; sumt[2] = a12[11];
    }
    // M^-1 nuall
    SR ma[3] = {nuall[0] * im, nuall[1] * im, nuall[2] * im};
    SR mb[3] = {Iinv[0] * nuall[3] + Iinv[1] * nuall[4] + Iinv[2] * nuall[5],
                Iinv[3] * nuall[3] + Iinv[4] * nuall[4] + Iinv[5] * nuall[5],
                Iinv[6] * nuall[3] + Iinv[7] * nuall[4] + Iinv[8] * nuall[5]};
    // (1/m)bar and Iinv bar from nu+ = nu* + M^-1 J^T r
    mbar += -(nuall[0] * sumf[0] + nuall[1] * sumf[1] + nuall[2] * sumf[2]) * im * im;
    SR Iinvb[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Iinvb[3 * i + j] = nuall[3 + i] * sumt[j];

    // ---- (F) per-contact geometry adjoint ------------------------------
    SR xbar_c[3] = {0, 0, 0};
    SR Rbar_c[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (act) {
        // J row i = [F_i, rho x F_i];  Jbar row i = ub_i nu^T + r_i (ma, mb)^T
        SR rhob[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            SR jl[3] = {ub[i] * nu[0] + r[i] * ma[0], ub[i] * nu[1] + r[i] * ma[1], ub[i] * nu[2] + r[i] * ma[2]};
            SR ja[3] = {ub[i] * nu[3] + r[i] * mb[0], ub[i] * nu[4] + r[i] * mb[1], ub[i] * nu[5] + r[i] * mb[2]};
            SR t1c[3], t2c[3];
            cross3(ja, rho, t1c);
            cross3(F + 3 * i, ja, t2c);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                Fbar[3 * i + j] += jl[j] + t1c[j];
                rhob[j] += t2c[j];
            }
        }
        // ucst = -F vl + (b_n, 0, 0), ucst_bar = ub
        SR vl[3] = {st.vl[0], st.vl[1], st.vl[2]};
        SR vlb[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            vlb[j] = -(ub[0] * F[j] + ub[1] * F[3 + j] + ub[2] * F[6 + j]);
#pragma unroll
            for (int i = 0; i < 3; ++i) Fbar[3 * i + j] += -ub[i] * vl[j];
        }
        SR db = ub[0] * (st.d >= 0.f ? SR(1) / dt : SR(P.erp) / dt);
        // frame: rows n, t1, t2;  t2 = n x t1;  t1 = normalize(n x e)
        SR n[3] = {F[0], F[1], F[2]}, t1[3] = {F[3], F[4], F[5]};
        SR nb[3] = {Fbar[0], Fbar[1], Fbar[2]}, t1b[3] = {Fbar[3], Fbar[4], Fbar[5]}, t2b[3] = {Fbar[6], Fbar[7], Fbar[8]};
        {
            SR a3[3], b3[3];
            cross3(t1, t2b, a3);
            cross3(t2b, n, b3);
#pragma unroll
            for (int j = 0; j < 3; ++j) { nb[j] += a3[j]; t1b[j] += b3[j]; }
            SR ev[3] = {st.e_axis == 0 ? SR(1) : SR(0), st.e_axis == 1 ? SR(1) : SR(0), st.e_axis == 2 ? SR(1) : SR(0)};
            SR uu[3];
            cross3(n, ev, uu);
            SR nuu = sqrt(uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2]);
            SR tt = t1[0] * t1b[0] + t1[1] * t1b[1] + t1[2] * t1b[2];
            SR ubb[3] = {(t1b[0] - t1[0] * tt) / nuu, (t1b[1] - t1[1] * tt) / nuu, (t1b[2] - t1[2] * tt) / nuu};
            SR c3[3];
            cross3(ev, ubb, c3);
#pragma unroll
            for (int j = 0; j < 3; ++j) nb[j] += c3[j];
        }
        // rho = p - x
        SR pb[3] = {rhob[0], rhob[1], rhob[2]};
        xbar_c[0] -= rhob[0]; xbar_c[1] -= rhob[1]; xbar_c[2] -= rhob[2];
        const int k = st.k, l = st.l;
        const float4 s4 = *reinterpret_cast<const float4 *>(sph + 4 * k);
        const SR rhok = s4.w;
        SR cb[3] = {0, 0, 0};
        if (l < L) {
            const float *sg = seg + l * SEG_STRIDE;
            // p = c - rho_k n
            cb[0] += pb[0]; cb[1] += pb[1]; cb[2] += pb[2];
            nb[0] += -rhok * pb[0]; nb[1] += -rhok * pb[1]; nb[2] += -rhok * pb[2];
            SR dist = st.dist;
            SR nn = n[0] * nb[0] + n[1] * nb[1] + n[2] * nb[2];
            SR delb[3];
            if (dist >= SR(1e-7)) {
#pragma unroll
                for (int j = 0; j < 3; ++j) delb[j] = (nb[j] - n[j] * nn) / dist + db * n[j];
            } else {
#pragma unroll
                for (int j = 0; j < 3; ++j) delb[j] = db * n[j];
            }
            SR ab[3] = {sg[4], sg[5], sg[6]};
            SR va[3] = {sg[8], sg[9], sg[10]}, vb[3] = {sg[12], sg[13], sg[14]};
            SR tb = vlb[0] * (vb[0] - va[0]) + vlb[1] * (vb[1] - va[1]) + vlb[2] * (vb[2] - va[2]);
            tb += -(ab[0] * delb[0] + ab[1] * delb[1] + ab[2] * delb[2]);
            cb[0] += delb[0]; cb[1] += delb[1]; cb[2] += delb[2];
            if (st.interior) {
                SR il2 = sg[7];
                cb[0] += tb * ab[0] * il2; cb[1] += tb * ab[1] * il2; cb[2] += tb * ab[2] * il2;
            }
        } else {
            // table: d = c_z - rho_k, p = c - rho_k e_z, n and v_link constant
            cb[0] += pb[0]; cb[1] += pb[1]; cb[2] += pb[2] + db;
        }
        // c = x + R s_k
        xbar_c[0] += cb[0]; xbar_c[1] += cb[1]; xbar_c[2] += cb[2];
        SR sk[3] = {s4.x, s4.y, s4.z};
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Rbar_c[3 * i + j] = cb[i] * sk[j];
    }
    {
        SR a13[13] = {xbar_c[0], xbar_c[1], xbar_c[2], Rbar_c[0], Rbar_c[1], Rbar_c[2], Rbar_c[3], Rbar_c[4],
                      Rbar_c[5], Rbar_c[6], Rbar_c[7], Rbar_c[8], mub_c};
        wave_sum<SR, 13>(a13, span);
        xbar[0] += a13[0]; xbar[1] += a13[1]; xbar[2] += a13[2];
#pragma unroll
        for (int i = 0; i < 9; ++i) Rbar[i] += a13[3 + i];
        mubar += a13[12];
    }

    // ---- (G) uniform tail ------------------------------------------------
    // vs = v + dt (g + f/m);  ws = w
    SR vsb[3] = {nuall[0], nuall[1], nuall[2]};
    mbar += -dt * (SR(B.f[0]) * vsb[0] + SR(B.f[1]) * vsb[1] + SR(B.f[2]) * vsb[2]) * im * im;
    if (fbar) {
        fbar[0] += dt * im * vsb[0];
        fbar[1] += dt * im * vsb[1];
        fbar[2] += dt * im * vsb[2];
    }
    // Iinv = R diag(ii) R^T, ii = inv/m
    SR ii[3] = {st.ii[0], st.ii[1], st.ii[2]};
    SR iib[3] = {0, 0, 0};
    rdr_adj(R, ii, Iinvb, Rbar, iib);
    mbar += -(iib[0] * SR(inv_in[0]) + iib[1] * SR(inv_in[1]) + iib[2] * SR(inv_in[2])) * im * im;
    quat_to_mat_adj(q, Rbar, qbar);
    // q_hat = q / |q|
    SR qn = sqrt(SR(B.q[0]) * B.q[0] + SR(B.q[1]) * B.q[1] + SR(B.q[2]) * B.q[2] + SR(B.q[3]) * B.q[3]);
    SR dqq = q[0] * qbar[0] + q[1] * qbar[1] + q[2] * qbar[2] + q[3] * qbar[3];
#pragma unroll
    for (int i = 0; i < 4; ++i) bar.q[i] = (qbar[i] - q[i] * dqq) / qn;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        bar.x[i] = xbar[i];
        bar.v[i] = vsb[i];
        bar.w[i] = nuall[3 + i];
    }
}

}  // namespace pt
