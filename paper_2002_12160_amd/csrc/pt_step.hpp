// pt_step.hpp -- one simulation step executed by one wavefront, split into
// phases so that the adjoint can re-run the forward step with the same code:
//   step_setup   pose, free velocity, narrow phase, cap, contact setup, warm start
//   step_solve   smoothed Fischer-Burmeister Newton on the 6x6 Schur system
//   step_finish  integration, warm cache and contact outputs
// Geometry runs in float32; the contact solve runs in SR (float or double).
#pragma once

#include "pt_device.hpp"

namespace pt {

template <typename SR>
struct StepState {
    // uniform
    float q[4];        // normalised pre-step orientation
    float R[9];
    float ii[3];       // principal inverse inertia / m
    float Iinv[9];     // world inverse inertia
    float vs[3], ws[3];// free velocity
    float m, im;
    int C, span, ncand;
    // per lane (contact slot)
    bool act;
    int key, link, k, l;
    float c[3];        // sphere centre
    float d, n[3], p[3], vl[3], tpar, dist;
    bool interior;     // closest point strictly inside the segment
    int e_axis;        // axis used for the tangent frame
    SR F[9];           // rows n, t1, t2
    SR rho[3];         // p - x
    SR ucst[3];        // -F v_link + (b_n, 0, 0)
    SR r[3];           // impulse
    SR nu[6];          // body velocity after the solve (fresh sum)
    SR psi_end;        // merit |Phi|^2 / 2 at the returned impulses (0 without
                       // contacts, -1 if no iteration ran)
};

// M^-1 J^T x summed over contacts, for an impulse x held by this lane
template <typename SR>
__device__ __forceinline__ void body_dv(const StepState<SR> &st, const SR *x, SR *dn)
{
    const SR *F = st.F;
    SR f[3] = {F[0] * x[0] + F[3] * x[1] + F[6] * x[2], F[1] * x[0] + F[4] * x[1] + F[7] * x[2],
               F[2] * x[0] + F[5] * x[1] + F[8] * x[2]};
    SR tq[3];
    cross3(st.rho, f, tq);
    SR a6[6] = {f[0], f[1], f[2], tq[0], tq[1], tq[2]};
    wave_sum<SR, 6>(a6, st.span);
    const SR imS = SR(1) / SR(st.m);
    dn[0] = a6[0] * imS; dn[1] = a6[1] * imS; dn[2] = a6[2] * imS;
    dn[3] = SR(st.Iinv[0]) * a6[3] + SR(st.Iinv[1]) * a6[4] + SR(st.Iinv[2]) * a6[5];
    dn[4] = SR(st.Iinv[3]) * a6[3] + SR(st.Iinv[4]) * a6[4] + SR(st.Iinv[5]) * a6[5];
    dn[5] = SR(st.Iinv[6]) * a6[3] + SR(st.Iinv[7]) * a6[4] + SR(st.Iinv[8]) * a6[5];
}

// relative velocity u = F (v + w x rho) + ucst + eps r for body velocity nu
template <typename SR>
__device__ __forceinline__ void rel_velocity(const StepState<SR> &st, const SR *nu, const SR *r, SR eps, SR *u)
{
    SR pv[3];
    SR nw3[3] = {nu[3], nu[4], nu[5]};
    cross3(nw3, st.rho, pv);
    pv[0] += nu[0]; pv[1] += nu[1]; pv[2] += nu[2];
    const SR *F = st.F;
    u[0] = dot3(F, pv) + st.ucst[0] + eps * r[0];
    u[1] = dot3(F + 3, pv) + st.ucst[1] + eps * r[1];
    u[2] = dot3(F + 6, pv) + st.ucst[2] + eps * r[2];
}

// phase 1: pose, rotation, inverse inertia, free velocity (wave-uniform)
template <typename SR>
__device__ __forceinline__ void step_pose(const Consts &P, const float *inv_in, const Body &B, StepState<SR> &st)
{
    const float dt = P.dt;
    float qn = rsqrtf(B.q[0] * B.q[0] + B.q[1] * B.q[1] + B.q[2] * B.q[2] + B.q[3] * B.q[3]);
    float *q = st.q;
    q[0] = B.q[0] * qn; q[1] = B.q[1] * qn; q[2] = B.q[2] * qn; q[3] = B.q[3] * qn;
    float *R = st.R;
    quat_to_mat(q, R);
    st.m = B.m;
    st.im = 1.f / st.m;
    const float im = st.im;
    st.ii[0] = inv_in[0] * im; st.ii[1] = inv_in[1] * im; st.ii[2] = inv_in[2] * im;
    const float *ii = st.ii;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            st.Iinv[3 * i + j] = R[3 * i] * ii[0] * R[3 * j] + R[3 * i + 1] * ii[1] * R[3 * j + 1] +
                                 R[3 * i + 2] * ii[2] * R[3 * j + 2];
    st.vs[0] = B.v[0] + dt * (P.gx + B.f[0] * im);
    st.vs[1] = B.v[1] + dt * (P.gy + B.f[1] * im);
    st.vs[2] = B.v[2] + dt * (P.gz + B.f[2] * im);
    st.ws[0] = B.w[0]; st.ws[1] = B.w[1]; st.ws[2] = B.w[2];
    // wave-uniform values to scalar registers (they stay live through the
    // whole step)
#pragma unroll
    for (int i = 0; i < 4; ++i) st.q[i] = uniform(st.q[i]);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        st.R[i] = uniform(st.R[i]);
        st.Iinv[i] = uniform(st.Iinv[i]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        st.ii[i] = uniform(st.ii[i]);
        st.vs[i] = uniform(st.vs[i]);
        st.ws[i] = uniform(st.ws[i]);
    }
    st.m = uniform(st.m);
    st.im = uniform(st.im);
}

// phase 4: geometry of the contact with key `key` held by this lane (key < 0:
// an empty slot), impulse reset to 0
template <typename SR, bool SDF = false>
__device__ __forceinline__ void contact_setup(const Consts &P, const float *__restrict__ seg,
                                              const float *__restrict__ sph, const Body &B, int key,
                                              StepState<SR> &st, const SdfRef &sdf = SdfRef())
{
    const int L = P.L;
    const float dt = P.dt;
    const float *R = st.R;
    st.act = key >= 0;
    st.key = key;
    SR *F = st.F;
    F[0] = 0; F[1] = 0; F[2] = 1; F[3] = 0; F[4] = 1; F[5] = 0; F[6] = 1; F[7] = 0; F[8] = 0;
    st.rho[0] = st.rho[1] = st.rho[2] = SR(0);
    st.ucst[0] = st.ucst[1] = st.ucst[2] = SR(0);
    st.r[0] = st.r[1] = st.r[2] = SR(0);
    st.link = -1;
    st.k = 0;
    st.l = L;
    st.interior = false;
    st.e_axis = 0;
    st.tpar = 0.f;
    st.dist = 0.f;
    st.d = 0.f;
    if (st.act) {
        int k = st.key / (L + 1);
        int l = st.key - k * (L + 1);
        st.k = k;
        st.l = l;
        float d, *n = st.n, *p = st.p, *vl = st.vl;
        if (SDF && l < L) {
            // sample k of link l against the object's distance field
            float t;
            sdf_contact(sdf, seg, l, k, B.x, R, d, n, p, vl, t);
            st.tpar = t;
            st.c[0] = st.c[1] = st.c[2] = 0.f;
        } else {
            const float4 t = *reinterpret_cast<const float4 *>(sph + 4 * k);
            const float s4[4] = {t.x, t.y, t.z, t.w};
            float *c = st.c;
            c[0] = B.x[0] + R[0] * s4[0] + R[1] * s4[1] + R[2] * s4[2];
            c[1] = B.x[1] + R[3] * s4[0] + R[4] * s4[1] + R[5] * s4[2];
            c[2] = B.x[2] + R[6] * s4[0] + R[7] * s4[1] + R[8] * s4[2];
            pair_contact(seg, l, L, c, s4[3], d, n, p, vl);
            if (l < L) {
                const float *sg = seg + l * SEG_STRIDE;
                float ca[3] = {c[0] - sg[0], c[1] - sg[1], c[2] - sg[2]};
                float tr = (ca[0] * sg[4] + ca[1] * sg[5] + ca[2] * sg[6]) * sg[7];
                st.interior = tr > 0.f && tr < 1.f;
                st.tpar = fminf(fmaxf(tr, 0.f), 1.f);
                st.dist = d + s4[3] + sg[3];
            }
        }
        st.d = d;
        float t1[3], t2[3];
        tangent_frame(n, t1, t2);
        {
            float an0 = fabsf(n[0]), an1 = fabsf(n[1]), an2 = fabsf(n[2]);
            int e = 0;
            float best = an0;
            if (an1 < best) { e = 1; best = an1; }
            if (an2 < best) { e = 2; }
            st.e_axis = e;
        }
        F[0] = n[0]; F[1] = n[1]; F[2] = n[2];
        F[3] = t1[0]; F[4] = t1[1]; F[5] = t1[2];
        F[6] = t2[0]; F[7] = t2[1]; F[8] = t2[2];
        st.rho[0] = p[0] - B.x[0]; st.rho[1] = p[1] - B.x[1]; st.rho[2] = p[2] - B.x[2];
        float bn = d >= 0.f ? d / dt : P.erp * d / dt;
        st.ucst[0] = -(n[0] * vl[0] + n[1] * vl[1] + n[2] * vl[2]) + bn;
        st.ucst[1] = -(t1[0] * vl[0] + t1[1] * vl[1] + t1[2] * vl[2]);
        st.ucst[2] = -(t2[0] * vl[0] + t2[1] * vl[1] + t2[2] * vl[2]);
        st.link = l < L ? l : -1;
    }
}

// The cap's ranking for ncand <= 64 H candidates (H = 1 .. 4): lane i
// holds candidates i, i + 64, ... as packed (d, key) words (lanes past
// ncand the largest word, never below a candidate's, so the counts run over
// whole groups of four lanes); every word is broadcast once and each lane
// counts the lower ones for each word it holds.  Keys are unique, so the ranks are a
// permutation; the C_max lowest candidates' keys land in sel[rank].
template <int H>
__device__ __forceinline__ void cap_rank(const WaveLds &lds, int ncand, int C_max)
{
    const int lane = lane_id();
    uint64_t w[H];
    int ki[H], rank[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int i = lane + WAVE * h;
        w[h] = ~0ull;
        ki[h] = 0;
        rank[h] = 0;
        if (i < ncand) {
            ki[h] = lds.cand_k[i];
            w[h] = pack_gap_key(lds.cand_d[i], ki[h]);
        }
    }
#pragma unroll
    for (int hb = 0; hb < H; ++hb) {
        const int n = min(WAVE, ncand - WAVE * hb);
        for (int j = 0; j < n; j += 4) {
            const uint64_t a = bcast_lane(w[hb], j), b = bcast_lane(w[hb], j + 1);
            const uint64_t c = bcast_lane(w[hb], j + 2), d = bcast_lane(w[hb], j + 3);
#pragma unroll
            for (int h = 0; h < H; ++h)
                rank[h] += (a < w[h] ? 1 : 0) + (b < w[h] ? 1 : 0) + (c < w[h] ? 1 : 0) + (d < w[h] ? 1 : 0);
        }
    }
#pragma unroll
    for (int h = 0; h < H; ++h)
        if (lane + WAVE * h < ncand && rank[h] < C_max) lds.sel[rank[h]] = ki[h];
}

// The cap for C_max < ncand <= 64 H (H = 2..4), with the same sel[] as
// cap_rank<H>: the C_max-th lowest packed (d, key) word is found bit by bit
// (radix select: a bit of the boundary stays set while fewer than C_max
// words lie below the trial value, counted by ballots), first over the 32
// gap bits and, only when several words share the boundary gap, over their
// key bits; the C_max words up to the boundary move to the front of the
// list and cap_rank<1> ranks them among themselves, which is their rank
// among all candidates (every lower word is kept too).  32 rounds of H
// compares instead of ncand broadcasts against H words per lane.
template <int H>
__device__ __forceinline__ void cap_select(const WaveLds &lds, int ncand, int C_max)
{
    const int lane = lane_id();
    uint32_t hi[H], lo[H];
    float d[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int i = lane + WAVE * h;
        hi[h] = lo[h] = ~0u;   // above every candidate: gaps are finite
        d[h] = 0.f;
        if (i < ncand) {
            d[h] = lds.cand_d[i];
            const uint64_t w = pack_gap_key(d[h], lds.cand_k[i]);
            hi[h] = (uint32_t)(w >> 32);
            lo[h] = (uint32_t)w;
        }
    }
    uint32_t ph = 0;
    for (int b = 31; b >= 0; --b) {
        const uint32_t t = ph | (1u << b);
        int cnt = 0;
#pragma unroll
        for (int h = 0; h < H; ++h) cnt += __popcll(__ballot(hi[h] < t));
        if (cnt < C_max) ph = t;
    }
    // ph: the boundary gap word (fewer than C_max words below it, at least
    // C_max up to it)
    int below = 0, at = 0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        below += __popcll(__ballot(hi[h] < ph));
        at += __popcll(__ballot(hi[h] == ph));
    }
    uint32_t pl = ~0u;
    if (below + at > C_max) {
        const int need = C_max - below;
        pl = 0;
        for (int b = 31; b >= 0; --b) {
            const uint32_t t = pl | (1u << b);
            int cnt = 0;
#pragma unroll
            for (int h = 0; h < H; ++h) cnt += __popcll(__ballot(hi[h] == ph && lo[h] < t));
            if (cnt < need) pl = t;
        }
    }
    wave_sync();   // every lane has read its entries before the list is rewritten
    int base = 0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const bool keep = hi[h] < ph || (hi[h] == ph && lo[h] <= pl);
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int at2 = base + mask_rank(m);
            lds.cand_d[at2] = d[h];
            lds.cand_k[at2] = (int)lo[h];
        }
        base += __popcll(m);
    }
    wave_sync();
    cap_rank<1>(lds, C_max, C_max);
}

// The cap's ranking for any n: every lane ranks its candidates against the
// LDS list, eight per pair of 16-byte reads (entries past n padded with
// (+inf, INT_MAX), never below); the keys of the C_max lowest go to
// sel[rank] and, with dsel, their gaps to dsel[rank].
__device__ __forceinline__ void cap_rank_lds(const WaveLds &lds, int n, int C_max, float *dsel)
{
    const int lane = lane_id();
    if (lane < 8) {
        lds.cand_d[n + lane] = __int_as_float(0x7f800000);
        lds.cand_k[n + lane] = 0x7fffffff;
    }
    wave_sync();
    for (int i = lane; i < n; i += WAVE) {
        const float di = lds.cand_d[i];
        const int ki = lds.cand_k[i];
        int rank = 0;
        for (int j = 0; j < n; j += 8) {
            const float4 d4 = *reinterpret_cast<const float4 *>(lds.cand_d + j);
            const float4 e4 = *reinterpret_cast<const float4 *>(lds.cand_d + j + 4);
            const int4 k4 = *reinterpret_cast<const int4 *>(lds.cand_k + j);
            const int4 m4 = *reinterpret_cast<const int4 *>(lds.cand_k + j + 4);
            rank += (d4.x < di || (d4.x == di && k4.x < ki)) ? 1 : 0;
            rank += (d4.y < di || (d4.y == di && k4.y < ki)) ? 1 : 0;
            rank += (d4.z < di || (d4.z == di && k4.z < ki)) ? 1 : 0;
            rank += (d4.w < di || (d4.w == di && k4.w < ki)) ? 1 : 0;
            rank += (e4.x < di || (e4.x == di && m4.x < ki)) ? 1 : 0;
            rank += (e4.y < di || (e4.y == di && m4.y < ki)) ? 1 : 0;
            rank += (e4.z < di || (e4.z == di && m4.z < ki)) ? 1 : 0;
            rank += (e4.w < di || (e4.w == di && m4.w < ki)) ? 1 : 0;
        }
        if (rank < C_max) {
            lds.sel[rank] = ki;
            if (dsel) dsel[rank] = di;
        }
    }
}

// A full candidate list cut to its C_max lowest (d, key) entries, in that
// order at its head: every candidate dropped has C_max lower ones, so the
// cap over everything seen is unchanged.  Returns the new length; thr gets
// the packed word of the last kept entry (the bar for later candidates).
// The warm cache's LDS (written after the narrow phase) holds the kept gaps.
__device__ __forceinline__ int compact_candidates(const WaveLds &lds, int n, int C_max, uint64_t &thr)
{
    const int lane = lane_id();
    wave_sync();
    cap_rank_lds(lds, n, C_max, lds.wr);
    wave_sync();
    const int m = min(n, C_max);
    if (lane < m) {
        lds.cand_d[lane] = lds.wr[lane];
        lds.cand_k[lane] = lds.sel[lane];
    }
    wave_sync();
    thr = pack_gap_key(lds.cand_d[m - 1], lds.cand_k[m - 1]);
    return m;
}

// Narrow phase: lanes over spheres, candidates appended to LDS in (sphere
// block, link) order by ballot + prefix count, the table (l == L) after the
// links, two links' gaps at a time so that their arithmetic interleaves.
// A link that no sphere can reach is skipped: a sphere's gap to a link is
// at least the gap from the object centre x to the link less |c - x| + rho
// (the distance to a segment is 1-Lipschitz), so a link farther from x than
// the object's largest |c - x| + rho plus the margin (and 10 um for
// rounding) holds no candidate; the reachable links are paired in
// increasing order, so the candidates appended, and their order, are those
// of the full loop.
// Bounded: the list may fill up; a batch that would overflow it first cuts
// the list to its C_max lowest, and from then on only candidates below the
// last kept one are appended (removed counts the others).
template <bool Bounded>
__device__ __forceinline__ void narrow_phase(const Consts &P, const WaveLds &lds, const float (&sgr)[8],
                                             const float *__restrict__ sph, int S, const float *x, const float *R,
                                             int cap, int &ncand, int &removed)
{
    const int lane = lane_id();
    const int L = P.L;
    bool bar = false;
    uint64_t thr = 0;
    // the links any sphere can reach (bit l; wave-uniform)
    float reach = 0.f;
    for (int k = lane; k < S; k += WAVE) {
        const float4 t = *reinterpret_cast<const float4 *>(sph + 4 * k);
        reach = fmaxf(reach, sqrtf(t.x * t.x + t.y * t.y + t.z * t.z) + t.w);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) reach = fmaxf(reach, __shfl_xor(reach, o));
    const uint64_t near = __ballot(lane < L && segment_gap(sgr, x, 0.f) - reach < P.margin + 1e-5f);
    for (int kb = 0; kb < S; kb += WAVE) {
        const int k = kb + lane;
        const bool valid = k < S;
        float s4[4] = {0.f, 0.f, 0.f, 0.f};
        if (valid) {
            const float4 t = *reinterpret_cast<const float4 *>(sph + 4 * k);
            s4[0] = t.x; s4[1] = t.y; s4[2] = t.z; s4[3] = t.w;
        }
        const float c[3] = {x[0] + R[0] * s4[0] + R[1] * s4[1] + R[2] * s4[2],
                            x[1] + R[3] * s4[0] + R[4] * s4[1] + R[5] * s4[2],
                            x[2] + R[6] * s4[0] + R[7] * s4[1] + R[8] * s4[2]};
        auto append = [&](float d, int l) {
            bool cand = valid && (d < P.margin);
            uint64_t mask = __ballot(cand);
            if constexpr (Bounded) {
                if (bar) {
                    removed += __popcll(mask);
                    cand = cand && pack_gap_key(d, k * (L + 1) + l) < thr;
                    mask = __ballot(cand);
                    removed -= __popcll(mask);
                }
                if (ncand + __popcll(mask) > cap) {
                    removed += ncand;
                    ncand = compact_candidates(lds, ncand, P.C_max, thr);
                    removed -= ncand;
                    bar = true;
                    cand = cand && pack_gap_key(d, k * (L + 1) + l) < thr;
                    const uint64_t m2 = __ballot(cand);
                    removed += __popcll(mask) - __popcll(m2);
                    mask = m2;
                }
            }
            if (cand) {
                const int pos = ncand + mask_rank(mask);
                lds.cand_d[pos] = d;
                lds.cand_k[pos] = k * (L + 1) + l;
            }
            ncand += __popcll(mask);
        };
        // the reachable links in increasing order, two at a time
        for (uint64_t m = near; m;) {
            const int l = __builtin_ctzll(m);
            m &= m - 1;
            const int l1 = m ? __builtin_ctzll(m) : l;
            if (m) m &= m - 1;
            float sa[8], sb[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                sa[i] = bcast_lane(sgr[i], l);
                sb[i] = bcast_lane(sgr[i], l1);
            }
            const float da = segment_gap(sa, c, s4[3]), db = segment_gap(sb, c, s4[3]);
            append(da, l);
            if (l1 != l) append(db, l1);
        }
        append(c[2] - s4[3], L);
    }
}

// Narrow phase against the object's distance field: lanes over the links'
// (link, sample) pairs, then over the spheres for the table, candidates
// appended to LDS by ballot + prefix count (the list holds them all: the
// batch is created only when L x samples + S_max fit).
__device__ __forceinline__ void narrow_phase_sdf(const Consts &P, const WaveLds &lds, const SdfRef &sdf,
                                                 const float *__restrict__ seg, const float *__restrict__ sph, int S,
                                                 const float *x, const float *R, int &ncand)
{
    const int lane = lane_id();
    const int L = P.L, M = sdf.M, nq = L * M;
    auto append = [&](bool cand, float d, int key) {
        const uint64_t mask = __ballot(cand);
        if (cand) {
            const int pos = ncand + mask_rank(mask);
            lds.cand_d[pos] = d;
            lds.cand_k[pos] = key;
        }
        ncand += __popcll(mask);
    };
    for (int i0 = 0; i0 < nq; i0 += WAVE) {
        const int i = i0 + lane;
        const bool valid = i < nq;
        float d = 0.f;
        int key = 0;
        if (valid) {
            const int l = i / M, m = i - (i / M) * M;
            const float *s = seg + l * SEG_STRIDE;
            const float t = sdf_sample_t(m, M);
            const float r[3] = {s[0] + t * s[4] - x[0], s[1] + t * s[5] - x[1], s[2] + t * s[6] - x[2]};
            const float po[3] = {R[0] * r[0] + R[3] * r[1] + R[6] * r[2], R[1] * r[0] + R[4] * r[1] + R[7] * r[2],
                                 R[2] * r[0] + R[5] * r[1] + R[8] * r[2]};
            d = sdf_eval(sdf, po, nullptr) - s[3];
            key = m * (L + 1) + l;
        }
        append(valid && d < P.margin, d, key);
    }
    for (int kb = 0; kb < S; kb += WAVE) {
        const int k = kb + lane;
        const bool valid = k < S;
        float d = 0.f;
        if (valid) {
            const float4 t = *reinterpret_cast<const float4 *>(sph + 4 * k);
            const float cz = x[2] + R[6] * t.x + R[7] * t.y + R[8] * t.z;
            d = cz - t.w;
        }
        append(valid && d < P.margin, d, k * (L + 1) + L);
    }
}

// phases 1-4: pose, free velocity, narrow phase, cap, contact setup, warm start
template <typename SR, bool SDF = false>
__device__ __forceinline__ void step_setup(const Consts &P, const float *__restrict__ seg,
                                           const float *__restrict__ sph, int S, const float *inv_in, const Body &B,
                                           int wkey, const float *wr, const WaveLds &lds, StepStats &stats,
                                           StepState<SR> &st, const SdfRef &sdf = SdfRef())
{
    const int lane = lane_id();
    const int L = P.L;
    step_pose<SR>(P, inv_in, B, st);
    const float *R = st.R;

    // 2. narrow phase: lanes over spheres, candidates appended to LDS in
    //    (sphere block, link) order by ballot + prefix count.  The links'
    //    segment records (first 8 floats) sit in registers, one link per
    //    lane, and are broadcast link by link.
    float sgr[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (lane < L) {
        const float4 a = *reinterpret_cast<const float4 *>(seg + lane * SEG_STRIDE);
        const float4 b = *reinterpret_cast<const float4 *>(seg + lane * SEG_STRIDE + 4);
        sgr[0] = a.x; sgr[1] = a.y; sgr[2] = a.z; sgr[3] = a.w;
        sgr[4] = b.x; sgr[5] = b.y; sgr[6] = b.z; sgr[7] = b.w;
    }
    // list capacity (entries; 8 more are the cap's padding); a step that
    // can find more candidates than that runs the bounded form
    const int cap = P.max_cand - 8;
    int ncand = 0, removed = 0;
    if (SDF)
        narrow_phase_sdf(P, lds, sdf, seg, sph, S, B.x, R, ncand);
    else if (S * (L + 1) <= cap)
        narrow_phase<false>(P, lds, sgr, sph, S, B.x, R, cap, ncand, removed);
    else
        narrow_phase<true>(P, lds, sgr, sph, S, B.x, R, cap, ncand, removed);
    wave_sync();
    ncand = __builtin_amdgcn_readfirstlane(ncand);   // wave-uniform: loops on it stay scalar
    const int C = ncand < P.C_max ? ncand : P.C_max;
    st.C = C;
    st.ncand = ncand;
    st.span = lane_span(C);

    // 3. cap: rank of every candidate in (d, key) order; the C_max lowest
    //    land in sel[rank].  Up to one wave of candidates each lane holds
    //    one as a packed (d, key) word and counts the lower words,
    //    broadcast lane by lane; up to four, a radix select finds the
    //    C_max lowest first and only they are ranked; beyond, every lane
    //    ranks its candidates against the LDS list, eight per pair of
    //    16-byte reads (entries past ncand padded with (+inf, INT_MAX),
    //    never below).
    if (ncand <= WAVE) {
        cap_rank<1>(lds, ncand, P.C_max);
    } else if (ncand <= 2 * WAVE) {
        cap_select<2>(lds, ncand, P.C_max);
    } else if (ncand <= 3 * WAVE) {
        cap_select<3>(lds, ncand, P.C_max);
    } else if (ncand <= 4 * WAVE) {
        cap_select<4>(lds, ncand, P.C_max);
    } else {
        cap_rank_lds(lds, ncand, P.C_max, nullptr);
    }
    // previous warm cache to LDS for the key lookup
    lds.wkey[lane] = wkey;
    lds.wr[3 * lane + 0] = wr[0];
    lds.wr[3 * lane + 1] = wr[1];
    lds.wr[3 * lane + 2] = wr[2];
    wave_sync();

    stats.cand += ncand + removed;
    stats.contacts += C;
    stats.dropped += ncand + removed - C;

    // 4. contact setup, one contact per lane, and the warm start from the
    //    previous step's impulse of the same key
    //    (keys of the previous cache are unique; eight compared per round)
    contact_setup<SR, SDF>(P, seg, sph, B, lane < C ? lds.sel[lane] : -1, st, sdf);
    if (st.act) {
        int hit = -1;
        for (int j = 0; j < P.C_max; j += 8) {
            const int4 a = *reinterpret_cast<const int4 *>(lds.wkey + j);
            const int4 b = *reinterpret_cast<const int4 *>(lds.wkey + j + 4);
            hit = a.x == st.key ? j : hit;
            hit = a.y == st.key ? j + 1 : hit;
            hit = a.z == st.key ? j + 2 : hit;
            hit = a.w == st.key ? j + 3 : hit;
            hit = b.x == st.key ? j + 4 : hit;
            hit = b.y == st.key ? j + 5 : hit;
            hit = b.z == st.key ? j + 6 : hit;
            hit = b.w == st.key ? j + 7 : hit;
        }
        if (hit >= 0) {
            st.r[0] = lds.wr[3 * hit]; st.r[1] = lds.wr[3 * hit + 1]; st.r[2] = lds.wr[3 * hit + 2];
        }
    }
    // the solve's sum rows may run on over the cap slots and the lookup's words
    wave_sync();
}

// Newton on the smoothed FB system.  The 3C x 3C Newton matrix
// A = blkdiag(JX) + blkdiag(JY) W, W = J M^-1 J^T + eps I, is reduced to the
// 6x6 system (I + M^-1 sum_c J_c^T P_c^-1 B_c J_c) dnu =
// -M^-1 sum_c J_c^T P_c^-1 Phi_c with P_c = JX_c + eps JY_c, B_c = JY_c; then
// dr_c = -P_c^-1 (Phi_c + B_c J_c dnu).  Leaves st.r and the fresh st.nu.
// red: LDS for the cross-contact sum of the 6x6 system (the wave's candidate
// list, free once the cap has run); the 6x6 solve reads the sums there.
// PairTrials: with at most 32 contacts the line search runs its trials two
// at a time, one per half-wave (the same trials, sums and choice; the worst
// case of four trials costs two).
template <typename SR, bool PairTrials = false>
__device__ __forceinline__ void step_solve(const Consts &P, StepState<SR> &st, float mu_f, const float *inv_in,
                                           SR *red)
{
    const SR eps = P.compliance, kap = P.kappa, del = P.fb_delta, mu = mu_f;
    BodyMass<SR> Mb;
    body_mass<SR>(st.m, st.Iinv, inv_in, Mb);
    const bool act = st.act;
    const int span = st.span;
    SR *r = st.r;
    const SR *F = st.F, *rho = st.rho;
    // current body velocity nu = nu* + M^-1 J^T r
    SR nu[6];
    body_dv(st, r, nu);
    nu[0] += st.vs[0]; nu[1] += st.vs[1]; nu[2] += st.vs[2];
    nu[3] += st.ws[0]; nu[4] += st.ws[1]; nu[5] += st.ws[2];
    st.psi_end = st.C > 0 && P.newton_iters == 0 ? SR(-1) : SR(0);
    if (st.C > 0) {
        // relative velocity and FB value at the current impulses; after the
        // first iteration they are those of the line search's accepted trial
        SR u[3];
        rel_velocity(st, nu, r, eps, u);
        FBOut<SR> fo;
        fb_value(mu, kap, del, r, u, fo);
        for (int it = 0; it < P.newton_iters; ++it) {
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
            schur_contribution(Qw, gw, rho, acc);
            acc[42] = SR(0.5) * (fo.phi[0] * fo.phi[0] + fo.phi[1] * fo.phi[1] + fo.phi[2] * fo.phi[2]);
            if (!act) {
#pragma unroll
                for (int i = 0; i < 43; ++i) acc[i] = SR(0);
            }
            // the sums stay valid in LDS until the next iteration's rows; the
            // 6x6 solve reads them from there as it goes (fewer live
            // registers than loading all 43 at once)
            SR rhs[6];
            lds_colsum<SR, 43>(acc, st.C, red);
            const SR psi = red[42];
            schur_solve(red, Mb, rhs);
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
            // body-velocity change of the step, M^-1 J^T dr: in float64 the
            // 6x6 solution itself; in float32 summed afresh from dr, so that
            // the tracked velocity stays consistent with r (the 6x6 solution
            // equals it only up to the Schur system's conditioning)
            SR dn[6];
            if (sizeof(SR) == 8) {
#pragma unroll
                for (int i = 0; i < 6; ++i) dn[i] = rhs[i];
            } else {
                body_dv(st, dr, dn);
            }
            // du = W dr = F (dn_v + dn_w x rho) + eps dr
            SR du[3];
            {
                SR dq[3];
                SR dnw[3] = {dn[3], dn[4], dn[5]};
                cross3(dnw, rho, dq);
                dq[0] += dn[0]; dq[1] += dn[1]; dq[2] += dn[2];
                du[0] = dot3(F, dq) + eps * dr[0];
                du[1] = dot3(F + 3, dq) + eps * dr[1];
                du[2] = dot3(F + 6, dq) + eps * dr[2];
            }
            // Armijo backtracking over alpha = 1, 1/2, 1/4, 1/8 (1/8 if none
            // passes); the last trial evaluated is the accepted one, and its
            // impulses, relative velocity (u + alpha W dr) and FB value carry
            // into the next iteration
            SR alpha = SR(0.125);
            SR rt[3], ut[3];
            FBOut<SR> ft;
            if (PairTrials && span <= 32) {
                // the same four trials two at a time: the lower half-wave
                // at alpha = 1 (then 1/4), the upper half at 1/2 (then 1/8)
                // on a copy of the lower half's contacts, each half summed
                // by the tree wave_sum uses, accepted in the same order
                SR r2[3], dr2[3], u2[3], du2[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    r2[i] = half_bcast(r[i], false);
                    dr2[i] = half_bcast(dr[i], false);
                    u2[i] = half_bcast(u[i], false);
                    du2[i] = half_bcast(du[i], false);
                }
                const bool act2 = half_bcast((uint32_t)act, false) != 0u;
                const bool up = lane_id() >= 32;
                bool from_upper = true;   // 1/8, the fallback, is the upper half's last trial
                SR psi_acc = SR(0);
                for (int t = 0; t < 2; ++t) {
                    const SR alo = t == 0 ? SR(1) : SR(0.25), ahi = SR(0.5) * alo;
                    const SR a = up ? ahi : alo;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        rt[i] = r2[i] + a * dr2[i];
                        ut[i] = u2[i] + a * du2[i];
                    }
                    fb_value(mu, kap, del, rt, ut, ft);
                    const SR ptr = act2 ? SR(0.5) * (ft.phi[0] * ft.phi[0] + ft.phi[1] * ft.phi[1] +
                                                     ft.phi[2] * ft.phi[2])
                                        : SR(0);
                    SR slo, shi;
                    half_sums(ptr, span, slo, shi);
                    if (slo <= (SR(1) - SR(2) * SR(P.armijo_sigma) * alo) * psi) {
                        alpha = alo;
                        from_upper = false;
                        psi_acc = slo;
                        break;
                    }
                    psi_acc = shi;
                    if (shi <= (SR(1) - SR(2) * SR(P.armijo_sigma) * ahi) * psi) { alpha = ahi; break; }
                }
                st.psi_end = psi_acc;
                if (from_upper) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        rt[i] = half_bcast(rt[i], true);
                        ut[i] = half_bcast(ut[i], true);
                        ft.phi[i] = half_bcast(ft.phi[i], true);
                        ft.x[i] = half_bcast(ft.x[i], true);
                        ft.y[i] = half_bcast(ft.y[i], true);
                    }
                    ft.w0 = half_bcast(ft.w0, true); ft.w1 = half_bcast(ft.w1, true);
                    ft.w2 = half_bcast(ft.w2, true); ft.s = half_bcast(ft.s, true);
                    ft.st = half_bcast(ft.st, true); ft.rw = half_bcast(ft.rw, true);
                    ft.rs = half_bcast(ft.rs, true); ft.rst = half_bcast(ft.rst, true);
                }
            } else {
                SR a = SR(1);
                for (int t = 0; t < 4; ++t, a *= SR(0.5)) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        rt[i] = r[i] + a * dr[i];
                        ut[i] = u[i] + a * du[i];
                    }
                    fb_value(mu, kap, del, rt, ut, ft);
                    SR ptr = act ? SR(0.5) * (ft.phi[0] * ft.phi[0] + ft.phi[1] * ft.phi[1] +
                                              ft.phi[2] * ft.phi[2])
                                 : SR(0);
                    ptr = wave_sum1(ptr, span);
                    st.psi_end = ptr;    // the last trial evaluated is the one taken
                    if (ptr <= (SR(1) - SR(2) * SR(P.armijo_sigma) * a) * psi) { alpha = a; break; }
                }
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                r[i] = rt[i];
                u[i] = ut[i];
            }
            fo = ft;
#pragma unroll
            for (int i = 0; i < 6; ++i) nu[i] += alpha * dn[i];
        }
    }
    // fresh sum of the body velocity for the final impulses
    body_dv(st, r, st.nu);
    st.nu[0] += st.vs[0]; st.nu[1] += st.vs[1]; st.nu[2] += st.vs[2];
    st.nu[3] += st.ws[0]; st.nu[4] += st.ws[1]; st.nu[5] += st.ws[2];
}

// integrate: x += dt v+, q <- normalize(Exp(dt w+) q), angular-momentum-
// preserving w remap; new warm cache slot and contact output of this lane
template <typename SR>
__device__ __forceinline__ void step_finish(const Consts &P, const StepState<SR> &st, const float *inv_in, Body &B,
                                            int &wkey, float *wr, int &out_link, float *out_imp)
{
    const float dt = P.dt;
    const SR *F = st.F, *r = st.r;
    SR impS[3] = {F[0] * r[0] + F[3] * r[1] + F[6] * r[2], F[1] * r[0] + F[4] * r[1] + F[7] * r[2],
                  F[2] * r[0] + F[5] * r[1] + F[8] * r[2]};
    if (!st.act) { impS[0] = impS[1] = impS[2] = SR(0); }
    float vp[3] = {(float)st.nu[0], (float)st.nu[1], (float)st.nu[2]};
    float wp[3] = {(float)st.nu[3], (float)st.nu[4], (float)st.nu[5]};
    const float *q = st.q, *R = st.R;
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
    for (int i = 0; i < 3; ++i) hb[i] = inv_in[i] > 0.f ? wb[i] * st.m / inv_in[i] : 0.f;
    float h[3] = {R[0] * hb[0] + R[1] * hb[1] + R[2] * hb[2], R[3] * hb[0] + R[4] * hb[1] + R[5] * hb[2],
                  R[6] * hb[0] + R[7] * hb[1] + R[8] * hb[2]};
    float Rn[9];
    quat_to_mat(q2, Rn);
    float hn[3] = {Rn[0] * h[0] + Rn[3] * h[1] + Rn[6] * h[2], Rn[1] * h[0] + Rn[4] * h[1] + Rn[7] * h[2],
                   Rn[2] * h[0] + Rn[5] * h[1] + Rn[8] * h[2]};
#pragma unroll
    for (int i = 0; i < 3; ++i) hn[i] *= st.ii[i];
    B.w[0] = Rn[0] * hn[0] + Rn[1] * hn[1] + Rn[2] * hn[2];
    B.w[1] = Rn[3] * hn[0] + Rn[4] * hn[1] + Rn[5] * hn[2];
    B.w[2] = Rn[6] * hn[0] + Rn[7] * hn[1] + Rn[8] * hn[2];
    B.x[0] = xn[0]; B.x[1] = xn[1]; B.x[2] = xn[2];
    B.q[0] = q2[0]; B.q[1] = q2[1]; B.q[2] = q2[2]; B.q[3] = q2[3];
    B.v[0] = vp[0]; B.v[1] = vp[1]; B.v[2] = vp[2];
    B.f[0] = B.f[1] = B.f[2] = 0.f;

    wkey = st.act ? st.key : -1;
    wr[0] = st.act ? (float)r[0] : 0.f;
    wr[1] = st.act ? (float)r[1] : 0.f;
    wr[2] = st.act ? (float)r[2] : 0.f;
    out_link = st.act ? st.link : -1;
    out_imp[0] = (float)impS[0]; out_imp[1] = (float)impS[1]; out_imp[2] = (float)impS[2];
}

// one full step of one simulation
template <typename SR>
__device__ __forceinline__ void env_step(const Consts &P, const float *__restrict__ seg,
                                         const float *__restrict__ sph, int S, const float *inv_in, Body &B,
                                         int &wkey, float *wr, int &out_link, float *out_imp, const WaveLds &lds,
                                         StepStats &stats)
{
    StepState<SR> st;
    step_setup<SR>(P, seg, sph, S, inv_in, B, wkey, wr, lds, stats, st);
    step_solve<SR>(P, st, B.mu, inv_in, reinterpret_cast<SR *>(lds.cand_d));
    step_finish<SR>(P, st, inv_in, B, wkey, wr, out_link, out_imp);
}

}  // namespace pt
