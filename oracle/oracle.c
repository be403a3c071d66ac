/*
 * oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * Written to be checked by eye against the paper and the model reading listed
 * in oracle.h: every step is done in the most direct way (dense matrices, a
 * full sort of candidates, dense LU), with no blocking or fusion.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* small vector / quaternion helpers                                   */
/* ------------------------------------------------------------------ */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    double t0 = a[1] * b[2] - a[2] * b[1];
    double t1 = a[2] * b[0] - a[0] * b[2];
    double t2 = a[0] * b[1] - a[1] * b[0];
    o[0] = t0; o[1] = t1; o[2] = t2;
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

/* Hamilton product, quaternions stored (w, x, y, z). */
static void qmul(const double *a, const double *b, double *o)
{
    double w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    double x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
    double y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
    double z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
    o[0] = w; o[1] = x; o[2] = y; o[3] = z;
}

/* Rotation matrix of a unit quaternion, row-major. */
static void qmat(const double *q, double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}
static void matvec(const double R[9], const double *v, double *o)
{
    double a = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
    double b = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
    double c = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
    o[0] = a; o[1] = b; o[2] = c;
}
static void mattvec(const double R[9], const double *v, double *o)
{
    double a = R[0] * v[0] + R[3] * v[1] + R[6] * v[2];
    double b = R[1] * v[0] + R[4] * v[1] + R[7] * v[2];
    double c = R[2] * v[0] + R[5] * v[1] + R[8] * v[2];
    o[0] = a; o[1] = b; o[2] = c;
}

/* Quaternion of a rotation by angle th about unit axis a. */
static void qaxis(const double *a, double th, double *q)
{
    double s = sin(0.5 * th);
    q[0] = cos(0.5 * th); q[1] = s * a[0]; q[2] = s * a[1]; q[3] = s * a[2];
}

/* Exponential map of a rotation vector th (world frame), with the series
 * form near zero. */
static void qexp(const double *th, double *q)
{
    double a = norm3(th);
    if (a < 1e-4) {
        double a2 = a * a;
        double c = 1.0 - a2 / 8.0;
        double s = 0.5 - a2 / 48.0;
        q[0] = c; q[1] = s * th[0]; q[2] = s * th[1]; q[3] = s * th[2];
    } else {
        double s = sin(0.5 * a) / a;
        q[0] = cos(0.5 * a); q[1] = s * th[0]; q[2] = s * th[1]; q[3] = s * th[2];
    }
}

static void qnormalize(double *q)
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    q[0] /= n; q[1] /= n; q[2] /= n; q[3] /= n;
}

/* Diagnostic rounding of n geometric values to float32 (model flag
 * geom_f32): 1 rounds to the nearest float32; 2 also moves each rounded
 * value one float32 step up or down, the direction taken from a hash of its
 * bits (a second probe of the size of float32 arithmetic error). */
static void geom_round(const or_model *m, double *v, int n)
{
    if (!m->geom_f32) return;
    for (int i = 0; i < n; ++i) {
        float f = (float)v[i];
        if (m->geom_f32 == 2 && f != 0.0f && isfinite(f)) {
            uint32_t bits;
            memcpy(&bits, &f, sizeof bits);
            uint32_t h = bits * 0x9E3779B1u;
            f = nextafterf(f, (h >> 31) ? INFINITY : -INFINITY);
        }
        v[i] = (double)f;
    }
}

/* ------------------------------------------------------------------ */
/* hand forward kinematics                                             */
/* ------------------------------------------------------------------ */

/* Link table row (20 doubles): parent, joint0, joint1, axis0(3), axis1(3),
 * offset translation(3, in the parent's tip frame), offset rotation (w,x,y,z),
 * length, radius, 2 reserved.  A link's frame is the parent's tip frame, moved
 * by the offset, then turned about axis0 by u[joint0] and about axis1 by
 * u[joint1]; the capsule runs from the frame origin along local +x. */
void or_hand_fk(const or_model *m, const double *u, double *seg)
{
    int L = m->L;
    double *tipq = (double *)malloc(sizeof(double) * 4 * (size_t)L);
    double *tipp = (double *)malloc(sizeof(double) * 3 * (size_t)L);
    for (int l = 0; l < L; ++l) {
        const double *h = m->hand + (size_t)l * OR_HAND_STRIDE;
        int parent = (int)h[0], j0 = (int)h[1], j1 = (int)h[2];
        double pq[4] = {1, 0, 0, 0}, pp[3] = {0, 0, 0};
        if (parent >= 0) {
            memcpy(pq, tipq + 4 * parent, sizeof pq);
            memcpy(pp, tipp + 3 * parent, sizeof pp);
        }
        double Rp[9];
        qmat(pq, Rp);
        double off[3];
        matvec(Rp, h + 9, off);
        double o[3] = {pp[0] + off[0], pp[1] + off[1], pp[2] + off[2]};
        double q[4];
        qmul(pq, h + 12, q);
        if (j0 >= 0) {
            double qj[4], t[4];
            qaxis(h + 3, u[j0], qj);
            qmul(q, qj, t);
            memcpy(q, t, sizeof q);
        }
        if (j1 >= 0) {
            double qj[4], t[4];
            qaxis(h + 6, u[j1], qj);
            qmul(q, qj, t);
            memcpy(q, t, sizeof q);
        }
        double R[9];
        qmat(q, R);
        double len = h[16];
        double b[3] = {o[0] + len * R[0], o[1] + len * R[3], o[2] + len * R[6]};
        memcpy(tipq + 4 * l, q, sizeof q);
        memcpy(tipp + 3 * l, b, sizeof b);
        double *s = seg + 6 * l;
        s[0] = o[0]; s[1] = o[1]; s[2] = o[2];
        s[3] = b[0]; s[4] = b[1]; s[5] = b[2];
    }
    free(tipq);
    free(tipp);
}

/* ------------------------------------------------------------------ */
/* narrow phase                                                        */
/* ------------------------------------------------------------------ */

typedef struct {
    double d;
    int32_t key;
} cand_t;

static int cand_cmp(const void *pa, const void *pb)
{
    const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
    if (a->d < b->d) return -1;
    if (a->d > b->d) return 1;
    return (a->key > b->key) - (a->key < b->key);
}

/* Sphere (centre c, radius rho) against link l (capsule seg0[l], radius R)
 * or, for l == L, the table plane z = 0.  Fills d, n, p, vlink. */
static void pair_geometry(const or_model *m, const double *seg0, const double *seg1, int l,
                          const double *c, double rho, double *d, double *n, double *p, double *vl)
{
    int L = m->L;
    if (l == L) {
        *d = c[2] - rho;
        n[0] = 0; n[1] = 0; n[2] = 1;
        p[0] = c[0]; p[1] = c[1]; p[2] = c[2] - rho;
        vl[0] = vl[1] = vl[2] = 0;
        return;
    }
    const double *a = seg0 + 6 * l, *b = seg0 + 6 * l + 3;
    const double *a1 = seg1 + 6 * l, *b1 = seg1 + 6 * l + 3;
    double R = m->hand[(size_t)l * OR_HAND_STRIDE + 17];
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double ca[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double L2 = dot3(ab, ab);
    double s = 0.0;
    if (sqrt(L2) >= 1e-9) {
        s = dot3(ca, ab) / L2;
        if (s < 0) s = 0;
        if (s > 1) s = 1;
    }
    double ps[3] = {a[0] + s * ab[0], a[1] + s * ab[1], a[2] + s * ab[2]};
    double del[3] = {c[0] - ps[0], c[1] - ps[1], c[2] - ps[2]};
    double dist = norm3(del);
    *d = dist - rho - R;
    if (dist < 1e-7) {
        double ex[3] = {1, 0, 0}, ey[3] = {0, 1, 0}, t[3];
        cross3(ab, ex, t);
        if (norm3(t) <= 1e-12) cross3(ab, ey, t);
        if (norm3(t) <= 1e-12) { t[0] = 0; t[1] = 0; t[2] = 1; }
        double nt = norm3(t);
        n[0] = t[0] / nt; n[1] = t[1] / nt; n[2] = t[2] / nt;
    } else {
        n[0] = del[0] / dist; n[1] = del[1] / dist; n[2] = del[2] / dist;
    }
    p[0] = c[0] - rho * n[0]; p[1] = c[1] - rho * n[1]; p[2] = c[2] - rho * n[2];
    double dt = m->dt;
    for (int i = 0; i < 3; ++i) {
        double va = (a1[i] - a[i]) / dt, vb = (b1[i] - b[i]) / dt;
        vl[i] = (1 - s) * va + s * vb;
    }
}

/* Signed distance field of object type `type` at object-frame point p and
 * its gradient g: trilinear interpolation of the grid nodes (exact for
 * affine fields); outside the grid's box, the value at the nearest box
 * point plus the distance to it, with that point's gradient. */
static double sdf_eval(const or_model *m, int type, const double *p, double *g)
{
    const int n = m->sdf_n;
    const double *box = m->sdf_box + 4 * type;
    const double *v = m->sdf + (size_t)type * n * n * n;
    const double h = box[3];
    double out2 = 0.0, f[3];
    int i0[3];
    for (int a = 0; a < 3; ++a) {
        double hi = box[a] + (n - 1) * h;
        double c = p[a] < box[a] ? box[a] : (p[a] > hi ? hi : p[a]);
        out2 += (p[a] - c) * (p[a] - c);
        double u = (c - box[a]) / h;
        int i = (int)floor(u);
        if (i > n - 2) i = n - 2;
        if (i < 0) i = 0;
        i0[a] = i;
        f[a] = u - i;
    }
    double val = 0.0;
    g[0] = g[1] = g[2] = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double node = v[((size_t)(i0[2] + dz) * n + (i0[1] + dy)) * n + (i0[0] + dx)];
                double wx = dx ? f[0] : 1.0 - f[0], wy = dy ? f[1] : 1.0 - f[1], wz = dz ? f[2] : 1.0 - f[2];
                double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
                val += wx * wy * wz * node;
                g[0] += sx * wy * wz * node / h;
                g[1] += wx * sy * wz * node / h;
                g[2] += wx * wy * sz * node / h;
            }
    return val + sqrt(out2);
}

/* Geometry of sample k of link l against the object's distance field (the
 * object at pose x, R): the sample s on the link's axis, its object-frame
 * point, the field's value phi and gradient there; gap phi - radius, normal
 * (link -> object) minus the world unit gradient, contact point s - phi
 * times that gradient (the object's surface point nearest the sample), and
 * the link's velocity at s. */
static void sdf_link_geometry(const or_model *m, const double *seg0, const double *seg1, int type,
                              const double *R, const double *x, int l, int k, double *d, double *n, double *p,
                              double *vl)
{
    const int M = m->link_samples;
    const double t = M > 1 ? (double)k / (double)(M - 1) : 0.5;
    const double *a = seg0 + 6 * l, *b = seg0 + 6 * l + 3;
    const double *a1 = seg1 + 6 * l, *b1 = seg1 + 6 * l + 3;
    double s[3], rel[3], po[3], g[3];
    for (int i = 0; i < 3; ++i) s[i] = a[i] + t * (b[i] - a[i]);
    geom_round(m, s, 3);
    for (int i = 0; i < 3; ++i) rel[i] = s[i] - x[i];
    mattvec(R, rel, po);
    geom_round(m, po, 3);
    double phi = sdf_eval(m, type, po, g);
    geom_round(m, &phi, 1);
    geom_round(m, g, 3);
    double gn = norm3(g), go[3];
    if (gn < 1e-12) {
        go[0] = 0; go[1] = 0; go[2] = 1;
    } else {
        go[0] = g[0] / gn; go[1] = g[1] / gn; go[2] = g[2] / gn;
    }
    double gw[3];
    matvec(R, go, gw);
    *d = phi - m->hand[(size_t)l * OR_HAND_STRIDE + 17];
    for (int i = 0; i < 3; ++i) {
        n[i] = -gw[i];
        p[i] = s[i] - phi * gw[i];
    }
    const double dt = m->dt;
    for (int i = 0; i < 3; ++i) {
        double va = (a1[i] - a[i]) / dt, vb = (b1[i] - b[i]) / dt;
        vl[i] = (1 - t) * va + t * vb;
    }
}

/* the field and its gradient at an object-frame point (for the pins) */
double or_sdf_eval(const or_model *m, int type, const double *p, double *g) { return sdf_eval(m, type, p, g); }

/* Tangent frame: e is the axis where |n_i| is smallest (lowest index on ties),
 * t1 = normalize(n x e), t2 = n x t1. */
static void tangent_frame(const double *n, double *t1, double *t2)
{
    int e = 0;
    if (fabs(n[1]) < fabs(n[e])) e = 1;
    if (fabs(n[2]) < fabs(n[e])) e = 2;
    double ev[3] = {0, 0, 0};
    ev[e] = 1;
    cross3(n, ev, t1);
    double nt = norm3(t1);
    t1[0] /= nt; t1[1] /= nt; t1[2] /= nt;
    cross3(n, t1, t2);
}

/* ------------------------------------------------------------------ */
/* Fischer-Burmeister function for the second-order cone                */
/* ------------------------------------------------------------------ */

/* Jordan algebra on R x R^2: x o y = (x.y, x0 ybar + y0 xbar).
 * For one contact with impulse r and velocity u (both in n,t1,t2):
 *   x = kappa (mu r_n, r_t),  y = (u_n + mu sqrt(|u_t|^2 + delta^2), mu u_t),
 *   w = sqrt(x o x + y o y + 2 delta^2 e),  Phi = x + y - w.
 * If Jx / Jy are non-NULL they receive dPhi/dr and dPhi/du (3x3, row-major). */
static void fb_contact(const or_model *m, double mu, const double *r, const double *u,
                       double *Phi, double *Jx, double *Jy)
{
    double kap = m->kappa, del = m->fb_delta;
    double x[3] = {kap * mu * r[0], kap * r[1], kap * r[2]};
    double st = sqrt(u[1] * u[1] + u[2] * u[2] + del * del);
    double y[3] = {u[0] + mu * st, mu * u[1], mu * u[2]};
    /* z = x o x + y o y + 2 delta^2 e */
    double z0 = dot3(x, x) + dot3(y, y) + 2 * del * del;
    double zb[2] = {2 * (x[0] * x[1] + y[0] * y[1]), 2 * (x[0] * x[2] + y[0] * y[2])};
    double nz = sqrt(zb[0] * zb[0] + zb[1] * zb[1]);
    /* spectral values and square root */
    double l1 = z0 - nz, l2 = z0 + nz;
    double s1 = sqrt(l1), s2 = sqrt(l2);
    double w[3];
    w[0] = 0.5 * (s1 + s2);
    if (nz > 0) {
        double f = 0.5 * (s2 - s1) / nz;
        w[1] = f * zb[0];
        w[2] = f * zb[1];
    } else {
        w[1] = 0;
        w[2] = 0;
    }
    for (int i = 0; i < 3; ++i) Phi[i] = x[i] + y[i] - w[i];
    if (!Jx) return;

    /* L_a = [[a0, abar^T], [abar, a0 I]] (arrow matrix of a). */
    double Lx[9] = {x[0], x[1], x[2], x[1], x[0], 0, x[2], 0, x[0]};
    double Ly[9] = {y[0], y[1], y[2], y[1], y[0], 0, y[2], 0, y[0]};
    double Lw[9] = {w[0], w[1], w[2], w[1], w[0], 0, w[2], 0, w[0]};
    /* inverse of L_w by the textbook 3x3 adjugate formula */
    double inv[9];
    {
        const double *a = Lw;
        double c00 = a[4] * a[8] - a[5] * a[7];
        double c01 = a[5] * a[6] - a[3] * a[8];
        double c02 = a[3] * a[7] - a[4] * a[6];
        double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
        inv[0] = c00 / det;
        inv[1] = (a[2] * a[7] - a[1] * a[8]) / det;
        inv[2] = (a[1] * a[5] - a[2] * a[4]) / det;
        inv[3] = c01 / det;
        inv[4] = (a[0] * a[8] - a[2] * a[6]) / det;
        inv[5] = (a[2] * a[3] - a[0] * a[5]) / det;
        inv[6] = c02 / det;
        inv[7] = (a[1] * a[6] - a[0] * a[7]) / det;
        inv[8] = (a[0] * a[4] - a[1] * a[3]) / det;
    }
    double Dx[9], Dy[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double sx = 0, sy = 0;
            for (int k = 0; k < 3; ++k) {
                sx += inv[3 * i + k] * Lx[3 * k + j];
                sy += inv[3 * i + k] * Ly[3 * k + j];
            }
            Dx[3 * i + j] = (i == j ? 1.0 : 0.0) - sx;
            Dy[3 * i + j] = (i == j ? 1.0 : 0.0) - sy;
        }
    /* dx/dr = kappa diag(mu, 1, 1);  dy/du = [[1, mu that^T], [0, mu I]] */
    double Sx[9] = {kap * mu, 0, 0, 0, kap, 0, 0, 0, kap};
    double Sy[9] = {1, mu * u[1] / st, mu * u[2] / st, 0, mu, 0, 0, 0, mu};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0, b = 0;
            for (int k = 0; k < 3; ++k) {
                a += Dx[3 * i + k] * Sx[3 * k + j];
                b += Dy[3 * i + k] * Sy[3 * k + j];
            }
            Jx[3 * i + j] = a;
            Jy[3 * i + j] = b;
        }
}

/* Dense LU with partial pivoting: solves A z = rhs in place (A n x n,
 * row-major, destroyed).  Returns 0 on success, -1 on an exactly zero pivot. */
static int lu_solve(int n, double *A, double *rhs)
{
    for (int k = 0; k < n; ++k) {
        int piv = k;
        double best = fabs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(A[(size_t)i * n + k]);
            if (v > best) { best = v; piv = i; }
        }
        if (best == 0.0) return -1;
        if (piv != k) {
            for (int j = 0; j < n; ++j) {
                double t = A[(size_t)k * n + j];
                A[(size_t)k * n + j] = A[(size_t)piv * n + j];
                A[(size_t)piv * n + j] = t;
            }
            double t = rhs[k]; rhs[k] = rhs[piv]; rhs[piv] = t;
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[(size_t)i * n + k] / A[(size_t)k * n + k];
            A[(size_t)i * n + k] = f;
            for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
            rhs[i] -= f * rhs[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = rhs[k];
        for (int j = k + 1; j < n; ++j) s -= A[(size_t)k * n + j] * rhs[j];
        rhs[k] = s / A[(size_t)k * n + k];
    }
    return 0;
}

/* u = W r + u_free (n = 3C). */
static void apply_W(int n, const double *W, const double *r, const double *uf, double *u)
{
    for (int i = 0; i < n; ++i) {
        double s = uf[i];
        for (int j = 0; j < n; ++j) s += W[(size_t)i * n + j] * r[j];
        u[i] = s;
    }
}

static double merit(const or_model *m, int C, double mu, const double *W, const double *uf, const double *r,
                    double *ubuf)
{
    int n = 3 * C;
    apply_W(n, W, r, uf, ubuf);
    double psi = 0;
    for (int c = 0; c < C; ++c) {
        double Phi[3];
        fb_contact(m, mu, r + 3 * c, ubuf + 3 * c, Phi, NULL, NULL);
        psi += 0.5 * dot3(Phi, Phi);
    }
    return psi;
}

/* ------------------------------------------------------------------ */
/* one environment step                                                */
/* ------------------------------------------------------------------ */

typedef struct {
    double x[3], q[4], R[9], Iinv[9], vs[3], ws[3];
    double mass, mu;
    int ncand, C;
    double d_last_kept, d_first_dropped;
    double margin_gap, tangent_tie;
    or_contact *cc; /* [C] */
    double *J;      /* [3C][6] */
    double *uf;     /* [3C]    */
    double *W;      /* [3C][3C] */
} sys_t;

static void sys_free(sys_t *y)
{
    free(y->cc); free(y->J); free(y->uf); free(y->W);
}

/* Steps 1-8 of the model: pose, free velocity, candidates, the C_max cap,
 * contact frames, Jacobian, compliant Delassus matrix W and free velocity. */
static void build_system(const or_model *m, const double *seg0, const double *seg1, int type,
                         const double *st, const double *pr, sys_t *y)
{
    const int L = m->L, Cmax = m->C_max;
    const double dt = m->dt;
    const double mass = pr[0], mu = pr[1];
    const double *fp = pr + 2;
    const double *inv = m->inv_inertia + 3 * type;
    const int S = m->n_spheres[type];
    const double *sph = m->spheres + (size_t)type * m->S_max * 4;
    y->mass = mass;
    y->mu = mu;

    /* 1. pose, rotation, inverse mass matrix */
    double *x = y->x, *q = y->q, *R = y->R;
    x[0] = st[0]; x[1] = st[1]; x[2] = st[2];
    q[0] = st[3]; q[1] = st[4]; q[2] = st[5]; q[3] = st[6];
    qnormalize(q);
    qmat(q, R);
    geom_round(m, q, 4);
    geom_round(m, R, 9);
    double v[3] = {st[7], st[8], st[9]}, w[3] = {st[10], st[11], st[12]};
    /* I_w^{-1} = R diag(inv/m) R^T */
    double *Iinv = y->Iinv;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += R[3 * i + k] * (inv[k] / mass) * R[3 * j + k];
            Iinv[3 * i + j] = s;
        }
    geom_round(m, Iinv, 9);

    /* 2. free velocity */
    double *vs = y->vs, *ws = y->ws;
    for (int i = 0; i < 3; ++i) {
        vs[i] = v[i] + dt * (m->gravity[i] + fp[i] / mass);
        ws[i] = w[i];
    }
    geom_round(m, vs, 3);

    /* 3-5. candidates */
    int npair = S * (L + 1);
    cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)(npair > 0 ? npair : 1));
    int ncand = 0;
    y->margin_gap = INFINITY;
    for (int k = 0; k < S; ++k) {
        double c[3];
        matvec(R, sph + 4 * k, c);
        c[0] += x[0]; c[1] += x[1]; c[2] += x[2];
        geom_round(m, c, 3);
        double rho = sph[4 * k + 3];
        for (int l = m->collision_mode == 1 ? L : 0; l <= L; ++l) {
            double d, n[3], p[3], vl[3];
            pair_geometry(m, seg0, seg1, l, c, rho, &d, n, p, vl);
            geom_round(m, &d, 1);
            if (fabs(d - m->margin) < y->margin_gap) y->margin_gap = fabs(d - m->margin);
            if (d < m->margin) {
                cand[ncand].d = d;
                cand[ncand].key = k * (L + 1) + l;
                ++ncand;
            }
        }
    }
    /* links against the object's distance field */
    if (m->collision_mode == 1) {
        cand = (cand_t *)realloc(cand, sizeof(cand_t) * (size_t)(ncand + L * m->link_samples + 1));
        for (int l = 0; l < L; ++l)
            for (int k = 0; k < m->link_samples; ++k) {
                double d, n[3], p[3], vl[3];
                sdf_link_geometry(m, seg0, seg1, type, R, x, l, k, &d, n, p, vl);
                geom_round(m, &d, 1);
                if (fabs(d - m->margin) < y->margin_gap) y->margin_gap = fabs(d - m->margin);
                if (d < m->margin) {
                    cand[ncand].d = d;
                    cand[ncand].key = k * (L + 1) + l;
                    ++ncand;
                }
            }
    }
    /* 6. cap: the C_max smallest (d, key) */
    qsort(cand, (size_t)ncand, sizeof(cand_t), cand_cmp);
    int C = ncand < Cmax ? ncand : Cmax;
    y->ncand = ncand;
    y->C = C;
    y->d_last_kept = C > 0 ? cand[C - 1].d : -INFINITY;
    y->d_first_dropped = ncand > C ? cand[C].d : INFINITY;

    /* 7-8. contact frames, Jacobian, W, u_free */
    or_contact *cc = (or_contact *)calloc((size_t)(C > 0 ? C : 1), sizeof(or_contact));
    int n3 = 3 * C;
    double *J = (double *)calloc((size_t)(n3 > 0 ? n3 : 1) * 6, sizeof(double));
    double *uf = (double *)calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    y->tangent_tie = INFINITY;
    for (int c = 0; c < C; ++c) {
        int key = cand[c].key;
        int k = key / (L + 1), l = key % (L + 1);
        or_contact *o = cc + c;
        o->key = key;
        o->link = l;
        if (m->collision_mode == 1 && l < L) {
            sdf_link_geometry(m, seg0, seg1, type, R, x, l, k, &o->d, o->n, o->p, o->vlink);
        } else {
            double ctr[3];
            matvec(R, sph + 4 * k, ctr);
            ctr[0] += x[0]; ctr[1] += x[1]; ctr[2] += x[2];
            geom_round(m, ctr, 3);
            pair_geometry(m, seg0, seg1, l, ctr, sph[4 * k + 3], &o->d, o->n, o->p, o->vlink);
        }
        geom_round(m, &o->d, 1);
        geom_round(m, o->n, 3);
        geom_round(m, o->p, 3);
        geom_round(m, o->vlink, 3);
        tangent_frame(o->n, o->t1, o->t2);
        geom_round(m, o->t1, 3);
        geom_round(m, o->t2, 3);
        if (l < L) {
            /* distance of the tangent-axis rule from a tie: the two smallest
             * |n_i| (a table contact's normal is exactly e_z on any
             * implementation, so its tie of x and y is exact, not near) */
            double a0 = fabs(o->n[0]), a1 = fabs(o->n[1]), a2 = fabs(o->n[2]);
            double lo = fmin(a0, fmin(a1, a2)), hi = fmax(a0, fmax(a1, a2));
            double mid = a0 + a1 + a2 - lo - hi;
            if (mid - lo < y->tangent_tie) y->tangent_tie = mid - lo;
        }
        double rho[3] = {o->p[0] - x[0], o->p[1] - x[1], o->p[2] - x[2]};
        geom_round(m, rho, 3);
        const double *dirs[3] = {o->n, o->t1, o->t2};
        /* velocity of the object's material point at p under (vs, ws) */
        double wr_[3];
        cross3(ws, rho, wr_);
        double vp[3] = {vs[0] + wr_[0], vs[1] + wr_[1], vs[2] + wr_[2]};
        for (int i = 0; i < 3; ++i) {
            double *row = J + (size_t)(3 * c + i) * 6;
            double rc[3];
            cross3(rho, dirs[i], rc);
            row[0] = dirs[i][0]; row[1] = dirs[i][1]; row[2] = dirs[i][2];
            row[3] = rc[0]; row[4] = rc[1]; row[5] = rc[2];
            uf[3 * c + i] = dot3(dirs[i], vp) - dot3(dirs[i], o->vlink);
        }
        /* speculative gap d/dt for d >= 0, Baumgarte erp*d/dt when penetrating */
        double bn = o->d >= 0 ? o->d / dt : m->erp * o->d / dt;
        uf[3 * c] += bn;
    }
    /* W = J M^{-1} J^T + eps I with M^{-1} = diag(I3/m, Iinv) */
    double *W = (double *)calloc((size_t)(n3 > 0 ? n3 * n3 : 1), sizeof(double));
    for (int i = 0; i < n3; ++i) {
        const double *ri = J + (size_t)i * 6;
        double mi[6];
        mi[0] = ri[0] / mass; mi[1] = ri[1] / mass; mi[2] = ri[2] / mass;
        matvec(Iinv, ri + 3, mi + 3);
        for (int j = 0; j < n3; ++j) {
            const double *rj = J + (size_t)j * 6;
            double s = 0;
            for (int t = 0; t < 6; ++t) s += mi[t] * rj[t];
            W[(size_t)i * n3 + j] = s + (i == j ? m->compliance : 0.0);
        }
    }
    free(cand);
    y->cc = cc;
    y->J = J;
    y->uf = uf;
    y->W = W;
}

int or_env_system(const or_model *m, const double *seg0, const double *seg1, int type,
                  const double *st, const double *pr, or_contact *cont, double *W_out, double *uf_out)
{
    sys_t y;
    build_system(m, seg0, seg1, type, st, pr, &y);
    int n3 = 3 * y.C;
    for (int c = 0; c < y.C; ++c) cont[c] = y.cc[c];
    memcpy(W_out, y.W, sizeof(double) * (size_t)n3 * n3);
    memcpy(uf_out, y.uf, sizeof(double) * (size_t)n3);
    sys_free(&y);
    return y.C;
}

/* Step 10 of the model: warm start from the previous impulses of the same
 * keys, then the smoothed Fischer-Burmeister Newton iteration with the
 * Armijo schedule (fixed N, or until converged).  r [3C] receives the
 * impulses; the diagnostics go to nd. */
typedef struct {
    int iters, nfull, nfall;
    double psi_first, psi, armijo_margin;
} newton_diag;

static void newton_solve(const or_model *m, int C, double mu, double mass, const or_contact *cc, const double *W,
                         const double *uf, const int32_t *wkey, const double *wr, double *r, newton_diag *nd)
{
    const int Cmax = m->C_max;
    const double dt = m->dt;
    int n3 = 3 * C;
    for (int i = 0; i < n3; ++i) r[i] = 0.0;
    for (int c = 0; c < C; ++c)
        for (int j = 0; j < Cmax; ++j)
            if (wkey[j] == cc[c].key) {
                r[3 * c] = wr[3 * j]; r[3 * c + 1] = wr[3 * j + 1]; r[3 * c + 2] = wr[3 * j + 2];
                break;
            }
    double *u = (double *)calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    double *A = (double *)calloc((size_t)(n3 > 0 ? n3 * n3 : 1), sizeof(double));
    double *Phi = (double *)calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    double *dr = (double *)calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    double *rt = (double *)calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    int iters = 0, nfull = 0, nfall = 0;
    double psi_first = 0, psi = 0;
    double armijo_margin = INFINITY;
    if (C > 0) {
        int maxit = m->converged ? m->conv_max_iters : m->newton_iters;
        for (int it = 0; it < maxit; ++it) {
            apply_W(n3, W, r, uf, u);
            psi = 0;
            memset(A, 0, sizeof(double) * (size_t)n3 * n3);
            for (int c = 0; c < C; ++c) {
                double Jx[9], Jy[9];
                fb_contact(m, mu, r + 3 * c, u + 3 * c, Phi + 3 * c, Jx, Jy);
                psi += 0.5 * dot3(Phi + 3 * c, Phi + 3 * c);
                /* rows of block c: A = Jx (block diagonal) + Jy W */
                for (int i = 0; i < 3; ++i) {
                    double *Arow = A + (size_t)(3 * c + i) * n3;
                    for (int j = 0; j < 3; ++j) Arow[3 * c + j] += Jx[3 * i + j];
                    for (int col = 0; col < n3; ++col) {
                        double s = 0;
                        for (int k = 0; k < 3; ++k) s += Jy[3 * i + k] * W[(size_t)(3 * c + k) * n3 + col];
                        Arow[col] += s;
                    }
                }
            }
            if (it == 0) psi_first = psi;
            if (m->converged && psi < m->conv_tol) break;
            for (int i = 0; i < n3; ++i) dr[i] = -Phi[i];
            if (lu_solve(n3, A, dr) != 0) break;
            /* Armijo backtracking on Psi = 1/2 |Phi|^2 */
            double alpha = 0.125;
            double a = 1.0;
            double drmax = 0, rmax = 0;
            for (int i = 0; i < n3; ++i) {
                if (fabs(dr[i]) > drmax) drmax = fabs(dr[i]);
                if (fabs(r[i]) > rmax) rmax = fabs(r[i]);
            }
            double rscale = fmax(mass * norm3(m->gravity) * dt, rmax);
            int passed = 0;
            for (int t = 0; t < 4; ++t, a *= 0.5) {
                for (int i = 0; i < n3; ++i) rt[i] = r[i] + a * dr[i];
                double pt = merit(m, C, mu, W, uf, rt, u);
                double bound = (1.0 - 2.0 * m->armijo_sigma * a) * psi;
                /* diagnostics: how close this trial's decision is to flipping */
                if (t < 3 && psi > 0 && 0.5 * a * drmax > OR_ARMIJO_IMPACT * rscale) {
                    double rel = fabs(pt - bound) / psi;
                    if (rel < armijo_margin) armijo_margin = rel;
                }
                if (pt <= bound) { alpha = a; passed = 1; break; }
            }
            if (!passed) ++nfall;
            if (alpha == 1.0) ++nfull;
            for (int i = 0; i < n3; ++i) r[i] += alpha * dr[i];
            ++iters;
        }
        psi = merit(m, C, mu, W, uf, r, u);
    }

    nd->iters = iters;
    nd->nfull = nfull;
    nd->nfall = nfall;
    nd->psi_first = psi_first;
    nd->psi = psi;
    nd->armijo_margin = armijo_margin;
    free(u); free(A); free(Phi); free(dr); free(rt);
}

int or_env_step(const or_model *m, const double *seg0, const double *seg1, int type,
                double *st, double *pr, int32_t *wkey, double *wr,
                or_contact *cont_out, or_diag *dg)
{
    const int Cmax = m->C_max;
    const double dt = m->dt;
    const double *inv = m->inv_inertia + 3 * type;
    sys_t y;
    build_system(m, seg0, seg1, type, st, pr, &y);
    const double mass = y.mass, mu = y.mu;
    const double *x = y.x, *q = y.q, *R = y.R, *Iinv = y.Iinv, *vs = y.vs, *ws = y.ws;
    const int C = y.C, ncand = y.ncand;
    or_contact *cc = y.cc;
    const double *J = y.J, *uf = y.uf, *W = y.W;
    int n3 = 3 * C;

    /* 10. warm start and Newton */
    double *r = (double *)calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    double *u = (double *)calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    newton_diag nd;
    newton_solve(m, C, mu, mass, cc, W, uf, wkey, wr, r, &nd);

    /* 11. integrate */
    double dv[3] = {0, 0, 0}, dL[3] = {0, 0, 0};
    for (int c = 0; c < C; ++c)
        for (int i = 0; i < 3; ++i) {
            const double *row = J + (size_t)(3 * c + i) * 6;
            for (int t = 0; t < 3; ++t) { dv[t] += row[t] * r[3 * c + i]; dL[t] += row[3 + t] * r[3 * c + i]; }
        }
    double dw[3];
    matvec(Iinv, dL, dw);
    double vp[3], wp[3];
    for (int i = 0; i < 3; ++i) {
        vp[i] = vs[i] + dv[i] / mass;
        wp[i] = ws[i] + dw[i];
    }
    double xn[3] = {x[0] + dt * vp[0], x[1] + dt * vp[1], x[2] + dt * vp[2]};
    double th[3] = {dt * wp[0], dt * wp[1], dt * wp[2]};
    double eq[4], qn[4];
    qexp(th, eq);
    qmul(eq, q, qn);
    qnormalize(qn);
    /* omega remap that conserves world angular momentum:
     * h = I_w(q) w+, w_next = I_w(q_next)^{-1} h; locked axes (inv = 0) carry
     * no momentum. */
    double wb[3], hb[3], h[3];
    mattvec(R, wp, wb);
    for (int i = 0; i < 3; ++i) hb[i] = inv[i] > 0 ? wb[i] * mass / inv[i] : 0.0;
    matvec(R, hb, h);
    double Rn[9], hn[3], wn[3];
    qmat(qn, Rn);
    mattvec(Rn, h, hn);
    for (int i = 0; i < 3; ++i) hn[i] *= inv[i] / mass;
    matvec(Rn, hn, wn);

    st[0] = xn[0]; st[1] = xn[1]; st[2] = xn[2];
    st[3] = qn[0]; st[4] = qn[1]; st[5] = qn[2]; st[6] = qn[3];
    st[7] = vp[0]; st[8] = vp[1]; st[9] = vp[2];
    st[10] = wn[0]; st[11] = wn[1]; st[12] = wn[2];
    pr[2] = pr[3] = pr[4] = 0.0;

    /* warm cache for the next step */
    for (int j = 0; j < Cmax; ++j) {
        wkey[j] = -1;
        wr[3 * j] = wr[3 * j + 1] = wr[3 * j + 2] = 0;
    }
    for (int c = 0; c < C; ++c) {
        wkey[c] = cc[c].key;
        wr[3 * c] = r[3 * c]; wr[3 * c + 1] = r[3 * c + 1]; wr[3 * c + 2] = r[3 * c + 2];
    }
    if (cont_out) {
        if (C > 0) apply_W(n3, W, r, uf, u);
        for (int c = 0; c < C; ++c) {
            for (int i = 0; i < 3; ++i) { cc[c].r[i] = r[3 * c + i]; cc[c].u[i] = u[3 * c + i]; }
            cont_out[c] = cc[c];
        }
    }
    if (dg) {
        dg->n_candidates = ncand;
        dg->n_contacts = C;
        dg->iters = nd.iters;
        dg->n_full_steps = nd.nfull;
        dg->psi_first = nd.psi_first;
        dg->psi_final = nd.psi;
        dg->d_last_kept = y.d_last_kept;
        dg->d_first_dropped = y.d_first_dropped;
        dg->armijo_margin = nd.armijo_margin;
        dg->tangent_tie = y.tangent_tie;
        dg->margin_gap = y.margin_gap;
        dg->n_fallback = nd.nfall;
        dg->reserved = 0;
    }
    free(r); free(u);
    sys_free(&y);
    return C;
}

/* ------------------------------------------------------------------ */
/* PD-controlled articulated hand (hand_mode 1)                         */
/* ------------------------------------------------------------------ */

/* The hand at joint angles q: per link its frame rotation Rl, origin ol,
 * tip bl and centre of mass (the segment midpoint); per joint its world axis
 * and origin (the origin of the link it turns); chain[l][j] = 1 when joint j
 * moves link l (its own joints and its ancestors'). */
typedef struct {
    double *R, *o, *b, *com; /* [L][9], [L][3] x 3 */
    double *axis, *jo;       /* [D][3] */
    unsigned char *chain;    /* [L][D] */
} hand_kin;

static void hand_kin_alloc(const or_model *m, hand_kin *hk)
{
    size_t L = (size_t)m->L, D = (size_t)(m->D > 0 ? m->D : 1);
    hk->R = (double *)calloc(L * 9, sizeof(double));
    hk->o = (double *)calloc(L * 3, sizeof(double));
    hk->b = (double *)calloc(L * 3, sizeof(double));
    hk->com = (double *)calloc(L * 3, sizeof(double));
    hk->axis = (double *)calloc(D * 3, sizeof(double));
    hk->jo = (double *)calloc(D * 3, sizeof(double));
    hk->chain = (unsigned char *)calloc(L * D, 1);
}

static void hand_kin_free(hand_kin *hk)
{
    free(hk->R); free(hk->o); free(hk->b); free(hk->com); free(hk->axis); free(hk->jo); free(hk->chain);
}

static void hand_kinematics_pd(const or_model *m, const double *q, hand_kin *hk)
{
    int L = m->L, D = m->D;
    double *tipq = (double *)malloc(sizeof(double) * 4 * (size_t)L);
    for (int l = 0; l < L; ++l) {
        const double *h = m->hand + (size_t)l * OR_HAND_STRIDE;
        int parent = (int)h[0], j0 = (int)h[1], j1 = (int)h[2];
        double pq[4] = {1, 0, 0, 0}, pp[3] = {0, 0, 0};
        unsigned char *ch = hk->chain + (size_t)l * D;
        if (parent >= 0) {
            memcpy(pq, tipq + 4 * parent, sizeof pq);
            memcpy(pp, hk->b + 3 * parent, sizeof pp);
            memcpy(ch, hk->chain + (size_t)parent * D, (size_t)D);
        }
        double Rp[9];
        qmat(pq, Rp);
        double off[3];
        matvec(Rp, h + 9, off);
        double *o = hk->o + 3 * l;
        o[0] = pp[0] + off[0]; o[1] = pp[1] + off[1]; o[2] = pp[2] + off[2];
        double qf[4];
        qmul(pq, h + 12, qf);
        const int js[2] = {j0, j1};
        for (int k = 0; k < 2; ++k) {
            int j = js[k];
            if (j < 0) continue;
            const double *ax = h + 3 + 3 * k;
            double Rf[9];
            qmat(qf, Rf);
            matvec(Rf, ax, hk->axis + 3 * j);
            memcpy(hk->jo + 3 * j, o, 3 * sizeof(double));
            ch[j] = 1;
            double qj[4], t[4];
            qaxis(ax, q[j], qj);
            qmul(qf, qj, t);
            memcpy(qf, t, sizeof qf);
        }
        double *R = hk->R + 9 * l;
        qmat(qf, R);
        double len = h[16];
        for (int i = 0; i < 3; ++i) {
            hk->b[3 * l + i] = o[i] + len * R[3 * i];
            hk->com[3 * l + i] = o[i] + 0.5 * len * R[3 * i];
        }
        memcpy(tipq + 4 * l, qf, sizeof qf);
    }
    free(tipq);
}

/* Joint-space mass matrix M(q) [D][D]: sum over links of
 * m J_v^T J_v + J_w^T I_w J_w with J_w[:, j] = axis_j and
 * J_v[:, j] = axis_j x (com - origin_j) over the link's chain; a link is a
 * solid cylinder of the hand's link mass (axial inertia m R^2 / 2,
 * transverse m (3 R^2 + len^2) / 12 about its centre). */
static void hand_mass(const or_model *m, const hand_kin *hk, double *M)
{
    int L = m->L, D = m->D;
    memset(M, 0, sizeof(double) * (size_t)D * D);
    double ml = m->link_mass;
    for (int l = 0; l < L; ++l) {
        const double *h = m->hand + (size_t)l * OR_HAND_STRIDE;
        double len = h[16], rad = h[17];
        double Ib[3] = {0.5 * ml * rad * rad, ml * (3 * rad * rad + len * len) / 12.0,
                        ml * (3 * rad * rad + len * len) / 12.0};
        const double *R = hk->R + 9 * l;
        double Iw[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double s_ = 0;
                for (int k = 0; k < 3; ++k) s_ += R[3 * i + k] * Ib[k] * R[3 * j + k];
                Iw[3 * i + j] = s_;
            }
        const unsigned char *ch = hk->chain + (size_t)l * D;
        const double *c = hk->com + 3 * l;
        for (int i = 0; i < D; ++i) {
            if (!ch[i]) continue;
            double ri[3] = {c[0] - hk->jo[3 * i], c[1] - hk->jo[3 * i + 1], c[2] - hk->jo[3 * i + 2]}, vi[3];
            cross3(hk->axis + 3 * i, ri, vi);
            double Iwi[3];
            matvec(Iw, hk->axis + 3 * i, Iwi);
            for (int j = 0; j < D; ++j) {
                if (!ch[j]) continue;
                double rj[3] = {c[0] - hk->jo[3 * j], c[1] - hk->jo[3 * j + 1], c[2] - hk->jo[3 * j + 2]}, vj[3];
                cross3(hk->axis + 3 * j, rj, vj);
                M[(size_t)i * D + j] += ml * dot3(vi, vj) + dot3(hk->axis + 3 * j, Iwi);
            }
        }
    }
}

void or_hand_mass(const or_model *m, const double *q, double *M)
{
    hand_kin hk;
    hand_kin_alloc(m, &hk);
    hand_kinematics_pd(m, q, &hk);
    hand_mass(m, &hk, M);
    hand_kin_free(&hk);
}

/* inverse of an n x n matrix by LU with partial pivoting on the identity */
static int mat_inverse(int n, const double *A, double *Ainv)
{
    double *T = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *e = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = 0;
    for (int col = 0; col < n && rc == 0; ++col) {
        memcpy(T, A, sizeof(double) * (size_t)n * n);
        for (int i = 0; i < n; ++i) e[i] = i == col ? 1.0 : 0.0;
        rc = lu_solve(n, T, e);
        for (int i = 0; i < n; ++i) Ainv[(size_t)i * n + col] = e[i];
    }
    free(T);
    free(e);
    return rc;
}

/* One step of one environment with the PD-controlled hand: the object's
 * steps 1-9 and 11 of the model, with the hand's joint rates as further
 * degrees of freedom.  Generalised velocity nu = (v, w, qdot) (6 + D); the
 * hand's implicit PD law gives (M + dt kd I + dt^2 kp I) qdot+ =
 * M qdot + dt kp (u - q) + (contact impulses), q+ = q + dt qdot+.  A
 * contact between sphere k and link l at the object's contact point p has
 * the Jacobian rows F [I, -(p - x)^, -G_l(p)] with G_l(p)[:, j] =
 * axis_j x (p - origin_j) over the link's chain (the velocity of the
 * object's point relative to the link's material point at p); the table's
 * rows have no hand columns.  hq [2D]: q, qdot, updated in place. */
int or_env_step_pd(const or_model *m, const double *u_cmd, int type, double *st, double *pr, double *hq,
                   int32_t *wkey, double *wr, or_contact *cont_out, or_diag *dg)
{
    const int L = m->L, D = m->D, Cmax = m->C_max;
    const int nd = 6 + D;
    const double dt = m->dt;
    const double mass = pr[0], mu = pr[1];
    const double *fp = pr + 2;
    const double *inv = m->inv_inertia + 3 * type;
    const int S = m->n_spheres[type];
    const double *sph = m->spheres + (size_t)type * m->S_max * 4;
    const double *qh = hq, *qdh = hq + D;

    /* object pose, rotation, inverse inertia, free velocity */
    double x[3] = {st[0], st[1], st[2]}, q[4] = {st[3], st[4], st[5], st[6]}, R[9];
    qnormalize(q);
    qmat(q, R);
    geom_round(m, q, 4);
    geom_round(m, R, 9);
    double Iinv[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s_ = 0;
            for (int k = 0; k < 3; ++k) s_ += R[3 * i + k] * (inv[k] / mass) * R[3 * j + k];
            Iinv[3 * i + j] = s_;
        }
    geom_round(m, Iinv, 9);
    double *nus = (double *)calloc((size_t)nd, sizeof(double));
    double *nup = (double *)calloc((size_t)nd, sizeof(double));
    for (int i = 0; i < 3; ++i) {
        nus[i] = st[7 + i] + dt * (m->gravity[i] + fp[i] / mass);
        nus[3 + i] = st[10 + i];
    }
    geom_round(m, nus, 3);

    /* hand: kinematics at q, mass matrix, PD-implicit effective mass and
     * free joint rates */
    hand_kin hk;
    hand_kin_alloc(m, &hk);
    hand_kinematics_pd(m, qh, &hk);
    double *Mh = (double *)calloc((size_t)(D > 0 ? D * D : 1), sizeof(double));
    double *Ah = (double *)calloc((size_t)(D > 0 ? D * D : 1), sizeof(double));
    double *Ahinv = (double *)calloc((size_t)(D > 0 ? D * D : 1), sizeof(double));
    hand_mass(m, &hk, Mh);
    for (int i = 0; i < D * D; ++i) Ah[i] = Mh[i];
    for (int i = 0; i < D; ++i) Ah[(size_t)i * D + i] += dt * m->kd + dt * dt * m->kp;
    if (D > 0) mat_inverse(D, Ah, Ahinv);
    {
        double *pmom = (double *)calloc((size_t)(D > 0 ? D : 1), sizeof(double));
        for (int i = 0; i < D; ++i) {
            double s_ = dt * m->kp * (u_cmd[i] - qh[i]);
            for (int j = 0; j < D; ++j) s_ += Mh[(size_t)i * D + j] * qdh[j];
            pmom[i] = s_;
        }
        for (int i = 0; i < D; ++i) {
            double s_ = 0;
            for (int j = 0; j < D; ++j) s_ += Ahinv[(size_t)i * D + j] * pmom[j];
            nus[6 + i] = s_;
        }
        free(pmom);
    }

    /* segments of the links at q (velocities enter through the Jacobian) */
    double *seg = (double *)malloc(sizeof(double) * 6 * (size_t)L);
    for (int l = 0; l < L; ++l)
        for (int i = 0; i < 3; ++i) {
            seg[6 * l + i] = hk.o[3 * l + i];
            seg[6 * l + 3 + i] = hk.b[3 * l + i];
        }
    geom_round(m, seg, 6 * L);

    /* candidates and the cap, as in the kinematic model */
    int npair = S * (L + 1);
    cand_t *cand = (cand_t *)malloc(sizeof(cand_t) * (size_t)(npair > 0 ? npair : 1));
    int ncand = 0;
    double margin_gap = INFINITY;
    for (int k = 0; k < S; ++k) {
        double c[3];
        matvec(R, sph + 4 * k, c);
        c[0] += x[0]; c[1] += x[1]; c[2] += x[2];
        geom_round(m, c, 3);
        for (int l = m->collision_mode == 1 ? L : 0; l <= L; ++l) {
            double d, n[3], p[3], vl[3];
            pair_geometry(m, seg, seg, l, c, sph[4 * k + 3], &d, n, p, vl);
            geom_round(m, &d, 1);
            if (fabs(d - m->margin) < margin_gap) margin_gap = fabs(d - m->margin);
            if (d < m->margin) {
                cand[ncand].d = d;
                cand[ncand].key = k * (L + 1) + l;
                ++ncand;
            }
        }
    }
    if (m->collision_mode == 1) {
        cand = (cand_t *)realloc(cand, sizeof(cand_t) * (size_t)(ncand + L * m->link_samples + 1));
        for (int l = 0; l < L; ++l)
            for (int k = 0; k < m->link_samples; ++k) {
                double d, n[3], p[3], vl[3];
                sdf_link_geometry(m, seg, seg, type, R, x, l, k, &d, n, p, vl);
                geom_round(m, &d, 1);
                if (fabs(d - m->margin) < margin_gap) margin_gap = fabs(d - m->margin);
                if (d < m->margin) {
                    cand[ncand].d = d;
                    cand[ncand].key = k * (L + 1) + l;
                    ++ncand;
                }
            }
    }
    qsort(cand, (size_t)ncand, sizeof(cand_t), cand_cmp);
    int C = ncand < Cmax ? ncand : Cmax;
    int n3 = 3 * C;
    or_contact *cc = (or_contact *)calloc((size_t)(C > 0 ? C : 1), sizeof(or_contact));
    double *J = (double *)calloc((size_t)(n3 > 0 ? n3 : 1) * nd, sizeof(double));
    double *uf = (double *)calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    double tangent_tie = INFINITY;
    for (int c = 0; c < C; ++c) {
        int key = cand[c].key;
        int k = key / (L + 1), l = key % (L + 1);
        or_contact *o_ = cc + c;
        o_->key = key;
        o_->link = l;
        if (m->collision_mode == 1 && l < L) {
            sdf_link_geometry(m, seg, seg, type, R, x, l, k, &o_->d, o_->n, o_->p, o_->vlink);
        } else {
            double ctr[3];
            matvec(R, sph + 4 * k, ctr);
            ctr[0] += x[0]; ctr[1] += x[1]; ctr[2] += x[2];
            geom_round(m, ctr, 3);
            pair_geometry(m, seg, seg, l, ctr, sph[4 * k + 3], &o_->d, o_->n, o_->p, o_->vlink);
        }
        geom_round(m, &o_->d, 1);
        geom_round(m, o_->n, 3);
        geom_round(m, o_->p, 3);
        tangent_frame(o_->n, o_->t1, o_->t2);
        geom_round(m, o_->t1, 3);
        geom_round(m, o_->t2, 3);
        if (l < L) {
            /* distance of the tangent-axis rule from a tie (as in the
             * kinematic step) */
            double a0 = fabs(o_->n[0]), a1 = fabs(o_->n[1]), a2 = fabs(o_->n[2]);
            double lo = fmin(a0, fmin(a1, a2)), hi = fmax(a0, fmax(a1, a2));
            double mid = a0 + a1 + a2 - lo - hi;
            if (mid - lo < tangent_tie) tangent_tie = mid - lo;
        }
        double rho[3] = {o_->p[0] - x[0], o_->p[1] - x[1], o_->p[2] - x[2]};
        geom_round(m, rho, 3);
        const double *dirs[3] = {o_->n, o_->t1, o_->t2};
        for (int i = 0; i < 3; ++i) {
            double *row = J + (size_t)(3 * c + i) * nd;
            double rc[3];
            cross3(rho, dirs[i], rc);
            row[0] = dirs[i][0]; row[1] = dirs[i][1]; row[2] = dirs[i][2];
            row[3] = rc[0]; row[4] = rc[1]; row[5] = rc[2];
            if (l < L) {
                const unsigned char *ch = hk.chain + (size_t)l * D;
                for (int j = 0; j < D; ++j) {
                    if (!ch[j]) continue;
                    double rj[3] = {o_->p[0] - hk.jo[3 * j], o_->p[1] - hk.jo[3 * j + 1], o_->p[2] - hk.jo[3 * j + 2]};
                    double g[3];
                    cross3(hk.axis + 3 * j, rj, g);
                    row[6 + j] = -dot3(dirs[i], g);
                }
            }
            double s_ = 0;
            for (int t = 0; t < nd; ++t) s_ += row[t] * nus[t];
            uf[3 * c + i] = s_;
        }
        uf[3 * c] += o_->d >= 0 ? o_->d / dt : m->erp * o_->d / dt;
    }
    /* inverse generalised mass blockdiag(I3 / m, I_w^-1, A_h^-1) and
     * W = J M^-1 J^T + eps I */
    double *Minv = (double *)calloc((size_t)nd * nd, sizeof(double));
    for (int i = 0; i < 3; ++i) Minv[(size_t)i * nd + i] = 1.0 / mass;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Minv[(size_t)(3 + i) * nd + 3 + j] = Iinv[3 * i + j];
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) Minv[(size_t)(6 + i) * nd + 6 + j] = Ahinv[(size_t)i * D + j];
    double *MJt = (double *)calloc((size_t)nd * (n3 > 0 ? n3 : 1), sizeof(double)); /* [nd][3C] */
    for (int a = 0; a < nd; ++a)
        for (int c = 0; c < n3; ++c) {
            double s_ = 0;
            for (int t = 0; t < nd; ++t) s_ += Minv[(size_t)a * nd + t] * J[(size_t)c * nd + t];
            MJt[(size_t)a * n3 + c] = s_;
        }
    double *W = (double *)calloc((size_t)(n3 > 0 ? n3 * n3 : 1), sizeof(double));
    for (int i = 0; i < n3; ++i)
        for (int j = 0; j < n3; ++j) {
            double s_ = 0;
            for (int t = 0; t < nd; ++t) s_ += J[(size_t)i * nd + t] * MJt[(size_t)t * n3 + j];
            W[(size_t)i * n3 + j] = s_ + (i == j ? m->compliance : 0.0);
        }

    /* the contact solve */
    double *r = (double *)calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
    newton_diag ndg;
    newton_solve(m, C, mu, mass, cc, W, uf, wkey, wr, r, &ndg);

    /* integrate: nu+ = nu* + M^-1 J^T r */
    for (int a = 0; a < nd; ++a) {
        double s_ = nus[a];
        for (int c = 0; c < n3; ++c) s_ += MJt[(size_t)a * n3 + c] * r[c];
        nup[a] = s_;
    }
    double xn[3] = {x[0] + dt * nup[0], x[1] + dt * nup[1], x[2] + dt * nup[2]};
    double th[3] = {dt * nup[3], dt * nup[4], dt * nup[5]};
    double eq[4], qn[4];
    qexp(th, eq);
    qmul(eq, q, qn);
    qnormalize(qn);
    double wb[3], hb[3], hmom[3], Rn[9], hn[3], wn[3];
    mattvec(R, nup + 3, wb);
    for (int i = 0; i < 3; ++i) hb[i] = inv[i] > 0 ? wb[i] * mass / inv[i] : 0.0;
    matvec(R, hb, hmom);
    qmat(qn, Rn);
    mattvec(Rn, hmom, hn);
    for (int i = 0; i < 3; ++i) hn[i] *= inv[i] / mass;
    matvec(Rn, hn, wn);
    st[0] = xn[0]; st[1] = xn[1]; st[2] = xn[2];
    st[3] = qn[0]; st[4] = qn[1]; st[5] = qn[2]; st[6] = qn[3];
    st[7] = nup[0]; st[8] = nup[1]; st[9] = nup[2];
    st[10] = wn[0]; st[11] = wn[1]; st[12] = wn[2];
    pr[2] = pr[3] = pr[4] = 0.0;
    for (int j = 0; j < D; ++j) {
        hq[D + j] = nup[6 + j];
        hq[j] = qh[j] + dt * nup[6 + j];
    }

    /* warm cache and outputs */
    for (int j = 0; j < Cmax; ++j) {
        wkey[j] = -1;
        wr[3 * j] = wr[3 * j + 1] = wr[3 * j + 2] = 0;
    }
    for (int c = 0; c < C; ++c) {
        wkey[c] = cc[c].key;
        wr[3 * c] = r[3 * c]; wr[3 * c + 1] = r[3 * c + 1]; wr[3 * c + 2] = r[3 * c + 2];
    }
    if (cont_out) {
        double *uu = (double *)calloc((size_t)(n3 > 0 ? n3 : 1), sizeof(double));
        if (C > 0) apply_W(n3, W, r, uf, uu);
        for (int c = 0; c < C; ++c) {
            for (int i = 0; i < 3; ++i) { cc[c].r[i] = r[3 * c + i]; cc[c].u[i] = uu[3 * c + i]; }
            cont_out[c] = cc[c];
        }
        free(uu);
    }
    if (dg) {
        memset(dg, 0, sizeof *dg);
        dg->n_candidates = ncand;
        dg->n_contacts = C;
        dg->iters = ndg.iters;
        dg->n_full_steps = ndg.nfull;
        dg->psi_first = ndg.psi_first;
        dg->psi_final = ndg.psi;
        dg->d_last_kept = C > 0 ? cand[C - 1].d : -INFINITY;
        dg->d_first_dropped = ncand > C ? cand[C].d : INFINITY;
        dg->armijo_margin = ndg.armijo_margin;
        dg->tangent_tie = tangent_tie;
        dg->margin_gap = margin_gap;
        dg->n_fallback = ndg.nfall;
    }
    free(cand); free(cc); free(J); free(uf); free(Minv); free(MJt); free(W); free(r); free(seg);
    free(Mh); free(Ah); free(Ahinv); free(nus); free(nup);
    hand_kin_free(&hk);
    return C;
}

double or_step_cost_pd(const or_model *m, const double *obs, const double *qo, const double *obs_gt,
                       const double *q_gt)
{
    double s_ = or_step_cost(m, obs, obs_gt);
    for (int j = 0; j < m->D; ++j) s_ += m->w_q * (qo[j] - q_gt[j]) * (qo[j] - q_gt[j]);
    return s_;
}

void or_batch_step_pd(const or_model *m, int K, const int32_t *env_type, const double *u, double *state,
                      double *params, double *hstate, int32_t *wkey, double *wr, or_contact *cont, or_diag *diag,
                      double *obs)
{
    int L = m->L, Cmax = m->C_max, D = m->D;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < K; ++i) {
        or_contact local[OR_MAX_CMAX];
        or_contact *cp = cont ? cont + (size_t)i * Cmax : local;
        int nc = or_env_step_pd(m, u, env_type[i], state + 13 * (size_t)i, params + 5 * (size_t)i,
                                hstate + 2 * (size_t)D * i, wkey + (size_t)i * Cmax, wr + (size_t)i * Cmax * 3, cp,
                                diag ? diag + i : NULL);
        if (cont)
            for (int c = nc; c < Cmax; ++c) { memset(cp + c, 0, sizeof(or_contact)); cp[c].key = -1; }
        if (obs) or_observe(m, nc, cp, obs + (size_t)i * L * 4);
    }
}

/* ------------------------------------------------------------------ */
/* observation and cost                                                */
/* ------------------------------------------------------------------ */

/* Force on each sensor link exerted by the object over the step:
 * c_l = -(1/dt) sum_{contacts on l} (r_n n + r_t1 t1 + r_t2 t2);
 * obs = (|c_l|, c_l/|c_l|), with the direction zeroed at or below tau_c.
 * Table contacts are not sensed. */
void or_observe(const or_model *m, int nc, const or_contact *cont, double *obs)
{
    int L = m->L;
    double *f = (double *)calloc((size_t)L * 3, sizeof(double));
    for (int c = 0; c < nc; ++c) {
        int l = cont[c].link;
        if (l >= L) continue;
        for (int i = 0; i < 3; ++i)
            f[3 * l + i] -= (cont[c].r[0] * cont[c].n[i] + cont[c].r[1] * cont[c].t1[i] + cont[c].r[2] * cont[c].t2[i]) / m->dt;
    }
    for (int l = 0; l < L; ++l) {
        double mag = norm3(f + 3 * l);
        obs[4 * l] = mag;
        for (int i = 0; i < 3; ++i) obs[4 * l + 1 + i] = mag > m->tau_contact ? f[3 * l + i] / mag : 0.0;
    }
    free(f);
}

/* Step cost: sum over sensors of w_mag (|c|-|c_gt|)^2 + w_dir |c_hat - c_hat_gt|^2. */
double or_step_cost(const or_model *m, const double *obs, const double *obs_gt)
{
    double s = 0;
    for (int l = 0; l < m->L; ++l) {
        const double *a = obs + 4 * l, *b = obs_gt + 4 * l;
        double dm = a[0] - b[0];
        double dd[3] = {a[1] - b[1], a[2] - b[2], a[3] - b[3]};
        s += m->w_mag * dm * dm + m->w_dir * dot3(dd, dd);
    }
    return s;
}

/* Observation of Eq. 3 (see oracle.h): contact force, slip direction in the
 * sensor's surface frame, spin direction about the mean contact normal. */
void or_observe_eq3(const or_model *m, int nc, const or_contact *cont, const double *seg0, const double *seg1,
                    const double *omega_obj, double *obs)
{
    int L = m->L;
    double eps = m->compliance;
    double *f = (double *)calloc((size_t)L * 3, sizeof(double));
    double *N = (double *)calloc((size_t)L * 3, sizeof(double));
    double *S = (double *)calloc((size_t)L * 3, sizeof(double));
    double *W = (double *)calloc((size_t)L, sizeof(double));
    for (int c = 0; c < nc; ++c) {
        int l = cont[c].link;
        if (l >= L) continue;
        const or_contact *k = &cont[c];
        double rn = k->r[0];
        /* relative tangential velocity of the object's point against the
         * link's: the constraint velocity less the compliance term */
        double v1 = k->u[1] - eps * k->r[1], v2 = k->u[2] - eps * k->r[2];
        for (int i = 0; i < 3; ++i) {
            f[3 * l + i] -= (k->r[0] * k->n[i] + k->r[1] * k->t1[i] + k->r[2] * k->t2[i]) / m->dt;
            N[3 * l + i] += rn * k->n[i];
            S[3 * l + i] += rn * (v1 * k->t1[i] + v2 * k->t2[i]);
        }
        W[l] += rn;
    }
    for (int l = 0; l < L; ++l) {
        double *o = obs + 7 * l;
        double mag = norm3(f + 3 * l);
        o[0] = mag;
        for (int i = 0; i < 3; ++i) o[1 + i] = mag > m->tau_contact ? f[3 * l + i] / mag : 0.0;
        o[4] = o[5] = o[6] = 0.0;
        double nn = norm3(N + 3 * l);
        if (W[l] <= 0.0 || nn <= 0.0) continue;
        double nb[3] = {N[3 * l] / nn, N[3 * l + 1] / nn, N[3 * l + 2] / nn};
        const double *a0 = seg0 + 6 * l, *b0 = seg0 + 6 * l + 3, *a1 = seg1 + 6 * l, *b1 = seg1 + 6 * l + 3;
        double ab[3], va[3], vb[3], dv[3];
        for (int i = 0; i < 3; ++i) {
            ab[i] = b0[i] - a0[i];
            va[i] = (a1[i] - a0[i]) / m->dt;
            vb[i] = (b1[i] - b0[i]) / m->dt;
            dv[i] = vb[i] - va[i];
        }
        double sl[3] = {S[3 * l] / W[l], S[3 * l + 1] / W[l], S[3 * l + 2] / W[l]};
        if (norm3(sl) > m->tau_slip) {
            /* surface frame: the link axis projected on the tangent plane
             * (if the normal runs along the axis, the contact-frame rule) */
            double la = norm3(ab);
            double ea[3] = {ab[0] / la, ab[1] / la, ab[2] / la};
            double an = dot3(ea, nb);
            double e1[3] = {ea[0] - an * nb[0], ea[1] - an * nb[1], ea[2] - an * nb[2]};
            double n1 = norm3(e1);
            double e2[3];
            if (n1 < 1e-6) {
                tangent_frame(nb, e1, e2);
            } else {
                for (int i = 0; i < 3; ++i) e1[i] /= n1;
                cross3(nb, e1, e2);
            }
            double d1 = dot3(sl, e1), d2 = dot3(sl, e2);
            double dn = sqrt(d1 * d1 + d2 * d2);
            if (dn > 0.0) { o[4] = d1 / dn; o[5] = d2 / dn; }
        }
        double wl[3];
        cross3(ab, dv, wl);
        double l2 = dot3(ab, ab);
        double spin = 0.0;
        for (int i = 0; i < 3; ++i) spin += (omega_obj[i] - wl[i] / l2) * nb[i];
        o[6] = spin > m->tau_spin ? 1.0 : (spin < -m->tau_spin ? -1.0 : 0.0);
    }
    free(f); free(N); free(S); free(W);
}

/* the angle between two vectors of n = 2 or 3 components:
 * atan2(|a x b|, a . b), exact also when the inputs are unit vectors only up
 * to their rounding (where acos of the dot product is off by ~sqrt(2 ulp)) */
static double unit_angle(const double *a, const double *b, int n)
{
    double d = 0.0, c;
    for (int i = 0; i < n; ++i) d += a[i] * b[i];
    if (n == 2) {
        c = fabs(a[0] * b[1] - a[1] * b[0]);
    } else {
        double x[3];
        cross3(a, b, x);
        c = norm3(x);
    }
    return atan2(c, d);
}

double or_step_cost_eq3(const or_model *m, const double *obs, const double *obs_gt)
{
    const double *w = m->w_eq3;   /* w4 .. w10 */
    double s = 0;
    for (int l = 0; l < m->L; ++l) {
        const double *a = obs + 7 * l, *b = obs_gt + 7 * l;
        int in_a = a[0] > m->tau_contact, in_b = b[0] > m->tau_contact;
        int sl_a = a[4] != 0.0 || a[5] != 0.0, sl_b = b[4] != 0.0 || b[5] != 0.0;
        int ro_a = a[6] != 0.0, ro_b = b[6] != 0.0;
        if (in_a == in_b) {
            s += w[1] * fabs(a[0] - b[0]);
            if (in_a) s += w[2] * unit_angle(a + 1, b + 1, 3);
        } else {
            s += w[0];
        }
        if (sl_a == sl_b) {
            if (sl_a) s += w[4] * unit_angle(a + 4, b + 4, 2);
        } else {
            s += w[3];
        }
        if (ro_a == ro_b) {
            if (ro_a) s += w[6] * fabs((a[6] > 0.0 ? 1.0 : 0.0) - (b[6] > 0.0 ? 1.0 : 0.0));
        } else {
            s += w[5];
        }
    }
    return s;
}

void or_batch_step(const or_model *m, int K, const int32_t *env_type,
                   const double *u_prev, const double *u,
                   double *state, double *params, int32_t *wkey, double *wr,
                   or_contact *cont, or_diag *diag, double *obs)
{
    int L = m->L, Cmax = m->C_max;
    double *seg0 = (double *)malloc(sizeof(double) * 6 * (size_t)L);
    double *seg1 = (double *)malloc(sizeof(double) * 6 * (size_t)L);
    or_hand_fk(m, u_prev, seg0);
    or_hand_fk(m, u, seg1);
    geom_round(m, seg0, 6 * L);
    geom_round(m, seg1, 6 * L);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < K; ++i) {
        or_contact local[OR_MAX_CMAX];
        or_contact *cp = cont ? cont + (size_t)i * Cmax : local;
        int nc = or_env_step(m, seg0, seg1, env_type[i], state + 13 * (size_t)i, params + 5 * (size_t)i,
                             wkey + (size_t)i * Cmax, wr + (size_t)i * Cmax * 3, cp, diag ? diag + i : NULL);
        if (cont)
            for (int c = nc; c < Cmax; ++c) { memset(cp + c, 0, sizeof(or_contact)); cp[c].key = -1; }
        if (obs) {
            if (m->cost_mode == 1)
                or_observe_eq3(m, nc, cp, seg0, seg1, state + 13 * (size_t)i + 10, obs + (size_t)i * L * 7);
            else
                or_observe(m, nc, cp, obs + (size_t)i * L * 4);
        }
    }
    free(seg0);
    free(seg1);
}

void or_batch_cost(const or_model *m, int K, int G, const int32_t *group_start,
                   const double *obs, const double *obs_gt, double *cost_sum)
{
    int L = m->L;
    for (int g = 0; g < G; ++g)
        for (int i = group_start[g]; i < group_start[g + 1] && i < K; ++i)
            cost_sum[i] += m->cost_mode == 1
                               ? or_step_cost_eq3(m, obs + (size_t)i * L * 7, obs_gt + (size_t)g * L * 7)
                               : or_step_cost(m, obs + (size_t)i * L * 4, obs_gt + (size_t)g * L * 4);
}

int or_argmin(int n, const double *v)
{
    int best = 0;
    double bv = INFINITY;
    for (int i = 0; i < n; ++i) {
        double x = isnan(v[i]) ? INFINITY : v[i];
        if (x < bv) { bv = x; best = i; }
    }
    return best;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 and the population-based resampler                    */
/* ------------------------------------------------------------------ */

/* Philox4x32 with 10 rounds: each round multiplies words 0 and 2 by the two
 * published multipliers, mixes the high halves with the other words and the
 * round key, and the key is bumped by the two Weyl constants between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u01(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

/* Two standard normals from two Philox words (Box-Muller). */
static void box_muller(uint32_t a, uint32_t b, double *n0, double *n1)
{
    double u = u01(a), v = u01(b);
    double rad = sqrt(-2.0 * log(u));
    double ang = 2.0 * M_PI * v;
    *n0 = rad * cos(ang);
    *n1 = rad * sin(ang);
}

typedef struct {
    double c;
    int32_t i;
} rank_t;

static int rank_cmp(const void *pa, const void *pb)
{
    const rank_t *a = (const rank_t *)pa, *b = (const rank_t *)pb;
    if (a->c < b->c) return -1;
    if (a->c > b->c) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

void or_resample_pbo(const or_model *m, const or_resample_cfg *rc, int K, int G,
                     const int32_t *group_start, uint32_t window_idx,
                     double *cost_sum, double *state, double *params,
                     int32_t *wkey, double *wr, int32_t *parent)
{
    int Cmax = m->C_max;
    (void)K;
    uint32_t key[2] = {(uint32_t)(rc->seed & 0xffffffffu), (uint32_t)(rc->seed >> 32)};
    for (int g = 0; g < G; ++g) {
        int lo = group_start[g], hi = group_start[g + 1];
        int n = hi - lo;
        if (n <= 0) continue;
        /* rank by (cost, index) ascending; NaN ranks as +inf */
        rank_t *rk = (rank_t *)malloc(sizeof(rank_t) * (size_t)n);
        for (int j = 0; j < n; ++j) {
            double c = cost_sum[lo + j];
            rk[j].c = isnan(c) ? INFINITY : c;
            rk[j].i = lo + j;
        }
        qsort(rk, (size_t)n, sizeof(rank_t), rank_cmp);
        int kb = (int)floor((double)n * rc->elite_frac);
        if (kb < 1) kb = 1;
        if (kb > n) kb = n;
        for (int t = 0; t < kb; ++t) parent[rk[t].i] = -1;
        for (int t = kb; t < n; ++t) {
            int j = rk[t].i;
            uint32_t ctr[4] = {(uint32_t)j, window_idx, 0u, 0u}, w[4];
            or_philox4x32_10(ctr, key, w);
            int pr_rank = (int)(((uint64_t)w[0] * (uint64_t)kb) >> 32);
            int p = rk[pr_rank].i;
            parent[j] = p;
            memcpy(state + 13 * (size_t)j, state + 13 * (size_t)p, 13 * sizeof(double));
            memcpy(params + 5 * (size_t)j, params + 5 * (size_t)p, 5 * sizeof(double));
            memcpy(wkey + (size_t)j * Cmax, wkey + (size_t)p * Cmax, (size_t)Cmax * sizeof(int32_t));
            memcpy(wr + (size_t)j * Cmax * 3, wr + (size_t)p * Cmax * 3, (size_t)Cmax * 3 * sizeof(double));
            /* exploration: parameter noise (Sec. III-D, N(theta, Sigma_theta))
             * and a random force on the object (N(0, Sigma_v)) */
            double nrm[6];
            uint32_t c1[4] = {(uint32_t)j, window_idx, 1u, 0u}, c2[4] = {(uint32_t)j, window_idx, 2u, 0u}, w1[4], w2[4];
            or_philox4x32_10(c1, key, w1);
            or_philox4x32_10(c2, key, w2);
            box_muller(w1[0], w1[1], &nrm[0], &nrm[1]);
            box_muller(w1[2], w1[3], &nrm[2], &nrm[3]);
            box_muller(w2[0], w2[1], &nrm[4], &nrm[5]);
            double *pp = params + 5 * (size_t)j;
            double mu = pp[1] + rc->sigma_mu * nrm[0];
            double ms = pp[0] + rc->sigma_m * nrm[1];
            pp[1] = mu < rc->mu_lo ? rc->mu_lo : (mu > rc->mu_hi ? rc->mu_hi : mu);
            pp[0] = ms < rc->m_lo ? rc->m_lo : (ms > rc->m_hi ? rc->m_hi : ms);
            pp[2] = rc->sigma_f * nrm[2];
            pp[3] = rc->sigma_f * nrm[3];
            pp[4] = rc->sigma_f * nrm[4];
        }
        free(rk);
        for (int j = lo; j < hi; ++j) cost_sum[j] = 0.0;
    }
}

/* Resampling with replacement: copies from a snapshot of the envs before
 * the call (a parent may itself be overwritten), then explores every env. */
void or_resample_apply(const or_model *m, const or_resample_cfg *rc, int K, const int32_t *parent,
                       uint32_t window_idx, double *cost_sum, double *state, double *params,
                       int32_t *wkey, double *wr)
{
    int Cmax = m->C_max;
    uint32_t key[2] = {(uint32_t)(rc->seed & 0xffffffffu), (uint32_t)(rc->seed >> 32)};
    double *st0 = (double *)malloc(sizeof(double) * 13 * (size_t)K);
    double *pr0 = (double *)malloc(sizeof(double) * 5 * (size_t)K);
    int32_t *wk0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)K * Cmax);
    double *wr0 = (double *)malloc(sizeof(double) * (size_t)K * Cmax * 3);
    memcpy(st0, state, sizeof(double) * 13 * (size_t)K);
    memcpy(pr0, params, sizeof(double) * 5 * (size_t)K);
    memcpy(wk0, wkey, sizeof(int32_t) * (size_t)K * Cmax);
    memcpy(wr0, wr, sizeof(double) * (size_t)K * Cmax * 3);
    for (int j = 0; j < K; ++j) {
        int p = parent[j];
        memcpy(state + 13 * (size_t)j, st0 + 13 * (size_t)p, 13 * sizeof(double));
        memcpy(wkey + (size_t)j * Cmax, wk0 + (size_t)p * Cmax, (size_t)Cmax * sizeof(int32_t));
        memcpy(wr + (size_t)j * Cmax * 3, wr0 + (size_t)p * Cmax * 3, (size_t)Cmax * 3 * sizeof(double));
        double nrm[6];
        uint32_t c1[4] = {(uint32_t)j, window_idx, 1u, 0u}, c2[4] = {(uint32_t)j, window_idx, 2u, 0u}, w1[4], w2[4];
        or_philox4x32_10(c1, key, w1);
        or_philox4x32_10(c2, key, w2);
        box_muller(w1[0], w1[1], &nrm[0], &nrm[1]);
        box_muller(w1[2], w1[3], &nrm[2], &nrm[3]);
        box_muller(w2[0], w2[1], &nrm[4], &nrm[5]);
        const double *pp0 = pr0 + 5 * (size_t)p;
        double *pp = params + 5 * (size_t)j;
        double mu = pp0[1] + rc->sigma_mu * nrm[0];
        double ms = pp0[0] + rc->sigma_m * nrm[1];
        pp[1] = mu < rc->mu_lo ? rc->mu_lo : (mu > rc->mu_hi ? rc->mu_hi : mu);
        pp[0] = ms < rc->m_lo ? rc->m_lo : (ms > rc->m_hi ? rc->m_hi : ms);
        pp[2] = rc->sigma_f * nrm[2];
        pp[3] = rc->sigma_f * nrm[3];
        pp[4] = rc->sigma_f * nrm[4];
        cost_sum[j] = 0.0;
    }
    free(st0); free(pr0); free(wk0); free(wr0);
}

/* ------------------------------------------------------------------ */
/* ADD metric                                                          */
/* ------------------------------------------------------------------ */

double or_add(const or_model *m, int type, const double *pa, const double *pb)
{
    int S = m->n_spheres[type];
    const double *sph = m->spheres + (size_t)type * m->S_max * 4;
    double qa[4] = {pa[3], pa[4], pa[5], pa[6]}, qb[4] = {pb[3], pb[4], pb[5], pb[6]};
    qnormalize(qa);
    qnormalize(qb);
    double Ra[9], Rb[9];
    qmat(qa, Ra);
    qmat(qb, Rb);
    double s = 0;
    for (int k = 0; k < S; ++k) {
        double a[3], b[3];
        matvec(Ra, sph + 4 * k, a);
        matvec(Rb, sph + 4 * k, b);
        double d[3] = {(a[0] - b[0]) + (pa[0] - pb[0]), (a[1] - b[1]) + (pa[1] - pb[1]), (a[2] - b[2]) + (pa[2] - pb[2])};
        s += norm3(d);
    }
    return S > 0 ? s / S : 0.0;
}

/* ------------------------------------------------------------------ */
/* window cost of one environment (for finite-difference gradients)     */
/* ------------------------------------------------------------------ */

double or_window_cost(const or_model *m, int type, const double *st0, const double *pr0,
                      const int32_t *wkey0, const double *wr0, int T,
                      const double *u_seq, const double *obs_gt)
{
    int L = m->L, D = m->D, Cmax = m->C_max;
    double st[13], pr[5];
    memcpy(st, st0, sizeof st);
    memcpy(pr, pr0, sizeof pr);
    int32_t wkey[OR_MAX_CMAX];
    double wr[OR_MAX_CMAX * 3];
    for (int j = 0; j < Cmax; ++j) {
        wkey[j] = wkey0 ? wkey0[j] : -1;
        for (int i = 0; i < 3; ++i) wr[3 * j + i] = wr0 ? wr0[3 * j + i] : 0.0;
    }
    double *seg0 = (double *)malloc(sizeof(double) * 6 * (size_t)L);
    double *seg1 = (double *)malloc(sizeof(double) * 6 * (size_t)L);
    double *obs = (double *)malloc(sizeof(double) * 4 * (size_t)L);
    or_contact cont[OR_MAX_CMAX];
    double total = 0;
    for (int t = 0; t < T; ++t) {
        or_hand_fk(m, u_seq + (size_t)t * D, seg0);
        or_hand_fk(m, u_seq + (size_t)(t + 1) * D, seg1);
        geom_round(m, seg0, 6 * L);
        geom_round(m, seg1, 6 * L);
        int nc = or_env_step(m, seg0, seg1, type, st, pr, wkey, wr, cont, NULL);
        or_observe(m, nc, cont, obs);
        total += or_step_cost(m, obs, obs_gt + (size_t)t * L * 4);
    }
    free(seg0); free(seg1); free(obs);
    return total;
}

/* ------------------------------------------------------------------ */
/* threads (for timing the oracle)                                      */
/* ------------------------------------------------------------------ */

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
