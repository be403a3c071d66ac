/*
 * oracle.h -- plain FP64 CPU oracle for sample-based in-hand pose tracking
 * (Liang et al., "In-Hand Object Pose Tracking via Contact Feedback and
 * GPU-Accelerated Robotic Simulation", arXiv 2002.12160).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path
 * (libpt + its Python binding) never links, imports or calls it, and the two
 * share no source: no headers, helpers, tables or constants.
 *
 * What it computes (Sec. III-A..III-D, Alg. 1 of the paper): one step of the
 * world model s_{t+1} = f(s_t, u_t, theta) for each of K perturbed simulations
 * (a rigid object made of spheres, a kinematic capsule hand driven by the same
 * joint command u_t in every simulation, a table plane, Coulomb friction), the
 * per-sensor contact-force observation, the step cost against the observed
 * one, the running window cost and its argmin (Eq. 1-2), the population-based
 * resampler (Sec. III-D.3) and the ADD error metric (Sec. IV).
 *
 * The paper does not specify its simulator's internals; the discrete model
 * below is the reading fixed for this project (sphere-set object, capsule
 * links, speculative contacts with Baumgarte depenetration, a compliant
 * Delassus operator, Coulomb friction written as a second-order-cone
 * complementarity problem solved by a smoothed Fischer-Burmeister Newton
 * method with Armijo backtracking).  The oracle forms the full 3C x 3C Newton
 * matrix and solves it by dense LU with partial pivoting.
 *
 * Parity pins: closed forms (free fall, momentum, resting force, sliding
 * onset), the NCP certificate on converged solves, single-contact brute-force
 * mode enumeration, narrow-phase brute force, Philox known-answer vectors,
 * cost / argmin / ADD identities (see tests/test_oracle_*.py).
 *
 * Layouts are env-major (AoS), all doubles:
 *   state  [K][13]  x(3) q(4: w,x,y,z) v(3) w(3), world frame
 *   params [K][5]   m, mu, f_pert(3)
 *   warm   key [K][C_max] int32 (-1 = empty), r [K][C_max][3]
 *   obs    [K][L][4] |c|, c_hat(3)
 */
#ifndef PT_ORACLE_H
#define PT_ORACLE_H

#include <stdint.h>

#define OR_HAND_STRIDE 20
#define OR_MAX_CMAX 64

typedef struct {
    int32_t L, D, n_types, S_max, C_max;
    int32_t newton_iters;   /* fixed-N mode: exactly this many iterations      */
    int32_t converged;      /* 1: iterate until Psi < conv_tol or conv_max     */
    int32_t conv_max_iters;
    double conv_tol;
    double dt;
    double gravity[3];
    double margin, erp, compliance, kappa, fb_delta, armijo_sigma;
    double tau_contact, w_mag, w_dir;
    const double *hand;        /* [L][20] link table                            */
    const double *spheres;     /* [n_types][S_max][4] body-frame centre, radius */
    const int32_t *n_spheres;  /* [n_types]                                     */
    const double *inv_inertia; /* [n_types][3] principal inverse inertia per unit mass (0 = locked axis) */
    int32_t cost_mode;         /* 0: force magnitude / direction cost, obs [L][4];
                                * 1: Eq. 3 with contact-state, slip and spin terms, obs [L][7] */
    double tau_slip, tau_spin; /* slip thresholds: m/s, rad/s                    */
    double w_eq3[7];           /* w4 .. w10 of Eq. 3                             */
    int32_t geom_f32;          /* diagnostic only (0 = off): round to float32 every
                                * geometric quantity a float32 implementation holds
                                * (hand segments, rotation, inverse inertia, free
                                * velocity, sphere centres, contact gap, normal,
                                * frame, point and link velocity), to measure how
                                * far a step's result moves under such rounding;
                                * 2: also move each rounded value one float32
                                * step, up or down by a hash of its bits */
    /* PD-controlled hand (or_env_step_pd): joint gains, the mass of every
     * capsule link and the weight of the joint-angle term of the cost */
    double kp, kd, link_mass, w_q;
    /* Link-object collision (collision_mode): 0 = the object's sphere set;
     * 1 = the object's signed distance field, sampled on a regular grid in
     * the object frame and interpolated trilinearly, queried at link_samples
     * points along each link's axis (t = m / (link_samples - 1); the middle
     * for one sample): sample m of link l is a contact candidate with key
     * m*(L+1)+l and gap phi - radius_l, its normal minus the field's unit
     * gradient, its point on the object the sample moved by -phi along the
     * gradient.  Object-table contacts stay with the sphere set. */
    int32_t collision_mode, link_samples, sdf_n;
    const double *sdf;         /* [n_types][sdf_n^3] node values, x fastest, then y, z */
    const double *sdf_box;     /* [n_types][4] grid origin (object frame) and node spacing */
} or_model;

typedef struct {
    int32_t key, link;         /* key = k*(L+1)+l ; link == L is the table      */
    double d;                  /* signed gap                                    */
    double n[3], t1[3], t2[3]; /* contact frame, n points from link to object   */
    double p[3];               /* contact point on the object                   */
    double vlink[3];           /* velocity of the link surface point            */
    double r[3];               /* impulse on the object in (n,t1,t2)            */
    double u[3];               /* relative velocity W r + u_free in (n,t1,t2)   */
} or_contact;

typedef struct {
    int32_t n_candidates;      /* pairs with d < margin                         */
    int32_t n_contacts;        /* after the C_max cap                           */
    int32_t iters;             /* Newton iterations run                         */
    int32_t n_full_steps;      /* iterations that accepted alpha = 1            */
    double psi_first;          /* merit at the first iterate                    */
    double psi_final;          /* merit at the returned impulses                */
    double d_last_kept;        /* gap of the last contact kept by the cap       */
    double d_first_dropped;    /* gap of the first candidate the cap drops (+inf if none) */
    /* Distances of the step's discrete decisions from their thresholds (the
     * places where a rounding-level change of the inputs can change the
     * result by more than rounding):
     * armijo_margin: smallest |Psi(r + a dr) - (1 - 2 sigma a) Psi(r)| / Psi(r)
     *   over the line-search trials whose outcome decides the step taken
     *   (every trial evaluated except a = 1/8, which is taken either way)
     *   and whose flip would move the impulses by more than ARMIJO_IMPACT of
     *   the impulse scale max(m |g| dt, max |r|): a flip changes the step by
     *   at least a/2 |dr|_inf; +inf if there is no such trial;
     * tangent_tie: smallest difference between the two smallest |n_i| of a
     *   kept sphere-link contact's normal (the tangent-axis rule; a table
     *   contact's normal is exactly e_z); +inf without such contacts;
     * margin_gap: smallest |d - margin| over all pairs (whether a pair is a
     *   candidate at all). */
    double armijo_margin;
    double tangent_tie;
    double margin_gap;
    int32_t n_fallback;        /* iterations where no trial passed (a = 1/8)    */
    int32_t reserved;
} or_diag;

/* Flips of an Armijo decision that move the impulses by less than this
 * fraction of the impulse scale are not counted in armijo_margin. */
#define OR_ARMIJO_IMPACT 1e-6

/* Forward kinematics of the kinematic hand at joint vector u[D]:
 * seg[L][6] = segment endpoints a(3), b(3) in the world frame. */
void or_hand_fk(const or_model *m, const double *u, double *seg);

/* One step of one environment.  seg0 = FK(u_{t-1}), seg1 = FK(u_t).
 * st[13], pr[5], wkey[C_max], wr[C_max*3] are updated in place.
 * cont[C_max] (may be NULL) receives the solved contacts; dg may be NULL.
 * Returns the number of contacts. */
int or_env_step(const or_model *m, const double *seg0, const double *seg1, int type,
                double *st, double *pr, int32_t *wkey, double *wr,
                or_contact *cont, or_diag *dg);

/* The contact system of one environment at its current state, without
 * stepping: the capped contacts cont[C], the compliant Delassus matrix
 * W[3C][3C] and the free relative velocity uf[3C] (callers size the buffers
 * for C_max).  Returns C. */
int or_env_system(const or_model *m, const double *seg0, const double *seg1, int type,
                  const double *st, const double *pr, or_contact *cont, double *W, double *uf);

/* Per-sensor observation from a step's contacts: obs[L][4]. */
void or_observe(const or_model *m, int nc, const or_contact *cont, double *obs);

/* Step cost of one simulation's observation against the observed one. */
double or_step_cost(const or_model *m, const double *obs, const double *obs_gt);

/* PD-controlled hand (the hand's joints are state; Sec. IV-A's PD hand).
 * Every joint of the link table is revolute; q and qdot [D] are per
 * simulation (hq = [q, qdot]).  Each capsule link is a solid cylinder of
 * mass link_mass; the controller compensates the hand's gravity and the
 * step neglects velocity-product forces.  Implicit PD toward the command u:
 * (M(q) + dt kd I + dt^2 kp I) qdot+ = M(q) qdot + dt kp (u - q) + J_h^T r,
 * q+ = q + dt qdot+.  A sphere-link contact couples the object's velocity
 * and the joint rates of the link's chain (the velocity of the object's
 * contact point relative to the link's material point there); the contact
 * model, cap, solve and object integration are those of or_env_step.  Links
 * touch the object only.  u [D] is the step's command.  Returns C. */
int or_env_step_pd(const or_model *m, const double *u, int type, double *st, double *pr, double *hq,
                   int32_t *wkey, double *wr, or_contact *cont, or_diag *dg);

/* Joint-space mass matrix M(q) [D][D] of the PD hand (sum over links of
 * m J_v^T J_v + J_w^T I_w J_w at the link's centre of mass). */
void or_hand_mass(const or_model *m, const double *q, double *M);

/* K environments of or_env_step_pd (OpenMP); hstate [K][2D]; obs [K][L][4]
 * the force observation (the joint angles are hstate's first D columns). */
void or_batch_step_pd(const or_model *m, int K, const int32_t *env_type, const double *u, double *state,
                      double *params, double *hstate, int32_t *wkey, double *wr, or_contact *cont, or_diag *diag,
                      double *obs);

/* Step cost with the joint-angle term: or_step_cost + w_q |q - q_gt|^2
 * (Eq. 3's first term, squared like the force terms). */
double or_step_cost_pd(const or_model *m, const double *obs, const double *q, const double *obs_gt,
                       const double *q_gt);

/* Observation of Eq. 3 (cost_mode 1), per sensor l, obs[l][7]:
 * |c|, c/|c| (0 when |c| <= tau_contact), d (2), rot, where, over the
 * link's contacts with normal impulses r_n (weights W = sum r_n):
 * n_bar = normalised sum r_n n, the slip velocity s = sum r_n (relative
 * tangential velocity of the object's contact point against the link's,
 * u - eps r in (t1, t2)) / W; when |s| > tau_slip, d = s in the sensor's
 * surface frame (e1 = the link axis projected on the plane normal to n_bar,
 * e2 = n_bar x e1), normalised, else 0; rot = sign of
 * (omega_obj - omega_link) . n_bar when its size exceeds tau_spin, else 0.
 * omega_link = ((b - a) x (vb - va)) / |b - a|^2 from the segment's end
 * velocities; omega_obj is the object's angular velocity after the step.
 * seg0 / seg1: the step's segments at u_prev and u ([L][6]). */
void or_observe_eq3(const or_model *m, int nc, const or_contact *cont, const double *seg0, const double *seg1,
                    const double *omega_obj, double *obs);

/* Step cost of Eq. 3 (cost_mode 1), obs [L][7] each: per sensor
 * w4 (1 - a) + a (w5 |dM| + w6 angle(c, c_gt)) + w7 (1 - b) + b w8 angle(d, d_gt)
 * + w9 (1 - g) + g w10 |r - r_gt|, a / b / g = agreement of the contact,
 * slip and spin states, the angles and |r - r_gt| counted where both sides
 * are in that state (r = 1 for a positive spin). */
double or_step_cost_eq3(const or_model *m, const double *obs, const double *obs_gt);

/* Batched step over K environments (OpenMP over environments).
 * u_prev/u: [D].  cont [K][C_max], diag [K], obs [K][L][4] may be NULL. */
void or_batch_step(const or_model *m, int K, const int32_t *env_type,
                   const double *u_prev, const double *u,
                   double *state, double *params, int32_t *wkey, double *wr,
                   or_contact *cont, or_diag *diag, double *obs);

/* cost_sum[i] += step cost of obs[i] against obs_gt[group(i)] for K envs in
 * G contiguous groups (group_start[G+1]). */
void or_batch_cost(const or_model *m, int K, int G, const int32_t *group_start,
                   const double *obs, const double *obs_gt, double *cost_sum);

/* Lowest index of the minimum over n values (NaN counts as +inf). */
int or_argmin(int n, const double *v);

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

typedef struct {
    double elite_frac, sigma_mu, sigma_m, sigma_f, mu_lo, mu_hi, m_lo, m_hi;
    uint64_t seed;
} or_resample_cfg;

/* Population-based resampling (Sec. III-D.3) of K envs in G contiguous groups.
 * parent[K] receives -1 for kept elites, else the source env index.
 * cost_sum is zeroed on exit. */
void or_resample_pbo(const or_model *m, const or_resample_cfg *rc, int K, int G,
                     const int32_t *group_start, uint32_t window_idx,
                     double *cost_sum, double *state, double *params,
                     int32_t *wkey, double *wr, int32_t *parent);

/* Resampling with replacement (Sec. III-D.1, III-D.2): env j becomes a copy
 * of env parent[j] as it was before the call (state, params, warm-start
 * cache), then every env is explored: mu and m get N(0, sigma^2) noise
 * around the copied values (clamped to their ranges) and the perturbation
 * force is drawn from N(0, sigma_f^2 I), with the same Philox counters as the
 * population-based resampler.  cost_sum is zeroed. */
void or_resample_apply(const or_model *m, const or_resample_cfg *rc, int K, const int32_t *parent,
                       uint32_t window_idx, double *cost_sum, double *state, double *params,
                       int32_t *wkey, double *wr);

/* ADD (Sec. IV): mean distance of the object's sphere centres between pose a
 * and pose b (each x(3), q(4)). */
double or_add(const or_model *m, int type, const double *pose_a, const double *pose_b);

/* Window cost of a single environment over T steps (force cost, cost_mode
 * 0, the one the adjoint differentiates): sum of step costs
 * against obs_gt[T][L][4]; u_seq[T+1][D] with u_seq[0] the command before
 * the window.  Inputs are not modified. */
double or_window_cost(const or_model *m, int type, const double *st0, const double *pr0,
                      const int32_t *wkey0, const double *wr0, int T,
                      const double *u_seq, const double *obs_gt);

/* OpenMP threads the batched calls use, and a way to set them (timing). */
int or_max_threads(void);
void or_set_threads(int n);

/* Distance field of object type `type` at object-frame point p (value
 * returned, gradient into g[3]); collision_mode 1 only. */
double or_sdf_eval(const or_model *m, int type, const double *p, double *g);

#endif
