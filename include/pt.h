/*
 * pt.h -- C ABI of libpt, the MI355X (gfx950) library for the data-parallel
 * hot path of sample-based in-hand object pose tracking (Liang et al.,
 * arXiv 2002.12160).
 *
 * The method (Sec. III-B, Alg. 1): K simulations of a robot hand and an
 * object, initialised around a pose estimate with perturbed poses and
 * physics parameters, are stepped in lockstep with the real robot's joint
 * command u_t (s_{t+1} = f(s_t, u_t, theta), Sec. III-A); each simulation's
 * contact-sensor observation is compared with the observed one by a cost
 * (Eq. 3); costs are averaged over a window of T steps (Eq. 1) whose argmin
 * is the pose estimate (Eq. 2); every T steps a sample-based optimiser
 * resamples the population (Sec. III-D).
 *
 * World model (the paper leaves its simulator's internals open; this is the
 * reading implemented here and by the test oracle): a kinematic hand of L
 * capsule links driven by u_t, an object of spheres resting on a table plane
 * z = 0, speculative contacts kept when the signed gap d < margin and capped
 * at the C_max smallest (d, key) with key = k*(L+1)+l (l == L: the table),
 * Baumgarte depenetration erp*d/dt, a compliant Delassus operator
 * W = J M^-1 J^T + compliance*I and Coulomb friction written as a
 * second-order-cone complementarity problem, solved by exactly newton_iters
 * iterations of a smoothed Fischer-Burmeister Newton method (smoothing
 * fb_delta, impulse scale kappa) with Armijo backtracking over
 * alpha in {1, 1/2, 1/4, 1/8} (sigma = armijo_sigma, 1/8 if none passes),
 * warm-started from the previous step's impulses of the same keys; then
 * semi-implicit Euler with a quaternion exponential update and a remap of
 * the angular velocity that conserves world angular momentum.
 *
 * Conventions
 *   - Every buffer argument is a DEVICE pointer to caller-owned contiguous
 *     float32/int32 memory (torch tensors) unless stated "host".
 *   - Every call is asynchronous on the given HIP stream; nothing here
 *     synchronises the device except pt_read_stats and pt_autotune.
 *   - Device memory is allocated only by pt_create_batch (scene tables and
 *     the library's scratch: hand segments, contact buffer, counters, the
 *     autotuner's copies, gradient checkpoints for the elites, refinement
 *     buffers) and freed by pt_destroy_batch; no other call allocates.
 *   - Return value: PT_OK (0) or an error code; pt_last_error() returns a
 *     thread-local message for the last failing call on that thread.
 *     Argument and shape errors are detected before any launch.  Kernel
 *     faults surface as PT_E_HIP at a later call or at stream sync.
 *   - A simulation whose state becomes non-finite is not an error: its cost
 *     becomes NaN, which ranks as +inf in the argmin and the resampler (the
 *     paper's divergent samples, Sec. III-E), so it is replaced at the next
 *     resampling.  Contacts beyond C_max are dropped (counted in stats).
 *   - One host thread per batch at a time.
 *
 * Layouts (SoA, environment index fastest where it is per-environment):
 *   state  [13][K]    x(3), q(4: w,x,y,z), v(3), omega(3), world frame
 *   params [5][K]     mass, mu, f_pert(3) (f_pert acts for one step, then 0)
 *   warm   [K][C_max][4]  key (int32 bits, -1 = empty), r(3) in (n,t1,t2)
 *   obs    [4][L][K]  |c_l|, c_hat_l(3): force on sensor link l by the object
 *   obs_gt [4][L][G]  observed force per group (the layout pt_observe gives
 *                     for the batch of the G observed simulations)
 *   hand   [L][20]    host: parent, joint0, joint1, axis0(3), axis1(3),
 *                     offset(3), offset quaternion(4), length, radius, 2 spare
 */
#ifndef PT_H
#define PT_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define PT_API __attribute__((visibility("default")))
#else
#define PT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pt_batch_s *pt_batch;
typedef void *pt_stream; /* a hipStream_t; NULL = the null stream */

typedef enum {
    PT_OK = 0,
    PT_E_ARG = 1,         /* invalid argument, shape or size                 */
    PT_E_HIP = 2,         /* a HIP runtime call failed                       */
    PT_E_STATE = 3,       /* call not valid in the batch's current state     */
    PT_E_CAPTURE = 4,     /* graph capture / instantiation failed            */
    PT_E_UNSUPPORTED = 5  /* size beyond the library's limits                */
} pt_status;

#define PT_HAND_STRIDE 20
#define PT_MAX_CMAX 64
#define PT_MAX_LINKS 62
#define PT_MAX_SPHERES 256

typedef struct {
    /* sizes */
    int32_t K;            /* simulations in this batch, >= 1                      */
    int32_t G;            /* contiguous groups (one observed env each), >= 1      */
    int32_t L;            /* capsule links = contact sensors, 1..PT_MAX_LINKS     */
    int32_t D;            /* joints, >= 0                                         */
    int32_t n_types;      /* object types, >= 1                                   */
    int32_t S_max;        /* row stride of the sphere table, 1..PT_MAX_SPHERES    */
    int32_t C_max;        /* contact cap per simulation, 1..PT_MAX_CMAX           */
    int32_t newton_iters; /* Newton iterations per step, 0..100                   */
    int32_t T;            /* optimiser window length (steps), >= 1                */
    int32_t solve_precision; /* contact-solve arithmetic: 64 (float64, 0 = default)
                                or 32 (float32); geometry is float32 either way  */
    /* model constants */
    float dt, gravity[3], margin, erp, compliance, kappa, fb_delta, armijo_sigma;
    float tau_contact, w_mag, w_dir;
    /* population-based resampling (Sec. III-D.3) */
    float elite_frac, sigma_mu, sigma_m, sigma_f, mu_lo, mu_hi, m_lo, m_hi;
    uint64_t seed;                 /* Philox4x32-10 key                          */
    /* scene tables: HOST pointers, copied to the device by pt_create_batch  */
    const float *hand;             /* [L][20]                                    */
    const float *spheres;          /* [n_types][S_max][4] body-frame centre, radius */
    const int32_t *n_spheres;      /* [n_types], each 1..S_max                   */
    const float *inv_inertia;      /* [n_types][3] principal 1/I per unit mass, >= 0
                                      (0: the body does not turn about that axis) */
    const int32_t *env_type;       /* [K] in [0, n_types)                        */
    const int32_t *group_start;    /* [G+1], 0 = g0 < ... < gG = K               */
    /* simulation state: DEVICE pointers, caller-owned, bound for the batch's life */
    float *state;                  /* [13][K]                                    */
    float *params;                 /* [5][K]                                     */
    float *warm;                   /* [K][C_max][4]                              */
    /* nonzero: pt_run_window records a checkpoint of every simulation before
       every step (body, kept contacts' keys and float64 impulses; K * T *
       (64 + 32 C_max) bytes, allocated by pt_create_batch), from which
       pt_refine_elites takes the elites' first gradient instead of replaying
       their window */
    int32_t window_checkpoints;
    /* observation and cost: 0 = contact-force terms, obs [4][L][K] rows |c|,
       c/|c|; 1 = the full cost of Eq. 3 (Sec. III-C) with the terms a
       kinematic hand does not make identically zero: contact-state
       agreement, force magnitude and angle, translational slip (agreement
       and direction in the sensor's surface frame) and rotational slip
       (agreement and direction), obs [7][L][K] rows |c|, c/|c|, d (2), rot.
       Mode 1 has no gradient: pt_window_grad and pt_refine_elites return
       PT_E_UNSUPPORTED. */
    int32_t cost_mode;
    float tau_slip;       /* translational slip threshold [m/s], mode 1       */
    float tau_spin;       /* rotational slip threshold [rad/s], mode 1        */
    float w_eq3[7];       /* w4 .. w10 of Eq. 3, mode 1                       */
    /* hand model: 0 = kinematic hand, its joints follow the commands (the
       world model above); 1 = PD-controlled hand (Sec. III-A: the state
       holds the joint angles of the articulated hand and the observation the
       measured angles; Sec. IV-A: the simulated hand is driven by PD gains).
       With 1, every simulation's joints (q, qdot) are state in hand_state;
       each link is a solid cylinder of mass link_mass (axial inertia
       m r^2 / 2, transverse m (3 r^2 + len^2) / 12 about its centre), the
       hand's gravity compensated and its velocity-product terms dropped, so
       M(q) = sum over links of m J_v^T J_v + J_w^T I_w J_w is its only
       inertia; the PD law is taken implicitly,
         (M + dt kd I + dt^2 kp I) qdot+ = M qdot + dt kp (u - q) + J_h^T r,
         q+ = q + dt qdot+,
       and the contact solve runs over the generalised velocity (v, omega,
       qdot) of size 6 + D, a contact on link l adding the columns
       -F G_l(p), G_l(p)[:, j] = axis_j x (p - origin_j) over the joints that
       move link l (the object's point relative to the link's point at p).
       The observation gains the D joint angles after the step: obs
       [4 L + D][K] (the [4][L][K] force rows, then q [D][K]); obs_gt
       [4 L + D][G]; the step cost adds w_q sum_j (q_j - q^gt_j)^2 (Eq. 3's
       joint-angle term).  Limits (PT_E_UNSUPPORTED): D <= 64; a joint
       drives one link; at most 8 joints move a link; the joints split into
       independent groups (joints moving a common link, closed transitively:
       a finger) of at most 6; solve_precision 64; cost_mode 0.  With 1,
       pt_step reads u (the PD targets) and ignores u_prev; pt_observe,
       pt_cost and pt_resample (which copies hand_state with the rest of a
       simulation) take the layouts above, and so do pt_run_window and
       pt_run_window_static (one wavefront per simulation's window);
       window_checkpoints, pt_autotune, the gradient, refinement and
       weighted-resampling calls return PT_E_UNSUPPORTED. */
    int32_t hand_mode;
    float kp;             /* joint stiffness [N m / rad], >= 0                */
    float kd;             /* joint damping [N m s / rad], >= 0; kp + kd > 0  */
    float link_mass;      /* mass of every link [kg], > 0                     */
    float w_q;            /* weight of the joint-angle term [1 / rad^2], >= 0 */
    float *hand_state;    /* [2 D][K] q (D rows) then qdot (D rows), DEVICE,
                             caller-owned, used in place (hand_mode 1)       */
    /* link-object collision (Sec. IV-A simplifies the objects' collision
       geometry; here it may be a signed distance field): 0 = the sphere
       set; 1 = the object's signed distance field phi (negative inside),
       node values on a cubic grid in the object frame interpolated
       trilinearly (outside the grid: the value at the nearest grid point plus
       the distance to it), queried at link_samples points a + t (b - a),
       t = m / (link_samples - 1) (the middle for one sample), along each
       link's axis: sample m of link l is a contact candidate with key
       m*(L+1)+l and gap phi - radius_l, normal minus the world unit gradient
       of phi, contact point the sample moved by -phi along that gradient.
       Object-table contacts stay with the sphere set.  Limits
       (PT_E_UNSUPPORTED): L x link_samples + S_max <= 1536;
       solve_precision 64; cost_mode 0; the gradient and refinement calls
       return PT_E_UNSUPPORTED.  Both hand modes (the windowed calls with
       the kinematic hand only, as for the sphere set). */
    int32_t collision_mode;
    int32_t link_samples; /* 1..64                                             */
    int32_t sdf_n;        /* grid nodes per axis, 2..128                       */
    const float *sdf;     /* HOST [n_types][sdf_n][sdf_n][sdf_n] node values,
                             x fastest (index (k sdf_n + j) sdf_n + i for the
                             node origin + spacing (i, j, k)), copied        */
    const float *sdf_box; /* HOST [n_types][4] grid origin (object frame, 3)
                             and node spacing (> 0), copied                  */
} pt_batch_desc;

/* Creates a batch: validates the descriptor (PT_E_ARG / PT_E_UNSUPPORTED),
 * copies the scene tables to the device and allocates internal scratch
 * (hand segments, a contact buffer [K][C_max][4], counters).  The caller's
 * state/params/warm buffers are used in place and must outlive the batch.
 * On success *out receives the handle. */
PT_API pt_status pt_create_batch(const pt_batch_desc *desc, pt_batch *out);

/* Frees everything pt_create_batch allocated (after synchronising the
 * device); the caller's buffers are untouched.  NULL is accepted. */
PT_API pt_status pt_destroy_batch(pt_batch b);

/* One world step of all K simulations, every one with the same command
 * (Alg. 1, inner loop).  u_prev, u: device [D] joint commands
 * of the previous and the current step (the hand moves from FK(u_prev) to
 * FK(u) during the step; pass u_prev == u for the first step).  Updates
 * state, params (f_pert consumed) and warm in place and keeps the solved
 * contacts for pt_observe.  With the float64 solve and K at least eight per
 * compute unit, the step's hand kinematics run once, in a launch of their
 * own on s ahead of the step's; otherwise every simulation's wavefront
 * evaluates them (the same bits either way). */
PT_API pt_status pt_step(pt_batch b, const float *u_prev, const float *u, pt_stream s);

/* Per-sensor observation of the last pt_step (Sec. III-A: the force vector
 * of each contact sensor): obs[4][L][K] = (|c_l|, c_l/|c_l|) with
 * c_l = -(1/dt) sum over contacts on link l of the impulse on the object,
 * the direction set to 0 when |c_l| <= tau_contact.  Table contacts are not
 * sensed. */
PT_API pt_status pt_observe(pt_batch b, float *obs, pt_stream s);

/* Step cost (Eq. 3, here the force-magnitude and force-direction terms):
 * cost_sum[i] += sum_l w_mag (|c_l| - |c^gt_l|)^2 + w_dir |c_hat_l - c_hat^gt_l|^2
 * against obs_gt[.][l][g(i)] of its group g(i), then best[g] = argmin of cost_sum over group g
 * (Eq. 2; ties -> lowest index, NaN ranks as +inf).  best may be NULL. */
PT_API pt_status pt_cost(pt_batch b, const float *obs, const float *obs_gt, float *cost_sum, int32_t *best,
                  pt_stream s);

/* Population-based optimiser (PBO, Sec. III-D.3), per group: rank by
 * (cost_sum, index) with NaN as +inf; the K_best = max(1, floor(K_g *
 * elite_frac)) lowest are kept unchanged (parent = -1); every other
 * simulation j copies the state, params and warm cache of the elite of rank
 * floor(w0 * K_best / 2^32), w = Philox4x32-10(key = seed, counter =
 * (j, window_idx, 0, 0)), then explores: mu and mass get Gaussian noise
 * (sigma_mu, sigma_m; clamped to [mu_lo, mu_hi], [m_lo, m_hi]) and f_pert a
 * Gaussian force (sigma_f per axis; Sec. III-D: perturbation forces), the
 * normals drawn by Box-Muller from counters (j, window_idx, 1, 0) and
 * (j, window_idx, 2, 0).  cost_sum is zeroed.  parent [K] may be NULL. */
PT_API pt_status pt_resample(pt_batch b, float *cost_sum, uint32_t window_idx, int32_t *parent, pt_stream s);

/* Weighted resampling, WRS (Sec. III-D.1, Eq. 4), per group: with the
 * window-mean costs C_i = cost_sum[i] / n_steps, P(i) is proportional to
 * exp(-lambda (C_i - min_j C_j)) over the finite costs (a NaN or infinite
 * cost gets P = 0; a group without a finite cost draws uniformly).  Every
 * simulation j then draws its parent with replacement: the first index of
 * the group whose running sum of P exceeds u = (w0 + 1/2) 2^-32 of the
 * total, w = Philox4x32-10(key = seed, counter = (j, window_idx, 3, 0)), and
 * becomes a copy of that parent as it was before the call (state, params,
 * warm cache); every simulation is then explored as pt_resample explores a
 * copy (same counters).  cost_sum is zeroed.  parent [K] (required)
 * receives the drawn index; weights [K] (may be NULL) the group's P.
 * lambda: finite, >= 0 (0 draws uniformly); n_steps >= 1.  The copies go
 * through a snapshot buffer owned by the batch: no allocation. */
PT_API pt_status pt_resample_wrs(pt_batch b, float *cost_sum, int32_t n_steps, uint32_t window_idx, float lambda,
                                 int32_t *parent, float *weights, pt_stream s);

/* Relative Entropy Policy Search, REPS (Sec. III-D.2, Eqs. 5-6), per group:
 * rewards R_i = max_j C_j + min_j C_j - C_i over the finite window-mean
 * costs, eta* = argmin over eta > 0 of eta epsilon + eta log((1/K_f) sum_i
 * exp(R_i / eta)) (K_f finite costs), P(i) = softmax(R_i / eta*); then the
 * draw, copies and exploration of pt_resample_wrs.  eta* is found where the
 * dual's slope epsilon - KL(P_eta || uniform) vanishes, by bisection on
 * log(eta) to ~1e-13; when all finite costs are equal P is uniform over
 * them, and with no finite cost uniform over the group (eta* reported as
 * +inf in both cases); when epsilon >= log(K_f / #argmin) the
 * dual has no interior minimum and P is the eta -> 0+ limit, uniform over
 * the lowest costs (eta* reported as 0).  eta [G] and weights [K] may be
 * NULL.  epsilon: finite, > 0. */
PT_API pt_status pt_resample_reps(pt_batch b, float *cost_sum, int32_t n_steps, uint32_t window_idx, float epsilon,
                                  int32_t *parent, float *weights, float *eta, pt_stream s);

/* Batched execution of one optimiser window: T steps of every simulation
 * with the per-step observation and cost fused, in one persistent kernel
 * (environments pulled from a work queue, state kept on chip for all T
 * steps), replayed from a captured HIP graph when graph != 0.
 *   u_win      [T+1][D]   u_win[0] is the command before the window
 *   obs_gt_win [T][4][L][G]
 *   cost_sum   [K]        accumulated (not reset)
 *   best       [G]        argmin of cost_sum after the window (may be NULL)
 *   obs_out    [T][4][L][K] or NULL
 * Equivalent to T rounds of pt_step/pt_observe/pt_cost.
 * With the PD hand (hand_mode 1) the kinematics depend on each simulation's
 * joint angles: up to one simulation per SIMD (K <= 4 x compute units) one
 * wavefront runs each simulation's whole window; beyond, the call enqueues
 * the per-step kernels of the T steps (which fit two wavefronts per SIMD),
 * staging contacts and observations in buffers the batch allocated at
 * creation.  The rows are those of pt_observe and pt_cost for that hand,
 * obs_gt_win [T][4L + D][G] and obs_out [T][4L + D][K]; the joint state
 * advances in hand_state; the results are those of T rounds of
 * pt_step/pt_observe/pt_cost bit for bit either way. */
PT_API pt_status pt_run_window(pt_batch b, const float *u_win, const float *obs_gt_win, float *cost_sum,
                        int32_t *best, float *obs_out, int32_t graph, pt_stream s);

/* pt_run_window without allocation or graph capture, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  Runs the same kernels as pt_run_window
 * with graph == 0 and gives the same results bit for bit; the window's
 * scratch (the work-queue counters and the T x L hand segment records) lives
 * in a static device array of 256 KiB that every GPU the library runs on
 * holds until the process ends, instead of in the batch.  The array's
 * address on a device is resolved when the first batch is created on it.
 * Limits: T x L <= 4096 (PT_E_UNSUPPORTED beyond, before any launch).  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from different host threads) race and must not be
 * issued; calls in one stream are ordered and safe.  The counters are
 * cleared by a kernel at the start of every call (the PD hand's window
 * uses none of the array, only the batch's own buffers).  Arguments, layouts
 * and errors as pt_run_window. */
PT_API pt_status pt_run_window_static(pt_batch b, const float *u_win, const float *obs_gt_win, float *cost_sum,
                                      int32_t *best, float *obs_out, pt_stream s);

/* Chooses the persistent kernel's environments per workgroup (waves per
 * workgroup, {1,2,4,8}; at most 4 with the float64 solve) by timing windows
 * on scratch copies of the state; the widest choice is kept unless a
 * narrower one is at least 2% faster (fuller workgroups leave compute units
 * free for work on other streams).  The batch's own buffers are not
 * modified.  Synchronises the stream.  result (host, may be NULL) receives
 * the chosen value.  PT_E_UNSUPPORTED with the PD hand (its window has one
 * simulation per wavefront, nothing to choose). */
PT_API pt_status pt_autotune(pt_batch b, const float *u_win, const float *obs_gt_win, int32_t *result, pt_stream s);

/* Sets the persistent kernel's environments per workgroup (1, 2, 4 or 8)
 * by hand instead of through pt_autotune.  PT_E_UNSUPPORTED if that many
 * simulations' LDS does not fit in one workgroup, or above 4 with the
 * float64 solve. */
PT_API pt_status pt_set_tuning(pt_batch b, int32_t waves_per_workgroup);

/* Gradient of the window cost of n listed simulations with respect to their
 * window start.  The window cost is the sum over the window's T steps of the
 * step cost of pt_cost (Eq. 3 terms, accumulated as in Eq. 1 and Alg. 1).
 * The paper's optimisers are derivative-free (Sec. III-D); this gradient
 * serves pt_refine_elites.  Each simulation runs the window from the given
 * start exactly as pt_run_window does (the same bits for the same start),
 * writing a checkpoint of its body and warm cache before every step; the
 * reverse sweep re-runs each step from its checkpoint and propagates the
 * adjoint through the cost, the observation, the integration and the
 * contact solve.  The contact solve is differentiated implicitly: the
 * computed impulses are taken as the root of the smoothed Fischer-Burmeister
 * system, and its transposed Newton matrix is solved through the same 6x6
 * Schur reduction as the forward solve.  The contact set, the cap and the
 * branch choices of each step (tangent axis, clamps, depenetration) are held
 * fixed: the result is the gradient of the smooth piece of the window map
 * that contains the start.
 *   u_win      [T+1][D]       as in pt_run_window
 *   obs_gt_win [T][4][L][G]   as in pt_run_window
 *   n          >= 0 simulations listed
 *   env        [n] int32      batch index of each (gives its object type and
 *                             group); an index outside [0, K) yields cost NaN
 *                             and a zero gradient
 *   start      [18][n]        x(3) q(4) v(3) omega(3) mass mu f_pert(3)
 *   warm0      [n][C_max][4]  warm cache at the window start
 *   cost       [n]            out: window cost
 *   grad       [18][n]        out: d cost / d start (rows as start), or NULL
 *                             for the cost alone (no checkpoints, no reverse
 *                             sweep); the q rows are the gradient through the
 *                             normalisation of q (orthogonal to q)
 *   end_state  [13][n]        out: state after the window, or NULL
 *   end_warm   [n][C_max][4]  out: warm cache after the window, or NULL
 *   resid      [n]            out: the largest final merit |Phi|^2 / 2 of the
 *                             window's contact solves (0 for a step without
 *                             contacts), or NULL.  The gradient is exact for
 *                             the window map the forward sweep computes only
 *                             where these solves have converged: with a fixed
 *                             newton_iters a solve can stop short of the root
 *                             the reverse sweep assumes, and the gradient is
 *                             then that of the converged map at this start
 * The batch's own state, params and warm cache are neither read nor written.
 * The checkpoints (per simulation and step the body and the contacts' keys
 * and float64 impulses, 64 + 32 C_max bytes) live in a buffer the batch owns,
 * sized for pt_elite_count(b) simulations; longer lists run in chunks of that
 * many.  The buffer is shared between calls: calls on different streams must
 * not overlap. */
PT_API pt_status pt_window_grad(pt_batch b, const float *u_win, const float *obs_gt_win, int32_t n,
                                const int32_t *env, const float *start, const float *warm0, float *cost,
                                float *grad, float *end_state, float *end_warm, float *resid, pt_stream s);

/* Elite refinement by the window-cost gradient, run between pt_run_window
 * and pt_resample.  The elites of each group, ranked from cost_sum as
 * pt_resample ranks them, take `steps` scaled gradient steps from their
 * window start: delta = -rho (s o s o g) / |s o g| over (x, q, v, omega,
 * mass, mu), rho starting at `step`; a trial is kept when its replayed window
 * cost is lower than the current one, otherwise rho is halved; q is
 * renormalised, mass and mu are clamped to [m_lo, m_hi] and [mu_lo, mu_hi],
 * and f_pert is kept.  For each elite whose start changed, the batch's
 * state, params (f_pert 0) and warm cache become the end of the kept replay
 * and cost_sum its window cost; costs only decrease, so pt_resample keeps
 * the same elites.
 *   cost_sum       [K]   window costs from the pt_run_window just done
 *   start_state [13][K], start_params [5][K], start_warm [K][C_max][4]:
 *                        copies of the batch's buffers taken before it
 *   steps          >= 0 gradient steps; step > 0
 *   scale          host [15], or NULL for (1 mm x3, 0.01 x4, 1 cm/s x3,
 *                  0.1 rad/s x3, 5 g, 0.02)
 *   best           [G] argmin of cost_sum per group afterwards, or NULL
 *   elite_out      [pt_elite_count(b)] int32 batch index of each elite
 *                  (groups in order, by rank within a group), or NULL
 * The elites' starts, gradients and checkpoints use buffers the batch holds
 * from pt_create_batch on; calls on different streams must not overlap.
 * From 16 elites per compute unit on, the elites run in two parts, the second
 * on a stream the batch owns, forked from `s` and joined back to it with
 * events: the call is ordered on `s` as a whole (and can be captured there),
 * and its results are those of one launch over all elites. */
PT_API pt_status pt_refine_elites(pt_batch b, const float *u_win, const float *obs_gt_win, float *cost_sum,
                                  const float *start_state, const float *start_params, const float *start_warm,
                                  int32_t steps, float step, const float *scale, int32_t *best, int32_t *elite_out,
                                  pt_stream s);

/* Number of elites over all groups, sum over g of max(1, floor(K_g *
 * elite_frac)); -1 for a NULL batch. */
PT_API int32_t pt_elite_count(pt_batch b);

/* Reads the batch's cumulative counters (host out[4]): environment-steps,
 * narrow-phase candidates (d < margin), contacts solved, contacts dropped by
 * the cap.  Synchronises the stream. */
PT_API pt_status pt_read_stats(pt_batch b, int64_t *out, pt_stream s);

/* Message of the last failing call on this thread ("" if none). */
PT_API const char *pt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PT_H */
