// pt_api.hip -- host side of libpt: the C ABI declared in include/pt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pt.h"
#include "pt_internal.h"
#include "pt_pd.hpp"

using pt::Consts;
using pt::Tables;

namespace {

thread_local std::string g_err;

pt_status fail(pt_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
pt_status fail(pt_status code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(PT_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

struct GraphKey {
    const void *p[5];
    int wpb;
    bool operator==(const GraphKey &o) const
    {
        for (int i = 0; i < 5; ++i)
            if (p[i] != o.p[i]) return false;
        return wpb == o.wpb;
    }
};

// Scratch of pt_run_window_static, for callers that cannot allocate: the
// window's work-queue counters (the first 256 bytes) and its hand segment
// records, T x L of them at most.  Every GPU the library runs on holds its
// own copy until the process ends; host code never uses the array's name
// as an address, only the per-device address hipGetSymbolAddress returns.
constexpr size_t STATIC_COUNTER_INTS = 64;
constexpr size_t STATIC_SEG_RECORDS = 4096;
constexpr size_t STATIC_SCRATCH_FLOATS = STATIC_COUNTER_INTS + STATIC_SEG_RECORDS * pt::SEG_STRIDE;
static __device__ __align__(256) float scratch[STATIC_SCRATCH_FLOATS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// the scratch array's address on `device` (current), resolved once per device
hipError_t static_scratch(int device, void **out)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// n int32 words set to v (a kernel, so that a captured stream records no
// memset node)
__global__ void k_fill_i32(int32_t *p, int n, int32_t v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

struct pt_batch_s {
    Consts P;
    pt::ResampleArgs R;
    int n_types;
    int device;
    int num_cu;
    // device tables
    float *d_hand = nullptr, *d_spheres = nullptr, *d_inv = nullptr;
    int32_t *d_nsph = nullptr, *d_type = nullptr, *d_group_of = nullptr, *d_group_start = nullptr;
    int32_t *d_order = nullptr, *d_queue = nullptr;
    int64_t *d_stats = nullptr;
    // scratch
    float *d_seg_win = nullptr;  // [T][L][16]
    float *d_contacts = nullptr; // [K][C_max][4]
    float *d_seg_grad = nullptr; // [T][L][16] for the gradient and refinement calls
    float *d_tune = nullptr;     // autotuner's copies of state, params, warm cache and costs
    // gradient checkpoints (for n_elite simulations at a time) and refinement buffers
    float *d_ckpt = nullptr;
    float *d_wckpt = nullptr;    // per-step checkpoints of every simulation's window (window_checkpoints)
    float *d_cslip = nullptr;    // [K][C_max][8] per-contact slip data of the last step (cost_mode 1)
    float *d_seg = nullptr;      // [L][16] the last step's hand segments (kinematic hand)
    int n_elite = 0;
    int32_t *d_elite = nullptr;  // [n_elite]
    float *d_ref = nullptr;      // see refine_layout
    float *d_snap = nullptr;     // [18][K] + [K][C_max][4]: parents' copies for the weighted resamplers
    void *static_scratch = nullptr; // this device's pt_run_window_static scratch (not owned)
    // the PD-controlled hand (hand_mode 1)
    int hand_mode = 0;
    pt::PdConsts Q = {};
    int32_t *d_pd = nullptr;     // the hand's structure table (pt::PdTab)
    int32_t *d_parent = nullptr; // [K] parents of a resampling, for the joint state's copies
    float *d_pd_obs = nullptr;   // [4L + D][K] a step's observation inside a window of per-step kernels
    float *hstate = nullptr;     // caller-owned [2D][K]
    // the objects' distance fields (collision_mode 1)
    float *d_sdf = nullptr, *d_sdf_box = nullptr;
    // caller-owned state
    float *state, *params, *warm;
    // host copies
    std::vector<int32_t> group_start;
    int max_group = 0;
    // batched-path configuration
    int wpb = 4;
    int step_wpb = 4;
    bool step_fk_once = false;   // pt_step: hand kinematics in a launch of their own
    hipStream_t capture_stream = nullptr;
    // parts 1.. of the elite refinement run on these streams, forked from
    // and joined back to the caller's stream by the events
    static constexpr int REFINE_PARTS = 2;
    hipStream_t side_stream[REFINE_PARTS - 1] = {};
    hipEvent_t ev_fork = nullptr, ev_join[REFINE_PARTS - 1] = {};
    // captured windows, keyed by their buffers (a driver that double-buffers
    // its inputs alternates between a few); least recently used is evicted
    static constexpr int N_GRAPHS = 4;
    hipGraphExec_t graph_exec[N_GRAPHS] = {};
    GraphKey graph_key[N_GRAPHS] = {};
    uint64_t graph_used[N_GRAPHS] = {};
    uint64_t graph_clock = 0;
    void drop_graphs()
    {
        for (int i = 0; i < N_GRAPHS; ++i)
            if (graph_exec[i]) {
                (void)hipGraphExecDestroy(graph_exec[i]);
                graph_exec[i] = nullptr;
            }
    }
};

namespace {

pt_status validate(const pt_batch_desc *d)
{
    if (!d) return fail(PT_E_ARG, "desc is NULL");
    if (d->K < 1) return fail(PT_E_ARG, "K must be >= 1 (got %d)", d->K);
    if (d->G < 1 || d->G > d->K) return fail(PT_E_ARG, "G must be in [1, K] (got %d)", d->G);
    if (d->L < 1 || d->L > PT_MAX_LINKS) return fail(PT_E_UNSUPPORTED, "L must be in [1, %d] (got %d)", PT_MAX_LINKS, d->L);
    if (d->D < 0) return fail(PT_E_ARG, "D must be >= 0");
    if (d->n_types < 1) return fail(PT_E_ARG, "n_types must be >= 1");
    if (d->S_max < 1 || d->S_max > PT_MAX_SPHERES)
        return fail(PT_E_UNSUPPORTED, "S_max must be in [1, %d] (got %d)", PT_MAX_SPHERES, d->S_max);
    if (d->C_max < 1 || d->C_max > PT_MAX_CMAX)
        return fail(PT_E_UNSUPPORTED, "C_max must be in [1, %d] (got %d)", PT_MAX_CMAX, d->C_max);
    if (d->newton_iters < 0 || d->newton_iters > 100) return fail(PT_E_ARG, "newton_iters must be in [0, 100]");
    if (d->T < 1) return fail(PT_E_ARG, "T must be >= 1");
    if (d->solve_precision != 0 && d->solve_precision != 32 && d->solve_precision != 64)
        return fail(PT_E_ARG, "solve_precision must be 32 or 64 (or 0 for the default, 64)");
    if (!(d->dt > 0.f) || !std::isfinite(d->dt)) return fail(PT_E_ARG, "dt must be positive and finite");
    if (!(d->kappa > 0.f) || !(d->fb_delta > 0.f)) return fail(PT_E_ARG, "kappa and fb_delta must be positive");
    if (d->cost_mode != 0 && d->cost_mode != 1) return fail(PT_E_ARG, "cost_mode must be 0 or 1 (got %d)", d->cost_mode);
    if (d->cost_mode == 1) {
        if (!(d->tau_slip >= 0.f) || !std::isfinite(d->tau_slip) || !(d->tau_spin >= 0.f) ||
            !std::isfinite(d->tau_spin))
            return fail(PT_E_ARG, "tau_slip and tau_spin must be finite and >= 0");
        for (int i = 0; i < 7; ++i)
            if (!std::isfinite(d->w_eq3[i])) return fail(PT_E_ARG, "w_eq3[%d] is not finite", i);
    }
    if (!(d->compliance >= 0.f)) return fail(PT_E_ARG, "compliance must be >= 0");
    if (!(d->elite_frac > 0.f && d->elite_frac <= 1.f)) return fail(PT_E_ARG, "elite_frac must be in (0, 1]");
    if (!(d->mu_lo <= d->mu_hi) || !(d->m_lo <= d->m_hi) || !(d->m_lo > 0.f))
        return fail(PT_E_ARG, "invalid parameter clamp ranges");
    if (!d->hand || !d->spheres || !d->n_spheres || !d->inv_inertia || !d->env_type || !d->group_start)
        return fail(PT_E_ARG, "scene table pointer is NULL");
    if (!d->state || !d->params || !d->warm) return fail(PT_E_ARG, "state/params/warm pointer is NULL");
    if (d->hand_mode != 0 && d->hand_mode != 1) return fail(PT_E_ARG, "hand_mode must be 0 or 1 (got %d)", d->hand_mode);
    if (d->hand_mode == 1) {
        if (d->D > pt::PD_MAX_D) return fail(PT_E_UNSUPPORTED, "the PD hand has at most %d joints (got %d)", pt::PD_MAX_D, d->D);
        if (d->solve_precision == 32) return fail(PT_E_UNSUPPORTED, "the PD hand's solve is float64 only");
        if (d->cost_mode != 0) return fail(PT_E_UNSUPPORTED, "the PD hand supports cost_mode 0 only");
        if (!(d->kp >= 0.f) || !(d->kd >= 0.f) || !std::isfinite(d->kp) || !std::isfinite(d->kd) ||
            !(d->kp + d->kd > 0.f))
            return fail(PT_E_ARG, "kp and kd must be finite, >= 0 and not both 0");
        if (!(d->link_mass > 0.f) || !std::isfinite(d->link_mass)) return fail(PT_E_ARG, "link_mass must be positive and finite");
        if (!(d->w_q >= 0.f) || !std::isfinite(d->w_q)) return fail(PT_E_ARG, "w_q must be finite and >= 0");
        if (d->D > 0 && !d->hand_state) return fail(PT_E_ARG, "hand_state is NULL");
        if (d->window_checkpoints)
            return fail(PT_E_UNSUPPORTED, "the PD hand has no window gradient, so no window checkpoints");
    }
    if (d->collision_mode != 0 && d->collision_mode != 1)
        return fail(PT_E_ARG, "collision_mode must be 0 or 1 (got %d)", d->collision_mode);
    if (d->collision_mode == 1) {
        if (d->link_samples < 1 || d->link_samples > 64) return fail(PT_E_ARG, "link_samples must be in [1, 64]");
        if (d->sdf_n < 2 || d->sdf_n > 128) return fail(PT_E_UNSUPPORTED, "sdf_n must be in [2, 128] (got %d)", d->sdf_n);
        if (!d->sdf || !d->sdf_box) return fail(PT_E_ARG, "sdf/sdf_box is NULL");
        if (d->solve_precision == 32) return fail(PT_E_UNSUPPORTED, "the distance-field path solves in float64 only");
        if (d->cost_mode != 0) return fail(PT_E_UNSUPPORTED, "the distance-field path supports cost_mode 0 only");
        if (d->L * d->link_samples + d->S_max > pt::CAND_CAP)
            return fail(PT_E_UNSUPPORTED, "L x link_samples + S_max = %d exceeds %d candidates",
                        d->L * d->link_samples + d->S_max, pt::CAND_CAP);
        for (int t = 0; t < d->n_types; ++t) {
            const float *bx = d->sdf_box + 4 * t;
            if (!std::isfinite(bx[0]) || !std::isfinite(bx[1]) || !std::isfinite(bx[2]) || !(bx[3] > 0.f) ||
                !std::isfinite(bx[3]))
                return fail(PT_E_ARG, "sdf_box[%d]: origin must be finite and spacing positive", t);
        }
        const size_t nv = (size_t)d->n_types * d->sdf_n * d->sdf_n * d->sdf_n;
        for (size_t i = 0; i < nv; ++i)
            if (!std::isfinite(d->sdf[i])) return fail(PT_E_ARG, "sdf value %zu is not finite", i);
    }
    for (int l = 0; l < d->L; ++l) {
        const float *h = d->hand + (size_t)l * PT_HAND_STRIDE;
        int parent = (int)h[0], j0 = (int)h[1], j1 = (int)h[2];
        if (parent < -1 || parent >= l) return fail(PT_E_ARG, "link %d: parent %d must be -1 or a lower index", l, parent);
        if (j0 < -1 || j0 >= d->D || j1 < -1 || j1 >= d->D) return fail(PT_E_ARG, "link %d: joint index out of range", l);
        if (!(h[16] >= 0.f) || !(h[17] >= 0.f)) return fail(PT_E_ARG, "link %d: negative length or radius", l);
    }
    for (int t = 0; t < d->n_types; ++t)
        if (d->n_spheres[t] < 1 || d->n_spheres[t] > d->S_max)
            return fail(PT_E_ARG, "n_spheres[%d] = %d must be in [1, S_max]", t, d->n_spheres[t]);
    for (int t = 0; t < d->n_types; ++t)
        for (int a = 0; a < 3; ++a) {
            const float v = d->inv_inertia[3 * t + a];
            if (!(v >= 0.f) || !std::isfinite(v))
                return fail(PT_E_ARG, "inv_inertia[%d][%d] must be finite and >= 0", t, a);
        }
    for (int i = 0; i < d->K; ++i)
        if (d->env_type[i] < 0 || d->env_type[i] >= d->n_types) return fail(PT_E_ARG, "env_type[%d] out of range", i);
    if (d->group_start[0] != 0 || d->group_start[d->G] != d->K)
        return fail(PT_E_ARG, "group_start must begin at 0 and end at K");
    for (int g = 0; g < d->G; ++g)
        if (d->group_start[g + 1] <= d->group_start[g]) return fail(PT_E_ARG, "groups must be non-empty and increasing");
    return PT_OK;
}

// The PD hand's structure table (layout: pt::PdTab).  Joints that move a
// common link are joined (transitively) into a group; groups are numbered
// by their lowest joint and hold their joints in increasing order, which
// gives every joint its position.  Every joint drives at most one link.
pt_status build_pd_table(const pt_batch_desc *d, std::vector<int32_t> &tab, int &groups, int &dmax, int &gmax)
{
    const int L = d->L, D = d->D;
    std::vector<std::vector<int>> chain(L);
    std::vector<int> owner(D, -1), depth(L, 0), uf(D);
    for (int j = 0; j < D; ++j) uf[j] = j;
    auto find = [&](int j) {
        while (uf[j] != j) j = uf[j] = uf[uf[j]];
        return j;
    };
    dmax = 0;
    for (int l = 0; l < L; ++l) {
        const float *h = d->hand + (size_t)l * PT_HAND_STRIDE;
        const int parent = (int)h[0], js[2] = {(int)h[1], (int)h[2]};
        if (js[0] >= 0 && js[0] == js[1]) return fail(PT_E_UNSUPPORTED, "link %d: both joints are joint %d", l, js[0]);
        if (parent >= 0) {
            chain[l] = chain[parent];
            depth[l] = depth[parent] + 1;
        }
        dmax = std::max(dmax, depth[l]);
        for (int j : js) {
            if (j < 0) continue;
            if (owner[j] >= 0) return fail(PT_E_UNSUPPORTED, "joint %d drives links %d and %d", j, owner[j], l);
            owner[j] = l;
            chain[l].push_back(j);
        }
        if ((int)chain[l].size() > pt::PD_CHAIN)
            return fail(PT_E_UNSUPPORTED, "link %d is moved by %zu joints (at most %d)", l, chain[l].size(), pt::PD_CHAIN);
        for (int j : chain[l]) uf[find(j)] = find(chain[l][0]);
    }
    std::vector<int> group_of_root(D, -1);
    std::vector<std::vector<int>> members;
    for (int j = 0; j < D; ++j) {
        const int r = find(j);
        if (group_of_root[r] < 0) {
            group_of_root[r] = (int)members.size();
            members.emplace_back();
        }
        members[group_of_root[r]].push_back(j);
    }
    groups = (int)members.size();
    gmax = 0;
    for (const auto &m : members) gmax = std::max(gmax, (int)m.size());
    std::vector<int> jat, pos(D), gs(D), gn(D), gfirst;
    for (const auto &m : members) {
        if ((int)m.size() > pt::PD_GMAX)
            return fail(PT_E_UNSUPPORTED, "a group of %zu joints moves common links (at most %d)", m.size(), pt::PD_GMAX);
        gfirst.push_back((int)jat.size());
        for (int j : m) {
            pos[j] = (int)jat.size();
            gs[pos[j]] = gfirst.back();
            gn[pos[j]] = (int)m.size();
            jat.push_back(j);
        }
    }
    gfirst.push_back(D);
    std::vector<uint64_t> sub(D, 0);
    for (int l = 0; l < L; ++l)
        for (int j : chain[l]) sub[pos[j]] |= 1ull << l;
    tab.assign(pt::pd_tab_ints(L, D, groups), -1);
    for (int p = 0; p < D; ++p) {
        tab[p] = jat[p];
        tab[D + jat[p]] = p;
        tab[2 * D + p] = gs[p];
        tab[3 * D + p] = gn[p];
        tab[4 * D + p] = (int32_t)(uint32_t)(sub[p] & 0xffffffffu);
        tab[5 * D + p] = (int32_t)(uint32_t)(sub[p] >> 32);
    }
    for (int l = 0; l < L; ++l) {
        tab[6 * D + l] = depth[l];
        for (size_t i = 0; i < chain[l].size(); ++i) tab[6 * D + L + l * pt::PD_CHAIN + i] = pos[chain[l][i]];
    }
    for (int g = 0; g <= groups; ++g) tab[6 * D + L + L * pt::PD_CHAIN + g] = gfirst[g];
    return PT_OK;
}

int round_up(int a, int b) { return (a + b - 1) / b * b; }

// largest simulations-per-workgroup the step kernels are compiled for
int max_wpb(const Consts &P) { return P.solve_fp64 ? 4 : 8; }

}  // namespace

// refinement buffers of n elites, carved from one allocation (every block a
// multiple of 4 floats, so the warm caches stay 16-byte aligned)
struct RefineBufs {
    float *xi, *xi_try, *g, *cost, *cost_try, *rho, *end_state, *end_warm, *warm0;
    int32_t *flag;
};

static size_t pad4(size_t x) { return (x + 3) / 4 * 4; }

static size_t refine_floats(const Consts &P, int n)
{
    const size_t w = (size_t)n * P.C_max * 4;
    return 3 * pad4((size_t)pt::XI_ROWS * n) + 4 * pad4(n) + pad4(13 * (size_t)n) + 2 * w;
}

static RefineBufs refine_layout(float *base, const Consts &P, int n)
{
    RefineBufs r;
    const size_t x = pad4((size_t)pt::XI_ROWS * n), v = pad4(n), w = (size_t)n * P.C_max * 4;
    r.xi = base;
    r.xi_try = r.xi + x;
    r.g = r.xi_try + x;
    r.cost = r.g + x;
    r.cost_try = r.cost + v;
    r.rho = r.cost_try + v;
    r.flag = reinterpret_cast<int32_t *>(r.rho + v);
    r.end_state = r.rho + 2 * v;
    r.end_warm = r.end_state + pad4(13 * (size_t)n);
    r.warm0 = r.end_warm + w;
    return r;
}

// autotuner scratch: copies of state [13][K], params [5][K], warm cache
// [K][C_max][4] and costs [K]
static size_t tune_floats(const Consts &P)
{
    const size_t K = P.K;
    return 13 * K + 5 * K + K * P.C_max * 4 + K;
}

extern "C" {

const char *pt_last_error(void) { return g_err.c_str(); }

pt_status pt_create_batch(const pt_batch_desc *d, pt_batch *out)
{
    if (!out) return fail(PT_E_ARG, "out is NULL");
    *out = nullptr;
    pt_status st = validate(d);
    if (st != PT_OK) return st;
    // candidate list (every sphere-link pair up to pt::CAND_CAP entries -- a
    // step with more cuts its list to the C_max lowest and goes on -- plus 8
    // entries of padding for the cap's 16-byte reads); the same LDS holds,
    // once the cap has run, the rows of the solve's cross-contact sums
    // (rows of RedStride<double> = 44 doubles: one per contact slot for the
    // PD solve's per-link sums, at most 32 for the kinematic solve's sums,
    // which fold the upper half-wave's contacts onto the lower one's)
    const int red_rows = d->C_max <= 16 ? 16 : (d->C_max <= 32 || d->hand_mode == 0 ? 32 : 64);
    // the PD hand's structure
    std::vector<int32_t> pd_tab;
    int pd_groups = 0, pd_dmax = 0, pd_gmax = 0;
    if (d->hand_mode == 1) {
        st = build_pd_table(d, pd_tab, pd_groups, pd_dmax, pd_gmax);
        if (st != PT_OK) return st;
    }
    // ... and the step's hand kinematics, which use the same LDS first
    const size_t fk_bytes = d->hand_mode == 1 ? pt::pd_fk_bytes(d->L) : hand_fk_lds_bytes(d->L, d->D);
    const int n_pairs = d->collision_mode == 1 ? d->L * d->link_samples + d->S_max : d->S_max * (d->L + 1);
    const int list = std::min(n_pairs, pt::CAND_CAP) + 8, rows = red_rows * pt::RedStride<double>::value,
              fk = (int)((fk_bytes + 7) / 8);
    int max_cand, max_cand_rows;
    if (d->hand_mode == 1) {
        // the PD solve keeps its group solutions in the spare words
        max_cand = std::max({round_up(list, 64), round_up(rows, 64), round_up(fk, 64)});
        max_cand_rows = max_cand;
    } else {
        // the sum rows may run on into the spare words after a shorter
        // list; the reverse sweep, which stages its own data there, keeps
        // them whole in the list
        max_cand = std::max({round_up(list, 32), round_up(rows - pt::WAVE_SPARE_BYTES / 8, 32), round_up(fk, 32)});
        max_cand_rows = std::max(max_cand, round_up(rows, 32));
    }
    const size_t wave_lds = std::max(pt::wave_lds_bytes(max_cand, d->L), pt::wave_lds_bytes(max_cand_rows, 0)) +
                            (d->hand_mode == 1 ? pt::pd_lds_bytes(d->D) : 0);
    if (wave_lds > 160 * 1024)
        return fail(PT_E_UNSUPPORTED, "%zu B of LDS per simulation (> 160 KiB)", wave_lds);

    pt_batch b = new pt_batch_s();
    Consts &P = b->P;
    P.K = d->K; P.G = d->G; P.L = d->L; P.D = d->D; P.S_max = d->S_max; P.C_max = d->C_max;
    P.newton_iters = d->newton_iters; P.T = d->T; P.max_cand = max_cand; P.max_cand_rows = max_cand_rows;
    P.solve_fp64 = d->solve_precision == 32 ? 0 : 1;
    P.dt = d->dt; P.gx = d->gravity[0]; P.gy = d->gravity[1]; P.gz = d->gravity[2];
    P.margin = d->margin; P.erp = d->erp; P.compliance = d->compliance; P.kappa = d->kappa;
    P.fb_delta = d->fb_delta; P.armijo_sigma = d->armijo_sigma;
    P.tau_contact = d->tau_contact; P.w_mag = d->w_mag; P.w_dir = d->w_dir;
    P.cost_mode = d->cost_mode;
    P.tau_slip = d->tau_slip; P.tau_spin = d->tau_spin;
    for (int i = 0; i < 7; ++i) P.w_eq3[i] = d->cost_mode == 1 ? d->w_eq3[i] : 0.f;
    P.collision_mode = d->collision_mode;
    P.link_samples = d->collision_mode == 1 ? d->link_samples : 0;
    P.sdf_n = d->collision_mode == 1 ? d->sdf_n : 0;
    b->R = {d->elite_frac, d->sigma_mu, d->sigma_m, d->sigma_f, d->mu_lo, d->mu_hi, d->m_lo, d->m_hi, d->seed};
    b->n_types = d->n_types;
    b->hand_mode = d->hand_mode;
    if (d->hand_mode == 1) {
        b->Q = {pd_groups, pd_dmax, pd_gmax, d->kp, d->kd, d->link_mass, d->w_q};
        b->hstate = d->hand_state;
    }
    b->state = d->state;
    b->params = d->params;
    b->warm = d->warm;
    b->group_start.assign(d->group_start, d->group_start + d->G + 1);
    for (int g = 0; g < d->G; ++g) b->max_group = std::max(b->max_group, b->group_start[g + 1] - b->group_start[g]);
    if (pt::resample_lds_bytes(b->max_group) > 160 * 1024) {
        delete b;
        return fail(PT_E_UNSUPPORTED, "group of %d simulations exceeds the resampler's LDS (max 16384)", b->max_group);
    }

    auto cleanup = [&](pt_status code) {
        pt_destroy_batch(b);
        return code;
    };
#define HIP_TRY_C(expr)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return cleanup(fail(PT_E_HIP, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)

    HIP_TRY_C(hipGetDevice(&b->device));
    HIP_TRY_C(hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, b->device));
    // this device's copy of pt_run_window_static's scratch, once per device
    HIP_TRY_C(static_scratch(b->device, &b->static_scratch));
    HIP_TRY_C(set_lds_limits(160 * 1024));
    HIP_TRY_C(set_grad_lds_limits(160 * 1024));
    HIP_TRY_C(set_draw_lds_limits(160 * 1024));
    HIP_TRY_C(set_pd_lds_limits(160 * 1024));

    const size_t K = d->K;
    std::vector<int32_t> group_of(K), order(K);
    for (int g = 0; g < d->G; ++g)
        for (int i = d->group_start[g]; i < d->group_start[g + 1]; ++i) group_of[i] = g;
    // persistent-kernel work order: simulations with more spheres first
    for (size_t i = 0; i < K; ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return d->n_spheres[d->env_type[a]] > d->n_spheres[d->env_type[c]];
    });

    HIP_TRY_C(hipMalloc(&b->d_hand, sizeof(float) * d->L * PT_HAND_STRIDE));
    HIP_TRY_C(hipMalloc(&b->d_spheres, sizeof(float) * d->n_types * d->S_max * 4));
    HIP_TRY_C(hipMalloc(&b->d_inv, sizeof(float) * d->n_types * 3));
    HIP_TRY_C(hipMalloc(&b->d_nsph, sizeof(int32_t) * d->n_types));
    HIP_TRY_C(hipMalloc(&b->d_type, sizeof(int32_t) * K));
    HIP_TRY_C(hipMalloc(&b->d_group_of, sizeof(int32_t) * K));
    HIP_TRY_C(hipMalloc(&b->d_group_start, sizeof(int32_t) * (d->G + 1)));
    HIP_TRY_C(hipMalloc(&b->d_order, sizeof(int32_t) * K));
    HIP_TRY_C(hipMalloc(&b->d_queue, sizeof(int32_t) * 4));
    HIP_TRY_C(hipMalloc(&b->d_stats, sizeof(int64_t) * pt::STATS_SLOTS * pt::STATS_STRIDE));
    HIP_TRY_C(hipMalloc(&b->d_seg_win, sizeof(float) * (size_t)d->T * d->L * pt::SEG_STRIDE));
    HIP_TRY_C(hipMalloc(&b->d_contacts, sizeof(float) * K * d->C_max * 4));
    HIP_TRY_C(hipMalloc(&b->d_seg_grad, sizeof(float) * (size_t)d->T * d->L * pt::SEG_STRIDE));
    HIP_TRY_C(hipMalloc(&b->d_tune, sizeof(float) * tune_floats(P)));
    for (int g = 0; g < d->G; ++g)
        b->n_elite += pt::elite_count(d->group_start[g + 1] - d->group_start[g], d->elite_frac);
    HIP_TRY_C(hipMalloc(&b->d_ckpt, sizeof(float) * ckpt_floats(P, b->n_elite)));
    HIP_TRY_C(hipMalloc(&b->d_ref, sizeof(float) * refine_floats(P, b->n_elite)));
    HIP_TRY_C(hipMalloc(&b->d_elite, sizeof(int32_t) * b->n_elite));
    HIP_TRY_C(hipMalloc(&b->d_snap, sizeof(float) * K * (18 + (size_t)4 * d->C_max)));
    if (d->window_checkpoints) HIP_TRY_C(hipMalloc(&b->d_wckpt, sizeof(float) * ckpt_floats(P, (int)K)));
    if (d->collision_mode == 1) {
        const size_t nv = (size_t)d->n_types * d->sdf_n * d->sdf_n * d->sdf_n;
        HIP_TRY_C(hipMalloc(&b->d_sdf, sizeof(float) * nv));
        HIP_TRY_C(hipMalloc(&b->d_sdf_box, sizeof(float) * 4 * d->n_types));
        HIP_TRY_C(hipMemcpy(b->d_sdf, d->sdf, sizeof(float) * nv, hipMemcpyHostToDevice));
        HIP_TRY_C(hipMemcpy(b->d_sdf_box, d->sdf_box, sizeof(float) * 4 * d->n_types, hipMemcpyHostToDevice));
    }
    if (d->hand_mode == 1) {
        HIP_TRY_C(hipMalloc(&b->d_pd, sizeof(int32_t) * pd_tab.size()));
        HIP_TRY_C(hipMalloc(&b->d_parent, sizeof(int32_t) * K));
        HIP_TRY_C(hipMalloc(&b->d_pd_obs, sizeof(float) * (4 * (size_t)d->L + d->D) * K));
        HIP_TRY_C(hipMemcpy(b->d_pd, pd_tab.data(), sizeof(int32_t) * pd_tab.size(), hipMemcpyHostToDevice));
    }
    if (d->hand_mode == 0) HIP_TRY_C(hipMalloc(&b->d_seg, sizeof(float) * d->L * pt::SEG_STRIDE));
    if (d->cost_mode == 1) {
        HIP_TRY_C(hipMalloc(&b->d_cslip, sizeof(float) * K * d->C_max * 8));
        HIP_TRY_C(hipMemset(b->d_cslip, 0, sizeof(float) * K * d->C_max * 8));
    }
    HIP_TRY_C(hipMemcpy(b->d_hand, d->hand, sizeof(float) * d->L * PT_HAND_STRIDE, hipMemcpyHostToDevice));
    HIP_TRY_C(hipMemcpy(b->d_spheres, d->spheres, sizeof(float) * d->n_types * d->S_max * 4, hipMemcpyHostToDevice));
    HIP_TRY_C(hipMemcpy(b->d_inv, d->inv_inertia, sizeof(float) * d->n_types * 3, hipMemcpyHostToDevice));
    HIP_TRY_C(hipMemcpy(b->d_nsph, d->n_spheres, sizeof(int32_t) * d->n_types, hipMemcpyHostToDevice));
    HIP_TRY_C(hipMemcpy(b->d_type, d->env_type, sizeof(int32_t) * K, hipMemcpyHostToDevice));
    HIP_TRY_C(hipMemcpy(b->d_group_of, group_of.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice));
    HIP_TRY_C(hipMemcpy(b->d_group_start, d->group_start, sizeof(int32_t) * (d->G + 1), hipMemcpyHostToDevice));
    HIP_TRY_C(hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice));
    HIP_TRY_C(hipMemset(b->d_queue, 0, sizeof(int32_t) * 4));
    HIP_TRY_C(hipMemset(b->d_stats, 0, sizeof(int64_t) * pt::STATS_SLOTS * pt::STATS_STRIDE));
    HIP_TRY_C(hipMemset(b->d_contacts, 0, sizeof(float) * K * d->C_max * 4));
    HIP_TRY_C(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
    HIP_TRY_C(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    for (int k = 0; k < pt_batch_s::REFINE_PARTS - 1; ++k) {
        HIP_TRY_C(hipStreamCreateWithFlags(&b->side_stream[k], hipStreamNonBlocking));
        HIP_TRY_C(hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming));
    }
    // environments per workgroup within the LDS budget (autotuned later)
    b->wpb = 4;
    const size_t win_lds = pt::wave_lds_bytes(max_cand, 0);
    while (b->wpb > 1 && ((size_t)b->wpb * win_lds > 160 * 1024 || b->wpb > max_wpb(P))) b->wpb >>= 1;
    // the per-step launch: one simulation per workgroup, so that up to one
    // wavefront per compute unit has its LDS, caches and issue to itself
    // (measured faster than four per workgroup at 256 simulations)
    b->step_wpb = 1;
    // from a full round of the GPU's step wavefronts (eight per compute
    // unit) the hand kinematics run once per step in a launch of their own
    // rather than in every wavefront; below that the step is latency-bound
    // and the per-wavefront evaluation overlaps its state loads
    b->step_fk_once = d->hand_mode == 0 && P.solve_fp64 && K >= 8 * b->num_cu;
#undef HIP_TRY_C
    *out = b;
    return PT_OK;
}

pt_status pt_destroy_batch(pt_batch b)
{
    if (!b) return PT_OK;
    (void)hipDeviceSynchronize();
    b->drop_graphs();
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    for (int k = 0; k < pt_batch_s::REFINE_PARTS - 1; ++k) {
        if (b->side_stream[k]) (void)hipStreamDestroy(b->side_stream[k]);
        if (b->ev_join[k]) (void)hipEventDestroy(b->ev_join[k]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    void *ptrs[] = {b->d_hand, b->d_spheres, b->d_inv, b->d_nsph, b->d_type, b->d_group_of, b->d_group_start,
                    b->d_order, b->d_queue, b->d_stats, b->d_seg_win, b->d_contacts,
                    b->d_seg_grad, b->d_tune, b->d_ckpt, b->d_wckpt, b->d_elite, b->d_ref, b->d_snap,
                    b->d_cslip, b->d_seg, b->d_pd, b->d_parent, b->d_pd_obs, b->d_sdf, b->d_sdf_box};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete b;
    return PT_OK;
}

static Tables tables_of(const pt_batch b)
{
    Tables tb;
    tb.hand = b->d_hand;
    tb.spheres = b->d_spheres;
    tb.n_spheres = b->d_nsph;
    tb.inv_inertia = b->d_inv;
    tb.env_type = b->d_type;
    tb.group_of = b->d_group_of;
    tb.sdf = b->d_sdf;
    tb.sdf_box = b->d_sdf_box;
    return tb;
}

pt_status pt_step(pt_batch b, const float *u_prev, const float *u, pt_stream s)
{
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    hipStream_t st = (hipStream_t)s;
    if (b->hand_mode == 1) {
        if (b->P.D > 0 && !u) return fail(PT_E_ARG, "u is NULL");
        HIP_TRY(launch_step_pd(b->P, b->Q, tables_of(b), b->d_pd, u, b->state, b->params, b->warm, b->hstate,
                               b->d_contacts, b->d_stats, st));
        return PT_OK;
    }
    if (b->P.D > 0 && (!u_prev || !u)) return fail(PT_E_ARG, "u_prev/u is NULL");
    if (b->step_fk_once)
        HIP_TRY(launch_hand_fk(b->d_hand, b->P.L, b->P.D, b->P.dt, u_prev, u, 0, 1, b->d_seg, st));
    HIP_TRY(launch_step(b->P, tables_of(b), u_prev, u, b->state, b->params, b->warm, b->d_contacts, b->d_cslip,
                        b->d_seg, b->d_stats, b->step_wpb, b->step_fk_once, st));
    return PT_OK;
}

pt_status pt_observe(pt_batch b, float *obs, pt_stream s)
{
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    if (!obs) return fail(PT_E_ARG, "obs is NULL");
    if (b->hand_mode == 1) {
        HIP_TRY(launch_observe_pd(b->P, b->d_contacts, b->hstate, obs, (hipStream_t)s));
        return PT_OK;
    }
    HIP_TRY(launch_observe(b->P, b->d_contacts, b->d_cslip, b->d_seg, obs, (hipStream_t)s));
    return PT_OK;
}

pt_status pt_cost(pt_batch b, const float *obs, const float *obs_gt, float *cost_sum, int32_t *best, pt_stream s)
{
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    if (!obs || !obs_gt || !cost_sum) return fail(PT_E_ARG, "obs/obs_gt/cost_sum is NULL");
    hipStream_t st = (hipStream_t)s;
    if (b->hand_mode == 1) {
        HIP_TRY(launch_cost_pd(b->P, b->Q, b->d_group_of, obs, obs_gt, cost_sum, st));
        if (best) HIP_TRY(launch_argmin(b->P.G, b->d_group_start, cost_sum, best, st));
        return PT_OK;
    }
    // up to FUSED_ARGMIN_MAX simulations the cost kernel's last workgroup ranks
    // the groups itself; past that one workgroup's pass over the population
    // takes longer than a launch of the per-group argmin kernel
    const bool fused = best && b->P.K <= pt::FUSED_ARGMIN_MAX;
    HIP_TRY(launch_cost(b->P, b->d_group_of, b->d_group_start, obs, obs_gt, cost_sum, fused ? best : nullptr,
                        b->d_queue + 2, st));
    if (best && !fused) HIP_TRY(launch_argmin(b->P.G, b->d_group_start, cost_sum, best, st));
    return PT_OK;
}

pt_status pt_resample(pt_batch b, float *cost_sum, uint32_t window_idx, int32_t *parent, pt_stream s)
{
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    if (!cost_sum) return fail(PT_E_ARG, "cost_sum is NULL");
    // the PD hand's joint state follows each simulation's parent
    int32_t *par = b->hand_mode == 1 && !parent ? b->d_parent : parent;
    HIP_TRY(launch_resample(b->P, b->R, b->d_group_start, b->max_group, window_idx, cost_sum, b->state, b->params,
                            b->warm, par, (hipStream_t)s));
    if (b->hand_mode == 1 && b->P.D > 0)
        HIP_TRY(launch_copy_hand(b->P.K, 2 * b->P.D, par, b->hstate, (hipStream_t)s));
    return PT_OK;
}

static pt_status weighted_resample(pt_batch b, int kind, float hyper, float *cost_sum, int32_t n_steps,
                                   uint32_t window_idx, int32_t *parent, float *weights, float *eta, pt_stream s)
{
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    if (!cost_sum || !parent) return fail(PT_E_ARG, "cost_sum/parent is NULL");
    if (b->hand_mode == 1) return fail(PT_E_UNSUPPORTED, "the weighted resamplers do not carry the PD hand's state");
    if (n_steps < 1) return fail(PT_E_ARG, "n_steps must be >= 1 (got %d)", n_steps);
    if (!std::isfinite(hyper) || (kind == 0 ? hyper < 0.f : hyper <= 0.f))
        return fail(PT_E_ARG, kind == 0 ? "lambda must be finite and >= 0" : "epsilon must be finite and > 0");
    HIP_TRY(launch_weighted_resample(b->P, b->R, kind, hyper, b->d_group_start, b->max_group, n_steps, window_idx,
                                     cost_sum, b->state, b->params, b->warm, b->d_snap, parent, weights, eta,
                                     (hipStream_t)s));
    return PT_OK;
}

pt_status pt_resample_wrs(pt_batch b, float *cost_sum, int32_t n_steps, uint32_t window_idx, float lambda,
                          int32_t *parent, float *weights, pt_stream s)
{
    return weighted_resample(b, 0, lambda, cost_sum, n_steps, window_idx, parent, weights, nullptr, s);
}

pt_status pt_resample_reps(pt_batch b, float *cost_sum, int32_t n_steps, uint32_t window_idx, float epsilon,
                           int32_t *parent, float *weights, float *eta, pt_stream s)
{
    return weighted_resample(b, 1, epsilon, cost_sum, n_steps, window_idx, parent, weights, eta, s);
}

// the launches of one window, in stream order
static pt_status enqueue_window(pt_batch b, const float *u_win, const float *obs_gt_win, float *cost_sum,
                                int32_t *best, float *obs_out, int wpb, float *state, float *params, float *warm,
                                float *ckpt, hipStream_t st, float *seg_win = nullptr, int32_t *queue = nullptr)
{
    const Consts &P = b->P;
    if (b->hand_mode == 1) {
        // the PD hand (its kinematics depend on each simulation's joint
        // angles): up to one simulation per SIMD, one wavefront runs each
        // simulation's whole window; beyond, where occupancy counts, the
        // per-step kernels run it step by step (the window kernel holds one
        // wavefront per SIMD, the step kernel two), the same bits either way
        const Tables tb = tables_of(b);
        if (P.K <= 4 * b->num_cu) {
            HIP_TRY(launch_window_pd(P, b->Q, tb, b->d_pd, u_win, state, params, warm, b->hstate, obs_gt_win,
                                     cost_sum, obs_out, b->d_stats, st));
        } else {
            const size_t RG = (4 * (size_t)P.L + P.D) * P.G, RK = (4 * (size_t)P.L + P.D) * P.K;
            for (int t = 0; t < P.T; ++t) {
                float *obs = obs_out ? obs_out + (size_t)t * RK : b->d_pd_obs;
                HIP_TRY(launch_step_pd(P, b->Q, tb, b->d_pd, u_win + (size_t)(t + 1) * P.D, state, params, warm,
                                       b->hstate, b->d_contacts, b->d_stats, st));
                HIP_TRY(launch_observe_pd(P, b->d_contacts, b->hstate, obs, st));
                HIP_TRY(launch_cost_pd(P, b->Q, b->d_group_of, obs, obs_gt_win + (size_t)t * RG, cost_sum, st));
            }
        }
        if (best) HIP_TRY(launch_argmin(P.G, b->d_group_start, cost_sum, best, st));
        return PT_OK;
    }
    if (!seg_win) seg_win = b->d_seg_win;
    if (!queue) queue = b->d_queue;
    int bpc = 0;
    HIP_TRY(window_occupancy(P, wpb, &bpc));
    if (bpc < 1) return fail(PT_E_UNSUPPORTED, "persistent kernel does not fit with %d waves per workgroup", wpb);
    int want = (P.K + wpb - 1) / wpb;
    int blocks = std::min(want, bpc * b->num_cu);
    HIP_TRY(launch_hand_fk(b->d_hand, P.L, P.D, P.dt, u_win, u_win + P.D, P.D, P.T, seg_win, st));
    // the window kernel's last workgroup puts the work queue back to 0 and,
    // for populations up to FUSED_ARGMIN_MAX, ranks the groups
    const bool fused = best && P.K <= pt::FUSED_ARGMIN_MAX;
    HIP_TRY(launch_window(P, tables_of(b), seg_win, state, params, warm, obs_gt_win, cost_sum, obs_out,
                          b->d_order, queue, b->d_stats, wpb, blocks, ckpt, b->d_group_start,
                          fused ? best : nullptr, st));
    if (best && !fused) HIP_TRY(launch_argmin(P.G, b->d_group_start, cost_sum, best, st));
    return PT_OK;
}

pt_status pt_run_window(pt_batch b, const float *u_win, const float *obs_gt_win, float *cost_sum, int32_t *best,
                        float *obs_out, int32_t graph, pt_stream s)
{
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    if (!u_win || !obs_gt_win || !cost_sum) return fail(PT_E_ARG, "u_win/obs_gt_win/cost_sum is NULL");
    hipStream_t st = (hipStream_t)s;
    if (!graph)
        return enqueue_window(b, u_win, obs_gt_win, cost_sum, best, obs_out, b->wpb, b->state, b->params, b->warm,
                              b->d_wckpt, st);
    GraphKey key{{u_win, obs_gt_win, cost_sum, best, obs_out}, b->wpb};
    int slot = -1;
    for (int i = 0; i < pt_batch_s::N_GRAPHS; ++i)
        if (b->graph_exec[i] && b->graph_key[i] == key) slot = i;
    if (slot < 0) {
        // an empty entry, else the least recently used one
        int victim = -1;
        for (int i = 0; i < pt_batch_s::N_GRAPHS && victim < 0; ++i)
            if (!b->graph_exec[i]) victim = i;
        if (victim < 0) {
            victim = 0;
            for (int i = 1; i < pt_batch_s::N_GRAPHS; ++i)
                if (b->graph_used[i] < b->graph_used[victim]) victim = i;
        }
        slot = victim;
        if (b->graph_exec[slot]) {
            HIP_TRY(hipStreamSynchronize(st));
            HIP_TRY(hipGraphExecDestroy(b->graph_exec[slot]));
            b->graph_exec[slot] = nullptr;
        }
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
        pt_status cs = enqueue_window(b, u_win, obs_gt_win, cost_sum, best, obs_out, b->wpb, b->state, b->params,
                                      b->warm, b->d_wckpt, b->capture_stream);
        hipError_t ec = hipStreamEndCapture(b->capture_stream, &g);
        if (cs != PT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return cs;
        }
        if (ec != hipSuccess) return fail(PT_E_CAPTURE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
        hipError_t ei = hipGraphInstantiate(&b->graph_exec[slot], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            b->graph_exec[slot] = nullptr;
            return fail(PT_E_CAPTURE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
        }
        b->graph_key[slot] = key;
    }
    b->graph_used[slot] = ++b->graph_clock;
    HIP_TRY(hipGraphLaunch(b->graph_exec[slot], st));
    return PT_OK;
}

pt_status pt_run_window_static(pt_batch b, const float *u_win, const float *obs_gt_win, float *cost_sum,
                               int32_t *best, float *obs_out, pt_stream s)
{
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    if (!u_win || !obs_gt_win || !cost_sum) return fail(PT_E_ARG, "u_win/obs_gt_win/cost_sum is NULL");
    const Consts &P = b->P;
    if ((size_t)P.T * P.L > STATIC_SEG_RECORDS)
        return fail(PT_E_UNSUPPORTED, "T x L = %d x %d exceeds the static scratch's %zu hand segment records", P.T,
                    P.L, STATIC_SEG_RECORDS);
    if (!b->static_scratch) return fail(PT_E_STATE, "static scratch not resolved for device %d", b->device);
    hipStream_t st = (hipStream_t)s;
    int32_t *queue = static_cast<int32_t *>(b->static_scratch);
    float *seg_win = static_cast<float *>(b->static_scratch) + STATIC_COUNTER_INTS;
    // the work-queue and last-workgroup counters start at 0 (the array keeps
    // whatever the last call on this GPU left)
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, queue, 4, 0);
    HIP_TRY(hipGetLastError());
    return enqueue_window(b, u_win, obs_gt_win, cost_sum, best, obs_out, b->wpb, b->state, b->params, b->warm,
                          b->d_wckpt, st, seg_win, queue);
}

pt_status pt_autotune(pt_batch b, const float *u_win, const float *obs_gt_win, int32_t *result, pt_stream s)
{
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    if (b->hand_mode == 1)
        return fail(PT_E_UNSUPPORTED, "the PD hand's window runs one simulation per wavefront: nothing to tune");
    if (!u_win || !obs_gt_win) return fail(PT_E_ARG, "u_win/obs_gt_win is NULL");
    hipStream_t st = (hipStream_t)s;
    const Consts &P = b->P;
    const size_t K = P.K;
    const size_t n_state = 13 * K, n_params = 5 * K, n_warm = K * P.C_max * 4;
    float *ts = b->d_tune, *tp = ts + n_state, *tw = tp + n_params, *tc = tw + n_warm;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const size_t wave_lds = pt::wave_lds_bytes(P.max_cand, 0);
    int best_wpb = b->wpb;
    float best_ms = 1e30f;
    pt_status rc = PT_OK;
    // widest first: a narrower choice must be clearly faster (2%) to win,
    // since fewer, fuller workgroups leave compute units free for other work
    for (int wpb : {8, 4, 2, 1}) {
        if ((size_t)wpb * wave_lds > 160 * 1024 || wpb > max_wpb(P)) continue;
        float total = 0.f;
        for (int rep = 0; rep < 3 && rc == PT_OK; ++rep) {
            if (hipMemcpyAsync(ts, b->state, sizeof(float) * n_state, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(tp, b->params, sizeof(float) * n_params, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemcpyAsync(tw, b->warm, sizeof(float) * n_warm, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                hipMemsetAsync(tc, 0, sizeof(float) * K, st) != hipSuccess) {
                rc = fail(PT_E_HIP, "autotune scratch copy failed");
                break;
            }
            (void)hipEventRecord(e0, st);
            rc = enqueue_window(b, u_win, obs_gt_win, tc, nullptr, nullptr, wpb, ts, tp, tw, nullptr, st);
            (void)hipEventRecord(e1, st);
            if (rc != PT_OK) break;
            if (hipEventSynchronize(e1) != hipSuccess) {
                rc = fail(PT_E_HIP, "autotune: window failed");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) total += ms;  // first run warms up
        }
        if (rc != PT_OK) break;
        if (total < 0.98f * best_ms) {
            best_ms = total;
            best_wpb = wpb;
        }
    }
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PT_OK) return rc;
    b->wpb = best_wpb;
    if (result) *result = best_wpb;
    return PT_OK;
}

pt_status pt_set_tuning(pt_batch b, int32_t wpb)
{
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    if (wpb != 1 && wpb != 2 && wpb != 4 && wpb != 8) return fail(PT_E_ARG, "waves per workgroup must be 1, 2, 4 or 8");
    if ((size_t)wpb * pt::wave_lds_bytes(b->P.max_cand, 0) > 160 * 1024)
        return fail(PT_E_UNSUPPORTED, "%d simulations per workgroup exceed the LDS", wpb);
    if (wpb > max_wpb(b->P))
        return fail(PT_E_UNSUPPORTED, "at most %d simulations per workgroup with this solve precision", max_wpb(b->P));
    b->wpb = wpb;
    return PT_OK;
}

pt_status pt_window_grad(pt_batch b, const float *u_win, const float *obs_gt_win, int32_t n, const int32_t *env,
                         const float *start, const float *warm0, float *cost, float *grad, float *end_state,
                         float *end_warm, float *resid, pt_stream s)
{
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    if (b->hand_mode == 1) return fail(PT_E_UNSUPPORTED, "the window gradient is not built for the PD hand");
    if (b->P.collision_mode == 1) return fail(PT_E_UNSUPPORTED, "the window gradient is not built for the distance-field collision");
    if (b->P.cost_mode != 0) return fail(PT_E_UNSUPPORTED, "the window gradient is defined for cost_mode 0 only");
    if (n < 0) return fail(PT_E_ARG, "n must be >= 0 (got %d)", n);
    if (n == 0) return PT_OK;
    if (!u_win || !obs_gt_win || !env || !start || !warm0 || !cost)
        return fail(PT_E_ARG, "u_win/obs_gt_win/env/start/warm0/cost is NULL");
    hipStream_t st = (hipStream_t)s;
    const Consts &P = b->P;
    const Tables tb = tables_of(b);
    HIP_TRY(launch_hand_fk(b->d_hand, P.L, P.D, P.dt, u_win, u_win + P.D, P.D, P.T, b->d_seg_grad, st));
    if (!grad) {
        HIP_TRY(launch_window_fwd(P, tb, b->d_seg_grad, n, 0, n, env, start, warm0, obs_gt_win, cost, end_state,
                                  end_warm, nullptr, st, resid));
        return PT_OK;
    }
    // the checkpoint buffer holds n_elite simulations: forward and reverse
    // sweeps run in chunks of that many
    for (int i0 = 0; i0 < n; i0 += b->n_elite) {
        const int cnt = std::min(b->n_elite, n - i0);
        HIP_TRY(launch_window_fwd(P, tb, b->d_seg_grad, n, i0, cnt, env, start, warm0, obs_gt_win, cost, end_state,
                                  end_warm, b->d_ckpt, st, resid));
        HIP_TRY(launch_window_bwd(P, tb, b->d_seg_grad, n, i0, cnt, env, start, obs_gt_win, b->d_ckpt, false, nullptr,
                                  grad, st));
    }
    return PT_OK;
}

pt_status pt_refine_elites(pt_batch b, const float *u_win, const float *obs_gt_win, float *cost_sum,
                           const float *start_state, const float *start_params, const float *start_warm,
                           int32_t steps, float step, const float *scale, int32_t *best, int32_t *elite_out,
                           pt_stream s)
{
    if (b && b->P.cost_mode != 0)
        return fail(PT_E_UNSUPPORTED, "elite refinement needs the window gradient, defined for cost_mode 0 only");
    if (!b) return fail(PT_E_ARG, "batch is NULL");
    if (b->hand_mode == 1) return fail(PT_E_UNSUPPORTED, "elite refinement is not built for the PD hand");
    if (b->P.collision_mode == 1) return fail(PT_E_UNSUPPORTED, "elite refinement is not built for the distance-field collision");
    if (!u_win || !obs_gt_win || !cost_sum || !start_state || !start_params || !start_warm)
        return fail(PT_E_ARG, "u_win/obs_gt_win/cost_sum/start_state/start_params/start_warm is NULL");
    if (steps < 0) return fail(PT_E_ARG, "steps must be >= 0 (got %d)", steps);
    if (!(step > 0.f) || !std::isfinite(step)) return fail(PT_E_ARG, "step must be positive and finite");
    pt::RefineArgs A;
    static const float kScale[15] = {1e-3f, 1e-3f, 1e-3f, 0.01f, 0.01f, 0.01f, 0.01f, 0.01f,
                                     0.01f, 0.01f, 0.1f,  0.1f,  0.1f,  5e-3f, 0.02f};
    for (int i = 0; i < 15; ++i) {
        A.scale[i] = scale ? scale[i] : kScale[i];
        if (!(A.scale[i] >= 0.f) || !std::isfinite(A.scale[i])) return fail(PT_E_ARG, "scale[%d] must be finite and >= 0", i);
    }
    A.m_lo = b->R.m_lo; A.m_hi = b->R.m_hi; A.mu_lo = b->R.mu_lo; A.mu_hi = b->R.mu_hi;
    hipStream_t st = (hipStream_t)s;
    const Consts &P = b->P;
    const int n = b->n_elite;
    RefineBufs r = refine_layout(b->d_ref, P, n);
    const Tables tb = tables_of(b);
    HIP_TRY(launch_select_elites(P.G, b->max_group, b->R.elite_frac, b->d_group_start, cost_sum, b->d_elite, st));
    if (elite_out)
        HIP_TRY(hipMemcpyAsync(elite_out, b->d_elite, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    if (steps > 0) {
        HIP_TRY(launch_hand_fk(b->d_hand, P.L, P.D, P.dt, u_win, u_win + P.D, P.D, P.T, b->d_seg_grad, st));
        // the first gradient: from the checkpoints the population's window
        // recorded (window_checkpoints) or from a replay of the window
        const bool from_window = b->d_wckpt != nullptr;
        HIP_TRY(launch_refine_gather(n, P.K, P.C_max, b->d_elite, start_state, start_params, start_warm,
                                     from_window ? cost_sum : nullptr, r.xi, r.warm0, r.cost, r.rho, step, st));
        // every elite's chain of replays and sweeps is its own, so when the
        // elites outnumber what the GPU holds at once (from 16 per compute
        // unit: two or more rounds of the at most eight replay wavefronts a
        // compute unit holds) they go in parts on streams of their own:
        // one part's short kernels and the tail of its replay overlap the
        // others' replays (the same bits as one launch over all of them);
        // each part has its own checkpoints.  Fewer elites all run at once
        // in one launch, and parts would only add launches.
        constexpr int NP = pt_batch_s::REFINE_PARTS;
        const int parts = n >= 16 * b->num_cu ? NP : 1;
        struct Part {
            int i0, count;
            hipStream_t s;
            float *ckpt;
        } part[NP];
        int np = 0;
        for (int k = 0, i0 = 0; k < parts; ++k) {
            const int cnt = (n - i0) / (parts - k) + ((n - i0) % (parts - k) != 0);
            if (cnt <= 0) break;
            part[np++] = {i0, cnt, k == 0 ? st : b->side_stream[k - 1], b->d_ckpt + ckpt_floats(P, i0)};
            i0 += cnt;
        }
        if (np > 1) {
            HIP_TRY(hipEventRecord(b->ev_fork, st));
            for (int k = 1; k < np; ++k) HIP_TRY(hipStreamWaitEvent(part[k].s, b->ev_fork, 0));
        }
        for (int k = 0; k < np; ++k) {
            const Part &c = part[k];
            if (!from_window)
                HIP_TRY(launch_window_fwd(P, tb, b->d_seg_grad, n, c.i0, c.count, b->d_elite, r.xi, r.warm0,
                                          obs_gt_win, r.cost, nullptr, nullptr, c.ckpt, c.s));
            HIP_TRY(launch_window_bwd(P, tb, b->d_seg_grad, n, c.i0, c.count, b->d_elite, r.xi, obs_gt_win,
                                      from_window ? b->d_wckpt : c.ckpt, from_window, nullptr, r.g, c.s));
        }
        for (int it = 0; it < steps; ++it) {
            // trial, its replay (checkpointed unless it is the last), keep or
            // halve, then the gradient at the kept trials only
            const bool last = it == steps - 1;
            for (int k = 0; k < np; ++k) {
                const Part &c = part[k];
                HIP_TRY(launch_refine_propose(n, c.i0, c.count, A, r.xi, r.g, r.rho, r.xi_try, c.s));
                HIP_TRY(launch_window_fwd(P, tb, b->d_seg_grad, n, c.i0, c.count, b->d_elite, r.xi_try, r.warm0,
                                          obs_gt_win, r.cost_try, r.end_state, r.end_warm, last ? nullptr : c.ckpt,
                                          c.s));
                HIP_TRY(launch_refine_accept(n, c.i0, c.count, P.K, P.C_max, b->d_elite, r.cost, r.cost_try, r.xi,
                                             r.xi_try, r.rho, r.flag, r.end_state, r.end_warm, b->state, b->params,
                                             b->warm, cost_sum, c.s));
                if (!last)
                    HIP_TRY(launch_window_bwd(P, tb, b->d_seg_grad, n, c.i0, c.count, b->d_elite, r.xi, obs_gt_win,
                                              c.ckpt, false, r.flag, r.g, c.s));
            }
        }
        for (int k = 1; k < np; ++k) {
            HIP_TRY(hipEventRecord(b->ev_join[k - 1], part[k].s));
            HIP_TRY(hipStreamWaitEvent(st, b->ev_join[k - 1], 0));
        }
    }
    if (best) HIP_TRY(launch_argmin(P.G, b->d_group_start, cost_sum, best, st));
    return PT_OK;
}

int32_t pt_elite_count(pt_batch b) { return b ? b->n_elite : -1; }

pt_status pt_read_stats(pt_batch b, int64_t *out, pt_stream s)
{
    if (!b || !out) return fail(PT_E_ARG, "batch/out is NULL");
    HIP_TRY(hipStreamSynchronize((hipStream_t)s));
    std::vector<int64_t> slots((size_t)pt::STATS_SLOTS * pt::STATS_STRIDE);
    HIP_TRY(hipMemcpy(slots.data(), b->d_stats, sizeof(int64_t) * slots.size(), hipMemcpyDeviceToHost));
    for (int j = 0; j < 4; ++j) {
        int64_t t = 0;
        for (int k = 0; k < pt::STATS_SLOTS; ++k) t += slots[(size_t)k * pt::STATS_STRIDE + j];
        out[j] = t;
    }
    return PT_OK;
}

}  // extern "C"
