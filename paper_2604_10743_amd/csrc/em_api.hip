// Host runtime and C ABI of the EM/TM library: input validation, wire-tree
// partition of the netlist (Sec. IV-A), device layout, and the coupled outer
// loop of Fig. 2 (IR solve -> screen -> {stress steps, dR write-back,
// IR re-solve} -> time to failure).  All arithmetic of the method runs in the
// kernels of k_tree.hip and k_ir.hip; the host only does integer topology,
// memory management, launches and the convergence/retirement control flow.
#include "em_internal.h"
#include "../../include/em.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace em;

struct em_batch {
    em_material mat;
    em_run_params run;
    int S = 1;
    uint64_t seed = 0;
    double cov_k = 0, cov_s = 0, cov_r = 0, cov_l = 0, sd_ea = 0, sd_T = 0, cov_map = 0;
    bool trees_only = false;
    bool fp32 = false;
    hipStream_t stream = nullptr;
    em_allocator alloc{};
    bool has_alloc = false;
    std::string err;
    std::vector<void *> allocs;
    // host copies of the partition (read-back)
    int n_nodes = 0, n_res = 0, n_trees = 0, ns = 0, N = 0, max_tree_nodes = 0;
    std::vector<int> tree_off, parent, seg, dir, vert, kpos, seg_tree;
    Dev d{};
    Dev *d_dev = nullptr;         // device copy of d (read by kernels through a pointer)
    bool have_j = false;
    bool live_dirty = true;
    bool any_open = false;        // some segment of some sample has opened since creation/reset
    bool ir_valid = false;        // u, j, drop hold the solution for the current conductances
    bool ir_unchanged = false;    // the last IR solve was skipped: currents as before
    uint8_t *live0 = nullptr;     // reachability from the pads with every resistor conducting, per
                                  // node of the iterated system
    int cg_iters_last = 0;
    int n_outer_done = 0;
    int step_counter = 0;         // steps taken through em_stress_step
    int n_generic_trees = 0;      // trees the chain kernel does not take
    int n_br = 0;                 // of those, trees stepped by the workgroup tree kernel (stepper 0)
    int br_max_nodes = 0;         // their largest node count
    int n_inc = 0;                // node-incidence entries of the iterated system
    // CG iterations captured once in a HIP graph and replayed in blocks
    hipStream_t cap_stream = nullptr;
    hipGraph_t cg_graph = nullptr;
    hipGraphExec_t cg_exec = nullptr;
    // stream-time accounting with HIP events around each stepping launch and
    // each IR solve; folded in at the next synchronisation
    hipEvent_t ev_a = nullptr, ev_b = nullptr, ev_c = nullptr, ev_d = nullptr;
    bool step_pending = false, ir_pending = false;
    // catch-up replays of the learned screen run on a stream of their own,
    // beside the main stepping launch of the same interval
    hipStream_t rp_stream = nullptr;
    hipEvent_t ev_j = nullptr, ev_ra = nullptr, ev_rb = nullptr;
    bool replay_pending = false;
    double step_ms = 0.0, ir_ms = 0.0;
    long long step_launches = 0, cg_iters_total = 0;
    long long cg_sample_iters = 0;      // PCG iterations summed over samples (each sample's own count)
    uint8_t *h_flags = nullptr;   // pinned scratch for small read-backs
    size_t h_flags_cap = 0;
    // learned screen (model borrowed from the caller)
    em_mlp *sur = nullptr;
    double sur_margin = 2.0;
    bool sur_ready = false;       // its device buffers exist
    float *sur_y = nullptr;       // [inst] model output of the last evaluation
    double *jhist = nullptr;      // [n_hist][S][n_res] current densities of each aging interval
    int n_hist = 0;
    double sur_ms = 0.0;
    int n_def_list = 0;           // length of d.def_list from the t = 0 evaluation
    // multigrid preconditioner of the IR solve (device arrays owned through allocs)
    Amg amg;
    Amg *amg_dev = nullptr;             // device copy of amg (one-workgroup PCG)
    bool use_amg = false;
    bool ir_wg = false;                 // multigrid PCG with one workgroup per sample
    bool ir_lds = false;                // ... running from LDS
    // compaction of the active instances (screen, learned screen): the list
    // the forcing update walks and the lanes the chain kernel launches
    bool nominal = true;                // every sample still has the nominal resistances (no step taken
                                        // since creation or reset, no state set or restored)
    bool act_dirty = true;              // inst_active may have changed since the last compaction
    bool forcing_stale = false;         // dt*f lags the last IR solve's currents
    bool act_built = false;
    int n_act = 0;
    int *act_inst = nullptr;            // [IS] active instances, ascending
    std::vector<uint8_t> act_prev;      // active flags at the last compaction
    int *pl_inst = nullptr, *pl_L = nullptr;   // [IS] chain-lane placement (device staging)
    long long *pl_off = nullptr;
    std::vector<int> chain_L;           // lanes per instance of a chain tree (0: generic tree)
    std::vector<int> tree_perm_h;
    int chain_wg = 0;
    int chain_m = 8;                    // stress nodes per lane of the chain kernel
    int chain_occ = 1;                  // chain kernel register budget: 1 default, 3 (168 VGPRs), 4 (128)
    bool psi_shared = false;            // steady stress of the last screen only in column 0 (shared screen)
    std::vector<int> wg_cand;           // chain workgroup sizes that hold the longest chain tree
    long long lanes_cap = 0;            // lanes allocated for the chain kernel's table
    int *res_cnt = nullptr;             // [S][2] per-sample result counts (device)
    // chain condensation: the PCG iterates the terminal system rd; interior
    // voltages follow from the chains
    bool condensed = false;
    Dev rd{};
    Cond cond{};
    int n_term = 0, n_redge = 0, n_cchain = 0;
    // Monte Carlo sample index of each batch sample (empty: identity)
    std::vector<int> sid_h;
    // FP32 guard band: a host copy of the netlist for the FP64 re-run of the
    // samples that came within the band of the failure threshold
    struct GridCopy *gcopy = nullptr;
    int n_redecided = 0;
    int n_screen_rerun = 0;
    long long rerun_node_steps = 0;     // node-steps of the re-runs of the last em_run_to_ttf
    // steady-state skipping (em_run_params.ss_tol > 0)
    bool ss_ready = false;
    long long n_ss_skipped = 0, n_ss_woken = 0;
};

// Deep host copy of a netlist descriptor (the FP64 re-run builds a batch from it).
struct GridCopy {
    em_grid_desc g{};
    std::vector<double> xy, len, w, h, R0, sink, node_T, tmap;
    std::vector<int> layer, ra, rb, pad;
    std::vector<uint8_t> via;
    explicit GridCopy(const em_grid_desc &s)
    {
        const size_t n = s.n_nodes, m = s.n_res;
        xy.assign(s.xy, s.xy + 2 * n); layer.assign(s.layer, s.layer + n);
        ra.assign(s.res_a, s.res_a + m); rb.assign(s.res_b, s.res_b + m);
        len.assign(s.res_len, s.res_len + m); w.assign(s.res_w, s.res_w + m); h.assign(s.res_h, s.res_h + m);
        via.assign(s.res_is_via, s.res_is_via + m); R0.assign(s.res_R0, s.res_R0 + m);
        pad.assign(s.pad_node, s.pad_node + s.n_pads);
        if (s.sink_I) sink.assign(s.sink_I, s.sink_I + n);
        if (s.node_T) node_T.assign(s.node_T, s.node_T + n);
        if (s.tmap) tmap.assign(s.tmap, s.tmap + (size_t)s.tmap_nx * s.tmap_ny);
        g = s;
        g.xy = xy.data(); g.layer = layer.data(); g.res_a = ra.data(); g.res_b = rb.data();
        g.res_len = len.data(); g.res_w = w.data(); g.res_h = h.data(); g.res_is_via = via.data();
        g.res_R0 = R0.data(); g.pad_node = pad.data();
        g.sink_I = s.sink_I ? sink.data() : nullptr;
        g.node_T = s.node_T ? node_T.data() : nullptr;
        g.tmap = s.tmap ? tmap.data() : nullptr;
        g.seg_j = nullptr;
    }
};

namespace {

em_status fail(em_batch *b, em_status st, const std::string &msg)
{
    if (b) b->err = msg;
    return st;
}

#define HIPCHK(b, call)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail((b), EM_ERR_HIP, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK(b)                                                                      \
    do {                                                                                  \
        hipError_t e_ = hipGetLastError();                                                \
        if (e_ != hipSuccess)                                                             \
            return fail((b), EM_ERR_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e_)); \
    } while (0)

void *dalloc(em_batch *b, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (b->has_alloc) {
        p = b->alloc.alloc(bytes, b->alloc.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (!p) return nullptr;
    b->allocs.push_back(p);
    if (hipMemsetAsync(p, 0, bytes, b->stream) != hipSuccess) return nullptr;
    return p;
}

template <typename T>
T *upload(em_batch *b, const std::vector<T> &v)
{
    T *p = (T *)dalloc(b, v.size() * sizeof(T));
    if (!p) return nullptr;
    if (!v.empty() &&
        hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return nullptr;
    return p;
}

template <typename T>
T *upload_raw(em_batch *b, const T *src, size_t n)
{
    T *p = (T *)dalloc(b, n * sizeof(T));
    if (!p) return nullptr;
    if (n && hipMemcpyAsync(p, src, n * sizeof(T), hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return nullptr;
    return p;
}

uint8_t *pinned(em_batch *b, size_t n)
{
    if (n > b->h_flags_cap) {
        if (b->h_flags) (void)hipHostFree(b->h_flags);
        b->h_flags = nullptr;
        b->h_flags_cap = 0;
        if (hipHostMalloc((void **)&b->h_flags, n) != hipSuccess) return nullptr;
        b->h_flags_cap = n;
    }
    return b->h_flags;
}

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// --------------------------------------------------------------------------
// Wire-tree partition.  Wire segments on one layer form trees; the root is
// the lowest-index vertex, the walk is depth-first taking incident segments in
// ascending index order, and each segment is refined into N intervals whose
// FD nodes are numbered in visiting (pre-)order, so every parent precedes its
// children.  Iterative, with an explicit stack of (vertex, node, arrival
// segment, next incidence) frames.
// --------------------------------------------------------------------------
struct Partition {
    std::vector<int> tree_off, parent, seg, dir, vert, kpos, seg_tree;
    std::vector<int> inc_off, inc;   // vertex -> wire segments, ascending
};

em_status partition(em_batch *b, const em_grid_desc *g, int N, Partition &P)
{
    const int n = g->n_nodes, m = g->n_res;
    std::vector<uint8_t> wire(m);
    for (int r = 0; r < m; ++r)
        wire[r] = !g->res_is_via[r] && g->layer[g->res_a[r]] == g->layer[g->res_b[r]];
    P.inc_off.assign(n + 1, 0);
    for (int r = 0; r < m; ++r) {
        if (!wire[r]) continue;
        if (g->res_a[r] == g->res_b[r]) return fail(b, EM_ERR_ARG, "wire segment with both ends on one node");
        P.inc_off[g->res_a[r] + 1]++;
        P.inc_off[g->res_b[r] + 1]++;
    }
    for (int v = 0; v < n; ++v) P.inc_off[v + 1] += P.inc_off[v];
    P.inc.assign(P.inc_off[n], 0);
    {
        std::vector<int> pos(P.inc_off.begin(), P.inc_off.end() - 1);
        for (int r = 0; r < m; ++r) {
            if (!wire[r]) continue;
            P.inc[pos[g->res_a[r]]++] = r;
            P.inc[pos[g->res_b[r]]++] = r;
        }
    }
    P.seg_tree.assign(m, -1);
    std::vector<int> vnode(n, -1);
    struct Frame { int u, su, from, k; };
    std::vector<Frame> stack;
    P.tree_off.assign(1, 0);
    auto emit = [&](int par, int sg, int dr, int vt, int kp) {
        P.parent.push_back(par); P.seg.push_back(sg); P.dir.push_back(dr);
        P.vert.push_back(vt); P.kpos.push_back(kp);
        return (int)P.parent.size() - 1;
    };
    for (int v = 0; v < n; ++v) {
        if (vnode[v] >= 0 || P.inc_off[v + 1] == P.inc_off[v]) continue;
        int t = (int)P.tree_off.size() - 1;
        int s0 = emit(-1, -1, 0, v, 0);
        vnode[v] = s0;
        stack.clear();
        stack.push_back({v, s0, -1, P.inc_off[v]});
        while (!stack.empty()) {
            Frame &f = stack.back();
            if (f.k == P.inc_off[f.u + 1]) { stack.pop_back(); continue; }
            int e = P.inc[f.k++];
            if (e == f.from) continue;
            int a = g->res_a[e], bb = g->res_b[e];
            int u = f.u, su = f.su;
            int wv = (a == u) ? bb : a;
            if (vnode[wv] >= 0)
                return fail(b, EM_ERR_ARG, "wire component containing node " + std::to_string(u) +
                                               " has a cycle (not a tree)");
            P.seg_tree[e] = t;
            bool fwd = (a == u);
            int dr = fwd ? 1 : -1;
            int prev = su;
            for (int q = 1; q < N; ++q) prev = emit(prev, e, dr, -1, fwd ? q : N - q);
            int sw = emit(prev, e, dr, wv, fwd ? N : 0);
            vnode[wv] = sw;
            stack.push_back({wv, sw, e, P.inc_off[wv]});   // invalidates f
        }
        P.tree_off.push_back((int)P.parent.size());
        if ((long long)P.parent.size() > (1LL << 31) - 64) return fail(b, EM_ERR_ARG, "too many stress nodes");
    }
    return EM_OK;
}

em_status validate(em_batch *b, const em_grid_desc *g, const em_material *m, const em_run_params *r,
                   const em_mc_params *mc)
{
    if (!g || !m || !r) return fail(b, EM_ERR_ARG, "grid, material and run must be non-NULL");
    if (g->struct_size != sizeof(em_grid_desc) || m->struct_size != sizeof(em_material) ||
        r->struct_size != sizeof(em_run_params) || (mc && mc->struct_size != sizeof(em_mc_params)))
        return fail(b, EM_ERR_ARG, "struct_size mismatch (ABI version)");
    if (g->n_nodes <= 0 || g->n_res <= 0 || !g->xy || !g->layer || !g->res_a || !g->res_b ||
        !g->res_len || !g->res_w || !g->res_h || !g->res_is_via || !g->res_R0)
        return fail(b, EM_ERR_ARG, "netlist arrays missing or empty");
    int n_wire = 0;
    for (int i = 0; i < g->n_res; ++i) {
        int a = g->res_a[i], c = g->res_b[i];
        if (a < 0 || a >= g->n_nodes || c < 0 || c >= g->n_nodes) return fail(b, EM_ERR_ARG, "resistor node out of range");
        bool wire = !g->res_is_via[i] && g->layer[a] == g->layer[c];
        n_wire += wire ? 1 : 0;
        if (!(g->res_R0[i] > 0) || !std::isfinite(g->res_R0[i])) return fail(b, EM_ERR_ARG, "R0 must be positive and finite");
        if (wire && (!(g->res_len[i] > 0) || !(g->res_w[i] > 0) || !(g->res_h[i] > 0) ||
                     !std::isfinite(g->res_len[i]) || !std::isfinite(g->res_w[i]) || !std::isfinite(g->res_h[i])))
            return fail(b, EM_ERR_ARG, "wire geometry must be positive and finite");
    }
    if (n_wire == 0) return fail(b, EM_ERR_ARG, "no wire segment (every resistor is a via): nothing to age");
    if (!finite_all(g->xy, 2 * (size_t)g->n_nodes)) return fail(b, EM_ERR_ARG, "non-finite coordinates");
    if (g->node_T && !finite_all(g->node_T, g->n_nodes)) return fail(b, EM_ERR_ARG, "non-finite node_T");
    if (g->tmap) {
        if (g->tmap_nx < 1 || g->tmap_ny < 1 || !(g->tmap_dx > 0) || !(g->tmap_dy > 0))
            return fail(b, EM_ERR_ARG, "bad thermal raster");
        if (!finite_all(g->tmap, (size_t)g->tmap_nx * g->tmap_ny)) return fail(b, EM_ERR_ARG, "non-finite tmap");
    }
    if (g->seg_j) {
        if (!finite_all(g->seg_j, g->n_res)) return fail(b, EM_ERR_ARG, "non-finite seg_j");
    } else {
        if (g->n_pads <= 0 || !g->pad_node || !g->sink_I) return fail(b, EM_ERR_ARG, "coupled mode needs pads and sinks");
        for (int k = 0; k < g->n_pads; ++k)
            if (g->pad_node[k] < 0 || g->pad_node[k] >= g->n_nodes) return fail(b, EM_ERR_ARG, "pad out of range");
        if (!finite_all(g->sink_I, g->n_nodes)) return fail(b, EM_ERR_ARG, "non-finite sinks");
        if (!(g->vdd > 0)) return fail(b, EM_ERR_ARG, "vdd must be positive");
    }
    const double mv[] = {m->B, m->Omega, m->Z, m->rho_cu, m->Ea_eV, m->D0, m->sigma_crit, m->Q_eV,
                         m->sigma_T, m->delta, m->rho_ta, m->h_ta};
    if (!finite_all(mv, 12) || !(m->B > 0) || !(m->Omega > 0) || !(m->delta > 0) || !(m->D0 > 0) || !(m->h_ta > 0))
        return fail(b, EM_ERR_ARG, "bad material constants");
    if (r->intervals_per_seg < 1 || !(r->dt > 0) || !std::isfinite(r->dt) || r->n_steps < 0 || r->ir_every < 1 ||
        r->cg_max_iter < 1 || !(r->cg_rtol >= 0) || !std::isfinite(r->cg_rtol) ||
        (r->prec != EM_FP64 && r->prec != EM_FP32) ||
        r->max_voids_per_tree < 0 || r->max_voids_per_tree > MAXV || !(r->T_ambient > 0) ||
        r->stepper < 0 || r->stepper > 1 || r->ir_precond < 0 || r->ir_precond > 2 ||
        r->ir_launch < 0 || r->ir_launch > 3 || r->joule < 0 || r->joule > 1 ||
        !(r->dt_growth >= 0) || !std::isfinite(r->dt_growth) || !(r->guard_band >= 0) || !(r->guard_band < 1) ||
        !(r->guard_ttf >= 0) || !std::isfinite(r->guard_ttf) ||
        !(r->amg_alpha == 0.0 || (r->amg_alpha >= 1.0 && r->amg_alpha <= 4.0)) ||
        !(r->ss_tol >= 0) || !(r->ss_tol <= 1e-2) || r->krylov_q < 0 || r->krylov_q > KRY_RM_MAX / 2 ||
        !(r->krylov_eta >= 0) || !(r->krylov_eta <= 100.0))
        return fail(b, EM_ERR_ARG, "bad run parameters (max_voids_per_tree <= 4, 0 <= guard_band < 1, "
                                   "guard_ttf >= 0, amg_alpha 0 or in [1, 4], 0 <= ss_tol <= 1e-2, "
                                   "0 <= krylov_q <= 8, 0 <= krylov_eta <= 100)");
    if (r->krylov_q > 0 && r->ss_tol > 0)
        return fail(b, EM_ERR_ARG, "reduced (Krylov) stepping and steady-state skipping are exclusive");
    if (r->dt_adapt < 0 || r->dt_adapt > 12)
        return fail(b, EM_ERR_ARG, "bad run parameters (0 <= dt_adapt <= 12)");
    if (r->dt_adapt > 0 && r->dt_growth > 0 && r->dt_growth != 1.0)
        return fail(b, EM_ERR_ARG, "the adaptive and the graded time grids are exclusive");
    if (r->joule) {
        const double tv[] = {m->k_cu, m->k_ild, m->t_ild};
        if (!finite_all(tv, 3) || !(m->k_cu > 0) || !(m->k_ild > 0) || !(m->t_ild > 0))
            return fail(b, EM_ERR_ARG, "Joule pre-pass needs positive finite k_cu, k_ild and t_ild");
    }
    if (mc && (mc->n_samples < 1 || mc->n_samples > 65535 || mc->cov_kappa < 0 || mc->cov_scrit < 0 || !std::isfinite(mc->cov_kappa) ||
               !std::isfinite(mc->cov_scrit) || !(mc->cov_rho >= 0) || !(mc->cov_load >= 0) ||
               !std::isfinite(mc->cov_rho) || !std::isfinite(mc->cov_load) || !(mc->sd_ea_eV >= 0) ||
               !(mc->sd_ea_eV < 1.0) || !(mc->sd_T_K >= 0) || !(mc->sd_T_K <= 20.0) ||
               !(mc->cov_map >= 0) || !(mc->cov_map <= 1.0)))
        return fail(b, EM_ERR_ARG, "bad Monte Carlo parameters");
    if (mc && mc->cov_map > 0 && r->joule)
        return fail(b, EM_ERR_ARG, "a thermal-map amplitude spread cannot be combined with the Joule pre-pass");
    if (mc && mc->sample_ids)
        for (int s = 0; s < mc->n_samples; ++s)
            if (mc->sample_ids[s] < 0) return fail(b, EM_ERR_ARG, "Monte Carlo sample indices must be >= 0");
    return EM_OK;
}

em_status update_forcing(em_batch *b);

// After a solve of sample 0 for identical samples: its voltages, reachability,
// drop and currents, and (condensed) the reduced system it solved, become
// every sample's, so that later solves can skip unchanged samples.
em_status bcast_ir_state(em_batch *b, Dev &X)
{
    Dev &d = b->d;
    hipStream_t st = b->stream;
    const int S = d.S;
    launch_bcast0_f64(d.u, d.n_nodes, S, st);
    launch_bcast0_u8(d.live, d.n_nodes, S, st);
    launch_bcast0_f64(d.drop, 1, S, st);
    launch_bcast0_f64(d.jseg, d.n_res, S, st);
    if (b->condensed) {
        launch_bcast0_f64(X.G, X.n_res, S, st);
        launch_bcast0_f64(X.u, X.n_nodes, S, st);
        launch_bcast0_u8(X.live, X.n_nodes, S, st);
        launch_bcast0_f64(X.sink_s, X.n_nodes, S, st);
        launch_bcast0_f64(b->cond.cinj, 2LL * b->cond.n_chain, S, st);
    }
    LAUNCHCHK(b);
    return EM_OK;
}

em_status ir_solve_impl(em_batch *b)
{
    Dev &d = b->d;
    hipStream_t st = b->stream;
    HIPCHK(b, hipMemsetAsync(d.g_changed, 0, 4, st));
    // Per-sample change flags: samples whose conductances are those of the
    // last solve keep its solution (every sample counts as changed when the
    // state was replaced since: creation, reset, restore, set_seg_state).
    // When every sample carries the nominal network and the same warm start,
    // one solve (sample 0) serves all of them and its state is copied.
    const bool uniform = b->nominal && !b->ir_valid && d.S > 1;
    HIPCHK(b, hipMemsetAsync(d.g_chg_s, (b->ir_valid || uniform) ? 0 : 1, d.S, st));
    if (uniform) HIPCHK(b, hipMemsetAsync(d.g_chg_s, 1, 1, st));
    launch_ir_conductance(d, st);
    LAUNCHCHK(b);
    if (b->ir_valid && !b->live_dirty) {
        // no conductance changed since the last solve: its solution stands
        uint32_t *hg = (uint32_t *)pinned(b, std::max<size_t>(d.S, 8));
        if (!hg) return fail(b, EM_ERR_OOM, "pinned host buffer");
        HIPCHK(b, hipMemcpyAsync(hg, d.g_changed, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(b, hipStreamSynchronize(st));
        if (*hg == 0) {
            b->cg_iters_last = 0;
            b->ir_unchanged = true;
            return EM_OK;
        }
    }
    b->ir_unchanged = false;
    // the system the PCG iterates (with chain condensation: its terminals,
    // whose conductances, sinks and warm start the chain reduction forms)
    Dev &X = b->condensed ? b->rd : d;
    if (b->condensed) {
        launch_chain_reduce(d, X, b->cond, st);
        LAUNCHCHK(b);
    }
    if (b->live_dirty && !b->any_open && b->live0) {
        launch_ir_live_copy(X, b->live0, st);     // nothing open: the static reachability holds
        LAUNCHCHK(b);
        b->live_dirty = false;
    }
    if (b->live_dirty) {
        // connected components of the conducting network; labels only
        // decrease, so the rounds end (in practice after a few)
        launch_ir_cc_init(X, st);
        uint32_t *hc = (uint32_t *)pinned(b, std::max<size_t>(d.S, 8));
        if (!hc) return fail(b, EM_ERR_OOM, "pinned host buffer");
        for (int round = 0;; ++round) {
            HIPCHK(b, hipMemsetAsync(X.live_changed, 0, 4, st));
            launch_ir_cc_round(X, st);
            launch_ir_cc_round(X, st);
            LAUNCHCHK(b);
            HIPCHK(b, hipMemcpyAsync(hc, X.live_changed, 4, hipMemcpyDeviceToHost, st));
            HIPCHK(b, hipStreamSynchronize(st));
            if (*hc == 0) break;
            if (round > X.n_nodes) return fail(b, EM_ERR_HIP, "reachability did not settle");
        }
        launch_ir_cc_finish(X, st);
        LAUNCHCHK(b);
        b->live_dirty = false;
    }
    const double rtol = b->run.cg_rtol;
    const bool amg = b->use_amg;
    launch_ir_gather_inc(X, b->n_inc, st);
    launch_ir_setup(X, st);
    launch_ir_finalize0(X, rtol, st);
    if (uniform) launch_ir_only_sample0(X, st);
    LAUNCHCHK(b);
    uint8_t *hconv = pinned(b, std::max<size_t>(d.S, 8));
    if (!hconv) return fail(b, EM_ERR_OOM, "pinned host buffer");
    if (b->ir_wg) {
        // one workgroup per sample runs the whole PCG; converged samples exit
        HIPCHK(b, hipMemcpyAsync(hconv, X.conv, X.S, hipMemcpyDeviceToHost, st));
        HIPCHK(b, hipStreamSynchronize(st));
        bool all = true;
        for (int s = 0; s < X.S; ++s) all &= hconv[s] != 0;
        int itmax = 0;
        if (!all) {
            launch_amg_setup(X, b->amg, st);
            if (b->ir_lds) launch_ir_pcg_lds(X, b->n_inc, b->amg, b->amg_dev, rtol, b->run.cg_max_iter, st);
            else launch_ir_pcg_wg(X, b->amg_dev, rtol, b->run.cg_max_iter, st);
            LAUNCHCHK(b);
            std::vector<int> its(X.S);
            HIPCHK(b, hipMemcpyAsync(hconv, X.conv, X.S, hipMemcpyDeviceToHost, st));
            HIPCHK(b, hipMemcpyAsync(its.data(), X.ir_iters, 4 * (size_t)X.S, hipMemcpyDeviceToHost, st));
            HIPCHK(b, hipStreamSynchronize(st));
            all = true;
            for (int s = 0; s < X.S; ++s) {
                itmax = std::max(itmax, its[s]);
                b->cg_sample_iters += its[s];
                all &= hconv[s] != 0;
            }
            b->cg_iters_last = itmax;
            if (!all) return fail(b, EM_ERR_NOCONV, "PCG did not reach cg_rtol within cg_max_iter iterations");
        }
        b->cg_iters_last = itmax;
        if (b->condensed) launch_chain_expand(d, X, b->cond, st);
        launch_ir_finish(d, st);
        if (uniform) {
            em_status rb = bcast_ir_state(b, X);
            if (rb != EM_OK) return rb;
        }
        LAUNCHCHK(b);
        b->forcing_stale = true;          // dt*f follows before the next step
        b->have_j = true;
        b->ir_valid = true;
        return EM_OK;
    }
    if (amg) {
        // samples whose warm start already meets the tolerance need no
        // preconditioner; for the others: this solve's coarse operators, then
        // z = M^-1 r, p = z and r.z
        HIPCHK(b, hipMemcpyAsync(hconv, X.conv, X.S, hipMemcpyDeviceToHost, st));
        HIPCHK(b, hipStreamSynchronize(st));
        bool all = true;
        for (int s = 0; s < X.S; ++s) all &= hconv[s] != 0;
        if (!all) {
            launch_amg_setup(X, b->amg, st);
            launch_amg_vcycle(X, b->amg, true, st);
            launch_ir_finalize_rz(X, st);
            LAUNCHCHK(b);
        }
    }
    // CG_BLOCK iterations (an even count, so the r.z parity pattern repeats)
    // are captured once on a private stream and replayed as one graph launch.
    const int CG_BLOCK = amg ? 4 : 8;
    if (!b->cg_exec) {
        if (!b->cap_stream) HIPCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        HIPCHK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < CG_BLOCK; ++k) {
            launch_ir_spmv(X, b->cap_stream);
            launch_ir_update(X, k, amg ? b->amg.omega : 0.0, b->cap_stream);
            if (amg) launch_amg_vcycle(X, b->amg, false, b->cap_stream);
            launch_ir_pupdate(X, k, rtol, X.z, b->cap_stream);
        }
        HIPCHK(b, hipStreamEndCapture(b->cap_stream, &b->cg_graph));
        HIPCHK(b, hipGraphInstantiate(&b->cg_exec, b->cg_graph, nullptr, nullptr, 0));
    }
    int it = 0;
    for (;;) {
        HIPCHK(b, hipMemcpyAsync(hconv, X.conv, X.S, hipMemcpyDeviceToHost, st));
        HIPCHK(b, hipStreamSynchronize(st));
        bool all = true;
        int n_open = 0;
        for (int s = 0; s < X.S; ++s) {
            all &= hconv[s] != 0;
            n_open += hconv[s] == 0;
        }
        b->cg_sample_iters += (long long)n_open * (it > 0 ? CG_BLOCK : 0);
        if (all) break;
        if (it >= b->run.cg_max_iter) {
            b->cg_iters_last = it;
            return fail(b, EM_ERR_NOCONV, "PCG did not reach cg_rtol within cg_max_iter iterations");
        }
        HIPCHK(b, hipGraphLaunch(b->cg_exec, st));
        it += CG_BLOCK;
    }
    LAUNCHCHK(b);
    b->cg_iters_last = it;
    if (b->condensed) launch_chain_expand(d, X, b->cond, st);
    launch_ir_finish(d, st);
    if (uniform) {
        em_status rb = bcast_ir_state(b, X);
        if (rb != EM_OK) return rb;
    }
    LAUNCHCHK(b);
    b->forcing_stale = true;              // dt*f follows before the next step (active set known)
    b->have_j = true;
    b->ir_valid = true;
    return EM_OK;
}

em_status sync_open_dirty(em_batch *b)
{
    uint32_t *h = (uint32_t *)pinned(b, std::max<size_t>(b->d.S, 8));
    if (!h) return fail(b, EM_ERR_OOM, "pinned host buffer");
    HIPCHK(b, hipMemcpyAsync(h, b->d.open_dirty, 4, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    if (*h) {
        b->live_dirty = true;
        b->any_open = true;
        HIPCHK(b, hipMemsetAsync(b->d.open_dirty, 0, 4, b->stream));
    }
    return EM_OK;
}

void fold_timers(em_batch *b)
{
    float ms = 0.f;
    if (b->step_pending && hipEventElapsedTime(&ms, b->ev_a, b->ev_b) == hipSuccess) b->step_ms += ms;
    b->step_pending = false;
    if (b->replay_pending && hipEventElapsedTime(&ms, b->ev_ra, b->ev_rb) == hipSuccess) b->step_ms += ms;
    b->replay_pending = false;
    if (b->ir_pending && hipEventElapsedTime(&ms, b->ev_c, b->ev_d) == hipSuccess) b->ir_ms += ms;
    b->ir_pending = false;
}

// The steady-state screen; with the nominal resistances every sample has
// the same current densities and the steady stress is computed once per tree
// (not under resistivity variation: the electron-wind drive differs per sample).
em_status run_screen(em_batch *b, bool apply)
{
    Dev &d = b->d;
    if ((b->nominal || b->trees_only) && !d.xi_r && !d.map_a) {
        HIPCHK(b, hipMemsetAsync(d.tree_mortal, 0, (size_t)d.n_trees * d.S, b->stream));
        HIPCHK(b, hipMemsetAsync(d.seg_mortal, 0, (size_t)d.n_res * d.S, b->stream));
        launch_screen_shared(d, apply, b->stream);
        b->psi_shared = true;
    } else {
        launch_screen(d, apply, b->stream);
        b->psi_shared = false;
    }
    LAUNCHCHK(b);
    if (apply) b->act_dirty = true;
    return EM_OK;
}

// Lane layout of the chain kernel: instances of chain trees, L lanes each,
// never straddling a workgroup of cWG lanes; only the active ones when flags
// are given.  Best-fit decreasing: trees in tree_perm order (largest first),
// each tree's instances go to the open workgroups with the fewest free lanes
// that still hold one (as many per workgroup as fit), then to new ones.
// Every workgroup runs the same number of steps in about the same time, so
// fewer workgroups means fewer rounds of the chip.  Returns the lane count
// (whole workgroups) and, when asked, each placed instance's id, first lane
// and lane count.
long long place_chain_lanes(const std::vector<int> &perm, const std::vector<int> &chain_L, int S, int cWG,
                            const uint8_t *ia, const uint8_t *sa, std::vector<int> *pi,
                            std::vector<long long> *po, std::vector<int> *pL)
{
    if (pi) { pi->clear(); po->clear(); pL->clear(); }
    std::vector<std::vector<int>> open(cWG + 1);     // open[c]: workgroups with c free lanes
    std::vector<int> fill;                           // lanes used per workgroup
    std::vector<int> items;
    for (int t : perm) {
        const int L = chain_L[t];
        if (L == 0) continue;
        items.clear();
        for (int s = 0; s < S; ++s) {
            const size_t inst = (size_t)t * S + s;
            if (ia && !(ia[inst] && sa[s])) continue;
            items.push_back((int)inst);
        }
        size_t k = 0;
        auto put = [&](int wg, size_t q) {
            for (size_t r = 0; r < q; ++r, ++k) {
                if (pi) {
                    pi->push_back(items[k]);
                    po->push_back((long long)wg * cWG + fill[wg]);
                    pL->push_back(L);
                }
                fill[wg] += L;
            }
            if (cWG - fill[wg] > 0) open[cWG - fill[wg]].push_back(wg);
        };
        for (int c = L; c <= cWG && k < items.size(); ++c) {
            while (!open[c].empty() && k < items.size()) {
                const int wg = open[c].back();
                open[c].pop_back();
                put(wg, std::min(items.size() - k, (size_t)(c / L)));
            }
        }
        while (k < items.size()) {
            fill.push_back(0);
            put((int)fill.size() - 1, std::min(items.size() - k, (size_t)(cWG / L)));
        }
    }
    return (long long)fill.size() * cWG;
}

// Active-instance compaction (after the screen, the learned screen's
// deferrals and activations, a reset or a restore): the ascending list of
// active instances for the forcing update, and the chain kernel's lane table
// rebuilt over the active chain instances only (the kernel still checks the
// flags, so a superset would also be correct).  Instances that became active
// get their forcing from the present current densities.
em_status ensure_active(em_batch *b)
{
    if (!b->act_dirty) return EM_OK;
    Dev &d = b->d;
    hipStream_t st = b->stream;
    const int S = d.S;
    const size_t IS = (size_t)d.n_trees * S;
    std::vector<uint8_t> ia(IS), sa(S), cu;
    HIPCHK(b, hipMemcpyAsync(ia.data(), d.inst_active, IS, hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(sa.data(), d.sample_active, S, hipMemcpyDeviceToHost, st));
    if (b->sur_ready) {
        // instances activated by the learned screen are stepped in its
        // catch-up replay before they rejoin the active set
        cu.resize(IS);
        HIPCHK(b, hipMemcpyAsync(cu.data(), d.catchup, IS, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(b, hipStreamSynchronize(st));
    if (!cu.empty())
        for (size_t i = 0; i < IS; ++i) ia[i] |= cu[i];
    std::vector<int> lst, fresh;
    if (b->act_prev.size() != IS) b->act_prev.assign(IS, 0);
    for (size_t i = 0; i < IS; ++i) {
        const uint8_t a = ia[i] && sa[i % S];
        if (a) {
            lst.push_back((int)i);
            if (b->act_built && !b->act_prev[i]) fresh.push_back((int)i);
        }
        b->act_prev[i] = a;
    }
    b->n_act = (int)lst.size();
    if (!lst.empty())
        HIPCHK(b, hipMemcpyAsync(b->act_inst, lst.data(), 4 * lst.size(), hipMemcpyHostToDevice, st));
    // lanes: the placement rule of the full table (an instance never
    // straddles two workgroups), over the active chain instances
    const int cWG = b->chain_wg;
    std::vector<int> pi, pL;
    std::vector<long long> po;
    d.chain_wg = cWG;
    d.chain_occ = b->chain_occ;
    long long n_lanes = place_chain_lanes(b->tree_perm_h, b->chain_L, S, cWG, ia.data(), sa.data(), &pi, &po, &pL);
    if (n_lanes > b->lanes_cap)      // the full layout of any candidate size always fits
        n_lanes = place_chain_lanes(b->tree_perm_h, b->chain_L, S, cWG, nullptr, nullptr, &pi, &po, &pL);
    if (!pi.empty()) {
        HIPCHK(b, hipMemcpyAsync(b->pl_inst, pi.data(), 4 * pi.size(), hipMemcpyHostToDevice, st));
        HIPCHK(b, hipMemcpyAsync(b->pl_off, po.data(), 8 * po.size(), hipMemcpyHostToDevice, st));
        HIPCHK(b, hipMemcpyAsync(b->pl_L, pL.data(), 4 * pL.size(), hipMemcpyHostToDevice, st));
    }
    launch_place_lanes(const_cast<int *>(d.lane_inst), const_cast<int *>(d.lane_blk), n_lanes, b->pl_inst,
                       b->pl_off, b->pl_L, (int)pi.size(), st);
    d.n_chain_wg = cWG > 0 ? (int)(n_lanes / cWG) : 0;
    LAUNCHCHK(b);
    HIPCHK(b, hipMemcpyAsync(b->d_dev, &d, sizeof(Dev), hipMemcpyHostToDevice, st));
    HIPCHK(b, hipStreamSynchronize(st));          // host staging vectors go out of scope
    if (!fresh.empty() && b->have_j) {
        HIPCHK(b, hipMemcpyAsync(b->pl_inst, fresh.data(), 4 * fresh.size(), hipMemcpyHostToDevice, st));
        launch_update_f_list(d, b->fp32, b->pl_inst, (int)fresh.size(), st);
        LAUNCHCHK(b);
        HIPCHK(b, hipStreamSynchronize(st));
    }
    b->act_dirty = false;
    b->act_built = true;
    return EM_OK;
}

// dt*f from the present current densities: every node, or (when few are
// active) the nodes of the active instances only.
em_status update_forcing(em_batch *b)
{
    em_status rc = ensure_active(b);
    if (rc != EM_OK) return rc;
    Dev &d = b->d;
    if ((long long)b->n_act * 4 < (long long)d.n_trees * d.S)
        launch_update_f_list(d, b->fp32, b->act_inst, b->n_act, b->stream);
    else
        launch_update_f(d, b->fp32, b->stream);
    LAUNCHCHK(b);
    return EM_OK;
}

// Step the instances that `dd.inst_active` marks (the batch's own set, or the
// catch-up set of the learned screen with dd a modified copy of the batch's Dev).
em_status timed_step_dev(em_batch *b, const Dev &dd, int n_steps, int step0, bool void_dr = true)
{
    fold_timers(b);
    b->nominal = false;                   // voids may grow from here on
    HIPCHK(b, hipEventRecord(b->ev_a, b->stream));
    // long chains in reduced form first: an interval they take sits out the exact launch
    if (dd.kq > 0) launch_kry_step(dd, b->fp32, n_steps, b->stream);
    if (dd.n_chain_wg > 0) launch_chain(dd, b->d_dev, b->fp32, n_steps, step0, b->stream);
    if (b->n_br > 0) launch_branch(dd, b->fp32, b->n_br, b->br_max_nodes, n_steps, step0, b->stream);
    else if (b->n_generic_trees > 0) launch_step(dd, b->fp32, n_steps, step0, b->stream);
    if (dd.kq > 0) launch_kry_restore(dd, b->stream);
    LAUNCHCHK(b);
    HIPCHK(b, hipEventRecord(b->ev_b, b->stream));
    b->step_pending = true;
    b->step_launches++;
    if (void_dr) {
        launch_void_dR(b->d, b->stream);
        LAUNCHCHK(b);
    }
    return EM_OK;
}

em_status timed_step(em_batch *b, int n_steps, int step0, bool void_dr = true)
{
    em_status rc = ensure_active(b);
    if (rc != EM_OK) return rc;
    if (b->forcing_stale) {
        rc = update_forcing(b);
        if (rc != EM_OK) return rc;
        b->forcing_stale = false;
    }
    return timed_step_dev(b, b->d, n_steps, step0, void_dr);
}

em_status timed_ir(em_batch *b)
{
    HIPCHK(b, hipEventRecord(b->ev_c, b->stream));
    em_status st = ir_solve_impl(b);
    if (st != EM_OK) return st;
    if (b->d.kq > 0 && !b->ir_unchanged) launch_kry_invalidate(b->d, false, b->stream);   // new drive
    HIPCHK(b, hipEventRecord(b->ev_d, b->stream));
    b->ir_pending = true;
    b->cg_iters_total += b->cg_iters_last;
    return EM_OK;
}

// Device buffers of the learned screen (the per-interval current-density
// history for the catch-up replay included) and the per-tree static features.
em_status sur_buffers(em_batch *b)
{
    if (b->sur_ready) return EM_OK;
    if (!b->trees_only) {
        const int n_hist = (b->run.n_steps + b->run.ir_every - 1) / b->run.ir_every;
        b->jhist = (double *)dalloc(b, 8 * (size_t)std::max(n_hist, 1) * b->S * b->n_res);
        if (!b->jhist) return fail(b, EM_ERR_OOM, "current-density history");
        b->n_hist = n_hist;
    }
    Dev &d = b->d;
    const size_t IS = (size_t)d.n_trees * d.S;
    d.tstat = (double *)dalloc(b, 4 * 8 * (size_t)d.n_trees);
    d.rdist = (double *)dalloc(b, 8 * (size_t)d.ns);
    d.feat = (float *)dalloc(b, 4 * IS * NFEAT);
    d.yhat = (float *)dalloc(b, 4 * IS);
    d.deferred = (uint8_t *)dalloc(b, IS);
    d.catchup = (uint8_t *)dalloc(b, IS);
    d.def_list = (int *)dalloc(b, 4 * IS);
    d.def_k = (int *)dalloc(b, 4 * IS);
    d.sur_viol = (uint8_t *)dalloc(b, (size_t)d.S);
    d.act_list = (int *)dalloc(b, 4 * IS);
    d.sur_cnt = (unsigned int *)dalloc(b, 32);
    b->sur_y = (float *)dalloc(b, 4 * IS);
    if (!d.tstat || !d.rdist || !d.feat || !d.yhat || !d.deferred || !d.catchup || !d.def_list || !d.def_k ||
        !d.sur_viol ||
        !d.act_list || !d.sur_cnt || !b->sur_y)
        return fail(b, EM_ERR_OOM, "learned-screen buffers");
    if (!b->rp_stream) HIPCHK(b, hipStreamCreateWithFlags(&b->rp_stream, hipStreamNonBlocking));
    if (!b->ev_j) HIPCHK(b, hipEventCreate(&b->ev_j));
    if (!b->ev_ra) HIPCHK(b, hipEventCreate(&b->ev_ra));
    if (!b->ev_rb) HIPCHK(b, hipEventCreate(&b->ev_rb));
    launch_tree_static(d, b->stream);
    LAUNCHCHK(b);
    HIPCHK(b, hipMemcpyAsync(b->d_dev, &d, sizeof(Dev), hipMemcpyHostToDevice, b->stream));
    b->sur_ready = true;
    return EM_OK;
}

// Features of every (tree, sample) with the current densities: the screen's
// steady stress is refreshed first (without changing the active set); after a
// shared screen the features read its column 0.
em_status features_impl(em_batch *b, float *X, bool screen_current = false, bool candidates_only = false)
{
    if (!screen_current) {
        em_status rc = run_screen(b, false);
        if (rc != EM_OK) return rc;
    }
    launch_features(b->d, X, candidates_only, b->psi_shared, b->stream);
    LAUNCHCHK(b);
    return EM_OK;
}

// A deferred instance is re-evaluated once one of its segment currents has
// moved by more than this fraction of its largest since its last prediction
// (a 1 % change moves a nucleation time that scales as 1/j^2 by about 2 %).
constexpr double REEVAL_TOL = 0.01;

// Evaluate the attached model and defer the mortal active instances predicted
// to nucleate after thr; returns how many were deferred (synchronises).
em_status sur_evaluate(em_batch *b, double thr, int64_t *n_def, bool screen_current)
{
    Dev &d = b->d;
    auto t0 = std::chrono::steady_clock::now();
    em_status rc = features_impl(b, d.feat, screen_current, true);
    if (rc != EM_OK) return rc;
    int irc = mlp_forward_async(b->sur, d.feat, d.n_trees * d.S, b->sur_y, b->stream);
    if (irc != EM_OK) return fail(b, (em_status)irc, "learned-screen model evaluation failed");
    HIPCHK(b, hipMemsetAsync(d.sur_cnt, 0, 32, b->stream));
    launch_defer(d, b->sur_y, thr, b->stream);
    LAUNCHCHK(b);
    b->act_dirty = true;
    unsigned int *h = (unsigned int *)pinned(b, 32);
    if (!h) return fail(b, EM_ERR_OOM, "pinned host buffer");
    HIPCHK(b, hipMemcpyAsync(h, d.sur_cnt, 32, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    if (n_def) *n_def = h[0];
    b->n_def_list = (int)h[4];
    if (b->n_def_list > 0) {
        // the deferred list in instance order, so that the re-evaluations read
        // the [node][sample] arrays of one tree's samples together
        const size_t IS = (size_t)d.n_trees * d.S;
        std::vector<uint8_t> df(IS);
        HIPCHK(b, hipMemcpy(df.data(), d.deferred, IS, hipMemcpyDeviceToHost));
        std::vector<int> lst;
        lst.reserve(b->n_def_list);
        for (size_t i = 0; i < IS; ++i) if (df[i]) lst.push_back((int)i);
        b->n_def_list = (int)lst.size();
        HIPCHK(b, hipMemcpy(d.def_list, lst.data(), 4 * lst.size(), hipMemcpyHostToDevice));
        HIPCHK(b, hipMemset(d.def_k, 0xff, 4 * lst.size()));      // rows still by instance: evaluate all
    }
    b->sur_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return EM_OK;
}

// Catch-up of the instances just activated before interval k: their lanes
// join the lane table, the main set's forcing is brought up to date, then the
// stored aging intervals 0..k (interval k: nst steps with the present
// densities) are replayed for them on the replay stream, beside the main
// launch of interval k (which steps only the already active instances; the
// two sets share no node, segment or void).  sur_catch_up_end joins the two.
em_status sur_catch_up_begin(em_batch *b, int k, int n_new, int nst)
{
    Dev &d = b->d;
    const int K = b->run.ir_every;
    b->act_dirty = true;                  // the activated (catch-up) instances join the lane table
    em_status rc = ensure_active(b);
    if (rc != EM_OK) return rc;
    if (b->forcing_stale) {
        rc = update_forcing(b);
        if (rc != EM_OK) return rc;
        b->forcing_stale = false;
    }
    fold_timers(b);
    b->nominal = false;
    HIPCHK(b, hipEventRecord(b->ev_j, b->stream));
    HIPCHK(b, hipStreamWaitEvent(b->rp_stream, b->ev_j, 0));
    Dev dr = d;
    dr.inst_active = d.catchup;
    HIPCHK(b, hipEventRecord(b->ev_ra, b->rp_stream));
    for (int i = 0; i <= k; ++i) {
        dr.jseg = b->jhist + (size_t)i * d.S * d.n_res;
        launch_update_f_list(dr, b->fp32, d.act_list, n_new, b->rp_stream);
        LAUNCHCHK(b);
        const int n = i < k ? K : nst;
        if (dr.n_chain_wg > 0) launch_chain(dr, b->d_dev, b->fp32, n, i * K, b->rp_stream);
        if (b->n_br > 0) launch_branch(dr, b->fp32, b->n_br, b->br_max_nodes, n, i * K, b->rp_stream);
        else if (b->n_generic_trees > 0) launch_step(dr, b->fp32, n, i * K, b->rp_stream);
        LAUNCHCHK(b);
        b->step_launches++;
    }
    HIPCHK(b, hipEventRecord(b->ev_rb, b->rp_stream));
    return EM_OK;
}

// After the main launch of interval k: wait for the replays, return the
// caught-up instances to the active set (counting late activations) and
// update the resistances from every void.
em_status sur_catch_up_end(em_batch *b, int k)
{
    Dev &d = b->d;
    HIPCHK(b, hipStreamWaitEvent(b->stream, b->ev_rb, 0));
    b->replay_pending = true;
    launch_catchup_done(d, k * b->run.ir_every, b->stream);
    launch_void_dR(d, b->stream);
    LAUNCHCHK(b);
    return EM_OK;
}

}  // namespace

extern "C" {

const char *em_last_error(const em_batch *b)
{
    return b ? b->err.c_str() : "null batch";
}

// One-time thermal pre-pass (Sec. III-A): currents of the nominal network (one
// IR solve, or the prescribed densities) -> per-tree vertex temperatures and
// per-segment steady profiles -> node temperatures; the coefficients that
// depend on temperature (diffusivity, thermomigration drive, the factor, and
// in trees-only mode the forcing) are rebuilt from them, and the dynamic
// state returns to t = 0.
static em_status joule_prepass(em_batch *b)
{
    Dev &d = b->d;
    hipStream_t st = b->stream;
    if (!b->trees_only) {
        // the nominal network: sampled resistivity and loading left out
        double *xr = d.xi_r, *ss = d.sink_s;
        d.xi_r = nullptr; d.sink_s = nullptr;
        b->nominal = true;
        em_status s = em_ir_solve(b, nullptr);
        d.xi_r = xr; d.sink_s = ss;
        if (s != EM_OK) return s;
    }
    double *scr = (double *)dalloc(b, 16 * (size_t)d.ns);
    if (!scr) return fail(b, EM_ERR_OOM, "device allocation");
    launch_joule_T(d, d.jseg, scr, scr + d.ns, st);     // sample 0's currents
    launch_edge_static(d, st);
    if (b->trees_only) launch_update_f(d, b->fp32, st);
    LAUNCHCHK(b);
    if (!b->trees_only) return em_reset(b);              // refactors, voltages back to vdd
    launch_factor(d, b->fp32, st);
    LAUNCHCHK(b);
    HIPCHK(b, hipStreamSynchronize(st));
    return EM_OK;
}

em_status em_batch_create(const em_grid_desc *g, const em_material *m, const em_run_params *r,
                          const em_mc_params *mc, const em_allocator *alloc, void *hip_stream,
                          em_batch **out)
{
    if (!out) return EM_ERR_ARG;
    *out = nullptr;
    em_batch *b = new (std::nothrow) em_batch();
    if (!b) return EM_ERR_OOM;
    *out = b;                       // returned even on failure so em_last_error works
    em_status st = validate(b, g, m, r, mc);
    if (st != EM_OK) return st;
    b->mat = *m;
    b->run = *r;
    if (b->run.cg_rtol == 0.0)        // automatic: 1e-11 with FP64 stepping, 1e-8 with FP32
        b->run.cg_rtol = r->prec == EM_FP32 ? 1e-8 : 1e-11;
    b->S = mc ? mc->n_samples : 1;
    b->seed = mc ? mc->seed : 0;
    b->cov_k = mc ? mc->cov_kappa : 0.0;
    b->cov_s = mc ? mc->cov_scrit : 0.0;
    b->trees_only = g->seg_j != nullptr;
    b->cov_r = mc ? mc->cov_rho : 0.0;
    b->cov_l = (mc && !b->trees_only) ? mc->cov_load : 0.0;     // no sinks in trees-only mode
    b->sd_ea = mc ? mc->sd_ea_eV : 0.0;
    b->sd_T = mc ? mc->sd_T_K : 0.0;
    b->cov_map = mc ? mc->cov_map : 0.0;
    b->fp32 = r->prec == EM_FP32;
    if (mc && mc->sample_ids) b->sid_h.assign(mc->sample_ids, mc->sample_ids + mc->n_samples);
    b->stream = (hipStream_t)hip_stream;
    if (alloc && alloc->alloc && alloc->free) { b->alloc = *alloc; b->has_alloc = true; }

    const int N = r->intervals_per_seg;
    Partition P;
    st = partition(b, g, N, P);
    if (st != EM_OK) return st;
    b->n_nodes = g->n_nodes; b->n_res = g->n_res; b->N = N;
    b->n_trees = (int)P.tree_off.size() - 1;
    b->ns = (int)P.parent.size();
    if (b->n_trees == 0) return fail(b, EM_ERR_ARG, "netlist has no wire segment");
    b->tree_off = P.tree_off; b->parent = P.parent; b->seg = P.seg; b->dir = P.dir;
    b->vert = P.vert; b->kpos = P.kpos; b->seg_tree = P.seg_tree;
    const int ns = b->ns, nt = b->n_trees, S = b->S, nr = g->n_res, nn = g->n_nodes;
    for (int t = 0; t < nt; ++t) b->max_tree_nodes = std::max(b->max_tree_nodes, P.tree_off[t + 1] - P.tree_off[t]);
    // element counts of the [node][sample], [resistor][sample], [sample][node]
    // and per-incidence arrays stay below 2^31 (the kernels' 32-bit element
    // arithmetic); larger Monte Carlo studies run as several batches over
    // disjoint em_mc_params.sample_ids
    const long long lim = (1LL << 31) - (1LL << 20);
    if ((long long)nt * S > lim || (long long)ns * S > lim || (long long)g->n_res * S > lim ||
        (long long)g->n_nodes * S > lim || 2LL * g->n_res * S > lim)
        return fail(b, EM_ERR_ARG, "batch too large: stress nodes, resistors or incidences x samples must stay "
                                   "below 2^31 (split the samples over batches with em_mc_params.sample_ids)");

    // children of each stress node, ascending
    std::vector<int> child_off(ns + 1, 0), child;
    for (int i = 0; i < ns; ++i) if (P.parent[i] >= 0) child_off[P.parent[i] + 1]++;
    for (int i = 0; i < ns; ++i) child_off[i + 1] += child_off[i];
    child.assign(child_off[ns], 0);
    {
        std::vector<int> pos(child_off.begin(), child_off.end() - 1);
        for (int i = 0; i < ns; ++i) if (P.parent[i] >= 0) child[pos[P.parent[i]]++] = i;
    }
    // segments of each tree
    std::vector<int> tseg_off(nt + 1, 0), tseg;
    for (int e = 0; e < nr; ++e) if (P.seg_tree[e] >= 0) tseg_off[P.seg_tree[e] + 1]++;
    for (int t = 0; t < nt; ++t) tseg_off[t + 1] += tseg_off[t];
    tseg.assign(tseg_off[nt], 0);
    {
        std::vector<int> pos(tseg_off.begin(), tseg_off.end() - 1);
        for (int e = 0; e < nr; ++e) if (P.seg_tree[e] >= 0) tseg[pos[P.seg_tree[e]]++] = e;
    }
    // via map: a vertex with an inter-layer resistor to a strictly higher layer
    std::vector<uint8_t> via_up(nn, 0), is_wire(nr, 0), is_pad(nn, 0);
    for (int e = 0; e < nr; ++e) {
        int a = g->res_a[e], c = g->res_b[e];
        is_wire[e] = !g->res_is_via[e] && g->layer[a] == g->layer[c];
        if (is_wire[e]) continue;
        if (g->layer[c] > g->layer[a]) via_up[a] = 1;
        if (g->layer[a] > g->layer[c]) via_up[c] = 1;
    }
    if (!b->trees_only)
        for (int k = 0; k < g->n_pads; ++k) is_pad[g->pad_node[k]] = 1;
    // node incidence over all resistors (IR)
    std::vector<int> ninc_off(nn + 1, 0), ninc_res, ninc_nbr;
    for (int e = 0; e < nr; ++e) { ninc_off[g->res_a[e] + 1]++; ninc_off[g->res_b[e] + 1]++; }
    for (int v = 0; v < nn; ++v) ninc_off[v + 1] += ninc_off[v];
    ninc_res.assign(ninc_off[nn], 0); ninc_nbr.assign(ninc_off[nn], 0);
    {
        std::vector<int> pos(ninc_off.begin(), ninc_off.end() - 1);
        for (int e = 0; e < nr; ++e) {
            int a = g->res_a[e], c = g->res_b[e];
            ninc_res[pos[a]] = e; ninc_nbr[pos[a]++] = c;
            ninc_res[pos[c]] = e; ninc_nbr[pos[c]++] = a;
        }
    }
    // static reachability from the pads (breadth-first over every resistor)
    std::vector<uint8_t> live0(nn, 0);
    {
        std::vector<int> queue;
        for (int v = 0; v < nn; ++v) if (is_pad[v]) { live0[v] = 1; queue.push_back(v); }
        for (size_t q = 0; q < queue.size(); ++q) {
            int v = queue[q];
            for (int k = ninc_off[v]; k < ninc_off[v + 1]; ++k) {
                int u = ninc_nbr[k];
                if (!live0[u]) { live0[u] = 1; queue.push_back(u); }
            }
        }
    }
    // lane slots: larger trees first so a wavefront of trees has similar sizes
    std::vector<int> tree_perm(nt);
    for (int t = 0; t < nt; ++t) tree_perm[t] = t;
    std::stable_sort(tree_perm.begin(), tree_perm.end(), [&](int x, int y) {
        return (P.tree_off[x + 1] - P.tree_off[x]) > (P.tree_off[y + 1] - P.tree_off[y]);
    });
    // Chains (every FD node's parent is its predecessor: a straight wire
    // rooted at an end) that fit one workgroup go to the resident chain
    // kernel; instances are packed into workgroups without straddling.
    const int cWGmax = b->fp32 ? CHAIN_WG32 : CHAIN_WG64;
    std::vector<uint8_t> tree_chain(nt, 0);
    std::vector<int> chain_L(nt, 0);
    int need = 1;
    auto chain_layout = [&](int cM) {
        std::fill(tree_chain.begin(), tree_chain.end(), 0);
        std::fill(chain_L.begin(), chain_L.end(), 0);
        need = 1;
        if (r->stepper != 0) return;
        for (int t = 0; t < nt; ++t) {
            int i0 = P.tree_off[t], i1 = P.tree_off[t + 1];
            const int L = (i1 - i0 + cM - 1) / cM;
            if (L > cWGmax) continue;
            bool chain = true;
            for (int i = i0 + 1; i < i1 && chain; ++i) chain = P.parent[i] == i - 1;
            tree_chain[t] = chain;
            if (chain) { chain_L[t] = L; need = std::max(need, L); }
        }
    };
    // nodes per lane: 8, or in FP32 9 where every layout needs 1024-lane
    // workgroups (one per compute unit) and the 9-node blocks take fewer
    // rounds of the chip, weighting a round by its block length
    int cM = b->fp32 ? CHAIN_M32 : CHAIN_M64;
    if (r->chain_m != 0 && r->chain_m != cM && !(b->fp32 && r->chain_m == CHAIN_M32W))
        return fail(b, EM_ERR_ARG, "chain_m must be 0, 8, or 9 (FP32 with 1024-lane workgroups)");
    chain_layout(cM);
    const bool wide_ok = b->fp32 && (r->chain_wg == 0 || r->chain_wg == CHAIN_WG32);
    if (r->chain_m == CHAIN_M32W) {
        if (!wide_ok) return fail(b, EM_ERR_ARG, "chain_m 9 needs 1024-lane workgroups");
        cM = CHAIN_M32W;
        chain_layout(cM);
    } else if (r->chain_m == 0 && wide_ok && need > CHAIN_WG32 / 2) {
        int n_cu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
            n_cu = 256;
        const long long r8 = (place_chain_lanes(tree_perm, chain_L, S, CHAIN_WG32, nullptr, nullptr, nullptr,
                                                nullptr, nullptr) / CHAIN_WG32 + n_cu - 1) / n_cu;
        chain_layout(CHAIN_M32W);
        const long long r9 = (place_chain_lanes(tree_perm, chain_L, S, CHAIN_WG32, nullptr, nullptr, nullptr,
                                                nullptr, nullptr) / CHAIN_WG32 + n_cu - 1) / n_cu;
        if (r9 * CHAIN_M32W < r8 * CHAIN_M32) cM = CHAIN_M32W;
        else chain_layout(cM);
    }
    // workgroup sizes that hold the longest chain tree; by default the
    // smallest of 256 or more (64 and 128 lanes are candidates of the
    // autotuner and the caller) unless the caller (or the autotuner) names one
    std::vector<int> wg_cand;
    for (int w = 64; w <= cWGmax; w *= 2)
        if (w >= need && (cM == CHAIN_M32 || cM == CHAIN_M64 || w == CHAIN_WG32)) wg_cand.push_back(w);
    int cWG = wg_cand.back();
    for (int w : wg_cand)
        if (w >= 256) { cWG = w; break; }
    if (r->chain_wg != 0) {
        if (std::find(wg_cand.begin(), wg_cand.end(), r->chain_wg) == wg_cand.end())
            return fail(b, EM_ERR_ARG, "chain_wg must be a power of two from 64 to the precision's maximum "
                                       "(1024 FP32, 512 FP64) holding the longest chain tree");
        cWG = r->chain_wg;
    }
    if (r->chain_occ != 0 && r->chain_occ != 1 &&
        !(r->chain_occ == 4 && b->fp32 && cWG <= 512) &&
        !(r->chain_occ == 3 && b->fp32 && (cWG == 256 || cWG == 512)))
        return fail(b, EM_ERR_ARG, "chain_occ must be 0, 1, 3 (FP32 with 256 or 512 lanes) or 4 (FP32 with "
                                   "64 to 512 lanes)");
    // placement of each chain instance: first lane (global) and lane count;
    // the per-lane table itself is expanded on the device.  The table is
    // allocated for the largest of the candidate sizes' layouts.
    std::vector<int> place_inst, place_L;
    std::vector<long long> place_off;
    long long lanes_cap = 0;
    for (int w : wg_cand)
        lanes_cap = std::max(lanes_cap, place_chain_lanes(tree_perm, chain_L, S, w, nullptr, nullptr,
                                                          nullptr, nullptr, nullptr));
    const long long n_lanes = place_chain_lanes(tree_perm, chain_L, S, cWG, nullptr, nullptr,
                                                &place_inst, &place_off, &place_L);

    Dev &d = b->d;
    d.n_nodes = nn; d.n_res = nr; d.n_trees = nt; d.ns = ns; d.N = N; d.S = S;
    d.n_pads = b->trees_only ? 0 : g->n_pads;
    d.max_voids = r->max_voids_per_tree;
    d.dt = r->dt; d.vdd = g->vdd;
    d.B = m->B; d.Omega = m->Omega; d.Z = m->Z; d.rho = m->rho_cu; d.Ea_eV = m->Ea_eV; d.D0 = m->D0;
    d.scrit = m->sigma_crit; d.Q_eV = m->Q_eV; d.sigT = m->sigma_T; d.delta = m->delta;
    d.rho_ta = m->rho_ta; d.h_ta = m->h_ta;
    d.T_amb = r->T_ambient;
    d.k_cu = m->k_cu; d.k_ild = m->k_ild; d.t_ild = m->t_ild;

#define UP(dst, vec) do { auto *p_ = upload(b, vec); if (!p_) return fail(b, EM_ERR_OOM, "device upload"); dst = p_; } while (0)
#define UPR(dst, src, n) do { auto *p_ = upload_raw(b, src, n); if (!p_) return fail(b, EM_ERR_OOM, "device upload"); dst = p_; } while (0)
#define AL(dst, T, n) do { dst = (T *)dalloc(b, sizeof(T) * (size_t)(n)); if (!dst) return fail(b, EM_ERR_OOM, "device allocation"); } while (0)

    UPR(d.xy, g->xy, 2 * (size_t)nn);
    UPR(d.layer, g->layer, nn);
    UPR(d.ra, g->res_a, nr); UPR(d.rb, g->res_b, nr);
    UPR(d.len, g->res_len, nr); UPR(d.w, g->res_w, nr); UPR(d.h, g->res_h, nr); UPR(d.R0, g->res_R0, nr);
    UP(d.is_wire, is_wire); UP(d.is_pad, is_pad);
    if (g->sink_I) UPR(d.sink, g->sink_I, nn);
    else { double *z; AL(z, double, nn); d.sink = z; }
    UP(d.ninc_off, ninc_off); UP(d.ninc_res, ninc_res); UP(d.ninc_nbr, ninc_nbr);
    d.node_T = nullptr; d.tmap = nullptr;
    if (g->tmap) {
        UPR(d.tmap, g->tmap, (size_t)g->tmap_nx * g->tmap_ny);
        d.tnx = g->tmap_nx; d.tny = g->tmap_ny;
        d.tx0 = g->tmap_x0; d.ty0 = g->tmap_y0; d.tdx = g->tmap_dx; d.tdy = g->tmap_dy;
    } else if (g->node_T) {
        UPR(d.node_T, g->node_T, nn);
    }
    d.seg_j_in = nullptr;
    if (g->seg_j) UPR(d.seg_j_in, g->seg_j, nr);
    UP(d.tree_off, P.tree_off); UP(d.parent, P.parent); UP(d.seg, P.seg); UP(d.dir, P.dir);
    {
        std::vector<int> ntree(ns);
        for (int t = 0; t < nt; ++t)
            for (int i = P.tree_off[t]; i < P.tree_off[t + 1]; ++i) ntree[i] = t;
        UP(d.ntree, ntree);
    }
    UP(d.vert, P.vert); UP(d.kpos, P.kpos);
    UP(d.child_off, child_off); UP(d.child, child);
    UP(d.vinc_off, P.inc_off); UP(d.vinc, P.inc);
    UP(d.tseg_off, tseg_off); UP(d.tseg, tseg);
    UP(d.via_up, via_up); UP(d.tree_perm, tree_perm); UP(d.tree_chain, tree_chain);
    if (r->ss_tol > 0 && S >= 64) {
        // steady-state skipping with many samples: chunks of the chain trees
        std::vector<int> coff(nt + 1, 0), ctree, cstart;
        for (int t = 0; t < nt; ++t) {
            coff[t] = (int)ctree.size();
            if (!tree_chain[t]) continue;
            for (int i = P.tree_off[t]; i < P.tree_off[t + 1]; i += SS_CL) {
                ctree.push_back(t);
                cstart.push_back(i);
            }
        }
        coff[nt] = (int)ctree.size();
        d.ss_nc = (int)ctree.size();
        UP(d.ss_coff, coff);
        if (d.ss_nc > 0) {
            UP(d.ss_ctree, ctree);
            UP(d.ss_cstart, cstart);
        }
    }
    if (r->krylov_q > 0) {
        // reduced stepping: the chain instances of at least max(3q, 30) nodes (eq. 27)
        const int q = r->krylov_q;
        std::vector<int> kl;
        for (int t = 0; t < nt; ++t)
            if (tree_chain[t] && P.tree_off[t + 1] - P.tree_off[t] >= std::max(3 * q, 30))
                for (int s = 0; s < S; ++s) kl.push_back(t * S + s);
        d.kq = q;
        d.krm = 2 * q;
        d.keta = r->krylov_eta > 0 ? r->krylov_eta : 1.0;
        d.n_kry_list = (int)kl.size();
        const size_t ISk = (size_t)nt * S;
        if (!kl.empty()) {
            UP(d.kry_list, kl);
            AL(d.kv, double, (size_t)d.krm * ns * S);
            AL(d.kred, double, ISk * KRY_KS(d.krm));
            AL(d.kscr, double, 3 * (size_t)ns * S);
            AL(d.kbl, int, kl.size());
            AL(d.kfl, int, kl.size());
            AL(d.kze, double, ISk * d.krm);
            AL(d.kdist, double, ISk);
        }
        AL(d.kbn, unsigned int, 2);
        HIPCHK(b, hipMemsetAsync(d.kbn, 0, 2 * sizeof(unsigned int), b->stream));
        AL(d.kr, int, ISk);
        AL(d.kdone, uint8_t, ISk);
        AL(d.kcnt, unsigned long long, 4 * KRY_CNT_SLOTS);
        HIPCHK(b, hipMemsetAsync(d.kr, 0, 4 * ISk, b->stream));
        HIPCHK(b, hipMemsetAsync(d.kdone, 0, ISk, b->stream));
        HIPCHK(b, hipMemsetAsync(d.kcnt, 0, 4 * KRY_CNT_SLOTS * sizeof(unsigned long long), b->stream));
    }
    if (lanes_cap / 256 > (1LL << 30)) return fail(b, EM_ERR_ARG, "batch too large");
    d.n_chain_wg = (int)(n_lanes / cWG);
    b->n_generic_trees = 0;
    for (int t = 0; t < nt; ++t) b->n_generic_trees += tree_chain[t] ? 0 : 1;
    // Heavy-path order of the other trees for the workgroup tree kernel
    // (stepper 0): a node's path continues through its child with the
    // largest subtree (lowest index on ties); paths are listed by light
    // depth (the number of path changes from the root), head to bottom.
    if (r->stepper == 0 && b->n_generic_trees > 0) {
        std::vector<int> br_tree, br_nlev, br_lvl0, br_lvl, br_node(ns, 0), br_heavy(ns, -1), sz(ns, 0), ld(ns, 0);
        for (int t = 0; t < nt; ++t) {
            if (tree_chain[t]) continue;
            const int i0 = P.tree_off[t], i1 = P.tree_off[t + 1];
            for (int i = i1 - 1; i >= i0; --i) {
                sz[i] += 1;
                if (P.parent[i] >= 0) sz[P.parent[i]] += sz[i];
            }
            for (int i = i0; i < i1; ++i) {
                int h = -1;
                for (int k = child_off[i]; k < child_off[i + 1]; ++k) {
                    const int c = child[k];
                    if (h < 0 || sz[c] > sz[h]) h = c;
                }
                br_heavy[i] = h;
            }
            int nlev = 1;
            std::vector<std::vector<int>> heads(1);
            heads[0].push_back(i0);
            ld[i0] = 0;
            for (int i = i0 + 1; i < i1; ++i) {
                const int p = P.parent[i];
                ld[i] = ld[p] + (br_heavy[p] == i ? 0 : 1);
                if (br_heavy[p] != i) {
                    if (ld[i] >= nlev) { nlev = ld[i] + 1; heads.resize(nlev); }
                    heads[ld[i]].push_back(i);
                }
            }
            br_tree.push_back(t);
            b->br_max_nodes = std::max(b->br_max_nodes, i1 - i0);
            br_nlev.push_back(nlev);
            br_lvl0.push_back((int)br_lvl.size());
            int pos = i0;
            for (int L = 0; L < nlev; ++L) {
                br_lvl.push_back(pos - i0);
                for (int h : heads[L])
                    for (int i = h; i >= 0; i = br_heavy[i]) br_node[pos++] = i;
            }
            br_lvl.push_back(pos - i0);
            if (pos != i1) return fail(b, EM_ERR_HIP, "heavy-path order does not cover the tree");
        }
        b->n_br = (int)br_tree.size();
        UP(d.br_tree, br_tree); UP(d.br_nlev, br_nlev); UP(d.br_lvl0, br_lvl0); UP(d.br_lvl, br_lvl);
        UP(d.br_node, br_node); UP(d.br_heavy, br_heavy);
    }
    b->chain_wg = cWG;
    b->chain_m = cM;
    d.chain_m = cM;
    b->chain_occ = (r->chain_occ == 4 || r->chain_occ == 3) ? r->chain_occ : 1;
    b->wg_cand = wg_cand;
    b->lanes_cap = lanes_cap;
    b->tree_perm_h = tree_perm;
    b->chain_L = chain_L;
    d.chain_wg = cWG;
    d.chain_occ = b->chain_occ;
    {
        const size_t ISb = (size_t)nt * S;
        AL(b->act_inst, int, ISb); AL(b->pl_inst, int, ISb); AL(b->pl_L, int, ISb);
        AL(b->res_cnt, int, 2 * (size_t)S);
        AL(b->pl_off, long long, ISb);
    }
    {
        int *li, *lb;
        AL(li, int, lanes_cap); AL(lb, int, lanes_cap);
        const int *pi, *pL;
        const long long *po;
        UP(pi, place_inst); UP(po, place_off); UP(pL, place_L);
        launch_place_lanes(li, lb, n_lanes, pi, po, pL, (int)place_inst.size(), b->stream);
        LAUNCHCHK(b);
        d.lane_inst = li; d.lane_blk = lb;
    }

    const size_t rs = b->fp32 ? 4 : 8;
    const size_t NS = (size_t)ns * S, RS = (size_t)nr * S, IS = (size_t)nt * S, VS = (size_t)nn * S;
    AL(d.T, double, ns); AL(d.V, double, ns); AL(d.g0, double, ns); AL(d.rob0, double, ns);
    AL(d.gdx0, double, ns); AL(d.mdrv, double, ns); AL(d.tree_V, double, nt);
    d.Vr = dalloc(b, rs * ns);
    d.sigma = dalloc(b, rs * NS); d.dtf = dalloc(b, rs * NS); d.dinv = dalloc(b, rs * NS);
    d.sig_lo = nullptr;
    if (b->fp32) {
        d.sig_lo = (float *)dalloc(b, 4 * NS);
        if (!d.sig_lo) return fail(b, EM_ERR_OOM, "device allocation");
    }
    d.lfac = dalloc(b, rs * NS); d.sc = dalloc(b, rs * NS);
    if (!d.Vr || !d.sigma || !d.dtf || !d.dinv || !d.lfac || !d.sc) return fail(b, EM_ERR_OOM, "device allocation");
    AL(d.psi, double, NS);
    if (b->n_generic_trees > 0) { AL(d.wsp, double, NS); } else { d.wsp = nullptr; }
    AL(d.xi_k, double, RS); AL(d.xi_s, double, RS);
    d.xi_r = nullptr;
    if (b->cov_r > 0) AL(d.xi_r, double, RS);
    d.map_a = nullptr;
    if (b->cov_map > 0) AL(d.map_a, double, S);
    d.sink_s = nullptr;
    if (b->cov_l > 0) AL(d.sink_s, double, (size_t)S * nn);
    AL(d.jseg, double, RS);
    if (S > 1) AL(d.jT, double, RS);
    AL(d.dR, double, RS); AL(d.open, uint8_t, RS); AL(d.seg_mortal, uint8_t, RS);
    AL(d.inst_active, uint8_t, IS); AL(d.tree_mortal, uint8_t, IS); AL(d.nv, int, IS);
    AL(d.vnode, int, IS * MAXV); AL(d.vseg, int, IS * MAXV); AL(d.vphase, int, IS * MAXV);
    AL(d.vstep, int, IS * MAXV); AL(d.vearly, int, IS * MAXV);
    AL(d.vvol, double, IS * MAXV); AL(d.vlen, double, IS * MAXV); AL(d.vrob, double, IS * MAXV);
    AL(d.n_suppressed, int, IS);
    AL(d.sample_active, uint8_t, S); AL(d.open_dirty, uint32_t, 1);
    d.ev_cap = 1 << 20;
    AL(d.events, int, (size_t)d.ev_cap * EV_WORDS); AL(d.ev_count, unsigned int, 1);
    AL(d.node_steps, unsigned long long, NS_SLOTS);
    HIPCHK(b, hipEventCreate(&b->ev_a)); HIPCHK(b, hipEventCreate(&b->ev_b));
    HIPCHK(b, hipEventCreate(&b->ev_c)); HIPCHK(b, hipEventCreate(&b->ev_d));
    AL(d.G, double, RS); AL(d.u, double, VS);
    AL(d.live, uint8_t, VS); AL(d.g_changed, uint32_t, 1); AL(d.g_chg_s, uint8_t, S);
    d.ir_nblk = (nn + ir_nodes_per_block() - 1) / ir_nodes_per_block();
    AL(d.part, double, (size_t)S * d.ir_nblk * 4);
    AL(d.drop, double, S);
    AL(d.ttf, double, S); AL(d.final_drop, double, S); AL(d.init_drop, double, S);
    AL(d.t_prev, double, S); AL(d.d_prev, double, S); AL(d.failed, int, S); AL(d.outer_idx, int, S);
    AL(d.guard, uint8_t, S);
    d.guard_band = (b->fp32 && !b->trees_only) ? r->guard_band : 0.0;
    d.guard_ttf = d.guard_band > 0 ? r->guard_ttf : 0.0;
    d.sid = nullptr;
    if (!b->sid_h.empty()) UP(d.sid, b->sid_h);
    if (!b->trees_only) {            // for the guard-band and learned-screen re-runs
        b->gcopy = new (std::nothrow) GridCopy(*g);
        if (!b->gcopy) return fail(b, EM_ERR_OOM, "host copy of the netlist");
    }

    // The system the PCG iterates: the nodal network, or (multigrid on the
    // condensed network) its terminals with one reduced edge per two-ended
    // chain.
    CondHost C;
    if (!b->trees_only && r->ir_precond == 2) {
        // condensed only where it removes at least a quarter of the nodes:
        // below that the extra chain passes cost more than they save.  A
        // reduction to isolated terminals (every chain dangling, as on a
        // single pad feeding open-ended wires) leaves no system to iterate:
        // the nodal one is solved instead.
        C = cond_build(nn, nr, g->res_a, g->res_b, g->res_R0, is_pad.data());
        b->condensed = (long long)C.n_term * 4 <= (long long)nn * 3 && !C.red_a.empty();
    }
    Dev &X = b->condensed ? b->rd : d;
    int xn = nn, xr = nr;
    std::vector<int> xoff, xres, xnbr, xra, xrb;
    std::vector<uint8_t> xpad, xlive0;
    std::vector<double> xR0;
    if (b->condensed) {
        xn = C.n_term;
        xr = (int)C.red_a.size();
        xra = C.red_a; xrb = C.red_b; xR0 = C.red_R0; xpad = C.red_pad;
        xlive0.assign(xn, 0);
        for (int t = 0; t < xn; ++t) xlive0[t] = live0[C.term_node[t]];
        xoff.assign(xn + 1, 0);
        for (int e = 0; e < xr; ++e) { xoff[xra[e] + 1]++; xoff[xrb[e] + 1]++; }
        for (int v = 0; v < xn; ++v) xoff[v + 1] += xoff[v];
        xres.assign(xoff[xn], 0); xnbr.assign(xoff[xn], 0);
        {
            std::vector<int> pos(xoff.begin(), xoff.end() - 1);
            for (int e = 0; e < xr; ++e) {
                xres[pos[xra[e]]] = e; xnbr[pos[xra[e]]++] = xrb[e];
                xres[pos[xrb[e]]] = e; xnbr[pos[xrb[e]]++] = xra[e];
            }
        }
        Cond &c = b->cond;
        c.n_term = xn; c.n_chain = C.n_chain;
        UP(c.term_node, C.term_node); UP(c.eoff, C.eoff); UP(c.e, C.e); UP(c.voff, C.voff); UP(c.v, C.v);
        UP(c.cA, C.cA); UP(c.cB, C.cB); UP(c.cred, C.cred); UP(c.tce_off, C.tce_off); UP(c.tce, C.tce);
        AL(c.cinj, double, (size_t)S * C.n_chain * 2);
        X.n_nodes = xn; X.n_res = xr; X.S = S; X.vdd = g->vdd;
        X.sample_active = d.sample_active;
        UP(X.ra, xra); UP(X.rb, xrb); UP(X.is_pad, xpad);
        UP(X.ninc_off, xoff); UP(X.ninc_res, xres); UP(X.ninc_nbr, xnbr);
        X.sink = nullptr;
        AL(X.sink_s, double, (size_t)S * xn);
        AL(X.G, double, (size_t)S * xr); AL(X.u, double, (size_t)S * xn); AL(X.live, uint8_t, (size_t)S * xn);
        b->n_term = xn; b->n_redge = xr; b->n_cchain = C.n_chain;
    } else {
        xoff = ninc_off; xpad = is_pad; xlive0 = live0;
        xra.assign(g->res_a, g->res_a + nr); xrb.assign(g->res_b, g->res_b + nr);
        xR0.assign(g->res_R0, g->res_R0 + nr);
    }
    UP(b->live0, xlive0);
    const size_t XS = (size_t)S * xn;
    AL(X.G_inc, double, (size_t)S * xoff[xn]);
    b->n_inc = xoff[xn];
    AL(X.diag, double, XS); AL(X.rhs, double, XS); AL(X.r, double, XS);
    AL(X.z, double, XS); AL(X.p, double, XS); AL(X.q, double, XS);
    AL(X.live_changed, uint32_t, 1);
    AL(X.cc_label, int, (size_t)S * (xn + 1));
    if (b->condensed) {
        X.ir_nblk = (xn + ir_nodes_per_block() - 1) / ir_nodes_per_block();
        AL(X.part, double, (size_t)S * X.ir_nblk * 4);
    }
    AL(X.rz, double, 2 * (size_t)S); AL(X.bb, double, S); AL(X.conv, uint8_t, S);
    AL(X.ir_iters, int, S);
    if (!b->trees_only && r->ir_precond >= 1) {
        AmgHost H = amg_build(xn, xpad.data(), xr, xra.data(), xrb.data(), xR0.data());
        Amg &a = b->amg;
        a.nlev = (int)H.lev.size() - 1;
        if (a.nlev >= 1) {
            a.l0.ne0 = (int)H.e0_res.size();
            UP(a.l0.e0_res, H.e0_res); UP(a.l0.e0_a, H.e0_a); UP(a.l0.e0_b, H.e0_b);
            AL(a.l0.w0, mgreal, XS);
            for (int l = 1; l <= a.nlev; ++l) {
                const AmgHostLevel &h = H.lev[l];
                AmgLevel &L = a.lev[l];
                L.n = h.n; L.ne = h.ne; L.nf = h.nf; L.nef = h.nef; L.nmem = (int)h.mem.size();
                UP(L.agg, h.agg); UP(L.mem_off, h.mem_off); UP(L.mem, h.mem);
                UP(L.int_off, h.int_off); UP(L.int_e, h.int_e);
                UP(L.src_off, h.src_off); UP(L.src_e, h.src_e);
                UP(L.adj_off, h.adj_off); UP(L.adj_nbr, h.adj_nbr); UP(L.adj_e, h.adj_e);
                AL(L.D, mgreal, (size_t)S * h.n); AL(L.W, mgreal, (size_t)S * std::max(h.ne, 1));
                AL(L.Wa, mgreal, (size_t)S * std::max(2 * h.ne, 1));
                AL(L.b, mgreal, (size_t)S * h.n); AL(L.x, mgreal, (size_t)S * h.n);
                AL(L.y, mgreal, (size_t)S * h.n); AL(L.w, mgreal, (size_t)S * h.n);
            }
            const int nc = a.lev[a.nlev].n;
            a.dense = nc <= AMG_NC_MAX ? 1 : 0;
            if (a.dense) AL(a.Ainv, mgreal, (size_t)S * nc * nc);
            b->use_amg = true;
            a.omega = 0.9;          // Jacobi weight and coarse-correction scale chosen by
            a.alpha = r->amg_alpha > 0 ? r->amg_alpha : 1.4;   // measurement (PCG iterations)
            // one workgroup per sample pays off when the samples fill the chip
            // or the system is small; a single large system keeps every CU busy
            // only in the one-kernel-per-step form
            b->ir_wg = r->ir_launch >= 2 ||
                       (r->ir_launch == 0 && (xn <= 4096 || (S >= 32 && xn <= ir_wg_max_nodes())));
            // from LDS when the sample's system and hierarchy fit a workgroup
            b->ir_lds = b->ir_wg && r->ir_launch != 3 && ir_lds_bytes(X, xoff[xn], a) > 0;
            b->amg_dev = (Amg *)dalloc(b, sizeof(Amg));
            if (!b->amg_dev) return fail(b, EM_ERR_OOM, "device allocation");
            HIPCHK(b, hipMemcpyAsync(b->amg_dev, &a, sizeof(Amg), hipMemcpyHostToDevice, b->stream));
        }
    }

    hipStream_t stq = b->stream;
    b->d_dev = (Dev *)dalloc(b, sizeof(Dev));
    if (!b->d_dev) return fail(b, EM_ERR_OOM, "device allocation");
    HIPCHK(b, hipMemcpyAsync(b->d_dev, &d, sizeof(Dev), hipMemcpyHostToDevice, stq));
    HIPCHK(b, hipMemsetAsync(d.inst_active, 1, IS, stq));
    HIPCHK(b, hipMemsetAsync(d.sample_active, 1, S, stq));
    launch_fill_f64(d.u, VS, g->vdd, stq);
    launch_node_T(d, stq);
    launch_edge_static(d, stq);
    launch_node_V(d, b->fp32, stq);
    launch_draws(d, b->seed, b->cov_k, b->cov_s, b->cov_r, b->cov_l, b->sd_ea, b->sd_T, b->cov_map, stq);
    b->nominal = !d.xi_r && !d.sink_s;
    launch_node_sc(d, b->fp32, stq);
    launch_set_sigma_T(d, b->fp32, stq);
    LAUNCHCHK(b);
    if (b->trees_only) {
        for (int s = 0; s < S; ++s)
            HIPCHK(b, hipMemcpyAsync(d.jseg + (size_t)s * nr, d.seg_j_in, nr * 8, hipMemcpyDeviceToDevice, stq));
        launch_update_f(d, b->fp32, stq);
        b->have_j = true;
    }
    launch_factor(d, b->fp32, stq);
    LAUNCHCHK(b);
    HIPCHK(b, hipStreamSynchronize(stq));
    if (r->joule) {
        em_status js = joule_prepass(b);
        if (js != EM_OK) return js;
    }
    return EM_OK;
#undef UP
#undef UPR
#undef AL
}

em_status em_batch_destroy(em_batch *b)
{
    if (!b) return EM_OK;
    if (b->stream || !b->allocs.empty()) (void)hipStreamSynchronize(b->stream);
    for (void *p : b->allocs) {
        if (b->has_alloc) b->alloc.free(p, b->alloc.ctx);
        else (void)hipFree(p);
    }
    if (b->h_flags) (void)hipHostFree(b->h_flags);
    for (hipEvent_t e : {b->ev_a, b->ev_b, b->ev_c, b->ev_d, b->ev_j, b->ev_ra, b->ev_rb})
        if (e) (void)hipEventDestroy(e);
    if (b->rp_stream) (void)hipStreamDestroy(b->rp_stream);
    if (b->cg_exec) (void)hipGraphExecDestroy(b->cg_exec);
    if (b->cg_graph) (void)hipGraphDestroy(b->cg_graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b->gcopy;
    delete b;
    return EM_OK;
}

em_status em_get_info(em_batch *b, em_info *info)
{
    if (!b || !info) return EM_ERR_ARG;
    info->n_trees = b->n_trees; info->n_stress = b->ns; info->n_samples = b->S;
    info->n_nodes = b->n_nodes; info->n_res = b->n_res; info->max_tree_nodes = b->max_tree_nodes;
    info->prec = b->fp32 ? EM_FP32 : EM_FP64; info->trees_only = b->trees_only ? 1 : 0;
    unsigned int cnt = 0;
    if (b->d.ev_count) {
        HIPCHK(b, hipMemcpyAsync(&cnt, b->d.ev_count, 4, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(b, hipStreamSynchronize(b->stream));
    }
    info->n_events = cnt;
    info->cg_iters_last = b->cg_iters_last;
    info->n_outer_done = b->n_outer_done;
    unsigned long long nsd = 0, nss[NS_SLOTS];
    HIPCHK(b, hipMemcpyAsync(nss, b->d.node_steps, sizeof nss, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    for (int k = 0; k < NS_SLOTS; ++k) nsd += nss[k];
    fold_timers(b);
    info->node_steps = (int64_t)nsd + b->rerun_node_steps;
    info->step_launches = b->step_launches;
    info->step_kernel_ms = b->step_ms;
    info->cg_iters_total = b->cg_iters_total;
    info->ir_ms = b->ir_ms;
    info->cg_sample_iters = b->cg_sample_iters;
    info->chain_m = b->chain_m;
    info->chain_wg = b->chain_wg;
    info->n_chain_wg = b->d.n_chain_wg;
    info->ir_sys_nodes = b->condensed ? b->n_term : b->n_nodes;
    info->ir_sys_edges = b->condensed ? b->n_redge : b->n_res;
    unsigned int sc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (b->sur_ready) {
        HIPCHK(b, hipMemcpyAsync(sc, b->d.sur_cnt, 32, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(b, hipStreamSynchronize(b->stream));
    }
    info->n_deferred = sc[0];
    info->n_activated = sc[1];
    info->n_late = sc[2];
    info->n_violations = sc[3];
    info->surrogate_ms = b->sur_ms;
    info->n_redecided = b->n_redecided;
    info->n_screen_rerun = b->n_screen_rerun;
    info->n_ss_skipped = b->n_ss_skipped;
    info->n_ss_woken = b->n_ss_woken;
    {
        unsigned long long kc[4] = {0, 0, 0, 0};
        if (b->d.kq > 0) {
            std::vector<unsigned long long> slots(4 * KRY_CNT_SLOTS);
            HIPCHK(b, hipMemcpyAsync(slots.data(), b->d.kcnt, slots.size() * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost, b->stream));
            HIPCHK(b, hipStreamSynchronize(b->stream));
            for (int k = 0; k < 4; ++k)
                for (int j = 0; j < KRY_CNT_SLOTS; ++j) kc[k] += slots[(size_t)k * KRY_CNT_SLOTS + j];
        }
        info->n_krylov_bases = (int64_t)kc[0];
        info->n_krylov_intervals = (int64_t)kc[1];
        info->n_krylov_fallbacks = (int64_t)kc[2];
        info->krylov_node_steps = (int64_t)kc[3];
    }
    {
        const size_t IS = (size_t)b->n_trees * b->S;
        std::vector<int> sup(IS);
        HIPCHK(b, hipMemcpyAsync(sup.data(), b->d.n_suppressed, 4 * IS, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(b, hipStreamSynchronize(b->stream));
        long long n = 0;
        for (int v : sup) n += v;
        info->n_void_capped = n;
    }
    return EM_OK;
}

em_status em_ir_solve(em_batch *b, double *max_drop)
{
    if (!b) return EM_ERR_ARG;
    if (b->trees_only) return fail(b, EM_ERR_STATE, "trees-only batch has no IR network");
    em_status st = sync_open_dirty(b);
    if (st != EM_OK) return st;
    st = timed_ir(b);
    if (st != EM_OK) return st;
    if (max_drop) {
        HIPCHK(b, hipMemcpyAsync(max_drop, b->d.drop, 8 * (size_t)b->S, hipMemcpyDeviceToHost, b->stream));
    }
    HIPCHK(b, hipStreamSynchronize(b->stream));
    return EM_OK;
}

em_status em_screen(em_batch *b, uint8_t *tree_mortal)
{
    if (!b) return EM_ERR_ARG;
    if (!b->have_j) return fail(b, EM_ERR_STATE, "no current densities yet (call em_ir_solve first)");
    em_status rs = run_screen(b, true);
    if (rs != EM_OK) return rs;
    if (tree_mortal) {
        // device layout is [tree][sample]; output is [sample][tree]
        std::vector<uint8_t> tmp((size_t)b->n_trees * b->S);
        HIPCHK(b, hipMemcpyAsync(tmp.data(), b->d.tree_mortal, tmp.size(), hipMemcpyDeviceToHost, b->stream));
        HIPCHK(b, hipStreamSynchronize(b->stream));
        for (int t = 0; t < b->n_trees; ++t)
            for (int s = 0; s < b->S; ++s) tree_mortal[(size_t)s * b->n_trees + t] = tmp[(size_t)t * b->S + s];
    }
    HIPCHK(b, hipStreamSynchronize(b->stream));
    return EM_OK;
}

em_status em_stress_step(em_batch *b, int32_t n_steps, int32_t *n_events)
{
    if (!b || n_steps < 0) return fail(b, EM_ERR_ARG, "bad step count");
    if (!b->have_j) return fail(b, EM_ERR_STATE, "no current densities yet (call em_ir_solve first)");
    unsigned int before = 0, after = 0;
    HIPCHK(b, hipMemcpyAsync(&before, b->d.ev_count, 4, hipMemcpyDeviceToHost, b->stream));
    if (n_steps > 0) {
        em_status st = timed_step(b, n_steps, b->step_counter);
        if (st != EM_OK) return st;
        b->step_counter += n_steps;
    }
    HIPCHK(b, hipMemcpyAsync(&after, b->d.ev_count, 4, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    if (n_events) *n_events = (int32_t)(after - before);
    if (after > (unsigned)b->d.ev_cap) return fail(b, EM_ERR_OVERFLOW, "event ring overflow");
    return EM_OK;
}

// Step size of aging interval k of em_run_to_ttf (geometric time grid).
static double interval_dt(const em_batch *b, int k)
{
    const double g = b->run.dt_growth > 0 ? b->run.dt_growth : 1.0;
    return g == 1.0 ? b->run.dt : b->run.dt * std::pow(g, (double)k);
}

// A new backward-Euler step size: the generic kernel's factors and dt * f
// follow (the chain kernel factors at every launch from the step size it is
// given).
static em_status set_step_size(em_batch *b, double dt)
{
    if (b->d.dt == dt) return EM_OK;
    b->d.dt = dt;
    HIPCHK(b, hipMemcpyAsync(b->d_dev, &b->d, sizeof(Dev), hipMemcpyHostToDevice, b->stream));
    launch_factor(b->d, b->fp32, b->stream);
    LAUNCHCHK(b);
    b->forcing_stale = true;
    return EM_OK;
}

// Guard band of the FP32 form: the samples whose worst drop came within the
// band of the failure threshold are run again from t = 0 in FP64 (a batch over
// their Monte Carlo sample indices built from the same inputs); their results,
// resistance changes and opens replace the FP32 run's.
//
// The same re-run in the batch's own precision and chain-kernel layout, without
// the learned screen (fp64 false), replaces the results of the samples that a
// learned-screen violation hit; its own guard band applies as in the batch.
static em_status rerun_samples(em_batch *b, const std::vector<int> &pick, em_ttf_result *out, bool fp64)
{
    std::vector<int> ids(pick.size());
    for (size_t i = 0; i < pick.size(); ++i) ids[i] = b->sid_h.empty() ? pick[i] : b->sid_h[pick[i]];
    em_run_params r2 = b->run;
    if (fp64) {
        r2.prec = EM_FP64;
        r2.guard_band = 0.0;
        r2.guard_ttf = 0.0;
        r2.cg_rtol = std::min(r2.cg_rtol, 1e-11);     // the FP64 decision solves as tightly as FP64 runs
        r2.chain_wg = 0; r2.chain_occ = 0; r2.chain_m = 0;
    } else {
        r2.chain_wg = b->chain_wg; r2.chain_occ = b->chain_occ; r2.chain_m = b->chain_m;
    }
    if (b->use_amg) r2.amg_alpha = b->amg.alpha;     // the batch's (possibly tuned) preconditioner
    em_mc_params mc2{};
    mc2.struct_size = sizeof(em_mc_params);
    mc2.n_samples = (int)pick.size();
    mc2.seed = b->seed;
    mc2.cov_kappa = b->cov_k; mc2.cov_scrit = b->cov_s; mc2.cov_rho = b->cov_r; mc2.cov_load = b->cov_l;
    mc2.sd_ea_eV = b->sd_ea;
    mc2.sd_T_K = b->sd_T;
    mc2.cov_map = b->cov_map;
    mc2.sample_ids = ids.data();
    em_batch *sub = nullptr;
    em_status rc = em_batch_create(&b->gcopy->g, &b->mat, &r2, &mc2, b->has_alloc ? &b->alloc : nullptr,
                                   b->stream, &sub);
    std::vector<em_ttf_result> res(pick.size());
    if (rc == EM_OK) rc = em_run_to_ttf(sub, res.data());
    if (rc == EM_OK) {
        const size_t nr = b->n_res;
        for (size_t i = 0; i < pick.size() && rc == EM_OK; ++i) {
            out[pick[i]] = res[i];
            out[pick[i]].redecided = fp64 ? 1 : 2;
            if (hipMemcpyAsync(b->d.dR + pick[i] * nr, sub->d.dR + i * nr, 8 * nr, hipMemcpyDeviceToDevice,
                               b->stream) != hipSuccess ||
                hipMemcpyAsync(b->d.open + pick[i] * nr, sub->d.open + i * nr, nr, hipMemcpyDeviceToDevice,
                               b->stream) != hipSuccess)
                rc = EM_ERR_HIP;
        }
        if (rc == EM_OK && hipStreamSynchronize(b->stream) != hipSuccess) rc = EM_ERR_HIP;
    }
    const std::string msg = sub ? sub->err : std::string("batch creation");
    const int sub_redecided = sub ? sub->n_redecided : 0;
    if (rc == EM_OK) {
        em_info si{};
        if ((rc = em_get_info(sub, &si)) == EM_OK) b->rerun_node_steps += si.node_steps;
    }
    em_batch_destroy(sub);
    if (rc != EM_OK)
        return fail(b, rc, std::string(fp64 ? "FP64 re-run of the guard-band samples" :
                                              "re-run of the samples hit by a learned-screen violation") +
                               " failed: " + msg);
    if (fp64) b->n_redecided += (int)pick.size();
    else {
        b->n_screen_rerun = (int)pick.size();
        b->n_redecided += sub_redecided;
    }
    return EM_OK;
}

// Steady-state skipping: its flags and counters (allocated on first use).
static em_status ss_begin(em_batch *b)
{
    Dev &d = b->d;
    hipStream_t st = b->stream;
    const size_t IS = (size_t)d.n_trees * d.S;
    if (!b->ss_ready) {
        d.ss_skip = (uint8_t *)dalloc(b, IS);
        d.ss_cnt = (unsigned int *)dalloc(b, 8);
        if (!d.ss_skip || !d.ss_cnt) return fail(b, EM_ERR_OOM, "steady-state skipping buffers");
        if (d.ss_nc > 0) {
            d.ss_scr = (double *)dalloc(b, 8 * ((size_t)d.ss_nc * 11 * d.S + IS));
            if (!d.ss_scr) return fail(b, EM_ERR_OOM, "steady-state skipping buffers");
        }
        b->ss_ready = true;
    }
    HIPCHK(b, hipMemsetAsync(d.ss_skip, 0, IS, st));
    HIPCHK(b, hipMemsetAsync(d.ss_cnt, 0, 8, st));
    b->n_ss_skipped = b->n_ss_woken = 0;
    return EM_OK;
}

// Wakes every skipped instance (the run's end: em_stress_step and a later run
// step them again).
static em_status ss_end(em_batch *b)
{
    Dev &d = b->d;
    unsigned int c[2] = {0, 0};
    HIPCHK(b, hipMemcpyAsync(c, d.ss_cnt, 8, hipMemcpyDeviceToHost, b->stream));
    launch_ss_wake(d, true, b->stream);
    LAUNCHCHK(b);
    HIPCHK(b, hipStreamSynchronize(b->stream));
    b->n_ss_skipped = c[0];
    b->n_ss_woken = c[1];
    b->act_dirty = true;
    return EM_OK;
}

em_status em_run_to_ttf(em_batch *b, em_ttf_result *out)
{
    if (!b || !out) return fail(b, EM_ERR_ARG, "null output");
    if (b->trees_only) return fail(b, EM_ERR_STATE, "trees-only batch has no IR coupling");
    const bool graded = b->run.dt_growth > 0 && b->run.dt_growth != 1.0;
    const int amax = b->run.dt_adapt;          // adaptive grid: interval step dt 2^m, m <= amax
    if ((graded || amax > 0) && b->sur)
        return fail(b, EM_ERR_STATE, "a graded or adaptive time grid cannot be combined with the learned screen");
    const bool ssk = b->run.ss_tol > 0;
    if (ssk && b->sur)
        return fail(b, EM_ERR_STATE, "steady-state skipping cannot be combined with the learned screen");
    if (b->d.kq > 0 && b->sur)
        return fail(b, EM_ERR_STATE, "reduced (Krylov) stepping cannot be combined with the learned screen");
    Dev &d = b->d;
    hipStream_t st = b->stream;
    const int S = b->S;
    em_status rc = sync_open_dirty(b);
    if (rc != EM_OK) return rc;
    rc = timed_ir(b);
    if (rc != EM_OK) return rc;
    const double fail_frac = b->run.fail_frac;
    launch_ttf_init(d, fail_frac, st);
    if (b->run.screen) {
        rc = run_screen(b, true);
        if (rc != EM_OK) return rc;
    }
    const int n_steps = b->run.n_steps, K = b->run.ir_every;
    const bool sur = b->sur != nullptr;
    if (sur) {
        // learned screen at t = 0; the current densities of every aging
        // interval are kept for the catch-up replay of later activations
        rc = sur_buffers(b);
        if (rc != EM_OK) return rc;
        HIPCHK(b, hipMemsetAsync(d.deferred, 0, (size_t)b->n_trees * S, st));
        HIPCHK(b, hipMemsetAsync(d.sur_viol, 0, S, st));
        rc = sur_evaluate(b, b->sur_margin * std::min(K, n_steps) * b->run.dt, nullptr, b->run.screen != 0);
        if (rc != EM_OK) return rc;
    }
    const size_t cnt_off = (std::max<size_t>(S, 8) + 15) & ~(size_t)15;
    uint8_t *h = pinned(b, cnt_off + 64);
    if (!h) return fail(b, EM_ERR_OOM, "pinned host buffer");
    unsigned int *hcnt = (unsigned int *)(h + cnt_off);
    unsigned int *hss = hcnt + 8;
    unsigned int *hev = hss + 2;               // event count at the top of each interval
    unsigned int n_activated = 0, ss_seen = 0, ev_prev = 0;
    int m_adapt = 0;
    const double horizon = (double)n_steps * b->run.dt;
    if (ssk) {
        if ((rc = ss_begin(b)) != EM_OK) return rc;
        hss[0] = hss[1] = 0;
    }
    int done = 0, k = 0;
    double t_now = 0.0;                   // time at the end of the last interval
    while (amax > 0 ? t_now < horizon * (1.0 - 1e-12) : done < n_steps) {
        if (sur) {
            HIPCHK(b, hipMemcpyAsync(b->jhist + (size_t)k * S * b->n_res, d.jseg, 8 * (size_t)S * b->n_res,
                                     hipMemcpyDeviceToDevice, st));
            if (k > 0 && (k & (k - 1)) == 0 && (k & 0x55555555) != 0) {
                // activation checks before the intervals k = 1, 4, 16, 64, ...:
                // predictions of the deferred trees with the current densities
                // (only ever brought forward), then activation of those due by
                // the end of the interval before the next check (t_{4k}).  A
                // catch-up replays every interval before it one after the
                // other, at the latency of one stepping launch per interval
                // whatever the number of trees, so the checks are spaced
                // geometrically: the replays of a run add up to a third of its
                // intervals at most
                const int nl = b->n_def_list;
                if (nl > 0 && !b->ir_unchanged) {
                    launch_reeval_features(d, nl, d.feat, b->jhist, k, REEVAL_TOL, st);
                    LAUNCHCHK(b);
                    int irc = mlp_forward_async(b->sur, d.feat, nl, b->sur_y, st);
                    if (irc != EM_OK) return fail(b, (em_status)irc, "learned-screen model evaluation failed");
                    launch_yhat_min(d, nl, b->sur_y, st);
                }
                HIPCHK(b, hipMemsetAsync(d.sur_cnt + 5, 0, 4, st));
                launch_activate(d, b->sur_margin * std::min(4 * done, n_steps) * b->run.dt, st);
                LAUNCHCHK(b);
            }
            HIPCHK(b, hipMemcpyAsync(hcnt, d.sur_cnt, 32, hipMemcpyDeviceToHost, st));
        }
        HIPCHK(b, hipMemcpyAsync(h, d.sample_active, S, hipMemcpyDeviceToHost, st));
        if (ssk) HIPCHK(b, hipMemcpyAsync(hss, d.ss_cnt, 8, hipMemcpyDeviceToHost, st));
        if (amax > 0) HIPCHK(b, hipMemcpyAsync(hev, d.ev_count, 4, hipMemcpyDeviceToHost, st));
        HIPCHK(b, hipStreamSynchronize(st));
        if (amax > 0) {
            // adaptive grid: the step doubles after an interval without a new
            // nucleation (up to dt 2^amax) and returns to dt after one that had one
            if (k > 0) m_adapt = *hev != ev_prev ? 0 : std::min(m_adapt + 1, amax);
            ev_prev = *hev;
        }
        if (ssk && hss[0] + hss[1] != ss_seen) {       // skips or wakes: rebuild the lane table
            ss_seen = hss[0] + hss[1];
            b->act_dirty = true;
        }
        int n_active = 0;
        for (int s = 0; s < S; ++s) n_active += h[s] != 0;
        if (n_active == 0) break;
        int nst = std::min(K, n_steps - done);
        double dt_k = interval_dt(b, k);
        if (amax > 0) {
            // K steps of dt 2^m, the last interval shortened to end at the horizon
            dt_k = std::ldexp(b->run.dt, m_adapt);
            const double rem = horizon - t_now;
            nst = (int)std::min<double>(K, std::ceil(rem / dt_k - 1e-9));
            if (nst < 1) nst = 1;
            if (nst * dt_k > rem) dt_k = rem / nst;
        }
        if ((rc = set_step_size(b, dt_k)) != EM_OK) return rc;
        const bool catch_up = sur && hcnt[1] != n_activated;
        if (catch_up) {
            n_activated = hcnt[1];
            rc = sur_catch_up_begin(b, k, (int)hcnt[5], nst);
            if (rc != EM_OK) return rc;
        }
        rc = timed_step(b, nst, done, !catch_up);
        if (rc != EM_OK) return rc;
        if (catch_up && (rc = sur_catch_up_end(b, k)) != EM_OK) return rc;
        if (ssk) launch_ss_check(d, b->fp32, b->run.ss_tol * d.scrit, st);
        done += nst;
        t_now += nst * dt_k;
        ++k;
        rc = sync_open_dirty(b);
        if (rc != EM_OK) return rc;
        fold_timers(b);
        rc = timed_ir(b);
        if (rc != EM_OK) return rc;
        if (ssk) launch_ss_wake(d, false, st);      // samples whose currents changed
        launch_ttf_update(d, fail_frac, k, (graded || amax > 0) ? t_now : done * b->run.dt, st);
        LAUNCHCHK(b);
    }
    b->n_outer_done = k;
    if (ssk && (rc = ss_end(b)) != EM_OK) return rc;
    if ((rc = set_step_size(b, b->run.dt)) != EM_OK) return rc;   // em_stress_step steps with dt
    // per-sample results
    std::vector<double> ttf(S), fd(S), idr(S);
    std::vector<int> failed(S), oidx(S), cnt(2 * (size_t)S);
    HIPCHK(b, hipMemsetAsync(b->res_cnt, 0, 8 * (size_t)S, st));
    launch_result_counts(d, b->res_cnt, st);
    LAUNCHCHK(b);
    HIPCHK(b, hipMemcpyAsync(ttf.data(), d.ttf, 8 * S, hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(fd.data(), d.final_drop, 8 * S, hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(idr.data(), d.init_drop, 8 * S, hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(failed.data(), d.failed, 4 * S, hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(oidx.data(), d.outer_idx, 4 * S, hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(cnt.data(), b->res_cnt, 8 * (size_t)S, hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipStreamSynchronize(st));
    fold_timers(b);
    for (int s = 0; s < S; ++s) {
        em_ttf_result &o = out[s];
        o.ttf_s = ttf[s]; o.final_drop = fd[s]; o.init_drop = idr[s];
        o.failed = failed[s]; o.outer_idx = oidx[s];
        o.n_nucleated_trees = cnt[2 * (size_t)s];
        o.n_failed_segs = cnt[2 * (size_t)s + 1];
        o.redecided = 0;
    }
    b->n_redecided = 0;
    b->n_screen_rerun = 0;
    b->rerun_node_steps = 0;
    // samples a learned-screen violation hit: re-run without the screen
    std::vector<uint8_t> viol(S, 0);
    if (sur) {
        HIPCHK(b, hipMemcpyAsync(viol.data(), d.sur_viol, S, hipMemcpyDeviceToHost, st));
        HIPCHK(b, hipStreamSynchronize(st));
        std::vector<int> pick;
        for (int s = 0; s < S; ++s)
            if (viol[s]) pick.push_back(s);
        if (!pick.empty() && (rc = rerun_samples(b, pick, out, false)) != EM_OK) return rc;
    }
    if (d.guard_band > 0 && b->gcopy) {
        std::vector<uint8_t> gf(S);
        HIPCHK(b, hipMemcpyAsync(gf.data(), d.guard, S, hipMemcpyDeviceToHost, st));
        HIPCHK(b, hipStreamSynchronize(st));
        std::vector<int> pick;
        for (int s = 0; s < S; ++s)
            if (gf[s] && !viol[s]) pick.push_back(s);
        if (!pick.empty()) return rerun_samples(b, pick, out, true);
    }
    return EM_OK;
}

em_status em_reset(em_batch *b)
{
    if (!b) return EM_ERR_ARG;
    Dev &d = b->d;
    hipStream_t st = b->stream;
    const size_t IS = (size_t)d.n_trees * d.S, RS = (size_t)d.n_res * d.S, VS = (size_t)d.n_nodes * d.S;
    HIPCHK(b, hipStreamSynchronize(st));
    fold_timers(b);
    HIPCHK(b, hipMemsetAsync(d.nv, 0, 4 * IS, st));
    HIPCHK(b, hipMemsetAsync(d.n_suppressed, 0, 4 * IS, st));
    HIPCHK(b, hipMemsetAsync(d.inst_active, 1, IS, st));
    HIPCHK(b, hipMemsetAsync(d.sample_active, 1, d.S, st));
    b->act_dirty = true;
    b->nominal = !d.xi_r && !d.sink_s;     // samples differ from t = 0 under R / load variation
    HIPCHK(b, hipMemsetAsync(d.dR, 0, 8 * RS, st));
    HIPCHK(b, hipMemsetAsync(d.open, 0, RS, st));
    HIPCHK(b, hipMemsetAsync(d.ev_count, 0, 4, st));
    HIPCHK(b, hipMemsetAsync(d.node_steps, 0, 8 * NS_SLOTS, st));
    HIPCHK(b, hipMemsetAsync(d.open_dirty, 0, 4, st));
    if (b->sur_ready) {
        HIPCHK(b, hipMemsetAsync(d.deferred, 0, IS, st));
        HIPCHK(b, hipMemsetAsync(d.catchup, 0, IS, st));
        HIPCHK(b, hipMemsetAsync(d.sur_cnt, 0, 32, st));
    }
    b->n_def_list = 0;
    if (d.dt != b->run.dt) {               // a graded run left its last step size
        d.dt = b->run.dt;
        HIPCHK(b, hipMemcpyAsync(b->d_dev, &d, sizeof(Dev), hipMemcpyHostToDevice, st));
    }
    launch_fill_f64(d.u, VS, d.vdd, st);
    launch_set_sigma_T(d, b->fp32, st);
    launch_factor(d, b->fp32, st);
    LAUNCHCHK(b);
    HIPCHK(b, hipStreamSynchronize(st));
    b->sur_ms = 0.0;
    b->n_redecided = 0;
    b->n_screen_rerun = 0;
    b->rerun_node_steps = 0;
    b->n_ss_skipped = b->n_ss_woken = 0;
    if (b->ss_ready) HIPCHK(b, hipMemsetAsync(d.ss_skip, 0, IS, st));
    if (d.kq > 0) {
        HIPCHK(b, hipMemsetAsync(d.kr, 0, 4 * IS, st));
        HIPCHK(b, hipMemsetAsync(d.kdone, 0, IS, st));
        HIPCHK(b, hipMemsetAsync(d.kcnt, 0, 4 * KRY_CNT_SLOTS * sizeof(unsigned long long), st));
        HIPCHK(b, hipMemsetAsync(d.kbn, 0, 2 * sizeof(unsigned int), st));
    }
    b->live_dirty = true;
    b->any_open = false;
    b->ir_valid = false;
    b->have_j = b->trees_only;
    b->step_counter = 0;
    b->n_outer_done = 0;
    b->cg_iters_last = 0;
    b->cg_iters_total = 0;
    b->cg_sample_iters = 0;
    b->step_launches = 0;
    b->step_ms = b->ir_ms = 0.0;
    return EM_OK;
}

// The multigrid preconditioner's coarse-correction scale: the host copy, the
// device copy of the one-workgroup forms, and the captured PCG graph (whose
// launches carry it) re-captured at the next solve.
static em_status set_amg_alpha(em_batch *b, double alpha)
{
    if (!b->use_amg || b->amg.alpha == alpha) return EM_OK;
    b->amg.alpha = alpha;
    HIPCHK(b, hipMemcpyAsync(b->amg_dev, &b->amg, sizeof(Amg), hipMemcpyHostToDevice, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    if (b->cg_exec) { (void)hipGraphExecDestroy(b->cg_exec); b->cg_exec = nullptr; }
    if (b->cg_graph) { (void)hipGraphDestroy(b->cg_graph); b->cg_graph = nullptr; }
    return EM_OK;
}

em_status em_autotune(em_batch *b, int32_t n_steps, em_tune_info *out)
{
    if (!b || n_steps < 1) return fail(b, EM_ERR_ARG, "bad step count");
    if (b->step_counter != 0 || b->n_outer_done != 0)
        return fail(b, EM_ERR_STATE, "autotune needs the batch at t = 0 (just created or reset)");
    hipStream_t st = b->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(b, hipEventCreate(&e0));
    HIPCHK(b, hipEventCreate(&e1));
    auto stream_ms = [&](float &ms) -> em_status {
        HIPCHK(b, hipEventSynchronize(e1));
        HIPCHK(b, hipEventElapsedTime(&ms, e0, e1));
        return EM_OK;
    };
    em_tune_info info{};
    info.ir_ms[0] = info.ir_ms[1] = info.ir_ms[2] = -1.0;
    em_status rc = EM_OK;
    // IR launch shape: a cold solve (warm start at VDD) in each form
    if (!b->trees_only && b->use_amg) {
        double best = 1e300;
        bool best_wg = b->ir_wg, best_lds = b->ir_lds;
        const bool lds_ok = ir_lds_bytes(b->condensed ? b->rd : b->d, b->n_inc, b->amg) > 0;
        // the one-workgroup-per-sample forms are timed only where they can win:
        // one workgroup walking a system of more than ir_wg_max_nodes() (65 536)
        // nodes for fewer than 32 samples is tens of times slower than the
        // multi-kernel form
        const int xn = b->condensed ? b->n_term : b->n_nodes;
        const bool wg_ok = xn <= ir_wg_max_nodes() || b->S >= 32;
        for (int k = 0; k < 3 && rc == EM_OK; ++k) {
            if (k >= 1 && !wg_ok) break;
            if (k == 2 && !lds_ok) break;
            b->ir_wg = k >= 1;
            b->ir_lds = k == 2;
            for (int rep = 0; rep < 2 && rc == EM_OK; ++rep) {     // the first pass warms the code paths
                if ((rc = em_reset(b)) != EM_OK) break;
                HIPCHK(b, hipEventRecord(e0, st));
                if ((rc = ir_solve_impl(b)) != EM_OK) break;
                HIPCHK(b, hipEventRecord(e1, st));
                float ms = 0.f;
                if ((rc = stream_ms(ms)) != EM_OK) break;
                if (rep == 1) {
                    info.ir_ms[k] = ms;
                    if (ms < best) { best = ms; best_wg = b->ir_wg; best_lds = b->ir_lds; }
                }
            }
        }
        b->ir_wg = best_wg;
        b->ir_lds = best_lds;
        info.ir_launch = best_lds ? 2 : best_wg ? 3 : 1;
        // coarse-correction scale, in the chosen shape, unless the caller set one
        info.alpha_ms[0] = info.alpha_ms[1] = info.alpha_ms[2] = -1.0;
        if (b->run.amg_alpha == 0.0 && rc == EM_OK) {
            const double cand_a[3] = {1.4, 1.8, 2.2};
            double best_t = 1e300, best_a = b->amg.alpha;
            for (int k = 0; k < 3 && rc == EM_OK; ++k) {
                if ((rc = set_amg_alpha(b, cand_a[k])) != EM_OK) break;
                for (int rep = 0; rep < 2 && rc == EM_OK; ++rep) {
                    if ((rc = em_reset(b)) != EM_OK) break;
                    HIPCHK(b, hipEventRecord(e0, st));
                    if ((rc = ir_solve_impl(b)) != EM_OK) break;
                    HIPCHK(b, hipEventRecord(e1, st));
                    float ms = 0.f;
                    if ((rc = stream_ms(ms)) != EM_OK) break;
                    if (rep == 1) {
                        info.alpha_ms[k] = ms;
                        if (ms < best_t) { best_t = ms; best_a = cand_a[k]; }
                    }
                }
            }
            if (rc == EM_OK) rc = set_amg_alpha(b, best_a);
        }
        info.amg_alpha = b->amg.alpha;
    }
    // chain-kernel workgroup size: n_steps steps of the screened instances
    if (rc == EM_OK && b->d.n_chain_wg >= 0) {
        double best = 1e300;
        int best_w = b->chain_wg, best_o = b->chain_occ;
        std::vector<std::pair<int, int>> cand;          // (lanes, register budget)
        for (int w : b->wg_cand) {
            cand.push_back({w, 1});
            if (b->fp32 && w <= 512) cand.push_back({w, 4});
            if (b->fp32 && (w == 256 || w == 512)) cand.push_back({w, 3});
        }
        for (size_t k = 0; k < cand.size() && k < 12 && rc == EM_OK; ++k) {
            b->chain_wg = cand[k].first;
            b->chain_occ = cand[k].second;
            for (int rep = 0; rep < 2 && rc == EM_OK; ++rep) {
                if ((rc = em_reset(b)) != EM_OK) break;
                if (!b->trees_only && (rc = ir_solve_impl(b)) != EM_OK) break;
                if (b->run.screen && (rc = run_screen(b, true)) != EM_OK) break;
                b->act_dirty = true;
                if ((rc = ensure_active(b)) != EM_OK) break;
                HIPCHK(b, hipEventRecord(e0, st));
                if ((rc = timed_step(b, rep == 0 ? 1 : n_steps, 0)) != EM_OK) break;
                HIPCHK(b, hipEventRecord(e1, st));
                float ms = 0.f;
                if ((rc = stream_ms(ms)) != EM_OK) break;
                if (rep == 1) {
                    info.wg[info.n_wg] = b->chain_wg;
                    info.occ[info.n_wg] = b->chain_occ;
                    info.wg_ms[info.n_wg++] = ms;
                    if (ms < best) { best = ms; best_w = b->chain_wg; best_o = b->chain_occ; }
                }
            }
        }
        b->chain_wg = best_w;
        b->chain_occ = best_o;
        info.chain_wg = best_w;
        info.chain_occ = best_o;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != EM_OK) return rc;
    b->act_dirty = true;
    rc = em_reset(b);
    if (rc != EM_OK) return rc;
    if (out) *out = info;
    return EM_OK;
}

em_status em_get_topology(em_batch *b, int32_t *tree_off, int32_t *parent, int32_t *seg, int32_t *dir,
                          int32_t *vert, int32_t *kpos, int32_t *seg_tree)
{
    if (!b) return EM_ERR_ARG;
    auto cp = [](int32_t *dst, const std::vector<int> &v) { if (dst) std::memcpy(dst, v.data(), 4 * v.size()); };
    cp(tree_off, b->tree_off); cp(parent, b->parent); cp(seg, b->seg); cp(dir, b->dir);
    cp(vert, b->vert); cp(kpos, b->kpos); cp(seg_tree, b->seg_tree);
    return EM_OK;
}

static em_status column_io(em_batch *b, int sample, double *host, bool to_state, int which)
{
    if (!b || !host || sample < 0 || sample >= b->S) return fail(b, EM_ERR_ARG, "bad sample or buffer");
    double *buf = nullptr;
    HIPCHK(b, hipMalloc(&buf, 8 * (size_t)b->ns));
    hipError_t e = hipSuccess;
    if (to_state) e = hipMemcpyAsync(buf, host, 8 * (size_t)b->ns, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) {
        if (which < 0) launch_copy_sigma(b->d, b->fp32, sample, buf, to_state, b->stream);
        else launch_copy_node_col(b->d, b->fp32, which, sample, buf, b->stream);
        e = hipGetLastError();
    }
    if (e == hipSuccess && !to_state)
        e = hipMemcpyAsync(host, buf, 8 * (size_t)b->ns, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(b, EM_ERR_HIP, std::string("column copy: ") + hipGetErrorString(e));
    return EM_OK;
}

em_status em_get_stress(em_batch *b, int32_t sample, double *sigma) { return column_io(b, sample, sigma, false, -1); }
// A state replaced from outside the stepping leaves the reduced bases' span.
static void kry_drop_all(em_batch *b)
{
    if (b && b->d.kq > 0) launch_kry_invalidate(b->d, true, b->stream);
}

em_status em_set_stress(em_batch *b, int32_t sample, const double *sigma)
{
    kry_drop_all(b);
    return column_io(b, sample, const_cast<double *>(sigma), true, -1);
}

em_status em_get_node_state(em_batch *b, int32_t sample, double *T, double *V, double *sc)
{
    if (!b || sample < 0 || sample >= b->S) return fail(b, EM_ERR_ARG, "bad sample");
    if (T) HIPCHK(b, hipMemcpyAsync(T, b->d.T, 8 * (size_t)b->ns, hipMemcpyDeviceToHost, b->stream));
    if (V) HIPCHK(b, hipMemcpyAsync(V, b->d.V, 8 * (size_t)b->ns, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    if (sc) return column_io(b, sample, sc, false, 0);
    return EM_OK;
}

em_status em_get_voltages(em_batch *b, int32_t sample, double *u)
{
    if (!b || !u || sample < 0 || sample >= b->S) return fail(b, EM_ERR_ARG, "bad sample or buffer");
    HIPCHK(b, hipMemcpyAsync(u, b->d.u + (size_t)sample * b->n_nodes, 8 * (size_t)b->n_nodes,
                             hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    return EM_OK;
}

em_status em_get_seg_j(em_batch *b, int32_t sample, double *j)
{
    if (!b || !j || sample < 0 || sample >= b->S) return fail(b, EM_ERR_ARG, "bad sample or buffer");
    HIPCHK(b, hipMemcpyAsync(j, b->d.jseg + (size_t)sample * b->n_res, 8 * (size_t)b->n_res,
                             hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    return EM_OK;
}

em_status em_get_seg_state(em_batch *b, int32_t sample, double *dR, uint8_t *open)
{
    if (!b || sample < 0 || sample >= b->S) return fail(b, EM_ERR_ARG, "bad sample");
    if (dR) HIPCHK(b, hipMemcpyAsync(dR, b->d.dR + (size_t)sample * b->n_res, 8 * (size_t)b->n_res,
                                     hipMemcpyDeviceToHost, b->stream));
    if (open) HIPCHK(b, hipMemcpyAsync(open, b->d.open + (size_t)sample * b->n_res, (size_t)b->n_res,
                                       hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    return EM_OK;
}

em_status em_set_seg_state(em_batch *b, int32_t sample, const double *dR, const uint8_t *open)
{
    kry_drop_all(b);
    if (!b || sample < 0 || sample >= b->S || !dR || !open) return fail(b, EM_ERR_ARG, "bad sample or null state");
    if (b->trees_only) return fail(b, EM_ERR_STATE, "trees-only batch has no IR network");
    bool any = false;
    for (int e = 0; e < b->n_res; ++e) {
        if (!std::isfinite(dR[e]) || dR[e] < 0.0 || open[e] > 1) return fail(b, EM_ERR_ARG, "dR must be finite and >= 0, open 0 or 1");
        any |= open[e] != 0;
    }
    HIPCHK(b, hipStreamSynchronize(b->stream));
    HIPCHK(b, hipMemcpy(b->d.dR + (size_t)sample * b->n_res, dR, 8 * (size_t)b->n_res, hipMemcpyHostToDevice));
    HIPCHK(b, hipMemcpy(b->d.open + (size_t)sample * b->n_res, open, (size_t)b->n_res, hipMemcpyHostToDevice));
    b->live_dirty = true;
    b->any_open = b->any_open || any;
    b->ir_valid = false;
    b->nominal = false;
    return EM_OK;
}

em_status em_get_events(em_batch *b, int32_t *buf, int32_t cap, int32_t *n)
{
    if (!b || cap < 0 || (cap > 0 && !buf)) return fail(b, EM_ERR_ARG, "bad event buffer");
    unsigned int cnt = 0;
    HIPCHK(b, hipMemcpyAsync(&cnt, b->d.ev_count, 4, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    int avail = (int)std::min<unsigned int>(cnt, (unsigned)b->d.ev_cap);
    int k = std::min(avail, cap);
    if (k > 0) {
        HIPCHK(b, hipMemcpyAsync(buf, b->d.events, 4 * (size_t)k * EV_WORDS, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(b, hipStreamSynchronize(b->stream));
    }
    if (n) *n = k;
    if (cnt > (unsigned)b->d.ev_cap) return fail(b, EM_ERR_OVERFLOW, "event ring overflow");
    return EM_OK;
}

em_status em_get_voids(em_batch *b, int32_t sample, int32_t *iv, double *dv, int32_t cap, int32_t *n)
{
    if (!b || sample < 0 || sample >= b->S || cap < 0) return fail(b, EM_ERR_ARG, "bad arguments");
    const int S = b->S, nt = b->n_trees;
    std::vector<int> nv((size_t)nt * S), vn((size_t)nt * S * MAXV), vs(vn.size()), vp(vn.size()),
        vst(vn.size()), ve(vn.size());
    std::vector<double> vv(vn.size()), vl(vn.size());
    hipStream_t st = b->stream;
    HIPCHK(b, hipMemcpyAsync(nv.data(), b->d.nv, 4 * nv.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(vn.data(), b->d.vnode, 4 * vn.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(vs.data(), b->d.vseg, 4 * vn.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(vp.data(), b->d.vphase, 4 * vn.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(vst.data(), b->d.vstep, 4 * vn.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(ve.data(), b->d.vearly, 4 * vn.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(vv.data(), b->d.vvol, 8 * vn.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipMemcpyAsync(vl.data(), b->d.vlen, 8 * vn.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(b, hipStreamSynchronize(st));
    int c = 0;
    for (int t = 0; t < nt; ++t) {
        int inst = t * S + sample;
        for (int k = 0; k < nv[inst]; ++k) {
            int q = inst * MAXV + k;
            if (c < cap) {
                if (iv) {
                    int32_t *I = iv + 6 * (size_t)c;
                    I[0] = t; I[1] = vn[q]; I[2] = vs[q]; I[3] = vp[q]; I[4] = vst[q]; I[5] = ve[q];
                }
                if (dv) { dv[2 * (size_t)c] = vv[q]; dv[2 * (size_t)c + 1] = vl[q]; }
            }
            ++c;
        }
    }
    if (n) *n = c;
    return EM_OK;
}

em_status em_get_screen(em_batch *b, int32_t sample, uint8_t *tree_mortal, uint8_t *seg_mortal, double *sigma_ss)
{
    if (!b || sample < 0 || sample >= b->S) return fail(b, EM_ERR_ARG, "bad sample");
    const int S = b->S;
    hipStream_t st = b->stream;
    if (tree_mortal) {
        std::vector<uint8_t> tmp((size_t)b->n_trees * S);
        HIPCHK(b, hipMemcpyAsync(tmp.data(), b->d.tree_mortal, tmp.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(b, hipStreamSynchronize(st));
        for (int t = 0; t < b->n_trees; ++t) tree_mortal[t] = tmp[(size_t)t * S + sample];
    }
    if (seg_mortal)
        HIPCHK(b, hipMemcpyAsync(seg_mortal, b->d.seg_mortal + (size_t)sample * b->n_res, b->n_res,
                                 hipMemcpyDeviceToHost, st));
    if (sigma_ss) {
        std::vector<double> tmp((size_t)b->ns * S);
        HIPCHK(b, hipMemcpyAsync(tmp.data(), b->d.psi, 8 * tmp.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(b, hipStreamSynchronize(st));
        const int col = b->psi_shared ? 0 : sample;      // a shared screen wrote column 0 only
        for (int i = 0; i < b->ns; ++i) sigma_ss[i] = tmp[(size_t)i * S + col];
    }
    HIPCHK(b, hipStreamSynchronize(st));
    return EM_OK;
}

em_status em_inject_void(em_batch *b, int32_t sample, int32_t tree, int32_t node)
{
    kry_drop_all(b);
    if (!b || sample < 0 || sample >= b->S || tree < 0 || tree >= b->n_trees ||
        node < b->tree_off[tree] || node >= b->tree_off[tree + 1])
        return fail(b, EM_ERR_ARG, "bad void location");
    launch_inject_void(b->d, b->fp32, sample, tree, node, b->stream);
    LAUNCHCHK(b);
    HIPCHK(b, hipStreamSynchronize(b->stream));
    return EM_OK;
}

em_status em_get_failed_segments(em_batch *b, int32_t sample, int32_t *idx, int32_t cap, int32_t *n)
{
    if (!b || !n || sample < 0 || sample >= b->S || cap < 0 || (cap > 0 && !idx))
        return fail(b, EM_ERR_ARG, "bad arguments");
    std::vector<double> dR(b->n_res);
    std::vector<uint8_t> op(b->n_res);
    HIPCHK(b, hipMemcpyAsync(dR.data(), b->d.dR + (size_t)sample * b->n_res, 8 * (size_t)b->n_res,
                             hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipMemcpyAsync(op.data(), b->d.open + (size_t)sample * b->n_res, (size_t)b->n_res,
                             hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    int c = 0;
    for (int e = 0; e < b->n_res; ++e)
        if (dR[e] > 0.0 || op[e]) {
            if (c < cap) idx[c] = e;
            ++c;
        }
    *n = c;
    return EM_OK;
}

// ---- snapshot / restore -------------------------------------------------
namespace {
constexpr uint32_t SNAP_MAGIC = 0x31534d45u;    // "EMS1"

struct SnapIO {
    uint8_t *p;          // host buffer (null: size only)
    const uint8_t *q;    // restore source
    size_t cap, pos;
    bool ok = true;
};

// device <-> snapshot region of n bytes
em_status snap_dev(em_batch *b, SnapIO &io, void *dev, size_t n, bool restore)
{
    if (n == 0) return EM_OK;
    if (restore) {
        if (io.pos + n > io.cap) { io.ok = false; return EM_OK; }
        HIPCHK(b, hipMemcpy(dev, io.q + io.pos, n, hipMemcpyHostToDevice));
    } else if (io.p) {
        if (io.pos + n > io.cap) { io.ok = false; return EM_OK; }
        HIPCHK(b, hipMemcpy(io.p + io.pos, dev, n, hipMemcpyDeviceToHost));
    }
    io.pos += n;
    return EM_OK;
}

void snap_host(SnapIO &io, void *h, size_t n, bool restore)
{
    if (restore) {
        if (io.pos + n > io.cap) { io.ok = false; return; }
        std::memcpy(h, io.q + io.pos, n);
    } else if (io.p) {
        if (io.pos + n > io.cap) { io.ok = false; return; }
        std::memcpy(io.p + io.pos, h, n);
    }
    io.pos += n;
}

// The dynamic state in a fixed order (the netlist, draws and statics are
// rebuilt by em_batch_create from the same inputs).
em_status snap_walk(em_batch *b, SnapIO &io, bool restore)
{
    Dev &d = b->d;
    const size_t S = b->S, IS = (size_t)b->n_trees * S, NS = (size_t)b->ns * S, RS = (size_t)b->n_res * S,
                 VS = (size_t)b->n_nodes * S, rsz = b->fp32 ? 4 : 8, IV = IS * MAXV;
    struct Item { void *p; size_t n; } items[] = {
        {d.sigma, rsz * NS}, {d.sig_lo, d.sig_lo ? 4 * NS : 0}, {d.jseg, 8 * RS}, {d.u, 8 * VS}, {d.drop, 8 * S}, {d.dR, 8 * RS},
        {d.open, RS}, {d.inst_active, IS}, {d.tree_mortal, IS}, {d.seg_mortal, RS}, {d.sample_active, S},
        {d.nv, 4 * IS}, {d.vnode, 4 * IV}, {d.vseg, 4 * IV}, {d.vphase, 4 * IV}, {d.vstep, 4 * IV},
        {d.vearly, 4 * IV}, {d.vvol, 8 * IV}, {d.vlen, 8 * IV}, {d.vrob, 8 * IV}, {d.n_suppressed, 4 * IS},
        {d.ttf, 8 * S}, {d.final_drop, 8 * S}, {d.init_drop, 8 * S}, {d.t_prev, 8 * S}, {d.d_prev, 8 * S},
        {d.failed, 4 * S}, {d.outer_idx, 4 * S}, {d.node_steps, 8 * NS_SLOTS}, {d.ev_count, 4}};
    for (const Item &it : items) {
        em_status rc = snap_dev(b, io, it.p, it.n, restore);
        if (rc != EM_OK) return rc;
    }
    return EM_OK;
}
}  // namespace

em_status em_snapshot(em_batch *b, void *host_buf, size_t cap, size_t *used)
{
    if (!b || !used) return fail(b, EM_ERR_ARG, "null argument");
    HIPCHK(b, hipStreamSynchronize(b->stream));
    uint32_t hdr[12] = {SNAP_MAGIC, 1u, (uint32_t)b->n_trees, (uint32_t)b->ns, (uint32_t)b->S,
                        (uint32_t)b->n_nodes, (uint32_t)b->n_res, b->fp32 ? 1u : 0u, (uint32_t)MAXV,
                        (uint32_t)b->step_counter, (uint32_t)b->n_outer_done, b->have_j ? 1u : 0u};
    unsigned int nev = 0;
    HIPCHK(b, hipMemcpy(&nev, b->d.ev_count, 4, hipMemcpyDeviceToHost));
    const size_t ev_bytes = 4 * (size_t)EV_WORDS * std::min<unsigned int>(nev, (unsigned int)b->d.ev_cap);
    SnapIO io{(uint8_t *)host_buf, nullptr, host_buf ? cap : 0, 0};
    snap_host(io, hdr, sizeof hdr, false);
    em_status rc = snap_walk(b, io, false);
    if (rc != EM_OK) return rc;
    rc = snap_dev(b, io, b->d.events, ev_bytes, false);
    if (rc != EM_OK) return rc;
    *used = io.pos;
    if (host_buf && !io.ok) return fail(b, EM_ERR_ARG, "snapshot buffer too small (see *used)");
    return EM_OK;
}

em_status em_restore(em_batch *b, const void *host_buf, size_t n)
{
    kry_drop_all(b);
    if (!b || !host_buf) return fail(b, EM_ERR_ARG, "null argument");
    uint32_t hdr[12];
    if (n < sizeof hdr) return fail(b, EM_ERR_ARG, "snapshot too short");
    std::memcpy(hdr, host_buf, sizeof hdr);
    if (hdr[0] != SNAP_MAGIC || hdr[1] != 1u || hdr[2] != (uint32_t)b->n_trees || hdr[3] != (uint32_t)b->ns ||
        hdr[4] != (uint32_t)b->S || hdr[5] != (uint32_t)b->n_nodes || hdr[6] != (uint32_t)b->n_res ||
        hdr[7] != (b->fp32 ? 1u : 0u) || hdr[8] != (uint32_t)MAXV)
        return fail(b, EM_ERR_ARG, "snapshot does not belong to a batch of this shape");
    HIPCHK(b, hipStreamSynchronize(b->stream));
    SnapIO io{nullptr, (const uint8_t *)host_buf, n, sizeof hdr};
    em_status rc = snap_walk(b, io, true);
    if (rc != EM_OK) return rc;
    if (!io.ok) return fail(b, EM_ERR_ARG, "snapshot truncated");
    unsigned int nev = 0;
    HIPCHK(b, hipMemcpy(&nev, b->d.ev_count, 4, hipMemcpyDeviceToHost));
    const size_t ev_bytes = 4 * (size_t)EV_WORDS * std::min<unsigned int>(nev, (unsigned int)b->d.ev_cap);
    rc = snap_dev(b, io, b->d.events, ev_bytes, true);
    if (rc != EM_OK) return rc;
    if (!io.ok) return fail(b, EM_ERR_ARG, "snapshot truncated");
    b->step_counter = (int)hdr[9];
    b->n_outer_done = (int)hdr[10];
    b->have_j = hdr[11] != 0;
    // derived state: forcing from the restored currents, factors from the
    // restored void rows, reachability and the IR solution status
    std::vector<uint8_t> op((size_t)b->n_res * b->S);
    HIPCHK(b, hipMemcpy(op.data(), b->d.open, op.size(), hipMemcpyDeviceToHost));
    b->any_open = false;
    for (uint8_t o : op) b->any_open |= o != 0;
    b->live_dirty = true;
    b->ir_valid = false;
    b->act_dirty = true;
    b->nominal = false;
    HIPCHK(b, hipMemsetAsync(b->d.open_dirty, 0, 4, b->stream));
    if (b->have_j) launch_update_f(b->d, b->fp32, b->stream);
    launch_factor(b->d, b->fp32, b->stream);
    LAUNCHCHK(b);
    HIPCHK(b, hipStreamSynchronize(b->stream));
    return EM_OK;
}

em_status em_get_xi(em_batch *b, int32_t sample, int32_t param, double *xi)
{
    if (!b || !xi || sample < 0 || sample >= b->S || param < 0 || param > 3)
        return fail(b, EM_ERR_ARG, "bad arguments");
    const int S = b->S;
    const Dev &d = b->d;
    if (param == 3) {               // loading: per node, the sampled sink over the nominal one
        std::vector<double> snk(b->n_nodes), ss(b->n_nodes);
        if (!d.sink_s) { for (int v = 0; v < b->n_nodes; ++v) xi[v] = 1.0; return EM_OK; }
        HIPCHK(b, hipMemcpyAsync(snk.data(), d.sink, 8 * snk.size(), hipMemcpyDeviceToHost, b->stream));
        HIPCHK(b, hipMemcpyAsync(ss.data(), d.sink_s + (size_t)sample * b->n_nodes, 8 * ss.size(),
                                 hipMemcpyDeviceToHost, b->stream));
        HIPCHK(b, hipStreamSynchronize(b->stream));
        for (int v = 0; v < b->n_nodes; ++v) xi[v] = snk[v] != 0.0 ? ss[v] / snk[v] : 1.0;
        return EM_OK;
    }
    const double *src = param == 0 ? d.xi_k : param == 1 ? d.xi_s : d.xi_r;
    if (!src) { for (int e = 0; e < b->n_res; ++e) xi[e] = 1.0; return EM_OK; }
    std::vector<double> tmp((size_t)b->n_res * S);
    HIPCHK(b, hipMemcpyAsync(tmp.data(), src, 8 * tmp.size(), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    for (int e = 0; e < b->n_res; ++e) xi[e] = tmp[(size_t)e * S + sample];
    return EM_OK;
}

em_status em_features(em_batch *b, float *X)
{
    if (!b || !X) return fail(b, EM_ERR_ARG, "null feature buffer");
    if (!b->have_j) return fail(b, EM_ERR_STATE, "no current densities yet (call em_ir_solve first)");
    em_status rc = sur_buffers(b);
    if (rc != EM_OK) return rc;
    rc = features_impl(b, X, false, false);
    if (rc != EM_OK) return rc;
    HIPCHK(b, hipStreamSynchronize(b->stream));
    return EM_OK;
}

em_status em_surrogate_screen(em_batch *b, em_mlp *mlp, double margin, int64_t *n_deferred)
{
    if (!b) return EM_ERR_ARG;
    if (n_deferred) *n_deferred = 0;
    if (mlp && !(margin >= 1.0 && std::isfinite(margin))) return fail(b, EM_ERR_ARG, "margin must be finite and >= 1");
    b->sur = mlp;
    b->sur_margin = margin;
    if (!mlp) return EM_OK;
    em_status rc = sur_buffers(b);
    if (rc != EM_OK) return rc;
    if (mlp_reserve(mlp, b->n_trees * b->S) != EM_OK)     // model activations for every instance
        return fail(b, EM_ERR_OOM, "learned-screen model buffers");
    if (b->have_j && b->step_counter == 0 && b->n_outer_done == 0) {
        const int K = std::min(b->run.ir_every, b->run.n_steps);
        rc = sur_evaluate(b, margin * K * b->run.dt, n_deferred, false);
        if (rc != EM_OK) return rc;
    }
    return EM_OK;
}

em_status em_get_surrogate(em_batch *b, int32_t sample, float *y_hat, uint8_t *deferred)
{
    if (!b || sample < 0 || sample >= b->S) return fail(b, EM_ERR_ARG, "bad sample");
    if (!b->sur_ready) return fail(b, EM_ERR_STATE, "no learned screen has been evaluated on this batch");
    const size_t IS = (size_t)b->n_trees * b->S;
    std::vector<float> y(IS);
    std::vector<uint8_t> df(IS);
    HIPCHK(b, hipMemcpyAsync(y.data(), b->d.yhat, 4 * IS, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipMemcpyAsync(df.data(), b->d.deferred, IS, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    for (int t = 0; t < b->n_trees; ++t) {
        if (y_hat) y_hat[t] = y[(size_t)t * b->S + sample];
        if (deferred) deferred[t] = df[(size_t)t * b->S + sample];
    }
    return EM_OK;
}

em_status em_first_nucleation(em_batch *b, int32_t *step)
{
    if (!b || !step) return fail(b, EM_ERR_ARG, "null output");
    const size_t IS = (size_t)b->n_trees * b->S;
    std::vector<int> nv(IS), vs(IS * MAXV);
    HIPCHK(b, hipMemcpyAsync(nv.data(), b->d.nv, 4 * IS, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipMemcpyAsync(vs.data(), b->d.vstep, 4 * IS * MAXV, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    for (int t = 0; t < b->n_trees; ++t)
        for (int s = 0; s < b->S; ++s) {
            size_t inst = (size_t)t * b->S + s;
            step[(size_t)s * b->n_trees + t] = nv[inst] > 0 ? vs[inst * MAXV] : -1;
        }
    return EM_OK;
}

}  // extern "C"
