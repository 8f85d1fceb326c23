// Internal device-side data layout and kernel launchers of the EM/TM library.
//
// Layouts (S = number of Monte Carlo samples):
//   stress-node arrays   [node][S]  (sample fastest: the lanes of a wavefront
//                                    are samples of one tree, or trees when
//                                    S == 1)
//   IR node vectors      [S][node]  (node fastest: per-sample reductions over
//                                    contiguous ranges)
//   per-segment MC draws [res][S]
//   per-segment state    [S][res]   (dR, open, current density)
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

namespace em {

constexpr int MAXV = 4;                 // void slots per (tree, sample)
constexpr double E_CHG = 1.602176634e-19;
constexpr double K_B = 1.380649e-23;
constexpr int EV_WORDS = 5;             // sample, tree, step, node, host segment
// resident chain kernel: nodes per lane and the largest lanes per workgroup
#define CHAIN_M32 8
#define CHAIN_M32W 9                    // FP32 blocks of the 1024-lane form when they save rounds
#define CHAIN_WG32 1024
#define CHAIN_M64 8
#define CHAIN_WG64 512

struct Dev {
    // ---- sizes ----
    int n_nodes, n_res, n_trees, ns, N, S, n_pads;
    int max_voids;
    double dt, vdd;
    // material
    double B, Omega, Z, rho, Ea_eV, D0, scrit, Q_eV, sigT, delta, rho_ta, h_ta;
    double k_cu, k_ild, t_ild;          // thermal block of the Joule pre-pass
    // ---- netlist (shared) ----
    const double *xy;
    const int *layer;
    const int *ra, *rb;
    const double *len, *w, *h, *R0;
    const uint8_t *is_wire;             // 1 for a wire segment
    const double *sink;
    double *sink_s;                     // [S][n_nodes] per-sample sinks (condensed system; nodal
                                        // network under loading variation), or null
    const uint8_t *is_pad;              // [n_nodes]
    const int *ninc_off, *ninc_res, *ninc_nbr;   // node incidence (all resistors)
    // temperature inputs
    const double *node_T;               // may be null
    const double *tmap;                 // may be null
    int tnx, tny;
    double tx0, ty0, tdx, tdy, T_amb;
    const double *seg_j_in;             // trees-only prescribed j (null otherwise)
    // ---- tree topology (shared) ----
    const int *tree_off, *parent, *seg, *dir, *vert, *kpos;
    const int *ntree;                   // [ns] tree of each stress node
    const int *child_off, *child;       // children of each stress node, ascending
    const int *vinc_off, *vinc;         // wire segments incident to each vertex, ascending
    const int *tseg_off, *tseg;         // segments of each tree
    const uint8_t *via_up;              // vertex has a via to a strictly higher layer
    const int *tree_perm;               // lane slot -> tree id (larger trees first)
    const uint8_t *tree_chain;          // tree stepped by the resident chain kernel
    const int *lane_inst, *lane_blk;    // chain kernel lanes: instance, block index
    // workgroup tree stepper (trees the chain kernel does not take): heavy-path
    // order of each such tree's nodes, level by level, at the tree's node range
    const int *br_tree;                 // [n_br] tree id
    const int *br_nlev, *br_lvl0;       // [n_br] levels, start in br_lvl
    const int *br_lvl;                  // level offsets (relative to the tree's first node), nlev + 1 per tree
    const int *br_node;                 // [ns] node at each heavy-path position
    const int *br_heavy;                // [ns] child continuing the node's path (-1 at a leaf)
    int n_chain_wg;                     // workgroups of the chain kernel's launch
    int chain_wg;                       // its lanes per workgroup (64 to the precision's maximum)
    int chain_m;                        // stress nodes per lane (CHAIN_M32/CHAIN_M64, or CHAIN_M32W)
    int chain_occ;                      // 1, or 4: register budget of 128 VGPRs (FP32, 64-512 lanes)
    // ---- per stress node statics (FP64) ----
    double *T, *V, *g0, *rob0, *gdx0, *mdrv;
    double *tree_V;                     // [n_trees] total control volume
    // ---- per (node, sample) stepping state; element type float or double ----
    void *sigma, *dtf, *dinv, *lfac, *sc, *Vr;
    float *sig_lo;                      // FP32 form: low part of the stress state (null in FP64)
    double *psi;                        // screen scratch / steady stress [node][S]
    double *wsp;                        // stepping workspace [node][S] (generic tree kernel)
    // ---- Monte Carlo draws [res][S] ----
    const int *sid;                     // [S] Monte Carlo sample index of each batch sample, or null
                                        // (identity)
    double *xi_k, *xi_s;
    double *map_a;                      // [S] thermal-map amplitude of each sample (null: 1)
    double *xi_r;                       // resistivity multipliers (1 for vias), or null
    // ---- per (sample, segment) ----
    double *jseg;                       // [S][res]
    double *jT;                         // [res][S] transposed copy of jseg for the forcing update (S > 1)
    double *dR;                         // [S][res]
    uint8_t *open;                      // [S][res]
    uint8_t *seg_mortal;                // [S][res]
    // ---- per instance (tree, sample), inst = tree * S + sample ----
    uint8_t *inst_active;               // stepped at all (screen)
    uint8_t *tree_mortal;               // screen verdict
    int *nv;                            // voids in use
    int *vnode, *vseg, *vphase, *vstep, *vearly;   // [inst][MAXV]
    double *vvol, *vlen, *vrob;         // [inst][MAXV]
    int *n_suppressed;                  // [inst]
    // ---- per sample ----
    uint8_t *sample_active;             // not yet retired
    uint32_t *open_dirty;               // [1] set when a segment opened
    unsigned long long *node_steps;     // [NS_SLOTS] stepped (node, sample) x steps, spread over slots
                                        //     picked by workgroup (summed on readout)
    // ---- events ----
    int *events;                        // [ev_cap][EV_WORDS]
    unsigned int *ev_count;
    int ev_cap;
    // ---- IR ([S][n_nodes] unless noted) ----
    double *G;                          // [S][res] conductance
    double *G_inc;                      // [S][node incidence] conductance per SpMV entry
    double *diag, *rhs, *u, *r, *z, *p, *q;
    uint8_t *live;                      // [S][n_nodes]
    uint32_t *live_changed;
    uint32_t *g_changed;                // [1] some conductance differs from the last solve's
    uint8_t *g_chg_s;                   // [S] this sample's conductances differ (or: first solve)
    int *cc_label;                      // [S][n_nodes + 1] component labels (reachability)
    double *part;                       // [S][nblk][4] block partial sums
    double *rz;                         // [2][S] r.z, double-buffered by iteration parity
    double *bb;                         // [S]
    uint8_t *conv;                      // [S]
    int *ir_iters;                      // [S] PCG iterations of the last solve (one-workgroup form)
    double *drop;                       // [S]
    int ir_nblk;
    // ---- TTF ----
    double *ttf, *final_drop, *init_drop, *t_prev, *d_prev;
    int *failed, *outer_idx;
    uint8_t *guard;                     // [S] a re-solve's drop came within guard_band of the threshold
    double guard_band;                  // relative to the failure fraction (0: off)
    double guard_ttf;                   // relative TTF tolerance of the ill-conditioned-bracket rule
    // ---- learned screen (allocated when a model is attached) ----
    double *tstat;                      // [n_trees][4] Ltot, Lpath, nseg, njunc
    double *rdist;                      // [ns] distance from the tree root along the tree
    float *feat;                        // [inst][NFEAT]
    float *yhat;                        // [inst] predicted log10(t_nuc / T_REF)
    uint8_t *deferred, *catchup;        // [inst]
    int *def_list;                      // [inst] instances deferred at t = 0 (in no particular order)
    int *def_k;                         // [def_list] aging interval of each one's last prediction (-1: t = 0)
    uint8_t *sur_viol;                  // [S] a learned-screen violation hit the sample
    int *act_list;                      // [inst] instances activated by the last activation check
    unsigned int *sur_cnt;              // [8] deferred, activated, late, violations, def_list length,
                                        //     act_list length
    // ---- steady-state skipping (allocated when em_run_params.ss_tol > 0) ----
    uint8_t *ss_skip;                   // [inst] skipped at its steady state
    unsigned int *ss_cnt;               // [2] skips, wakes (cumulative)
    int ss_nc;                          // chunks of SS_CL nodes over the chain trees (64+ samples)
    const int *ss_coff, *ss_ctree, *ss_cstart;   // [n_trees+1] first chunk; [nc] tree, first node
    double *ss_scr;                     // [nc][11][S] chunk sums, carries, extremes; [IS] fm
    // ---- reduced (extended rational Krylov) stepping of long chains (kq > 0) ----
    int kq, krm;                        // reduction order q (blocks), columns at most 2q
    double keta;                        // shift-time scale eta (eq. 26)
    const int *kry_list;                // chain instances of at least max(3q, 30) nodes
    int n_kry_list;
    double *kv;                         // [krm][ns][S] basis columns
    double *kred;                       // [inst][KRY_KS(krm)] A_h, C_h, f_h, z, F, g, dt of F
    double *kscr;                       // [3][ns][S] inverse pivots and multipliers of K = s0 C - A
    int *kr;                            // [inst] basis columns (0: none)
    uint8_t *kdone;                     // [inst] interval taken in reduced form
    unsigned long long *kcnt;           // [4][KRY_CNT_SLOTS] bases built, reduced intervals, fallbacks,
                                        //     node-steps advanced in reduced form; each count spread over
                                        //     slots picked by workgroup (summed on readout), so that tens of
                                        //     thousands of workgroups do not queue on one address
    int *kbl, *kfl;                     // [n_kry_list] instances needing a basis / a step operator
    unsigned int *kbn;                  // [2] their lengths (cleared by the bound-and-lift launch)
    double *kze;                        // [inst][krm] reduced end state of the interval
    double *kdist;                      // [inst] largest distance of the interval's reduced states from it
};

constexpr int SS_CL = 64;                // nodes per chunk of the many-sample skipping check
constexpr int KRY_RM_MAX = 16;           // 2 q for q <= 8
constexpr int NS_SLOTS = 64;             // slots of the node-step count (a power of two): one address
                                        // taking an atomic from every wavefront of a launch queues them
constexpr int KRY_CNT_SLOTS = 256;       // slots per reduced-stepping counter (a power of two)
__host__ __device__ constexpr int KRY_KS(int rm) { return 3 * rm * rm + 3 * rm + 1; }

// Aggregation multigrid preconditioner of the IR solve.  Level 0 is the nodal
// system on the free nodes; level l >= 1 has one node per aggregate of level
// l - 1 nodes (heavy-edge pair matching applied twice, so aggregates of up to
// four) and the Galerkin operator of piecewise-constant prolongation.
constexpr int AMG_MAXLEV = 16;
constexpr int AMG_NC_MAX = 88;          // coarsest level inverted densely when this small

// Storage type of the multigrid preconditioner (operators, V-cycle vectors,
// coarsest inverse, level-0 scratch): float halves its memory traffic; every
// operation on it runs in double and the CG itself (iterate, residual,
// search direction, its operator, dot products, stopping rule) stays FP64,
// so the precision of the solution is set by the CG's FP64 residual alone.
using mgreal = float;

struct AmgLevel {
    int n, ne, nf, nef;                 // nodes, edges of this level; nodes, edges of the finer one
    int nmem;                           // member entries (mem_off[n])
    const int *agg;                     // [nf] finer node -> node of this level (-1: outside)
    const int *mem_off, *mem;           // members of each node
    const int *int_off, *int_e;         // finer edges inside each node
    const int *src_off, *src_e;         // finer edges merged into each edge
    const int *adj_off, *adj_nbr, *adj_e;   // this level's graph (both directions)
    mgreal *D, *W;                      // [S][n] diagonal, [S][ne] edge conductance
    mgreal *Wa;                         // [S][2 ne] conductance of each adjacency entry (W[adj_e]),
                                        // contiguous per node as the V-cycle's rows read it
    mgreal *b, *x, *y, *w;              // [S][n] V-cycle vectors
};

struct Amg0 {                           // level-0 edges: resistors with both ends off the pads
    int ne0;
    const int *e0_res, *e0_a, *e0_b;
    mgreal *w0;                         // [S][n_nodes] level-0 scratch
};

struct Amg {
    int nlev = 0;                       // coarse levels 1..nlev
    AmgLevel lev[AMG_MAXLEV + 1];
    Amg0 l0;
    mgreal *Ainv = nullptr;             // [S][n][n] inverse of the coarsest operator (dense case)
    int dense = 0;
    double omega = 2.0 / 3.0, alpha = 1.0;
};

// Chain condensation of the IR network: terminals (pads and nodes whose
// resistor count is neither 1 nor 2) and the chains of interior nodes
// between them; the condensed system has one reduced edge per two-ended
// chain joining two distinct terminals.
struct CondHost {
    int n_term = 0, n_chain = 0;
    std::vector<int> term_node, tid;    // terminal -> node, node -> terminal (-1: interior)
    std::vector<int> eoff, e;           // resistors of each chain, from end A
    std::vector<int> voff, v;           // interior nodes of each chain, from end A
    std::vector<int> cA, cB;            // terminal at each end (cB -1: dangling chain)
    std::vector<int> cred;              // reduced edge of each chain (-1: none)
    std::vector<int> red_a, red_b;      // reduced edges (terminal indices)
    std::vector<double> red_R0;         // nominal series resistance of each reduced edge
    std::vector<uint8_t> red_pad;       // terminal is a pad
    std::vector<int> tce_off, tce;      // chain ends at each terminal: 2 * chain + (end B)
};
CondHost cond_build(int nn, int nr, const int *ra, const int *rb, const double *R0, const uint8_t *is_pad);

struct Cond {
    int n_term, n_chain;
    const int *term_node;
    const int *eoff, *e, *voff, *v, *cA, *cB, *cred;
    const int *tce_off, *tce;
    double *cinj;                       // [S][n_chain][2] current drawn from end A, end B
};

// Host-side construction of the aggregation hierarchy on the nominal
// conductances (1/R0); every array is returned for upload.
struct AmgHostLevel {
    int n = 0, ne = 0, nf = 0, nef = 0;
    std::vector<int> agg, mem_off, mem, int_off, int_e, src_off, src_e, adj_off, adj_nbr, adj_e;
};
struct AmgHost {
    std::vector<int> e0_res, e0_a, e0_b;
    std::vector<AmgHostLevel> lev;      // lev[0] unused
};
AmgHost amg_build(int n_nodes, const uint8_t *is_pad, int n_res, const int *ra, const int *rb,
                  const double *R0);

constexpr int NFEAT = 16;               // learned-screen features per (tree, sample)
constexpr double T_REF = 1e8;           // s; the model predicts log10(t_nuc / T_REF)

// ---- launchers (defined in the kernel translation units) ----
void launch_node_T(const Dev &d, hipStream_t st);
// Joule pre-pass: vertex temperatures per tree (scratch D, r: [ns] each), then
// the steady profile at every interior node; j = [n_res] current densities.
void launch_joule_T(const Dev &d, const double *j, double *D, double *r, hipStream_t st);
void launch_edge_static(const Dev &d, hipStream_t st);
void launch_node_V(const Dev &d, bool fp32, hipStream_t st);   // also per-tree volume
void launch_ss_check(const Dev &d, bool fp32, double tol_abs, hipStream_t st);  // skip converged chain instances
void launch_ss_wake(const Dev &d, bool all, hipStream_t st);  // wake those of re-solved samples (all: every one)
void launch_kry_step(const Dev &d, bool fp32, int n_steps, hipStream_t st);   // reduced intervals
void launch_kry_restore(const Dev &d, hipStream_t st);                        // after the exact launch
void launch_kry_invalidate(const Dev &d, bool all, hipStream_t st);           // after an IR solve
void launch_draws(const Dev &d, uint64_t seed, double cov_k, double cov_s, double cov_r, double cov_l,
                  double sd_ea, double sd_T, double cov_map, hipStream_t st);
void launch_node_sc(const Dev &d, bool fp32, hipStream_t st);
void launch_update_f(const Dev &d, bool fp32, hipStream_t st);
void launch_factor(const Dev &d, bool fp32, hipStream_t st);
void launch_screen(const Dev &d, bool apply, hipStream_t st);
// the screen when every sample has the same current densities (sample 0's);
// tree_mortal and seg_mortal zeroed by the caller
void launch_screen_shared(const Dev &d, bool apply, hipStream_t st);
// copy the shared screen's steady stress (column 0) to every sample's column
void launch_step(const Dev &d, bool fp32, int n_steps, int step0, hipStream_t st);
void launch_branch(const Dev &d, bool fp32, int n_br, int max_nodes, int n_steps, int step0, hipStream_t st);
void launch_void_dR(const Dev &d, hipStream_t st);
void launch_chain(const Dev &d, const Dev *d_dev, bool fp32, int n_steps, int step0, hipStream_t st);
void launch_set_sigma_T(const Dev &d, bool fp32, hipStream_t st);
void launch_inject_void(const Dev &d, bool fp32, int sample, int tree, int node, hipStream_t st);
void launch_copy_sigma(const Dev &d, bool fp32, int sample, double *out_dev, bool to_state, hipStream_t st);
void launch_copy_node_col(const Dev &d, bool fp32, int which, int sample, double *out_dev, hipStream_t st);

// IR
void launch_ir_conductance(const Dev &d, hipStream_t st);
void launch_ir_gather_inc(const Dev &d, int ninc, hipStream_t st);
void launch_ir_live_copy(const Dev &d, const uint8_t *live0, hipStream_t st);
void launch_ir_cc_init(const Dev &d, hipStream_t st);
void launch_ir_cc_round(const Dev &d, hipStream_t st);    // hooking + pointer jumping, sets live_changed
void launch_ir_cc_finish(const Dev &d, hipStream_t st);   // live = label is the pads'
void launch_ir_setup(const Dev &d, hipStream_t st);       // diag, rhs, r = b - A x, z, p, partials
void launch_ir_finalize0(const Dev &d, double rtol, hipStream_t st);
void launch_ir_spmv(const Dev &d, hipStream_t st);        // q = A p, partial p.q
// x, r; z = r/diag and partials r.z, r.r (amg_omega == 0), or the multigrid
// pre-smoothing z = omega r/diag and partial r.r only
void launch_ir_update(const Dev &d, int it, double amg_omega, hipStream_t st);
// p = z + beta p (z read from zs: d.z, or the multigrid output), conv
void launch_ir_pupdate(const Dev &d, int it, double rtol, const double *zs, hipStream_t st);
int ir_nodes_per_block();
void launch_ir_finish(const Dev &d, hipStream_t st);      // u, j, drop
// multigrid: per-solve Galerkin operators and coarsest inverse; one V-cycle
// z = M^-1 r (init: also pre-smoothing and p = z), partial r.z
void launch_ir_finalize_rz(const Dev &d, hipStream_t st);
void launch_amg_pre0(const Dev &d, double omega, hipStream_t st);
void launch_amg_res0(const Dev &d, mgreal *w0, hipStream_t st);
void launch_amg_post0(const Dev &d, mgreal *w0, const AmgLevel &L1, const mgreal *r1, double alpha,
                      double omega, bool init, hipStream_t st);
void launch_amg_setup(const Dev &d, const Amg &a, hipStream_t st);
void launch_amg_vcycle(const Dev &d, const Amg &a, bool init, hipStream_t st);
int ir_wg_max_nodes();
// LDS-resident form: bytes of dynamic LDS one sample's system and hierarchy
// take (0 when it does not fit a workgroup), and its launch
int ir_lds_bytes(const Dev &d, int nnz, const Amg &a);
void launch_ir_pcg_lds(const Dev &d, int nnz, const Amg &a, const Amg *amg_dev, double rtol, int max_iter,
                       hipStream_t st);
// chain-kernel lane table: lane_inst = -1 everywhere, then instance i fills
// lanes off[i] .. off[i] + L[i] - 1 with (inst[i], block 0 .. L[i] - 1)
void launch_place_lanes(int *lane_inst, int *lane_blk, long long n_lanes, const int *inst,
                        const long long *off, const int *L, int n_place, hipStream_t st);
// condensed IR solve: chain reduction + reduced sinks and warm start; terminal
// scatter + interior back-substitution into the nodal u and live
void launch_chain_reduce(const Dev &d, const Dev &r, const Cond &c, hipStream_t st);
void launch_chain_expand(const Dev &d, const Dev &r, const Cond &c, hipStream_t st);
void launch_ir_pcg_wg(const Dev &d, const Amg *amg_dev, double rtol, int max_iter, hipStream_t st);
void launch_fill_f64(double *p, size_t n, double v, hipStream_t st);
void launch_ttf_init(const Dev &d, double fail, hipStream_t st);
void launch_ttf_update(const Dev &d, double fail, int k, double t, hipStream_t st);
// identical samples: iterate sample 0 only (conv of the others set), then
// copy its [S][n] state to every sample
void launch_ir_only_sample0(const Dev &d, hipStream_t st);
void launch_bcast0_f64(double *a, long long n, int S, hipStream_t st);
void launch_bcast0_u8(uint8_t *a, long long n, int S, hipStream_t st);
// cnt[2s] = trees of sample s holding a void, cnt[2s+1] = segments with dR > 0 or open
void launch_result_counts(const Dev &d, int *cnt, hipStream_t st);

// learned screen
void launch_tree_static(const Dev &d, hipStream_t st);                 // tstat, rdist
void launch_features(const Dev &d, float *X, bool candidates_only, bool psi_col0,
                     hipStream_t st);   // needs psi (column 0 only with psi_col0)
void launch_reeval_features(const Dev &d, int n, float *X, const double *jhist, int k_now, double tol,
                            hipStream_t st);   // def_list[0..n)
void launch_yhat_min(const Dev &d, int n, const float *y, hipStream_t st);
void launch_defer(const Dev &d, const float *y, double thr, hipStream_t st);
void launch_activate(const Dev &d, double thr, hipStream_t st);
void launch_update_f_list(const Dev &d, bool fp32, const int *list, int n, hipStream_t st);
void launch_catchup_done(const Dev &d, int step_lim, hipStream_t st);

}  // namespace em

// MLP forward on a caller's stream (X, y device; rows n); defined with the
// model in em_mlp.hip.
struct em_mlp;
namespace em {
int mlp_forward_async(em_mlp *m, const float *X, int n, float *y, hipStream_t st);
int mlp_reserve(em_mlp *m, int n);        // activation buffers for n rows (allocates)
}
