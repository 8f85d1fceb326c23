/*
 * em.h -- C ABI of the MI355X coupled EM/TM stress + IR-drop library.
 *
 * The library implements the transient hot path of EMSpice 3 (Lu & Tan,
 * arXiv 2604.10743): Korhonen stress evolution with electromigration,
 * stress-migration and thermomigration drives (Sec. III-D, eqs. 10-13),
 * discretised into the descriptor system C dsigma/dt = A sigma + f (eq. 18)
 * on every wire tree of an extracted power grid and stepped by backward Euler;
 * void nucleation against the critical stress, the Robin void row (eq. 20,
 * Sec. IV-D), void volume by atom conservation (eq. 15), incubation (eq. 16),
 * early/late failure (Sec. IV-C, eq. 17); periodic IR-drop re-solves of the
 * nodal system M u = P I (eq. 8) closing the loop to time-to-failure (Fig. 2),
 * the optional steady-state immortality screen (Sec. III-B) and Monte Carlo
 * over diffusivity and critical stress (Sec. IV-F).
 *
 * Conventions for every entry point:
 *   - Returns an em_status; never throws, never aborts.  em_last_error() gives a
 *     human-readable message for the last failing call on a batch.
 *   - Input arrays are HOST pointers, read during the call and copied; the
 *     caller may free them afterwards.  Output arrays are HOST pointers owned
 *     by the caller, sized as documented (counts come from em_get_info).
 *   - All device memory belongs to the batch and is released by
 *     em_batch_destroy.  Device work runs on the stream given at creation.
 *   - A batch is not thread-safe: calls on one batch must not overlap.
 *   - Asynchronous HIP failures surface as EM_ERR_HIP at the next call that
 *     synchronises.
 *   - Units are SI (m, s, K, Pa, A, ohm, V) unless stated.
 */
#ifndef EM_MI355X_H
#define EM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct em_batch em_batch;   /* opaque, library-owned */
typedef struct em_mlp em_mlp;       /* opaque learned-screen model, library-owned */

typedef enum {
    EM_OK = 0,
    EM_ERR_ARG = 1,       /* invalid argument: NULL, size, NaN, a cycle in a wire tree, ... */
    EM_ERR_OOM = 2,       /* device or host allocation failed */
    EM_ERR_HIP = 3,       /* a HIP runtime call or kernel failed */
    EM_ERR_NOCONV = 4,    /* conjugate gradients missed cg_rtol within cg_max_iter */
    EM_ERR_STATE = 5,     /* call out of order (e.g. a step on a batch with no currents) */
    EM_ERR_OVERFLOW = 6   /* event ring overflowed (events beyond its capacity were dropped);
                             the per-instance void cap is not an error, see em_info.n_void_capped */
} em_status;

typedef enum { EM_FP64 = 0, EM_FP32 = 1 } em_precision;

/* Extracted power-grid netlist (Sec. IV-A: netlist, optional thermal map).
 * A resistor is a via when res_is_via[r] != 0 or its two nodes lie on
 * different layers; every other resistor is a wire segment.  Wire segments
 * on one layer form the wire trees (connected components; a component with a
 * cycle is rejected with EM_ERR_ARG).  Temperatures: a raster (tmap != NULL,
 * row-major [tmap_ny][tmap_nx], sample (x,y) -> bilinear with edge clamping),
 * else per-node node_T (interior FD points interpolate along the segment),
 * else the uniform em_run_params.T_ambient.  seg_j != NULL switches the batch
 * to trees-only mode: per-resistor current density prescribed (A/m^2, signed
 * along res_a -> res_b), no IR solve and no time-to-failure.  A netlist
 * without any wire segment is rejected (EM_ERR_ARG). */
typedef struct {
    uint32_t struct_size;           /* sizeof(em_grid_desc) */
    int32_t n_nodes;
    const double *xy;               /* [n_nodes][2] node coordinates */
    const int32_t *layer;           /* [n_nodes] metal layer index (higher = upper) */
    int32_t n_res;
    const int32_t *res_a, *res_b;   /* [n_res] end nodes */
    const double *res_len, *res_w, *res_h;   /* [n_res] length, width, thickness */
    const uint8_t *res_is_via;      /* [n_res] */
    const double *res_R0;           /* [n_res] nominal resistance, > 0 */
    int32_t n_pads;
    const int32_t *pad_node;        /* [n_pads] ideal VDD sources */
    double vdd;
    const double *sink_I;           /* [n_nodes] current drawn at each node, A; may be NULL in trees-only mode */
    const double *node_T;           /* [n_nodes] K, or NULL */
    int32_t tmap_nx, tmap_ny;
    double tmap_x0, tmap_y0, tmap_dx, tmap_dy;
    const double *tmap;             /* raster, or NULL */
    const double *seg_j;            /* [n_res] or NULL */
} em_grid_desc;

/* Material (the paper's YAML material block). Ea and Q in eV. */
typedef struct {
    uint32_t struct_size;
    double B;          /* effective bulk modulus, Pa */
    double Omega;      /* atomic volume, m^3 */
    double Z;          /* effective charge number */
    double rho_cu;     /* copper resistivity, ohm m */
    double Ea_eV;      /* activation energy of D_a */
    double D0;         /* diffusion prefactor, m^2/s */
    double sigma_crit; /* nucleation threshold, Pa */
    double Q_eV;       /* heat of transport (thermomigration) */
    double sigma_T;    /* initial residual stress, Pa */
    double delta;      /* void-interface thickness of the Robin row, m */
    double rho_ta;     /* liner resistivity, ohm m */
    double h_ta;       /* liner thickness, m */
    /* Thermal block of the Joule-heating pre-pass (Sec. III-A, eqs. 2-4; read
     * only when em_run_params.joule != 0): wire and dielectric thermal
     * conductivities (W/(m K)) and the dielectric thickness t_ILD (m).  The
     * wire thickness t_cu of eq. 2 is each segment's res_h. */
    double k_cu, k_ild, t_ild;
} em_material;

/* Numerics (the paper's YAML numerical block). */
typedef struct {
    uint32_t struct_size;
    int32_t intervals_per_seg;   /* FD intervals per wire segment, >= 1 */
    double dt;                   /* backward-Euler step, s */
    int32_t n_steps;             /* horizon in steps for em_run_to_ttf */
    int32_t ir_every;            /* steps between IR re-solves */
    double fail_frac;            /* failure when worst IR-drop >= fail_frac * vdd */
    double cg_rtol;              /* PCG: ||r|| <= cg_rtol ||b|| per sample; 0 automatic: 1e-11 with
                                    FP64 stepping, 1e-8 with FP32 (four orders below the FP32
                                    stepping's own drop error; the guard band's FP64 re-runs
                                    solve to 1e-11) */
    int32_t cg_max_iter;
    int32_t prec;                /* em_precision of the stress stepping */
    int32_t screen;              /* 1: steady-state immortality screen before stepping */
    int32_t max_voids_per_tree;  /* 0 disables nucleation */
    double T_ambient;            /* K, used when no thermal data is given */
    int32_t stepper;             /* 0: resident chain kernel for chain trees (straight wires)
                                    that fit a workgroup, generic tree kernel otherwise;
                                    1: generic tree kernel for every tree */
    int32_t ir_precond;          /* IR solve: 0 Jacobi-preconditioned CG on the nodal system;
                                    1 CG with an aggregation-multigrid V-cycle on the nodal
                                    system; 2 the same on the chain-condensed system (exact
                                    Schur complement onto pads and nodes with other than one or
                                    two resistors; interior node voltages by back-substitution
                                    along each chain), applied when it removes at least a
                                    quarter of the nodes, else as 1.  Same solution to cg_rtol;
                                    2 iterates a far smaller, better conditioned system on P/G
                                    grids with sparse vias. */
    int32_t ir_launch;           /* launch shape of the multigrid PCG: 0 automatic (2 when the
                                    iterated system has at most 4096 nodes, or at most 65536
                                    nodes and 32 or more samples; else 1); 1 one kernel per
                                    V-cycle step over all samples, iterations replayed as a
                                    graph; 2 one workgroup per sample running its whole PCG in
                                    one launch, from LDS when the sample's system and hierarchy
                                    fit (else as 3); 3 the same with the vectors in HBM.  Same
                                    preconditioner and stopping rule; the reduction order of
                                    the dot products differs. */
    int32_t chain_wg;            /* lanes per workgroup of the resident chain kernel: 0 automatic
                                    (the smallest of 256, 512, 1024 that holds the longest chain
                                    tree; 1024 with 9-node blocks, see chain_m), or one of 64, 128,
                                    256, 512, 1024 (at most 512 in FP64) that holds it (64 and 128:
                                    one or two wavefronts per workgroup, short trees only).
                                    Results do not depend on it (instances never share a
                                    reduction: the couplings across their boundaries are zero),
                                    except that the FP32 1024-lane form keeps no low part of the
                                    stress state (no registers for it) and agrees with the
                                    others to float rounding of the state. */
    int32_t chain_occ;           /* register budget of the resident chain kernel: 0 or 1 as many
                                    registers as it uses (one or two workgroups per compute unit);
                                    4 at most 128 VGPRs (four waves per SIMD: four 256-lane or two
                                    512-lane workgroups share a compute unit, some values spill),
                                    FP32 with 64 to 512 lanes only.  Pays when a launch holds
                                    few instances (Monte Carlo after the screen); 3 at most 168
                                    VGPRs (three waves per SIMD, fewer spills), FP32 with 256 or
                                    512 lanes.  Same results. */
    int32_t joule;               /* 1: one-time Joule-heating thermal pre-pass at batch creation
                                    (Sec. III-A): the currents of a nominal IR solve (or the
                                    prescribed seg_j) heat every wire segment; each segment's
                                    steady profile solves k T'' + j^2 rho = k (T - T0)/Gamma^2,
                                    Gamma^2 = t_cu t_ILD k_cu / k_ILD, between its end
                                    temperatures.  A tree vertex with a via takes the map
                                    temperature; the other vertices follow from heat-flux
                                    balance over their segments (exact per-tree elimination).
                                    T0 of a segment is the map temperature at its midpoint
                                    (the uniform T_ambient without thermal data).  The stress
                                    nodes then take the profile's values; the field is fixed for
                                    the batch (resets keep it).  0: node temperatures sampled
                                    from the map directly. */
    double dt_growth;            /* time grid of em_run_to_ttf (the paper's non-uniform inner
                                    grid with a factor per step size, Sec. IV-E): aging interval
                                    k (ir_every steps, k = 0, 1, ...) steps with dt * dt_growth^k.
                                    0 or 1: uniform.  The backward-Euler factors are rebuilt at
                                    each change of step size.  Not with a learned screen attached
                                    (its catch-up replay assumes uniform steps: EM_ERR_STATE).
                                    em_stress_step always uses dt. */
    int32_t chain_m;             /* stress nodes per lane of the resident chain kernel: 0
                                    automatic, 8, or 9 (FP32 with 1024-lane workgroups only).
                                    Automatic takes 8 unless every layout needs 1024-lane
                                    workgroups (one per compute unit) and 9-node blocks pack the
                                    chain instances into fewer rounds of the chip (rounds times
                                    block length smaller).  Lanes hold whole blocks; results agree
                                    to float rounding of the state. */
    double guard_band;           /* FP32 runs of em_run_to_ttf: relative guard band around the
                                    failure threshold (0 = off).  A sample whose worst drop at any
                                    re-solve up to its retirement lies within
                                    guard_band x fail_frac of fail_frac has its failure decision
                                    and time bracket determined by stress values that FP32
                                    stepping does not resolve; after the FP32 run every such
                                    sample is run again from t = 0 in FP64 (an internal batch over
                                    those Monte Carlo sample indices, same inputs) and its
                                    em_ttf_result, resistance changes and opens are replaced by
                                    the FP64 run's (em_ttf_result.redecided = 1).  Its stress,
                                    voids and events keep the FP32 run's values.  The re-run has
                                    no learned screen (whose replay reproduces the unscreened run).
                                    Ignored in FP64 and in trees-only mode. */
    double guard_ttf;            /* with guard_band > 0: a failing FP32 sample is also re-run in
                                    FP64 when its time to failure is ill-conditioned, i.e. a drop
                                    error of guard_band x fail_frac at the bracketing re-solves
                                    could move the interpolated TTF by more than guard_ttf
                                    relative: guard_band fail_frac (t_k - t_k-1) >
                                    guard_ttf TTF (drop_k - drop_k-1).  0 = off. */
    double amg_alpha;            /* coarse-correction scale of the multigrid preconditioner: 0
                                    automatic (1.4), else in [1, 4].  The best value depends on the
                                    network (pg400 1.4, the full chip 2.2 in cold-solve iterations);
                                    em_autotune times 1.4, 1.8 and 2.2 when it is 0.  Same solution
                                    to cg_rtol. */
    double ss_tol;               /* em_run_to_ttf: steady-state skipping, 0 = off, else in
                                    (0, 1e-2].  After each aging interval a chain-stepped
                                    (tree, sample) instance without voids stops being stepped
                                    when the band its stress can still move in under the
                                    present currents is at most ss_tol x sigma_crit (nominal)
                                    wide and keeps every node below its critical stress.  The
                                    band is exact for backward Euler with constant forcing:
                                    each step maps the distance to the steady state by a
                                    nonnegative matrix with unit row sums, and that distance
                                    follows, up to a constant, from the residual's sums over
                                    the chain.  So a skipped instance could not have
                                    nucleated, and its frozen stress stays within
                                    ss_tol x sigma_crit of the stepped one's at every node (up
                                    to the stepping's rounding).  An IR re-solve that changes
                                    its sample's conductances wakes it; every instance is
                                    awake again when the call returns.  Not with a learned
                                    screen attached. */
    int32_t krylov_q;            /* extended rational Krylov reduced stepping (Sec. IV-E, Alg. 1):
                                    0 = off, else the reduction order q in [1, 8] (at most 2q
                                    basis columns).  Chain-stepped (tree, sample) instances of at
                                    least max(3q, 30) nodes (eq. 27) without voids build a basis
                                    of the block rational Krylov space over [K^-1 C s, K^-1 f],
                                    K = s0 C - A, s0 = 1/t_s (eq. 26), and step the reduced
                                    model by backward Euler, lifting the state at each call's
                                    end; an interval whose lifted states could reach a critical
                                    stress (bound: each node's row norm of the basis times the
                                    reduced states' distance from the end state) is stepped
                                    exactly instead and the basis dropped.  A
                                    basis is kept while the drive is unchanged (an IR re-solve
                                    that changes the sample's conductances, em_set_stress,
                                    em_set_seg_state, em_inject_void, em_restore and em_reset
                                    drop it).  An approximation of the stepping (the paper
                                    reports under 0.05 % TTF / final-drop error); not with
                                    ss_tol or a learned screen. */
    double krylov_eta;           /* shift-time scale eta of eq. 26, t_s = eta L^2 / (pi^2 kappa)
                                    with L the chain's length and kappa its volume-weighted
                                    diffusivity; 0 means 1, else in (0, 100] */
    int32_t dt_adapt;            /* em_run_to_ttf: adaptive time grid, 0 = off, else in [1, 12]:
                                    aging interval k takes ir_every steps of dt 2^m_k, m_0 = 0,
                                    m_(k+1) = 0 after an interval in which a void nucleated
                                    (any sample of the batch) and min(m_k + 1, dt_adapt)
                                    otherwise; the run ends at the horizon n_steps dt, its last
                                    interval's steps shortened to end there.  Coarse steps where
                                    nothing nucleates, fine ones while voids form and grow.  The
                                    batch's samples share the grid.  Not with dt_growth or a
                                    learned screen. */
} em_run_params;

/* Monte Carlo (Sec. IV-F): unit-mean lognormal multipliers with coefficient
 * of variation cov_*, drawn from Philox-4x32-10 with counter (index, sample,
 * param, 0) and key (seed low word, seed high word):
 *   param 0  kappa (diffusivity), per wire segment;
 *   param 1  sigma_crit, per wire segment;
 *   param 2  resistivity, per wire segment: the segment's resistance R0, its
 *            electron-wind drive (eZ rho j / Omega) and the copper term of the
 *            liner resistance change (eq. 17) scale with it; vias keep R0;
 *   param 3  current loading, per node: the node's sink current scales with it;
 *   param 4  activation energy, per wire segment: an offset dEa ~ N(0, sd_ea_eV)
 *            (standard normal from the same counter and Box-Muller branch)
 *            multiplies the segment's diffusivity by exp(-dEa / (k_B T)), T the
 *            map temperature at the segment's midpoint (T_ambient without
 *            thermal data); the factor joins the kappa multiplier;
 *   param 5  die temperature, per sample (counter index 0): the thermal map
 *            shifted by dT ~ N(0, sd_T_K) (a perturbation of the map, Sec.
 *            IV-F); every wire segment's diffusivity takes the Arrhenius
 *            factor kappa(T + dT) / kappa(T) = exp(Ea/k_B (1/T - 1/(T + dT)))
 *            T/(T + dT), T as for param 4, folded into the kappa multiplier.
 *            The thermomigration drive keeps the unshifted map (a uniform
 *            shift leaves dT/dx unchanged; its 1/T^2 factor moves by under
 *            2 % for |dT| <= 3 K at 330 K), and sigma_crit does not depend on T.
 *   param 6  thermal-map amplitude, per sample (counter index 0): the map's rise
 *            above T_ambient scaled by a unit-mean lognormal a (CoV cov_map),
 *            T_a = T_ambient + a (T - T_ambient).  Each wire segment's
 *            diffusivity takes kappa(T_a) / kappa(T) at its midpoint map
 *            temperature (folded into the kappa multiplier, as param 5), and
 *            every edge's thermomigration drive (Q / (Omega T)) dT/dx becomes
 *            that of the scaled field, a T_e / T_a,e times the nominal one
 *            (T_e the edge's midpoint temperature).  Not with the Joule
 *            pre-pass (whose temperatures are not the map's).
 * The paper's study perturbs kappa and sigma_crit; resistivity and loading are
 * two of the further sampled inputs it names for the same flow.  With
 * cov_rho = cov_load = 0 every sample starts on the nominal network. */
typedef struct {
    uint32_t struct_size;
    int32_t n_samples;
    uint64_t seed;
    double cov_kappa, cov_scrit;
    double cov_rho, cov_load;
    double sd_ea_eV;             /* activation-energy spread, eV, 0 <= sd < 1 */
    double sd_T_K;               /* die-temperature spread, K, 0 <= sd <= 20 */
    const int32_t *sample_ids;   /* [n_samples] host, or NULL: the Monte Carlo sample index
                                    (the Philox counter's sample word) of each batch sample;
                                    NULL = 0 .. n_samples-1.  Entries >= 0, copied at creation.
                                    Lets a batch re-run any subset of a study's samples. */
    double cov_map;              /* thermal-map amplitude CoV (param 6), 0 <= cov <= 1 */
} em_mc_params;

typedef struct {
    double ttf_s;          /* time to failure, s; NaN when censored */
    double final_drop;     /* worst IR-drop fraction at retirement or at the horizon */
    double init_drop;      /* worst IR-drop fraction at t = 0 */
    int32_t failed;        /* 1 if the failure threshold was reached */
    int32_t outer_idx;     /* IR re-solves done (the one that failed, if failed) */
    int32_t n_nucleated_trees;
    int32_t n_failed_segs; /* segments with dR > 0 or open */
    int32_t redecided;     /* 1: the FP32 run came within the guard band of the threshold and
                              this result is that of the FP64 re-run (em_run_params.guard_band);
                              2: a learned-screen violation hit this sample and this result is
                              that of its re-run without the screen (see em_surrogate_screen) */
} em_ttf_result;

typedef struct {
    int32_t n_trees, n_stress, n_samples, n_nodes, n_res;
    int32_t max_tree_nodes;
    int32_t prec;
    int32_t trees_only;
    int64_t n_events;      /* nucleation events recorded so far (all samples) */
    int32_t cg_iters_last; /* PCG iterations of the last IR solve */
    int32_t n_outer_done;
    int64_t node_steps;    /* stress-node-steps taken: sum over stepped (tree, sample) of nodes x steps,
                              the re-runs of the last em_run_to_ttf (guard band, learned-screen
                              violations) included */
    int64_t step_launches; /* launches of the stepping kernel */
    double step_kernel_ms; /* summed stream time of those launches (HIP events around each) */
    int64_t cg_iters_total;/* PCG iterations over all IR solves */
    double ir_ms;          /* summed stream time of the IR solves (HIP events) */
    int64_t n_deferred;    /* learned screen: instances deferred at t = 0 */
    int64_t n_activated;   /* learned screen: deferred instances activated (and caught up) later */
    int64_t n_late;        /* learned screen: activated instances that had nucleated before
                              the interval they were activated for */
    int64_t n_violations;  /* learned screen: late activations whose void had also reached the
                              growth phase (a resistance change that earlier IR solves missed);
                              the samples they hit are re-run without the screen, so results
                              equal those of the unscreened run either way */
    double surrogate_ms;   /* wall time of the learned-screen evaluations (features + model) */
    int32_t ir_sys_nodes;  /* nodes of the system the IR PCG iterates (n_nodes, or the terminals
                              of the chain condensation) */
    int32_t ir_sys_edges;  /* its resistors (or reduced edges) */
    int64_t cg_sample_iters; /* PCG iterations summed over samples (one-kernel form: counted in
                              blocks of the graph's iterations per unconverged sample) */
    int32_t chain_m;       /* stress nodes per lane of the chain kernel */
    int32_t chain_wg;      /* its lanes per workgroup */
    int32_t n_chain_wg;    /* workgroups of its present lane layout */
    int32_t n_redecided;   /* samples of the last em_run_to_ttf re-run in FP64 (guard band) */
    int64_t n_void_capped; /* nucleation candidates not turned into a void because their
                              (tree, sample) already held max_voids_per_tree voids, summed over
                              instances since creation or reset.  Reaching the cap is not an
                              error: the run continues with the voids it has (the paper gives no
                              cap; the cap bounds the per-instance void records) */
    int32_t n_screen_rerun;/* samples of the last em_run_to_ttf re-run without the learned screen
                              after a violation */
    int64_t n_ss_skipped;  /* steady-state skipping: instances skipped in the last em_run_to_ttf
                              (an instance woken and skipped again counts twice) */
    int64_t n_ss_woken;    /* of those, woken by an IR re-solve of their sample */
    int64_t n_krylov_bases;      /* reduced stepping: bases built since creation or reset */
    int64_t n_krylov_intervals;  /* instance-intervals taken in reduced form */
    int64_t n_krylov_fallbacks;  /* instance-intervals handed back to exact stepping */
    int64_t krylov_node_steps;   /* stress-node-steps advanced in reduced form (not in node_steps) */
} em_info;

/* Allocator hook: device memory for the batch (e.g. a framework's caching
 * allocator).  NULL => hipMalloc/hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} em_allocator;

/* Build a batch (Sec. IV-A and Fig. 2: the flow's three inputs -- extracted
 * power-grid netlist, material and numerical parameters, optional thermal map
 * -- and the partition of the netlist into wire trees; Sec. IV-F for the
 * Monte Carlo draws): copies the netlist, partitions it into wire trees
 * (same-layer components, root = lowest vertex, depth-first in ascending
 * segment order, each segment refined into intervals_per_seg FD intervals),
 * and on the device evaluates temperatures, diffusivities, control volumes,
 * Monte Carlo draws (mc == NULL: one nominal sample) and the tree factors.
 * Stress starts at sigma_T.  hip_stream: a hipStream_t, or NULL for the null
 * stream.  *out receives the batch (NULL on failure); errors: EM_ERR_ARG for
 * a NULL or inconsistent argument, a struct_size other than this library's
 * sizeof of that struct, more than 2^31 - 2^20 stress nodes, resistors, node
 * incidences or trees times samples (split a larger Monte Carlo study into
 * batches over em_mc_params.sample_ids), non-finite or non-positive geometry, a wire component with a
 * cycle or a netlist without wire segments; EM_ERR_OOM when device or pinned
 * host memory runs out; EM_ERR_HIP for a failing HIP call.  The paper
 * re-partitions the degraded netlist at every aging step; the partition is
 * fixed here (resistance changes never alter which segments share a layer
 * component), so it is done once. */
em_status em_batch_create(const em_grid_desc *grid, const em_material *mat,
                          const em_run_params *run, const em_mc_params *mc,
                          const em_allocator *alloc, void *hip_stream, em_batch **out);
em_status em_batch_destroy(em_batch *b);
em_status em_get_info(em_batch *b, em_info *info);
const char *em_last_error(const em_batch *b);

/* IR solve (eq. 8) for every sample with R = R0 + dR (open segments conduct
 * nothing; nodes with no conducting path to a pad read 0 V), preconditioned
 * CG in FP64 (em_run_params.ir_precond) warm-started from the previous
 * solution.  Updates the per-segment
 * current densities and the stress forcing.  max_drop: [n_samples] host, may
 * be NULL.  Trees-only batches: EM_ERR_STATE. */
em_status em_ir_solve(em_batch *b, double *max_drop);

/* Steady-state immortality screen (Sec. III-B) with the current densities of
 * the last IR solve (or the prescribed ones): a tree is kept for stepping iff
 * some node's zero-flux steady stress exceeds its critical stress.
 * tree_mortal: [n_samples][n_trees] host, may be NULL. */
em_status em_screen(em_batch *b, uint8_t *tree_mortal);

/* Advance every active (sample, tree) by n_steps backward-Euler steps with the
 * current densities held fixed (quasi-static coupling, Sec. IV-A), checking
 * nucleation and growing voids after each step.  n_events: new nucleations in
 * this call, may be NULL. */
em_status em_stress_step(em_batch *b, int32_t n_steps, int32_t *n_events);

/* Full coupled loop (Fig. 2): IR solve, optional screen, then repeated
 * {ir_every steps, dR write-back, IR re-solve} until the worst drop reaches
 * fail_frac (TTF by linear interpolation between re-solves) or the horizon
 * (censored).  out: [n_samples] host. */
em_status em_run_to_ttf(em_batch *b, em_ttf_result *out);

/* Return the batch to its state right after creation: stress sigma_T, no
 * voids, no resistance change, every sample and tree active, IR warm start
 * at vdd, events and counters cleared.  Netlist, draws and statics are kept. */
em_status em_reset(em_batch *b);

/* ---- read-back (host outputs) ---- */
/* Tree partition: tree_off [n_trees+1]; per stress node parent (-1 at a root),
 * seg (segment of the edge to the parent, -1 at a root), dir (+1 if parent->node
 * runs res_a->res_b), vert (grid node or -1 for interior FD nodes), kpos (FD
 * index from res_a); seg_tree [n_res] (-1 for vias).  Any pointer may be NULL. */
em_status em_get_topology(em_batch *b, int32_t *tree_off, int32_t *parent, int32_t *seg,
                          int32_t *dir, int32_t *vert, int32_t *kpos, int32_t *seg_tree);
em_status em_get_stress(em_batch *b, int32_t sample, double *sigma /* [n_stress] */);
em_status em_set_stress(em_batch *b, int32_t sample, const double *sigma /* [n_stress] */);
em_status em_get_voltages(em_batch *b, int32_t sample, double *u /* [n_nodes] */);
em_status em_get_seg_j(em_batch *b, int32_t sample, double *j /* [n_res] */);
/* dR [n_res] (ohm), open [n_res] (0/1) */
em_status em_get_seg_state(em_batch *b, int32_t sample, double *dR, uint8_t *open);
/* Replace one sample's resistance state (the R = R0 + dR of eq. 17 and the
 * open resistors of early failures) that the next IR solve uses: a what-if
 * degradation state.  dR [n_res] finite and >= 0, open [n_res] 0 or 1; host
 * arrays, copied.  Void growth during later steps adds to this dR. */
em_status em_set_seg_state(em_batch *b, int32_t sample, const double *dR, const uint8_t *open);
/* Autotuner: on a batch at t = 0 (just created or reset), time every
 * launch shape this batch can use -- each feasible chain-kernel workgroup
 * size over n_steps steps of the screened instances, and (multigrid IR) the
 * multi-kernel and the one-workgroup-per-sample PCG on a cold solve -- keep
 * the fastest of each and reset the batch.  Results do not depend on the
 * choice beyond the rounding of the IR dot products.  out may be NULL. */
typedef struct {
    int32_t chain_wg;            /* chosen lanes per workgroup */
    int32_t chain_occ;           /* chosen register budget (em_run_params.chain_occ) */
    int32_t ir_launch;           /* chosen IR launch shape (1, 2 or 3; 0: not tuned) */
    int32_t n_wg;                /* chain-kernel candidates tried */
    int32_t wg[12], occ[12];     /* each candidate's lanes per workgroup and register budget */
    double wg_ms[12];            /* stream time of the n_steps steps per candidate */
    double amg_alpha;            /* chosen coarse-correction scale (em_run_params.amg_alpha) */
    double alpha_ms[3];          /* cold IR solve in the chosen launch shape with 1.4, 1.8, 2.2
                                    (-1: not tried) */
    double ir_ms[3];             /* cold IR solve: multi-kernel, one workgroup per sample from HBM,
                                    from LDS (-1: not tried; the one-workgroup forms are not tried
                                    on an iterated system of more than 65 536 nodes with fewer
                                    than 32 samples) */
} em_tune_info;
em_status em_autotune(em_batch *b, int32_t n_steps, em_tune_info *out);
/* Per-node temperature, control volume and critical stress for one sample. */
em_status em_get_node_state(em_batch *b, int32_t sample, double *T, double *V, double *sc);
/* Nucleation events, each 5 int32: sample, tree, step, node, host segment;
 * in no particular order.  *n = number copied (<= cap). */
em_status em_get_events(em_batch *b, int32_t *buf, int32_t cap, int32_t *n);
/* Voids of one sample: iv [cap][6] = tree, node, host seg, phase (0 incubation,
 * 1 growth), nucleation step, early-failure flag; dv [cap][2] = volume (m^3),
 * length (m).  Ordered by tree, then nucleation order. */
em_status em_get_voids(em_batch *b, int32_t sample, int32_t *iv, double *dv, int32_t cap, int32_t *n);
/* Screen output of one sample: tree_mortal [n_trees], seg_mortal [n_res],
 * sigma_ss [n_stress]; any may be NULL. */
em_status em_get_screen(em_batch *b, int32_t sample, uint8_t *tree_mortal, uint8_t *seg_mortal,
                        double *sigma_ss);
/* Test hook: place a void at stress node `node` of `tree` in `sample` as a
 * nucleation there would (host segment and failure mode chosen the same way). */
em_status em_inject_void(em_batch *b, int32_t sample, int32_t tree, int32_t node);
/* Monte Carlo multipliers of one sample: param 0 kappa (with the activation-energy
 * factor when sd_ea_eV > 0), 1 sigma_crit, 2 resistivity
 * (xi [n_res]; 1 for vias and where the CoV is 0), 3 current loading (xi [n_nodes]). */
em_status em_get_xi(em_batch *b, int32_t sample, int32_t param, double *xi);
/* Failed segments of one sample (dR > 0 or open; the set counted by
 * em_ttf_result.n_failed_segs), ascending: *n = their number, the first
 * min(*n, cap) written to idx (idx may be NULL when cap == 0). */
em_status em_get_failed_segments(em_batch *b, int32_t sample, int32_t *idx, int32_t cap, int32_t *n);

/* ---- checkpoint ----
 * em_snapshot copies the batch's dynamic state (stress, currents, IR
 * solution, void records, resistance changes, screen and retirement flags,
 * time-to-failure bookkeeping, step counters, event ring) into host_buf;
 * with host_buf NULL (or cap too small: EM_ERR_ARG) it only reports the size
 * in *used.  em_restore loads such a snapshot into a batch created from the
 * same inputs (EM_ERR_ARG otherwise) and rebuilds the derived state (forcing,
 * factors, reachability).  em_stress_step and em_ir_solve then continue
 * exactly where the snapshot was taken; em_run_to_ttf always starts from
 * t = 0.  The learned-screen attachment and the screen's steady-stress
 * scratch are not part of a snapshot. */
em_status em_snapshot(em_batch *b, void *host_buf, size_t cap, size_t *used);
em_status em_restore(em_batch *b, const void *host_buf, size_t n);

/* ---- learned screen ----
 * A small model, not part of EMSpice 3, that sits in front of the transient
 * stage: from 16 features of a (tree, sample) it predicts the nucleation time
 * of the steady-state-mortal trees, so trees predicted to nucleate long after
 * the current aging interval need not be stepped yet.  Feature vector
 * (float32, in this order): log10 total wire length/1um; log10 longest
 * root-to-node distance/1um; segments/8; junctions (degree >= 3)/4;
 * log10 max|j|/1e9 A/m^2; log10 length-weighted mean |j|/1e9 (both |j|
 * floored at 1e3); log10 mean diffusivity/1e-15 m^2/s (the Arrhenius kappa
 * of Sec. III-D at edge-midpoint temperature, times the Monte Carlo
 * multiplier); log10 mean diffusivity of the edges at the peak node p/1e-15;
 * r = peak over nodes of the zero-flux steady stress of the screen
 * (Sec. III-B) / node critical stress, clamped to [-10, 10] (p = first node of
 * the largest ratio); log10 max(r - 1, 1e-6); log10(Lpk^2 / (pi^2 kappa_pk)
 * / 1 s) - 8 with Lpk the difference of root distances from p to the nearest
 * node whose steady stress is at or below sigma_T (floored at 0.1 um);
 * (temperature at p - 300 K)/100; then early-time scales over the edges
 * (parent(i), i) of length l = segment length / N, diffusivity kappa_e and
 * steady drive g = |steady stress difference| / l: log10 of the least over
 * the edges of pi ds^2 / (4 kappa_e g^2) in seconds (the time a blocked end
 * of a semi-infinite wire with that drive takes to reach the critical stress
 * by the Korhonen solution sigma(0, t) = 2 g sqrt(kappa t / pi); ds = the
 * smaller critical stress of the two ends - sigma_T, floored at 1e3 Pa;
 * clamped to [1, 1e16] s) - 8; log10 kappa_max/1e-15; over the fast edges
 * (kappa_e >= kappa_max / 4) the stress they could build if blocked on both
 * sides, sum of g l / 2, over the least node critical stress - sigma_T
 * (floored at 1e3 Pa, clamped to 10); log10(L_f^2 / (pi^2 kappa_max) / 1 s)
 * - 8 with L_f their total length (floored at 0.1 um).
 * Model: 16 -> 256 -> 256 -> 256 -> 1 perceptron with exact (erf) GELU,
 * output y = log10(t_nuc / 1e8 s).  Hidden-layer products run on bfloat16
 * matrix cores with float32 accumulation (operands rounded to nearest even);
 * bias, GELU, output layer, loss and Adam are float32, with a float32 master
 * copy of every parameter.  Parameter vector (float32, em_mlp_num_params()):
 * W1 [256][16], b1 [256], W2 [256][256], b2, W3 [256][256], b3, w4 [256], b4
 * ([out][in] row-major).  X, t, y arguments of the em_mlp_* calls are DEVICE
 * pointers (X [n][16] row-major); calls on one model must not overlap. */
em_status em_mlp_create(void *hip_stream, em_mlp **out);   /* parameters start at zero */
em_status em_mlp_destroy(em_mlp *m);
const char *em_mlp_last_error(const em_mlp *m);
int32_t em_mlp_num_params(void);
/* Host float32 copies of the parameters; set also clears the Adam moments. */
em_status em_mlp_set_params(em_mlp *m, const float *params, int32_t n);
em_status em_mlp_get_params(em_mlp *m, float *params, int32_t n);
/* y [n] (device) = model(X). */
em_status em_mlp_forward(em_mlp *m, const float *X, int32_t n, float *y);
/* Mean squared error (1/n) sum (y - t)^2 of the model on (X, t) and its
 * gradient; grad [em_mlp_num_params()] host, loss host; either may be NULL. */
em_status em_mlp_grad(em_mlp *m, const float *X, const float *t, int32_t n, float *grad, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * mean squared error of the minibatch (X, t).  loss: host, may be NULL (then
 * the call does not synchronise). */
em_status em_mlp_train_step(em_mlp *m, const float *X, const float *t, int32_t n, float lr, float *loss);

/* ---- allocation-free entry point ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * em_mlp_forward_noalloc computes y [n] = model(X) exactly as em_mlp_forward
 * does (same kernels, same result bit for bit), but keeps the activations in a
 * fixed device array of the library instead of the model's buffers, which
 * em_mlp_forward grows with hipMalloc when n grows.  X [n][16] and y [n] are
 * caller-owned DEVICE pointers; 1 <= n <= em_mlp_noalloc_max_rows() (4096),
 * else EM_ERR_ARG.  Asynchronous on the model's stream (no synchronisation);
 * no device or pinned memory is allocated or freed.  The array (17 MB) exists
 * once per GPU that runs the call and is held until the process ends; every
 * call on that GPU, from any model or thread, uses the same array, so calls
 * that overlap on one GPU race (serialise them, e.g. on one stream), and each
 * call overwrites what the last one left there.  Errors: EM_ERR_ARG for a NULL
 * pointer or a bad n, EM_ERR_HIP when a HIP call fails. */
int32_t em_mlp_noalloc_max_rows(void);
em_status em_mlp_forward_noalloc(em_mlp *m, const float *X, int32_t n, float *y);

/* Features of every (tree, sample) for the current densities, written to X
 * (DEVICE, [n_trees * n_samples][16], row tree * n_samples + sample).
 * Refreshes the screen verdict (em_get_screen) without changing which trees
 * are stepped.  EM_ERR_STATE before any currents exist. */
em_status em_features(em_batch *b, float *X);
/* Attach a learned screen with safety margin m >= 1 (mlp NULL detaches it;
 * the model must outlive its use by the batch).  em_run_to_ttf then, at
 * t = 0, defers every steady-state-mortal tree whose predicted nucleation
 * time exceeds m x (end of the first aging interval); before the aging
 * intervals k = 1, 4, 16, 64, ... (interval k ends at t_{k+1}) it activates
 * every deferred tree with prediction <= m x t_{4k}, the end of the interval
 * before the next check, and catches it up from t = 0 by replaying the stored
 * current densities of the earlier intervals and of interval k on a stream
 * of its own, beside the main launch of interval k (the replays of a run add
 * up to a third of its intervals at most).  Every tree is thus active before
 * the first interval k with prediction <= m x t_{k+1}.  Before each
 * activation check a deferred tree is re-evaluated with the current
 * densities once one of its segment currents has moved by more than 1 % of
 * its largest since its last prediction (a prediction can only move
 * earlier).  The replay reproduces the unscreened run exactly unless an
 * activated tree's void had already reached the growth phase before its
 * activation (a violation, counted in em_info.n_violations; nucleation alone
 * before activation is counted in n_late and is harmless): em_run_to_ttf
 * then re-runs the samples a violation hit without the screen, in a batch
 * over their Monte Carlo sample indices with the same precision and chain
 * kernel layout, and takes their results, resistance changes and opens from
 * it (em_ttf_result.redecided = 2, em_info.n_screen_rerun), so its results
 * equal those of the unscreened run.  Called on a batch that has currents
 * and has not been stepped since creation or reset, it also evaluates the
 * model at once, so that em_stress_step skips the deferred trees;
 * *n_deferred (may be NULL) is then their number, else 0. */
em_status em_surrogate_screen(em_batch *b, em_mlp *mlp, double margin, int64_t *n_deferred);
/* Model output y (log10 of the predicted nucleation time / 1e8 s) and the
 * deferred flags of one sample: [n_trees] host each, either may be NULL.
 * Only trees that were deferral candidates (steady-state mortal and active)
 * are evaluated; y of the others is unspecified. */
em_status em_get_surrogate(em_batch *b, int32_t sample, float *y_hat, uint8_t *deferred);
/* Step of the first nucleation of every (sample, tree), -1 if none:
 * [n_samples][n_trees] host.  The nucleation time is (step + 1) x dt. */
em_status em_first_nucleation(em_batch *b, int32_t *step);

#ifdef __cplusplus
}
#endif
#endif /* EM_MI355X_H */
