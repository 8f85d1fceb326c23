/*
 * em_oracle.c -- plain, slow, obviously correct FP64 reference for the
 * coupled EM/TM stress path (EMSpice 3, arXiv 2604.10743).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * path.
 *
 * Every routine follows the paper's definitions in the paper's order, with
 * scalar loops and no blocking or fusion:
 *   - topology           : wire trees of the extracted netlist (Sec. IV-A)
 *   - node temperatures  : sampled from the thermal map (Sec. III-A), or given
 *                          by the Joule-heating pre-pass (oracle/thermal.py)
 *   - diffusivity        : kappa = D_a(T) B Omega / (k_B T), D_a = D0 exp(-Ea/k_B T)
 *                          (Korhonen PDE, eqs. 10-13)
 *   - descriptor system  : C dsigma/dt = A sigma + f (eq. 18), vertex-centred
 *                          finite volume on the tree graph, blocking ends
 *   - screen             : zero-flux steady state, classify against sigma_crit
 *                          (Sec. III-B)
 *   - BE step            : (C - dt A) sigma^{n+1} = C sigma^n + dt f, solved
 *                          exactly by Gaussian elimination in leaf-to-root order
 *   - nucleation         : peak-stress node with sigma >= sigma_crit; Robin row
 *                          stamped over all incident edges (eq. 20, Sec. IV-D)
 *   - void volume        : atom conservation V_v = -int sigma/B dV (eq. 15),
 *                          accumulated from the flux the Robin row removes
 *   - incubation / growth: critical size = width (eq. 16); early failure through
 *                          an upward via (Sec. IV-C); late-failure dR (eq. 17)
 *   - Monte Carlo draws  : Philox-4x32-10 (Salmon et al., SC'11) -> Box-Muller
 *                          -> unit-mean lognormal with the prescribed CoV (Sec. IV-F)
 *
 * Readings where the paper is silent are listed in the design notes and
 * repeated at the routine that takes them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_E   1.602176634e-19   /* C, exact SI */
#define ORA_KB  1.380649e-23      /* J/K, exact SI */
#define ORA_PI  3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Problem description (caller keeps every array alive while the state is). */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n_nodes;
    const double *xy;          /* [n_nodes*2] */
    const int *layer;          /* [n_nodes]   */
    int n_res;
    const int *ra, *rb;        /* [n_res] */
    const double *len, *w, *h; /* [n_res] */
    const unsigned char *is_via;
    /* temperature source: raster if tmap != NULL, else node_T if != NULL, else T_amb */
    const double *node_T;
    int tnx, tny;
    double tx0, ty0, tdx, tdy;
    const double *tmap;        /* [tny*tnx] row-major */
    double T_amb;
    /* material */
    double B, Omega, Z, rho, Ea_eV, D0, scrit, Q_eV, sigT, delta, rho_ta, h_ta;
    /* numerics */
    int N;                     /* FD intervals per segment */
    double dt;
    int max_voids;
    /* per-segment Monte Carlo multipliers; NULL means 1 */
    const double *xi_k, *xi_s;
    /* stress-node temperatures [ns] from the Joule-heating pre-pass (Sec. III-A,
     * oracle/thermal.py); NULL: sampled from the map as below */
    const double *T_stress;
    /* per-segment resistivity multipliers of the sample (Sec. IV-F sampled
     * input); NULL means 1.  They scale the electron-wind drive and the
     * copper term of eq. 17 (the IR resistances are scaled by the caller). */
    const double *xi_r;
    /* thermal-map amplitude of the sample (Sec. IV-F map perturbation): the
     * rise above T_amb scaled by map_a; 0 means 1 (unscaled).  Scales each
     * edge's thermomigration drive as the scaled field would; the diffusivity
     * factor is in xi_k. */
    double map_a;
} ora_problem;

/* thermomigration drive of an edge at midpoint temperature Te under the
 * sample's map amplitude: (Q/(Omega T)) dT/dx of the scaled field over the
 * nominal one */
static double tm_factor(const ora_problem *P, double Te)
{
    if (!(P->map_a > 0)) return 1.0;
    const double a = P->map_a;
    return a * Te / (P->T_amb + a * (Te - P->T_amb));
}

static double seg_rho(const ora_problem *P, int e)
{
    return P->rho * (P->xi_r ? P->xi_r[e] : 1.0);
}

static int res_is_wire(const ora_problem *P, int r)
{
    return !P->is_via[r] && P->layer[P->ra[r]] == P->layer[P->rb[r]];
}

/* ======================================================================== */
/* Topology: same-layer connected components of the wire resistors form the */
/* trees (Sec. IV-A).  Root = lowest-index vertex; DFS visits incident      */
/* segments in ascending segment index; each segment is refined into N      */
/* intervals and stress nodes are numbered in DFS pre-order.                */
/* ======================================================================== */
typedef struct {
    const ora_problem *P;
    int *inc_off, *inc;        /* vertex -> incident wire segments (ascending) */
    int *vnode;                /* vertex -> stress node (or -1) */
    int *parent, *seg, *dir, *vert, *kpos;
    int *seg_tree;
    int ns, cap, err, cur_tree;
} topo_ctx;

static int topo_emit(topo_ctx *c, int parent, int seg, int dir, int vert, int kpos)
{
    if (c->ns >= c->cap) { c->err = 2; return -1; }
    int i = c->ns++;
    c->parent[i] = parent; c->seg[i] = seg; c->dir[i] = dir;
    c->vert[i] = vert; c->kpos[i] = kpos;
    return i;
}

/* Recursive DFS from vertex u whose stress node is su; arrived through segment `from`. */
static void topo_dfs(topo_ctx *c, int u, int su, int from)
{
    const ora_problem *P = c->P;
    for (int k = c->inc_off[u]; k < c->inc_off[u + 1] && !c->err; ++k) {
        int e = c->inc[k];
        if (e == from) continue;
        int a = P->ra[e], b = P->rb[e];
        int wv = (a == u) ? b : a;
        if (c->vnode[wv] >= 0) { c->err = 1; return; }   /* a cycle: not a tree */
        c->seg_tree[e] = c->cur_tree;
        int from_a = (a == u);                           /* walking a -> b ? */
        int d = from_a ? +1 : -1;
        int prev = su;
        for (int q = 1; q < P->N; ++q) {                 /* interior nodes */
            int kp = from_a ? q : P->N - q;
            prev = topo_emit(c, prev, e, d, -1, kp);
            if (prev < 0) return;
        }
        int sw = topo_emit(c, prev, e, d, wv, from_a ? P->N : 0);
        if (sw < 0) return;
        c->vnode[wv] = sw;
        topo_dfs(c, wv, sw, e);
    }
}

/* Returns 0 on success, 1 if a component has a cycle, 2 if a capacity is exceeded. */
int ora_topology(const ora_problem *P, int cap_trees, int cap_stress,
                 int *n_trees, int *n_stress, int *tree_off,
                 int *parent, int *seg, int *dir, int *vert, int *kpos, int *seg_tree)
{
    topo_ctx c;
    memset(&c, 0, sizeof c);
    c.P = P;
    c.inc_off = calloc((size_t)P->n_nodes + 1, sizeof(int));
    c.inc = malloc(sizeof(int) * (size_t)(2 * P->n_res + 1));
    c.vnode = malloc(sizeof(int) * (size_t)(P->n_nodes + 1));
    for (int r = 0; r < P->n_res; ++r) {
        seg_tree[r] = -1;
        if (!res_is_wire(P, r)) continue;
        c.inc_off[P->ra[r] + 1]++; c.inc_off[P->rb[r] + 1]++;
    }
    for (int v = 0; v < P->n_nodes; ++v) c.inc_off[v + 1] += c.inc_off[v];
    int *fill = calloc((size_t)P->n_nodes + 1, sizeof(int));
    for (int r = 0; r < P->n_res; ++r) {           /* ascending r => ascending lists */
        if (!res_is_wire(P, r)) continue;
        int a = P->ra[r], b = P->rb[r];
        c.inc[c.inc_off[a] + fill[a]++] = r;
        if (b != a) c.inc[c.inc_off[b] + fill[b]++] = r;
        else { c.err = 1; }                          /* self loop */
    }
    free(fill);
    for (int v = 0; v < P->n_nodes; ++v) c.vnode[v] = -1;
    c.parent = parent; c.seg = seg; c.dir = dir; c.vert = vert; c.kpos = kpos;
    c.seg_tree = seg_tree; c.cap = cap_stress;
    int nt = 0;
    tree_off[0] = 0;
    for (int v = 0; v < P->n_nodes && !c.err; ++v) {
        if (c.vnode[v] >= 0 || c.inc_off[v + 1] == c.inc_off[v]) continue;
        if (nt >= cap_trees) { c.err = 2; break; }
        c.cur_tree = nt;
        int s0 = topo_emit(&c, -1, -1, 0, v, 0);
        if (s0 < 0) break;
        c.vnode[v] = s0;
        topo_dfs(&c, v, s0, -1);
        tree_off[++nt] = c.ns;
    }
    *n_trees = nt;
    *n_stress = c.ns;
    free(c.inc_off); free(c.inc); free(c.vnode);
    return c.err;
}

/* ======================================================================== */
/* Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the     */
/* published round function: two 32x32->64 multiplies, a Feistel-like      */
/* swap with key injection, and a Weyl-sequence key schedule.              */
/* ======================================================================== */
void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Unit-mean lognormal multiplier with coefficient of variation `cov` for
 * (seed, sample, segment, param); param 0 = diffusivity, 1 = critical stress.
 * Counter = (segment, sample, param, 0), key = (seed low word, seed high word).
 * Box-Muller on u1 = (x0 + 1) 2^-32 in (0,1], u2 = x1 2^-32 in [0,1). */
double ora_lognormal_xi(uint64_t seed, int sample, int segment, int param, double cov)
{
    if (cov == 0.0) return 1.0;
    uint32_t ctr[4] = {(uint32_t)segment, (uint32_t)sample, (uint32_t)param, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    ora_philox4x32_10(ctr, key, x);
    double u1 = ((double)x[0] + 1.0) * (1.0 / 4294967296.0);
    double u2 = (double)x[1] * (1.0 / 4294967296.0);
    double z = sqrt(-2.0 * log(u1)) * cos(2.0 * ORA_PI * u2);
    double s2 = log(1.0 + cov * cov);
    return exp(-0.5 * s2 + sqrt(s2) * z);
}

void ora_fill_xi(uint64_t seed, int sample, int n_seg, int param, double cov, double *out)
{
    for (int e = 0; e < n_seg; ++e) out[e] = ora_lognormal_xi(seed, sample, e, param, cov);
}

/* Standard normal deviate of counter (index, sample, param, 0): the same
 * Box-Muller branch as above, without the lognormal map. */
double ora_normal_z(uint64_t seed, int sample, int index, int param)
{
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)sample, (uint32_t)param, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    ora_philox4x32_10(ctr, key, x);
    double u1 = ((double)x[0] + 1.0) * (1.0 / 4294967296.0);
    double u2 = (double)x[1] * (1.0 / 4294967296.0);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * ORA_PI * u2);
}

void ora_fill_normal(uint64_t seed, int sample, int n, int param, double *out)
{
    for (int e = 0; e < n; ++e) out[e] = ora_normal_z(seed, sample, e, param);
}

/* ======================================================================== */
/* One sample's state.                                                      */
/* ======================================================================== */
typedef struct {
    ora_problem P;
    int n_trees, ns;
    const int *tree_off, *parent, *seg, *dir, *vert, *kpos, *seg_tree;
    double *T, *V, *kap, *g, *rob, *gsum, *robsum, *phi, *f, *sc, *sigma;
    double *jseg;
    unsigned char *active, *via_up;
    /* voids, max_voids slots per tree */
    int *nv, *vnode, *vseg, *vphase, *vstep, *vearly;
    double *vvol, *vlen;
    double *dR; unsigned char *open;
    int n_ev, cap_ev, *ev;      /* (tree, step, node, host_seg) */
    int n_suppressed;
    double *b, *d;              /* scratch for one tree */
} ora_state;

static double bilinear(const ora_problem *P, double x, double y)
{
    double fx = (x - P->tx0) / P->tdx, fy = (y - P->ty0) / P->tdy;
    if (fx < 0) fx = 0;
    if (fy < 0) fy = 0;
    if (fx > P->tnx - 1) fx = P->tnx - 1;
    if (fy > P->tny - 1) fy = P->tny - 1;
    int ix = (int)floor(fx), iy = (int)floor(fy);
    if (ix > P->tnx - 2) ix = P->tnx - 2;
    if (iy > P->tny - 2) iy = P->tny - 2;
    if (ix < 0) ix = 0;
    if (iy < 0) iy = 0;
    double tx = fx - ix, ty = fy - iy;
    int ix1 = (P->tnx > 1) ? ix + 1 : ix, iy1 = (P->tny > 1) ? iy + 1 : iy;
    const double *M = P->tmap;
    double t00 = M[iy * P->tnx + ix], t01 = M[iy * P->tnx + ix1];
    double t10 = M[iy1 * P->tnx + ix], t11 = M[iy1 * P->tnx + ix1];
    return (1 - ty) * ((1 - tx) * t00 + tx * t01) + ty * ((1 - tx) * t10 + tx * t11);
}

/* Temperature at every stress node.  Raster: bilinear sample at the node's
 * position.  Vertex temperatures: interior nodes interpolate linearly along
 * the segment.  Neither: uniform ambient. */
static void node_temperatures(ora_state *S)
{
    const ora_problem *P = &S->P;
    if (P->T_stress) {
        for (int i = 0; i < S->ns; ++i) S->T[i] = P->T_stress[i];
        return;
    }
    for (int i = 0; i < S->ns; ++i) {
        int e = S->seg[i];
        double x, y;
        if (S->vert[i] >= 0) {
            x = P->xy[2 * S->vert[i]]; y = P->xy[2 * S->vert[i] + 1];
        } else {
            double t = (double)S->kpos[i] / P->N;
            int a = P->ra[e], b = P->rb[e];
            x = P->xy[2 * a] + t * (P->xy[2 * b] - P->xy[2 * a]);
            y = P->xy[2 * a + 1] + t * (P->xy[2 * b + 1] - P->xy[2 * a + 1]);
        }
        if (P->tmap) S->T[i] = bilinear(P, x, y);
        else if (P->node_T) {
            if (S->vert[i] >= 0) S->T[i] = P->node_T[S->vert[i]];
            else {
                double t = (double)S->kpos[i] / P->N;
                S->T[i] = P->node_T[P->ra[e]] + t * (P->node_T[P->rb[e]] - P->node_T[P->ra[e]]);
            }
        } else S->T[i] = P->T_amb;
    }
}

ora_state *ora_create(const ora_problem *Pin, int n_trees, int ns, const int *tree_off,
                      const int *parent, const int *seg, const int *dir, const int *vert,
                      const int *kpos, const int *seg_tree, int cap_events)
{
    ora_state *S = calloc(1, sizeof *S);
    S->P = *Pin;
    const ora_problem *P = &S->P;
    S->n_trees = n_trees; S->ns = ns;
    S->tree_off = tree_off; S->parent = parent; S->seg = seg; S->dir = dir;
    S->vert = vert; S->kpos = kpos; S->seg_tree = seg_tree;
    size_t n = (size_t)ns;
    S->T = calloc(n, 8); S->V = calloc(n, 8); S->kap = calloc(n, 8); S->g = calloc(n, 8);
    S->rob = calloc(n, 8); S->gsum = calloc(n, 8); S->robsum = calloc(n, 8);
    S->phi = calloc(n, 8); S->f = calloc(n, 8); S->sc = calloc(n, 8); S->sigma = calloc(n, 8);
    S->b = calloc(n, 8); S->d = calloc(n, 8);
    S->jseg = calloc((size_t)P->n_res, 8);
    S->dR = calloc((size_t)P->n_res, 8);
    S->open = calloc((size_t)P->n_res, 1);
    S->active = malloc((size_t)n_trees + 1);
    memset(S->active, 1, (size_t)n_trees + 1);
    S->via_up = calloc((size_t)P->n_nodes + 1, 1);
    int mv = P->max_voids > 0 ? P->max_voids : 1;
    size_t nvs = (size_t)n_trees * mv + 1;
    S->nv = calloc((size_t)n_trees + 1, sizeof(int));
    S->vnode = calloc(nvs, sizeof(int)); S->vseg = calloc(nvs, sizeof(int));
    S->vphase = calloc(nvs, sizeof(int)); S->vstep = calloc(nvs, sizeof(int));
    S->vearly = calloc(nvs, sizeof(int));
    S->vvol = calloc(nvs, 8); S->vlen = calloc(nvs, 8);
    S->cap_ev = cap_events; S->ev = calloc((size_t)cap_events * 4 + 4, sizeof(int));

    /* Via map (Sec. IV-C): a vertex has an upward via if some inter-layer
     * resistor joins it to a node on a strictly higher layer. */
    for (int r = 0; r < P->n_res; ++r) {
        if (res_is_wire(P, r)) continue;
        int a = P->ra[r], b = P->rb[r];
        if (P->layer[b] > P->layer[a]) S->via_up[a] = 1;
        if (P->layer[a] > P->layer[b]) S->via_up[b] = 1;
    }

    node_temperatures(S);

    /* Per-edge diffusivity and conductance; per-node control volume; Robin
     * weights a*kappa/delta; critical stress = sigma_crit x min over incident
     * segments of the sample's multiplier. */
    for (int i = 0; i < ns; ++i) S->sc[i] = INFINITY;
    for (int i = 0; i < ns; ++i) {
        int p = parent[i];
        if (p < 0) continue;
        int e = seg[i];
        double dx = P->len[e] / P->N;
        double a = P->w[e] * P->h[e];
        double Te = 0.5 * (S->T[i] + S->T[p]);
        double xk = P->xi_k ? P->xi_k[e] : 1.0;
        double Da = P->D0 * exp(-P->Ea_eV * ORA_E / (ORA_KB * Te));
        double kap = xk * Da * P->B * P->Omega / (ORA_KB * Te);
        S->kap[i] = kap;
        S->g[i] = a * kap / dx;
        S->rob[i] = a * kap / P->delta;
        S->V[i] += 0.5 * a * dx;  S->V[p] += 0.5 * a * dx;
        S->gsum[i] += S->g[i];    S->gsum[p] += S->g[i];
        S->robsum[i] += S->rob[i]; S->robsum[p] += S->rob[i];
        double xs = P->xi_s ? P->xi_s[e] : 1.0;
        double sce = P->scrit * xs;
        if (sce < S->sc[i]) S->sc[i] = sce;
        if (sce < S->sc[p]) S->sc[p] = sce;
    }
    for (int i = 0; i < ns; ++i) S->sigma[i] = P->sigT;
    return S;
}

void ora_destroy(ora_state *S)
{
    if (!S) return;
    free(S->T); free(S->V); free(S->kap); free(S->g); free(S->rob); free(S->gsum);
    free(S->robsum); free(S->phi); free(S->f); free(S->sc); free(S->sigma);
    free(S->b); free(S->d); free(S->jseg); free(S->dR); free(S->open); free(S->active);
    free(S->via_up); free(S->nv); free(S->vnode); free(S->vseg); free(S->vphase);
    free(S->vstep); free(S->vearly); free(S->vvol); free(S->vlen); free(S->ev);
    free(S);
}

/* Drive terms from the current densities (eq. 13 notation): S = eZ rho j / Omega
 * along a->b; M = (Q/(Omega T_e)) dT/dx along a->b (edge-midpoint T, edge
 * difference for the gradient).  For the edge from parent p to child i with
 * orientation dir (+1 if p->i runs a->b): phi = dir * g dx (S + M) enters the
 * child's balance and leaves the parent's, which is the FV form of the flux
 * kappa (dsigma/dx - S - M) and makes every end blocking (eq. 12). */
void ora_set_j(ora_state *S, const double *jseg)
{
    const ora_problem *P = &S->P;
    memcpy(S->jseg, jseg, sizeof(double) * (size_t)P->n_res);
    for (int i = 0; i < S->ns; ++i) S->f[i] = 0.0;
    for (int i = 0; i < S->ns; ++i) {
        int p = S->parent[i];
        if (p < 0) { S->phi[i] = 0; continue; }
        int e = S->seg[i];
        double dx = P->len[e] / P->N;
        double Te = 0.5 * (S->T[i] + S->T[p]);
        double Sd = ORA_E * P->Z * seg_rho(P, e) * jseg[e] / P->Omega;
        double Md = S->dir[i] * (P->Q_eV * ORA_E / (P->Omega * Te)) * (S->T[i] - S->T[p]) / dx;
        Md *= tm_factor(P, Te);
        double phi = S->dir[i] * S->g[i] * dx * (Sd + Md);
        S->phi[i] = phi;
        S->f[i] += phi;
        S->f[p] -= phi;
    }
}

/* Steady-state screen (Sec. III-B): the zero-flux steady state satisfies
 * sigma_child - sigma_parent = dir dx (S + M) on every edge, independent of
 * kappa; the constant follows from conservation, sum V sigma = sum V sigma_T.
 * Node mortal iff its finite steady stress exceeds its critical stress;
 * segment mortal iff any of its nodes is; tree mortal iff any node is. */
void ora_screen(ora_state *S, unsigned char *tree_mortal, unsigned char *seg_mortal, double *sig_ss)
{
    const ora_problem *P = &S->P;
    for (int r = 0; r < P->n_res; ++r) seg_mortal[r] = 0;
    for (int t = 0; t < S->n_trees; ++t) {
        int i0 = S->tree_off[t], i1 = S->tree_off[t + 1];
        double *psi = S->b;
        psi[i0] = 0.0;
        for (int i = i0 + 1; i < i1; ++i) {
            int p = S->parent[i], e = S->seg[i];
            double dx = P->len[e] / P->N;
            double Te = 0.5 * (S->T[i] + S->T[p]);
            double Sd = ORA_E * P->Z * seg_rho(P, e) * S->jseg[e] / P->Omega;
            double Md = S->dir[i] * (P->Q_eV * ORA_E / (P->Omega * Te)) * (S->T[i] - S->T[p]) / dx;
            Md *= tm_factor(P, Te);
            psi[i] = psi[p] + S->dir[i] * dx * (Sd + Md);
        }
        double num = 0, den = 0;
        for (int i = i0; i < i1; ++i) { num += S->V[i] * psi[i]; den += S->V[i]; }
        double mean = num / den;
        int mortal = 0;
        for (int i = i0; i < i1; ++i) {
            double s = P->sigT + psi[i] - mean;
            sig_ss[i] = s;
            if (isfinite(s) && s > S->sc[i]) {
                mortal = 1;
                /* the node belongs to its parent edge's segment and to every
                 * child edge's segment */
                if (S->parent[i] >= 0) seg_mortal[S->seg[i]] = 1;
            }
        }
        for (int i = i0 + 1; i < i1; ++i) {
            int p = S->parent[i];
            double s = P->sigT + psi[p] - mean;
            if (isfinite(s) && s > S->sc[p]) seg_mortal[S->seg[i]] = 1;
        }
        tree_mortal[t] = (unsigned char)mortal;
    }
}

void ora_set_active(ora_state *S, const unsigned char *tree_active)
{
    for (int t = 0; t < S->n_trees; ++t) S->active[t] = tree_active[t];
}

static int void_slot(const ora_state *S, int t, int i)
{
    int mv = S->P.max_voids;
    for (int k = 0; k < S->nv[t]; ++k)
        if (S->vnode[t * mv + k] == i) return k;
    return -1;
}

/* Late-failure resistance increase (eq. 17) with V_v - V_crit = (l - W) W H:
 * dR = (l - W) [rho_Ta / (h_Ta (2H + W)) - rho_Cu / (W H)], clamped at 0. */
double ora_late_dR(double l, double W, double H, double h_ta, double rho_ta, double rho_cu)
{
    double ex = l - W;
    if (ex <= 0) return 0.0;
    return ex * (rho_ta / (h_ta * (2 * H + W)) - rho_cu / (W * H));
}

static double late_dR(const ora_problem *P, int e, double l, double W, double H)
{
    return ora_late_dR(l, W, H, P->h_ta, P->rho_ta, seg_rho(P, e));
}

/* Host segment of a new void: the node's own segment for an interior node;
 * for a vertex, the incident tree segment whose electron wind drives atoms
 * away from it hardest (signed j with the vertex at the b end, -j at the a
 * end), ties to the lowest segment index. */
static int host_segment(const ora_state *S, int t, int v)
{
    const ora_problem *P = &S->P;
    if (S->vert[v] < 0) return S->seg[v];
    int x = S->vert[v];
    int best = -1; double bd = 0;
    for (int e = 0; e < P->n_res; ++e) {
        if (S->seg_tree[e] != t) continue;
        if (P->ra[e] != x && P->rb[e] != x) continue;
        double d = (P->rb[e] == x) ? S->jseg[e] : -S->jseg[e];
        if (best < 0 || d > bd) { best = e; bd = d; }
    }
    return best;
}

static void refresh_dR(ora_state *S)
{
    const ora_problem *P = &S->P;
    int mv = P->max_voids;
    for (int r = 0; r < P->n_res; ++r) S->dR[r] = 0.0;
    for (int t = 0; t < S->n_trees; ++t)
        for (int k = 0; k < S->nv[t]; ++k) {
            int q = t * mv + k, e = S->vseg[q];
            if (!S->vearly[q]) S->dR[e] += late_dR(P, e, S->vlen[q], P->w[e], P->h[e]);
        }
}

/* Step size of the following ora_steps calls (a non-uniform time grid is a
 * sequence of calls with their own dt; nothing here depends on a previous dt). */
void ora_set_dt(ora_state *S, double dt)
{
    S->P.dt = dt;
}

/* Advance every active tree by n_steps backward-Euler steps starting at step
 * index step0.  After each step: grow existing voids, then test nucleation. */
int ora_steps(ora_state *S, int n_steps, int step0)
{
    const ora_problem *P = &S->P;
    const double dt = P->dt;
    int mv = P->max_voids;
    int new_ev = 0;
    for (int t = 0; t < S->n_trees; ++t) {
        if (!S->active[t]) continue;
        int i0 = S->tree_off[t], i1 = S->tree_off[t + 1];
        for (int st = 0; st < n_steps; ++st) {
            /* Backward Euler for the increment: (C - dt A) (sigma^{n+1} - sigma^n)
             * = dt (A sigma^n + f), the same equation as (C - dt A) sigma^{n+1} =
             * C sigma^n + dt f.  The right-hand side is assembled edge by edge from
             * the net flux of each edge (diffusion plus drive), so its rounding
             * shrinks with the flux and the stress content does not drift once a
             * tree is at steady state.  A void row keeps only the diffusion of its
             * edges and adds the Robin sink (eq. 20). */
            for (int i = i0; i < i1; ++i) {
                int isv = void_slot(S, t, i) >= 0;
                S->b[i] = isv ? -dt * S->robsum[i] * S->sigma[i] : 0.0;
                S->d[i] = S->V[i] + dt * S->gsum[i] + (isv ? dt * S->robsum[i] : 0.0);
            }
            for (int i = i0 + 1; i < i1; ++i) {
                int p = S->parent[i];
                double diff = S->g[i] * (S->sigma[p] - S->sigma[i]);  /* into i */
                double full = diff + S->phi[i];
                S->b[i] += dt * (void_slot(S, t, i) >= 0 ? diff : full);
                S->b[p] -= dt * (void_slot(S, t, p) >= 0 ? diff : full);
            }
            /* eliminate leaves into parents (reverse pre-order) */
            for (int i = i1 - 1; i > i0; --i) {
                int p = S->parent[i];
                double c = dt * S->g[i];            /* -(C - dt A)_{p,i} */
                double m = c / S->d[i];
                S->d[p] -= m * c;
                S->b[p] += m * S->b[i];
            }
            /* back substitution root-to-leaves (pre-order); b becomes the increment */
            S->b[i0] = S->b[i0] / S->d[i0];
            for (int i = i0 + 1; i < i1; ++i)
                S->b[i] = (S->b[i] + dt * S->g[i] * S->b[S->parent[i]]) / S->d[i];
            for (int i = i0; i < i1; ++i) S->sigma[i] += S->b[i];

            /* void growth from atom conservation (eq. 15): the Robin row removes
             * dt*(robsum*sigma_v + f_v) of stress content per step */
            for (int k = 0; k < S->nv[t]; ++k) {
                int q = t * mv + k, v = S->vnode[q], e = S->vseg[q];
                S->vvol[q] += dt / P->B * (S->robsum[v] * S->sigma[v] + S->f[v]);
                double W = P->w[e], H = P->h[e];
                double l = S->vvol[q] / (W * H);
                if (l > P->len[e]) l = P->len[e];
                S->vlen[q] = l;
                if (S->vphase[q] == 0 && l >= W) {
                    S->vphase[q] = 1;                 /* incubation over (eq. 16) */
                    if (S->vearly[q]) S->open[e] = 1; /* early failure: open */
                }
            }

            /* nucleation: peak stress among non-void nodes at or above their
             * critical stress; ties (relative 1e-12) go to the lowest index */
            if (S->nv[t] < mv || mv <= 0) {
                double m = -INFINITY; int any = 0;
                for (int i = i0; i < i1; ++i) {
                    if (void_slot(S, t, i) >= 0) continue;
                    if (S->sigma[i] >= S->sc[i]) { any = 1; if (S->sigma[i] > m) m = S->sigma[i]; }
                }
                if (any && mv > 0) {
                    double thr = m - 1e-12 * fabs(m);
                    int v = -1;
                    for (int i = i0; i < i1 && v < 0; ++i) {
                        if (void_slot(S, t, i) >= 0) continue;
                        if (S->sigma[i] >= S->sc[i] && S->sigma[i] >= thr) v = i;
                    }
                    int q = t * mv + S->nv[t];
                    S->vnode[q] = v;
                    S->vseg[q] = host_segment(S, t, v);
                    S->vphase[q] = 0;
                    S->vstep[q] = step0 + st;
                    S->vearly[q] = (S->vert[v] >= 0) ? S->via_up[S->vert[v]] : 0;
                    S->vvol[q] = 0; S->vlen[q] = 0;
                    S->nv[t]++;
                    if (S->n_ev < S->cap_ev) {
                        int *E = S->ev + 4 * S->n_ev;
                        E[0] = t; E[1] = step0 + st; E[2] = v; E[3] = S->vseg[q];
                    }
                    S->n_ev++;
                    new_ev++;
                } else if (any) {
                    S->n_suppressed++;
                }
            } else {
                for (int i = i0; i < i1; ++i)
                    if (void_slot(S, t, i) < 0 && S->sigma[i] >= S->sc[i]) { S->n_suppressed++; break; }
            }
        }
    }
    refresh_dR(S);
    return new_ev;
}

/* ---------------------------- accessors --------------------------------- */
int ora_n_events(const ora_state *S) { return S->n_ev; }
int ora_n_suppressed(const ora_state *S) { return S->n_suppressed; }
void ora_get_events(const ora_state *S, int *out)
{
    int n = S->n_ev < S->cap_ev ? S->n_ev : S->cap_ev;
    memcpy(out, S->ev, sizeof(int) * 4 * (size_t)n);
}
void ora_get_sigma(const ora_state *S, double *out) { memcpy(out, S->sigma, 8 * (size_t)S->ns); }
void ora_set_sigma(ora_state *S, const double *in) { memcpy(S->sigma, in, 8 * (size_t)S->ns); }
void ora_get_node_arrays(const ora_state *S, double *T, double *V, double *g, double *f,
                         double *sc, double *robsum)
{
    size_t n = 8 * (size_t)S->ns;
    if (T) memcpy(T, S->T, n);
    if (V) memcpy(V, S->V, n);
    if (g) memcpy(g, S->g, n);
    if (f) memcpy(f, S->f, n);
    if (sc) memcpy(sc, S->sc, n);
    if (robsum) memcpy(robsum, S->robsum, n);
}
void ora_get_seg_state(const ora_state *S, double *dR, unsigned char *open)
{
    memcpy(dR, S->dR, 8 * (size_t)S->P.n_res);
    memcpy(open, S->open, (size_t)S->P.n_res);
}
/* voids: per slot (tree, node, seg, phase, step, early) ints and (vol, len) doubles */
int ora_get_voids(const ora_state *S, int *iv, double *dv)
{
    int mv = S->P.max_voids, n = 0;
    for (int t = 0; t < S->n_trees; ++t)
        for (int k = 0; k < S->nv[t]; ++k) {
            int q = t * mv + k;
            if (iv) {
                int *I = iv + 6 * n;
                I[0] = t; I[1] = S->vnode[q]; I[2] = S->vseg[q]; I[3] = S->vphase[q];
                I[4] = S->vstep[q]; I[5] = S->vearly[q];
            }
            if (dv) { dv[2 * n] = S->vvol[q]; dv[2 * n + 1] = S->vlen[q]; }
            ++n;
        }
    return n;
}
/* Inject a void at stress node v of tree t (test hook for junction and
 * early-failure cases); host segment chosen as at a real nucleation. */
int ora_inject_void(ora_state *S, int t, int v, int step)
{
    int mv = S->P.max_voids;
    if (S->nv[t] >= mv) return -1;
    int q = t * mv + S->nv[t];
    S->vnode[q] = v; S->vseg[q] = host_segment(S, t, v); S->vphase[q] = 0; S->vstep[q] = step;
    S->vearly[q] = (S->vert[v] >= 0) ? S->via_up[S->vert[v]] : 0;
    S->vvol[q] = 0; S->vlen[q] = 0;
    S->nv[t]++;
    return S->vseg[q];
}
