// Aggregation multigrid preconditioner for the IR solve (the PCG of eq. 8).
//
// Hierarchy (host, once per batch, on the nominal conductances 1/R0): the
// level-0 graph is the resistor network restricted to the non-pad nodes.
// Each coarsening applies heavy-edge pair matching twice (a node pairs with
// its strongest unmatched neighbour when that coupling is at least a quarter
// of its strongest one), so an aggregate holds up to four nodes of the finer
// level, until at most AMG_NC_MAX nodes remain or coarsening stalls.
//
// Operators (device, every solve, per Monte Carlo sample): with piecewise-
// constant prolongation P the Galerkin operator P^T A P of a graph Laplacian
// plus a diagonal is again one: the conductance of a coarse edge is the sum of
// the finer edges it merges, and the diagonal of an aggregate is the sum of
// its members' diagonals minus twice its internal conductances.  At level 0 a
// free node's diagonal is the IR diagonal, a dead node (no path to a pad)
// carries 1 and no couplings.  The coarsest operator is inverted densely in
// LDS (symmetrised), or reduced to its diagonal when coarsening stalled above
// AMG_NC_MAX nodes.
//
// V-cycle (symmetric, so PCG stays valid): damped Jacobi pre-smoothing from
// zero, residual, restriction by summing over members, recursion, prolongation
// of the coarse correction scaled by alpha, damped Jacobi post-smoothing.  The
// result is zeroed off the free nodes, which keeps the PCG direction zero on
// pads and dead nodes.  Vectors are [S][n] per level; converged samples skip.
// One thread per node and level step.  At the coarse levels the prolongation
// is formed on the fly inside the post-smoother (one kernel per level on the
// way up); fusing a level's residual into the restriction instead serialises
// several SpMV rows per thread and measured slower, as did running the small
// levels in one workgroup per sample.
#include "em_internal.h"

#include <algorithm>
#include <cmath>
#include <unordered_map>

namespace em {

// ------------------------------------------------------------------------
// host: hierarchy
// ------------------------------------------------------------------------
namespace {

struct Graph {
    int n = 0;
    std::vector<int> ea, eb;
    std::vector<double> w;
    std::vector<char> excl;             // node outside the system (level 0: pads)
};

void csr_adj(const Graph &g, std::vector<int> &off, std::vector<int> &nbr, std::vector<int> &eid)
{
    off.assign(g.n + 1, 0);
    for (size_t e = 0; e < g.ea.size(); ++e) { off[g.ea[e] + 1]++; off[g.eb[e] + 1]++; }
    for (int i = 0; i < g.n; ++i) off[i + 1] += off[i];
    nbr.assign(off[g.n], 0);
    eid.assign(off[g.n], 0);
    std::vector<int> fill(off.begin(), off.end() - 1);
    for (size_t e = 0; e < g.ea.size(); ++e) {
        int a = g.ea[e], b = g.eb[e];
        nbr[fill[a]] = b; eid[fill[a]++] = (int)e;
        nbr[fill[b]] = a; eid[fill[b]++] = (int)e;
    }
}

// One pass of heavy-edge matching; map[i] = pair index (-1 for excluded nodes).
int match_pass(const Graph &g, std::vector<int> &map)
{
    std::vector<int> off, nbr, eid;
    csr_adj(g, off, nbr, eid);
    std::vector<int> mate(g.n, -1);
    for (int i = 0; i < g.n; ++i) {
        if (g.excl[i] || mate[i] != -1) continue;
        double wmax = 0.0;
        for (int k = off[i]; k < off[i + 1]; ++k)
            if (nbr[k] != i && !g.excl[nbr[k]]) wmax = std::max(wmax, g.w[eid[k]]);
        int best = -1;
        double bw = 0.0;
        for (int k = off[i]; k < off[i + 1]; ++k) {
            int j = nbr[k];
            if (j == i || g.excl[j] || mate[j] != -1) continue;
            if (g.w[eid[k]] > bw) { bw = g.w[eid[k]]; best = j; }
        }
        if (best >= 0 && bw >= 0.25 * wmax) { mate[i] = best; mate[best] = i; }
        else mate[i] = i;
    }
    map.assign(g.n, -1);
    int c = 0;
    for (int i = 0; i < g.n; ++i) {
        if (g.excl[i] || map[i] != -1) continue;
        map[i] = c;
        if (mate[i] != i) map[mate[i]] = c;
        ++c;
    }
    return c;
}

// Collapse g through map (nc coarse nodes): coarse graph + the level maps.
Graph collapse(const Graph &g, const std::vector<int> &map, int nc, AmgHostLevel *L)
{
    Graph c;
    c.n = nc;
    c.excl.assign(nc, 0);
    std::unordered_map<uint64_t, int> key;
    std::vector<std::vector<int>> src, internal(nc);
    for (size_t e = 0; e < g.ea.size(); ++e) {
        int I = map[g.ea[e]], J = map[g.eb[e]];
        if (I < 0 || J < 0) continue;
        if (I == J) { internal[I].push_back((int)e); continue; }
        if (I > J) std::swap(I, J);
        uint64_t k = ((uint64_t)I << 32) | (uint32_t)J;
        auto it = key.find(k);
        int E;
        if (it == key.end()) {
            E = (int)c.ea.size();
            key.emplace(k, E);
            c.ea.push_back(I); c.eb.push_back(J); c.w.push_back(0.0);
            src.emplace_back();
        } else {
            E = it->second;
        }
        c.w[E] += g.w[e];
        src[E].push_back((int)e);
    }
    if (L) {
        L->n = nc; L->ne = (int)c.ea.size(); L->nf = g.n; L->nef = (int)g.ea.size();
        L->agg = map;
        L->mem_off.assign(nc + 1, 0);
        for (int i = 0; i < g.n; ++i) if (map[i] >= 0) L->mem_off[map[i] + 1]++;
        for (int I = 0; I < nc; ++I) L->mem_off[I + 1] += L->mem_off[I];
        L->mem.assign(L->mem_off[nc], 0);
        std::vector<int> fill(L->mem_off.begin(), L->mem_off.end() - 1);
        for (int i = 0; i < g.n; ++i) if (map[i] >= 0) L->mem[fill[map[i]]++] = i;
        L->int_off.assign(nc + 1, 0);
        L->int_e.clear();
        for (int I = 0; I < nc; ++I) {
            L->int_e.insert(L->int_e.end(), internal[I].begin(), internal[I].end());
            L->int_off[I + 1] = (int)L->int_e.size();
        }
        L->src_off.assign(L->ne + 1, 0);
        L->src_e.clear();
        for (int E = 0; E < L->ne; ++E) {
            L->src_e.insert(L->src_e.end(), src[E].begin(), src[E].end());
            L->src_off[E + 1] = (int)L->src_e.size();
        }
        csr_adj(c, L->adj_off, L->adj_nbr, L->adj_e);
    }
    return c;
}

}  // namespace

AmgHost amg_build(int n_nodes, const uint8_t *is_pad, int n_res, const int *ra, const int *rb,
                  const double *R0)
{
    AmgHost H;
    Graph g;
    g.n = n_nodes;
    g.excl.assign(n_nodes, 0);
    for (int i = 0; i < n_nodes; ++i) g.excl[i] = is_pad[i] ? 1 : 0;
    for (int r = 0; r < n_res; ++r) {
        int a = ra[r], b = rb[r];
        if (a == b || is_pad[a] || is_pad[b]) continue;
        H.e0_res.push_back(r); H.e0_a.push_back(a); H.e0_b.push_back(b);
        g.ea.push_back(a); g.eb.push_back(b); g.w.push_back(1.0 / R0[r]);
    }
    H.lev.resize(1);
    int n_sys = 0;
    for (int i = 0; i < n_nodes; ++i) n_sys += !g.excl[i];
    if (n_sys < 2) return H;
    const int npass = 2;          // matching passes per level (3 or 4 measured slower)
    while ((int)H.lev.size() <= AMG_MAXLEV) {
        std::vector<int> agg(g.n), mk;
        for (int i = 0; i < g.n; ++i) agg[i] = g.excl[i] ? -1 : i;
        Graph gk = g;
        int n2 = 0;
        for (int pass = 0; pass < npass; ++pass) {
            n2 = match_pass(gk, mk);
            for (int i = 0; i < g.n; ++i) agg[i] = agg[i] < 0 ? -1 : mk[agg[i]];
            if (pass + 1 < npass) gk = collapse(gk, mk, n2, nullptr);
        }
        AmgHostLevel L;
        Graph c = collapse(g, agg, n2, &L);
        int n_prev = 0;
        for (int i = 0; i < g.n; ++i) n_prev += !g.excl[i];
        H.lev.push_back(std::move(L));
        if (n2 <= AMG_NC_MAX || n2 * 5 > n_prev * 4) break;   // small enough, or stalled
        g = std::move(c);
    }
    return H;
}

// ------------------------------------------------------------------------
// device
// ------------------------------------------------------------------------
#define AMG_BS 256

// level-0 values of one sample: diagonal of a system node, conductance of a
// level-0 edge (zero unless both ends are free)
__device__ inline bool free0(const Dev &d, int s, int i)
{
    return d.live[(size_t)s * d.n_nodes + i] && !d.is_pad[i];
}
__device__ inline double D0(const Dev &d, int s, int i)
{
    return free0(d, s, i) ? d.diag[(size_t)s * d.n_nodes + i] : 1.0;
}
__device__ inline double g0(const Dev &d, const Amg0 &z, int s, int e)
{
    int a = z.e0_a[e], b = z.e0_b[e];
    return (free0(d, s, a) && free0(d, s, b)) ? d.G[(size_t)s * d.n_res + z.e0_res[e]] : 0.0;
}

__global__ __launch_bounds__(AMG_BS) void k_amg_asm_nodes(Dev d, Amg0 z, AmgLevel L, AmgLevel F, int lvl)
{
    int I = blockIdx.x * AMG_BS + threadIdx.x, s = blockIdx.y;
    if (I >= L.n || d.conv[s]) return;
    double acc = 0.0;
    for (int k = L.mem_off[I]; k < L.mem_off[I + 1]; ++k) {
        int m = L.mem[k];
        acc += lvl == 1 ? D0(d, s, m) : F.D[(size_t)s * F.n + m];
    }
    double in = 0.0;
    for (int k = L.int_off[I]; k < L.int_off[I + 1]; ++k) {
        int e = L.int_e[k];
        in += lvl == 1 ? g0(d, z, s, e) : F.W[(size_t)s * F.ne + e];
    }
    L.D[(size_t)s * L.n + I] = acc - 2.0 * in;
}

__global__ __launch_bounds__(AMG_BS) void k_amg_asm_edges(Dev d, Amg0 z, AmgLevel L, AmgLevel F, int lvl)
{
    int E = blockIdx.x * AMG_BS + threadIdx.x, s = blockIdx.y;
    if (E >= L.ne || d.conv[s]) return;
    double acc = 0.0;
    for (int k = L.src_off[E]; k < L.src_off[E + 1]; ++k) {
        int e = L.src_e[k];
        acc += lvl == 1 ? g0(d, z, s, e) : F.W[(size_t)s * F.ne + e];
    }
    L.W[(size_t)s * L.ne + E] = acc;
}

// Conductances in adjacency order: row I's couplings contiguous, as the
// residual and smoothing passes read them (the edge numbering scatters them).
__global__ __launch_bounds__(AMG_BS) void k_amg_asm_adj(Dev d, AmgLevel L)
{
    int k = blockIdx.x * AMG_BS + threadIdx.x, s = blockIdx.y;
    if (k >= 2 * L.ne || d.conv[s]) return;
    L.Wa[(size_t)s * 2 * L.ne + k] = L.W[(size_t)s * L.ne + L.adj_e[k]];
}

// Dense inverse of the coarsest operator of one sample (Gauss-Jordan in LDS,
// no pivoting: the operator is symmetric positive definite), symmetrised.
__global__ __launch_bounds__(AMG_BS) void k_amg_coarse_inv(AmgLevel C, mgreal *Ainv, const uint8_t *conv)
{
    __shared__ double A[AMG_NC_MAX][AMG_NC_MAX];
    __shared__ double prow[AMG_NC_MAX], pcol[AMG_NC_MAX];
    const int s = blockIdx.x, n = C.n, t = threadIdx.x;
    if (conv[s]) return;                    // converged samples take no V-cycle
    for (int k = t; k < n * n; k += AMG_BS) A[k / n][k % n] = 0.0;
    __syncthreads();
    for (int i = t; i < n; i += AMG_BS) {
        A[i][i] = C.D[(size_t)s * n + i];
        for (int k = C.adj_off[i]; k < C.adj_off[i + 1]; ++k)
            A[i][C.adj_nbr[k]] -= C.W[(size_t)s * C.ne + C.adj_e[k]];
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double piv = A[k][k];
        for (int j = t; j < n; j += AMG_BS) {
            prow[j] = (j == k ? 1.0 : A[k][j]) / piv;
            pcol[j] = A[j][k];
        }
        __syncthreads();
        for (int q = t; q < n * n; q += AMG_BS) {
            int i = q / n, j = q % n;
            if (i == k) A[i][j] = prow[j];
            else A[i][j] = (j == k ? 0.0 : A[i][j]) - pcol[i] * prow[j];
        }
        __syncthreads();
    }
    mgreal *O = Ainv + (size_t)s * n * n;
    for (int q = t; q < n * n; q += AMG_BS) {
        int i = q / n, j = q % n;
        O[q] = 0.5 * (A[i][j] + A[j][i]);
    }
}

__device__ inline double amg_Av(const AmgLevel &L, int s, int I, const mgreal *v)
{
    const mgreal *Wa = L.Wa + (size_t)s * 2 * L.ne;
    double a = (double)L.D[(size_t)s * L.n + I] * (double)v[I];
    for (int k = L.adj_off[I]; k < L.adj_off[I + 1]; ++k) a -= (double)Wa[k] * (double)v[L.adj_nbr[k]];
    return a;
}

// Per-element bodies of the V-cycle, shared by the per-level kernels and the
// one-workgroup tail below (same arithmetic, same order).

// b = sum of the finer level's residual w over the members; pre-smoothing
// from zero, x = omega b / D.
__device__ inline void amg_restrict_one(const AmgLevel &L, const mgreal *wf, double omega, int s, int I)
{
    const mgreal *w = wf + (size_t)s * L.nf;
    double acc = 0.0;
    for (int k = L.mem_off[I]; k < L.mem_off[I + 1]; ++k) acc += w[L.mem[k]];
    size_t x = (size_t)s * L.n + I;
    L.b[x] = acc;
    L.x[x] = omega * acc / L.D[x];
}

// w = b - A x
__device__ inline void amg_res_one(const AmgLevel &L, int s, int I)
{
    size_t x = (size_t)s * L.n + I;
    L.w[x] = L.b[x] - amg_Av(L, s, I, L.x + (size_t)s * L.n);
}

// coarsest level: x = A^-1 b (dense), or b / D
__device__ inline void amg_coarse_one(const AmgLevel &C, const mgreal *Ainv, int dense, int s, int i)
{
    const int n = C.n;
    size_t x = (size_t)s * n + i;
    double v;
    if (dense) {
        const mgreal *row = Ainv + ((size_t)s * n + i) * n;
        const mgreal *b = C.b + (size_t)s * n;
        v = 0.0;
        for (int j = 0; j < n; ++j) v += (double)row[j] * (double)b[j];
    } else {
        v = (double)C.b[x] / (double)C.D[x];
    }
    C.x[x] = v;
}

// Up-sweep at a coarse level: y = x + alpha P rc, formed on the fly for the
// node and its neighbours, then post-smoothing out = y + omega (b - A y) / D.
// out (the level's result) is the level's y array.
__device__ inline void amg_up_one(const AmgLevel &L, const AmgLevel &C, const mgreal *rc, double alpha,
                                  double omega, int s, int I)
{
    const mgreal *xl = L.x + (size_t)s * L.n, *Wa = L.Wa + (size_t)s * 2 * L.ne;
    const mgreal *rcs = rc + (size_t)s * C.n;
    auto yv = [&](int J) {
        int K = C.agg[J];
        return (double)xl[J] + (K >= 0 ? alpha * (double)rcs[K] : 0.0);
    };
    size_t x = (size_t)s * L.n + I;
    const double yi = yv(I), Dd = (double)L.D[x];
    double a = Dd * yi;
    for (int k = L.adj_off[I]; k < L.adj_off[I + 1]; ++k) a -= (double)Wa[k] * yv(L.adj_nbr[k]);
    L.y[x] = yi + omega * (L.b[x] - a) / Dd;
}

__global__ __launch_bounds__(AMG_BS) void k_amg_restrict(Dev d, AmgLevel L, const mgreal *wf, double omega)
{
    int I = blockIdx.x * AMG_BS + threadIdx.x, s = blockIdx.y;
    if (I >= L.n || d.conv[s]) return;
    amg_restrict_one(L, wf, omega, s, I);
}

__global__ __launch_bounds__(AMG_BS) void k_amg_res(Dev d, AmgLevel L)
{
    int I = blockIdx.x * AMG_BS + threadIdx.x, s = blockIdx.y;
    if (I >= L.n || d.conv[s]) return;
    amg_res_one(L, s, I);
}

__global__ __launch_bounds__(AMG_BS) void k_amg_coarse_solve(Dev d, AmgLevel C, const mgreal *Ainv, int dense)
{
    int s = blockIdx.x;
    if (d.conv[s]) return;
    for (int i = threadIdx.x; i < C.n; i += AMG_BS) amg_coarse_one(C, Ainv, dense, s, i);
}

__global__ __launch_bounds__(AMG_BS) void k_amg_up(Dev d, AmgLevel L, AmgLevel C, const mgreal *rc,
                                                   double alpha, double omega)
{
    int I = blockIdx.x * AMG_BS + threadIdx.x, s = blockIdx.y;
    if (I >= L.n || d.conv[s]) return;
    amg_up_one(L, C, rc, alpha, omega, s, I);
}

// The small levels lt..nlev of a V-cycle in one workgroup per sample: their
// per-level launches cost far more than their work.  Phases are separated by
// workgroup barriers; each element is computed by the same body as in the
// per-level kernels.
constexpr int AMG_TAIL_LEV = 8;          // levels a tail holds
constexpr int AMG_TAIL_N = 512;          // largest level a tail starts at
struct AmgTail {
    int lt, nlev, dense;
    double omega, alpha;
    const mgreal *Ainv;
    AmgLevel lev[AMG_TAIL_LEV];          // lev[k] = level lt + k
};

template <int BS>
__global__ __launch_bounds__(BS) void k_amg_tail(Dev d, AmgTail t)
{
    const int s = blockIdx.x, T = threadIdx.x;
    if (d.conv[s]) return;                      // the same for the whole workgroup
    const int top = t.nlev - t.lt;              // index of the coarsest level in t.lev
    for (int k = 0; k < top; ++k) {
        const AmgLevel &L = t.lev[k], &C = t.lev[k + 1];
        for (int I = T; I < L.n; I += BS) amg_res_one(L, s, I);
        __syncthreads();
        for (int I = T; I < C.n; I += BS) amg_restrict_one(C, L.w, t.omega, s, I);
        __syncthreads();
    }
    for (int i = T; i < t.lev[top].n; i += BS) amg_coarse_one(t.lev[top], t.Ainv, t.dense, s, i);
    __syncthreads();
    for (int k = top - 1; k >= 0; --k) {
        const AmgLevel &L = t.lev[k], &C = t.lev[k + 1];
        const mgreal *rc = (k + 1 == top) ? C.x : C.y;
        for (int I = T; I < L.n; I += BS) amg_up_one(L, C, rc, t.alpha, t.omega, s, I);
        __syncthreads();
    }
}

static inline dim3 grid_of(int n, int S) { return dim3((n + AMG_BS - 1) / AMG_BS, S); }

void launch_amg_setup(const Dev &d, const Amg &a, hipStream_t st)
{
    for (int l = 1; l <= a.nlev; ++l) {
        const AmgLevel &L = a.lev[l];
        const AmgLevel &F = a.lev[l > 1 ? l - 1 : 1];
        k_amg_asm_nodes<<<grid_of(L.n, d.S), AMG_BS, 0, st>>>(d, a.l0, L, F, l);
        if (L.ne > 0) {
            k_amg_asm_edges<<<grid_of(L.ne, d.S), AMG_BS, 0, st>>>(d, a.l0, L, F, l);
            k_amg_asm_adj<<<grid_of(2 * L.ne, d.S), AMG_BS, 0, st>>>(d, L);
        }
    }
    if (a.dense) k_amg_coarse_inv<<<d.S, AMG_BS, 0, st>>>(a.lev[a.nlev], a.Ainv, d.conv);
}

void launch_amg_vcycle(const Dev &d, const Amg &a, bool init, hipStream_t st)
{
    const int L = a.nlev;
    // first level small enough for the one-workgroup tail (two levels at least)
    int lt = L;
    for (int l = 1; l < L; ++l)
        if (a.lev[l].n <= AMG_TAIL_N && L - l + 1 <= AMG_TAIL_LEV) { lt = l; break; }
    if (init) launch_amg_pre0(d, a.omega, st);
    launch_amg_res0(d, a.l0.w0, st);
    k_amg_restrict<<<grid_of(a.lev[1].n, d.S), AMG_BS, 0, st>>>(d, a.lev[1], a.l0.w0, a.omega);
    for (int l = 1; l < lt; ++l) {
        k_amg_res<<<grid_of(a.lev[l].n, d.S), AMG_BS, 0, st>>>(d, a.lev[l]);
        k_amg_restrict<<<grid_of(a.lev[l + 1].n, d.S), AMG_BS, 0, st>>>(d, a.lev[l + 1], a.lev[l].w, a.omega);
    }
    if (lt < L) {
        AmgTail t;
        t.lt = lt; t.nlev = L; t.dense = a.dense; t.omega = a.omega; t.alpha = a.alpha; t.Ainv = a.Ainv;
        for (int l = lt; l <= L; ++l) t.lev[l - lt] = a.lev[l];
        if (d.S < 64) k_amg_tail<1024><<<d.S, 1024, 0, st>>>(d, t);
        else k_amg_tail<AMG_BS><<<d.S, AMG_BS, 0, st>>>(d, t);
    } else {
        k_amg_coarse_solve<<<d.S, AMG_BS, 0, st>>>(d, a.lev[L], a.Ainv, a.dense);
    }
    // result of level l: x at the coarsest level, y above it
    for (int l = lt - 1; l >= 1; --l)
        k_amg_up<<<grid_of(a.lev[l].n, d.S), AMG_BS, 0, st>>>(d, a.lev[l], a.lev[l + 1],
                                                             l + 1 == L ? a.lev[l + 1].x : a.lev[l + 1].y,
                                                             a.alpha, a.omega);
    launch_amg_post0(d, a.l0.w0, a.lev[1], L == 1 ? a.lev[1].x : a.lev[1].y, a.alpha, a.omega, init, st);
}

}  // namespace em
