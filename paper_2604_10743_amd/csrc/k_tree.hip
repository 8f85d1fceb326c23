// Per-tree kernels: temperatures, diffusivities, control volumes, Monte Carlo
// draws, forcing, tree factorisation, steady-state screen, and the
// backward-Euler stepping loop with nucleation, Robin void rows and void growth.
//
// Lanes map to instances (tree, sample).  With S >= 64 the 64 lanes of a
// wavefront are 64 samples of one tree: identical control flow and coalesced
// [node][sample] accesses.  With S == 1 lanes are trees, ordered largest
// first so that a wavefront holds trees of similar size.
#include "em_internal.h"
#include <algorithm>
#include <cmath>

namespace em {

#define EM_KERNEL __global__ __launch_bounds__(256)

static inline int nblocks(long long n, int bs = 256) { return (int)((n + bs - 1) / bs); }

// ------------------------------------------------------------------------
// Temperature at every stress node (Sec. III-A: per-tree profile from the
// thermal map).  Raster: bilinear with clamping at the raster edge; vertex
// temperatures: linear along the segment; otherwise the ambient value.
// ------------------------------------------------------------------------
__device__ inline void node_position(const Dev &d, int i, double &x, double &y)
{
    int v = d.vert[i];
    if (v >= 0) { x = d.xy[2 * v]; y = d.xy[2 * v + 1]; return; }
    int e = d.seg[i];
    double f = (double)d.kpos[i] / d.N;
    int a = d.ra[e], b = d.rb[e];
    x = d.xy[2 * a] + f * (d.xy[2 * b] - d.xy[2 * a]);
    y = d.xy[2 * a + 1] + f * (d.xy[2 * b + 1] - d.xy[2 * a + 1]);
}

__device__ inline double raster_T(const Dev &d, double x, double y)
{
    double fx = (x - d.tx0) / d.tdx, fy = (y - d.ty0) / d.tdy;
    fx = fmin(fmax(fx, 0.0), (double)(d.tnx - 1));
    fy = fmin(fmax(fy, 0.0), (double)(d.tny - 1));
    int ix = (int)floor(fx), iy = (int)floor(fy);
    ix = max(0, min(ix, d.tnx - 2));
    iy = max(0, min(iy, d.tny - 2));
    double tx = fx - ix, ty = fy - iy;
    int ix1 = d.tnx > 1 ? ix + 1 : ix, iy1 = d.tny > 1 ? iy + 1 : iy;
    const double *M = d.tmap;
    double lo = (1 - tx) * M[iy * d.tnx + ix] + tx * M[iy * d.tnx + ix1];
    double hi = (1 - tx) * M[iy1 * d.tnx + ix] + tx * M[iy1 * d.tnx + ix1];
    return (1 - ty) * lo + ty * hi;
}

EM_KERNEL void k_node_T(Dev d)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.ns) return;
    double T;
    if (d.tmap) {
        double x, y;
        node_position(d, i, x, y);
        T = raster_T(d, x, y);
    } else if (d.node_T) {
        int v = d.vert[i];
        if (v >= 0) T = d.node_T[v];
        else {
            int e = d.seg[i];
            double f = (double)d.kpos[i] / d.N;
            T = d.node_T[d.ra[e]] + f * (d.node_T[d.rb[e]] - d.node_T[d.ra[e]]);
        }
    } else {
        T = d.T_amb;
    }
    d.T[i] = T;
}

// ------------------------------------------------------------------------
// Joule-heating thermal pre-pass (Sec. III-A, eqs. 1-4).  Along a wire segment
// of length L the steady temperature solves k T'' + j^2 rho = k (T - T0)/G^2
// (heat conduction, Joule source, loss through the dielectric to the local
// ambient T0), G^2 = t_cu t_ILD k_cu / k_ILD (eq. 2).  With c = T0 + Tm,
// Tm = j^2 rho G^2 / k_cu, and the end temperatures T1 (res_a end, x = -L/2)
// and T2 (res_b end, x = +L/2):
//   T(x) = c + (Tbar - c) cosh(x/G)/cosh(L/2G) + (T2 - T1)/2 sinh(x/G)/sinh(L/2G).
// The temperature gradient entering the segment at an end is
//   [-(T_here - c) coth(L/G) + (T_there - c) csch(L/G)] / G,
// so heat-flux balance at a vertex without a via (no heat exchanged there
// other than through its segments; a free wire end is adiabatic) reads
//   T_v sum_e w_e coth_e - sum_e w_e csch_e T_u = sum_e w_e c_e tanh(L_e/2G_e),
// w_e = (cross-section)/G_e: a diagonally dominant system on the tree's vertex
// graph, eliminated exactly leaf to root.  Vertices with a via are held at
// the map temperature.
// ------------------------------------------------------------------------

// map temperature at a grid node / at the midpoint of segment e
__device__ inline double map_T_vertex(const Dev &d, int v)
{
    if (d.tmap) return raster_T(d, d.xy[2 * v], d.xy[2 * v + 1]);
    if (d.node_T) return d.node_T[v];
    return d.T_amb;
}
__device__ inline double map_T_mid(const Dev &d, int e)
{
    const int a = d.ra[e], b = d.rb[e];
    if (d.tmap)
        return raster_T(d, 0.5 * (d.xy[2 * a] + d.xy[2 * b]), 0.5 * (d.xy[2 * a + 1] + d.xy[2 * b + 1]));
    if (d.node_T) return 0.5 * (d.node_T[a] + d.node_T[b]);
    return d.T_amb;
}

struct SegHeat { double G, c, w, cth, csh, th; };   // G, c, w; coth, csch of L/G; tanh(L/2G)

__device__ inline SegHeat seg_heat(const Dev &d, int e, const double *j)
{
    SegHeat q;
    q.G = sqrt(d.h[e] * d.t_ild * d.k_cu / d.k_ild);
    q.c = map_T_mid(d, e) + j[e] * j[e] * d.rho * q.G * q.G / d.k_cu;
    q.w = d.w[e] * d.h[e] / q.G;
    const double y = d.len[e] / q.G;
    const double em2 = expm1(-2.0 * y);                 // e^{-2y} - 1 < 0
    q.cth = (2.0 + em2) / -em2;                          // (1 + e^{-2y}) / (1 - e^{-2y})
    q.csh = 2.0 * exp(-y) / -em2;                        // 2 e^{-y} / (1 - e^{-2y})
    q.th = -expm1(-y) / (2.0 + expm1(-y));               // (1 - e^{-y}) / (1 + e^{-y})
    return q;
}

__device__ inline bool vertex_has_via(const Dev &d, int v)
{
    for (int k = d.ninc_off[v]; k < d.ninc_off[v + 1]; ++k)
        if (!d.is_wire[d.ninc_res[k]]) return true;
    return false;
}

// One thread per tree: vertex temperatures into d.T (vertex nodes only).
// A vertex node i other than the root reached its tree walk through segment
// seg[i], whose N - 1 interior nodes precede it, so its neighbour vertex on
// that segment is parent[i - N + 1].
EM_KERNEL void k_joule_vertices(Dev d, const double *j, double *D, double *r)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d.n_trees) return;
    const int o0 = d.tree_off[t], o1 = d.tree_off[t + 1], N = d.N;
    for (int i = o0; i < o1; ++i)
        if (d.vert[i] >= 0) { D[i] = 0.0; r[i] = 0.0; }
    for (int i = o0 + 1; i < o1; ++i) {
        if (d.vert[i] < 0) continue;
        const int p = d.parent[i - N + 1];
        const SegHeat q = seg_heat(d, d.seg[i], j);
        D[i] += q.w * q.cth; D[p] += q.w * q.cth;
        r[i] += q.w * q.c * q.th; r[p] += q.w * q.c * q.th;
    }
    // leaf to root (reverse walk order: children before parents)
    for (int i = o1 - 1; i > o0; --i) {
        const int v = d.vert[i];
        if (v < 0) continue;
        const int p = d.parent[i - N + 1];
        const SegHeat q = seg_heat(d, d.seg[i], j);
        const double beta = q.w * q.csh;
        if (vertex_has_via(d, v)) {
            d.T[i] = map_T_vertex(d, v);
            r[p] += beta * d.T[i];
        } else {
            r[p] += beta * r[i] / D[i];
            D[p] -= beta * beta / D[i];
        }
    }
    const int v0 = d.vert[o0];
    d.T[o0] = vertex_has_via(d, v0) ? map_T_vertex(d, v0) : r[o0] / D[o0];
    // root to leaves
    for (int i = o0 + 1; i < o1; ++i) {
        const int v = d.vert[i];
        if (v < 0 || vertex_has_via(d, v)) continue;
        const int p = d.parent[i - N + 1];
        const SegHeat q = seg_heat(d, d.seg[i], j);
        d.T[i] = (r[i] + q.w * q.csh * d.T[p]) / D[i];
    }
}

// One thread per interior node: the segment's steady profile between its
// end temperatures.  The interior node at walk position q (1..N-1) of a
// segment lies q nodes after the segment's first vertex node and N - q
// before its second.
EM_KERNEL void k_joule_nodes(Dev d, const double *j)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.ns || d.vert[i] >= 0) return;
    const int e = d.seg[i], N = d.N, kp = d.kpos[i];
    const int q = d.dir[i] > 0 ? kp : N - kp;
    const int sw = i + N - q;
    const int su = d.parent[sw - N + 1];
    const double T1 = d.dir[i] > 0 ? d.T[su] : d.T[sw];    // res_a end
    const double T2 = d.dir[i] > 0 ? d.T[sw] : d.T[su];    // res_b end
    const SegHeat h = seg_heat(d, e, j);
    const double hl = 0.5 * d.len[e] / h.G;                // L / 2G
    const double x = ((double)kp / N - 0.5) * d.len[e] / h.G;
    const double ax = fabs(x);
    // cosh(x)/cosh(hl) and sinh(x)/sinh(hl) without overflow
    const double ed = exp(ax - hl);
    const double ch = ed * (1.0 + exp(-2.0 * ax)) / (1.0 + exp(-2.0 * hl));
    double sh = ed * expm1(-2.0 * ax) / expm1(-2.0 * hl);
    if (x < 0) sh = -sh;
    d.T[i] = h.c + (0.5 * (T1 + T2) - h.c) * ch + 0.5 * (T2 - T1) * sh;
}

// ------------------------------------------------------------------------
// Per-edge statics for the edge (parent(i), i): diffusivity at the edge
// midpoint temperature, kappa = D0 exp(-Ea/kT) B Omega/(kT) (eqs. 10-11),
// conductance g0 = a kappa/dx, Robin weight a kappa/delta (eq. 20), and the
// thermomigration drive M = (Q/(Omega T)) dT/dx along res_a -> res_b (eq. 13).
// Monte Carlo multipliers scale kappa later, per sample.
// ------------------------------------------------------------------------
EM_KERNEL void k_edge_static(Dev d)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.ns) return;
    int p = d.parent[i];
    if (p < 0) { d.g0[i] = 0; d.rob0[i] = 0; d.gdx0[i] = 0; d.mdrv[i] = 0; return; }
    int e = d.seg[i];
    double dx = d.len[e] / d.N;
    double a = d.w[e] * d.h[e];
    double Te = 0.5 * (d.T[i] + d.T[p]);
    double kT = K_B * Te;
    double kap = d.D0 * exp(-d.Ea_eV * E_CHG / kT) * d.B * d.Omega / kT;
    d.g0[i] = a * kap / dx;
    d.rob0[i] = a * kap / d.delta;
    d.gdx0[i] = a * kap;
    d.mdrv[i] = d.dir[i] * (d.Q_eV * E_CHG / (d.Omega * Te)) * (d.T[i] - d.T[p]) / dx;
}

// Control volume of a node: half of every incident interval's volume.
EM_KERNEL void k_node_V(Dev d, int fp32)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.ns) return;
    double V = 0;
    if (d.parent[i] >= 0) {
        int e = d.seg[i];
        V += 0.5 * d.w[e] * d.h[e] * (d.len[e] / d.N);
    }
    for (int k = d.child_off[i]; k < d.child_off[i + 1]; ++k) {
        int e = d.seg[d.child[k]];
        V += 0.5 * d.w[e] * d.h[e] * (d.len[e] / d.N);
    }
    d.V[i] = V;
    if (fp32) ((float *)d.Vr)[i] = (float)V; else ((double *)d.Vr)[i] = V;
}

// Total control volume of each tree (fixed summation order).
// One wavefront per tree: strided partial sums, then a fixed butterfly.
EM_KERNEL void k_tree_V(Dev d)
{
    const int lane = threadIdx.x & 63;
    const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t >= d.n_trees) return;
    double s = 0.0;
    for (int i = d.tree_off[t] + lane; i < d.tree_off[t + 1]; i += 64) s += d.V[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) d.tree_V[t] = s;
}

// ------------------------------------------------------------------------
// Monte Carlo multipliers (Sec. IV-F): Philox-4x32-10 (Salmon et al., SC'11)
// counter (segment, sample, param, 0), key (seed lo, seed hi); Box-Muller on
// u1 = (x0 + 1) 2^-32, u2 = x1 2^-32; unit-mean lognormal with CoV `cov`.
// ------------------------------------------------------------------------
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        uint32_t hi0 = __umulhi(m0, c[0]), lo0 = m0 * c[0];
        uint32_t hi1 = __umulhi(m1, c[2]), lo1 = m1 * c[2];
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
}

// standard normal deviate of counter (index, sample, param, 0)
__device__ inline double normal_z(uint64_t seed, int sample, int index, int param)
{
    uint32_t c[4] = {(uint32_t)index, (uint32_t)sample, (uint32_t)param, 0u};
    philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
    double u1 = ((double)c[0] + 1.0) * (1.0 / 4294967296.0);
    double u2 = (double)c[1] * (1.0 / 4294967296.0);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

__device__ inline double lognormal_xi(uint64_t seed, int sample, int segment, int param, double cov)
{
    if (cov == 0.0) return 1.0;
    const double z = normal_z(seed, sample, segment, param);
    double s2 = log(1.0 + cov * cov);
    return exp(-0.5 * s2 + sqrt(s2) * z);
}

// The activation-energy offset dEa ~ N(0, sd_ea) of a wire segment (param 4)
// scales its diffusivity by exp(-dEa / (k_B T)), T the map temperature at the
// segment's midpoint; the sample's die-temperature offset dT ~ N(0, sd_T)
// (param 5, one per sample) by the Arrhenius ratio kappa(T + dT) / kappa(T);
// the sample's map amplitude a (param 6, unit-mean lognormal) by
// kappa(T_a) / kappa(T), T_a = T_amb + a (T - T_amb).  All join the kappa
// multiplier; a itself scales the thermomigration drive (tm_scale).
EM_KERNEL void k_draws(Dev d, uint64_t seed, double cov_k, double cov_s, double cov_r, double sd_ea, double sd_T,
                       double cov_map, int use_mc)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.n_res * d.S) return;
    int s = (int)(g % d.S), e = (int)(g / d.S);
    const int sm = d.sid ? d.sid[s] : s;       // Monte Carlo sample index of the counter
    double xk = use_mc ? lognormal_xi(seed, sm, e, 0, cov_k) : 1.0;
    if (sd_ea > 0.0 && d.is_wire[e])
        xk *= exp(-sd_ea * normal_z(seed, sm, e, 4) / ((K_B / E_CHG) * map_T_mid(d, e)));
    if (sd_T > 0.0 && d.is_wire[e]) {
        const double T = map_T_mid(d, e), dT = sd_T * normal_z(seed, sm, 0, 5);
        xk *= exp(d.Ea_eV / (K_B / E_CHG) * (1.0 / T - 1.0 / (T + dT))) * T / (T + dT);
    }
    if (cov_map > 0.0) {
        const double a = lognormal_xi(seed, sm, 0, 6, cov_map);
        if (e == 0) d.map_a[s] = a;
        if (d.is_wire[e]) {
            const double T = map_T_mid(d, e), Ta = d.T_amb + a * (T - d.T_amb);
            xk *= exp(d.Ea_eV / (K_B / E_CHG) * (1.0 / T - 1.0 / Ta)) * T / Ta;
        }
    }
    d.xi_k[g] = xk;
    d.xi_s[g] = use_mc ? lognormal_xi(seed, sm, e, 1, cov_s) : 1.0;
    if (d.xi_r) d.xi_r[g] = d.is_wire[e] ? lognormal_xi(seed, sm, e, 2, cov_r) : 1.0;
}

// Per-sample sinks under current-loading variation: [S][n_nodes].
EM_KERNEL void k_draws_load(Dev d, uint64_t seed, double cov_l)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.n_nodes * d.S) return;
    int s = (int)(g / d.n_nodes), v = (int)(g % d.n_nodes);
    d.sink_s[g] = d.sink[v] * lognormal_xi(seed, d.sid ? d.sid[s] : s, v, 3, cov_l);
}

// Resistivity multiplier of wire segment e in sample s (1 without that variation).
__device__ inline double xi_rho(const Dev &d, int e, int s)
{
    return d.xi_r ? d.xi_r[(size_t)e * d.S + s] : 1.0;
}

// Critical stress of a node: sigma_crit x the smallest multiplier over the
// segments meeting at it.
__device__ inline double node_scrit(const Dev &d, int i, int s)
{
    double m = INFINITY;
    if (d.parent[i] >= 0) m = d.xi_s[(size_t)d.seg[i] * d.S + s];
    for (int k = d.child_off[i]; k < d.child_off[i + 1]; ++k)
        m = fmin(m, d.xi_s[(size_t)d.seg[d.child[k]] * d.S + s]);
    return d.scrit * m;
}

template <typename R>
EM_KERNEL void k_node_sc(Dev d)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.ns * d.S) return;
    int s = (int)(g % d.S), i = (int)(g / d.S);
    ((R *)d.sc)[g] = (R)node_scrit(d, i, s);
}

// The same with one node per block row (node uniform across the block, so
// its topology is read once) and samples along x; for many samples.
template <typename R>
EM_KERNEL void k_node_sc_rows(Dev d)
{
    const int i = blockIdx.y + blockIdx.z * 65535;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.ns || s >= d.S) return;
    ((R *)d.sc)[(size_t)i * d.S + s] = (R)node_scrit(d, i, s);
}

// The thermomigration drive of the edge (parent(i), i) in sample s relative
// to the nominal map's: with the map's rise scaled by the sample's amplitude
// a, (Q / (Omega T)) dT/dx becomes a T_e / (T_amb + a (T_e - T_amb)) times
// itself, T_e the edge's midpoint temperature.
__device__ inline double tm_scale(const Dev &d, int i, int s)
{
    if (!d.map_a) return 1.0;
    const double a = d.map_a[s], Te = 0.5 * (d.T[i] + d.T[d.parent[i]]);
    return a * Te / (d.T_amb + a * (Te - d.T_amb));
}

// ------------------------------------------------------------------------
// Forcing f of the descriptor system (eq. 18): the edge (p, i) carries
// phi = dir * g dx (S + M) from p into i, with S = eZ rho j/Omega along
// res_a -> res_b; f_i = phi_i - sum over children c of phi_c.  Stored as dt*f.
// ------------------------------------------------------------------------
__device__ inline double edge_phi(const Dev &d, int i, int s)
{
    int e = d.seg[i];
    double j = d.S == 1 ? d.jseg[e] : d.jT[(size_t)e * d.S + s];
    double Sd = E_CHG * d.Z * d.rho * xi_rho(d, e, s) * j / d.Omega;
    return d.dir[i] * d.xi_k[(size_t)e * d.S + s] * d.gdx0[i] * (Sd + tm_scale(d, i, s) * d.mdrv[i]);
}

__device__ inline double node_dtf(const Dev &d, int i, int s)
{
    double f = 0.0;
    if (d.parent[i] >= 0) f += edge_phi(d, i, s);
    for (int k = d.child_off[i]; k < d.child_off[i + 1]; ++k) f -= edge_phi(d, d.child[k], s);
    return d.dt * f;
}

// jT = jseg transposed ([S][res] -> [res][S]) through 32 x 32 LDS tiles, so
// that the forcing update reads the current density of a segment for
// consecutive samples from consecutive addresses
__global__ __launch_bounds__(256) void k_transpose_j(Dev d, const double *jseg)
{
    __shared__ double tile[32][33];
    const int r0 = blockIdx.x * 32, s0 = blockIdx.y * 32, tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int s = s0 + k, r = r0 + tx;
        if (s < d.S && r < d.n_res) tile[k][tx] = jseg[(size_t)s * d.n_res + r];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int r = r0 + k, s = s0 + tx;
        if (r < d.n_res && s < d.S) d.jT[(size_t)r * d.S + s] = tile[tx][k];
    }
}

static void transpose_j(const Dev &d, hipStream_t st)
{
    if (d.S == 1) return;
    k_transpose_j<<<dim3((d.n_res + 31) / 32, (d.S + 31) / 32), 256, 0, st>>>(d, d.jseg);
}

template <typename R>
EM_KERNEL void k_update_f(Dev d)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.ns * d.S) return;
    int s = (int)(g % d.S), i = (int)(g / d.S);
    ((R *)d.dtf)[g] = (R)node_dtf(d, i, s);
}

// dt*f of the nodes of the listed instances only (one block per instance)
template <typename R>
EM_KERNEL void k_update_f_list(Dev d, const int *list)
{
    const int inst = list[blockIdx.x];
    const int t = inst / d.S, s = inst - t * d.S;
    for (int i = d.tree_off[t] + threadIdx.x; i < d.tree_off[t + 1]; i += blockDim.x)
        ((R *)d.dtf)[(size_t)i * d.S + s] = (R)node_dtf(d, i, s);
}

// ------------------------------------------------------------------------
// Tree factorisation of M = C - dt A (SPD on the tree): leaf-to-root
// elimination in reverse pre-order with no fill,
//   d_i = V_i + dt g_i + sum_c dt g_c (1 - l_c) [+ dt * Robin weight at a void],
//   l_i = dt g_i / d_i,
// stored as dinv = 1/d and l.
// ------------------------------------------------------------------------
__device__ inline bool in_list(int i, const int *vn, int nv)
{
    bool r = false;
#pragma unroll
    for (int k = 0; k < MAXV; ++k) r |= (k < nv) && (vn[k] == i);
    return r;
}

__device__ inline double robin_weight(const Dev &d, int v, int s)
{
    double r = 0.0;
    if (d.parent[v] >= 0) r += d.xi_k[(size_t)d.seg[v] * d.S + s] * d.rob0[v];
    for (int k = d.child_off[v]; k < d.child_off[v + 1]; ++k) {
        int c = d.child[k];
        r += d.xi_k[(size_t)d.seg[c] * d.S + s] * d.rob0[c];
    }
    return r;
}

template <typename R>
__device__ void factor_instance(const Dev &d, int t, int s, const int *vn, const double *vrob, int nv)
{
    const int S = d.S;
    R *dinv = (R *)d.dinv, *lf = (R *)d.lfac;
    int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
    const double dt = d.dt;
    for (int i = i1 - 1; i >= i0; --i) {
        double gi = 0.0;
        if (d.parent[i] >= 0) gi = dt * d.xi_k[(size_t)d.seg[i] * S + s] * d.g0[i];
        double dd = d.V[i] + gi;
        for (int k = d.child_off[i]; k < d.child_off[i + 1]; ++k) {
            int c = d.child[k];
            double gc = dt * d.xi_k[(size_t)d.seg[c] * S + s] * d.g0[c];
            dd += gc * (1.0 - (double)lf[(size_t)c * S + s]);
        }
        for (int k = 0; k < nv; ++k)
            if (vn[k] == i) dd += dt * vrob[k];
        dinv[(size_t)i * S + s] = (R)(1.0 / dd);
        lf[(size_t)i * S + s] = (R)(gi / dd);
    }
}

__device__ inline int inst_of_slot(const Dev &d, int slot, int &t, int &s)
{
    s = slot % d.S;
    t = d.tree_perm[slot / d.S];
    return t * d.S + s;
}

// Stress state: R per (node, sample), plus (FP32 form) a float low part, so
// that the state carries the increments that fall below half an ulp of the
// stored value (near saturation the per-step increments shrink to a few Pa,
// which float alone would drop: the approach to sigma_crit would stall).
template <typename R>
__device__ inline double ld_sig(const Dev &d, const R *hi, size_t x)
{
    return (double)hi[x] + (d.sig_lo ? (double)d.sig_lo[x] : 0.0);
}
template <typename R>
__device__ inline void st_sig(const Dev &d, R *hi, size_t x, double v)
{
    const R h = (R)v;
    hi[x] = h;
    if (d.sig_lo) d.sig_lo[x] = (float)(v - (double)h);
}

template <typename R>
EM_KERNEL void k_factor(Dev d)
{
    int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= d.n_trees * d.S) return;
    int t, s;
    int inst = inst_of_slot(d, slot, t, s);
    if (d.tree_chain[t]) return;         // the chain kernel factors in place
    int vn[MAXV];
    double vr[MAXV];
    int nv = d.nv[inst];
    for (int k = 0; k < MAXV; ++k) {
        vn[k] = k < nv ? d.vnode[inst * MAXV + k] : -1;
        vr[k] = k < nv ? d.vrob[inst * MAXV + k] : 0.0;
    }
    factor_instance<R>(d, t, s, vn, vr, nv);
}

// ------------------------------------------------------------------------
// Steady-state immortality screen (Sec. III-B).  Zero flux on every edge:
// psi_i = psi_p + dir dx (S + M); the constant follows from conservation
// (sum V sigma = sum V sigma_T), so sigma_ss = sigma_T + psi - <psi>_V.
// A node is mortal iff its finite sigma_ss exceeds its critical stress;
// segments through a mortal node and its tree are flagged.
// ------------------------------------------------------------------------
// The per-(tree, sample) passes below run one instance per 64-lane
// wavefront, lanes over the tree's nodes in chunks of 64.
__device__ inline double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wmax(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline double wmin(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// psi_i = psi_parent + dir dx (S + M) from the root (pre-order: a parent
// precedes its children).  Within a chunk the parent links are followed by
// pointer jumping; a parent in an earlier chunk is the previous chunk's last
// node (carried) or is read back.  Then sigma_ss = sigma_T + psi - <psi>_V.
__device__ void steady_stress_wave(const Dev &d, int t, int s, int lane)
{
    const int S = d.S;
    const int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
    double *psi = d.psi;
    double num = 0.0, den = 0.0, last = 0.0;
    for (int c = i0; c < i1; c += 64) {
        const int i = c + lane;
        const bool ok = i < i1;
        double v = 0.0;
        int a = -1;
        if (ok && i > i0) {
            const int e = d.seg[i];
            const double dx = d.len[e] / d.N;
            const double Sd = E_CHG * d.Z * d.rho * xi_rho(d, e, s) * d.jseg[(size_t)s * d.n_res + e] / d.Omega;
            v = d.dir[i] * dx * (Sd + tm_scale(d, i, s) * d.mdrv[i]);
            a = d.parent[i];
        }
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const bool in = a >= c;
            const int src = in ? a - c : lane;
            const double vo = __shfl(v, src, 64);
            const int ao = __shfl(a, src, 64);
            if (in) { v += vo; a = ao; }
        }
        if (a >= 0) v += (a == c - 1) ? last : psi[(size_t)a * S + s];
        if (ok) {
            psi[(size_t)i * S + s] = v;
            num += d.V[i] * v;
            den += d.V[i];
        }
        last = __shfl(v, 63, 64);
        __threadfence_block();
    }
    const double mean = wsum(num) / wsum(den);
    for (int i = i0 + lane; i < i1; i += 64) psi[(size_t)i * S + s] = d.sigT + psi[(size_t)i * S + s] - mean;
}

// Steady-state immortality screen of one instance per wavefront.
EM_KERNEL void k_screen(Dev d, int apply)
{
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slot >= d.n_trees * d.S) return;
    int t, s;
    const int inst = inst_of_slot(d, slot, t, s);
    const int S = d.S;
    steady_stress_wave(d, t, s, lane);
    const int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
    uint8_t *sm = d.seg_mortal + (size_t)s * d.n_res;
    for (int k = d.tseg_off[t] + lane; k < d.tseg_off[t + 1]; k += 64) sm[d.tseg[k]] = 0;
    __threadfence_block();
    bool mortal = false;
    for (int i = i0 + lane; i < i1; i += 64) {
        double v = d.psi[(size_t)i * S + s];
        if (isfinite(v) && v > node_scrit(d, i, s)) {
            mortal = true;
            if (d.parent[i] >= 0) sm[d.seg[i]] = 1;
            for (int k = d.child_off[i]; k < d.child_off[i + 1]; ++k) sm[d.seg[d.child[k]]] = 1;
        }
    }
    const bool any = __any(mortal);
    if (lane == 0) {
        d.tree_mortal[inst] = any ? 1 : 0;
        if (apply) d.inst_active[inst] = any ? 1 : 0;
    }
}

// The same screen when every sample carries the same current densities
// (nominal resistances: the t = 0 screen of a Monte Carlo run): the steady
// stress does not depend on the diffusivity, so it is computed once per tree
// (sample 0, a wavefront per tree) and then compared with each sample's
// critical stress, one thread per (node, sample).
EM_KERNEL void k_screen_ss0(Dev d)
{
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slot >= d.n_trees) return;
    steady_stress_wave(d, d.tree_perm[slot], 0, lane);
}

// Every sample's verdict from sample 0's steady stress.  The steady stress
// itself stays in column 0 (its readers take that column).
__device__ inline void screen_verdict(const Dev &d, int i, int s)
{
    const int S = d.S;
    const double v = d.psi[(size_t)i * S];
    if (isfinite(v) && v > node_scrit(d, i, s)) {
        d.tree_mortal[(size_t)d.ntree[i] * S + s] = 1;
        uint8_t *sm = d.seg_mortal + (size_t)s * d.n_res;
        if (d.parent[i] >= 0) sm[d.seg[i]] = 1;
        for (int k = d.child_off[i]; k < d.child_off[i + 1]; ++k) sm[d.seg[d.child[k]]] = 1;
    }
}
// one node per block row (its topology read once per block), samples along x
EM_KERNEL void k_screen_bcast_rows(Dev d)
{
    const int i = blockIdx.y + blockIdx.z * 65535;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d.ns && s < d.S) screen_verdict(d, i, s);
}
EM_KERNEL void k_screen_bcast_flat(Dev d)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < (long long)d.ns * d.S) screen_verdict(d, (int)(g / d.S), (int)(g % d.S));
}

EM_KERNEL void k_screen_activate(Dev d)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < (long long)d.n_trees * d.S) d.inst_active[g] = d.tree_mortal[g];
}

// ------------------------------------------------------------------------
// Late-failure resistance (eq. 17) with V_v - V_crit = (l - W) W H.
// ------------------------------------------------------------------------
__device__ inline double late_dR(const Dev &d, double l, double W, double H, double rho_cu)
{
    double ex = l - W;
    if (ex <= 0) return 0.0;
    return ex * (d.rho_ta / (d.h_ta * (2 * H + W)) - rho_cu / (W * H));
}

// Host segment of a void at node v: its own segment for an interior node; at
// a vertex, the incident segment with the largest wind away from it (signed
// j with the vertex at res_b, -j at res_a), ties to the lowest index.
__device__ inline int host_segment(const Dev &d, int v, int s)
{
    int x = d.vert[v];
    if (x < 0) return d.seg[v];
    int best = -1;
    double bd = 0.0;
    for (int k = d.vinc_off[x]; k < d.vinc_off[x + 1]; ++k) {
        int e = d.vinc[k];
        double j = d.jseg[(size_t)s * d.n_res + e];
        double drv = (d.rb[e] == x) ? j : -j;
        if (best < 0 || drv > bd) { best = e; bd = drv; }
    }
    return best;
}

template <typename R>
__device__ void add_void(const Dev &d, int inst, int t, int s, int v, int step, int *vn, double *vvol,
                         double *vlen, double *vrob, int *vseg, int *vphase, int *vearly, int &nv)
{
    int k = nv;
    vn[k] = v;
    vvol[k] = 0.0;
    vlen[k] = 0.0;
    vrob[k] = robin_weight(d, v, s);
    vseg[k] = host_segment(d, v, s);
    vphase[k] = 0;
    vearly[k] = d.vert[v] >= 0 ? d.via_up[d.vert[v]] : 0;
    d.vstep[inst * MAXV + k] = step;
    nv = k + 1;
    unsigned int q = atomicAdd(d.ev_count, 1u);
    if ((int)q < d.ev_cap) {
        int *E = d.events + (size_t)q * EV_WORDS;
        E[0] = s; E[1] = t; E[2] = step; E[3] = v; E[4] = vseg[k];
    }
    factor_instance<R>(d, t, s, vn, vrob, nv);
}

// The factor of one (tree, sample) after a Robin row was stamped at node v:
// only v and its ancestors change (a node's pivot depends on its own row and
// its children's multipliers), walked from v to the root.
template <typename R>
__device__ void refactor_path(const Dev &d, int v, int s, const int *vn, const double *vrob, int nv)
{
    const int S = d.S;
    R *dinv = (R *)d.dinv, *lf = (R *)d.lfac;
    const double dt = d.dt;
    for (int i = v; i >= 0; i = d.parent[i]) {
        double gi = 0.0;
        if (d.parent[i] >= 0) gi = dt * d.xi_k[(size_t)d.seg[i] * S + s] * d.g0[i];
        double dd = d.V[i] + gi;
        for (int k = d.child_off[i]; k < d.child_off[i + 1]; ++k) {
            int c = d.child[k];
            double gc = dt * d.xi_k[(size_t)d.seg[c] * S + s] * d.g0[c];
            dd += gc * (1.0 - (double)lf[(size_t)c * S + s]);
        }
        for (int k = 0; k < nv; ++k)
            if (vn[k] == i) dd += dt * vrob[k];
        dinv[(size_t)i * S + s] = (R)(1.0 / dd);
        lf[(size_t)i * S + s] = (R)(gi / dd);
    }
}

template <typename R>
__device__ void add_void_path(const Dev &d, int inst, int t, int s, int v, int step, int *vn, double *vvol,
                              double *vlen, double *vrob, int *vseg, int *vphase, int *vearly, int &nv)
{
    int k = nv;
    vn[k] = v;
    vvol[k] = 0.0;
    vlen[k] = 0.0;
    vrob[k] = robin_weight(d, v, s);
    vseg[k] = host_segment(d, v, s);
    vphase[k] = 0;
    vearly[k] = d.vert[v] >= 0 ? d.via_up[d.vert[v]] : 0;
    d.vstep[inst * MAXV + k] = step;
    nv = k + 1;
    unsigned int q = atomicAdd(d.ev_count, 1u);
    if ((int)q < d.ev_cap) {
        int *E = d.events + (size_t)q * EV_WORDS;
        E[0] = s; E[1] = t; E[2] = step; E[3] = v; E[4] = vseg[k];
    }
    refactor_path<R>(d, v, s, vn, vrob, nv);
}

// ------------------------------------------------------------------------
// Backward-Euler stepping, one (tree, sample) per lane, n_steps steps per
// launch with the current densities fixed.  Each step solves the BE equation
// (C - dt A) sigma^{n+1} = C sigma^n + dt f in increment form,
// (C - dt A) delta = dt (A sigma^n + f): the residual is assembled in FP64
// from exact flux differences, eliminated leaf-to-root into an FP64
// workspace, back-substituted root-to-leaf, and added to the stored stress.
// The rounding of the solve then scales with the residual, which vanishes at
// steady state (for FP32 storage this acts as iterative refinement inside the
// time stepping).  After each step: void growth from atom conservation
// (eq. 15), then the nucleation check (peak stress at or above the node's
// critical stress; ties within 1e-12 relative go to the lowest node), which
// stamps the Robin row (eq. 20) and refactors the tree.
//
// Conservation projection: the scheme keeps sum_i V_i sigma_i + B * (void
// volumes) equal to its value at the start of the launch exactly; the content
// is accumulated in FP64 during the back substitution and the uniform
// correction restoring it is folded into the next step (and into the stored
// stress at the end of the launch).  It changes the solution only at the
// rounding level.
// ------------------------------------------------------------------------
template <typename R>
EM_KERNEL void k_step(Dev d, int n_steps, int step0)
{
    int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= d.n_trees * d.S) return;
    int t, s;
    int inst = inst_of_slot(d, slot, t, s);
    if (!d.sample_active[s] || !d.inst_active[inst] || d.tree_chain[t]) return;
    const int S = d.S;
    R *sig = (R *)d.sigma;
    const R *dtf = (const R *)d.dtf, *dinv = (const R *)d.dinv, *lf = (const R *)d.lfac;
    const R *sc = (const R *)d.sc;
    const int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
    atomicAdd(&d.node_steps[blockIdx.x & (NS_SLOTS - 1)], (unsigned long long)(i1 - i0) * (unsigned long long)n_steps);

    int nv = d.nv[inst];
    int vn[MAXV], vseg[MAXV], vphase[MAXV], vearly[MAXV];
    double vvol[MAXV], vlen[MAXV], vrob[MAXV];
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
        int q = inst * MAXV + k;
        bool u = k < nv;
        vn[k] = u ? d.vnode[q] : -1;
        vseg[k] = u ? d.vseg[q] : -1;
        vphase[k] = u ? d.vphase[q] : 0;
        vearly[k] = u ? d.vearly[q] : 0;
        vvol[k] = u ? d.vvol[q] : 0.0;
        vlen[k] = u ? d.vlen[q] : 0.0;
        vrob[k] = u ? d.vrob[q] : 0.0;
    }
    int suppressed = 0;
    const double Vsum = d.tree_V[t];
    // conserved content at launch start: sum V sigma + B * void volume
    double Q0 = 0.0;
    for (int i = i0; i < i1; ++i) Q0 += d.V[i] * ld_sig(d, sig, (size_t)i * S + s);
    for (int k = 0; k < nv; ++k) Q0 += d.B * vvol[k];
    double corr = 0.0;

    double *W = d.wsp;              // FP64 workspace [node][S]
    for (int st = 0; st < n_steps; ++st) {
        // Increment form: (C - dt A) delta = dt (A sigma + f), residual in FP64
        // from exact flux differences.  Pass 1 (leaf-to-root) assembles the
        // residual and eliminates it into the parents: b_i = r_i + sum_c l_c b_c.
        double b_next = 0.0, s_next = 0.0;
        for (int i = i1 - 1; i >= i0; --i) {
            const size_t x = (size_t)i * S + s;
            const double si = ld_sig(d, sig, x) + corr;
            const bool isv = in_list(i, vn, nv);
            double r = isv ? 0.0 : (double)dtf[x];
            const int p = d.parent[i];
            if (p >= 0) r += d.dt * d.xi_k[(size_t)d.seg[i] * S + s] * d.g0[i] * ((ld_sig(d, sig, (size_t)p * S + s) + corr) - si);
            for (int k = d.child_off[i]; k < d.child_off[i + 1]; ++k) {
                const int c = d.child[k];
                const size_t y = (size_t)c * S + s;
                const double gc = d.dt * d.xi_k[(size_t)d.seg[c] * S + s] * d.g0[c];
                const double sc_ = (c == i + 1) ? s_next : ld_sig(d, sig, y) + corr;
                const double bc = (c == i + 1) ? b_next : W[y];
                r += gc * (sc_ - si) + (double)lf[y] * bc;
            }
            if (isv) {
                for (int k = 0; k < nv; ++k) if (vn[k] == i) r -= d.dt * vrob[k] * si;
            }
            W[x] = r;
            b_next = r;
            s_next = si;
        }
        // Pass 2 (root-to-leaf): delta_i = b_i / d_i + l_i delta_parent;
        // sigma += delta; track the nucleation candidate peak.
        double mx = 0.0;
        bool any = false;
        double Q = 0.0;
        double dprev = 0.0;
        for (int i = i0; i < i1; ++i) {
            const size_t x = (size_t)i * S + s;
            double dl = W[x] * (double)dinv[x];
            if (i > i0) {
                const int p = d.parent[i];
                dl += (double)lf[x] * (p == i - 1 ? dprev : W[(size_t)p * S + s]);
            }
            W[x] = dl;
            dprev = dl;
            const double v = ld_sig(d, sig, x) + corr + dl;
            st_sig(d, sig, x, v);
            Q += d.V[i] * v;
            if (v >= (double)sc[x] && !in_list(i, vn, nv)) {
                mx = any ? (v > mx ? v : mx) : v;
                any = true;
            }
        }
        // void growth: dV = (dt/B) (Robin weight * sigma_v + f_v)
        for (int k = 0; k < nv; ++k) {
            size_t x = (size_t)vn[k] * S + s;
            vvol[k] += (d.dt * vrob[k] * ld_sig(d, sig, x) + (double)dtf[x]) / d.B;
            int e = vseg[k];
            double Wd = d.w[e], H = d.h[e];
            double l = fmin(vvol[k] / (Wd * H), d.len[e]);
            vlen[k] = l;
            if (vphase[k] == 0 && l >= Wd) {
                vphase[k] = 1;
                if (vearly[k]) {
                    d.open[(size_t)s * d.n_res + e] = 1;
                    *d.open_dirty = 1u;
                }
            }
        }
        {
            double vtot = 0.0;
            for (int k = 0; k < nv; ++k) vtot += vvol[k];
            corr = (Q0 - d.B * vtot - Q) / Vsum;
        }
        // nucleation
        if (any) {
            if (nv < d.max_voids) {
                const double thr = mx - 1e-12 * (mx < 0 ? -mx : mx);
                int v = -1;
                for (int i = i0; i < i1 && v < 0; ++i) {
                    size_t x = (size_t)i * S + s;
                    const double val = ld_sig(d, sig, x);
                    if (val >= (double)sc[x] && val >= thr && !in_list(i, vn, nv)) v = i;
                }
                add_void<R>(d, inst, t, s, v, step0 + st, vn, vvol, vlen, vrob, vseg, vphase, vearly, nv);
            } else {
                ++suppressed;
            }
        }
    }
    if (corr != 0.0)
        for (int i = i0; i < i1; ++i) {
            const size_t x = (size_t)i * S + s;
            st_sig(d, sig, x, ld_sig(d, sig, x) + corr);
        }
    d.nv[inst] = nv;
    for (int k = 0; k < nv; ++k) {
        int q = inst * MAXV + k;
        d.vnode[q] = vn[k]; d.vseg[q] = vseg[k]; d.vphase[q] = vphase[k]; d.vearly[q] = vearly[k];
        d.vvol[q] = vvol[k]; d.vlen[q] = vlen[k]; d.vrob[q] = vrob[k];
    }
    d.n_suppressed[inst] += suppressed;
}

// ------------------------------------------------------------------------
// Workgroup stepper for the trees the chain kernel does not take (trees with
// junctions, and chains too long for it): one workgroup per (tree, sample),
// the same equation, residual, factors and event logic as k_step, with the
// two sweeps of the tree elimination run in parallel.
//
// The tree is cut into heavy paths (a node continues its path through the
// child with the largest subtree, so every root-to-leaf path crosses at most
// log2(n) path changes), grouped by light depth.  Each level lists its nodes
// path by path, head to bottom (hp_node).  Along that list the elimination
// b_i = r_i + sum_c l_c b_c is the reverse affine recurrence
// x_k = c_k + lambda_k x_{k+1}, where c_k adds the light children's b (from
// deeper levels) and lambda_k = l of the next node (0 at a path's bottom);
// the back substitution delta_i = b_i / d_i + l_i delta_parent is the
// forward recurrence y_k = c'_k + mu_k y_{k-1}, mu_k = l_i (0 at a path's
// head, whose parent's delta -- one level up -- enters c'_k).  Each
// recurrence is a workgroup scan of affine maps: every thread composes its
// chunk serially, the threads' maps are scanned in LDS (Hillis-Steele), and
// every thread applies the incoming value along its chunk.  Any order that
// eliminates children before parents uses the same factors, so they are
// those of factor_instance; only the rounding order of the solve differs.
// After a nucleation only the void's path to the root is refactored.
// ------------------------------------------------------------------------
// y -> c + a y over the threads: suffix (rev) or prefix composition; returns
// the composed map's constant of the neighbouring thread (the value entering
// this thread's chunk): thread t+1's for a suffix scan, t-1's for a prefix.
template <int BR_WG, bool REV>
__device__ inline double br_scan(double a, double c, double (*sa)[BR_WG], double (*sc)[BR_WG])
{
    const int t = threadIdx.x;
    int buf = 0;
    sa[0][t] = a;
    sc[0][t] = c;
    __syncthreads();
#pragma unroll
    for (int dd = 1; dd < BR_WG; dd <<= 1) {
        const int o = REV ? t + dd : t - dd;
        if (REV ? (o < BR_WG) : (o >= 0)) {
            const double a2 = sa[buf][o], c2 = sc[buf][o];
            c = c + a * c2;
            a = a * a2;
        }
        sa[buf ^ 1][t] = a;
        sc[buf ^ 1][t] = c;
        buf ^= 1;
        __syncthreads();
    }
    const int o = REV ? t + 1 : t - 1;
    const double in = (REV ? (o < BR_WG) : (o >= 0)) ? sc[buf][o] : 0.0;
    __syncthreads();             // the buffers are rewritten by the next call
    return in;
}

template <int BR_WG>
__device__ inline double br_sum(double v, double *red)
{
    v = wsum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < BR_WG / 64; ++k) a += red[k];
    __syncthreads();
    return a;
}
template <int BR_WG>
__device__ inline double br_max(double v, double *red)
{
    v = wmax(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double a = -INFINITY;
#pragma unroll
    for (int k = 0; k < BR_WG / 64; ++k) a = fmax(a, red[k]);
    __syncthreads();
    return a;
}

template <typename R, int BR_WG>
__global__ __launch_bounds__(BR_WG) void k_branch(Dev d, int n_steps, int step0)
{
    __shared__ double s_a[2][BR_WG], s_c[2][BR_WG];
    __shared__ double s_red[BR_WG / 64];
    __shared__ int s_vn[MAXV], s_vseg[MAXV], s_vphase[MAXV], s_vearly[MAXV], s_nv;
    __shared__ double s_vvol[MAXV], s_vlen[MAXV], s_vrob[MAXV];
    const int S = d.S;
    const int g = blockIdx.x / S, s = blockIdx.x - g * S;
    const int t = d.br_tree[g];
    const int inst = t * S + s;
    if (!d.sample_active[s] || !d.inst_active[inst]) return;     // uniform over the workgroup
    const int tid = threadIdx.x;
    R *sig = (R *)d.sigma;
    const R *dtf = (const R *)d.dtf, *dinv = (const R *)d.dinv, *lf = (const R *)d.lfac;
    const R *sc = (const R *)d.sc;
    double *W = d.wsp;
    const int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
    const int nlev = d.br_nlev[g];
    const int *lvl = d.br_lvl + d.br_lvl0[g];            // level L: hp positions [i0 + lvl[L], i0 + lvl[L+1])
    if (tid == 0) {
        atomicAdd(&d.node_steps[blockIdx.x & (NS_SLOTS - 1)], (unsigned long long)(i1 - i0) * (unsigned long long)n_steps);
        const int nv = d.nv[inst];
        s_nv = nv;
        for (int k = 0; k < MAXV; ++k) {
            const int q = inst * MAXV + k;
            const bool u = k < nv;
            s_vn[k] = u ? d.vnode[q] : -1;
            s_vseg[k] = u ? d.vseg[q] : -1;
            s_vphase[k] = u ? d.vphase[q] : 0;
            s_vearly[k] = u ? d.vearly[q] : 0;
            s_vvol[k] = u ? d.vvol[q] : 0.0;
            s_vlen[k] = u ? d.vlen[q] : 0.0;
            s_vrob[k] = u ? d.vrob[q] : 0.0;
        }
    }
    __syncthreads();
    int suppressed = 0;
    const double Vsum = d.tree_V[t];
    double q0 = 0.0;
    for (int i = i0 + tid; i < i1; i += BR_WG) q0 += d.V[i] * ld_sig(d, sig, (size_t)i * S + s);
    double Q0 = br_sum<BR_WG>(q0, s_red);
    for (int k = 0; k < s_nv; ++k) Q0 += d.B * s_vvol[k];
    double corr = 0.0;
    const double dt = d.dt;

    for (int st = 0; st < n_steps; ++st) {
        const int nv = s_nv;
        // residual dt (A sigma + f) in FP64 from exact flux differences
        for (int i = i0 + tid; i < i1; i += BR_WG) {
            const size_t x = (size_t)i * S + s;
            const double si = ld_sig(d, sig, x) + corr;
            const bool isv = in_list(i, s_vn, nv);
            double r = isv ? 0.0 : (double)dtf[x];
            const int p = d.parent[i];
            if (p >= 0) r += dt * d.xi_k[(size_t)d.seg[i] * S + s] * d.g0[i] * ((ld_sig(d, sig, (size_t)p * S + s) + corr) - si);
            for (int k = d.child_off[i]; k < d.child_off[i + 1]; ++k) {
                const int c = d.child[k];
                r += dt * d.xi_k[(size_t)d.seg[c] * S + s] * d.g0[c] * ((ld_sig(d, sig, (size_t)c * S + s) + corr) - si);
            }
            if (isv)
                for (int k = 0; k < nv; ++k) if (s_vn[k] == i) r -= dt * s_vrob[k] * si;
            W[x] = r;
        }
        __syncthreads();
        // elimination, deepest level first: b along each path, bottom up
        for (int L = nlev - 1; L >= 0; --L) {
            const int lo = i0 + lvl[L], hi = i0 + lvl[L + 1];
            const int ch = (hi - lo + BR_WG - 1) / BR_WG;
            const int p0 = lo + tid * ch, p1 = min(p0 + ch, hi);
            double A = 1.0, C = 0.0;
            for (int k = p1 - 1; k >= p0; --k) {
                const int i = d.br_node[k];
                const size_t x = (size_t)i * S + s;
                const int hv = d.br_heavy[i];
                double c = W[x];
                for (int m = d.child_off[i]; m < d.child_off[i + 1]; ++m) {
                    const int h = d.child[m];
                    if (h != hv) c += (double)lf[(size_t)h * S + s] * W[(size_t)h * S + s];
                }
                W[x] = c;
                const double lam = hv >= 0 ? (double)lf[(size_t)hv * S + s] : 0.0;
                C = c + lam * C;
                A = lam * A;
            }
            double xin = br_scan<BR_WG, true>(A, C, s_a, s_c);
            for (int k = p1 - 1; k >= p0; --k) {
                const int i = d.br_node[k];
                const size_t x = (size_t)i * S + s;
                const int hv = d.br_heavy[i];
                const double lam = hv >= 0 ? (double)lf[(size_t)hv * S + s] : 0.0;
                xin = W[x] + lam * xin;
                W[x] = xin;
            }
            __syncthreads();
        }
        // back substitution, root level first: delta along each path, top down
        for (int L = 0; L < nlev; ++L) {
            const int lo = i0 + lvl[L], hi = i0 + lvl[L + 1];
            const int ch = (hi - lo + BR_WG - 1) / BR_WG;
            const int p0 = lo + tid * ch, p1 = min(p0 + ch, hi);
            double M = 1.0, D = 0.0;
            for (int k = p0; k < p1; ++k) {
                const int i = d.br_node[k];
                const size_t x = (size_t)i * S + s;
                const bool head = k == lo || d.br_node[k - 1] != d.parent[i];
                double c = W[x] * (double)dinv[x];
                double mu = 0.0;
                if (head) {
                    const int p = d.parent[i];
                    if (p >= 0) c += (double)lf[x] * W[(size_t)p * S + s];
                } else {
                    mu = (double)lf[x];
                }
                W[x] = c;
                D = c + mu * D;
                M = mu * M;
            }
            double yin = br_scan<BR_WG, false>(M, D, s_a, s_c);
            for (int k = p0; k < p1; ++k) {
                const int i = d.br_node[k];
                const size_t x = (size_t)i * S + s;
                const bool head = k == lo || d.br_node[k - 1] != d.parent[i];
                yin = W[x] + (head ? 0.0 : (double)lf[x] * yin);
                W[x] = yin;
            }
            __syncthreads();
        }
        // new stress, stress content, nucleation candidates
        double qs = 0.0, mx = -INFINITY;
        for (int i = i0 + tid; i < i1; i += BR_WG) {
            const size_t x = (size_t)i * S + s;
            const double v = ld_sig(d, sig, x) + corr + W[x];
            st_sig(d, sig, x, v);
            qs += d.V[i] * v;
            if (v >= (double)sc[x] && !in_list(i, s_vn, nv)) mx = fmax(mx, v);
        }
        __syncthreads();            // stores published before the void pass reads them
        // void growth: dV = (dt/B) (Robin weight * sigma_v + f_v) (eq. 15 accounting)
        if (tid < nv) {
            const int k = tid;
            const size_t x = (size_t)s_vn[k] * S + s;
            s_vvol[k] += (dt * s_vrob[k] * ld_sig(d, sig, x) + (double)dtf[x]) / d.B;
            const int e = s_vseg[k];
            const double Wd = d.w[e], H = d.h[e];
            const double l = fmin(s_vvol[k] / (Wd * H), d.len[e]);
            s_vlen[k] = l;
            if (s_vphase[k] == 0 && l >= Wd) {
                s_vphase[k] = 1;
                if (s_vearly[k]) {
                    d.open[(size_t)s * d.n_res + e] = 1;
                    *d.open_dirty = 1u;
                }
            }
        }
        const double Q = br_sum<BR_WG>(qs, s_red);        // its barriers also publish the void records
        {
            double vtot = 0.0;
            for (int k = 0; k < nv; ++k) vtot += s_vvol[k];
            corr = (Q0 - d.B * vtot - Q) / Vsum;
        }
        // nucleation: peak candidate, ties within 1e-12 to the lowest node
        const double pk = br_max<BR_WG>(mx, s_red);
        if (pk != -INFINITY) {
            if (nv < d.max_voids) {
                const double thr = pk - 1e-12 * (pk < 0 ? -pk : pk);
                double lowest = INFINITY;
                for (int i = i0 + tid; i < i1; i += BR_WG) {
                    const size_t x = (size_t)i * S + s;
                    const double val = ld_sig(d, sig, x);
                    if (val >= (double)sc[x] && val >= thr && !in_list(i, s_vn, nv)) lowest = fmin(lowest, (double)i);
                }
                lowest = -br_max<BR_WG>(-lowest, s_red);
                if (tid == 0) {
                    int vn[MAXV], vseg[MAXV], vphase[MAXV], vearly[MAXV], nv2 = nv;
                    double vvol[MAXV], vlen[MAXV], vrob[MAXV];
                    for (int k = 0; k < MAXV; ++k) {
                        vn[k] = s_vn[k]; vseg[k] = s_vseg[k]; vphase[k] = s_vphase[k]; vearly[k] = s_vearly[k];
                        vvol[k] = s_vvol[k]; vlen[k] = s_vlen[k]; vrob[k] = s_vrob[k];
                    }
                    const int v = (int)lowest;
                    add_void_path<R>(d, inst, t, s, v, step0 + st, vn, vvol, vlen, vrob, vseg, vphase, vearly, nv2);
                    for (int k = 0; k < MAXV; ++k) {
                        s_vn[k] = vn[k]; s_vseg[k] = vseg[k]; s_vphase[k] = vphase[k]; s_vearly[k] = vearly[k];
                        s_vvol[k] = vvol[k]; s_vlen[k] = vlen[k]; s_vrob[k] = vrob[k];
                    }
                    s_nv = nv2;
                    __threadfence_block();
                }
                __syncthreads();
            } else {
                ++suppressed;
            }
        }
    }
    if (corr != 0.0)
        for (int i = i0 + tid; i < i1; i += BR_WG) {
            const size_t x = (size_t)i * S + s;
            st_sig(d, sig, x, ld_sig(d, sig, x) + corr);
        }
    if (tid == 0) {
        const int nv = s_nv;
        d.nv[inst] = nv;
        for (int k = 0; k < nv; ++k) {
            const int q = inst * MAXV + k;
            d.vnode[q] = s_vn[k]; d.vseg[q] = s_vseg[k]; d.vphase[q] = s_vphase[k]; d.vearly[q] = s_vearly[k];
            d.vvol[q] = s_vvol[k]; d.vlen[q] = s_vlen[k]; d.vrob[q] = s_vrob[k];
        }
        d.n_suppressed[inst] += suppressed;
    }
}

// Resistance write-back of one (tree, sample): dR of each segment of the tree
// is the sum of its late-failure voids' eq. 17 increments.
EM_KERNEL void k_void_dR(Dev d)
{
    int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= d.n_trees * d.S) return;
    int t, s;
    int inst = inst_of_slot(d, slot, t, s);
    double *dR = d.dR + (size_t)s * d.n_res;
    // voids never disappear, so only their host segments can carry a change
    int nv = d.nv[inst];
    for (int k = 0; k < nv; ++k) dR[d.vseg[inst * MAXV + k]] = 0.0;
    for (int k = 0; k < nv; ++k) {
        int q = inst * MAXV + k;
        if (d.vearly[q]) continue;
        int e = d.vseg[q];
        dR[e] += late_dR(d, d.vlen[q], d.w[e], d.h[e], d.rho * xi_rho(d, e, s));
    }
}

template <typename R>
EM_KERNEL void k_set_sigma_T(Dev d)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.ns * d.S) return;
    ((R *)d.sigma)[g] = (R)d.sigT;
    if (d.sig_lo) d.sig_lo[g] = (float)(d.sigT - (double)(R)d.sigT);
}

template <typename R>
EM_KERNEL void k_inject_void(Dev d, int s, int t, int v)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int inst = t * d.S + s;
    int nv = d.nv[inst];
    if (nv >= d.max_voids) return;
    int vn[MAXV], vseg[MAXV], vphase[MAXV], vearly[MAXV];
    double vvol[MAXV], vlen[MAXV], vrob[MAXV];
    for (int k = 0; k < MAXV; ++k) {
        int q = inst * MAXV + k;
        bool u = k < nv;
        vn[k] = u ? d.vnode[q] : -1; vseg[k] = u ? d.vseg[q] : -1;
        vphase[k] = u ? d.vphase[q] : 0; vearly[k] = u ? d.vearly[q] : 0;
        vvol[k] = u ? d.vvol[q] : 0.0; vlen[k] = u ? d.vlen[q] : 0.0; vrob[k] = u ? d.vrob[q] : 0.0;
    }
    add_void<R>(d, inst, t, s, v, 0, vn, vvol, vlen, vrob, vseg, vphase, vearly, nv);
    d.nv[inst] = nv;
    for (int k = 0; k < nv; ++k) {
        int q = inst * MAXV + k;
        d.vnode[q] = vn[k]; d.vseg[q] = vseg[k]; d.vphase[q] = vphase[k]; d.vearly[q] = vearly[k];
        d.vvol[q] = vvol[k]; d.vlen[q] = vlen[k]; d.vrob[q] = vrob[k];
    }
}

// Copy one sample's column of a [node][S] array to/from a dense FP64 vector.
template <typename R>
EM_KERNEL void k_copy_col(Dev d, void *arr, int s, double *out, int to_state)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.ns) return;
    R *a = (R *)arr;
    const size_t x = (size_t)i * d.S + s;
    if (arr == d.sigma) {               // the stress state (with its low part)
        if (to_state) st_sig(d, a, x, out[i]);
        else out[i] = ld_sig(d, (const R *)a, x);
    } else {
        if (to_state) a[x] = (R)out[i];
        else out[i] = (double)a[x];
    }
}

// ------------------------------------------------------------------------
// Learned screen.  Per tree (sample-independent): total wire length, the
// longest root-to-node distance along the tree, segment count and junction
// count (nodes of degree >= 3).  Per (tree, sample): current densities, the
// Arrhenius diffusivity of Sec. III-D at edge-midpoint temperature times the
// Monte Carlo multiplier, the peak p of the screen's zero-flux steady stress
// over the node critical stress (Sec. III-B, first node of the largest ratio),
// and the slowest-mode diffusion time Lpk^2/(pi^2 kappa_pk) over the
// distance Lpk (difference of root distances, floored at 0.1 um) from p to
// the nearest node whose steady stress is at or below sigma_T, kappa_pk the
// mean diffusivity of the edges at p; and the temperature at p.
// ------------------------------------------------------------------------
EM_KERNEL void k_tree_static(Dev d)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d.n_trees) return;
    int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
    double lpath = 0.0, nj = 0.0, prev = 0.0;
    d.rdist[i0] = 0.0;
    for (int i = i0; i < i1; ++i) {
        int p = d.parent[i];
        int deg = (p >= 0 ? 1 : 0) + (d.child_off[i + 1] - d.child_off[i]);
        nj += deg >= 3 ? 1.0 : 0.0;
        if (p >= 0) {
            double r = ((p == i - 1) ? prev : d.rdist[p]) + d.len[d.seg[i]] / d.N;
            d.rdist[i] = r;
            prev = r;
            lpath = fmax(lpath, r);
        }
    }
    double lt = 0.0;
    for (int k = d.tseg_off[t]; k < d.tseg_off[t + 1]; ++k) lt += d.len[d.tseg[k]];
    double *o = d.tstat + (size_t)t * 4;
    o[0] = lt;
    o[1] = lpath;
    o[2] = (double)(d.tseg_off[t + 1] - d.tseg_off[t]);
    o[3] = nj;
}

__device__ inline double kappa_arrhenius(const Dev &d, double T)
{
    double kT = K_B * T;
    return d.D0 * exp(-d.Ea_eV * E_CHG / kT) * d.B * d.Omega / kT;
}

// ---- per-instance passes by a workgroup of FB threads (four wavefronts):
// a tree of a few thousand nodes is read four times as fast as by one wave.
constexpr int FB = 256, FB_LOG = 8;
static_assert((1 << FB_LOG) == FB, "FB_LOG");

// Workgroup reductions over FB threads (every thread gets the result; sh is
// an LDS scratch of FB/64 doubles; the leading barrier guards its reuse).
__device__ inline double bsum(double v, double *sh)
{
    v = wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < FB / 64; ++k) r += sh[k];
    return r;
}
__device__ inline double bmax(double v, double *sh)
{
    v = wmax(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int k = 1; k < FB / 64; ++k) r = fmax(r, sh[k]);
    return r;
}
__device__ inline double bmin(double v, double *sh)
{
    return -bmax(-v, sh);
}

// psi_i = psi_parent + dir dx (S + M) from the root by a workgroup: chunks of
// FB nodes in pre-order; within a chunk the parent links are followed by
// pointer jumping through LDS; a parent in an earlier chunk is read back from
// psi (written by this workgroup before the chunk's barrier).  Then
// sigma_ss = sigma_T + psi - <psi>_V.
__device__ void steady_stress_blk(const Dev &d, int t, int s, double (*vs)[FB], int (*as)[FB], double *sh)
{
    const int S = d.S, tid = threadIdx.x;
    const int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
    double *psi = d.psi;
    double num = 0.0, den = 0.0;
    for (int c = i0; c < i1; c += FB) {
        const int i = c + tid;
        const bool ok = i < i1;
        double v = 0.0;
        int a = -1;
        if (ok && i > i0) {
            const int e = d.seg[i];
            const double dx = d.len[e] / d.N;
            const double Sd = E_CHG * d.Z * d.rho * xi_rho(d, e, s) * d.jseg[(size_t)s * d.n_res + e] / d.Omega;
            v = d.dir[i] * dx * (Sd + tm_scale(d, i, s) * d.mdrv[i]);
            a = d.parent[i];
        }
        int buf = 0;
#pragma unroll
        for (int r = 0; r < FB_LOG; ++r) {
            vs[buf][tid] = v;
            as[buf][tid] = a;
            __syncthreads();
            if (a >= c) {
                v += vs[buf][a - c];
                a = as[buf][a - c];
            }
            buf ^= 1;
        }
        if (a >= 0) v += psi[(size_t)a * S + s];
        if (ok) {
            psi[(size_t)i * S + s] = v;
            num += d.V[i] * v;
            den += d.V[i];
        }
        __threadfence_block();
        __syncthreads();
    }
    const double mean = bsum(num, sh) / bsum(den, sh);
    for (int i = i0 + tid; i < i1; i += FB) psi[(size_t)i * S + s] = d.sigT + psi[(size_t)i * S + s] - mean;
    __threadfence_block();
    __syncthreads();
}

// Features of one instance by a workgroup (the screen's steady stress must
// be current in column pc of psi); thread 0 writes the NFEAT values.
__device__ void features_blk(const Dev &d, int t, int s, int pc, float *x, double *sh, int *shi)
{
    const int S = d.S, tid = threadIdx.x;
    const double *ts = d.tstat + (size_t)t * 4;
    auto PSI = [&](int i) { return d.psi[(size_t)i * S + pc]; };
    double jmax = 0.0, jl = 0.0;
    for (int k = d.tseg_off[t] + tid; k < d.tseg_off[t + 1]; k += FB) {
        int e = d.tseg[k];
        double j = fabs(d.jseg[(size_t)s * d.n_res + e]);
        jmax = fmax(jmax, j);
        jl += d.len[e] * j;
    }
    jmax = bmax(jmax, sh);
    jl = bsum(jl, sh);
    // edge (parent(i), i): Arrhenius diffusivity at the midpoint temperature
    auto edge_kappa = [&](int i) {
        return d.xi_k[(size_t)d.seg[i] * S + s] * kappa_arrhenius(d, 0.5 * (d.T[i] + d.T[d.parent[i]]));
    };
    const int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
    // pass 1: mean diffusivity, peak ratio, least critical stress, the
    // blocked-end time and the largest diffusivity
    double ksum = 0.0, ne = 0.0, r = -INFINITY, dsmin = INFINITY, tblk = INFINITY, kmax = 0.0;
    int pk = 0x7fffffff;
    for (int i = i0 + tid; i < i1; i += FB) {
        const int p = d.parent[i];
        const double ss = PSI(i);
        const double sci = node_scrit(d, i, s);
        dsmin = fmin(dsmin, sci - d.sigT);
        if (p >= 0) {
            const double ke = edge_kappa(i);
            ksum += ke;
            ne += 1.0;
            kmax = fmax(kmax, ke);
            const double le = d.len[d.seg[i]] / d.N;
            const double g = fabs(ss - PSI(p)) / le;
            if (isfinite(g) && g > 0.0) {
                const double ds = fmax(fmin(sci, node_scrit(d, p, s)) - d.sigT, 1e3);
                tblk = fmin(tblk, M_PI * ds * ds / (4.0 * ke * g * g));
            }
        }
        if (isfinite(ss)) {
            double q = ss / sci;
            if (q > r) { r = q; pk = i; }          // threads visit ascending nodes: first max
        }
    }
    ksum = bsum(ksum, sh);
    ne = bsum(ne, sh);
    dsmin = fmax(bmin(dsmin, sh), 1e3);
    tblk = bmin(tblk, sh);
    kmax = bmax(kmax, sh);
    // peak: largest ratio, lowest node on ties
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ro = __shfl_xor(r, o, 64);
        const int po = __shfl_xor(pk, o, 64);
        if (ro > r || (ro == r && po < pk)) { r = ro; pk = po; }
    }
    __syncthreads();
    if ((tid & 63) == 0) { sh[tid >> 6] = r; shi[tid >> 6] = pk; }
    __syncthreads();
    r = sh[0]; pk = shi[0];
#pragma unroll
    for (int k = 1; k < FB / 64; ++k)
        if (sh[k] > r || (sh[k] == r && shi[k] < pk)) { r = sh[k]; pk = shi[k]; }
    if (pk == 0x7fffffff) { pk = i0; r = -10.0; }
    r = fmin(fmax(r, -10.0), 10.0);
    // pass 2: distance from the peak to the nearest node at or below sigma_T;
    // the fast edges (kappa >= kappa_max / 4): their length and the stress
    // they could build if blocked on both sides (sum of g l / 2)
    double lpk = INFINITY, lf = 0.0, sf = 0.0;
    const double dp = d.rdist[pk];
    for (int i = i0 + tid; i < i1; i += FB) {
        const double ss = PSI(i);
        if (ss <= d.sigT) lpk = fmin(lpk, fabs(d.rdist[i] - dp));
        const int p = d.parent[i];
        if (p < 0 || !(edge_kappa(i) >= 0.25 * kmax)) continue;
        const double dpsi = fabs(ss - PSI(p));
        lf += d.len[d.seg[i]] / d.N;
        if (isfinite(dpsi)) sf += 0.5 * dpsi;
    }
    lpk = bmin(lpk, sh);
    lf = bsum(lf, sh);
    sf = bsum(sf, sh);
    if (tid != 0) return;
    if (!isfinite(lpk)) lpk = ts[1];
    lpk = fmax(lpk, 1e-7);
    double kp = 0.0;
    int np_ = 0;
    for (int k = d.child_off[pk]; k < d.child_off[pk + 1]; ++k) { kp += edge_kappa(d.child[k]); ++np_; }
    if (d.parent[pk] >= 0) { kp += edge_kappa(pk); ++np_; }
    kp /= np_;
    double kmean = ksum / ne;
    double tau = lpk * lpk / (M_PI * M_PI * kp);
    x[0] = (float)log10(ts[0] / 1e-6);
    x[1] = (float)log10(ts[1] / 1e-6);
    x[2] = (float)(ts[2] / 8.0);
    x[3] = (float)(ts[3] / 4.0);
    x[4] = (float)log10(fmax(jmax, 1e3) / 1e9);
    x[5] = (float)log10(fmax(jl / ts[0], 1e3) / 1e9);
    x[6] = (float)log10(kmean / 1e-15);
    x[7] = (float)log10(kp / 1e-15);
    x[8] = (float)r;
    x[9] = (float)log10(fmax(r - 1.0, 1e-6));
    x[10] = (float)(log10(tau) - 8.0);
    x[11] = (float)((d.T[pk] - 300.0) / 100.0);
    // early-time scales: the time a blocked end of a semi-infinite wire with
    // an edge's steady drive g and diffusivity would take to reach the
    // critical stress (sigma(0, t) = 2 g sqrt(kappa t / pi)), least over the
    // edges; the largest diffusivity; the fast edges' blocked stress over the
    // least critical stress; their diffusion time L_f^2 / (pi^2 kappa_max)
    x[12] = (float)(log10(fmin(fmax(tblk, 1.0), 1e16)) - 8.0);
    x[13] = (float)log10(fmax(kmax, 1e-30) / 1e-15);
    x[14] = (float)fmin(sf / dsmin, 10.0);
    lf = fmax(lf, 1e-7);
    x[15] = (float)(log10(lf * lf / (M_PI * M_PI * fmax(kmax, 1e-30))) - 8.0);
}

// every instance, or only those a deferral could apply to (mortal, and
// active or already deferred); one instance per workgroup.  psi_col0: the
// steady stress of a shared screen (column 0 holds every sample's).
__global__ __launch_bounds__(FB) void k_features(Dev d, float *X, int candidates_only, int psi_col0)
{
    __shared__ double sh[FB / 64];
    __shared__ int shi[FB / 64];
    const int slot = blockIdx.x;
    int t, s;
    int inst = inst_of_slot(d, slot, t, s);
    if (candidates_only && !(d.tree_mortal[inst] && (d.inst_active[inst] || d.deferred[inst]))) return;
    features_blk(d, t, s, psi_col0 ? 0 : s, X + (size_t)inst * NFEAT, sh, shi);
}

// Features of the still-deferred instances of def_list[0..n) with the current
// densities (their steady stress is refreshed first, in their own column),
// row k for def_list[k], one instance per workgroup.  An instance whose
// segment currents have all stayed within tol x the largest of them since its
// last evaluation (interval def_k[k], densities in jhist) keeps that row: its
// prediction would hardly move.
__global__ __launch_bounds__(FB) void k_reeval_features(Dev d, int n, float *X, const double *jhist, int k_now,
                                                        double tol)
{
    __shared__ double vs[2][FB];
    __shared__ int as[2][FB];
    __shared__ double sh[FB / 64];
    __shared__ int shi[FB / 64];
    const int k = blockIdx.x, tid = threadIdx.x;
    int inst = d.def_list[k];
    if (!d.deferred[inst]) return;
    int t = inst / d.S, s = inst - (inst / d.S) * d.S;
    const int kp = d.def_k[k];
    if (kp >= 0) {
        const double *jp = jhist + ((size_t)kp * d.S + s) * d.n_res;
        const double *jn = d.jseg + (size_t)s * d.n_res;
        double jm = 0.0, dj = 0.0;
        for (int q = d.tseg_off[t] + tid; q < d.tseg_off[t + 1]; q += FB) {
            const int e = d.tseg[q];
            jm = fmax(jm, fabs(jp[e]));
            dj = fmax(dj, fabs(jn[e] - jp[e]));
        }
        dj = bmax(dj, sh);
        jm = bmax(jm, sh);
        if (dj <= tol * jm) return;
    }
    steady_stress_blk(d, t, s, vs, as, sh);
    features_blk(d, t, s, s, X + (size_t)k * NFEAT, sh, shi);
    if (tid == 0) d.def_k[k] = k_now;
}

// A re-evaluated prediction can only bring a deferred instance's activation forward.
EM_KERNEL void k_yhat_min(Dev d, int n, const float *y)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int inst = d.def_list[k];
    if (d.deferred[inst]) d.yhat[inst] = fminf(d.yhat[inst], y[k]);
}

__device__ inline double t_hat(float y) { return T_REF * pow(10.0, (double)y); }

// Defer the steady-state-mortal active instances predicted to nucleate after thr.
EM_KERNEL void k_defer(Dev d, const float *y, double thr)
{
    int inst = blockIdx.x * blockDim.x + threadIdx.x;
    if (inst >= d.n_trees * d.S) return;
    d.yhat[inst] = y[inst];
    d.catchup[inst] = 0;
    uint8_t df = 0;
    const uint8_t act = d.inst_active[inst] | d.deferred[inst];   // a repeated evaluation starts over
    d.inst_active[inst] = act;
    if (act && d.tree_mortal[inst] && t_hat(y[inst]) > thr) {
        d.inst_active[inst] = 0;
        df = 1;
        atomicAdd(&d.sur_cnt[0], 1u);
        d.def_list[atomicAdd(&d.sur_cnt[4], 1u)] = inst;
    }
    d.deferred[inst] = df;
}

// Mark deferred instances of running samples whose prediction falls due by
// thr and list them (sur_cnt[5] counts this activation's list).
EM_KERNEL void k_activate(Dev d, double thr)
{
    int inst = blockIdx.x * blockDim.x + threadIdx.x;
    if (inst >= d.n_trees * d.S) return;
    if (!d.deferred[inst] || !d.sample_active[inst % d.S]) return;
    if (t_hat(d.yhat[inst]) <= thr) {
        d.deferred[inst] = 0;
        d.catchup[inst] = 1;
        atomicAdd(&d.sur_cnt[1], 1u);
        d.act_list[atomicAdd(&d.sur_cnt[5], 1u)] = inst;
    }
}

// Caught-up instances join the active set.  One that nucleated before the
// interval it was activated for is a late activation; if one of its voids had
// also reached the growth phase (a resistance change the earlier IR solves
// did not see), it is a violation: only then can the screened run differ from
// the unscreened one, and its sample is flagged for a re-run without the screen.
EM_KERNEL void k_catchup_done(Dev d, int step_lim)
{
    int inst = blockIdx.x * blockDim.x + threadIdx.x;
    if (inst >= d.n_trees * d.S) return;
    if (!d.catchup[inst]) return;
    const int nv = d.nv[inst];
    if (nv > 0 && d.vstep[(size_t)inst * MAXV] < step_lim) {
        atomicAdd(&d.sur_cnt[2], 1u);
        bool grown = false;
        for (int k = 0; k < nv; ++k) grown |= d.vphase[(size_t)inst * MAXV + k] != 0;
        if (grown) {
            atomicAdd(&d.sur_cnt[3], 1u);
            d.sur_viol[inst % d.S] = 1;
        }
    }
    d.catchup[inst] = 0;
    d.inst_active[inst] = 1;
}

// ------------------------------------------------------------------------
// Steady-state skipping.  Between two IR solves an instance without voids
// steps C s' = f - A s by backward Euler: C = diag(V) the node volumes, A the
// Laplacian of the edge conductances g (positive).  A step of any size maps
// the distance e = s - s_inf to the steady state by (C + dt A)^-1 C, a
// nonnegative matrix (C + dt A is an M-matrix) with unit row sums (A 1 = 0),
// so every later e lies componentwise within [min e_n, max e_n].  On a tree e
// is known up to a constant from the residual: across the edge above a
// subtree, g (e_child - e_parent) is the sum of A s - f over the subtree.  On
// a chain (node i's parent i - 1) with r = dt (f - A s), the edge (i - 1, i)
// carries dt g (e_i - e_i-1) = sum of r over the nodes before i, and the
// potential P_i = sum over edges up to i of that sum / (dt g) equals e + const.
// Every later state then satisfies
//   s_n,i - (P_i - min P) <= s_m,i <= s_n,i + (max P - P_i),
// a band the steady state itself reaches (exact arithmetic; the stepping adds
// its rounding).  The forcing's total (zero but for rounding) is taken out in
// proportion to V first, as the stepping's content projection does; dt*f and
// dt*g are those the chain kernel steps with (the state's precision), the
// sums are FP64.  Skipped: an active chain instance without voids whose
// band is within tol_abs and keeps every node below its critical stress.
//
// Two launch forms.  With 64 samples or more, the chunked passes below.  With
// fewer samples, the chain kernel's lane table (each lane its block of chain_m
// consecutive nodes, instances never straddling a workgroup): the lane's
// loads issued together, then segmented scans over the instance's lanes in
// LDS.
// ------------------------------------------------------------------------
// Many-sample form: one lane per sample, the wavefront over 64 consecutive
// samples of one chain (every load coalesced), the chain cut into chunks of
// SS_CL nodes walked in parallel.  Per chunk (pass a): sums of dt f, V and
// the raw residual r, and of 1/(dt g), (the chunk's raw residual before the
// node)/(dt g) and (its volume before the node)/(dt g) over the chunk's
// edges.  Per instance (pass b): the forcing mean fm, then the chunks'
// carries in order -- r' before the chunk, and P where it starts, since the
// chunk adds carry G + H - fm K to P.  Per chunk (pass c): P at its nodes,
// its extremes and the margin.  Per instance (pass d): the decision.
// Scratch per (chunk, sample): 6 + 2 + 3 doubles; fm per instance.
template <typename R>
struct SsView {
    const Dev &d;
    int S, s;
    __device__ double sv(int i) const
    {
        const size_t x = (size_t)i * S + s;
        double v = (double)((const R *)d.sigma)[x];
        if (d.sig_lo) v += (double)d.sig_lo[x];
        return v;
    }
    __device__ double dtg(int i) const        // edge (i - 1, i)
    {
        return (double)(R)(d.dt * d.xi_k[(size_t)d.seg[i] * S + s] * d.g0[i]);
    }
    __device__ double fv(int i) const { return (double)((const R *)d.dtf)[(size_t)i * S + s]; }
    __device__ double vr(int i) const { return (double)((const R *)d.Vr)[i]; }
    __device__ double sc(int i) const { return (double)((const R *)d.sc)[(size_t)i * S + s]; }
};

__device__ inline bool ss_lane(const Dev &d, long long w, bool by_chunk, int &t, int &s, int &cg, size_t &inst)
{
    const int S = d.S, SW = (S + 63) / 64, lane = threadIdx.x & 63;
    const long long u = w / SW;
    const int s0 = (int)(w - u * SW) * 64;
    cg = by_chunk ? (int)u : -1;
    t = by_chunk ? d.ss_ctree[cg] : (int)u;
    s = min(s0 + lane, S - 1);                 // lanes past S repeat the last sample, unused
    inst = (size_t)t * S + s;
    return s0 + lane < S && d.tree_chain[t] && d.inst_active[inst] && d.sample_active[s] && d.nv[inst] == 0;
}

template <typename R>
EM_KERNEL void k_ssc_a(Dev d)
{
    const long long w = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= (long long)d.ss_nc * ((d.S + 63) / 64)) return;
    int t, s, cg;
    size_t inst;
    const bool act = ss_lane(d, w, true, t, s, cg, inst);
    if (!__any(act)) return;
    const SsView<R> v{d, d.S, s};
    const int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
    const int c0 = d.ss_cstart[cg], c1 = min(c0 + SS_CL, i1);
    double F = 0.0, Vs = 0.0, lr = 0.0, lv = 0.0, G = 0.0, H = 0.0, K = 0.0;
    double sp = c0 > i0 ? v.sv(c0 - 1) : 0.0, si = v.sv(c0), gl = c0 > i0 ? v.dtg(c0) : 0.0;
    for (int c = c0; c < c1; c += 8) {
        double sn[8], gr[8], f[8], vv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = c + k;
            const bool in = i < c1, nx = i + 1 < i1;
            sn[k] = in && nx ? v.sv(i + 1) : 0.0;
            gr[k] = in && nx ? v.dtg(i + 1) : 0.0;
            f[k] = in ? v.fv(i) : 0.0;
            vv[k] = in ? v.vr(i) : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = c + k;
            if (i >= c1) break;
            double r = f[k] + gr[k] * (sn[k] - si);
            if (i > i0) {
                r += gl * (sp - si);
                const double ig = 1.0 / gl;
                G += ig;
                H += lr * ig;
                K += lv * ig;
            }
            F += f[k];
            Vs += vv[k];
            lr += r;
            lv += vv[k];
            sp = si;
            si = sn[k];
            gl = gr[k];
        }
    }
    if (!act) return;
    const size_t S = d.S;
    double *o = d.ss_scr + (size_t)cg * 6 * S + s;
    o[0] = F; o[S] = Vs; o[2 * S] = lr; o[3 * S] = G; o[4 * S] = H; o[5 * S] = K;
}

EM_KERNEL void k_ssc_b(Dev d)
{
    const long long w = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= (long long)d.n_trees * ((d.S + 63) / 64)) return;
    int t, s, cg;
    size_t inst;
    if (!ss_lane(d, w, false, t, s, cg, inst)) return;
    const size_t S = d.S, NC = d.ss_nc;
    const int k0 = d.ss_coff[t], k1 = d.ss_coff[t + 1];
    const double *a = d.ss_scr;
    double *b = d.ss_scr + NC * 6 * S;
    double F = 0.0, V = 0.0;
    for (int c = k0; c < k1; ++c) {
        F += a[(size_t)c * 6 * S + s];
        V += a[((size_t)c * 6 + 1) * S + s];
    }
    const double fm = F / V;
    double cr = 0.0, cp = 0.0;
    for (int c = k0; c < k1; ++c) {
        const double *q = a + (size_t)c * 6 * S + s;
        b[(size_t)c * 2 * S + s] = cr;
        b[((size_t)c * 2 + 1) * S + s] = cp;
        cp += cr * q[3 * S] + q[4 * S] - fm * q[5 * S];
        cr += q[2 * S] - fm * q[S];
    }
    d.ss_scr[NC * 11 * S + inst] = fm;
}

template <typename R>
EM_KERNEL void k_ssc_c(Dev d)
{
    const long long w = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= (long long)d.ss_nc * ((d.S + 63) / 64)) return;
    int t, s, cg;
    size_t inst;
    const bool act = ss_lane(d, w, true, t, s, cg, inst);
    if (!__any(act)) return;
    const SsView<R> v{d, d.S, s};
    const size_t S = d.S, NC = d.ss_nc;
    const int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
    const int c0 = d.ss_cstart[cg], c1 = min(c0 + SS_CL, i1);
    const double fm = act ? d.ss_scr[NC * 11 * S + inst] : 0.0;
    const double *b = d.ss_scr + NC * 6 * S;
    double pre = act ? b[(size_t)cg * 2 * S + s] : 0.0, lp = act ? b[((size_t)cg * 2 + 1) * S + s] : 0.0;
    double pmax = -INFINITY, pmin = INFINITY, mmax = -INFINITY;
    double sp = c0 > i0 ? v.sv(c0 - 1) : 0.0, si = v.sv(c0), gl = c0 > i0 ? v.dtg(c0) : 0.0;
    for (int c = c0; c < c1; c += 8) {
        double sn[8], gr[8], f[8], vv[8], q[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = c + k;
            const bool in = i < c1, nx = i + 1 < i1;
            sn[k] = in && nx ? v.sv(i + 1) : 0.0;
            gr[k] = in && nx ? v.dtg(i + 1) : 0.0;
            f[k] = in ? v.fv(i) : 0.0;
            vv[k] = in ? v.vr(i) : 0.0;
            q[k] = in ? v.sc(i) : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = c + k;
            if (i >= c1) break;
            double r = f[k] - vv[k] * fm + gr[k] * (sn[k] - si);
            if (i > i0) {
                r += gl * (sp - si);
                lp += pre / gl;
            }
            pre += r;
            pmax = fmax(pmax, lp);
            pmin = fmin(pmin, lp);
            mmax = fmax(mmax, si - q[k] - lp);
            sp = si;
            si = sn[k];
            gl = gr[k];
        }
    }
    if (!act) return;
    double *o = d.ss_scr + NC * 8 * S + (size_t)cg * 3 * S + s;
    o[0] = pmax; o[S] = pmin; o[2 * S] = mmax;
}

EM_KERNEL void k_ssc_d(Dev d, double tol_abs)
{
    const long long w = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= (long long)d.n_trees * ((d.S + 63) / 64)) return;
    int t, s, cg;
    size_t inst;
    if (!ss_lane(d, w, false, t, s, cg, inst)) return;
    const size_t S = d.S, NC = d.ss_nc;
    const double *c3 = d.ss_scr + NC * 8 * S;
    double pmax = -INFINITY, pmin = INFINITY, mmax = -INFINITY;
    for (int c = d.ss_coff[t]; c < d.ss_coff[t + 1]; ++c) {
        const double *o = c3 + (size_t)c * 3 * S + s;
        pmax = fmax(pmax, o[0]);
        pmin = fmin(pmin, o[S]);
        mmax = fmax(mmax, o[2 * S]);
    }
    if (pmax - pmin <= tol_abs && mmax + pmax < 0.0) {
        d.inst_active[inst] = 0;
        d.ss_skip[inst] = 1;
        atomicAdd(&d.ss_cnt[0], 1u);
    }
}

constexpr int SS_WG_MAX = 1024, SS_M_MAX = CHAIN_M32W > CHAIN_M64 ? CHAIN_M32W : CHAIN_M64;

template <typename R>
__global__ __launch_bounds__(SS_WG_MAX) void k_ss_check(Dev d, double tol_abs)
{
    __shared__ double sa[SS_WG_MAX], sb[SS_WG_MAX];
    const int WG = blockDim.x, lane = threadIdx.x, S = d.S, M = d.chain_m;
    const size_t gl = (size_t)blockIdx.x * WG + lane;
    const int inst = d.lane_inst[gl];
    int s = 0, i0 = 0, i1 = 0, start = 0, cnt = 0, lo = lane, hi = lane;
    bool act = false;
    if (inst >= 0) {
        const int t = inst / S;
        s = inst - t * S;
        i0 = d.tree_off[t];
        i1 = d.tree_off[t + 1];
        const int kb = d.lane_blk[gl];
        start = i0 + kb * M;
        cnt = min(M, i1 - start);
        lo = lane - kb;
        hi = lo + (i1 - i0 + M - 1) / M - 1;
        act = d.inst_active[inst] && d.sample_active[s] && d.nv[inst] == 0;
    }
    if (!act) cnt = 0;
    // segmented inclusive scans of two values over the lanes [lo, lane]
    // (sums, or maxima), and the segment's results at its last lane
    auto scan2 = [&](double &x, double &y, bool mx) {
        sa[lane] = x;
        sb[lane] = y;
        __syncthreads();
        for (int dd = 1; dd < WG; dd <<= 1) {
            const bool in = lane - dd >= lo;
            const double u = in ? sa[lane - dd] : 0.0, w = in ? sb[lane - dd] : 0.0;
            __syncthreads();
            if (in) {
                x = mx ? fmax(x, u) : x + u;
                y = mx ? fmax(y, w) : y + w;
            }
            sa[lane] = x;
            sb[lane] = y;
            __syncthreads();
        }
    };
    auto totals = [&](double &x, double &y) {
        x = sa[hi];
        y = sb[hi];
        __syncthreads();
    };
    const R *sig = (const R *)d.sigma, *fv = (const R *)d.dtf, *sc = (const R *)d.sc, *Vr = (const R *)d.Vr;
    const float *slo = d.sig_lo;
    auto sv = [&](int i) -> double {
        const size_t x = (size_t)i * S + s;
        double v = (double)sig[x];
        if (slo) v += (double)slo[x];
        return v;
    };
    auto dtg = [&](int i) -> double {        // edge (i - 1, i)
        return (double)(R)(d.dt * d.xi_k[(size_t)d.seg[i] * S + s] * d.g0[i]);
    };
    // the lane's nodes and their neighbours: xs[j + 1] = state of node
    // start + j, xs[0] and xs[cnt + 1] the neighbours (0 past the chain's
    // ends, where ge = 0); ge[j] = dt g of the edge (start + j - 1, start + j)
    double xs[SS_M_MAX + 2], ge[SS_M_MAX + 1], fr[SS_M_MAX], vv[SS_M_MAX], cr[SS_M_MAX];
#pragma unroll
    for (int j = 0; j <= SS_M_MAX; ++j) {
        const int i = start - 1 + j;
        xs[j] = (j <= cnt + 1 && i >= i0 && i < i1 && cnt > 0) ? sv(i) : 0.0;
        ge[j] = (j <= cnt && start + j > i0 && start + j < i1 && cnt > 0) ? dtg(start + j) : 0.0;
    }
    xs[SS_M_MAX + 1] = (cnt == SS_M_MAX && start + cnt < i1) ? sv(start + cnt) : 0.0;
#pragma unroll
    for (int j = 0; j < SS_M_MAX; ++j) {
        const size_t x = (size_t)(start + j) * S + s;
        fr[j] = j < cnt ? (double)fv[x] : 0.0;
        vv[j] = j < cnt ? (double)Vr[start + j] : 0.0;
        cr[j] = j < cnt ? (double)sc[x] : 0.0;
    }
    double fs = 0.0, vs = 0.0, rs = 0.0;
#pragma unroll
    for (int j = 0; j < SS_M_MAX; ++j)
        if (j < cnt) {
            fs += fr[j];
            vs += vv[j];
            fr[j] += ge[j] * (xs[j] - xs[j + 1]) + ge[j + 1] * (xs[j + 2] - xs[j + 1]);   // dt f - dt A s
            rs += fr[j];
        }
    double ft = fs, vt = vs;
    scan2(ft, vt, false);
    totals(ft, vt);
    const double fm = act ? ft / vt : 0.0;
    const double rl = rs - fm * vs;
    double rinc = rl, dummy = 0.0;
    scan2(rinc, dummy, false);
    double pre = rinc - rl;                    // sum of r' over the instance's nodes before this lane's
    double lp = 0.0, lmax = -INFINITY, lmin = INFINITY, lm = -INFINITY;
#pragma unroll
    for (int j = 0; j < SS_M_MAX; ++j)
        if (j < cnt) {
            if (start + j > i0) lp += pre / ge[j];
            pre += fr[j] - vv[j] * fm;
            lmax = fmax(lmax, lp);
            lmin = fmin(lmin, lp);
            lm = fmax(lm, xs[j + 1] - cr[j] - lp);
        }
    double pinc = lp;
    scan2(pinc, dummy, false);
    const double cp = pinc - lp;               // the potential where this lane's nodes start
    double pmax = cp + lmax, mmax = lm - cp;   // largest P; largest s - sigma_crit - P
    scan2(pmax, mmax, true);
    totals(pmax, mmax);
    double npmin = -(cp + lmin), unused = -INFINITY;
    scan2(npmin, unused, true);
    totals(npmin, unused);
    if (act && lane == lo && pmax + npmin <= tol_abs && mmax + pmax < 0.0) {
        d.inst_active[inst] = 0;
        d.ss_skip[inst] = 1;
        atomicAdd(&d.ss_cnt[0], 1u);
    }
}

EM_KERNEL void k_ss_wake(Dev d, int all)
{
    const int inst = blockIdx.x * blockDim.x + threadIdx.x;
    if (inst >= d.n_trees * d.S) return;
    if (!d.ss_skip[inst] || !(all || d.g_chg_s[inst % d.S])) return;
    d.ss_skip[inst] = 0;
    d.inst_active[inst] = 1;
    atomicAdd(&d.ss_cnt[1], 1u);
}

// ---------------------------- launchers ---------------------------------
void launch_ss_check(const Dev &d, bool fp32, double tol_abs, hipStream_t st)
{
    if (d.n_chain_wg <= 0 || d.chain_wg <= 0 || d.chain_wg > SS_WG_MAX) return;
    if (d.S >= 64 && d.ss_nc > 0 && d.ss_scr) {
        const long long SW = (d.S + 63) / 64;
        const int nbc = (int)((d.ss_nc * SW + 3) / 4), nbt = (int)(((long long)d.n_trees * SW + 3) / 4);
        if (fp32) k_ssc_a<float><<<nbc, 256, 0, st>>>(d);
        else k_ssc_a<double><<<nbc, 256, 0, st>>>(d);
        k_ssc_b<<<nbt, 256, 0, st>>>(d);
        if (fp32) k_ssc_c<float><<<nbc, 256, 0, st>>>(d);
        else k_ssc_c<double><<<nbc, 256, 0, st>>>(d);
        k_ssc_d<<<nbt, 256, 0, st>>>(d, tol_abs);
        return;
    }
    if (fp32) k_ss_check<float><<<d.n_chain_wg, d.chain_wg, 0, st>>>(d, tol_abs);
    else k_ss_check<double><<<d.n_chain_wg, d.chain_wg, 0, st>>>(d, tol_abs);
}
void launch_ss_wake(const Dev &d, bool all, hipStream_t st)
{
    k_ss_wake<<<nblocks((long long)d.n_trees * d.S), 256, 0, st>>>(d, all ? 1 : 0);
}
void launch_node_T(const Dev &d, hipStream_t st)
{
    k_node_T<<<nblocks(d.ns), 256, 0, st>>>(d);
}
void launch_joule_T(const Dev &d, const double *j, double *D, double *r, hipStream_t st)
{
    k_joule_vertices<<<nblocks(d.n_trees, 64), 64, 0, st>>>(d, j, D, r);
    k_joule_nodes<<<nblocks(d.ns), 256, 0, st>>>(d, j);
}
void launch_edge_static(const Dev &d, hipStream_t st)
{
    k_edge_static<<<nblocks(d.ns), 256, 0, st>>>(d);
}
void launch_node_V(const Dev &d, bool fp32, hipStream_t st)
{
    k_node_V<<<nblocks(d.ns), 256, 0, st>>>(d, fp32 ? 1 : 0);
    k_tree_V<<<nblocks(d.n_trees, 4), 256, 0, st>>>(d);
}
void launch_draws(const Dev &d, uint64_t seed, double cov_k, double cov_s, double cov_r, double cov_l,
                  double sd_ea, double sd_T, double cov_map, hipStream_t st)
{
    int use = (cov_k != 0.0 || cov_s != 0.0) ? 1 : 0;
    k_draws<<<nblocks((long long)d.n_res * d.S), 256, 0, st>>>(d, seed, cov_k, cov_s, cov_r, sd_ea, sd_T, cov_map,
                                                               use);
    if (d.sink_s) k_draws_load<<<nblocks((long long)d.n_nodes * d.S), 256, 0, st>>>(d, seed, cov_l);
}
// grid of one block row per node (rows beyond 65535 folded into z) and the
// samples along x
static dim3 node_rows_grid(const Dev &d, int bs)
{
    return dim3((unsigned)((d.S + bs - 1) / bs), (unsigned)std::min(d.ns, 65535),
                (unsigned)((d.ns + 65534) / 65535));
}
static int rows_bs(const Dev &d) { return d.S >= 256 ? 256 : d.S >= 128 ? 128 : 64; }

void launch_node_sc(const Dev &d, bool fp32, hipStream_t st)
{
    if (d.S >= 64) {
        const int bs = rows_bs(d);
        if (fp32) k_node_sc_rows<float><<<node_rows_grid(d, bs), bs, 0, st>>>(d);
        else k_node_sc_rows<double><<<node_rows_grid(d, bs), bs, 0, st>>>(d);
        return;
    }
    long long n = (long long)d.ns * d.S;
    if (fp32) k_node_sc<float><<<nblocks(n), 256, 0, st>>>(d);
    else k_node_sc<double><<<nblocks(n), 256, 0, st>>>(d);
}
void launch_update_f(const Dev &d, bool fp32, hipStream_t st)
{
    long long n = (long long)d.ns * d.S;
    transpose_j(d, st);
    if (fp32) k_update_f<float><<<nblocks(n), 256, 0, st>>>(d);
    else k_update_f<double><<<nblocks(n), 256, 0, st>>>(d);
}
void launch_factor(const Dev &d, bool fp32, hipStream_t st)
{
    int n = d.n_trees * d.S;
    if (fp32) k_factor<float><<<nblocks(n), 256, 0, st>>>(d);
    else k_factor<double><<<nblocks(n), 256, 0, st>>>(d);
}
void launch_screen(const Dev &d, bool apply, hipStream_t st)
{
    k_screen<<<nblocks((long long)d.n_trees * d.S, 4), 256, 0, st>>>(d, apply ? 1 : 0);
}
void launch_screen_shared(const Dev &d, bool apply, hipStream_t st)
{
    k_screen_ss0<<<nblocks((long long)d.n_trees, 4), 256, 0, st>>>(d);
    if (d.S >= 64) {
        const int bs = rows_bs(d);
        k_screen_bcast_rows<<<node_rows_grid(d, bs), bs, 0, st>>>(d);
    } else {
        k_screen_bcast_flat<<<nblocks((long long)d.ns * d.S), 256, 0, st>>>(d);
    }
    if (apply) k_screen_activate<<<nblocks((long long)d.n_trees * d.S), 256, 0, st>>>(d);
}
void launch_step(const Dev &d, bool fp32, int n_steps, int step0, hipStream_t st)
{
    int n = d.n_trees * d.S;
    if (fp32) k_step<float><<<nblocks(n), 256, 0, st>>>(d, n_steps, step0);
    else k_step<double><<<nblocks(n), 256, 0, st>>>(d, n_steps, step0);
}
// Workgroup size by the largest tree stepped: about four nodes or fewer per
// thread in each pass (the passes walk a thread's nodes one after another).
void launch_branch(const Dev &d, bool fp32, int n_br, int max_nodes, int n_steps, int step0, hipStream_t st)
{
    if (n_br <= 0) return;
    const int nb = n_br * d.S;
    if (max_nodes > 2048) {
        if (fp32) k_branch<float, 1024><<<nb, 1024, 0, st>>>(d, n_steps, step0);
        else k_branch<double, 1024><<<nb, 1024, 0, st>>>(d, n_steps, step0);
    } else {
        if (fp32) k_branch<float, 256><<<nb, 256, 0, st>>>(d, n_steps, step0);
        else k_branch<double, 256><<<nb, 256, 0, st>>>(d, n_steps, step0);
    }
}
void launch_void_dR(const Dev &d, hipStream_t st)
{
    k_void_dR<<<nblocks(d.n_trees * d.S), 256, 0, st>>>(d);
}
void launch_set_sigma_T(const Dev &d, bool fp32, hipStream_t st)
{
    long long n = (long long)d.ns * d.S;
    if (fp32) k_set_sigma_T<float><<<nblocks(n), 256, 0, st>>>(d);
    else k_set_sigma_T<double><<<nblocks(n), 256, 0, st>>>(d);
}
void launch_inject_void(const Dev &d, bool fp32, int sample, int tree, int node, hipStream_t st)
{
    if (fp32) k_inject_void<float><<<1, 64, 0, st>>>(d, sample, tree, node);
    else k_inject_void<double><<<1, 64, 0, st>>>(d, sample, tree, node);
}
void launch_copy_sigma(const Dev &d, bool fp32, int sample, double *buf, bool to_state, hipStream_t st)
{
    if (fp32) k_copy_col<float><<<nblocks(d.ns), 256, 0, st>>>(d, d.sigma, sample, buf, to_state);
    else k_copy_col<double><<<nblocks(d.ns), 256, 0, st>>>(d, d.sigma, sample, buf, to_state);
}
void launch_copy_node_col(const Dev &d, bool fp32, int which, int sample, double *buf, hipStream_t st)
{
    void *arr = which == 0 ? d.sc : d.dtf;
    if (fp32) k_copy_col<float><<<nblocks(d.ns), 256, 0, st>>>(d, arr, sample, buf, 0);
    else k_copy_col<double><<<nblocks(d.ns), 256, 0, st>>>(d, arr, sample, buf, 0);
}

void launch_tree_static(const Dev &d, hipStream_t st)
{
    k_tree_static<<<nblocks(d.n_trees), 256, 0, st>>>(d);
}
void launch_features(const Dev &d, float *X, bool candidates_only, bool psi_col0, hipStream_t st)
{
    k_features<<<d.n_trees * d.S, FB, 0, st>>>(d, X, candidates_only ? 1 : 0, psi_col0 ? 1 : 0);
}
void launch_reeval_features(const Dev &d, int n, float *X, const double *jhist, int k_now, double tol,
                            hipStream_t st)
{
    k_reeval_features<<<n, FB, 0, st>>>(d, n, X, jhist, k_now, tol);
}
void launch_yhat_min(const Dev &d, int n, const float *y, hipStream_t st)
{
    k_yhat_min<<<nblocks(n), 256, 0, st>>>(d, n, y);
}
void launch_defer(const Dev &d, const float *y, double thr, hipStream_t st)
{
    k_defer<<<nblocks(d.n_trees * d.S), 256, 0, st>>>(d, y, thr);
}
void launch_update_f_list(const Dev &d, bool fp32, const int *list, int n, hipStream_t st)
{
    if (n <= 0) return;
    transpose_j(d, st);
    if (fp32) k_update_f_list<float><<<n, 256, 0, st>>>(d, list);
    else k_update_f_list<double><<<n, 256, 0, st>>>(d, list);
}
void launch_activate(const Dev &d, double thr, hipStream_t st)
{
    k_activate<<<nblocks(d.n_trees * d.S), 256, 0, st>>>(d, thr);
}
void launch_catchup_done(const Dev &d, int step_lim, hipStream_t st)
{
    k_catchup_done<<<nblocks(d.n_trees * d.S), 256, 0, st>>>(d, step_lim);
}

// ---- chain-kernel lane table (built once per batch) ----
__global__ void k_fill_i32(int *p, long long n, int v)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) p[g] = v;
}

// one block per placed instance; its threads stride over the instance's lanes
__global__ void k_place_lanes(int *lane_inst, int *lane_blk, const int *inst, const long long *off,
                              const int *L)
{
    const int i = blockIdx.x;
    for (int k = threadIdx.x; k < L[i]; k += blockDim.x) {
        lane_inst[off[i] + k] = inst[i];
        lane_blk[off[i] + k] = k;
    }
}

void launch_place_lanes(int *lane_inst, int *lane_blk, long long n_lanes, const int *inst,
                        const long long *off, const int *L, int n_place, hipStream_t st)
{
    if (n_lanes > 0) k_fill_i32<<<(int)((n_lanes + 255) / 256), 256, 0, st>>>(lane_inst, n_lanes, -1);
    if (n_place > 0) k_place_lanes<<<n_place, 64, 0, st>>>(lane_inst, lane_blk, inst, off, L);
}

}  // namespace em
