// Chain condensation of the IR network (exact Schur complement of the nodal
// system of Sec. III-C, eq. 8, onto its terminal nodes).
//
// A node that is not a pad and has one or two incident resistors carries no
// branching: the interior of a wire between vias is a chain of such nodes.
// Terminals are the pads and every node of another degree.  Each chain runs
// from a terminal A through interior nodes v_1..v_m to a terminal B, or ends
// at a leaf (dangling).  With the terminal voltages fixed, a chain is a series
// resistor ladder with current sinks at its interior nodes, solved in closed
// form:
//   * all of its resistors conduct and it has two ends: it couples A and B by
//     the series conductance 1 / R_tot, and the sink I_j at resistance P_j
//     from A draws I_j (R_tot - P_j) / R_tot from A and I_j P_j / R_tot from
//     B (current divider);
//   * otherwise the nodes before the first open resistor hang from A, those
//     after the last open one from B, each piece drawing its sinks from its
//     terminal, and nodes between two opens (or past the open or leaf end of
//     a dangling chain) are cut off from every pad.
// The condensed system on the non-pad terminals (reduced edges = two-ended
// chains between distinct terminals, sinks = own sink plus the chain draws)
// is solved by the same PCG; interior voltages then follow by walking each
// chain: from A, u_j = u_A + (u_B - u_A) P_j / R_tot - sum_{k<j} R_k i_k with
// i_k the ladder current of the sinks alone, or by the drop along a piece
// towards its terminal.  On the P/G grids most nodes are interior (a via
// every few dozen nodes), so the iterated system is many times smaller and
// better conditioned than the nodal one.
#include "em_internal.h"

#include <algorithm>

namespace em {

// ------------------------------------------------------------------------
// host: chains and terminals
// ------------------------------------------------------------------------
CondHost cond_build(int nn, int nr, const int *ra, const int *rb, const double *R0, const uint8_t *is_pad)
{
    CondHost H;
    std::vector<int> deg(nn, 0), off(nn + 1, 0), inc;
    for (int e = 0; e < nr; ++e) { deg[ra[e]]++; deg[rb[e]]++; }
    for (int v = 0; v < nn; ++v) off[v + 1] = off[v] + deg[v];
    inc.assign(off[nn], 0);
    {
        std::vector<int> pos(off.begin(), off.end() - 1);
        for (int e = 0; e < nr; ++e) { inc[pos[ra[e]]++] = e; inc[pos[rb[e]]++] = e; }
    }
    std::vector<char> term(nn, 0), used(nr, 0);
    H.tid.assign(nn, -1);
    auto add_term = [&](int v) {
        term[v] = 1;
        H.tid[v] = (int)H.term_node.size();
        H.term_node.push_back(v);
    };
    for (int v = 0; v < nn; ++v)
        if (is_pad[v] || (deg[v] != 1 && deg[v] != 2)) add_term(v);
    H.eoff.push_back(0);
    H.voff.push_back(0);
    auto walk = [&](int t, int e0) {
        H.cA.push_back(H.tid[t]);
        used[e0] = 1;
        H.e.push_back(e0);
        int prev = e0, cur = ra[e0] == t ? rb[e0] : ra[e0], B = -1;
        for (;;) {
            if (term[cur]) { B = H.tid[cur]; break; }
            H.v.push_back(cur);
            if (deg[cur] == 1) break;                       // leaf: dangling chain
            const int e1 = inc[off[cur]], e2 = inc[off[cur] + 1];
            const int nx = e1 == prev ? e2 : e1;
            if (nx == prev || used[nx]) break;             // cannot occur on a valid netlist
            used[nx] = 1;
            H.e.push_back(nx);
            prev = nx;
            cur = ra[nx] == cur ? rb[nx] : ra[nx];
        }
        H.cB.push_back(B);
        H.eoff.push_back((int)H.e.size());
        H.voff.push_back((int)H.v.size());
    };
    for (size_t q = 0; q < H.term_node.size(); ++q) {
        const int t = H.term_node[q];
        for (int k = off[t]; k < off[t + 1]; ++k)
            if (!used[inc[k]]) walk(t, inc[k]);
    }
    // closed rings of interior nodes reach no terminal: one of their nodes
    // becomes a terminal (with no path to a pad)
    for (int e = 0; e < nr; ++e) {
        if (used[e]) continue;
        const int x = ra[e];
        add_term(x);
        for (int k = off[x]; k < off[x + 1]; ++k)
            if (!used[inc[k]]) walk(x, inc[k]);
    }
    H.n_term = (int)H.term_node.size();
    H.n_chain = (int)H.cA.size();
    H.cred.assign(H.n_chain, -1);
    for (int c = 0; c < H.n_chain; ++c) {
        if (H.cB[c] < 0 || H.cB[c] == H.cA[c]) continue;
        H.cred[c] = (int)H.red_a.size();
        H.red_a.push_back(H.cA[c]);
        H.red_b.push_back(H.cB[c]);
        double R = 0.0;
        for (int k = H.eoff[c]; k < H.eoff[c + 1]; ++k) R += R0[H.e[k]];
        H.red_R0.push_back(R);
    }
    H.red_pad.assign(H.n_term, 0);
    for (int t = 0; t < H.n_term; ++t) H.red_pad[t] = is_pad[H.term_node[t]];
    H.tce_off.assign(H.n_term + 1, 0);
    for (int c = 0; c < H.n_chain; ++c) {
        H.tce_off[H.cA[c] + 1]++;
        if (H.cB[c] >= 0) H.tce_off[H.cB[c] + 1]++;
    }
    for (int t = 0; t < H.n_term; ++t) H.tce_off[t + 1] += H.tce_off[t];
    H.tce.assign(H.tce_off[H.n_term], 0);
    {
        std::vector<int> pos(H.tce_off.begin(), H.tce_off.end() - 1);
        for (int c = 0; c < H.n_chain; ++c) {
            H.tce[pos[H.cA[c]]++] = 2 * c;
            if (H.cB[c] >= 0) H.tce[pos[H.cB[c]]++] = 2 * c + 1;
        }
    }
    return H;
}

// ------------------------------------------------------------------------
// device
// ------------------------------------------------------------------------
#define CH_BS 256

static inline int cnb(long long n) { return (int)((n + CH_BS - 1) / CH_BS); }

// First and last open resistor of a chain (-1: none) and the series
// resistance of its conducting resistors.
__device__ inline void chain_scan(const Cond &c, const double *G, int ch, int &k1, int &k2, double &Rt)
{
    const int e0 = c.eoff[ch], K = c.eoff[ch + 1] - e0;
    k1 = -1; k2 = -1; Rt = 0.0;
    for (int k = 0; k < K; ++k) {
        const double g = G[c.e[e0 + k]];
        if (g > 0.0) Rt += 1.0 / g;
        else { if (k1 < 0) k1 = k; k2 = k; }
    }
}

// Sink current of node x in sample s (per-sample under loading variation).
__device__ inline double sink_at(const Dev &d, int s, int x)
{
    return d.sink_s ? d.sink_s[(size_t)s * d.n_nodes + x] : d.sink[x];
}

// Per (chain, sample): reduced-edge conductance and the currents the chain
// draws from its two terminals.
__global__ __launch_bounds__(CH_BS) void k_chain_reduce(Dev d, Dev r, Cond c)
{
    long long g = (long long)blockIdx.x * CH_BS + threadIdx.x;
    if (g >= (long long)d.S * c.n_chain) return;
    const int s = (int)(g / c.n_chain), ch = (int)(g % c.n_chain);
    if (!d.sample_active[s] || !d.g_chg_s[s]) return;    // unchanged: as at the last solve
    const double *G = d.G + (size_t)s * d.n_res;
    const int e0 = c.eoff[ch], v0 = c.voff[ch], m = c.voff[ch + 1] - v0;
    const bool two = c.cB[ch] >= 0;
    int k1, k2;
    double Rt;
    chain_scan(c, G, ch, k1, k2, Rt);
    double IA = 0.0, IB = 0.0, geq = 0.0;
    if (two && k1 < 0) {
        double P = 0.0;
        for (int j = 1; j <= m; ++j) {
            P += 1.0 / G[c.e[e0 + j - 1]];
            const double I = sink_at(d, s, c.v[v0 + j - 1]);
            IA += I * (Rt - P);
            IB += I * P;
        }
        IA /= Rt;
        IB /= Rt;
        geq = 1.0 / Rt;
    } else {
        const int a_end = (!two && k1 < 0) ? m : k1;      // nodes 1..a_end hang from A
        for (int j = 1; j <= a_end; ++j) IA += sink_at(d, s, c.v[v0 + j - 1]);
        if (two)
            for (int j = k2 + 1; j <= m; ++j) IB += sink_at(d, s, c.v[v0 + j - 1]);
    }
    if (c.cred[ch] >= 0) r.G[(size_t)s * r.n_res + c.cred[ch]] = geq;
    c.cinj[((size_t)s * c.n_chain + ch) * 2 + 0] = IA;
    c.cinj[((size_t)s * c.n_chain + ch) * 2 + 1] = IB;
}

// Per (terminal, sample): own sink plus the draws of the chains ending there;
// the warm start of the condensed solve is the terminal's present voltage.
__global__ __launch_bounds__(CH_BS) void k_red_assemble(Dev d, Dev r, Cond c)
{
    long long g = (long long)blockIdx.x * CH_BS + threadIdx.x;
    if (g >= (long long)d.S * c.n_term) return;
    const int s = (int)(g / c.n_term), t = (int)(g % c.n_term);
    if (!d.g_chg_s[s]) return;
    const int node = c.term_node[t];
    double acc = sink_at(d, s, node);
    const double *ci = c.cinj + (size_t)s * c.n_chain * 2;
    for (int k = c.tce_off[t]; k < c.tce_off[t + 1]; ++k) acc += ci[c.tce[k]];
    r.sink_s[g] = acc;
    r.u[g] = d.u[(size_t)s * d.n_nodes + node];
}

// Terminal voltages and reachability back into the nodal arrays (pads at
// VDD, terminals without a path to a pad at 0 V).
__global__ __launch_bounds__(CH_BS) void k_red_scatter(Dev d, Dev r, Cond c)
{
    long long g = (long long)blockIdx.x * CH_BS + threadIdx.x;
    if (g >= (long long)d.S * c.n_term) return;
    const int s = (int)(g / c.n_term), t = (int)(g % c.n_term);
    if (!d.sample_active[s] || !d.g_chg_s[s]) return;    // unchanged: as at the last solve
    const size_t x = (size_t)s * d.n_nodes + c.term_node[t];
    const bool pad = r.is_pad[t], live = pad || r.live[g];
    d.u[x] = pad ? d.vdd : (live ? r.u[g] : 0.0);
    d.live[x] = live ? 1 : 0;
}

// Per (chain, sample): interior voltages and reachability from the terminal
// voltages (after the scatter).
__global__ __launch_bounds__(CH_BS) void k_chain_backsub(Dev d, Cond c)
{
    long long g = (long long)blockIdx.x * CH_BS + threadIdx.x;
    if (g >= (long long)d.S * c.n_chain) return;
    const int s = (int)(g / c.n_chain), ch = (int)(g % c.n_chain);
    if (!d.sample_active[s] || !d.g_chg_s[s]) return;    // unchanged: as at the last solve
    const double *G = d.G + (size_t)s * d.n_res;
    double *u = d.u + (size_t)s * d.n_nodes;
    uint8_t *live = d.live + (size_t)s * d.n_nodes;
    const int e0 = c.eoff[ch], v0 = c.voff[ch], m = c.voff[ch + 1] - v0;
    const bool two = c.cB[ch] >= 0;
    const int nA = c.term_node[c.cA[ch]], nB = two ? c.term_node[c.cB[ch]] : -1;
    const double uA = u[nA], uB = two ? u[nB] : 0.0;
    const bool lA = live[nA], lB = two && live[nB];
    const double IA = c.cinj[((size_t)s * c.n_chain + ch) * 2 + 0];
    const double IB = c.cinj[((size_t)s * c.n_chain + ch) * 2 + 1];
    int k1, k2;
    double Rt;
    chain_scan(c, G, ch, k1, k2, Rt);
    if (two && k1 < 0) {
        const bool lv = lA || lB;
        double P = 0.0, vj = 0.0, i = IA;
        for (int j = 1; j <= m; ++j) {
            const double R = 1.0 / G[c.e[e0 + j - 1]];
            P += R;
            vj -= R * i;
            const int x = c.v[v0 + j - 1];
            u[x] = lv ? uA + (uB - uA) * (P / Rt) + vj : 0.0;
            live[x] = lv ? 1 : 0;
            i -= sink_at(d, s, x);
        }
        return;
    }
    const int a_end = (!two && k1 < 0) ? m : k1;
    {
        double uj = uA, i = IA;
        for (int j = 1; j <= a_end; ++j) {
            uj -= (1.0 / G[c.e[e0 + j - 1]]) * i;
            const int x = c.v[v0 + j - 1];
            u[x] = lA ? uj : 0.0;
            live[x] = lA ? 1 : 0;
            i -= sink_at(d, s, x);
        }
    }
    const int b_start = two ? k2 + 1 : m + 1;             // nodes b_start..m hang from B
    for (int j = a_end + 1; j < b_start; ++j) {
        const int x = c.v[v0 + j - 1];
        u[x] = 0.0;
        live[x] = 0;
    }
    if (two) {
        double uj = uB, i = IB;
        for (int j = m; j >= b_start; --j) {
            uj -= (1.0 / G[c.e[e0 + j]]) * i;
            const int x = c.v[v0 + j - 1];
            u[x] = lB ? uj : 0.0;
            live[x] = lB ? 1 : 0;
            i -= sink_at(d, s, x);
        }
    }
}

void launch_chain_reduce(const Dev &d, const Dev &r, const Cond &c, hipStream_t st)
{
    if (c.n_chain > 0)
        k_chain_reduce<<<cnb((long long)d.S * c.n_chain), CH_BS, 0, st>>>(d, r, c);
    k_red_assemble<<<cnb((long long)d.S * c.n_term), CH_BS, 0, st>>>(d, r, c);
}

void launch_chain_expand(const Dev &d, const Dev &r, const Cond &c, hipStream_t st)
{
    k_red_scatter<<<cnb((long long)d.S * c.n_term), CH_BS, 0, st>>>(d, r, c);
    if (c.n_chain > 0)
        k_chain_backsub<<<cnb((long long)d.S * c.n_chain), CH_BS, 0, st>>>(d, c);
}

}  // namespace em
