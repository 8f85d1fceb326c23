// IR-drop solve (Sec. III-C, eq. 8): nodal analysis M u = P I of the resistor
// network with ideal VDD pads, batched over Monte Carlo samples.  Jacobi-
// preconditioned conjugate gradients in FP64 on the free nodes (live, not a
// pad); an open segment conducts nothing and a node with no conducting path
// to a pad reads 0 V.  Vectors are [S][node]; a block covers 256 nodes of one
// sample and per-sample dot products are reduced deterministically through
// per-block partials.  The time-to-failure bookkeeping of the outer loop
// (Fig. 2, Table I caption) lives here too.
#include "em_internal.h"
#include <algorithm>
#include <cmath>

namespace em {

#define IR_BS 256
#define IR_NPT 4                      // nodes per thread in the CG kernels
#define IR_NPB (IR_BS * IR_NPT)       // nodes per block
#define EM_KERNEL __global__ __launch_bounds__(IR_BS)

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum of up to 4 per-thread values over the block; thread 0 writes them to
// part[(s*nblk + bx)*4 + slot].
__device__ inline void block_partials(const Dev &d, int s, int bx, double v0, double v1, double v2,
                                      double v3, int mask)
{
    __shared__ double red[4][IR_BS / 64];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double v[4] = {v0, v1, v2, v3};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (!(mask & (1 << c))) continue;
        double x = wave_sum(v[c]);
        if (lane == 0) red[c][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *P = d.part + ((size_t)s * d.ir_nblk + bx) * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!(mask & (1 << c))) continue;
            double acc = 0.0;
            for (int w = 0; w < IR_BS / 64; ++w) acc += red[c][w];
            P[c] = acc;
        }
    }
}

// Deterministic sum of partial `slot` over all blocks of sample s, broadcast
// to every thread of the block.
__device__ inline double sum_partials(const Dev &d, int s, int slot)
{
    __shared__ double bc;
    if (threadIdx.x < 64) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < d.ir_nblk; b += 64)
            acc += d.part[((size_t)s * d.ir_nblk + b) * 4 + slot];
        acc = wave_sum(acc);
        if (threadIdx.x == 0) bc = acc;
    }
    __syncthreads();
    double r = bc;
    __syncthreads();
    return r;
}

__device__ inline bool is_free(const Dev &d, int s, int i)
{
    return d.live[(size_t)s * d.n_nodes + i] && !d.is_pad[i];
}

EM_KERNEL void k_ir_conductance(Dev d)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.S * d.n_res) return;
    int r = (int)(g % d.n_res);
    const double R0 = d.xi_r ? d.R0[r] * d.xi_r[(size_t)r * d.S + g / d.n_res] : d.R0[r];
    const double Gn = d.open[g] ? 0.0 : 1.0 / (R0 + d.dR[g]);
    if (Gn != d.G[g]) {
        d.G[g] = Gn;
        *d.g_changed = 1u;
        d.g_chg_s[g / d.n_res] = 1;
    }
}

// Conductance of every node-incidence entry, contiguous per node (SpMV rows).
EM_KERNEL void k_ir_gather_inc(Dev d)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int ninc = d.ninc_off[d.n_nodes];
    if (g >= (long long)d.S * ninc) return;
    int s = (int)(g / ninc), k = (int)(g % ninc);
    d.G_inc[g] = d.G[(size_t)s * d.n_res + d.ninc_res[k]];
}

EM_KERNEL void k_ir_live_copy(Dev d, const uint8_t *live0)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.S * d.n_nodes) return;
    d.live[g] = live0[g % d.n_nodes];
}

// Reachability from the pads as connected components of the conducting
// network (min-label hooking with pointer jumping): node i has index i + 1,
// index 0 stands for all pads; a node is live iff its final label is 0.
EM_KERNEL void k_ir_cc_init(Dev d)
{
    const long long n1 = d.n_nodes + 1;
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.S * n1) return;
    const int x = (int)(g % n1);
    d.cc_label[g] = (x == 0 || d.is_pad[x - 1]) ? 0 : x;
}

EM_KERNEL void k_ir_cc_hook(Dev d)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.S * d.n_res) return;
    const int s = (int)(g / d.n_res), e = (int)(g % d.n_res);
    if (!(d.G[g] > 0.0)) return;
    int *L = d.cc_label + (size_t)s * (d.n_nodes + 1);
    const int a = d.ra[e] + 1, b = d.rb[e] + 1;
    const int la = L[a], lb = L[b];
    if (la == lb) return;
    // any edge whose ends disagree keeps the rounds going: a round that
    // sees none has reached equal labels on every conducting component
    *d.live_changed = 1u;
    const int lo = min(la, lb), hi = max(la, lb);
    atomicMin(&L[hi], lo);
    atomicMin(&L[a], lo);
    atomicMin(&L[b], lo);
}

EM_KERNEL void k_ir_cc_jump(Dev d)
{
    const long long n1 = d.n_nodes + 1;
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.S * n1) return;
    int *L = d.cc_label + (g / n1) * n1;
    int x = L[g % n1];
    for (int k = 0; k < 32 && L[x] < x; ++k) x = L[x];
    L[g % n1] = x;
}

EM_KERNEL void k_ir_cc_finish(Dev d)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.S * d.n_nodes) return;
    const int s = (int)(g / d.n_nodes), i = (int)(g % d.n_nodes);
    d.live[g] = d.cc_label[(size_t)s * (d.n_nodes + 1) + i + 1] == 0 ? 1 : 0;
}

// Diagonal, right-hand side (sinks and pad injections), residual of the warm
// start, z = r/diag, p = z; partials r.z, r.r, b.b.
EM_KERNEL void k_ir_setup(Dev d)
{
    int s = blockIdx.y, bx = blockIdx.x;
    double rz = 0, rr = 0, bbv = 0;
    for (int c = 0; c < IR_NPT; ++c) {
        int i = bx * IR_NPB + c * IR_BS + threadIdx.x;
        if (i >= d.n_nodes) break;
        size_t x = (size_t)s * d.n_nodes + i;
        const double *G = d.G + (size_t)s * d.n_res;
        const double *u = d.u + (size_t)s * d.n_nodes;
        double dg = 0.0;
        for (int k = d.ninc_off[i]; k < d.ninc_off[i + 1]; ++k) dg += G[d.ninc_res[k]];
        d.diag[x] = dg;
        if (is_free(d, s, i)) {
            double b = -(d.sink_s ? d.sink_s[x] : d.sink[i]), Ax = dg * u[i];
            for (int k = d.ninc_off[i]; k < d.ninc_off[i + 1]; ++k) {
                int nb = d.ninc_nbr[k];
                double gk = G[d.ninc_res[k]];
                if (d.is_pad[nb]) b += gk * d.vdd;
                else if (is_free(d, s, nb)) Ax -= gk * u[nb];
            }
            double r = b - Ax, z = r / dg;
            d.rhs[x] = b; d.r[x] = r; d.z[x] = z; d.p[x] = z;
            rz += r * z; rr += r * r; bbv += b * b;
        } else {
            d.rhs[x] = 0; d.r[x] = 0; d.z[x] = 0; d.p[x] = 0;
        }
    }
    block_partials(d, s, bx, 0.0, rz, rr, bbv, 0xE);
}

EM_KERNEL void k_ir_finalize0(Dev d, double rtol)
{
    int s = blockIdx.x;
    double rz = sum_partials(d, s, 1);
    double rr = sum_partials(d, s, 2);
    double bb = sum_partials(d, s, 3);
    if (threadIdx.x == 0) {
        d.rz[s] = rz;
        d.bb[s] = bb;
        d.conv[s] = (!d.sample_active[s] || rr <= rtol * rtol * bb) ? 1 : 0;
    }
}

// q = A p on the free nodes; partial p.q.
EM_KERNEL void k_ir_spmv(Dev d)
{
    int s = blockIdx.y, bx = blockIdx.x;
    if (d.conv[s]) return;
    double pq = 0;
    for (int c = 0; c < IR_NPT; ++c) {
        int i = bx * IR_NPB + c * IR_BS + threadIdx.x;
        if (i >= d.n_nodes) break;
        size_t x = (size_t)s * d.n_nodes + i;
        double q = 0.0;
        if (is_free(d, s, i)) {
            // p vanishes on pads and dead nodes, so every neighbour can be summed
            const double *Gi = d.G_inc + (size_t)s * d.ninc_off[d.n_nodes];
            const double *p = d.p + (size_t)s * d.n_nodes;
            const double pi = p[i];
            q = d.diag[x] * pi;
            for (int k = d.ninc_off[i]; k < d.ninc_off[i + 1]; ++k) q -= Gi[k] * p[d.ninc_nbr[k]];
            pq += pi * q;
        }
        d.q[x] = q;
    }
    block_partials(d, s, bx, pq, 0.0, 0.0, 0.0, 0x1);
}

// alpha = (r.z)/(p.q) from the partials (every block sums them in the same
// order); x += alpha p, r -= alpha q, z = r/diag; partials r.z and r.r.
EM_KERNEL void k_ir_update(Dev d, int it, double amg_omega)
{
    int s = blockIdx.y, bx = blockIdx.x;
    if (d.conv[s]) return;
    const double pq = sum_partials(d, s, 0);
    const double alpha = pq > 0.0 ? d.rz[(it & 1) * d.S + s] / pq : 0.0;
    const bool amg = amg_omega > 0.0;
    double rz = 0, rr = 0;
    for (int c = 0; c < IR_NPT; ++c) {
        int i = bx * IR_NPB + c * IR_BS + threadIdx.x;
        if (i >= d.n_nodes) break;
        if (!is_free(d, s, i)) continue;
        size_t x = (size_t)s * d.n_nodes + i;
        d.u[x] += alpha * d.p[x];
        double r = d.r[x] - alpha * d.q[x];
        double z = (amg ? amg_omega * r : r) / d.diag[x];
        d.r[x] = r; d.z[x] = z;
        rz += r * z; rr += r * r;
    }
    block_partials(d, s, bx, 0.0, rz, rr, 0.0, amg ? 0x4 : 0x6);
}

// ---- multigrid V-cycle, level 0 (the free nodes of the nodal system) ----
// r.z of the preconditioned start of the not yet converged samples
EM_KERNEL void k_ir_finalize_rz(Dev d)
{
    int s = blockIdx.x;
    if (d.conv[s]) return;
    double rz = sum_partials(d, s, 1);
    if (threadIdx.x == 0) d.rz[s] = rz;
}

// z = omega r / diag (pre-smoothing from zero)
EM_KERNEL void k_amg_pre0(Dev d, double omega)
{
    int s = blockIdx.y, bx = blockIdx.x;
    if (d.conv[s]) return;
    for (int c = 0; c < IR_NPT; ++c) {
        int i = bx * IR_NPB + c * IR_BS + threadIdx.x;
        if (i >= d.n_nodes) break;
        size_t x = (size_t)s * d.n_nodes + i;
        d.z[x] = is_free(d, s, i) ? omega * d.r[x] / d.diag[x] : 0.0;
    }
}

// A v at free node i (v vanishes off the free nodes)
template <typename V>
__device__ inline double A0v(const Dev &d, int s, int i, const V *v)
{
    const double *Gi = d.G_inc + (size_t)s * d.ninc_off[d.n_nodes];
    double a = d.diag[(size_t)s * d.n_nodes + i] * (double)v[i];
    for (int k = d.ninc_off[i]; k < d.ninc_off[i + 1]; ++k) a -= Gi[k] * (double)v[d.ninc_nbr[k]];
    return a;
}

// w0 = r - A z (z the pre-smoothed vector)
EM_KERNEL void k_amg_res0(Dev d, mgreal *w0)
{
    int s = blockIdx.y, bx = blockIdx.x;
    if (d.conv[s]) return;
    const double *z = d.z + (size_t)s * d.n_nodes;
    for (int c = 0; c < IR_NPT; ++c) {
        int i = bx * IR_NPB + c * IR_BS + threadIdx.x;
        if (i >= d.n_nodes) break;
        size_t x = (size_t)s * d.n_nodes + i;
        w0[x] = is_free(d, s, i) ? d.r[x] - A0v(d, s, i, z) : 0.0;
    }
}

// w0 = z + alpha r1[agg] on the free nodes, 0 elsewhere (r1: level 1's result)
EM_KERNEL void k_amg_prolong0(Dev d, mgreal *w0, AmgLevel L1, const mgreal *r1, double alpha)
{
    int s = blockIdx.y, bx = blockIdx.x;
    if (d.conv[s]) return;
    for (int c = 0; c < IR_NPT; ++c) {
        int i = bx * IR_NPB + c * IR_BS + threadIdx.x;
        if (i >= d.n_nodes) break;
        size_t x = (size_t)s * d.n_nodes + i;
        int J = L1.agg[i];
        w0[x] = (is_free(d, s, i) && J >= 0) ? d.z[x] + alpha * (double)r1[(size_t)s * L1.n + J] : 0.0;
    }
}

// z = w0 + omega (r - A w0) / diag on the free nodes, 0 elsewhere; partial
// r.z; at the start of a solve also p = z
EM_KERNEL void k_amg_smooth0(Dev d, const mgreal *w0, double omega, int init)
{
    int s = blockIdx.y, bx = blockIdx.x;
    if (d.conv[s]) return;
    const mgreal *w = w0 + (size_t)s * d.n_nodes;
    double rz = 0.0;
    for (int c = 0; c < IR_NPT; ++c) {
        int i = bx * IR_NPB + c * IR_BS + threadIdx.x;
        if (i >= d.n_nodes) break;
        size_t x = (size_t)s * d.n_nodes + i;
        double z = 0.0;
        if (is_free(d, s, i)) {
            z = (double)w[i] + omega * (d.r[x] - A0v(d, s, i, w)) / d.diag[x];
            rz += d.r[x] * z;
        }
        d.z[x] = z;
        if (init) d.p[x] = z;
    }
    block_partials(d, s, bx, 0.0, rz, 0.0, 0.0, 0x2);
}

// beta = (new r.z)/(old r.z); p = z + beta p; convergence flag.
EM_KERNEL void k_ir_pupdate(Dev d, int it, double rtol, const double *zs)
{
    int s = blockIdx.y, bx = blockIdx.x;
    if (d.conv[s]) return;
    const double rz_new = sum_partials(d, s, 1);
    const double rr = sum_partials(d, s, 2);
    const double rz_old = d.rz[(it & 1) * d.S + s];
    const double beta = rz_old != 0.0 ? rz_new / rz_old : 0.0;
    for (int c = 0; c < IR_NPT; ++c) {
        int i = bx * IR_NPB + c * IR_BS + threadIdx.x;
        if (i >= d.n_nodes) break;
        if (!is_free(d, s, i)) continue;
        size_t x = (size_t)s * d.n_nodes + i;
        d.p[x] = zs[x] + beta * d.p[x];
    }
    if (bx == 0 && threadIdx.x == 0) {
        d.rz[((it + 1) & 1) * d.S + s] = rz_new;
        if (rr <= rtol * rtol * d.bb[s]) d.conv[s] = 1;
    }
}

// Fixed nodes, worst drop partials.
EM_KERNEL void k_ir_finish_nodes(Dev d)
{
    int s = blockIdx.y, bx = blockIdx.x;
    if (!d.g_chg_s[s]) return;              // voltages as at the last solve
    double dm = -INFINITY;
    for (int c = 0; c < IR_NPT; ++c) {
        int i = bx * IR_NPB + c * IR_BS + threadIdx.x;
        if (i >= d.n_nodes) break;
        size_t x = (size_t)s * d.n_nodes + i;
        if (d.is_pad[i]) d.u[x] = d.vdd;
        else if (!d.live[x]) d.u[x] = 0.0;
        dm = fmax(dm, (d.vdd - d.u[x]) / d.vdd);
    }
    __shared__ double red[IR_BS / 64];
    double m = wave_max(dm);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = red[0];
        for (int w = 1; w < IR_BS / 64; ++w) acc = fmax(acc, red[w]);
        d.part[((size_t)s * d.ir_nblk + bx) * 4 + 0] = acc;
    }
}

EM_KERNEL void k_ir_finalize_drop(Dev d)
{
    int s = blockIdx.x;
    if (!d.g_chg_s[s]) return;
    double m = -INFINITY;
    for (int b = threadIdx.x; b < d.ir_nblk; b += 64)
        m = fmax(m, d.part[((size_t)s * d.ir_nblk + b) * 4 + 0]);
    m = wave_max(m);
    if (threadIdx.x == 0) d.drop[s] = m;
}

// Branch currents and signed current densities along res_a -> res_b.
EM_KERNEL void k_ir_currents(Dev d)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long long)d.S * d.n_res) return;
    int s = (int)(g / d.n_res), r = (int)(g % d.n_res);
    if (!d.sample_active[s] || !d.g_chg_s[s]) return;
    const double *u = d.u + (size_t)s * d.n_nodes;
    double I = (u[d.ra[r]] - u[d.rb[r]]) * d.G[g];
    d.jseg[g] = I / (d.w[r] * d.h[r]);
}

// ---------------------------- TTF ----------------------------------------
EM_KERNEL void k_ttf_init(Dev d, double fail)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.S) return;
    double dr = d.drop[s];
    d.init_drop[s] = dr; d.final_drop[s] = dr;
    d.t_prev[s] = 0.0; d.d_prev[s] = dr;
    d.outer_idx[s] = 0;
    d.guard[s] = fabs(dr - fail) < d.guard_band * fail;
    if (dr >= fail) { d.failed[s] = 1; d.ttf[s] = 0.0; d.sample_active[s] = 0; }
    else { d.failed[s] = 0; d.ttf[s] = NAN; }
}

// After re-solve k at time t: failure when the worst drop reaches the
// threshold; TTF interpolates linearly between the bracketing re-solves.
EM_KERNEL void k_ttf_update(Dev d, double fail, int k, double t)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.S || !d.sample_active[s]) return;
    double dr = d.drop[s];
    d.final_drop[s] = dr;
    d.outer_idx[s] = k;
    if (fabs(dr - fail) < d.guard_band * fail) d.guard[s] = 1;
    if (dr >= fail) {
        double tp = d.t_prev[s], dp = d.d_prev[s];
        const double ttf = tp + (fail - dp) / (dr - dp) * (t - tp);
        d.ttf[s] = ttf;
        // a drop error of guard_band x fail at either re-solve moves the
        // interpolated time by about that over the bracket's drop increase
        if (d.guard_ttf > 0.0 && d.guard_band * fail * (t - tp) > d.guard_ttf * ttf * (dr - dp)) d.guard[s] = 1;
        d.failed[s] = 1;
        d.sample_active[s] = 0;
    } else {
        d.t_prev[s] = t;
        d.d_prev[s] = dr;
    }
}

EM_KERNEL void k_fill_f64(double *p, long long n, double v)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) p[g] = v;
}

// ---------------------------- launchers ---------------------------------
static inline int nb(long long n) { return (int)((n + IR_BS - 1) / IR_BS); }

void launch_ir_conductance(const Dev &d, hipStream_t st)
{
    k_ir_conductance<<<nb((long long)d.S * d.n_res), IR_BS, 0, st>>>(d);
}
void launch_ir_gather_inc(const Dev &d, int ninc, hipStream_t st)
{
    k_ir_gather_inc<<<nb((long long)d.S * ninc), IR_BS, 0, st>>>(d);
}
void launch_ir_live_copy(const Dev &d, const uint8_t *live0, hipStream_t st)
{
    long long n = (long long)d.S * d.n_nodes;
    k_ir_live_copy<<<(int)((n + IR_BS - 1) / IR_BS), IR_BS, 0, st>>>(d, live0);
}
void launch_ir_cc_init(const Dev &d, hipStream_t st)
{
    k_ir_cc_init<<<nb((long long)d.S * (d.n_nodes + 1)), IR_BS, 0, st>>>(d);
}
void launch_ir_cc_round(const Dev &d, hipStream_t st)
{
    k_ir_cc_hook<<<nb((long long)d.S * d.n_res), IR_BS, 0, st>>>(d);
    k_ir_cc_jump<<<nb((long long)d.S * (d.n_nodes + 1)), IR_BS, 0, st>>>(d);
}
void launch_ir_cc_finish(const Dev &d, hipStream_t st)
{
    k_ir_cc_finish<<<nb((long long)d.S * d.n_nodes), IR_BS, 0, st>>>(d);
}
void launch_ir_setup(const Dev &d, hipStream_t st)
{
    k_ir_setup<<<dim3(d.ir_nblk, d.S), IR_BS, 0, st>>>(d);
}
void launch_ir_finalize0(const Dev &d, double rtol, hipStream_t st)
{
    k_ir_finalize0<<<d.S, 64, 0, st>>>(d, rtol);
}
void launch_ir_spmv(const Dev &d, hipStream_t st)
{
    k_ir_spmv<<<dim3(d.ir_nblk, d.S), IR_BS, 0, st>>>(d);
}
void launch_ir_update(const Dev &d, int it, double amg_omega, hipStream_t st)
{
    k_ir_update<<<dim3(d.ir_nblk, d.S), IR_BS, 0, st>>>(d, it, amg_omega);
}
void launch_ir_finalize_rz(const Dev &d, hipStream_t st)
{
    k_ir_finalize_rz<<<d.S, 64, 0, st>>>(d);
}
void launch_amg_pre0(const Dev &d, double omega, hipStream_t st)
{
    k_amg_pre0<<<dim3(d.ir_nblk, d.S), IR_BS, 0, st>>>(d, omega);
}
void launch_amg_res0(const Dev &d, mgreal *w0, hipStream_t st)
{
    k_amg_res0<<<dim3(d.ir_nblk, d.S), IR_BS, 0, st>>>(d, w0);
}
void launch_amg_post0(const Dev &d, mgreal *w0, const AmgLevel &L1, const mgreal *r1, double alpha,
                      double omega, bool init, hipStream_t st)
{
    k_amg_prolong0<<<dim3(d.ir_nblk, d.S), IR_BS, 0, st>>>(d, w0, L1, r1, alpha);
    k_amg_smooth0<<<dim3(d.ir_nblk, d.S), IR_BS, 0, st>>>(d, w0, omega, init ? 1 : 0);
}
void launch_ir_pupdate(const Dev &d, int it, double rtol, const double *zs, hipStream_t st)
{
    k_ir_pupdate<<<dim3(d.ir_nblk, d.S), IR_BS, 0, st>>>(d, it, rtol, zs);
}
int ir_nodes_per_block() { return IR_NPB; }
void launch_ir_finish(const Dev &d, hipStream_t st)
{
    k_ir_finish_nodes<<<dim3(d.ir_nblk, d.S), IR_BS, 0, st>>>(d);
    k_ir_finalize_drop<<<d.S, 64, 0, st>>>(d);
    k_ir_currents<<<nb((long long)d.S * d.n_res), IR_BS, 0, st>>>(d);
}
void launch_fill_f64(double *p, size_t n, double v, hipStream_t st)
{
    k_fill_f64<<<nb((long long)n), IR_BS, 0, st>>>(p, (long long)n, v);
}
void launch_ttf_init(const Dev &d, double fail, hipStream_t st)
{
    k_ttf_init<<<nb(d.S), IR_BS, 0, st>>>(d, fail);
}
// All samples share the nominal network: only sample 0 iterates ...
EM_KERNEL void k_ir_only_sample0(Dev d)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= 1 && s < d.S) d.conv[s] = 1;
}
// ... and its per-sample IR state ([S][n] arrays) is every sample's.
template <typename T>
EM_KERNEL void k_bcast0(T *a, long long n, int S)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n || g >= n * S) return;
    a[g] = a[g % n];
}
void launch_ir_only_sample0(const Dev &d, hipStream_t st)
{
    k_ir_only_sample0<<<nb(d.S), IR_BS, 0, st>>>(d);
}
void launch_bcast0_f64(double *a, long long n, int S, hipStream_t st)
{
    if (n > 0 && S > 1) k_bcast0<double><<<nb(n * S), IR_BS, 0, st>>>(a, n, S);
}
void launch_bcast0_u8(uint8_t *a, long long n, int S, hipStream_t st)
{
    if (n > 0 && S > 1) k_bcast0<uint8_t><<<nb(n * S), IR_BS, 0, st>>>(a, n, S);
}

// Per-sample result counts (one block per sample): segments with a
// resistance change or open, and trees holding a void.
EM_KERNEL void k_result_counts(Dev d, int *cnt)
{
    const int s = blockIdx.y;
    int nf = 0, nt = 0;
    for (int e = blockIdx.x * IR_BS + threadIdx.x; e < d.n_res; e += gridDim.x * IR_BS) {
        const size_t x = (size_t)s * d.n_res + e;
        nf += (d.dR[x] > 0.0 || d.open[x]) ? 1 : 0;
    }
    for (int t = blockIdx.x * IR_BS + threadIdx.x; t < d.n_trees; t += gridDim.x * IR_BS)
        nt += d.nv[(size_t)t * d.S + s] > 0 ? 1 : 0;
    __shared__ int red[2][IR_BS / 64];
    for (int o = 32; o > 0; o >>= 1) { nf += __shfl_xor(nf, o, 64); nt += __shfl_xor(nt, o, 64); }
    if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = nf; red[1][threadIdx.x >> 6] = nt; }
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0, b = 0;
        for (int w = 0; w < IR_BS / 64; ++w) { a += red[0][w]; b += red[1][w]; }
        if (b) atomicAdd(&cnt[2 * s], b);
        if (a) atomicAdd(&cnt[2 * s + 1], a);
    }
}
void launch_result_counts(const Dev &d, int *cnt, hipStream_t st)
{
    // cnt zeroed by the caller; blocks per sample sized to the segment count
    const int bx = std::min(64, std::max(1, d.n_res / (8 * IR_BS)));
    k_result_counts<<<dim3(bx, d.S), IR_BS, 0, st>>>(d, cnt);
}
void launch_ttf_update(const Dev &d, double fail, int k, double t, hipStream_t st)
{
    k_ttf_update<<<nb(d.S), IR_BS, 0, st>>>(d, fail, k, t);
}

}  // namespace em
