// IR solve of small networks (Sec. II-C, eq. 8) with one workgroup per Monte
// Carlo sample: the whole preconditioned CG, multigrid V-cycle included, runs
// inside one launch, with workgroup barriers where the multi-kernel form ends
// a kernel.  The arithmetic is that of the multi-kernel form (same
// preconditioner, same stopping rule ||r|| <= rtol ||b|| per sample); only
// the reduction order of the dot products differs.
//
// Why: a Monte Carlo re-solve moves only the samples whose conductances
// changed, often a few dozen of a thousand, and the multi-kernel form then
// pays about two dozen launches per iteration for little work each.  Here a
// sample's iterations cost barriers, and samples that are already converged
// cost one early-exiting workgroup.  Per-sample vectors are contiguous
// ([S][n] layout), so a workgroup streams its own slices; the index arrays
// of the network and the hierarchy are shared by every sample and stay in
// the L2 of each XCD.
#include "em_internal.h"

namespace em {

#define WG_BS 1024

__device__ inline double wg_wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup, returned to every thread (fixed summation order).
__device__ inline double wg_sum(double v, double *red)
{
    v = wg_wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < WG_BS / 64; ++k) acc += red[k];
    __syncthreads();
    return acc;
}

struct WgSample {                       // one sample's level-0 slices
    int n;
    const uint8_t *live, *is_pad;
    const int *off, *nbr;
    const double *G, *D;                // incidence conductances, diagonal
    __device__ bool free_(int i) const { return live[i] && !is_pad[i]; }
    // (A v)_i at a free node (v vanishes off the free nodes)
    __device__ double Av(int i, const double *v) const
    {
        double a = D[i] * v[i];
        for (int k = off[i]; k < off[i + 1]; ++k) a -= G[k] * v[nbr[k]];
        return a;
    }
};

__device__ inline double lev_Av(const AmgLevel &L, int s, int I, const double *v)
{
    const double *W = L.W + (size_t)s * L.ne;
    double a = L.D[(size_t)s * L.n + I] * v[I];
    for (int k = L.adj_off[I]; k < L.adj_off[I + 1]; ++k) a -= W[L.adj_e[k]] * v[L.adj_nbr[k]];
    return a;
}

// z = M^-1 r by one V-cycle; returns r.z (every thread).  When p is given it
// also receives z (start of a solve).
__device__ double wg_vcycle(const WgSample &S0, const Amg &a, int s, const double *r, double *z,
                            double *w0, double *p, double *red)
{
    const int T = threadIdx.x, n = S0.n, nl = a.nlev;
    const double om = a.omega, al = a.alpha;
    // pre-smoothing from zero
    for (int i = T; i < n; i += WG_BS) z[i] = S0.free_(i) ? om * r[i] / S0.D[i] : 0.0;
    __syncthreads();
    for (int i = T; i < n; i += WG_BS) w0[i] = S0.free_(i) ? r[i] - S0.Av(i, z) : 0.0;
    __syncthreads();
    // down: restriction by member sums, pre-smoothing, residual
    for (int l = 1; l <= nl; ++l) {
        const AmgLevel &L = a.lev[l];
        const double *wf = l == 1 ? w0 : a.lev[l - 1].w + (size_t)s * a.lev[l - 1].n;
        double *b = L.b + (size_t)s * L.n, *x = L.x + (size_t)s * L.n;
        const double *D = L.D + (size_t)s * L.n;
        for (int I = T; I < L.n; I += WG_BS) {
            double acc = 0.0;
            for (int k = L.mem_off[I]; k < L.mem_off[I + 1]; ++k) acc += wf[L.mem[k]];
            b[I] = acc;
            x[I] = om * acc / D[I];
        }
        __syncthreads();
        if (l < nl) {
            double *w = L.w + (size_t)s * L.n;
            for (int I = T; I < L.n; I += WG_BS) w[I] = b[I] - lev_Av(L, s, I, x);
            __syncthreads();
        }
    }
    // coarsest level
    {
        const AmgLevel &C = a.lev[nl];
        const int nc = C.n;
        const double *b = C.b + (size_t)s * nc;
        double *x = C.x + (size_t)s * nc;
        const double *D = C.D + (size_t)s * nc;
        for (int i = T; i < nc; i += WG_BS) {
            double v;
            if (a.dense) {
                const double *row = a.Ainv + ((size_t)s * nc + i) * nc;
                v = 0.0;
                for (int j = 0; j < nc; ++j) v += row[j] * b[j];
            } else {
                v = b[i] / D[i];
            }
            x[i] = v;
        }
        __syncthreads();
    }
    // up: prolongation of the coarse result, post-smoothing
    for (int l = nl - 1; l >= 1; --l) {
        const AmgLevel &L = a.lev[l], &C = a.lev[l + 1];
        const double *rc = (l + 1 == nl ? C.x : C.y) + (size_t)s * C.n;
        const double *xl = L.x + (size_t)s * L.n, *W = L.W + (size_t)s * L.ne;
        const double *b = L.b + (size_t)s * L.n, *D = L.D + (size_t)s * L.n;
        double *y = L.y + (size_t)s * L.n;
        for (int I = T; I < L.n; I += WG_BS) {
            auto yv = [&](int J) {
                const int K = C.agg[J];
                return xl[J] + (K >= 0 ? al * rc[K] : 0.0);
            };
            const double yi = yv(I), Dd = D[I];
            double acc = Dd * yi;
            for (int k = L.adj_off[I]; k < L.adj_off[I + 1]; ++k) acc -= W[L.adj_e[k]] * yv(L.adj_nbr[k]);
            y[I] = yi + om * (b[I] - acc) / Dd;
        }
        __syncthreads();
    }
    // level 0: w0 = z0 + alpha P y1, then z = w0 + omega (r - A w0) / D
    {
        const AmgLevel &L1 = a.lev[1];
        const double *r1 = (nl == 1 ? L1.x : L1.y) + (size_t)s * L1.n;
        for (int i = T; i < n; i += WG_BS) {
            const int J = L1.agg[i];
            w0[i] = (S0.free_(i) && J >= 0) ? z[i] + al * r1[J] : 0.0;
        }
        __syncthreads();
    }
    double rz = 0.0;
    for (int i = T; i < n; i += WG_BS) {
        double zi = 0.0;
        if (S0.free_(i)) {
            zi = w0[i] + om * (r[i] - S0.Av(i, w0)) / S0.D[i];
            rz += r[i] * zi;
        }
        z[i] = zi;
        if (p) p[i] = zi;
    }
    return wg_sum(rz, red);     // its barriers also publish z (and p)
}

// PCG of the samples not yet converged (conv[s] == 0), from the residual,
// diagonal and incidence conductances of the solve's set-up; iters[s]
// receives the iteration count, conv[s] 1 once ||r||^2 <= rtol^2 ||b||^2.
__global__ __launch_bounds__(WG_BS, 8) void k_ir_pcg_wg(Dev d, const Amg *__restrict__ ap, double rtol,
                                                    int max_iter)
{
    __shared__ double red[2 * (WG_BS / 64)];
    const int s = blockIdx.x, T = threadIdx.x;
    if (d.conv[s]) {
        if (T == 0) d.ir_iters[s] = 0;
        return;
    }
    const Amg &a = *ap;
    const int n = d.n_nodes;
    const size_t o = (size_t)s * n;
    WgSample S0;
    S0.n = n;
    S0.live = d.live + o;
    S0.is_pad = d.is_pad;
    S0.off = d.ninc_off;
    S0.nbr = d.ninc_nbr;
    S0.G = d.G_inc + (size_t)s * d.ninc_off[n];
    S0.D = d.diag + o;
    double *u = d.u + o, *r = d.r + o, *z = d.z + o, *p = d.p + o, *q = d.q + o;
    double *w0 = a.l0.w0 + o;
    const double bb = d.bb[s], tol2 = rtol * rtol * bb;
    double rz = wg_vcycle(S0, a, s, r, z, w0, p, red);
    int it = 0;
    bool done = false;
    while (it < max_iter) {
        double pq = 0.0;
        for (int i = T; i < n; i += WG_BS) {
            double qi = 0.0;
            if (S0.free_(i)) {
                qi = S0.Av(i, p);
                pq += p[i] * qi;
            }
            q[i] = qi;
        }
        pq = wg_sum(pq, red);
        const double alpha = pq > 0.0 ? rz / pq : 0.0;
        double rr = 0.0;
        for (int i = T; i < n; i += WG_BS) {
            if (!S0.free_(i)) continue;
            u[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            rr += ri * ri;
        }
        rr = wg_sum(rr, red);
        ++it;
        if (rr <= tol2) { done = true; break; }
        const double rz_new = wg_vcycle(S0, a, s, r, z, w0, nullptr, red);
        const double beta = rz != 0.0 ? rz_new / rz : 0.0;
        rz = rz_new;
        for (int i = T; i < n; i += WG_BS)
            if (S0.free_(i)) p[i] = z[i] + beta * p[i];
        __syncthreads();
    }
    if (T == 0) {
        d.ir_iters[s] = it;
        d.conv[s] = done ? 1 : 0;
    }
}

int ir_wg_max_nodes() { return 1 << 16; }

void launch_ir_pcg_wg(const Dev &d, const Amg *amg_dev, double rtol, int max_iter, hipStream_t st)
{
    k_ir_pcg_wg<<<d.S, WG_BS, 0, st>>>(d, amg_dev, rtol, max_iter);
}

}  // namespace em
