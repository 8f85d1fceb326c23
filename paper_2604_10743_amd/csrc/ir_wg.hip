// IR solve of small systems (Sec. III-C, eq. 8) with one workgroup per Monte
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
// cost one early-exiting workgroup.
//
// Two forms share the code below through views of a sample's arrays:
//   * global: the vectors stay in the [S][n] arrays in HBM (any size);
//   * LDS-resident: when the sample's system, its hierarchy and the coarsest
//     inverse fit the LDS of one workgroup, they are loaded once, the PCG
//     runs from LDS, and only the voltages are written back.  On the chain-
//     condensed P/G grids (a few hundred terminals per sample) this removes
//     the global-memory latency that bounds the other form.
#include "em_internal.h"

namespace em {

__device__ inline double wg_wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup, returned to every thread (fixed summation order).
// The wavefront partials alternate between two halves of the buffer from
// call to call, so one barrier per call suffices: a half is written again
// only after every thread has passed the next call's barrier, that is after
// it read the half.  Every thread makes the same sequence of calls.
struct WgRed {
    double *buf;                        // 2 * (BS / 64) doubles
    int par;
};
template <int BS>
__device__ inline double wg_sum(double v, WgRed &red)
{
    v = wg_wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double *b = red.buf + red.par * (BS / 64);
    red.par ^= 1;
    if (lane == 0) b[w] = v;
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < BS / 64; ++k) acc += b[k];
    return acc;
}

struct L0View {                         // level 0 (the iterated system) of one sample
    int n;
    const int *off, *nbr;
    const double *G, *D;                // incidence conductances, diagonal
    const uint8_t *fr;                  // free flags (LDS form), or null: live and not a pad
    const uint8_t *live, *is_pad;
    double *u, *r, *z, *p, *q;
    mgreal *w0;
    __device__ bool free_(int i) const { return fr ? fr[i] != 0 : (live[i] && !is_pad[i]); }
    // (A v)_i at a free node (v vanishes off the free nodes)
    template <typename V>
    __device__ double Av(int i, const V *v) const
    {
        double a = D[i] * (double)v[i];
        for (int k = off[i]; k < off[i + 1]; ++k) a -= G[k] * (double)v[nbr[k]];
        return a;
    }
};

struct LView {                          // coarse level l >= 1 of one sample
    int n;
    const int *agg, *mem_off, *mem, *adj_off, *adj_nbr;
    const mgreal *D, *Wa;               // diagonal; conductance of each adjacency entry
    mgreal *b, *x, *y, *w;
    __device__ double Av(int I, const mgreal *v) const
    {
        double a = (double)D[I] * (double)v[I];
        for (int k = adj_off[I]; k < adj_off[I + 1]; ++k) a -= (double)Wa[k] * (double)v[adj_nbr[k]];
        return a;
    }
};

// Level views straight from the [S][n] arrays of the hierarchy.
struct GlobalLevels {
    const Amg *a;
    int s;
    __device__ LView lev(int l) const
    {
        const AmgLevel &L = a->lev[l];
        const size_t o = (size_t)s * L.n;
        return LView{L.n, L.agg, L.mem_off, L.mem, L.adj_off, L.adj_nbr,
                     L.D + o, L.Wa + (size_t)s * 2 * L.ne, L.b + o, L.x + o, L.y + o, L.w + o};
    }
    __device__ const mgreal *Ainv() const
    {
        const size_t nc = a->lev[a->nlev].n;
        return a->Ainv + (size_t)s * nc * nc;
    }
};

// Byte offsets of everything the LDS form keeps in shared memory.
struct LdsLayout {
    int bytes;
    int off, nbr, G, D, fr, u, r, z, p, q, w0;
    int agg[AMG_MAXLEV + 1], mem_off[AMG_MAXLEV + 1], mem[AMG_MAXLEV + 1], adj_off[AMG_MAXLEV + 1],
        adj_nbr[AMG_MAXLEV + 1], LD[AMG_MAXLEV + 1], LWa[AMG_MAXLEV + 1],
        b[AMG_MAXLEV + 1], x[AMG_MAXLEV + 1], y[AMG_MAXLEV + 1], w[AMG_MAXLEV + 1];
    int Ainv;
};

struct LdsLevels {
    char *sm;
    const LdsLayout *ly;
    const Amg *a;
    __device__ LView lev(int l) const
    {
        const LdsLayout &y = *ly;
        return LView{a->lev[l].n, (const int *)(sm + y.agg[l]), (const int *)(sm + y.mem_off[l]),
                     (const int *)(sm + y.mem[l]), (const int *)(sm + y.adj_off[l]),
                     (const int *)(sm + y.adj_nbr[l]),
                     (const mgreal *)(sm + y.LD[l]), (const mgreal *)(sm + y.LWa[l]),
                     (mgreal *)(sm + y.b[l]), (mgreal *)(sm + y.x[l]), (mgreal *)(sm + y.y[l]),
                     (mgreal *)(sm + y.w[l])};
    }
    __device__ const mgreal *Ainv() const { return (const mgreal *)(sm + ly->Ainv); }
};

// z = M^-1 r by one V-cycle; returns r.z (every thread).  When setp is set
// p also receives z (start of a solve).
template <int BS, class Lev>
__device__ double wg_vcycle(const L0View &S0, const Amg &a, const Lev &lv, bool setp, WgRed &red)
{
    const int T = threadIdx.x, n = S0.n, nl = a.nlev;
    const double om = a.omega, al = a.alpha;
    const double *r = S0.r;
    double *z = S0.z;
    mgreal *w0 = S0.w0;
    // pre-smoothing from zero
    for (int i = T; i < n; i += BS) z[i] = S0.free_(i) ? om * r[i] / S0.D[i] : 0.0;
    __syncthreads();
    for (int i = T; i < n; i += BS) w0[i] = S0.free_(i) ? r[i] - S0.Av(i, z) : 0.0;
    __syncthreads();
    // down: restriction by member sums, pre-smoothing, residual
    const mgreal *wf = w0;
    for (int l = 1; l <= nl; ++l) {
        const LView L = lv.lev(l);
        for (int I = T; I < L.n; I += BS) {
            double acc = 0.0;
            for (int k = L.mem_off[I]; k < L.mem_off[I + 1]; ++k) acc += wf[L.mem[k]];
            L.b[I] = acc;
            L.x[I] = om * acc / (double)L.D[I];
        }
        __syncthreads();
        if (l < nl) {
            for (int I = T; I < L.n; I += BS) L.w[I] = L.b[I] - L.Av(I, L.x);
            __syncthreads();
            wf = L.w;
        }
    }
    // coarsest level
    {
        const LView C = lv.lev(nl);
        const mgreal *Ai = a.dense ? lv.Ainv() : nullptr;
        if (Ai) {
            // eight lanes per row (aligned groups of one wavefront, active or
            // idle together), each a strided part of the row's dot product
            constexpr int TPR = 8;
            for (int idx = T; idx < C.n * TPR; idx += BS) {
                const int i = idx / TPR, part = idx - i * TPR;
                const mgreal *row = Ai + (size_t)i * C.n;
                double v = 0.0;
                for (int j = part; j < C.n; j += TPR) v += (double)row[j] * (double)C.b[j];
                v += __shfl_xor(v, 4, 64);
                v += __shfl_xor(v, 2, 64);
                v += __shfl_xor(v, 1, 64);
                if (part == 0) C.x[i] = v;
            }
        } else {
            for (int i = T; i < C.n; i += BS) C.x[i] = (double)C.b[i] / (double)C.D[i];
        }
        __syncthreads();
    }
    // up: prolongation of the coarse result, post-smoothing
    for (int l = nl - 1; l >= 1; --l) {
        const LView L = lv.lev(l), C = lv.lev(l + 1);
        const mgreal *rc = l + 1 == nl ? C.x : C.y;
        for (int I = T; I < L.n; I += BS) {
            auto yv = [&](int J) {
                const int K = C.agg[J];
                return (double)L.x[J] + (K >= 0 ? al * (double)rc[K] : 0.0);
            };
            const double yi = yv(I), Dd = (double)L.D[I];
            double acc = Dd * yi;
            for (int k = L.adj_off[I]; k < L.adj_off[I + 1]; ++k) acc -= (double)L.Wa[k] * yv(L.adj_nbr[k]);
            L.y[I] = yi + om * (L.b[I] - acc) / Dd;
        }
        __syncthreads();
    }
    // level 0: w0 = z0 + alpha P y1, then z = w0 + omega (r - A w0) / D
    {
        const LView L1 = lv.lev(1);
        const mgreal *r1 = nl == 1 ? L1.x : L1.y;
        for (int i = T; i < n; i += BS) {
            const int J = L1.agg[i];
            w0[i] = (S0.free_(i) && J >= 0) ? z[i] + al * (double)r1[J] : 0.0;
        }
        __syncthreads();
    }
    double rz = 0.0;
    for (int i = T; i < n; i += BS) {
        double zi = 0.0;
        if (S0.free_(i)) {
            zi = (double)w0[i] + om * (r[i] - S0.Av(i, w0)) / S0.D[i];
            rz += r[i] * zi;
        }
        z[i] = zi;
        if (setp) S0.p[i] = zi;
    }
    return wg_sum<BS>(rz, red);     // its barriers also publish z (and p)
}

// PCG from the residual of the solve's set-up; returns the iteration count,
// *done when ||r||^2 <= tol2.
template <int BS, class Lev>
__device__ int wg_pcg(const L0View &S0, const Amg &a, const Lev &lv, double tol2, int max_iter, bool *done,
                      double *red_buf)
{
    const int T = threadIdx.x, n = S0.n;
    double *u = S0.u, *r = S0.r, *z = S0.z, *p = S0.p, *q = S0.q;
    WgRed red{red_buf, 0};
    double rz = wg_vcycle<BS>(S0, a, lv, true, red);
    int it = 0;
    *done = false;
    while (it < max_iter) {
        double pq = 0.0;
        for (int i = T; i < n; i += BS) {
            double qi = 0.0;
            if (S0.free_(i)) {
                qi = S0.Av(i, p);
                pq += p[i] * qi;
            }
            q[i] = qi;
        }
        pq = wg_sum<BS>(pq, red);
        const double alpha = pq > 0.0 ? rz / pq : 0.0;
        double rr = 0.0;
        for (int i = T; i < n; i += BS) {
            if (!S0.free_(i)) continue;
            u[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            rr += ri * ri;
        }
        rr = wg_sum<BS>(rr, red);
        ++it;
        if (rr <= tol2) { *done = true; break; }
        const double rz_new = wg_vcycle<BS>(S0, a, lv, false, red);
        const double beta = rz != 0.0 ? rz_new / rz : 0.0;
        rz = rz_new;
        for (int i = T; i < n; i += BS)
            if (S0.free_(i)) p[i] = z[i] + beta * p[i];
        __syncthreads();
    }
    return it;
}

// ---- global form ----
#define WG_BS 1024

__global__ __launch_bounds__(WG_BS, 8) void k_ir_pcg_wg(Dev d, const Amg *__restrict__ ap, double rtol,
                                                       int max_iter)
{
    __shared__ double red[2 * (WG_BS / 64)];
    const int s = blockIdx.x;
    if (d.conv[s]) {
        if (threadIdx.x == 0) d.ir_iters[s] = 0;
        return;
    }
    const Amg &a = *ap;
    const int n = d.n_nodes;
    const size_t o = (size_t)s * n;
    L0View S0;
    S0.n = n;
    S0.off = d.ninc_off;
    S0.nbr = d.ninc_nbr;
    S0.G = d.G_inc + (size_t)s * d.ninc_off[n];
    S0.D = d.diag + o;
    S0.fr = nullptr;
    S0.live = d.live + o;
    S0.is_pad = d.is_pad;
    S0.u = d.u + o; S0.r = d.r + o; S0.z = d.z + o; S0.p = d.p + o; S0.q = d.q + o;
    S0.w0 = a.l0.w0 + o;
    bool done;
    const int it = wg_pcg<WG_BS>(S0, a, GlobalLevels{ap, s}, rtol * rtol * d.bb[s], max_iter, &done, red);
    if (threadIdx.x == 0) {
        d.ir_iters[s] = it;
        d.conv[s] = done ? 1 : 0;
    }
}

// ---- LDS-resident form ----
// The passes are bound by LDS latency along each node's row, so the
// workgroup has about one thread per node (256 to 1024 threads).
constexpr int LDS_BYTES_MAX = 160 * 1024 - 1024;    // dynamic share of the 160 KB (reductions aside)

template <int BS>
__device__ inline void cp_i32(int *dst, const int *src, int n)
{
    for (int i = threadIdx.x; i < n; i += BS) dst[i] = src[i];
}
template <int BS, typename T>
__device__ inline void cp_arr(T *dst, const T *src, int n)
{
    for (int i = threadIdx.x; i < n; i += BS) dst[i] = src[i];
}

template <int LDS_BS>
__global__ __launch_bounds__(LDS_BS) void k_ir_pcg_lds(Dev d, const Amg *__restrict__ ap, LdsLayout ly,
                                                       double rtol, int max_iter)
{
    extern __shared__ __align__(16) char sm[];
    __shared__ double red[2 * (LDS_BS / 64)];
    const int s = blockIdx.x;
    if (d.conv[s]) {
        if (threadIdx.x == 0) d.ir_iters[s] = 0;
        return;
    }
    const Amg &a = *ap;
    const int n = d.n_nodes, nnz = d.ninc_off[n];
    const size_t o = (size_t)s * n;
    // load the sample's system and hierarchy
    cp_i32<LDS_BS>((int *)(sm + ly.off), d.ninc_off, n + 1);
    cp_i32<LDS_BS>((int *)(sm + ly.nbr), d.ninc_nbr, nnz);
    cp_arr<LDS_BS>((double *)(sm + ly.G), d.G_inc + (size_t)s * nnz, nnz);
    cp_arr<LDS_BS>((double *)(sm + ly.D), d.diag + o, n);
    cp_arr<LDS_BS>((double *)(sm + ly.u), d.u + o, n);
    cp_arr<LDS_BS>((double *)(sm + ly.r), d.r + o, n);
    for (int i = threadIdx.x; i < n; i += LDS_BS)
        ((uint8_t *)(sm + ly.fr))[i] = (d.live[o + i] && !d.is_pad[i]) ? 1 : 0;
    for (int l = 1; l <= a.nlev; ++l) {
        const AmgLevel &L = a.lev[l];
        cp_i32<LDS_BS>((int *)(sm + ly.agg[l]), L.agg, L.nf);
        cp_i32<LDS_BS>((int *)(sm + ly.mem_off[l]), L.mem_off, L.n + 1);
        cp_i32<LDS_BS>((int *)(sm + ly.mem[l]), L.mem, L.nmem);
        cp_i32<LDS_BS>((int *)(sm + ly.adj_off[l]), L.adj_off, L.n + 1);
        cp_i32<LDS_BS>((int *)(sm + ly.adj_nbr[l]), L.adj_nbr, 2 * L.ne);
        cp_arr<LDS_BS>((mgreal *)(sm + ly.LD[l]), L.D + (size_t)s * L.n, L.n);
        cp_arr<LDS_BS>((mgreal *)(sm + ly.LWa[l]), L.Wa + (size_t)s * 2 * L.ne, 2 * L.ne);
    }
    if (a.dense) {
        const int nc = a.lev[a.nlev].n;
        cp_arr<LDS_BS>((mgreal *)(sm + ly.Ainv), a.Ainv + (size_t)s * nc * nc, nc * nc);
    }
    __syncthreads();
    L0View S0;
    S0.n = n;
    S0.off = (const int *)(sm + ly.off);
    S0.nbr = (const int *)(sm + ly.nbr);
    S0.G = (const double *)(sm + ly.G);
    S0.D = (const double *)(sm + ly.D);
    S0.fr = (const uint8_t *)(sm + ly.fr);
    S0.live = nullptr;
    S0.is_pad = nullptr;
    S0.u = (double *)(sm + ly.u); S0.r = (double *)(sm + ly.r); S0.z = (double *)(sm + ly.z);
    S0.p = (double *)(sm + ly.p); S0.q = (double *)(sm + ly.q); S0.w0 = (mgreal *)(sm + ly.w0);
    bool done;
    const int it = wg_pcg<LDS_BS>(S0, a, LdsLevels{sm, &ly, ap}, rtol * rtol * d.bb[s], max_iter, &done, red);
    for (int i = threadIdx.x; i < n; i += LDS_BS) d.u[o + i] = S0.u[i];
    if (threadIdx.x == 0) {
        d.ir_iters[s] = it;
        d.conv[s] = done ? 1 : 0;
    }
}

// Host: the LDS layout of a system (offsets 16-byte aligned); bytes = 0 when
// it does not fit.
static LdsLayout lds_layout(const Dev &d, int nnz, const Amg &a)
{
    LdsLayout y{};
    long long at = 0;
    auto take = [&](long long bytes) {
        const int o = (int)at;
        at += (bytes + 15) & ~15LL;
        return o;
    };
    const int n = d.n_nodes;
    y.off = take(4LL * (n + 1));
    y.nbr = take(4LL * nnz);
    y.G = take(8LL * nnz);
    y.D = take(8LL * n);
    y.fr = take(n);
    y.u = take(8LL * n); y.r = take(8LL * n); y.z = take(8LL * n);
    y.p = take(8LL * n); y.q = take(8LL * n); y.w0 = take((long long)sizeof(mgreal) * n);
    for (int l = 1; l <= a.nlev; ++l) {
        const AmgLevel &L = a.lev[l];
        y.agg[l] = take(4LL * L.nf);
        y.mem_off[l] = take(4LL * (L.n + 1));
        y.mem[l] = take(4LL * L.nmem);
        y.adj_off[l] = take(4LL * (L.n + 1));
        y.adj_nbr[l] = take(8LL * L.ne);
        const long long m = sizeof(mgreal);
        y.LD[l] = take(m * L.n);
        y.LWa[l] = take(2 * m * L.ne);
        y.b[l] = take(m * L.n); y.x[l] = take(m * L.n);
        y.y[l] = take(m * L.n); y.w[l] = take(m * L.n);
    }
    if (a.dense) {
        const long long nc = a.lev[a.nlev].n;
        y.Ainv = take((long long)sizeof(mgreal) * nc * nc);
    }
    y.bytes = at <= LDS_BYTES_MAX ? (int)at : 0;
    return y;
}

int ir_lds_bytes(const Dev &d, int nnz, const Amg &a)
{
    if (a.nlev < 1) return 0;
    return lds_layout(d, nnz, a).bytes;
}

void launch_ir_pcg_lds(const Dev &d, int nnz, const Amg &a, const Amg *amg_dev, double rtol, int max_iter,
                       hipStream_t st)
{
    const LdsLayout y = lds_layout(d, nnz, a);
    if (d.n_nodes <= 256) k_ir_pcg_lds<256><<<d.S, 256, y.bytes, st>>>(d, amg_dev, y, rtol, max_iter);
    else if (d.n_nodes <= 512) k_ir_pcg_lds<512><<<d.S, 512, y.bytes, st>>>(d, amg_dev, y, rtol, max_iter);
    else k_ir_pcg_lds<1024><<<d.S, 1024, y.bytes, st>>>(d, amg_dev, y, rtol, max_iter);
}

int ir_wg_max_nodes() { return 1 << 16; }

void launch_ir_pcg_wg(const Dev &d, const Amg *amg_dev, double rtol, int max_iter, hipStream_t st)
{
    k_ir_pcg_wg<<<d.S, WG_BS, 0, st>>>(d, amg_dev, rtol, max_iter);
}

}  // namespace em
