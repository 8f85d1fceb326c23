// Extended rational Krylov reduced stepping of long chains (Sec. IV-E,
// Alg. 1, eqs. 21-27), for (tree, sample) instances without voids.
//
// Between two IR solves a chain's stress obeys C s' = A s + f (C = diag(V),
// A = -L the negated Laplacian of the edge conductances g = xi_k g0, f the
// constant drive).  With the shift s0 = 1/t_s, t_s = eta L^2 / (pi^2 kappa)
// (eq. 26: L the chain's length, kappa its volume-weighted diffusivity) and
// K = s0 C - A, the basis V spans the block rational Krylov space of R C over
// the starting block [K^-1 C s, K^-1 f] (eq. 23): block Gram-Schmidt, two
// passes, a column kept when its norm after orthogonalisation exceeds 1e-10
// of its norm before, at most q blocks.  The reduced model
// A_h = V^T A V, C_h = V^T C V, f_h = V^T f (eq. 25) is stepped by backward
// Euler, z <- (C_h - dt A_h)^-1 (C_h z + dt f_h), and lifted as s = V z.
//
// The basis is built from the state and drive of the instance's first
// reduced interval and kept while both stay in its span: the state does (it
// is V z), the drive until an IR re-solve changes the sample's conductances.
// An interval is taken in reduced form only when the lifted states provably
// stay below every critical stress: |V_i . (z_k - z_end)| <= |V_i|_2
// |z_k - z_end|_2 (V_i the node's row of V), so
// max_i (s_end,i - sigma_crit,i + |V_i|_2 max_k |z_k - z_end|_2) < 0 suffices;
// otherwise the interval is stepped by the exact chain kernel and the basis
// dropped (the exact state leaves the span).
//
// Layout: V columns [(c ns + i) S + s] (samples fastest, as the state); per
// instance KS doubles: A_h, C_h (RM x RM), f_h, z (RM), the step operator F
// (RM x RM), g (RM) and the step size they were formed for; pivots of K's
// tridiagonal factorisation [i S + s]; per instance the interval's reduced
// end state (RM) and the largest distance of its states from it.  Everything
// in FP64; the state is written back in the batch's precision (FP32: high and
// low parts).
//
// Per aging interval: k_kry_need lists the instances that need a basis or a
// step operator; k_kry_basis and k_kry_form work through those lists only;
// k_kry_rec runs the reduced recurrence (one instance per lane); k_kry_step
// checks the bound and lifts (one wavefront per instance).  Every count the
// kernels keep is spread over slots (see KRY_CNT_SLOTS): tens of thousands of
// workgroups adding to one device-scope counter queue on its address.
#include "em_internal.h"

#include <type_traits>

namespace em {

constexpr int KB = 256;                 // threads per workgroup of the per-instance flag kernels
constexpr double KRY_EPS = 1e-10;
#define EM_KERNEL_KB __global__ __launch_bounds__(256)

constexpr int KBW = 64;                 // one wavefront per basis build
constexpr int KRY_BASIS_GRID = 8192;    // workgroups of the basis launch (grid-stride over the builds)

// lane b's value on every lane (b uniform): two scalar lane reads
__device__ inline double kry_bcast(double v, int b)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), b);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// A strided node loop (first, first + step, ... below end) in batches of KU
// nodes: the batch's values are all computed (their loads issued together)
// before any is stored, so a long chain costs one memory round trip per batch
// rather than per node.  load(i) must not read what op(j, .) writes for
// another node j of the batch.
template <int KU, typename L, typename O>
__device__ inline void kw_batched(int first, int end, int step, L load, O op)
{
    for (int i = first; i < end; i += KU * step) {
        double v[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int ii = i + u * step;
            v[u] = ii < end ? load(ii) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int ii = i + u * step;
            if (ii < end) op(ii, v[u]);
        }
    }
}

// sum over the wavefront, every lane gets it
__device__ inline double kw_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// N sums over the wavefront at once (independent shuffles in flight together)
template <int N>
__device__ inline void kw_sum_n(double (&v)[N], int n)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < N; ++k)
            if (k < n) v[k] += __shfl_xor(v[k], o, 64);
}

// Lane L holds the affine map x -> m x + b of its segment (the composite of
// its nodes in sweep order).  Returns the value entering the segment: the maps
// of lanes 0 .. L-1 applied in order to 0 (an inclusive scan of the
// compositions, then the previous lane's composite).
__device__ inline double kw_affine_entry(double m, double b)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double pm = __shfl_up(m, o, 64), pb = __shfl_up(b, o, 64);
        if (lane >= o) {
            b = m * pb + b;
            m = m * pm;
        }
    }
    const double e = __shfl_up(b, 1, 64);
    return lane == 0 ? 0.0 : e;
}

// a 2x2 matrix rescaled by a power of two (exact) so that its largest entry
// is of order one: only ratios carry meaning, and products stay finite
__device__ inline void kw_mat_rescale(double &a, double &b, double &c, double &e)
{
    const double m = fmax(fmax(fabs(a), fabs(b)), fmax(fabs(c), fabs(e)));
    if (m > 0.0 && isfinite(m)) {
        const int k = -ilogb(m);
        a = ldexp(a, k);
        b = ldexp(b, k);
        c = ldexp(c, k);
        e = ldexp(e, k);
    }
}

// For 2x2 matrices [a b; c e] acting on (num, den) vectors (a continued
// fraction p -> 1 / (D - h p) is the projective map [0 1; -h D]): the
// composites of lanes 0 .. L-1 applied to (0, 1), returned on lane L as
// num / den.  The vector is carried through the lanes' matrices in order
// (one lane's matrix per pass, read by broadcast), not by a tree of matrix
// products: near the double root of a weakly shifted chain (s0 V << g) the
// tree's regrouping of the products loses several digits that the ordered
// product keeps.  The vector is rescaled by a power of two (exact).
__device__ inline double kw_projective_entry(double a, double b, double c, double e)
{
    const int lane = threadIdx.x & 63;
    double v0 = 0.0, v1 = 1.0, n0 = 0.0, n1 = 1.0;
    for (int L = 0; L < 63; ++L) {
        const double la = kry_bcast(a, L), lb = kry_bcast(b, L), lc = kry_bcast(c, L), le = kry_bcast(e, L);
        double w0 = la * v0 + lb * v1, w1 = lc * v0 + le * v1;
        const double m = fmax(fabs(w0), fabs(w1));
        if (m > 0.0 && isfinite(m)) {
            const int k = -ilogb(m);
            w0 = ldexp(w0, k);
            w1 = ldexp(w1, k);
        }
        v0 = w0;
        v1 = w1;
        if (lane == L + 1) {
            n0 = v0;
            n1 = v1;
        }
    }
    return n0 / n1;
}

// a chain instance the reduced path may take: active, without voids, of at
// least max(3q, 30) nodes (eq. 27)
__device__ inline bool kry_eligible(const Dev &d, int inst, int &s, int &i0, int &i1)
{
    const int t = inst / d.S;
    s = inst - t * d.S;
    if (!d.tree_chain[t] || !d.inst_active[inst] || !d.sample_active[s] || d.nv[inst] > 0) return false;
    i0 = d.tree_off[t];
    i1 = d.tree_off[t + 1];
    return i1 - i0 >= max(3 * d.kq, 30);
}

template <typename R>
__device__ inline double kry_state(const Dev &d, int i, int s)
{
    const size_t x = (size_t)i * d.S + s;
    double v = (double)((const R *)d.sigma)[x];
    if (d.sig_lo) v += (double)d.sig_lo[x];
    return v;
}

// The chain instances of the reduced list that need a basis (eligible, none
// kept) go to kbl, those that need their step operator formed (a new basis or
// a new step size) to kfl; the orders are free (the instances are independent).
EM_KERNEL_KB void k_kry_need(Dev d)
{
    const int j = blockIdx.x * KB + threadIdx.x;
    if (j >= d.n_kry_list) return;
    const int inst = d.kry_list[j];
    int s, i0, i1;
    if (!kry_eligible(d, inst, s, i0, i1)) return;
    const bool build = d.kr[inst] <= 0;
    if (build) d.kbl[atomicAdd(&d.kbn[0], 1u)] = inst;
    const double *dtF = d.kred + (size_t)inst * KRY_KS(d.krm) + 3 * d.krm * d.krm + 3 * d.krm;
    if (build || *dtF != d.dt) d.kfl[atomicAdd(&d.kbn[1], 1u)] = inst;
}

// One wavefront per chain instance needing a basis (grid-stride over the
// list k_kry_need wrote).  K = s0 C - A is tridiagonal along the chain; its
// pivots (a continued fraction) and the two sweeps of each solve (first-order
// recurrences) run as scans over the lanes, each lane holding a contiguous
// segment of the chain; Gram-Schmidt and the projections are wavefront sums.
template <typename R>
__global__ __launch_bounds__(KBW) void k_kry_basis(Dev d)
{
    const int nb = (int)*(volatile const unsigned int *)&d.kbn[0];
    for (int jb = blockIdx.x; jb < nb; jb += gridDim.x) {
        const int inst = d.kbl[jb];
        const int t = inst / d.S, s = inst - t * d.S;
        const int i0 = d.tree_off[t], i1 = d.tree_off[t + 1];
        const int lane = threadIdx.x, S = d.S, RM = d.krm;
        auto col = [&](int c, int i) -> double & { return d.kv[((size_t)c * d.ns + i) * S + s]; };
        auto ge = [&](int i) -> double { return d.xi_k[(size_t)d.seg[i] * S + s] * d.g0[i]; };   // edge (i-1, i)
        // per node: inverse pivot, forward multiplier m_i = g_i / p_(i-1) and
        // backward multiplier u_i = g_(i+1) / p_i of K's tridiagonal factorisation
        double *ip = d.kscr, *mf = ip + (size_t)d.ns * S, *ub = mf + (size_t)d.ns * S;   // [i S + s]
        // shift (eq. 26)
        double a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 4
        for (int i = i0 + lane; i < i1; i += KBW) {
            a2 += d.V[i];
            if (i > i0) {
                const double dx = d.len[d.seg[i]] / d.N;
                a1 += ge(i) * dx * dx;
                a3 += dx;
            }
        }
        const double kap = kw_sum(a1) / kw_sum(a2);
        const double L = kw_sum(a3);
        const double s0 = M_PI * M_PI * kap / (d.keta * L * L);
        // this lane's contiguous segment [lo, hi) of the chain
        const int chunk = (i1 - i0 + KBW - 1) / KBW;
        const int lo = min(i0 + lane * chunk, i1), hi = min(lo + chunk, i1);
        // pivots p_i = 1 / (D_i - g_i^2 p_(i-1)), D_i = s0 V_i + g_i + g_(i+1)
        {
            double a = 1.0, b = 0.0, c = 0.0, e = 1.0;
#pragma unroll 4
            for (int i = lo; i < hi; ++i) {
                const double gl = i > i0 ? ge(i) : 0.0, gr = i + 1 < i1 ? ge(i + 1) : 0.0;
                const double D = s0 * d.V[i] + gl + gr, h = gl * gl;
                double na = c, nb2 = e, nc = D * c - h * a, ne = D * e - h * b;
                kw_mat_rescale(na, nb2, nc, ne);
                a = na;
                b = nb2;
                c = nc;
                e = ne;
            }
            double p = kw_projective_entry(a, b, c, e);
            for (int i = lo; i < hi; i += 4) {
                double glv[4], grv[4], Vv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int ii = i + u;
                    glv[u] = ii < hi && ii > i0 ? ge(ii) : 0.0;
                    grv[u] = ii < hi && ii + 1 < i1 ? ge(ii + 1) : 0.0;
                    Vv[u] = ii < hi ? d.V[ii] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int ii = i + u;
                    if (ii >= hi) break;
                    const double gl = glv[u], gr = grv[u];
                    const double D = s0 * Vv[u] + gl + gr;
                    const double np = 1.0 / (ii > i0 ? D - gl * gl * p : D);
                    const size_t x = (size_t)ii * S + s;
                    ip[x] = np;
                    ub[x] = gr * np;
                    mf[x] = ii > i0 ? gl * p : 0.0;
                    p = np;
                }
            }
        }
        __syncthreads();                       // lanes read other lanes' nodes from here on
        // column c <- K^-1 column c: y_i = b_i + m_i y_(i-1) over the chain, then
        // x_i = p_i^-1 y_i + u_i x_(i+1) from its end (lane L takes segment 63 - L)
        const int rlo = min(i0 + (KBW - 1 - lane) * chunk, i1), rhi = min(rlo + chunk, i1);
        auto solve = [&](int c) {
            __syncthreads();
            double m = 1.0, b = 0.0;
#pragma unroll 4
            for (int i = lo; i < hi; ++i) {
                const double mi = mf[(size_t)i * S + s];
                b = mi * b + col(c, i);
                m = mi * m;
            }
            double y = kw_affine_entry(m, b);
            for (int i = lo; i < hi; i += 4) {
                double bv[4], mv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    bv[u] = i + u < hi ? col(c, i + u) : 0.0;
                    mv[u] = i + u < hi ? mf[(size_t)(i + u) * S + s] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    y = bv[u] + mv[u] * y;                // m = 0 at the chain's first node
                    if (i + u < hi) col(c, i + u) = y;
                }
            }
            __syncthreads();
            m = 1.0;
            b = 0.0;
#pragma unroll 4
            for (int i = rhi - 1; i >= rlo; --i) {
                const size_t x = (size_t)i * S + s;
                b = ub[x] * b + ip[x] * col(c, i);
                m = ub[x] * m;
            }
            double xv = kw_affine_entry(m, b);
            for (int i = rhi - 1; i >= rlo; i -= 4) {
                double yv[4], pv[4], uv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool in = i - u >= rlo;
                    const size_t x = (size_t)(i - u) * S + s;
                    yv[u] = in ? col(c, i - u) : 0.0;
                    pv[u] = in ? ip[x] : 0.0;
                    uv[u] = in ? ub[x] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    xv = pv[u] * yv[u] + uv[u] * xv;       // u = 0 at the chain's last node
                    if (i - u >= rlo) col(c, i - u) = xv;
                }
            }
            __syncthreads();
        };
        // orthonormalise column c against columns 0 .. c-1 (classical
        // Gram-Schmidt, two passes); true when kept
        auto accept = [&](int c) -> bool {
            double n0 = 0.0;
#pragma unroll 4
            for (int i = i0 + lane; i < i1; i += KBW) n0 += col(c, i) * col(c, i);
            n0 = sqrt(kw_sum(n0));
            if (!(n0 > 0.0)) return false;
            for (int pass = 0; pass < 2; ++pass) {
                double h[KRY_RM_MAX];
#pragma unroll
                for (int q = 0; q < KRY_RM_MAX; ++q) h[q] = 0.0;
                for (int i = i0 + lane; i < i1; i += KBW) {
                    const double w = col(c, i);
#pragma unroll
                    for (int q = 0; q < KRY_RM_MAX; ++q)
                        if (q < c) h[q] += col(q, i) * w;
                }
                kw_sum_n(h, c);
                kw_batched<2>(i0 + lane, i1, KBW, [&](int i) {
                    double w = col(c, i);
#pragma unroll
                    for (int q = 0; q < KRY_RM_MAX; ++q)
                        if (q < c) w -= h[q] * col(q, i);
                    return w;
                }, [&](int i, double w) { col(c, i) = w; });
            }
            double nw = 0.0;
#pragma unroll 4
            for (int i = i0 + lane; i < i1; i += KBW) nw += col(c, i) * col(c, i);
            nw = sqrt(kw_sum(nw));
            if (!(nw > KRY_EPS * n0)) return false;
            const double inv = 1.0 / nw;
            kw_batched<4>(i0 + lane, i1, KBW, [&](int i) { return col(c, i) * inv; },
                          [&](int i, double w) { col(c, i) = w; });
            return true;
        };
        const R *fv = (const R *)d.dtf;
        int r = 0;
        // starting block (eq. 23): K^-1 C s, K^-1 f
        kw_batched<4>(i0 + lane, i1, KBW, [&](int i) { return d.V[i] * kry_state<R>(d, i, s); },
                      [&](int i, double w) { col(r, i) = w; });
        solve(r);
        if (accept(r)) ++r;
        kw_batched<4>(i0 + lane, i1, KBW, [&](int i) { return (double)fv[(size_t)i * S + s] / d.dt; },
                      [&](int i, double w) { col(r, i) = w; });
        solve(r);
        if (accept(r)) ++r;
        int b0 = 0, b1 = r;
        for (int j = 1; j < d.kq && b1 > b0; ++j) {
            const int nbk = r;
            for (int c = b0; c < b1 && r < RM; ++c) {
                kw_batched<4>(i0 + lane, i1, KBW, [&](int i) { return d.V[i] * col(c, i); },
                              [&](int i, double w) { col(r, i) = w; });
                solve(r);
                if (accept(r)) ++r;
            }
            b0 = nbk;
            b1 = r;
        }
        // reduced matrices (eq. 25) and the reduced state V^T s
        __syncthreads();
        double *kh = d.kred + (size_t)inst * KRY_KS(RM);
        double *Ah = kh, *Ch = kh + RM * RM, *fh = kh + 2 * RM * RM, *z = fh + RM;
        for (int b = 0; b < r; ++b) {
            double aa[KRY_RM_MAX], cc[KRY_RM_MAX];
#pragma unroll
            for (int q = 0; q < KRY_RM_MAX; ++q) aa[q] = cc[q] = 0.0;
            for (int i = i0 + lane; i < i1; i += KBW) {
                const double vb = col(b, i), db = i > i0 ? vb - col(b, i - 1) : 0.0;
                const double w = d.V[i] * vb, gi = i > i0 ? ge(i) : 0.0;
#pragma unroll
                for (int q = 0; q < KRY_RM_MAX; ++q)
                    if (q >= b && q < r) {
                        const double vc = col(q, i);
                        cc[q] += w * vc;
                        if (i > i0) aa[q] -= gi * db * (vc - col(q, i - 1));
                    }
            }
            kw_sum_n(aa, r);
            kw_sum_n(cc, r);
            if (lane == 0)
                for (int q = b; q < r; ++q) {
                    Ah[b * RM + q] = Ah[q * RM + b] = aa[q];
                    Ch[b * RM + q] = Ch[q * RM + b] = cc[q];
                }
        }
        {
            double ff[KRY_RM_MAX], zz[KRY_RM_MAX];
#pragma unroll
            for (int q = 0; q < KRY_RM_MAX; ++q) ff[q] = zz[q] = 0.0;
#pragma unroll 2
            for (int i = i0 + lane; i < i1; i += KBW) {
                const double fi = (double)fv[(size_t)i * S + s] / d.dt, si = kry_state<R>(d, i, s);
#pragma unroll
                for (int q = 0; q < KRY_RM_MAX; ++q)
                    if (q < r) {
                        const double vq = col(q, i);
                        ff[q] += fi * vq;
                        zz[q] += si * vq;
                    }
            }
            kw_sum_n(ff, r);
            kw_sum_n(zz, r);
            if (lane == 0)
                for (int q = 0; q < r; ++q) {
                    fh[q] = ff[q];
                    z[q] = zz[q];
                }
        }
        if (lane == 0) {
            kh[3 * RM * RM + 3 * RM] = 0.0;    // step operator not formed yet
            d.kr[inst] = r;
            atomicAdd(&d.kcnt[0 * KRY_CNT_SLOTS + (blockIdx.x & (KRY_CNT_SLOTS - 1))], 1ull);
        }
        __syncthreads();
    }
}

// The step operator F = (C_h - dt A_h)^-1 C_h and g = dt (C_h - dt A_h)^-1 f_h
// of every instance in kfl (one wavefront each, grid-stride): LU without
// pivoting on one lane (C_h - dt A_h is symmetric positive definite), then
// column c of F on lane c and g on lane r, one triangular pair each.  Kept
// with the basis until the basis or the step size changes.
constexpr int KW = 64;

__global__ __launch_bounds__(KW) void k_kry_form(Dev d)
{
    __shared__ double M[KRY_RM_MAX * KRY_RM_MAX];
    const int nf = (int)*(volatile const unsigned int *)&d.kbn[1];
    const int lane = threadIdx.x, RM = d.krm;
    const double dt = d.dt;
    for (int jf = blockIdx.x; jf < nf; jf += gridDim.x) {
        const int inst = d.kfl[jf];
        const int r = d.kr[inst];
        if (r <= 0) continue;                   // the build kept no column
        double *kh = d.kred + (size_t)inst * KRY_KS(RM);
        const double *Ah = kh, *Ch = kh + RM * RM, *fh = kh + 2 * RM * RM;
        double *z = kh + 2 * RM * RM + RM, *F = z + RM, *g = F + RM * RM, *dtF = g + RM;
        if (lane == 0) {
            for (int a = 0; a < r; ++a)
                for (int b = 0; b < r; ++b) M[a * r + b] = Ch[a * RM + b] - dt * Ah[a * RM + b];
            for (int k = 0; k < r; ++k)
                for (int a = k + 1; a < r; ++a) {
                    const double l = M[a * r + k] / M[k * r + k];
                    M[a * r + k] = l;
                    for (int b = k + 1; b < r; ++b) M[a * r + b] -= l * M[k * r + b];
                }
        }
        __syncthreads();
        if (lane <= r) {
            double x[KRY_RM_MAX];
            for (int a = 0; a < r; ++a) x[a] = lane < r ? Ch[a * RM + lane] : dt * fh[a];
            for (int a = 1; a < r; ++a)
                for (int b = 0; b < a; ++b) x[a] -= M[a * r + b] * x[b];
            for (int a = r - 1; a >= 0; --a) {
                for (int b = a + 1; b < r; ++b) x[a] -= M[a * r + b] * x[b];
                x[a] /= M[a * r + a];
            }
            for (int a = 0; a < r; ++a) {
                if (lane < r) F[a * RM + lane] = x[a];
                else g[a] = x[a];
            }
        }
        if (lane == 0) *dtF = dt;
        __syncthreads();
    }
}

// n_steps of reduced backward Euler, z <- F z + g, for every instance with a
// basis, one lane per instance (64 instances to a wavefront) with F, g and z
// zero-padded to NR x NR in registers: the end state z_end to kze and the
// largest distance max_k |z_k - z_end|_2 of the interval's states (k = 0 ..
// n_steps) to kdist, the recurrence run a second time for the distances.  Per
// row the products are added in column order, as in the wavefront form below,
// and the padding adds exact zeros, so both forms give the same values.
constexpr int KRY_LANE_RM = 12;              // columns held per lane in registers

template <int NR>
__global__ __launch_bounds__(KW) void k_kry_rec(Dev d, int n_steps)
{
    const int j = blockIdx.x * KW + threadIdx.x;
    if (j >= d.n_kry_list) return;
    const int inst = d.kry_list[j];
    int s, i0, i1;
    if (!kry_eligible(d, inst, s, i0, i1)) return;
    const int r = d.kr[inst];
    if (r <= 0) return;
    const int RM = d.krm;
    const double *kh = d.kred + (size_t)inst * KRY_KS(RM);
    const double *z = kh + 2 * RM * RM + RM, *F = z + RM, *g = F + RM * RM;
    double f[NR][NR], gg[NR], zc[NR];
#pragma unroll
    for (int a = 0; a < NR; ++a) {
#pragma unroll
        for (int b = 0; b < NR; ++b) f[a][b] = (a < r && b < r) ? F[a * RM + b] : 0.0;
        gg[a] = a < r ? g[a] : 0.0;
        zc[a] = a < r ? z[a] : 0.0;
    }
    auto step = [&]() {
        double zn[NR];
#pragma unroll
        for (int a = 0; a < NR; ++a) {
            double v = gg[a];
#pragma unroll
            for (int b = 0; b < NR; ++b) v += f[a][b] * zc[b];
            zn[a] = v;
        }
#pragma unroll
        for (int a = 0; a < NR; ++a) zc[a] = zn[a];
    };
    for (int k = 0; k < n_steps; ++k) step();
    double ze[NR];
#pragma unroll
    for (int a = 0; a < NR; ++a) {
        ze[a] = zc[a];
        zc[a] = a < r ? z[a] : 0.0;            // the start state again (read back, not held)
    }
    auto gap = [&]() -> double {
        double q = 0.0;
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            const double e = zc[c] - ze[c];
            q += e * e;
        }
        return sqrt(q);
    };
    double dist = gap();
    for (int k = 0; k < n_steps; ++k) {
        step();
        dist = fmax(dist, gap());
    }
    double *out = d.kze + (size_t)inst * RM;
#pragma unroll
    for (int a = 0; a < NR; ++a)
        if (a < RM) out[a] = ze[a];
    d.kdist[inst] = dist;
}

// The bound and the lift, one wavefront per instance: the lifted end state
// replaces the state when the interval provably stays below every critical
// stress (the instance then sits out the exact launch).  With more than
// KRY_LANE_RM columns the recurrence runs here instead: lane a holds row a of
// F in registers and a step is r multiply-adds per lane against lane b's
// component read as a uniform broadcast (two scalar lane reads per
// component); the interval's reduced states go to LDS when they fit, so that
// the distance of each from the end state is one lane's sum over the
// components.
constexpr int KRY_ZS_BYTES = 32768;          // LDS for the interval's reduced states
constexpr int KRY_LC = 4;                    // blocks of 64 nodes whose lifted values stay in registers

// n_steps of z <- F z + g with NT >= r terms per row (rows and components
// beyond r are zero, so the padding adds exact zeros); state k (k = 0 ..
// n_steps) stored at zs[k RM + lane] for lanes below RM when zs is given
template <int NT>
__device__ inline double kry_interval(const double (&fr)[KRY_RM_MAX], double gl, double z0, int n_steps,
                                      double *zs, int RM, int lane)
{
    double zc = z0;
    if (zs && lane < RM) zs[lane] = zc;
    for (int k = 0; k < n_steps; ++k) {
        double v = gl;
#pragma unroll
        for (int b = 0; b < NT; ++b) v += fr[b] * kry_bcast(zc, b);
        zc = v;
        if (zs && lane < RM) zs[(k + 1) * RM + lane] = zc;
    }
    return zc;
}

template <typename R>
__global__ __launch_bounds__(KW) void k_kry_step(Dev d, int n_steps)
{
    __shared__ double ze_s[KRY_RM_MAX];
    extern __shared__ double zs_dyn[];
    if (blockIdx.x == 0 && threadIdx.x < 2) d.kbn[threadIdx.x] = 0;   // the launches that read them are done
    const int inst = d.kry_list[blockIdx.x];
    int s, i0, i1;
    if (!kry_eligible(d, inst, s, i0, i1)) return;
    const int r = d.kr[inst];
    if (r <= 0) return;
    const int lane = threadIdx.x, S = d.S, RM = d.krm;
    double *kh = d.kred + (size_t)inst * KRY_KS(RM);
    double *z = kh + 2 * RM * RM + RM, *F = z + RM, *g = F + RM * RM;
    double ze, dist = 0.0;
    if (RM <= KRY_LANE_RM) {
        ze = lane < r ? d.kze[(size_t)inst * RM + lane] : 0.0;
        dist = d.kdist[inst];
        if (lane < KRY_RM_MAX) ze_s[lane] = ze;   // zero beyond r
        __syncthreads();
    } else {
        // row `lane` of F in registers (zero beyond r)
        double fr[KRY_RM_MAX];
#pragma unroll
        for (int b = 0; b < KRY_RM_MAX; ++b) fr[b] = (lane < r && b < r) ? F[lane * RM + b] : 0.0;
        const double gl = lane < r ? g[lane] : 0.0, z0 = lane < r ? z[lane] : 0.0;
        const bool keep = (size_t)(n_steps + 1) * RM * sizeof(double) <= KRY_ZS_BYTES;
        double *zs = keep ? zs_dyn : nullptr;
        auto run = [&](double *out) -> double {
            if (r <= 4) return kry_interval<4>(fr, gl, z0, n_steps, out, RM, lane);
            if (r <= 8) return kry_interval<8>(fr, gl, z0, n_steps, out, RM, lane);
            if (r <= 12) return kry_interval<12>(fr, gl, z0, n_steps, out, RM, lane);
            return kry_interval<16>(fr, gl, z0, n_steps, out, RM, lane);
        };
        ze = run(zs);
        if (lane < KRY_RM_MAX) ze_s[lane] = ze;   // zero beyond r
        __syncthreads();
        // the largest distance of a reduced state of the interval from its end
        if (keep) {
            for (int k = lane; k <= n_steps; k += KW) {
                double q = 0.0;
                for (int c = 0; c < r; ++c) {
                    const double e = zs[k * RM + c] - ze_s[c];
                    q += e * e;
                }
                dist = fmax(dist, sqrt(q));
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) dist = fmax(dist, __shfl_xor(dist, o, 64));
        } else {
            // too many states for LDS: the recurrence again, one norm per state
            double zc = z0;
            for (int k = 0; k <= n_steps; ++k) {
                double q = lane < r ? (zc - ze) * (zc - ze) : 0.0;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
                dist = fmax(dist, sqrt(q));
                if (k < n_steps) {
                    double v = gl;
#pragma unroll
                    for (int b = 0; b < KRY_RM_MAX; ++b) v += fr[b] * kry_bcast(zc, b);
                    zc = v;
                }
            }
        }
    }
    const R *sc = (const R *)d.sc;
    auto run_lift = [&](auto nt) {
        constexpr int NT = decltype(nt)::value;
        // node i: the lifted end state V_i . z_end and |V_i|_2 (the columns'
        // loads issued together); the first KRY_LC blocks of 64 nodes keep
        // their lifted values in registers for the write-back
        auto row = [&](int i, double &w) -> double {
            double e[NT];
#pragma unroll
            for (int c = 0; c < NT; ++c) e[c] = c < r ? d.kv[((size_t)c * d.ns + i) * S + s] : 0.0;
            double v = 0.0;
            w = 0.0;
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                v += e[c] * ze_s[c];              // both zero beyond r
                w += e[c] * e[c];
            }
            return v;
        };
        double keep_v[KRY_LC];
        // node i moves by |V_i . (z_k - z_end)| <= |V_i|_2 |z_k - z_end|_2 during the interval
        double mg = -INFINITY;
        int blk = 0;
        for (int i = i0 + lane; i - lane < i1; i += KW, ++blk) {
            double w, v = 0.0;
            if (i < i1) {
                v = row(i, w);
                mg = fmax(mg, v - (double)sc[(size_t)i * S + s] + sqrt(w) * dist);
            }
#pragma unroll
            for (int k = 0; k < KRY_LC; ++k)
                if (k == blk) keep_v[k] = v;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mg = fmax(mg, __shfl_xor(mg, o, 64));
        const bool ok = mg < 0.0;
        if (ok) {
            R *sig = (R *)d.sigma;
            blk = 0;
            for (int i = i0 + lane; i < i1; i += KW, ++blk) {
                const size_t x = (size_t)i * S + s;
                double v = 0.0, w;
#pragma unroll
                for (int k = 0; k < KRY_LC; ++k)
                    if (k == blk) v = keep_v[k];
                if (blk >= KRY_LC) v = row(i, w);
                sig[x] = (R)v;
                if (d.sig_lo) d.sig_lo[x] = (float)(v - (double)(R)v);
            }
            if (lane < r) z[lane] = ze;
        }
        return ok;
    };
    bool ok;
    if (r <= 4) ok = run_lift(std::integral_constant<int, 4>());
    else if (r <= 8) ok = run_lift(std::integral_constant<int, 8>());
    else if (r <= 12) ok = run_lift(std::integral_constant<int, 12>());
    else ok = run_lift(std::integral_constant<int, 16>());
    if (lane == 0) {
        if (ok) {
            d.kdone[inst] = 1;
            d.inst_active[inst] = 0;
            const int slot = blockIdx.x & (KRY_CNT_SLOTS - 1);
            atomicAdd(&d.kcnt[1 * KRY_CNT_SLOTS + slot], 1ull);
            atomicAdd(&d.kcnt[3 * KRY_CNT_SLOTS + slot], (unsigned long long)(i1 - i0) * (unsigned long long)n_steps);
        } else {
            d.kr[inst] = 0;
            atomicAdd(&d.kcnt[2 * KRY_CNT_SLOTS + (blockIdx.x & (KRY_CNT_SLOTS - 1))], 1ull);
        }
    }
}

// the instances taken in reduced form rejoin the active set
EM_KERNEL_KB void k_kry_restore(Dev d)
{
    const int inst = blockIdx.x * KB + threadIdx.x;
    if (inst >= d.n_trees * d.S || !d.kdone[inst]) return;
    d.kdone[inst] = 0;
    d.inst_active[inst] = 1;
}

// bases of the samples whose conductances changed at the last IR solve (all:
// every basis) are dropped: the drive left their span
EM_KERNEL_KB void k_kry_invalidate(Dev d, int all)
{
    const int inst = blockIdx.x * KB + threadIdx.x;
    if (inst >= d.n_trees * d.S) return;
    if (all || d.g_chg_s[inst % d.S]) d.kr[inst] = 0;
}

void launch_kry_step(const Dev &d, bool fp32, int n_steps, hipStream_t st)
{
    const int n = d.n_kry_list;
    if (n <= 0 || d.kq <= 0) return;
    // the instances needing a basis or a step operator, the builds, the
    // operators, the reduced intervals, then the bound and lift (which also
    // clears the two list lengths for the next interval)
    k_kry_need<<<(n + KB - 1) / KB, KB, 0, st>>>(d);
    const int gb = std::min(n, KRY_BASIS_GRID);
    if (fp32) k_kry_basis<float><<<gb, KBW, 0, st>>>(d);
    else k_kry_basis<double><<<gb, KBW, 0, st>>>(d);
    k_kry_form<<<gb, KW, 0, st>>>(d);
    unsigned zs_bytes = 0;
    if (d.krm <= 8) k_kry_rec<8><<<(n + KW - 1) / KW, KW, 0, st>>>(d, n_steps);
    else if (d.krm <= KRY_LANE_RM) k_kry_rec<KRY_LANE_RM><<<(n + KW - 1) / KW, KW, 0, st>>>(d, n_steps);
    else {
        const size_t zs = (size_t)(n_steps + 1) * d.krm * sizeof(double);
        zs_bytes = zs <= (size_t)KRY_ZS_BYTES ? (unsigned)zs : 0u;
    }
    if (fp32) k_kry_step<float><<<n, KW, zs_bytes, st>>>(d, n_steps);
    else k_kry_step<double><<<n, KW, zs_bytes, st>>>(d, n_steps);
}

void launch_kry_restore(const Dev &d, hipStream_t st)
{
    const int n = d.n_trees * d.S;
    if (n > 0 && d.kq > 0) k_kry_restore<<<(n + KB - 1) / KB, KB, 0, st>>>(d);
}

void launch_kry_invalidate(const Dev &d, bool all, hipStream_t st)
{
    const int n = d.n_trees * d.S;
    if (n > 0 && d.kq > 0) k_kry_invalidate<<<(n + KB - 1) / KB, KB, 0, st>>>(d, all ? 1 : 0);
}

}  // namespace em
