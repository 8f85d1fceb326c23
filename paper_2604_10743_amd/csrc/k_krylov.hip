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
// tridiagonal factorisation [i S + s].  Everything in FP64; the state is
// written back in the batch's precision (FP32: high and low parts).
#include "em_internal.h"

namespace em {

constexpr int KB = 256;                 // threads per instance workgroup
constexpr double KRY_EPS = 1e-10;
#define EM_KERNEL_KB __global__ __launch_bounds__(256)

__device__ inline double kb_sum(double v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < KB / 64; ++k) r += sh[k];
    return r;
}

__device__ inline double kb_max(double v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int k = 1; k < KB / 64; ++k) r = fmax(r, sh[k]);
    return r;
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

template <typename R>
EM_KERNEL_KB void k_kry_basis(Dev d)
{
    __shared__ double sh[KB / 64];
    const int inst = d.kry_list[blockIdx.x];
    int s, i0, i1;
    if (!kry_eligible(d, inst, s, i0, i1) || d.kr[inst] > 0) return;
    const int tid = threadIdx.x, S = d.S, RM = d.krm;
    auto col = [&](int c, int i) -> double & { return d.kv[((size_t)c * d.ns + i) * S + s]; };
    auto ge = [&](int i) -> double { return d.xi_k[(size_t)d.seg[i] * S + s] * d.g0[i]; };   // edge (i-1, i)
    // per node: inverse pivot, forward multiplier m_i = g_i / p_(i-1) and
    // backward multiplier u_i = g_(i+1) / p_i of K's tridiagonal factorisation
    double *ip = d.kscr, *mf = ip + (size_t)d.ns * S, *ub = mf + (size_t)d.ns * S;   // [i S + s]
    // shift (eq. 26)
    double a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int i = i0 + tid; i < i1; i += KB) {
        a2 += d.V[i];
        if (i > i0) {
            const double dx = d.len[d.seg[i]] / d.N;
            a1 += ge(i) * dx * dx;
            a3 += dx;
        }
    }
    const double kap = kb_sum(a1, sh) / kb_sum(a2, sh);
    const double L = kb_sum(a3, sh);
    const double s0 = M_PI * M_PI * kap / (d.keta * L * L);
    // K = s0 C + L is tridiagonal along the chain: the edge conductances in
    // parallel, then the pivots in order (one thread)
    for (int i = i0 + tid; i < i1; i += KB) mf[(size_t)i * S + s] = i > i0 ? ge(i) : 0.0;
    __syncthreads();
    if (tid == 0) {
        double p = 0.0;
        for (int i = i0; i < i1; ++i) {
            const double gl = mf[(size_t)i * S + s], gr = i + 1 < i1 ? mf[(size_t)(i + 1) * S + s] : 0.0;
            const double D = s0 * d.V[i] + gl + gr;
            const double np = 1.0 / (i > i0 ? D - gl * gl * p : D);    // p: the previous inverse pivot
            ip[(size_t)i * S + s] = np;
            ub[(size_t)i * S + s] = gr * np;
            if (i > i0) mf[(size_t)i * S + s] = gl * p;
            p = np;
        }
    }
    __syncthreads();
    // column c <- K^-1 column c: y_i = b_i + m_i y_(i-1), then
    // x_i = p_i^-1 y_i + u_i x_(i+1) (one thread, loads issued eight nodes at a time)
    auto solve = [&](int c) {
        if (tid == 0) {
            double y = 0.0;
            for (int i = i0; i < i1; i += 8) {
                double b[8], m[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    b[k] = i + k < i1 ? col(c, i + k) : 0.0;
                    m[k] = i + k < i1 ? mf[(size_t)(i + k) * S + s] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    y = b[k] + m[k] * y;              // m = 0 at the chain's first node
                    b[k] = y;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (i + k < i1) col(c, i + k) = b[k];
            }
            double x = 0.0;
            for (int i = i1 - 1; i >= i0; i -= 8) {
                double yv[8], pv[8], uv[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const bool in = i - k >= i0;
                    yv[k] = in ? col(c, i - k) : 0.0;
                    pv[k] = in ? ip[(size_t)(i - k) * S + s] : 0.0;
                    uv[k] = in ? ub[(size_t)(i - k) * S + s] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    x = pv[k] * yv[k] + uv[k] * x;     // u = 0 at the chain's last node
                    yv[k] = x;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (i - k >= i0) col(c, i - k) = yv[k];
            }
        }
        __syncthreads();
    };
    auto dot = [&](int b, int c) -> double {
        double a = 0.0;
        for (int i = i0 + tid; i < i1; i += KB) a += col(b, i) * col(c, i);
        return kb_sum(a, sh);
    };
    // orthonormalise column c against columns 0 .. c-1; true when kept
    auto accept = [&](int c) -> bool {
        const double n0 = sqrt(dot(c, c));
        if (!(n0 > 0.0)) return false;
        for (int pass = 0; pass < 2; ++pass)
            for (int b = 0; b < c; ++b) {
                const double h = dot(b, c);
                for (int i = i0 + tid; i < i1; i += KB) col(c, i) -= h * col(b, i);
                __syncthreads();
            }
        const double nw = sqrt(dot(c, c));
        if (!(nw > KRY_EPS * n0)) return false;
        const double inv = 1.0 / nw;
        for (int i = i0 + tid; i < i1; i += KB) col(c, i) *= inv;
        __syncthreads();
        return true;
    };
    const R *fv = (const R *)d.dtf;
    int r = 0;
    // starting block (eq. 23): K^-1 C s, K^-1 f
    for (int i = i0 + tid; i < i1; i += KB) col(r, i) = d.V[i] * kry_state<R>(d, i, s);
    __syncthreads();
    solve(r);
    if (accept(r)) ++r;
    for (int i = i0 + tid; i < i1; i += KB) col(r, i) = (double)fv[(size_t)i * S + s] / d.dt;
    __syncthreads();
    solve(r);
    if (accept(r)) ++r;
    int b0 = 0, b1 = r;
    for (int j = 1; j < d.kq && b1 > b0; ++j) {
        const int nb = r;
        for (int c = b0; c < b1 && r < RM; ++c) {
            for (int i = i0 + tid; i < i1; i += KB) col(r, i) = d.V[i] * col(c, i);
            __syncthreads();
            solve(r);
            if (accept(r)) ++r;
        }
        b0 = nb;
        b1 = r;
    }
    // reduced matrices (eq. 25) and the reduced state V^T s
    double *kh = d.kred + (size_t)inst * KRY_KS(RM);
    double *Ah = kh, *Ch = kh + RM * RM, *fh = kh + 2 * RM * RM, *z = fh + RM;
    for (int b = 0; b < r; ++b)
        for (int c = b; c < r; ++c) {
            double aa = 0.0, cc = 0.0;
            for (int i = i0 + tid; i < i1; i += KB) {
                cc += d.V[i] * col(b, i) * col(c, i);
                if (i > i0) aa -= ge(i) * (col(b, i) - col(b, i - 1)) * (col(c, i) - col(c, i - 1));
            }
            aa = kb_sum(aa, sh);
            cc = kb_sum(cc, sh);
            if (tid == 0) {
                Ah[b * RM + c] = Ah[c * RM + b] = aa;
                Ch[b * RM + c] = Ch[c * RM + b] = cc;
            }
        }
    for (int b = 0; b < r; ++b) {
        double ff = 0.0, zz = 0.0;
        for (int i = i0 + tid; i < i1; i += KB) {
            ff += (double)fv[(size_t)i * S + s] / d.dt * col(b, i);
            zz += kry_state<R>(d, i, s) * col(b, i);
        }
        ff = kb_sum(ff, sh);
        zz = kb_sum(zz, sh);
        if (tid == 0) {
            fh[b] = ff;
            z[b] = zz;
        }
    }
    if (tid == 0) {
        kh[3 * RM * RM + 3 * RM] = 0.0;        // step operator not formed yet
        d.kr[inst] = r;
        atomicAdd(&d.kcnt[0], 1ull);
    }
}

// n_steps of reduced backward Euler for every instance with a basis; the
// lifted end state replaces the state when the interval provably stays below
// every critical stress (the instance then sits out the exact launch).  One
// wavefront per instance: the step operator F = (C_h - dt A_h)^-1 C_h and
// g = dt (C_h - dt A_h)^-1 f_h are formed once per basis and step size (one
// lane, LU without pivoting: C_h - dt A_h is symmetric positive definite) and
// kept with the basis; lane a holds row a of F in registers, so a step is r
// shuffles and multiply-adds per lane.
constexpr int KW = 64;

template <typename R>
__global__ __launch_bounds__(KW) void k_kry_step(Dev d, int n_steps)
{
    __shared__ double M[KRY_RM_MAX * KRY_RM_MAX], ze_s[KRY_RM_MAX];
    const int inst = d.kry_list[blockIdx.x];
    int s, i0, i1;
    if (!kry_eligible(d, inst, s, i0, i1)) return;
    const int r = d.kr[inst];
    if (r <= 0) return;
    const int lane = threadIdx.x, S = d.S, RM = d.krm;
    double *kh = d.kred + (size_t)inst * KRY_KS(RM);
    const double *Ah = kh, *Ch = kh + RM * RM, *fh = kh + 2 * RM * RM;
    double *z = kh + 2 * RM * RM + RM, *F = z + RM, *g = F + RM * RM, *dtF = g + RM;
    const double dt = d.dt;
    if (*dtF != dt) {                          // a new basis or a new step size
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
        // column c of F (c < r) and, on lane r, g: one triangular pair each
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
        __syncthreads();
        if (lane == 0) *dtF = dt;
        __threadfence_block();
        __syncthreads();
    }
    // row `lane` of F in registers
    double fr[KRY_RM_MAX];
#pragma unroll
    for (int b = 0; b < KRY_RM_MAX; ++b) fr[b] = (lane < r && b < r) ? F[lane * RM + b] : 0.0;
    const double gl = lane < r ? g[lane] : 0.0, z0 = lane < r ? z[lane] : 0.0;
    auto step = [&](double zc) -> double {
        double v = gl;
#pragma unroll
        for (int b = 0; b < KRY_RM_MAX; ++b)
            if (b < r) v += fr[b] * __shfl(zc, b, 64);
        return v;
    };
    double zc = z0;
    for (int k = 0; k < n_steps; ++k) zc = step(zc);
    const double ze = zc;
    // the largest distance of a reduced state of the interval from its end
    double dist = 0.0;
    zc = z0;
    for (int k = 0; k <= n_steps; ++k) {
        double q = lane < r ? (zc - ze) * (zc - ze) : 0.0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
        dist = fmax(dist, sqrt(q));
        if (k < n_steps) zc = step(zc);
    }
    if (lane < r) ze_s[lane] = ze;
    __syncthreads();
    const R *sc = (const R *)d.sc;
    auto lift = [&](int i) -> double {
        double v = 0.0;
        for (int c = 0; c < r; ++c) v += d.kv[((size_t)c * d.ns + i) * S + s] * ze_s[c];
        return v;
    };
    // node i moves by |V_i . (z_k - z_end)| <= |V_i|_2 |z_k - z_end|_2 during the interval
    double mg = -INFINITY;
    for (int i = i0 + lane; i < i1; i += KW) {
        double v = 0.0, w = 0.0;
        for (int c = 0; c < r; ++c) {
            const double e = d.kv[((size_t)c * d.ns + i) * S + s];
            v += e * ze_s[c];
            w += e * e;
        }
        mg = fmax(mg, v - (double)sc[(size_t)i * S + s] + sqrt(w) * dist);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mg = fmax(mg, __shfl_xor(mg, o, 64));
    const bool ok = mg < 0.0;
    if (ok) {
        R *sig = (R *)d.sigma;
        for (int i = i0 + lane; i < i1; i += KW) {
            const size_t x = (size_t)i * S + s;
            const double v = lift(i);
            sig[x] = (R)v;
            if (d.sig_lo) d.sig_lo[x] = (float)(v - (double)(R)v);
        }
        if (lane < r) z[lane] = ze;
    }
    if (lane == 0) {
        if (ok) {
            d.kdone[inst] = 1;
            d.inst_active[inst] = 0;
            atomicAdd(&d.kcnt[1], 1ull);
            atomicAdd(&d.kcnt[3], (unsigned long long)(i1 - i0) * (unsigned long long)n_steps);
        } else {
            d.kr[inst] = 0;
            atomicAdd(&d.kcnt[2], 1ull);
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
    if (fp32) {
        k_kry_basis<float><<<n, KB, 0, st>>>(d);
        k_kry_step<float><<<n, KW, 0, st>>>(d, n_steps);
    } else {
        k_kry_basis<double><<<n, KB, 0, st>>>(d);
        k_kry_step<double><<<n, KW, 0, st>>>(d, n_steps);
    }
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
