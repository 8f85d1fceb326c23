// Resident chain kernel: backward-Euler stepping of wire trees that are
// chains (every FD node has at most one child in pre-order, i.e. a straight
// wire split into segments -- the common case of power stripes), held on chip
// for a whole aging interval.
//
// Layout.  A workgroup of WG lanes holds whole instances (tree, sample); each
// lane owns a block of at most M consecutive FD nodes of one instance.  The
// first node of every block is a separator; the others are the block's
// interior.  Per step:
//   1. rhs b = V (sigma + corr) + dt f                        (registers)
//   2. interior Thomas solve with zero separator values      (registers)
//      -> y, plus the precomputed responses alpha, beta to the left and
//      right separators (interior = y + alpha x_k + beta x_{k+1})
//   3. reduced tridiagonal system on the separators, solved by parallel
//      cyclic reduction through LDS; instance boundaries have zero coupling,
//      so one reduction serves every instance packed in the workgroup
//   4. back-out of the interior; void growth; nucleation test
// The elimination is exact (a reordering of the tree elimination); only the
// rounding order differs.  The factors (interior Thomas multipliers, alpha,
// beta, cyclic-reduction multipliers) are built in the kernel at launch start
// and rebuilt when a void row is stamped, so HBM is touched once per launch.
// The stress content sum V sigma + B * void volume is projected back to its
// launch-start value every `proj_every` steps (rounding-level correction, see
// the tree kernel).
#include "em_internal.h"
#include <cmath>

namespace em {

__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Workgroup-wide OR with one barrier: each wavefront's vote in its own LDS
// word, then every lane ORs the words.  A caller needs at least one other
// barrier between two calls (the words are rewritten by the next call).
template <int WG>
__device__ __forceinline__ bool wg_any(bool p, unsigned *s_w, int lane)
{
    const bool wave = __any(p ? 1 : 0) != 0;
    if ((lane & 63) == 0) s_w[lane >> 6] = wave ? 1u : 0u;
    lds_barrier();
    unsigned a = 0;
#pragma unroll
    for (int w = 0; w < WG / 64; ++w) a |= s_w[w];
    return a != 0;
}

template <int N>
struct Log2 { static constexpr int v = 1 + Log2<N / 2>::v; };
template <>
struct Log2<1> { static constexpr int v = 0; };

__device__ inline int chain_host_segment(const Dev &d, int v, int s)
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

__device__ inline double chain_robin_weight(const Dev &d, int v, int s)
{
    double r = 0.0;
    if (d.parent[v] >= 0) r += d.xi_k[(size_t)d.seg[v] * d.S + s] * d.rob0[v];
    for (int k = d.child_off[v]; k < d.child_off[v + 1]; ++k) {
        int c = d.child[k];
        r += d.xi_k[(size_t)d.seg[c] * d.S + s] * d.rob0[c];
    }
    return r;
}

struct ChainHot {
    void *sigma;
    float *sig_lo;           // FP32 form: low part of the stress state
    const void *Vr, *dtf, *sc;
    const int *lane_inst, *lane_blk, *tree_off;
    const uint8_t *sample_active, *inst_active;
    const Dev *dev;          // device-resident copy of every other field
    int S, n_steps, step0, proj_every;
    double dt;
};

// dt * kappa-scaled conductance of the edge (parent(i), i) for sample s
__device__ inline double edge_dtg(const Dev *d, int i, int s, double dt)
{
    return dt * d->xi_k[(size_t)d->seg[i] * d->S + s] * d->g0[i];
}

// OCC: waves per SIMD the register budget must allow (1: as many registers
// as the kernel wants; 4: at most 128 VGPRs, so that several workgroups share
// a CU when the launch holds few instances).
template <typename R, int M, int WG, int OCC>
__global__ __launch_bounds__(WG, OCC) void k_chain(ChainHot h)
{
    constexpr int LEV = Log2<WG>::v;
    // FP32 form: the state carries a float low part sl (sg + sl), which keeps
    // the increments that fall below half an ulp of sg (near saturation the
    // per-step increments shrink to a few Pa and float alone would stall the
    // approach to sigma_crit, moving nucleation by steps).  With 1024 lanes
    // (chains of more than 4096 nodes) the register file has no room for it:
    // there the low part is folded in at load and the state rounds to float
    // every step.  (Keeping it in LDS instead doubled the spills and cost 60 %
    // per launch, while the nucleation steps still moved by up to 3 against
    // FP64 stepping: the float separator solve, not the state, dominates there.)
    constexpr bool LO = sizeof(R) == 4 && WG < 1024;
    __shared__ R s_al[LEV][WG];
    __shared__ R s_ga[LEV][WG];
    // separator exchange of the per-step reduction, padded by WG/2 zeros on
    // each side: the neighbours at lane -+ 2^l are read at a constant offset
    // from one lane address (no per-level index registers, no clamping)
    __shared__ R s_xp[2][2 * WG];
    __shared__ R s_e[3][WG];
    // neighbour exchange of the factorisation and of the separator values:
    // shares s_e's storage (every use is separated from the uses of s_e by a
    // barrier that all lanes pass after their reads)
    R (*const s_x)[WG] = s_e;
    __shared__ double s_q[WG];
    __shared__ unsigned s_vote[WG / 64];

    const Dev *d = h.dev;
    const int lane = threadIdx.x;
    s_xp[0][lane] = 0; s_xp[0][lane + WG] = 0;
    s_xp[1][lane] = 0; s_xp[1][lane + WG] = 0;      // pads stay zero (ordered by the barriers below)
    const size_t gl = (size_t)blockIdx.x * WG + lane;
    const int S = h.S;
    const int inst = h.lane_inst[gl];
    const int kb = inst >= 0 ? h.lane_blk[gl] : 0;
    int t = 0, s = 0, start = 0, cnt = 0, lo = lane, hi = lane, nT = 0;
    bool act = false;
    if (inst >= 0) {
        t = inst / S;
        s = inst - t * S;
        int base = h.tree_off[t];
        nT = h.tree_off[t + 1] - base;
        start = base + kb * M;
        cnt = min(M, nT - kb * M);
        lo = lane - kb;
        hi = lo + (nT + M - 1) / M - 1;
        act = h.sample_active[s] && h.inst_active[inst];
    }
    if (!__syncthreads_or(act ? 1 : 0)) return;   // nothing to step in this workgroup
    const bool first = act && kb == 0;
    const bool last = act && (kb * M + cnt == nT);
    if (!act) cnt = 0;
    if (act && lane == lo)
        atomicAdd(&d->node_steps[blockIdx.x & (NS_SLOTS - 1)], (unsigned long long)nT * (unsigned long long)h.n_steps);

    R *sig = (R *)h.sigma;
    float *sig_lo = h.sig_lo;
    const R *dtf_g = (const R *)h.dtf;
    const R *sc_g = (const R *)h.sc;
    const R *Vr_g = (const R *)h.Vr;
    const R *Vr_b = Vr_g + start;   // this lane's block: one base address, constant offsets
    const double dt = h.dt;

    // ---- per-lane node data (registers for the whole launch) ----
    R sg[M], fv[M], dinv[M], al[M], be[M];
    float slr[LO ? M : 1];          // the low part (registers)
    auto SL = [&](int j) -> float {
        if constexpr (LO) return slr[j];
        else return 0.f;
    };
    auto SLset = [&](int j, float v) {
        if constexpr (LO) slr[j] = v;
    };
    R gE[M + 1];                    // gE[j] = dt*g of edge (j-1, j); gE[0] previous block, gE[cnt] next block
    R scmin = (R)INFINITY;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        // nodes past cnt (a short last block, an idle lane) keep zeros here:
        // the step below computes them without branches, and zero pivots and
        // multipliers map them to zero increments
        sg[j] = 0; fv[j] = 0; dinv[j] = 0; al[j] = 0; be[j] = 0;
        float lo0 = 0.f;
        if (j < cnt) {
            size_t x = (size_t)(start + j) * S + s;
            sg[j] = sig[x];
            if constexpr (LO) {
                lo0 = sig_lo ? sig_lo[x] : 0.f;
            } else if constexpr (sizeof(R) == 4) {
                if (sig_lo) sg[j] = (R)((double)sg[j] + (double)sig_lo[x]);
            }
            fv[j] = dtf_g[x];
            R scj = sc_g[x];
            scmin = scj < scmin ? scj : scmin;
        }
        SLset(j, lo0);
    }
    // nucleation pre-test on the high part alone: sg + sl >= sc implies
    // sg >= sc - |sl| >= the float below sc (|sl| <= half an ulp of sg)
    const R scpre = LO ? nextafterf((float)scmin, -INFINITY) : scmin;
#pragma unroll
    for (int j = 0; j <= M; ++j) {
        gE[j] = 0;
        if (act && j <= cnt) {
            bool exists = (j == 0) ? !first : (j == cnt ? !last : true);
            if (exists) gE[j] = (R)edge_dtg(d, start + j, s, dt);
        }
    }
    int nv = act ? d->nv[inst] : 0;
    unsigned vmask = 0;             // block nodes carrying a void
    // a void node's row has no drive (its Robin row replaces it): its dt*f
    // register is zeroed here once (the void growth reads it from memory)
    auto refresh_vmask = [&]() {
        vmask = 0;
        for (int k = 0; k < nv; ++k) {
            int jv = d->vnode[inst * MAXV + k] - start;
            if (jv >= 0 && jv < cnt) vmask |= 1u << jv;
        }
#pragma unroll
        for (int j = 0; j < M; ++j)
            if ((vmask >> j) & 1u) fv[j] = 0;
    };
    if (act) refresh_vmask();
    auto e_first = [&]() -> R {     // coupling from the separator to what follows it
        R e = gE[1];
        if (cnt == 1) e = gE[1];   // gE[cnt] is the next block's edge
        return e;
    };

    // ---- factorisation (interior Thomas, alpha/beta, reduced row, PCR) ----
    R dfin = 1;
    auto factor = [&]() {
        R Dg[M], w[M];       // forward multipliers w[j] = gE[j] dinv[j-1] (recomputed per step)
#pragma unroll
        for (int j = 0; j < M; ++j) Dg[j] = (j < cnt ? Vr_b[j] : (R)0) + gE[j] + gE[j + 1];
        for (int k = 0; k < nv; ++k) {          // Robin rows of the block's voids
            int jv = d->vnode[inst * MAXV + k] - start;
            R rw = (R)(dt * d->vrob[inst * MAXV + k]);
#pragma unroll
            for (int j = 0; j < M; ++j)
                if (j == jv) Dg[j] += rw;
        }
        // interior nodes 1..cnt-1: forward multipliers and pivots
#pragma unroll
        for (int j = 1; j < M; ++j) {
            if (j < cnt) {
                R dp = Dg[j];
                if (j >= 2) { w[j] = gE[j] * dinv[j - 1]; dp = Dg[j] - w[j] * gE[j]; }
                else w[j] = 0;
                dinv[j] = (R)1 / dp;
            }
        }
        // alpha = T^-1 (gE[1] e_first), beta = T^-1 (gE[cnt] e_last)
        {
            R a = 0;
#pragma unroll
            for (int j = 1; j < M; ++j)
                if (j < cnt) { a = (j == 1) ? gE[1] : w[j] * a; al[j] = a; }
            R an = 0, bn = 0;
#pragma unroll
            for (int j = M - 1; j >= 1; --j) {
                if (j < cnt) {
                    const R uj = (j + 1 < cnt) ? gE[j + 1] * dinv[j] : (R)0;
                    const R bj = (j == cnt - 1) ? gE[cnt] : (R)0;
                    an = al[j] * dinv[j] + uj * an;
                    bn = bj * dinv[j] + uj * bn;
                    al[j] = an;
                    be[j] = bn;
                }
            }
        }
        // the block's first interior node (F) and last node (L) in terms of
        // (own separator, next separator)
        R aF, bF, aL, bL;
        if (cnt >= 2) {
            aF = al[1]; bF = be[1];
            aL = 0; bL = 0;
#pragma unroll
            for (int j = 1; j < M; ++j) if (j == cnt - 1) { aL = al[j]; bL = be[j]; }
        } else {
            aF = 0; bF = 1;
            aL = 1; bL = 0;
        }
        s_x[0][lane] = aL;
        s_x[1][lane] = bL;
        lds_barrier();
        const R aLp = (act && !first) ? s_x[0][lane - 1] : (R)0;
        const R bLp = (act && !first) ? s_x[1][lane - 1] : (R)0;
        lds_barrier();
        R A = 0, Dd = 1, C = 0;
        if (act) {
            const R e1 = e_first();
            A = -gE[0] * aLp;
            Dd = Dg[0] - gE[0] * bLp - e1 * aF;
            C = -e1 * bF;
        }
        // cyclic reduction of the separator matrix; keep the rhs multipliers
#pragma unroll
        for (int l = 0; l < LEV; ++l) {
            const int dd = 1 << l;
            s_e[0][lane] = A; s_e[1][lane] = Dd; s_e[2][lane] = C;
            lds_barrier();
            R al_l = 0, ga_l = 0, Am = 0, Cm = 0, Ap = 0, Cp = 0;
            if (A != (R)0) {
                al_l = -A / s_e[1][lane - dd];
                Am = s_e[0][lane - dd]; Cm = s_e[2][lane - dd];
            }
            if (C != (R)0) {
                ga_l = -C / s_e[1][lane + dd];
                Ap = s_e[0][lane + dd]; Cp = s_e[2][lane + dd];
            }
            lds_barrier();
            Dd = Dd + al_l * Cm + ga_l * Ap;
            A = al_l * Am;
            C = ga_l * Cp;
            s_al[l][lane] = al_l;
            s_ga[l][lane] = ga_l;
        }
        dfin = (R)1 / Dd;
        lds_barrier();
    };
    factor();

    // ---- segmented (per-instance) sums over the lanes of the workgroup ----
    auto seg_sum = [&](double v) -> double {
        s_q[lane] = v;
        lds_barrier();
#pragma unroll
        for (int l = 0; l < LEV; ++l) {
            const int dd = 1 << l;
            if (act && ((lane - lo) & ((dd << 1) - 1)) == 0 && lane + dd <= hi) s_q[lane] += s_q[lane + dd];
            lds_barrier();
        }
        double r = act ? s_q[lo] : 0.0;
        lds_barrier();
        return r;
    };
    auto sv = [&](int j) -> double {
        if constexpr (LO) return (double)sg[j] + (double)SL(j);
        else return (double)sg[j];
    };
    // stress content of this lane: its nodes plus the voids on them (a void's
    // volume is only ever written by the lane that owns its node)
    auto content = [&]() -> double {
        double q = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) if (j < cnt) q += (double)Vr_b[j] * sv(j);
        if (vmask) {
            for (int k = 0; k < nv; ++k) {
                int jv = d->vnode[inst * MAXV + k] - start;
                if (jv >= 0 && jv < cnt) q += d->B * d->vvol[inst * MAXV + k];
            }
        }
        return q;
    };
    double vs = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) if (j < cnt) vs += (double)Vr_b[j];
    const double Vtot = seg_sum(vs);
    const double Q0 = seg_sum(content());
    // stress at the next block's separator (kept in step with that lane)
    s_x[0][lane] = sg[0];
    if constexpr (LO) s_x[1][lane] = SL(0);
    lds_barrier();
    R sn = (act && !last) ? s_x[0][lane + 1] : (R)0;
    float snl = 0.f;                   // its low part (FP32 form)
    if constexpr (LO) snl = (act && !last) ? s_x[1][lane + 1] : 0.f;
    lds_barrier();

    for (int st = 0; st < h.n_steps; ++st) {
        // 1. residual dt (A sigma + f) in FP64 (flux differences are exact),
        //    rounded once for the solve: the step solves for the increment
        //    Each edge's flux dt g (s_right - s_left) is formed once and
        //    enters its two nodes with opposite signs.  Every node, past cnt
        //    too (finite values, zero increments below).
        R y[M];
        double r0_part = 0.0, qprev = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            y[j] = 0;
            const double sj = sv(j);
            const double sr = (j + 1 < cnt) ? sv(j + 1) : (LO ? (double)sn + (double)snl : (double)sn);
            const double qn = (double)gE[j + 1] * (sr - sj);
            double r = (double)fv[j] + qn;
            if (j > 0) r -= qprev;
            qprev = qn;
            if (j == 0) r0_part = r; else y[j] = (R)r;
        }
        if (vmask) {                           // Robin sinks at void nodes
            for (int k = 0; k < nv; ++k) {
                const int jv = d->vnode[inst * MAXV + k] - start;
                const double rb = dt * d->vrob[inst * MAXV + k];     // loaded with the node
                if (jv < 0 || jv >= cnt) continue;
#pragma unroll
                for (int j = 0; j < M; ++j)
                    if (j == jv) {
                        if (j == 0) r0_part -= rb * sv(0);
                        else y[j] = (R)((double)y[j] - rb * sv(j));
                    }
            }
        }
        // 2. interior solve with zero separator values (y overwrites the rhs).
        //    Past cnt: w = dinv = 0, so the backward sweep leaves y = 0 there
        //    and carries yn = 0 into the last node (whose coupling to the next
        //    block is the separator's, not the interior solve's).
        R yp = 0;
#pragma unroll
        for (int j = 1; j < M; ++j) { yp = (j == 1) ? y[1] : y[j] + (gE[j] * dinv[j - 1]) * yp; y[j] = yp; }
        R yn = 0;
#pragma unroll
        for (int j = M - 1; j >= 1; --j) {
            const R uj = gE[j + 1] * dinv[j];
            yn = y[j] * dinv[j] + uj * yn;
            y[j] = yn;
        }
        R yF = 0, yL = 0, sL = sg[0];
        float sLl = 0.f;
        if constexpr (LO) sLl = SL(0);
        if (cnt >= 2) {
            yF = y[1];
#pragma unroll
            for (int j = 1; j < M; ++j)
                if (j == cnt - 1) {
                    yL = y[j]; sL = sg[j];
                    if constexpr (LO) sLl = SL(j);
                }
        }
        // 3. exchange with the previous block: its last interior value and its
        //    last node's stress (for the separator's residual), then PCR
        s_e[0][lane] = yL;
        s_e[1][lane] = sL;
        if constexpr (LO) s_e[2][lane] = sLl;
        lds_barrier();
        R Rk = 0;
        if (act) {
            double r0 = r0_part;
            R yLp = 0;
            if (!first) {
                yLp = s_e[0][lane - 1];
                double sp = (double)s_e[1][lane - 1];
                if constexpr (LO) sp += (double)s_e[2][lane - 1];
                r0 += (double)gE[0] * (sp - sv(0));
            }
            Rk = (R)r0 + gE[0] * yLp + e_first() * yF;
        }
        int buf = 1;
#pragma unroll
        for (int l = 0; l < LEV; ++l) {
            const int dd = 1 << l;
            constexpr int P = WG / 2;
            s_xp[buf][P + lane] = Rk;
            lds_barrier();
            // both neighbours read unconditionally (past the workgroup's ends
            // the zero pads; every lane wrote a finite value): a missing
            // coupling has a zero multiplier
            const R al_l = s_al[l][lane], ga_l = s_ga[l][lane];
            const R xm = s_xp[buf][P + lane - dd];
            const R xp = s_xp[buf][P + lane + dd];
            Rk = Rk + al_l * xm + ga_l * xp;
            buf ^= 1;
        }
        const R xk = Rk * dfin;
        s_x[buf][lane] = xk;
        lds_barrier();
        const R xn = (act && !last) ? s_x[buf][lane + 1] : (R)0;
        // 4. increments and new stress
        if constexpr (LO) {
            auto put = [&](int j, double v) {      // state <- v as sg + sl
                const R hv = (R)v;
                sg[j] = hv;
                SLset(j, (float)(v - (double)hv));
            };
            put(0, sv(0) + (double)xk);
#pragma unroll
            for (int j = 1; j < M; ++j) put(j, sv(j) + (double)(y[j] + al[j] * xk + be[j] * xn));
            const double v = (double)sn + (double)snl + (double)xn;
            sn = (R)v;
            snl = (float)(v - (double)sn);
        } else {
            sg[0] += xk;
#pragma unroll
            for (int j = 1; j < M; ++j) sg[j] += y[j] + al[j] * xk + be[j] * xn;
            sn += xn;
        }

        // void growth on the lanes owning void nodes (eq. 15 accounting)
        if (vmask) {
            for (int k = 0; k < nv; ++k) {
                // every load of the void's record issued before the test and
                // the stores: two dependent rounds (record, then its node's
                // drive and its segment's geometry) instead of a chain
                const int q = inst * MAXV + k;
                const int jv = d->vnode[q] - start;
                const int e = d->vseg[q];
                const double vol0 = d->vvol[q], rob = d->vrob[q];
                const int phase = d->vphase[q];
                if (jv < 0 || jv >= cnt) continue;
                const R fvv = dtf_g[(size_t)(start + jv) * S + s];
                const double W = d->w[e], H = d->h[e], Le = d->len[e];
                R sh = 0;
                float slo = 0.f;
#pragma unroll
                for (int j = 0; j < M; ++j)
                    if (j == jv) {
                        sh = sg[j];
                        if constexpr (LO) slo = SL(j);
                    }
                double svv = (double)sh;
                if constexpr (LO) svv += (double)slo;
                const double vol = vol0 + (dt * rob * svv + (double)fvv) / d->B;
                d->vvol[q] = vol;
                const double l = fmin(vol / (W * H), Le);
                d->vlen[q] = l;
                if (phase == 0 && l >= W) {
                    d->vphase[q] = 1;
                    if (d->vearly[q]) {
                        d->open[(size_t)s * d->n_res + e] = 1;
                        *d->open_dirty = 1u;
                    }
                }
            }
        }

        // nucleation: any non-void node at or above its critical stress?
        bool cand = false;
        if (act) {
            if constexpr (LO) {
#pragma unroll
                for (int j = 0; j < M; ++j)
                    if (j < cnt && sg[j] >= scpre && !((vmask >> j) & 1u)) cand = true;
                if (cand) {
                    cand = false;
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        if (j < cnt && !((vmask >> j) & 1u) && sv(j) >= (double)sc_g[(size_t)(start + j) * S + s])
                            cand = true;
                }
            } else {
#pragma unroll
                for (int j = 0; j < M; ++j)
                    if (j < cnt && sg[j] >= scmin && !((vmask >> j) & 1u)) cand = true;
                if (cand) {
                    cand = false;
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        if (j < cnt && !((vmask >> j) & 1u) && sg[j] >= sc_g[(size_t)(start + j) * S + s])
                            cand = true;
                }
            }
        }
        if (wg_any<WG>(cand, s_vote, lane)) {    // the step's reduction barriers separate two calls
            // peak candidate per instance, then the lowest node within the tie window
            if constexpr (LO) {
                double lm = -INFINITY;
                if (cand) {
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        if (j < cnt && !((vmask >> j) & 1u) && sv(j) >= (double)sc_g[(size_t)(start + j) * S + s])
                            lm = sv(j) > lm ? sv(j) : lm;
                }
                s_q[lane] = lm;
            } else {
                R lm = (R)(-INFINITY);
                if (cand) {
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        if (j < cnt && !((vmask >> j) & 1u) && sg[j] >= sc_g[(size_t)(start + j) * S + s])
                            lm = sg[j] > lm ? sg[j] : lm;
                }
                s_q[lane] = (double)lm;
            }
            lds_barrier();
#pragma unroll
            for (int l = 0; l < LEV; ++l) {
                const int dd = 1 << l;
                if (act && ((lane - lo) & ((dd << 1) - 1)) == 0 && lane + dd <= hi)
                    s_q[lane] = fmax(s_q[lane], s_q[lane + dd]);
                lds_barrier();
            }
            const double mxd = act ? s_q[lo] : -INFINITY;
            lds_barrier();
            const bool any = act && mxd != -INFINITY;
            const bool has = any && nv < d->max_voids;
            int loc = 0x7fffffff;
            if constexpr (LO) {
                const double thr = mxd - 1e-12 * (mxd < 0 ? -mxd : mxd);
                if (has && cand) {
#pragma unroll
                    for (int j = M - 1; j >= 0; --j)
                        if (j < cnt && !((vmask >> j) & 1u) && sv(j) >= thr &&
                            sv(j) >= (double)sc_g[(size_t)(start + j) * S + s])
                            loc = start + j;
                }
            } else {
                const R mx = (R)mxd;
                const R thr = mx - (R)1e-12 * (mx < 0 ? -mx : mx);
                if (has && cand) {
#pragma unroll
                    for (int j = M - 1; j >= 0; --j)
                        if (j < cnt && !((vmask >> j) & 1u) && sg[j] >= thr &&
                            sg[j] >= sc_g[(size_t)(start + j) * S + s])
                            loc = start + j;
                }
            }
            s_q[lane] = (double)loc;
            lds_barrier();
#pragma unroll
            for (int l = 0; l < LEV; ++l) {
                const int dd = 1 << l;
                if (act && ((lane - lo) & ((dd << 1) - 1)) == 0 && lane + dd <= hi)
                    s_q[lane] = fmin(s_q[lane], s_q[lane + dd]);
                lds_barrier();
            }
            const int v = act ? (int)s_q[lo] : 0x7fffffff;
            lds_barrier();
            if (any && !has && lane == lo) d->n_suppressed[inst] += 1;
            if (has && v != 0x7fffffff) {
                if (lane == lo) {
                    const int k = nv;
                    const int q = inst * MAXV + k;
                    d->vnode[q] = v;
                    d->vvol[q] = 0.0;
                    d->vlen[q] = 0.0;
                    d->vrob[q] = chain_robin_weight(*d, v, s);
                    const int hs = chain_host_segment(*d, v, s);
                    d->vseg[q] = hs;
                    d->vphase[q] = 0;
                    d->vearly[q] = d->vert[v] >= 0 ? d->via_up[d->vert[v]] : 0;
                    d->vstep[q] = h.step0 + st;
                    d->nv[inst] = k + 1;
                    const unsigned int qe = atomicAdd(d->ev_count, 1u);
                    if ((int)qe < d->ev_cap) {
                        int *E = d->events + (size_t)qe * EV_WORDS;
                        E[0] = s; E[1] = t; E[2] = h.step0 + st; E[3] = v; E[4] = hs;
                    }
                }
                nv += 1;
            }
            __syncthreads();   // void records written by lane `lo` visible to the owner lane
            if (act) refresh_vmask();
            factor();
        }

        // conservation projection (rounding-level)
        if (h.proj_every > 0 && ((st + 1) % h.proj_every == 0 || st + 1 == h.n_steps)) {
            const double Q = seg_sum(content());
            if constexpr (LO) {
                const double corr = act ? (Q0 - Q) / Vtot : 0.0;
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    const double v = sv(j) + corr;
                    sg[j] = (R)v;
                    SLset(j, (float)(v - (double)sg[j]));
                }
                const double v = (double)sn + (double)snl + corr;
                sn = (R)v;
                snl = (float)(v - (double)sn);
            } else {
                const R corr = act ? (R)((Q0 - Q) / Vtot) : (R)0;
#pragma unroll
                for (int j = 0; j < M; ++j) sg[j] += corr;
                sn += corr;
            }
        }
    }
    // ---- write back ----
#pragma unroll
    for (int j = 0; j < M; ++j)
        if (j < cnt) {
            const size_t x = (size_t)(start + j) * S + s;
            sig[x] = sg[j];
            if constexpr (LO) {
                if (sig_lo) sig_lo[x] = SL(j);
            } else if constexpr (sizeof(R) == 4) {
                if (sig_lo) sig_lo[x] = 0.f;
            }
        }
}

void launch_chain(const Dev &d, const Dev *d_dev, bool fp32, int n_steps, int step0, hipStream_t st)
{
    ChainHot h;
    h.sigma = d.sigma; h.sig_lo = d.sig_lo; h.Vr = d.Vr; h.dtf = d.dtf; h.sc = d.sc;
    h.lane_inst = d.lane_inst; h.lane_blk = d.lane_blk; h.tree_off = d.tree_off;
    h.sample_active = d.sample_active; h.inst_active = d.inst_active;
    h.dev = d_dev;
    h.S = d.S; h.n_steps = n_steps; h.step0 = step0; h.proj_every = 16;
    h.dt = d.dt;
    // the batch's workgroup size (lanes): the smallest that holds its longest
    // chain, or the one the autotuner measured fastest
    const bool dense = d.chain_occ == 4;    // FP32 64-512 lanes only (checked at creation)
    const bool mid = d.chain_occ == 3;      // FP32 256 and 512 lanes only
    const int G = d.n_chain_wg;
    if (G > 0) {
        if (fp32) {
            if (d.chain_wg == 64) {
                if (dense) k_chain<float, CHAIN_M32, 64, 4><<<G, 64, 0, st>>>(h);
                else k_chain<float, CHAIN_M32, 64, 1><<<G, 64, 0, st>>>(h);
            } else if (d.chain_wg == 128) {
                if (dense) k_chain<float, CHAIN_M32, 128, 4><<<G, 128, 0, st>>>(h);
                else k_chain<float, CHAIN_M32, 128, 1><<<G, 128, 0, st>>>(h);
            } else if (d.chain_wg == 256) {
                if (dense) k_chain<float, CHAIN_M32, 256, 4><<<G, 256, 0, st>>>(h);
                else if (mid) k_chain<float, CHAIN_M32, 256, 3><<<G, 256, 0, st>>>(h);
                else k_chain<float, CHAIN_M32, 256, 1><<<G, 256, 0, st>>>(h);
            } else if (d.chain_wg == 512) {
                if (dense) k_chain<float, CHAIN_M32, 512, 4><<<G, 512, 0, st>>>(h);
                else if (mid) k_chain<float, CHAIN_M32, 512, 3><<<G, 512, 0, st>>>(h);
                else k_chain<float, CHAIN_M32, 512, 1><<<G, 512, 0, st>>>(h);
            } else {
                if (d.chain_m == CHAIN_M32W)
                    k_chain<float, CHAIN_M32W, CHAIN_WG32, 1><<<G, CHAIN_WG32, 0, st>>>(h);
                else
                    k_chain<float, CHAIN_M32, CHAIN_WG32, 1><<<G, CHAIN_WG32, 0, st>>>(h);
            }
        } else {
            if (d.chain_wg == 64) k_chain<double, CHAIN_M64, 64, 1><<<G, 64, 0, st>>>(h);
            else if (d.chain_wg == 128) k_chain<double, CHAIN_M64, 128, 1><<<G, 128, 0, st>>>(h);
            else if (d.chain_wg == 256) k_chain<double, CHAIN_M64, 256, 1><<<G, 256, 0, st>>>(h);
            else k_chain<double, CHAIN_M64, CHAIN_WG64, 1><<<G, CHAIN_WG64, 0, st>>>(h);
        }
    }
}

}  // namespace em
