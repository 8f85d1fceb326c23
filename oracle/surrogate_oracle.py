"""FP64 CPU oracle of the learned screen: per-tree features, the MLP forward
and backward passes, Adam, and the lazy-activation schedule.

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark's
CPU-baseline leg, never by the product package; it shares no code with the
HIP path.

The learned screen has no counterpart in EMSpice 3; it is this library's own
addition in front of the transient stage.  What it computes is defined here in
plain numpy:

* Features (16 per (tree, sample)) from quantities the paper defines: segment
  lengths and current densities (Sec. III-C), the Arrhenius diffusivity
  kappa = D0 exp(-Ea/kT) B Omega/(kT) (Sec. III-D), the zero-flux steady
  stress of the immortality screen (Sec. III-B) against the critical stress,
  and the diffusion time L^2/(pi^2 kappa) of the slowest Korhonen mode over
  the span between the stress peak and the neutral point of the steady
  profile; early-time scales from the Korhonen solution of a semi-infinite
  wire with a blocked end, sigma(0, t) = 2 g sqrt(kappa t / pi) for a drive
  (steady stress gradient) g, and the fast part of the tree (edges within a
  factor 4 of the largest diffusivity).
* A multilayer perceptron 16 -> 256 -> 256 -> 256 -> 1 with GELU activations
  in the exact erf form (Hendrycks & Gimpel, 2016), predicting
  log10(t_nuc / 1e8 s).  Precision contract of the device path, mirrored
  here: the operands of the three hidden-layer products (forward and
  backward) are rounded to float32 and then to bfloat16 (round to nearest,
  ties to even) before an exact-product, wide-accumulation contraction; the
  output layer, bias, GELU and loss are unrounded.  ``rnd=None`` switches the
  rounding off, which makes the backward pass the exact gradient of the
  float64 network (pinned by central finite differences).
* Mean-squared-error loss and Adam with bias-corrected moments (Kingma & Ba,
  ICLR 2015, Algorithm 1).
* Lazy activation: a steady-state-mortal tree whose predicted nucleation time
  exceeds margin x (end of the first aging interval) is deferred; it must be
  active before the aging interval ending at the first t_{k+1} with
  t_hat <= margin x t_{k+1}.  Activation is checked before the intervals
  k = 1, 4, 16, 64, ... only, each check activating what is due by t_{4k}, and
  an activated tree is caught up by replaying the stored per-interval current
  densities from t = 0.
"""
from __future__ import annotations

import math

import numpy as np

NF, HID = 16, 256
T_REF = 1e8            # s; the network predicts log10(t_nuc / T_REF)
E_CHG = 1.602176634e-19
K_B = 1.380649e-23

# flat parameter layout (row-major [out][in] weights)
SHAPES = [("W1", (HID, NF)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (HID, HID)), ("b3", (HID,)), ("w4", (HID,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


# ---------------------------------------------------------------------------
# bfloat16 rounding: float64 -> float32 (IEEE round to nearest) -> the upper
# 16 bits of the float32 pattern, rounding to nearest with ties to even.
# ---------------------------------------------------------------------------
def bf16(x):
    x32 = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


def _erf(z):
    return np.vectorize(math.erf, otypes=[np.float64])(z)


def gelu(z):
    z = np.asarray(z, np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz of z Phi(z) = Phi(z) + z phi(z)."""
    z = np.asarray(z, np.float64)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _ident(x):
    return np.asarray(x, np.float64)


def forward(p, X, rnd=bf16):
    """Network output y [n] and the cache of pre-/post-activations."""
    r = rnd if rnd is not None else _ident
    P = unpack(p)
    X = np.asarray(X, np.float64)
    Z1 = r(X) @ r(P["W1"]).T + P["b1"]
    H1 = gelu(Z1)
    Z2 = r(H1) @ r(P["W2"]).T + P["b2"]
    H2 = gelu(Z2)
    Z3 = r(H2) @ r(P["W3"]).T + P["b3"]
    H3 = gelu(Z3)
    y = H3 @ P["w4"] + P["b4"][0]
    return y, dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2, Z3=Z3, H3=H3)


def loss_and_grad(p, X, t, rnd=bf16):
    """Mean squared error (1/n) sum (y - t)^2 and its gradient (flat layout)
    by the chain rule through the three GELU layers."""
    r = rnd if rnd is not None else _ident
    P = unpack(p)
    y, c = forward(p, X, rnd)
    t = np.asarray(t, np.float64)
    n = y.size
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / n
    g = {}
    g["w4"] = c["H3"].T @ dy
    g["b4"] = np.array([dy.sum()])
    dZ3 = np.outer(dy, P["w4"]) * gelu_grad(c["Z3"])
    g["W3"] = r(dZ3).T @ r(c["H2"])
    g["b3"] = dZ3.sum(axis=0)
    dZ2 = (r(dZ3) @ r(P["W3"])) * gelu_grad(c["Z2"])
    g["W2"] = r(dZ2).T @ r(c["H1"])
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (r(dZ2) @ r(P["W2"])) * gelu_grad(c["Z1"])
    g["W1"] = r(dZ1).T @ r(c["X"])
    g["b1"] = dZ1.sum(axis=0)
    return loss, pack(g)


def grad_magnitude(p, X, t, rnd=bf16):
    """Per-parameter sum of the magnitudes of the terms that make up the
    gradient of loss_and_grad: the same chain rule with every factor replaced
    by its absolute value (the upstream signals |dZ| themselves built from
    magnitudes).  A perturbation of relative size e of every operand of those
    sums moves each gradient entry by at most about e times this value, which
    is the scale of the element-wise bound on a reduced-precision gradient."""
    r = rnd if rnd is not None else _ident
    P = unpack(p)
    y, c = forward(p, X, rnd)
    t = np.asarray(t, np.float64)
    n = y.size
    ady = 2.0 * np.abs(y - t) / n
    g = {}
    g["w4"] = np.abs(c["H3"]).T @ ady
    g["b4"] = np.array([ady.sum()])
    a3 = np.outer(ady, np.abs(P["w4"])) * np.abs(gelu_grad(c["Z3"]))
    g["W3"] = np.abs(r(a3)).T @ np.abs(r(c["H2"]))
    g["b3"] = a3.sum(axis=0)
    a2 = (np.abs(r(a3)) @ np.abs(r(P["W3"]))) * np.abs(gelu_grad(c["Z2"]))
    g["W2"] = np.abs(r(a2)).T @ np.abs(r(c["H1"]))
    g["b2"] = a2.sum(axis=0)
    a1 = (np.abs(r(a2)) @ np.abs(r(P["W2"]))) * np.abs(gelu_grad(c["Z1"]))
    g["W1"] = np.abs(r(a1)).T @ np.abs(r(c["X"]))
    g["b1"] = a1.sum(axis=0)
    return pack(g)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected first and second moments); t >= 1 is
    the step number.  Returns the new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Features
# ---------------------------------------------------------------------------
def kappa0(T, mat):
    """Arrhenius diffusivity kappa = D0 exp(-Ea/kT) B Omega / (kT) (Sec. III-D)."""
    T = np.asarray(T, np.float64)
    kT = K_B * T
    return mat["D0"] * np.exp(-mat["Ea_eV"] * E_CHG / kT) * mat["B"] * mat["Omega"] / kT


FEATURE_NAMES = ["log10 Ltot/um", "log10 Lpath/um", "nseg/8", "njunc/4", "log10 jmax/1e9",
                 "log10 jmean/1e9", "log10 kmean/1e-15", "log10 kpk/1e-15", "r = max sss/sc",
                 "log10 max(r-1,1e-6)", "log10 tau_pk/s - 8", "(Tpk-300)/100"]


def features(topo, grid, mat, jseg, xi_k, T, sig_ss, sc):
    """[n_trees][16] features of one sample.

    topo: the tree partition; jseg [n_res] current density; xi_k [n_res]
    diffusivity multipliers; T, sig_ss, sc [n_stress]: node temperature, the
    screen's zero-flux steady stress, and the node critical stress.

    The peak node p is the first node (lowest index) of largest finite
    sig_ss / sc.  Its length scale Lpk is the distance along the root path
    coordinate, |d(i) - d(p)| with d the distance from the root, to the
    nearest node whose steady stress does not exceed sigma_T (floored at
    0.1 um); on a straight line this is the distance to the neutral point of
    the steady profile.  kappa_pk is the mean diffusivity of the edges at p,
    tau_pk = Lpk^2 / (pi^2 kappa_pk).

    Early-time scales over the edges e = (parent(i), i) of length l_e =
    segment length / N and diffusivity kappa_e: the steady drive g_e =
    |sig_ss(i) - sig_ss(parent)| / l_e; with ds_e = max(min(sc) of the two
    ends - sigma_T, 1e3 Pa) the time pi ds_e^2 / (4 kappa_e g_e^2) at which a
    blocked end of a semi-infinite wire with that drive reaches sc (edges
    with g_e > 0; the least one, clamped to [1, 1e16] s); kappa_max; the fast
    edges (kappa_e >= kappa_max / 4): their length L_f (floored at 0.1 um)
    and the stress they could build if blocked on both sides, sum of
    g_e l_e / 2, over ds_min = max(min over nodes of sc - sigma_T, 1e3 Pa)
    (clamped to 10); and L_f^2 / (pi^2 kappa_max).
    """
    N = topo.N
    out = np.zeros((topo.n_trees, NF))
    nchild = np.zeros(topo.n_stress, np.int64)
    for i in range(topo.n_stress):
        if topo.parent[i] >= 0:
            nchild[topo.parent[i]] += 1
    children = [[] for _ in range(topo.n_stress)]
    for i in range(topo.n_stress):
        if topo.parent[i] >= 0:
            children[topo.parent[i]].append(i)

    def edge_kappa(i):          # edge (parent(i), i)
        p = int(topo.parent[i])
        return xi_k[int(topo.seg[i])] * kappa0(0.5 * (T[i] + T[p]), mat)

    for t in range(topo.n_trees):
        i0, i1 = int(topo.tree_off[t]), int(topo.tree_off[t + 1])
        segs = sorted({int(topo.seg[i]) for i in range(i0, i1) if topo.parent[i] >= 0})
        lens = np.array([grid.res_len[e] for e in segs])
        js = np.array([abs(jseg[e]) for e in segs])
        Ltot = lens.sum()
        dist = {i0: 0.0}
        kap = []
        njunc = 0
        for i in range(i0, i1):
            p = int(topo.parent[i])
            deg = nchild[i] + (1 if p >= 0 else 0)
            njunc += deg >= 3
            if p >= 0:
                dist[i] = dist[p] + grid.res_len[int(topo.seg[i])] / N
                kap.append(edge_kappa(i))
        Lpath = max(dist.values())
        kmean = float(np.mean(kap))
        # peak of the steady stress over the critical stress
        pk, rr = -1, -np.inf
        for i in range(i0, i1):
            if np.isfinite(sig_ss[i]):
                q = sig_ss[i] / sc[i]
                if q > rr:
                    pk, rr = i, q
        if pk < 0:
            pk, rr = i0, -10.0
        rr = min(max(rr, -10.0), 10.0)
        lpk = np.inf
        for i in range(i0, i1):
            if sig_ss[i] <= mat["sigma_T"]:
                lpk = min(lpk, abs(dist[i] - dist[pk]))
        lpk = max(lpk if np.isfinite(lpk) else Lpath, 1e-7)
        ke = [edge_kappa(c) for c in children[pk]]
        if topo.parent[pk] >= 0:
            ke.append(edge_kappa(pk))
        kpk = float(np.mean(ke))
        tau = lpk ** 2 / (math.pi ** 2 * kpk)
        # early-time scales
        ds_min = max(min(sc[i] for i in range(i0, i1)) - mat["sigma_T"], 1e3)
        edges = [(i, int(topo.parent[i])) for i in range(i0, i1) if topo.parent[i] >= 0]
        k_e = {i: edge_kappa(i) for i, _ in edges}
        l_e = {i: grid.res_len[int(topo.seg[i])] / N for i, _ in edges}
        kmax = max(k_e.values()) if edges else 0.0
        t_blk = math.inf
        Lf, Sf = 0.0, 0.0
        for i, p in edges:
            dpsi = abs(sig_ss[i] - sig_ss[p])
            g = dpsi / l_e[i]
            if math.isfinite(g) and g > 0:
                ds = max(min(sc[i], sc[p]) - mat["sigma_T"], 1e3)
                t_blk = min(t_blk, math.pi * ds ** 2 / (4 * k_e[i] * g ** 2))
            if k_e[i] >= 0.25 * kmax:
                Lf += l_e[i]
                if math.isfinite(dpsi):
                    Sf += 0.5 * dpsi
        t_blk = min(max(t_blk, 1.0), 1e16)
        kmax = max(kmax, 1e-30)
        Lf = max(Lf, 1e-7)
        out[t] = [math.log10(Ltot / 1e-6), math.log10(Lpath / 1e-6), len(segs) / 8.0, njunc / 4.0,
                  math.log10(max(js.max(), 1e3) / 1e9), math.log10(max((lens * js).sum() / Ltot, 1e3) / 1e9),
                  math.log10(kmean / 1e-15), math.log10(kpk / 1e-15), rr,
                  math.log10(max(rr - 1.0, 1e-6)), math.log10(tau) - 8.0,
                  (float(T[pk]) - 300.0) / 100.0,
                  math.log10(t_blk) - 8.0, math.log10(kmax / 1e-15), min(Sf / ds_min, 10.0),
                  math.log10(Lf ** 2 / (math.pi ** 2 * kmax)) - 8.0]
    return out


# ---------------------------------------------------------------------------
# Lazy activation
# ---------------------------------------------------------------------------
def t_hat(y):
    return T_REF * np.power(10.0, np.asarray(y, np.float64))


def activation_interval(that, margin, K, dt):
    """Index k of the aging interval (ending at t_{k+1} = (k+1) K dt) before
    which a tree predicted to nucleate at ``that`` must be active: the
    smallest k >= 0 with that <= margin t_{k+1}."""
    T1 = margin * K * dt
    return np.maximum(0, np.ceil(np.asarray(that) / T1) - 1).astype(np.int64)


def activation_check(a):
    """Interval before which a deferred tree whose activation interval is
    a >= 1 is activated when the checks run only before the intervals
    c = 1, 4, 16, 64, ... and each activates what is due by t_{4c}, the end of
    the interval before the next check: the largest power of four <= a (the
    check c with c <= a < 4c)."""
    a = np.asarray(a, np.int64)
    out = np.zeros_like(a)
    for idx, v in np.ndenumerate(a):
        c = 1
        while 4 * c <= v:
            c *= 4
        out[idx] = c
    return out
