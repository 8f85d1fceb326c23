"""Benchmark of the coupled EM/TM stress + IR-drop hot path on one MI355X.

A step is one full pass of the hot path over the four-layer full-chip grid
(2000x2000 routing grid, 84k trees, 8.8M stress nodes): IR solve,
backward-Euler stress stepping of every tree (2000 steps over ten years,
FP32 stress with FP64 void/dR accumulators), nucleation and void growth,
resistance write-back and an IR re-solve every 50 steps, until the 10 %
IR-drop failure or the horizon.  The batch is built (netlist copied, trees
partitioned, statics and the Joule pre-pass evaluated) before the timed
region; each timed step resets it to t = 0 and runs it to time-to-failure.

Prints ONE JSON line (rank 0).  Metric: stress-node-steps/s (sum over stepped
trees of stress nodes x steps, divided by wall time).  Also reported: the
roofline of the dominant kernel (the stepping kernel, timed with HIP events on
its stream inside the library; against the streamed HBM roofline, or the FP32
vector-ALU bound where the resident kernel beats the former), the plain FP64
GPU form (one tree per lane, FP64) over one aging interval, the FP64 oracle on
host cores over a bounded sample of the same workload, the same measurement
on the 400x400 two-layer grid with and without voids, and Monte Carlo
samples/s to TTF: 64 samples of the full chip, 1024 samples of the 96x96
sparse-via grid (failures within the horizon; checked against the FP64
oracle on 64 samples), the 32x32 mesh, further sampled inputs, a thermal-map
sweep and the learned screen.
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, TFLOP/s
# BE step of a node with the factorisation reused: right-hand side V s + dt f,
# forward elimination, back substitution -- about four fused multiply-adds
FLOPS_PER_NODE_STEP = 8
BYTES_PER_NODE_STEP = {0: 40.0, 1: 20.0}   # sigma r/w, 1/d, l, dt*f (FP64 / FP32)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _oracle_grid(name):
    """The CPU baseline's input: the named workload's grid in trees-only mode
    with seeded prescribed current densities (the stepping cost does not
    depend on their values), FP64 numerics."""
    from paper_2604_10743_amd import synth
    g, mat, run, _ = synth.workload(name)
    run = dict(run, prec=0, joule=0)
    return synth.with_prescribed_j(g, synth.seeded_current_density(g, 777)), mat, run


def _oracle_trees_worker(job):
    """One host process of the all-core oracle baseline: BE steps of trees
    [t0, t1) of the named workload; returns node-steps."""
    name, t0, t1, n_steps = job
    import numpy as np
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    g, mat, run = _oracle_grid(name)
    topo = O.topology(g, run["intervals_per_seg"])
    sim = O.SampleSim(g, mat, run, topo)
    sim.set_j(g.seg_j)
    act = np.zeros(topo.n_trees, np.uint8)
    act[t0:t1] = 1
    sim.set_active(act)
    sim.steps(n_steps, 0)
    return int(topo.tree_off[t1] - topo.tree_off[t0]) * n_steps


def _oracle_mc_worker(job):
    """One host process of the all-core Monte Carlo oracle baseline: the
    named workload's samples ``ids`` run to TTF by the FP64 oracle."""
    name, ids, var = job
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    from paper_2604_10743_amd import synth
    g, mat, run, mc = synth.workload(name)
    mc = dict(mc, **(var or {}))
    topo = O.topology(g, run["intervals_per_seg"])
    for s in ids:
        O.run_sample(g, mat, run, mc, s, topo=topo)
    return len(ids)


def host_cpu():
    """Host CPU model and logical core count (for the oracle baselines)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cores": os.cpu_count()}


def kernel_code_sha(kernel_src: str) -> str:
    """SHA-256 (first 16 hex digits) of a kernel source's device code: the
    file up to its host-side launcher (`void launch_`), so that a change of
    the launch dispatch alone does not void the counters."""
    import hashlib
    txt = open(os.path.join(ROOT, kernel_src)).read()
    cut = txt.find("\nvoid launch_")
    return hashlib.sha256((txt if cut < 0 else txt[:cut + 1]).encode()).hexdigest()[:16]


def measured_traffic(kernel_src: str, profile_md: str, kernel: str | None = None):
    """HBM bytes per launch from the committed PMC summary (one JSON block per
    instantiation measured), or None when the kernel's device code changed
    since the counters were taken (or none was taken on this instantiation)."""
    try:
        txt = open(os.path.join(ROOT, profile_md)).read()
        sha = kernel_code_sha(kernel_src)
        for part in txt.split("```json")[1:]:
            pm = json.loads(part.split("```", 1)[0])
            if pm.get("source_sha256_16") != sha:
                continue
            if kernel is not None and pm.get("kernel", kernel) != kernel:
                continue
            return pm["traffic_bytes_per_launch"]
        return None
    except (OSError, ValueError, KeyError):
        return None


def surrogate_leg(args):
    """Learned screen: labels from the library's own transient runs on random
    cold long-line grids (trees-only, currents of the t = 0 IR solve held
    fixed, labels to 100 years), training with the BF16 MFMA kernels, a bias
    shift calibrated on the held-out pairs whose tree nucleated within the
    label horizon, then the screened and the unscreened Monte Carlo run to TTF
    of the screen_cold workload (results compared sample by sample)."""
    import numpy as np
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import surrogate, synth

    g, mat, run, mc = synth.workload("screen_cold")
    mc = dict(mc, n_samples=args.sur_samples)
    lab_run = dict(run, dt=run["dt"] * 2.5)      # label steps of 2.5 dt, to 100 years
    # the FP32 guard band re-runs the same samples in FP64 with and without
    # the screen (and costs more than the FP32 run on this workload): off in
    # both runs compared here
    run = dict(run, guard_band=0.0, guard_ttf=0.0)
    horizon = 4 * run["n_steps"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, y, infos = surrogate.training_set(11, args.sur_grids, mat, lab_run, args.sur_label_samples, horizon,
                                         log=log, family="cold_lines")
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    Xv, yv, _ = surrogate.training_set(12, 4, mat, lab_run, 256, horizon, family="cold_lines")
    model = P.MLP(synth.init_mlp_params(1, out_bias=float(y.mean().item())))
    n = int(X.shape[0])
    batch = min(4096, max(256, n // 16))
    steps = args.sur_steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    surrogate.train(model, X, y, steps, batch=batch, lr=1e-3, lr_final=1e-4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    flop_step = 3 * 2 * batch * (16 * 256 + 2 * 256 * 256)      # hidden-layer GEMMs, fwd + 2x bwd
    train_loss = model.grad(X, y)[0]
    val_loss = model.grad(Xv, yv)[0]
    ratio = 10.0 ** (model.forward(Xv).cpu().numpy() - yv.cpu().numpy())
    # bias shift: a fraction q of the held-out trees that nucleated within the
    # label horizon are predicted no later than they nucleated
    q = args.sur_quantile
    shift = surrogate.calibrate(model, Xv, yv, q, y_cap=surrogate.label_cap(lab_run, horizon))
    margin = 1.0
    log(f"bench: surrogate trained on {n} pairs: loss {train_loss:.4f}, held-out {val_loss:.4f}")

    def mc_run(with_model, reps=3):
        B = P.Batch(g, mat, run, mc)
        best = None
        for _ in range(reps):                   # the first run of a batch builds its solver state
            B.reset()
            if with_model:
                B.surrogate_screen(model, margin)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = B.run_to_ttf()
            torch.cuda.synchronize()
            w = time.perf_counter() - t0
            if best is None or w < best[2]:
                best = (res, B.info(), w)
        B.close()
        return best

    r0, i0, w0 = mc_run(False)
    r1, i1, w1 = mc_run(True)
    # inference throughput of the screen model on this workload's feature rows
    Bf = P.Batch(g, mat, run, mc)
    Bf.ir_solve()
    Xf = Bf.features()
    Bf.close()
    model.forward(Xf)
    torch.cuda.synchronize()
    reps = 20
    t0 = time.perf_counter()
    for _ in range(reps):
        model.forward(Xf)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / reps
    flop_inf = 2 * int(Xf.shape[0]) * (16 * 256 + 2 * 256 * 256)
    same = all((a["failed"] == b["failed"]) and (a["outer_idx"] == b["outer_idx"]) and
               (np.isnan(a["ttf_s"]) and np.isnan(b["ttf_s"]) or a["ttf_s"] == b["ttf_s"]) and
               a["final_drop"] == b["final_drop"] and a["n_failed_segs"] == b["n_failed_segs"]
               for a, b in zip(r0, r1))
    ttf = np.array([r["ttf_s"] for r in r1 if r["failed"]])
    S = mc["n_samples"]
    return {"metric": "MC samples/s to TTF, learned screen on", "value": S / w1, "unit": "samples/s",
            "workload": f"screen_cold: 64 x 257 long-line grid at 310 K with two hotspots, {S} samples, "
                        f"20% CoV on kappa and sigma_crit, FP32 (guard band off), margin {margin:g}, "
                        f"best of 3 runs each",
            "unscreened_samples_per_s": S / w0, "speedup": w0 / w1,
            "node_steps": i1["node_steps"], "node_steps_unscreened": i0["node_steps"],
            "n_deferred": i1["n_deferred"], "n_activated": i1["n_activated"],
            "n_late": i1["n_late"], "n_violations": i1["n_violations"], "n_screen_rerun": i1["n_screen_rerun"],
            "results_identical": bool(same), "calibration_quantile": q,
            "ir_ms": i1["ir_ms"], "ir_ms_unscreened": i0["ir_ms"], "step_kernel_ms": i1["step_kernel_ms"],
            "step_kernel_ms_unscreened": i0["step_kernel_ms"],
            "n_fail": int(ttf.size), "ttf_mean_y": float(ttf.mean() / 3.15576e7) if ttf.size else None,
            "surrogate_ms": i1["surrogate_ms"],
            "inference": {"rows": int(Xf.shape[0]), "ms": t_inf * 1e3, "mfma_tflops": flop_inf / t_inf / 1e12,
                          "mfma_frac_of_bf16_peak": flop_inf / t_inf / 2.5e15},
            "training": {"pairs": n, "label_grids": args.sur_grids, "label_samples": args.sur_label_samples,
                         "label_s": t_label, "batch": batch, "steps": steps, "train_s": t_train,
                         "mfma_tflops": flop_step * steps / t_train / 1e12,
                         "mfma_frac_of_bf16_peak": flop_step * steps / t_train / 2.5e15,
                         "loss": train_loss, "heldout_loss": val_loss,
                         "heldout_ratio_pct_0.1_1_50_99": np.percentile(ratio, [0.1, 1, 50, 99]).tolist(),
                         "calibration_shift_decades": shift}}


MC_DESC = {
    "mc_grid": "96x96 two-layer sparse-via P/G grid (via every 32 nodes, 16 pads, 12309 nodes, "
               "169 line trees), 330 K + 6 hotspots, worst initial drop 7 %",
    "mc_mesh": "32x32 two-layer mesh with 4 corner pads, M1 rows cut into 213 trees, 378 K",
    "fullchip": "the full-chip grid of the headline (84k trees, 8.8M stress nodes, 515k grid nodes), "
                "340 K + 12 hotspots with the Joule pre-pass, IR re-solve every 50 steps",
}


# further sampled inputs of the Monte Carlo leg with them (Sec. IV-F)
MC_VAR = {"cov_rho": 0.1, "cov_load": 0.15}


def mc_leg(args, name, oracle, plain, var=None, joule=False, n_samples=None):
    """Monte Carlo samples/s to TTF: batch creation and the run of every
    sample to its 10 % IR-drop failure or the 10-year horizon, FP32 stepping,
    steady-state screen on.  One untimed run first (code paths warm), then the
    timed one.  With ``oracle``: every 16th sample (64) recomputed by the FP64
    CPU oracle, compared and timed (the CPU baseline of this metric).  With
    ``plain``: the plain FP64 GPU form (generic tree kernel, no screen,
    Jacobi-CG on the nodal system) on a subset of the samples.  ``var``: further
    sampled inputs (resistivity / current-loading CoV); ``joule``: with the
    Joule-heating thermal pre-pass (inside the timed batch creation)."""
    import numpy as np
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import synth

    g, mat, run, mc = synth.workload(name)
    mc = dict(mc, n_samples=n_samples or args.mc_samples, **(var or {}))
    if joule:
        run = dict(run, joule=1)
    S = mc["n_samples"]
    label = {"sd_T_K": "die-temperature sd {:g} K", "sd_ea_eV": "activation-energy sd {:g} eV",
             "cov_map": "thermal-map amplitude CoV {:g}"}
    extra = "".join(", " + (label[k].format(v) if k in label else f"{k[4:]} CoV {v:g}")
                    for k, v in (var or {}).items()) + (", Joule pre-pass" if joule else "")

    def one(run_, mc_):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B = P.Batch(g, mat, run_, mc_)
        res = B.run_to_ttf()
        torch.cuda.synchronize()
        return B, res, time.perf_counter() - t0

    # the multigrid's coarse-correction scale is a property of the network:
    # tuned once on a one-sample batch of the same design (outside the timed
    # region) and passed to the Monte Carlo batch
    t0 = time.perf_counter()
    Bt = P.Batch(g, mat, run)
    tune = Bt.autotune(run["ir_every"])
    Bt.close()
    t_tune = time.perf_counter() - t0
    run = dict(run, amg_alpha=tune["amg_alpha"] if tune["amg_alpha"] > 0 else 0.0)
    B, _, _ = one(run, mc)
    B.close()
    B, res, wall = one(run, mc)
    info = B.info()
    segs = {s: B.failed_segments(s) for s in range(0, S, 16)}
    B.close()
    ttf = np.array([r["ttf_s"] for r in res if r["failed"]])
    yr = 365.25 * 86400.0
    o = {"metric": "MC samples/s to TTF", "value": S / wall, "unit": "samples/s",
         "workload": f"{name}: {MC_DESC[name]}; {S} samples, 20% lognormal CoV on kappa and sigma_crit{extra}, "
                     f"2000 BE steps over 10 y, IR re-solve every {run['ir_every']} steps, FP32 stepping, screen on",
         "wall_s": wall, "n_fail": int(ttf.size), "n_censored": int(S - ttf.size),
         "ttf_mean_y": float(ttf.mean() / yr) if ttf.size else None,
         "ttf_cov": float(ttf.std(ddof=1) / ttf.mean()) if ttf.size > 1 else None,
         "final_drop_mean": float(np.mean([r["final_drop"] for r in res])),
         "node_steps": info["node_steps"], "ir_ms": info["ir_ms"], "step_kernel_ms": info["step_kernel_ms"],
         "amg_alpha": run["amg_alpha"], "tune_s": t_tune,
         "ir_system_nodes": info["ir_sys_nodes"], "cg_iters_total": info["cg_iters_total"],
         "redecided_in_fp64": info["n_redecided"]}
    # roofline of the whole Monte Carlo job: algorithmic HBM bytes per sample =
    # 20 B per FP32 node-step actually stepped + 124 B per iterated-system node
    # and PCG iteration of that sample (both streamed once), at 8 TB/s
    bps = (BYTES_PER_NODE_STEP[1] * info["node_steps"] + 124.0 * info["ir_sys_nodes"] * info["cg_sample_iters"]) / S
    o["roofline"] = {"bound": "hbm", "algorithmic_bytes_per_sample": bps,
                     "roofline_samples_per_s": HBM_PEAK_GBS * 1e9 / bps, "frac": (S / wall) / (HBM_PEAK_GBS * 1e9 / bps),
                     "note": "latency-bound: a few hundred-node system per sample and few active trees"}
    if oracle:
        from oracle import oracle as O
        O.build(force=False)
        topo = O.topology(g, run["intervals_per_seg"])
        t0 = time.perf_counter()
        refs = {s: O.run_sample(g, mat, run, mc, s, topo=topo) for s in range(0, S, 16)}
        t_or = time.perf_counter() - t0
        n_cmp = n_red = flag_mis = seg_mis = 0
        e_ttf = e_fd = 0.0
        for s, ref in refs.items():
            r = res[s]
            n_cmp += 1
            n_red += int(r["redecided"])
            flag_mis += int(r["failed"] != ref["failed"])
            e_fd = max(e_fd, abs(r["final_drop"] - ref["final_drop"]) / ref["final_drop"])
            if r["failed"] and ref["failed"]:
                e_ttf = max(e_ttf, abs(r["ttf_s"] - ref["ttf"]) / ref["ttf"])
            seg_mis += int(not np.array_equal(segs[s], ref["failed_segs"]))
        o["vs_fp64_oracle"] = {"samples": len(refs), "compared": n_cmp, "redecided_in_fp64": n_red,
                               "failure_flag_mismatches": flag_mis, "failed_segment_set_mismatches": seg_mis,
                               "max_rel_err_ttf": e_ttf, "max_rel_err_final_drop": e_fd,
                               "oracle_failed": int(sum(refs[s]["failed"] for s in refs))}
        o["cpu_baseline"] = {"value": len(refs) / t_or, "unit": "samples/s", "cores": 1, "kind": "oracle",
                             "cpu": host_cpu(),
                             "sample": f"every 16th of the {S} samples ({len(refs)}), FP64 oracle, "
                                      f"{t_or:.1f} s incl. its IR direct solves"}
        # the same samples over the host's cores (one spawned process each)
        import concurrent.futures as cf
        import multiprocessing as mp
        ids = list(refs)
        n_proc = max(1, min(16, os.cpu_count() or 1, len(ids)))
        jobs = [(name, ids[k::n_proc], var) for k in range(n_proc)]
        t0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=n_proc, mp_context=mp.get_context("spawn")) as ex:
            n_done = sum(ex.map(_oracle_mc_worker, jobs))
        ta = time.perf_counter() - t0
        o["cpu_baseline"]["all_cores"] = {"value": n_done / ta, "unit": "samples/s", "cores": n_proc,
                                          "sample": f"the same {n_done} samples over {n_proc} spawned processes "
                                                    f"({ta:.1f} s incl. each process's setup)"}
    if plain:
        Sp = min(64, S)
        runp = dict(run, prec=0, stepper=1, screen=0, ir_precond=0)
        Bp, resp, wp = one(runp, dict(mc, n_samples=Sp))
        Bp.close()
        o["plain_fp64_gpu"] = {"value": Sp / wp, "unit": "samples/s",
                               "sample": f"first {Sp} samples, FP64, generic tree kernel, every tree stepped, "
                                         "Jacobi-preconditioned CG on the nodal system",
                               "speedup_of_value": (S / wall) / (Sp / wp)}
    return o


STEP_DESC = {
    "fullchip": "fullchip: 2000x2000 routing grid (1 um tracks, 2 mm die), 4 metal layers (M1/M2 stripes "
                "every 4th track cut into trees of 2-8 segments, M3/M4 every 20th track cut into lines of "
                "40-99 segments, M3-M4 vias every 4th node), 16 VDD pads on M4, thermal map 340 K + 12 hotspots (+20..70 K) with the "
                "Joule-heating pre-pass, 2000 BE steps over 10 y, IR re-solve every 50 steps, run to the "
                "first 10 % IR-drop failure or the horizon",
    "pg400": "pg400: 400x400 two-layer P/G grid, 798 line trees, 2000 BE steps over 10 y, IR re-solve every "
             "100 steps, thermal map 330 K + 6 hotspots",
}
PROFILE_OF = {"fullchip": "profiles/k_chain_fullchip.md", "pg400": "profiles/k_chain_pg400.md"}


def stepping_leg(args, name, headline):
    """Stress-node-steps/s of one sample's full coupled run (IR solve, every
    tree stepped -- the steady-state screen off, as the plain method without
    its optional pruning --, nucleation, void growth, resistance write-back,
    IR re-solves, to failure or the horizon).  The batch is built before the
    timed region; each timed step resets it to t = 0 and runs it to TTF.  The
    roofline is that of the stepping kernel (HIP events around each launch
    inside the library); for the headline also the plain FP64 GPU form and
    the FP64 oracle on host cores."""
    import numpy as np
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import synth

    g, mat, run, _ = synth.workload(name)
    run = dict(run, prec=args.prec, screen=0)
    log(f"bench: building batch for {g.name} ({g.n_nodes} nodes, {g.n_res} resistors)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B = P.Batch(g, mat, run)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = B.info()
    log(f"bench: {info['n_trees']} trees, {info['n_stress']} stress nodes, setup {t_setup:.2f} s")
    # the library's autotuner picks the chain kernel's workgroup size and
    # register budget and the IR launch shape on this batch (outside the timed region)
    t0 = time.perf_counter()
    tune = B.autotune(run["ir_every"])
    t_tune = time.perf_counter() - t0
    log(f"bench: autotune {t_tune:.2f} s: chain_wg {tune['chain_wg']}, chain_occ {tune['chain_occ']}, "
        f"ir_launch {tune['ir_launch']}")
    steps = args.steps if headline else max(1, min(args.steps, 2))
    warm = args.warmup if headline else 1
    for w in range(warm):
        B.reset()
        B.run_to_ttf()
    torch.cuda.synchronize()
    B.reset()
    t0 = time.perf_counter()
    results = None
    for k in range(steps):
        if k:
            B.reset()
        results = B.run_to_ttf()
        if headline:
            log(f"bench: step {k + 1}/{steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # counters are cleared by reset: every step replays the same run, so the
    # last step's counters times the step count is exact
    i1 = B.info()
    value = i1["node_steps"] * steps / wall
    bytes_ns = BYTES_PER_NODE_STEP[args.prec]
    step_ms = i1["step_kernel_ms"]
    launches = i1["step_launches"]
    achieved = (bytes_ns * i1["node_steps"] / 1e9) / (step_ms / 1e3) if step_ms > 0 else None
    kernel = (f"k_chain<float,{i1['chain_m']},{i1['chain_wg']},{tune['chain_occ']}>" if args.prec == 1
              else "k_chain<double>")
    traffic = (measured_traffic("paper_2604_10743_amd/csrc/k_chain.hip", PROFILE_OF[name], kernel)
               if args.prec == 1 else None)
    streamed = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "bytes_per_node_step": bytes_ns}
    if achieved and achieved > HBM_PEAK_GBS:
        # the resident kernel moves its state once per launch and can beat any
        # streaming stepper: then it is measured against the vector-ALU bound
        tf = FLOPS_PER_NODE_STEP * i1["node_steps"] / (step_ms / 1e3) / 1e12
        roofline = {"bound": "alu", "achieved": tf, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tf / FP32_VALU_PEAK_TFLOPS, "flops_per_node_step": FLOPS_PER_NODE_STEP,
                    "streamed_hbm": streamed}
    else:
        roofline = dict(streamed)
    roofline.update({"traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-scaled)",
                     "kernel": kernel, "launches_per_step": launches,
                     "avg_launch_ms": step_ms / max(launches, 1), "workgroups": i1["n_chain_wg"],
                     "algorithmic_bytes_per_launch": bytes_ns * i1["node_steps"] / max(launches, 1)})
    r0 = results[0]
    out = {
        "metric": "stress-node-steps/s", "value": value, "unit": "node-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": warm, "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.prec == 1 else "f64", "data": "synthetic",
        "config": {"workload": f"{STEP_DESC[name]}; {info['n_trees']} trees, {info['n_stress']} stress nodes, "
                               f"{info['n_nodes']} grid nodes; steady-state screen off (every tree stepped), "
                               "FP32 stress with FP64 void volumes, resistance changes, IR and TTF",
                   "node_steps_per_step": i1["node_steps"], "setup_s": t_setup,
                   "autotune": {"s": t_tune, "chain_wg": tune["chain_wg"], "chain_occ": tune["chain_occ"],
                                "ir_launch": tune["ir_launch"]},
                   "ir_ms_per_step": i1["ir_ms"], "cg_iters_per_step": i1["cg_iters_total"],
                   "ir_system_nodes": i1["ir_sys_nodes"], "step_kernel_ms_per_step": step_ms,
                   "ttf_s": r0["ttf_s"], "final_drop": r0["final_drop"], "init_drop": r0["init_drop"],
                   "outer_idx": r0["outer_idx"], "n_nucleated_trees": r0["n_nucleated_trees"],
                   "n_failed_segs": r0["n_failed_segs"]},
        "roofline": roofline,
    }
    B.close()
    if headline and not args.no_plain:
        # the plain FP64 GPU FDTD form (generic tree kernel, one (tree) per
        # lane, FP64) on one aging interval of the same workload
        Bp = P.Batch(g, mat, dict(run, prec=0, stepper=1, joule=0))
        Bp.ir_solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Bp.stress_step(run["ir_every"])
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        ip = Bp.info()
        out["plain_fp64_gpu"] = {"value": ip["node_steps"] / tp, "unit": "node-steps/s",
                                 "sample": f"{name}, {run['ir_every']} BE steps of every tree, FP64, "
                                           "one (tree) per lane tree-elimination kernel",
                                 "speedup_of_value": value / (ip["node_steps"] / tp)}
        Bp.close()
        log("bench: plain fp64 done")
    if headline and not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_stepping(name, run["ir_every"])
        log("bench: cpu baseline done")
    return out


def cpu_baseline_stepping(name, n_steps):
    """The FP64 oracle stepping every tree of the workload for one aging
    interval (seeded prescribed currents in trees-only mode: the oracle's
    sparse direct IR solve does not finish on the full-chip grid in 20
    minutes, so it is left out and the figure is stepping only), on one core
    and with the trees split over every host core."""
    import numpy as np
    from oracle import oracle as O
    O.build(force=False)
    g, mat, run = _oracle_grid(name)
    topo = O.topology(g, run["intervals_per_seg"])
    t0 = time.perf_counter()
    sim = O.SampleSim(g, mat, run, topo)
    sim.set_j(g.seg_j)
    sim.steps(n_steps, 0)
    t1 = time.perf_counter() - t0
    ns = int(topo.n_stress) * n_steps
    out = {"value": ns / t1, "unit": "node-steps/s", "cores": 1, "kind": "oracle", "cpu": host_cpu(),
           "sample": f"{name}: FP64 oracle BE stepping of all {topo.n_trees} trees ({topo.n_stress} stress "
                     f"nodes) for one aging interval of {n_steps} steps, seeded prescribed currents, "
                     f"{t1:.1f} s on one core; IR solve excluded (the GPU value includes its IR re-solves)"}
    import concurrent.futures as cf
    import multiprocessing as mp
    n_proc = max(1, min(16, os.cpu_count() or 1))
    bounds = np.linspace(0, topo.n_trees, n_proc + 1).astype(int)
    jobs = [(name, int(bounds[k]), int(bounds[k + 1]), n_steps) for k in range(n_proc) if bounds[k + 1] > bounds[k]]
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
        ns_all = sum(ex.map(_oracle_trees_worker, jobs))
    ta = time.perf_counter() - t0
    out["all_cores"] = {"value": ns_all / ta, "unit": "node-steps/s", "cores": len(jobs),
                        "sample": f"the same interval with the trees split over {len(jobs)} spawned processes "
                                  f"({ns_all} node-steps, {ta:.1f} s incl. each process's setup)"}
    return out


def branched_leg(args):
    """Branched trees: 200 comb/stub trees (about 200 branches and 4000 FD
    nodes each, trees-only with prescribed currents, 378 K), 200 BE steps of
    every tree with nucleation and void growth, FP32; the workgroup tree
    stepper against the per-lane tree kernel (the plain form), both timed
    with HIP events around each launch inside the library."""
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import synth

    g, mat, run, _ = synth.workload("combs")
    out = {"metric": "stress-node-steps/s", "unit": "node-steps/s",
           "workload": "combs: 200 comb/stub trees (trunks of 20-100 segments, teeth and stubs; 200 branches "
                       "and 4016 FD nodes per tree on average, up to 418 and 8361), prescribed currents, 378 K, "
                       f"FP{'32' if args.prec else '64'}"}
    for stepper, key, n in ((0, "workgroup_tree_kernel", 200), (1, "per_lane_tree_kernel", 20)):
        B = P.Batch(g, mat, dict(run, prec=args.prec, stepper=stepper))
        B.stress_step(2)
        torch.cuda.synchronize()
        i0 = B.info()
        t0 = time.perf_counter()
        B.stress_step(n)
        torch.cuda.synchronize()
        w = time.perf_counter() - t0
        i1 = B.info()
        ns = i1["node_steps"] - i0["node_steps"]
        ms = i1["step_kernel_ms"] - i0["step_kernel_ms"]
        bn = BYTES_PER_NODE_STEP[args.prec]
        out[key] = {"value": ns / w, "steps": n, "kernel_ms": ms, "kernel_node_steps_per_s": ns / (ms * 1e-3),
                    "roofline": {"bound": "hbm", "achieved": ns * bn / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": ns * bn / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 "bytes_per_node_step": bn},
                    "n_events": i1["n_events"]}
        B.close()
    out["value"] = out["workgroup_tree_kernel"]["value"]
    out["speedup_over_per_lane"] = out["workgroup_tree_kernel"]["value"] / out["per_lane_tree_kernel"]["value"]
    return out


def voids_leg(args, name="pg400", sigma_crit=200e6, screen=1):
    """A grid with voids: the critical stress lowered (pg400: 200 MPa, the
    full chip: 250 MPa) so that the mortal lines nucleate within the horizon;
    void growth, liner resistance changes and IR re-solves run inside the
    timed region (one untimed run first)."""
    import numpy as np
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import synth

    g, mat, run, _ = synth.workload(name)
    mat = dict(mat, sigma_crit=sigma_crit)
    run = dict(run, prec=args.prec, screen=screen)
    B = P.Batch(g, mat, run)
    tune = B.autotune(run["ir_every"])           # outside the timed region
    B.run_to_ttf()
    B.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = B.run_to_ttf()[0]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    i = B.info()
    B.close()
    return {"metric": "stress-node-steps/s", "value": i["node_steps"] / wall, "unit": "node-steps/s",
            "workload": f"{name} with sigma_crit {sigma_crit / 1e6:g} MPa, screen {'on' if screen else 'off'}, "
                        f"FP32, one run to failure or the horizon",
            "wall_ms": wall * 1e3, "ir_ms": i["ir_ms"], "step_kernel_ms": i["step_kernel_ms"],
            "autotune": {k: tune[k] for k in ("chain_wg", "chain_occ", "ir_launch", "amg_alpha")},
            "cg_iters": i["cg_iters_total"], "node_steps": i["node_steps"], "ttf_s": r["ttf_s"],
            "failed": r["failed"], "outer_idx": r["outer_idx"], "init_drop": r["init_drop"],
            "final_drop": r["final_drop"], "n_nucleated_trees": r["n_nucleated_trees"],
            "n_failed_segs": r["n_failed_segs"]}


def skip_leg(args, name, n_samples=None, tol=1e-6, reps=3):
    """Steady-state skipping (ss_tol) against the full run: the immortality
    screen off (every tree stepped), the same batch run to the horizon with
    and without skipping (best of reps each, after an untimed run), results
    compared sample by sample and the largest stress difference reported."""
    import numpy as np
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import synth

    g, mat, run, mc = synth.workload(name)
    mc = dict(mc, n_samples=n_samples) if (mc is not None and n_samples) else None
    legs = {}
    for label, ss in (("full", 0.0), ("skip", tol)):
        B = P.Batch(g, mat, dict(run, prec=args.prec, screen=0, ss_tol=ss), mc)
        B.autotune(run["ir_every"])
        B.run_to_ttf()
        best, res = 1e30, None
        for _ in range(reps):
            B.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = B.run_to_ttf()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        i = B.info()
        st = [B.stress(s) for s in range(min(len(res), 8))]
        B.close()
        legs[label] = (best, res, i, st)
    (tf, rf, i_f, sf), (ts, rs, i_s, ss_) = legs["full"], legs["skip"]
    same = all(a["failed"] == b["failed"] and a["outer_idx"] == b["outer_idx"] and
               a["n_nucleated_trees"] == b["n_nucleated_trees"] and
               abs(a["final_drop"] - b["final_drop"]) <= 1e-6 * abs(a["final_drop"]) for a, b in zip(rf, rs))
    dmax = max(float(np.max(np.abs(a - b))) for a, b in zip(sf, ss_))
    return {"workload": f"{name}{f' x {len(rf)} Monte Carlo samples' if mc else ''}, screen off, "
                        f"FP32, run to the horizon, ss_tol {tol:g}",
            "full_ms": tf * 1e3, "skip_ms": ts * 1e3, "speedup": tf / ts,
            "node_steps_full": i_f["node_steps"], "node_steps_skip": i_s["node_steps"],
            "full_node_steps_per_s_at_skip_time": i_f["node_steps"] / ts,
            "n_skipped": i_s["n_ss_skipped"], "n_woken": i_s["n_ss_woken"],
            "results_identical": bool(same), "max_stress_diff_Pa": dmax,
            "stress_bound_Pa": tol * mat["sigma_crit"]}


def krylov_leg(args, name, n_samples=None, q=6, reps=3):
    """Reduced (extended rational Krylov) stepping of the long chains against
    exact elimination: the immortality screen off, the same batch run to the
    horizon with krylov_q = q and without (best of reps each, after an
    untimed run), results and stress compared."""
    import numpy as np
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import synth

    g, mat, run, mc = synth.workload(name)
    mc = dict(mc, n_samples=n_samples) if (mc is not None and n_samples) else None
    legs = {}
    for label, kq in (("exact", 0), ("krylov", q)):
        B = P.Batch(g, mat, dict(run, prec=args.prec, screen=0, krylov_q=kq), mc)
        B.autotune(run["ir_every"])
        B.run_to_ttf()
        best, res = 1e30, None
        for _ in range(reps):
            B.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = B.run_to_ttf()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        i = B.info()
        st = [B.stress(s) for s in range(min(len(res), 8))]
        B.close()
        legs[label] = (best, res, i, st)
    (te, re_, ie, se), (tk, rk, ik, sk) = legs["exact"], legs["krylov"]
    same = all(a["failed"] == b["failed"] and a["outer_idx"] == b["outer_idx"] for a, b in zip(re_, rk))
    drop_err = max(abs(a["final_drop"] - b["final_drop"]) / a["final_drop"] for a, b in zip(re_, rk))
    srel = max(float(np.max(np.abs(a - b)) / np.max(np.abs(a))) for a, b in zip(se, sk))
    return {"workload": f"{name}{f' x {len(re_)} Monte Carlo samples' if mc else ''}, screen off, "
                        f"FP32, run to the horizon, krylov_q {q}",
            "exact_ms": te * 1e3, "krylov_ms": tk * 1e3, "speedup": te / tk,
            "exact_step_ms": ie["step_kernel_ms"], "krylov_step_ms": ik["step_kernel_ms"],
            "node_steps_exact": ie["node_steps"], "node_steps_exact_in_krylov_run": ik["node_steps"],
            "krylov_node_steps": ik["krylov_node_steps"], "bases_built": ik["n_krylov_bases"],
            "reduced_intervals": ik["n_krylov_intervals"], "fallbacks": ik["n_krylov_fallbacks"],
            "decisions_identical": bool(same), "max_final_drop_rel_err": drop_err,
            "max_stress_rel_err": srel}


def adaptive_leg(args, name, sigma_crit=None, screen=0, levels=3, reps=3):
    """The adaptive time grid (dt_adapt: up to dt 2^levels between
    nucleations, back to dt after one) against the uniform grid on the same
    one-sample batch: run time to failure or the horizon (best of reps, after
    an untimed run), re-solves, and the TTF / final drop difference (the
    adaptive grid's discretisation error against the uniform one)."""
    import numpy as np
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import synth

    g, mat, run, _ = synth.workload(name)
    if sigma_crit:
        mat = dict(mat, sigma_crit=sigma_crit)
    legs = {}
    for label, lv in (("uniform", 0), ("adaptive", levels)):
        B = P.Batch(g, mat, dict(run, prec=args.prec, screen=screen, dt_adapt=lv))
        B.autotune(run["ir_every"])
        B.run_to_ttf()
        best, res = 1e30, None
        for _ in range(reps):
            B.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = B.run_to_ttf()[0]
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        i = B.info()
        B.close()
        legs[label] = (best, res, i)
    (tu, ru, iu), (ta, ra, ia) = legs["uniform"], legs["adaptive"]
    o = {"workload": f"{name}{f' with sigma_crit {sigma_crit / 1e6:g} MPa' if sigma_crit else ''}, "
                     f"screen {'on' if screen else 'off'}, FP32, one run to failure or the horizon, "
                     f"dt_adapt {levels}",
         "uniform_ms": tu * 1e3, "adaptive_ms": ta * 1e3, "speedup": tu / ta,
         "resolves_uniform": ru["outer_idx"], "resolves_adaptive": ra["outer_idx"],
         "node_steps_uniform": iu["node_steps"], "node_steps_adaptive": ia["node_steps"],
         "failed": [ru["failed"], ra["failed"]], "ttf_s": [ru["ttf_s"], ra["ttf_s"]],
         "final_drop": [ru["final_drop"], ra["final_drop"]]}
    if ru["failed"] and ra["failed"]:
        o["ttf_rel_diff"] = abs(ra["ttf_s"] - ru["ttf_s"]) / ru["ttf_s"]
    return o


def thermal_leg(args):
    """Equal-average thermal maps (the paper's thermal-profile observation):
    the mc_grid network under a uniform map, four hotspots over the wires of
    highest current density, the same hotspots over the wires of lowest
    current density, the latter 5 K hotter on average, and no map at all
    (Joule heating over the uniform ambient); each with the Joule-heating
    pre-pass, Monte Carlo to TTF for each (256 samples; batch creation, which
    runs the pre-pass, inside the timed region)."""
    import numpy as np
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import synth

    g, mat, run, mc = synth.workload("mc_grid")
    mc = dict(mc, n_samples=256)
    B = P.Batch(g, mat, run)
    B.ir_solve()
    j = B.seg_j(0)
    B.close()
    hot = synth.hotspot_centers(g, j, 4, 150e-6, highest=True)
    cold = synth.hotspot_centers(g, j, 4, 150e-6, highest=False)
    out = {"workload": "mc_grid network, 256 samples per map, hotspots 4 x +60 K (sigma 60 um, 150 um apart), "
                       "die-average 335 K (hotter variant 340 K); Joule-heating pre-pass on every map "
                       "(k_cu 400, k_ILD 1.4 W/(m K), t_ILD 0.2 um)", "maps": {}}
    yr = 365.25 * 86400.0
    t_all = 0.0
    maps = synth.thermal_variants(g, hot, cold, 335.0, 60.0, 60e-6, hotter_K=5.0)
    maps["joule_only"] = copy.deepcopy(maps["uniform"])
    maps["joule_only"].tmap = None
    for name, h in maps.items():
        rn = dict(run, joule=1, T_ambient=335.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Bm = P.Batch(h, mat, rn, mc)
        res = Bm.run_to_ttf()
        torch.cuda.synchronize()
        t_all += time.perf_counter() - t0
        Tn = Bm.node_state(0)[0]
        ttf = np.array([r["ttf_s"] for r in res if r["failed"]])
        out["maps"][name] = {"map_mean_K": float(h.tmap.mean()) if h.tmap is not None else 335.0,
                             "map_max_K": float(h.tmap.max()) if h.tmap is not None else 335.0,
                             "wire_T_mean_K": float(Tn.mean()), "wire_T_max_K": float(Tn.max()),
                             "n_fail": int(ttf.size), "n_censored": int(len(res) - ttf.size),
                             "ttf_mean_y": float(ttf.mean() / yr) if ttf.size else None,
                             "nucleated_trees_per_sample": float(np.mean([r["n_nucleated_trees"] for r in res])),
                             "final_drop_mean": float(np.mean([r["final_drop"] for r in res]))}
        Bm.close()
    out["samples_per_s"] = len(maps) * 256 / t_all
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", type=int, default=1, help="1 = FP32 stepping, 0 = FP64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mc", action="store_true")
    ap.add_argument("--only-mc", action="store_true",
                    help="run only the Monte Carlo legs (no oracle, no plain form) and print them")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--mc-samples", type=int, default=1024)
    ap.add_argument("--fc-samples", type=int, default=64, help="Monte Carlo samples of the full-chip leg")
    ap.add_argument("--workload", default="fullchip", choices=sorted(STEP_DESC),
                    help="workload of the headline stepping measurement")
    ap.add_argument("--only-headline", action="store_true", help="run the headline measurement only")
    ap.add_argument("--no-sur", action="store_true", help="skip the learned-screen leg")
    ap.add_argument("--only-sur", action="store_true", help="run the learned-screen leg only")
    ap.add_argument("--only-skip", action="store_true", help="run the steady-state skipping legs only")
    ap.add_argument("--only-krylov", action="store_true", help="run the reduced (Krylov) stepping legs only")
    ap.add_argument("--only-adaptive", action="store_true", help="run the adaptive time grid legs only")
    ap.add_argument("--sur-grids", type=int, default=24, help="label grids for the learned screen")
    ap.add_argument("--sur-label-samples", type=int, default=1024)
    ap.add_argument("--sur-steps", type=int, default=3000, help="Adam steps of the screen model")
    ap.add_argument("--sur-samples", type=int, default=256, help="MC samples of the screened run")
    ap.add_argument("--sur-quantile", type=float, default=0.995,
                    help="held-out quantile of the learned screen's calibration")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only copy this many bytes device-to-device (a plain copy kernel of known "
                         "size, to scale the FETCH_SIZE/WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is described in the design notes, not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.only_mc:
        out = {"mc": mc_leg(args, "mc_grid", oracle=False, plain=False),
               "mc_mesh": mc_leg(args, "mc_mesh", oracle=False, plain=False),
               "mc_rho_load": mc_leg(args, "mc_grid", oracle=False, plain=False, var=MC_VAR),
               "mc_joule": mc_leg(args, "mc_grid", oracle=False, plain=False, joule=True),
               "mc_die_T": mc_leg(args, "mc_grid", oracle=False, plain=False, var={"sd_T_K": 3.0}),
               "mc_map": mc_leg(args, "mc_grid", oracle=False, plain=False, var={"cov_map": 0.2})}
        print(json.dumps(out), flush=True)
        return

    if args.only_sur:
        print(json.dumps({"surrogate": surrogate_leg(args)}), flush=True)
        return

    if args.only_skip:
        print(json.dumps({"fullchip_skip": skip_leg(args, "fullchip"),
                          "mc_skip": skip_leg(args, "mc_grid", n_samples=256)}), flush=True)
        return

    if args.only_adaptive:
        print(json.dumps({"fullchip_adaptive": adaptive_leg(args, "fullchip"),
                          "pg400_voids_adaptive": adaptive_leg(args, "pg400", sigma_crit=200e6, screen=1)}),
              flush=True)
        return

    if args.only_krylov:
        print(json.dumps({"fullchip_krylov": krylov_leg(args, "fullchip"),
                          "pg400_krylov": krylov_leg(args, "pg400")}), flush=True)
        return

    out = stepping_leg(args, args.workload, headline=True)
    log(f"bench: headline ({args.workload}) done")
    if args.only_headline:
        print(json.dumps(out), flush=True)
        return
    if args.workload != "pg400":
        out["pg400"] = stepping_leg(args, "pg400", headline=False)
        log("bench: pg400 done")
    out["pg400_voids"] = voids_leg(args)
    log("bench: pg400 with voids done")
    out["fullchip_voids"] = voids_leg(args, "fullchip", 250e6, screen=0)
    log("bench: fullchip with voids done")
    out["branched"] = branched_leg(args)
    log("bench: branched trees done")
    out["fullchip_skip"] = skip_leg(args, "fullchip")
    log("bench: fullchip steady-state skipping done")
    out["fullchip_krylov"] = krylov_leg(args, "fullchip")
    out["pg400_krylov"] = krylov_leg(args, "pg400")
    log("bench: reduced (Krylov) stepping legs done")
    out["fullchip_adaptive"] = adaptive_leg(args, "fullchip")
    out["pg400_voids_adaptive"] = adaptive_leg(args, "pg400", sigma_crit=200e6, screen=1)
    log("bench: adaptive time grid legs done")
    if not args.no_mc:
        out["fullchip_mc"] = mc_leg(args, "fullchip", oracle=False, plain=False, n_samples=args.fc_samples)
        log("bench: fullchip mc done")
        out["mc"] = mc_leg(args, "mc_grid", oracle=not args.no_cpu, plain=not args.no_plain)
        log("bench: mc (mc_grid) done")
        out["mc_mesh"] = mc_leg(args, "mc_mesh", oracle=False, plain=False)
        out["mc_rho_load"] = mc_leg(args, "mc_grid", oracle=False, plain=False, var=MC_VAR)
        out["mc_joule"] = mc_leg(args, "mc_grid", oracle=False, plain=False, joule=True)
        out["mc_die_T"] = mc_leg(args, "mc_grid", oracle=False, plain=False, var={"sd_T_K": 3.0})
        out["mc_map"] = mc_leg(args, "mc_grid", oracle=False, plain=False, var={"cov_map": 0.2})
        log("bench: mc (mc_mesh, variations) done")
        out["mc_skip"] = skip_leg(args, "mc_grid", n_samples=256)
        log("bench: mc_grid steady-state skipping done")
        out["thermal_sweep"] = thermal_leg(args)
        log("bench: thermal sweep done")
    if not args.no_sur:
        out["surrogate"] = surrogate_leg(args)
        log("bench: surrogate done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
