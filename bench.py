"""Benchmark of the coupled EM/TM stress + IR-drop hot path on one MI355X.

A step is one full pass of the hot path over the 400x400 two-layer P/G grid:
IR solve, backward-Euler stress stepping of every tree (2000 steps over ten
years, FP32 stress with FP64 void/dR accumulators), nucleation and void
growth, resistance write-back and an IR re-solve every 100 steps, until the
10 % IR-drop failure or the horizon.  The batch is built (netlist copied,
trees partitioned, statics evaluated) before the timed region; each timed
step resets it to t = 0 and runs it to time-to-failure.

Prints ONE JSON line (rank 0).  Metric: stress-node-steps/s (sum over stepped
trees of stress nodes x steps, divided by wall time).  Also reported: the
roofline of the dominant kernel (the stepping kernel, timed with HIP events on
its own stream inside the library; against the streamed HBM roofline, or the
FP32 vector-ALU bound where the resident kernel beats the former), the plain FP64 GPU form (one tree per
lane, FP64) over one aging interval, the FP64 oracle on host cores over a
bounded sample of the same workload, and Monte Carlo samples/s to TTF with 1024
samples on the 96x96 sparse-via grid (failures within the horizon; checked
against the FP64 oracle on 64 samples) and on the 32x32 mesh.
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


def _oracle_trees_worker(job):
    """One host process of the all-core oracle baseline: the pg400 grid, the
    nominal currents j, 100 BE steps of trees [t0, t1); returns node-steps."""
    t0, t1, j, n_steps = job
    import numpy as np
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    from paper_2604_10743_amd import synth
    g, mat, run, _ = synth.workload("pg400_fp64")
    topo = O.topology(g, run["intervals_per_seg"])
    sim = O.SampleSim(g, mat, run, topo)
    sim.set_j(j)
    act = np.zeros(topo.n_trees, np.uint8)
    act[t0:t1] = 1
    sim.set_active(act)
    sim.steps(n_steps, 0)
    return int(topo.tree_off[t1] - topo.tree_off[t0]) * n_steps


def measured_traffic(kernel_src: str, profile_md: str):
    """HBM bytes per launch from the committed PMC summary, or None when the
    kernel source changed since the counters were taken."""
    import hashlib
    try:
        txt = open(os.path.join(ROOT, profile_md)).read()
        block = txt.split("```json", 1)[1].split("```", 1)[0]
        pm = json.loads(block)
        sha = hashlib.sha256(open(os.path.join(ROOT, kernel_src), "rb").read()).hexdigest()[:16]
        if pm.get("source_sha256_16") != sha:
            return None
        return pm["traffic_bytes_per_launch"]
    except (OSError, IndexError, ValueError, KeyError):
        return None


def surrogate_leg(args):
    """Learned screen: labels from the library's own transient runs on random
    sparse-via grids, training with the BF16 MFMA kernels, then the screened
    and the unscreened Monte Carlo run of the screen_mc workload."""
    import numpy as np
    import torch
    import paper_2604_10743_amd as P
    from paper_2604_10743_amd import surrogate, synth

    g, mat, run, mc = synth.workload("screen_mc")
    mc = dict(mc, n_samples=args.sur_samples)
    horizon = 4 * run["n_steps"]                  # labels up to 40 years
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, y, infos = surrogate.training_set(11, args.sur_grids, mat, run, args.sur_label_samples, horizon,
                                         log=log)
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    Xv, yv, _ = surrogate.training_set(12, 2, mat, run, args.sur_label_samples, horizon)
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
    # bias shift so that 99.5 % of held-out predictions are not later than the label
    shift = surrogate.calibrate(model, Xv, yv, 0.995)
    log(f"bench: surrogate trained on {n} pairs: loss {train_loss:.4f}, held-out {val_loss:.4f}")

    def mc_run(with_model):
        B = P.Batch(g, mat, run, mc)
        if with_model:
            B.surrogate_screen(model, 2.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = B.run_to_ttf()
        torch.cuda.synchronize()
        w = time.perf_counter() - t0
        inf = B.info()
        B.close()
        return res, inf, w

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
            "workload": f"screen_mc: 200x200 sparse-via grid (via every 64 nodes), 330 K + 6 hotspots, "
                        f"{S} samples, 20% CoV on kappa and sigma_crit, FP32, margin 2",
            "unscreened_samples_per_s": S / w0, "speedup": w0 / w1,
            "node_steps": i1["node_steps"], "node_steps_unscreened": i0["node_steps"],
            "n_deferred": i1["n_deferred"], "n_activated": i1["n_activated"],
            "n_late": i1["n_late"], "n_violations": i1["n_violations"], "results_identical": bool(same),
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
}


# further sampled inputs of the Monte Carlo leg with them (Sec. IV-F)
MC_VAR = {"cov_rho": 0.1, "cov_load": 0.15}


def mc_leg(args, name, oracle, plain, var=None, joule=False):
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
    mc = dict(mc, n_samples=args.mc_samples, **(var or {}))
    if joule:
        run = dict(run, joule=1)
    S = mc["n_samples"]
    extra = "".join(f", {k[4:]} CoV {v:g}" for k, v in (var or {}).items()) + (", Joule pre-pass" if joule else "")

    def one(run_, mc_):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B = P.Batch(g, mat, run_, mc_)
        res = B.run_to_ttf()
        torch.cuda.synchronize()
        return B, res, time.perf_counter() - t0

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
                     "2000 BE steps over 10 y, IR re-solve every 100 steps, FP32 stepping, screen on",
         "wall_s": wall, "n_fail": int(ttf.size), "n_censored": int(S - ttf.size),
         "ttf_mean_y": float(ttf.mean() / yr) if ttf.size else None,
         "ttf_cov": float(ttf.std(ddof=1) / ttf.mean()) if ttf.size > 1 else None,
         "final_drop_mean": float(np.mean([r["final_drop"] for r in res])),
         "node_steps": info["node_steps"], "ir_ms": info["ir_ms"], "step_kernel_ms": info["step_kernel_ms"],
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
                             "sample": f"every 16th of the {S} samples ({len(refs)}), FP64 oracle, "
                                      f"{t_or:.1f} s incl. its IR direct solves"}
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
    ap.add_argument("--no-sur", action="store_true", help="skip the learned-screen leg")
    ap.add_argument("--sur-grids", type=int, default=24, help="label grids for the learned screen")
    ap.add_argument("--sur-label-samples", type=int, default=128)
    ap.add_argument("--sur-steps", type=int, default=3000, help="Adam steps of the screen model")
    ap.add_argument("--sur-samples", type=int, default=256, help="MC samples of the screened run")
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
               "mc_joule": mc_leg(args, "mc_grid", oracle=False, plain=False, joule=True)}
        print(json.dumps(out), flush=True)
        return

    g, mat, run, _ = synth.workload("pg400")
    run = dict(run, prec=args.prec, screen=0)
    log(f"bench: building batch for {g.name} ({g.n_nodes} nodes, {g.n_res} resistors)")
    t0 = time.perf_counter()
    B = P.Batch(g, mat, run)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = B.info()
    log(f"bench: {info['n_trees']} trees, {info['n_stress']} stress nodes, setup {t_setup:.2f} s")

    for w in range(args.warmup):
        B.reset()
        B.run_to_ttf()
        log(f"bench: warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    B.reset()
    i0 = B.info()
    t0 = time.perf_counter()
    results = None
    for k in range(args.steps):
        if k:
            B.reset()
        results = B.run_to_ttf()
        log(f"bench: step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # counters are cleared by reset: accumulate per step instead
    # (node_steps of the last step x steps is exact: every step replays the same run)
    i1 = B.info()
    node_steps_total = i1["node_steps"] * args.steps
    value = node_steps_total / wall
    bytes_ns = BYTES_PER_NODE_STEP[args.prec]
    step_ms = i1["step_kernel_ms"]
    launches = i1["step_launches"]
    achieved = (bytes_ns * i1["node_steps"] / 1e9) / (step_ms / 1e3) if step_ms > 0 else None
    traffic = (measured_traffic("paper_2604_10743_amd/csrc/k_chain.hip", "profiles/k_chain_pg400.md")
               if args.prec == 1 else None)
    kernel = (f"k_chain<float,{i1['chain_m']},{i1['chain_wg']}>" if args.prec == 1 else "k_step<double>")
    streamed = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "bytes_per_node_step": bytes_ns}
    if achieved and achieved > HBM_PEAK_GBS:
        # the resident kernel moves its state once per launch and beats any
        # streaming stepper: measure it against the vector-ALU bound instead
        tf = FLOPS_PER_NODE_STEP * i1["node_steps"] / (step_ms / 1e3) / 1e12
        roofline = {"bound": "alu", "achieved": tf, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tf / FP32_VALU_PEAK_TFLOPS, "flops_per_node_step": FLOPS_PER_NODE_STEP,
                    "streamed_hbm": streamed}
    else:
        roofline = dict(streamed)
    roofline.update({"traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-scaled)",
                     "kernel": kernel, "launches_per_step": launches,
                     "avg_launch_ms": step_ms / max(launches, 1), "workgroups": i1["n_chain_wg"]})
    r0 = results[0]
    out = {
        "metric": "stress-node-steps/s", "value": value, "unit": "node-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.prec == 1 else "f64", "data": "synthetic",
        "config": {"workload": f"pg400: 400x400 two-layer P/G grid, {info['n_trees']} line trees, "
                               f"{info['n_stress']} stress nodes, 2000 BE steps over 10 y, "
                               "IR re-solve every 100 steps, thermal map 330 K + 6 hotspots, "
                               "screen off (every tree stepped)",
                   "node_steps_per_step": i1["node_steps"], "setup_s": t_setup,
                   "ir_ms_per_step": i1["ir_ms"], "cg_iters_per_step": i1["cg_iters_total"],
                   "ttf_s": r0["ttf_s"], "final_drop": r0["final_drop"], "init_drop": r0["init_drop"],
                   "n_nucleated_trees": r0["n_nucleated_trees"]},
        "roofline": roofline,
    }
    B.close()

    if not args.no_mc:
        out["mc"] = mc_leg(args, "mc_grid", oracle=not args.no_cpu, plain=not args.no_plain)
        log("bench: mc (mc_grid) done")
        out["mc_mesh"] = mc_leg(args, "mc_mesh", oracle=False, plain=False)
        out["mc_rho_load"] = mc_leg(args, "mc_grid", oracle=False, plain=False, var=MC_VAR)
        out["mc_joule"] = mc_leg(args, "mc_grid", oracle=False, plain=False, joule=True)
        log("bench: mc (mc_mesh) done")

    if not args.no_mc:
        out["thermal_sweep"] = thermal_leg(args)
        log("bench: thermal sweep done")

    if not args.no_sur:
        out["surrogate"] = surrogate_leg(args)
        log("bench: surrogate done")

    if not args.no_plain:
        # the plain FP64 GPU FDTD form (generic tree kernel, FP64) on one aging
        # interval of the same workload, for the speedup of the batched form
        Bp = P.Batch(g, mat, dict(run, prec=0, stepper=1))
        Bp.ir_solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Bp.stress_step(run["ir_every"])
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        ip = Bp.info()
        out["plain_fp64_gpu"] = {"value": ip["node_steps"] / tp, "unit": "node-steps/s",
                                 "sample": f"pg400, {run['ir_every']} BE steps of every tree, FP64, "
                                           "one (tree) per lane tree-elimination kernel",
                                 "speedup_of_value": value / (ip["node_steps"] / tp)}
        Bp.close()
        log("bench: plain fp64 done")

    if not args.no_cpu:
        import numpy as np
        from oracle import oracle as O
        O.build(force=False)
        topo = O.topology(g, run["intervals_per_seg"])
        # one aging interval of pg400 as the GPU job counts it: the IR solve
        # plus ir_every BE steps of every tree.  One core steps the first
        # quarter of the trees (the rest scales with their node count).
        n_tr = max(1, topo.n_trees // 4)
        t0 = time.perf_counter()
        u, I, j, d0 = O.ir_solve(g, g.res_R0)
        t_ir = time.perf_counter() - t0
        t0 = time.perf_counter()
        sim = O.SampleSim(g, mat, run, topo)
        sim.set_j(j)
        act = np.zeros(topo.n_trees, np.uint8)
        act[:n_tr] = 1
        sim.set_active(act)
        sim.steps(run["ir_every"], 0)
        t_st = time.perf_counter() - t0
        ns_c = int(topo.tree_off[n_tr]) * run["ir_every"]
        ns_full = int(topo.tree_off[topo.n_trees]) * run["ir_every"]
        t_full = t_ir + t_st * ns_full / ns_c
        out["cpu_baseline"] = {"value": ns_full / t_full, "unit": "node-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"pg400, FP64 oracle, one aging interval: IR solve (sparse direct, "
                                         f"{t_ir:.1f} s) + {run['ir_every']} BE steps of the first {n_tr} of "
                                         f"{topo.n_trees} trees ({ns_c} node-steps, {t_st:.1f} s), stepping "
                                         f"time scaled to all {ns_full} node-steps by node count"}
        log("bench: cpu baseline done")
        # the same oracle on every host core: the trees split over processes
        # (spawned: no GPU state in them), each building the grid itself
        import concurrent.futures as cf
        import multiprocessing as mp
        n_proc = max(1, min(16, os.cpu_count() or 1))
        bounds = np.linspace(0, topo.n_trees, n_proc + 1).astype(int)
        jobs = [(int(bounds[k]), int(bounds[k + 1]), j, run["ir_every"]) for k in range(n_proc)
                if bounds[k + 1] > bounds[k]]
        t0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
            ns_all = sum(ex.map(_oracle_trees_worker, jobs))
        ta = time.perf_counter() - t0
        out["cpu_baseline"]["all_cores"] = {
            "value": ns_all / (t_ir + ta), "unit": "node-steps/s", "cores": len(jobs),
            "sample": f"pg400, FP64 oracle, one aging interval: the same IR solve on one core ({t_ir:.1f} s) + "
                      f"{run['ir_every']} BE steps of all {topo.n_trees} trees split over {len(jobs)} processes "
                      f"({ns_all} node-steps, {ta:.1f} s incl. each process's setup)"}
        log("bench: cpu baseline (all cores) done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
