#!/usr/bin/env python3
"""Benchmark: Barnes-Hut force evaluation on one MI355X.

Metric: bodies/s (and body-cell interactions/s) of the force evaluation at an
rms relative force error of 1e-3 against FP64 direct summation.

Workload (default): Plummer sphere, N = 2^22 equal masses (G = M = a = 1,
seed 4), eps 0.005, leaf 16, FP32 walk with FP64 cell moments, quadrupole
order, KDK leapfrog dt 5e-4: the configuration the learned criterion is
compared with the opening angle on.  Before timing, the force-evaluation
methods are calibrated on the initial state against the FP64 direct sum
over a seeded 4096-body subsample:
  body-theta    the per-body walk of Sec. 3 (opening angle theta);
  body-theta-guard  the same with a containment guard: a cell whose cube
                holds the body is opened whatever its angle (a variant);
  group-theta   one opening-angle decision per wavefront of 64 bodies;
  group-budget  one error-budget decision per wavefront (error model
                M l^3 / d_g^5 against tau times the group's smallest |a|,
                each |a_i| floored at half the mean |a|, 0.3 of it for
                the monopole terms over Hilbert groups);
  group-learned one learned decision per wavefront and cell: the network's
                predicted error of the particle-cell term on the group
                against the same budget (bf16 MFMA inside the walk),
                trained first on the library's own FP64 simulations of
                Plummer spheres;
  body-theta-o3, group-theta-o3  the two opening-angle walks with the
                octopole term added to each particle-cell interaction;
  group-budget-mono  the group error budget with monopole terms: a cell is
                also charged the bound (7/2) |Q|_F / d_g^4 of the
                quadrupole term it drops;
  group-budget-mixed the group error budget with the mixed order: per cell
                the monopole term where that charged budget holds, else the
                quadrupole term where the plain budget holds, else open;
  body-theta-hilbert, group-theta-hilbert, group-budget-hilbert,
  group-budget-mono-hilbert, group-budget-mixed-hilbert,
  group-learned-hilbert  six of the walks over bodies sorted along the
                Peano-Hilbert curve (a group is 64 consecutive bodies of
                that curve).
Each is swept over its parameter grid from accurate to cheap; the cheapest
grid value with rms <= 1e-3 is kept, and the method with the fastest walk
at that value is the one timed.  After the timed steps the rms error is
measured again at the final state.  The per-body walk of Sec. 3 is also
reported at theta = 0.4, 0.5 and 0.7 and at the theta where its rms error
is 1e-3 (log-log interpolation of the sweep), each with its walk time.

A timed step is one kick-drift-kick leapfrog step, the paper's loop body:
kick + drift, tree rebuild (bbox, keys, radix sort, topology, FP64 upward
pass, pack), the wavefront tree walk (accelerations), the second kick.
value = N / (time per step): one force evaluation per step, tree build
included; the per-phase HIP-event breakdown and the interaction counts of
the simulation's walks are taken over up to 20 further steps, and the
roofline figure is their counted FLOPs over the walk kernel's event time in
those same steps.  Inputs are resident on the GPU before timing starts.  The FP64
energy diagnostic (its potential from one more walk) is taken before and
after the timed steps, and its relative change reported.

After the timed steps the direct method (every pair, FP32, no tree) is
timed once on the same bodies as the O(N^2) reference point (up to
N = 2^22).

Prints ONE JSON line.  --gpus N with N > 1 is refused: the library targets
one GPU.

--energy-table runs the paper's validation experiment instead (Sec. 5):
two Plummer clusters colliding, in standard units, theta 0.5, dt 0.01, 500
steps, FP64, one body per leaf as in the paper's tree, softening 0.003 (the
paper gives none), for N = 10000 ... 80000, with the tree code and with the
direct method; it prints one JSON line with |dE/E| in percent per run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "body-cell interactions/s and bodies/s force eval at rms rel force err 1e-3"
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# VALU issue: 256 CUs x 4 SIMDs, a wavefront instruction every four cycles
# on a SIMD (16 lanes), 2.4 GHz
VALU_SIMDS, VALU_CYCLES_PER_INSTR, CLOCK_HZ = 1024, 4, 2.4e9
# algorithmic FLOPs per interaction: particle-particle 20; particle-cell 20
# (monopole), 60 (monopole + quadrupole) or 125 (and octopole: its contraction
# with x x costs 39, the rest of the term 26)
FLOP_PP = 20
FLOP_PC = {0: 20, 2: 60, 3: 125}

# force-evaluation methods compared at the target error, with the parameter
# grid each is swept over (from accurate to cheap)
METHODS = {
    "body-theta": [round(0.5 + 0.005 * k, 3) for k in range(61)],     # Sec. 3 walk
    # the same walk with a containment guard (a cell holding the body is opened)
    "body-theta-guard": [round(0.5 + 0.005 * k, 3) for k in range(101)],
    "group-theta": [round(0.6 + 0.00625 * k, 5) for k in range(57)],  # one decision per wave
    "group-budget": [round(-2.5 + 0.03125 * k, 5) for k in range(49)],  # log10 tau
    "group-learned": [round(-5.0 + 0.03125 * k, 5) for k in range(113)],  # log10 tau
    # the opening angle with the octopole term (l = 3 of the expansion)
    "body-theta-o3": [round(0.5 + 0.005 * k, 3) for k in range(81)],
    "group-theta-o3": [round(0.6 + 0.00625 * k, 5) for k in range(73)],
    # the budget with monopole terms (the dropped quadrupole's bound charged)
    "group-budget-mono": [round(-4.0 + 0.03125 * k, 5) for k in range(89)],  # log10 tau
    # the mixed order (monopole or quadrupole per cell)
    "group-budget-mixed": [round(-4.0 + 0.03125 * k, 5) for k in range(89)],  # log10 tau
}
# the same methods over bodies sorted along the Peano-Hilbert curve
for _m in ("body-theta", "group-theta", "group-budget", "group-budget-mono",
           "group-budget-mixed", "group-learned"):
    METHODS[_m + "-hilbert"] = METHODS[_m]
PARAM_NAME = {"body-theta": "theta", "body-theta-guard": "theta", "group-theta": "theta",
              "group-budget": "log10_tau", "group-budget-mono": "log10_tau",
              "group-budget-mixed": "log10_tau",
              "group-learned": "log10_tau", "body-theta-o3": "theta", "group-theta-o3": "theta"}
for _m in ("body-theta", "group-theta", "group-budget", "group-budget-mono",
           "group-budget-mixed", "group-learned"):
    PARAM_NAME[_m + "-hilbert"] = PARAM_NAME[_m]


def order_of(method):
    """Expansion order of a method: octopole for the -o3 variants,
    monopole for the -mono ones, the mixed order (1) for the -mixed ones."""
    if method.endswith("-o3"):
        return 3
    if "-mixed" in method:
        return 1
    return 0 if "-mono" in method else 2


def hilbert(method):
    """Whether a method sorts the bodies along the Peano-Hilbert curve."""
    return method.endswith("-hilbert")


def base_of(method):
    """The method without its curve suffix."""
    return method[:-len("-hilbert")] if hilbert(method) else method
BUDGET_THETA_MAX = 1.5
# |a_i| in the budget tests is max(|a_i|, f <|a|>): f = 0.3 for the budget
# with monopole terms over Hilbert groups, 0.5 for the others (each the
# faster at rms 1e-3 on the 2^22 Plummer sphere)
ACC_FLOOR = 0.5
ACC_FLOOR_MONO_HILBERT = 0.3


def acc_floor_of(method, override=None):
    """The |a| floor of a budget method (``override`` if given)."""
    if override is not None:
        return override
    return ACC_FLOOR_MONO_HILBERT if method == "group-budget-mono-hilbert" else ACC_FLOOR
# steps after the timed ones that record the per-phase HIP events
PHASE_STEPS = 20
# fixed opening angles the per-body walk is also reported at
THETA_POINTS = (0.4, 0.5, 0.7)
# the direct method (every pair) is timed once up to this N
DIRECT_MAX_N = 1 << 22


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="c4")
    ap.add_argument("--n", type=int, default=None, help="override N")
    ap.add_argument("--leaf", type=int, default=None, help="override the leaf capacity")
    ap.add_argument("--theta", type=float, default=None,
                    help="per-body walk: skip the sweep and use this theta")
    ap.add_argument("--method", default=None,
                    help="calibrate only this method, or a comma-separated list of them, and "
                    "time the fastest (default: all of " + ", ".join(METHODS) + ")")
    ap.add_argument("--target-err", type=float, default=1e-3)
    ap.add_argument("--acc-floor", type=float, default=None,
                    help="budget criteria: |a_i| floored at this fraction of the mean |a| "
                    f"(default {ACC_FLOOR_MONO_HILBERT} for group-budget-mono-hilbert, else "
                    f"{ACC_FLOOR})")
    ap.add_argument("--theta-max", type=float, default=BUDGET_THETA_MAX,
                    help="budget criteria: cells above this opening angle are opened")
    ap.add_argument("--walk-cap", type=int, default=0,
                    help="group walk work cap (0: the library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20,
                    help="bodies the CPU oracle walks (the tree is built in full)")
    ap.add_argument("--energy-table", action="store_true",
                    help="run the two-cluster energy-conservation experiment and exit")
    ap.add_argument("--table-n", default="10000,20000,40000,60000,80000")
    ap.add_argument("--table-steps", type=int, default=500)
    ap.add_argument("--table-eps", type=float, default=0.003)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (to scale "
                         "the profiler's FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def copy_calibration(mib: int):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "reps": 3}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        log("bench.py: only --gpus 1 is supported (single-GPU build)")
        sys.exit(2)

    import torch

    from paper_2203_08966_amd import binding as B
    from paper_2203_08966_amd import workloads as W

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if not torch.cuda.is_available():
        log("bench.py needs a GPU")
        sys.exit(1)
    B.load()
    if args.energy_table:
        energy_table(args)
        return
    bodies, cfg = W.config(args.config, n=args.n)
    if args.leaf is not None:
        cfg = dict(cfg, leaf=args.leaf)
    n = bodies.n
    eps, leaf, dt, order = cfg["eps"], cfg["leaf"], cfg["dt"], 2
    dtype = torch.float32 if cfg["dtype"] == "f32" else torch.float64
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(np.ascontiguousarray(bodies.pos)).to(dev)
    vel = torch.from_numpy(np.ascontiguousarray(bodies.vel)).to(dev)
    mass = torch.from_numpy(np.ascontiguousarray(bodies.mass)).to(dev)
    ctx = B.bh_ctx_create(0)
    log(f"workload {cfg['workload']} N={n} eps={eps} leaf={leaf} dtype={cfg['dtype']}")

    # ---- error reference: FP64 direct sum on a seeded subsample (GPU)
    sample = W.subsample(n, 4096, cfg.get("sub_seed", 100))
    tg = torch.from_numpy(sample).to(dev)
    tg_long = tg.to(torch.int64)
    acc_dir = torch.empty((len(sample), 3), dtype=torch.float64, device=dev)
    B.bh_direct(ctx, pos, mass, tg, eps, acc_dir)
    torch.cuda.synchronize()
    ref = acc_dir.cpu().numpy()

    tree = B.bh_build(ctx, pos, mass, leaf)
    acc = torch.empty_like(pos)
    npp = torch.zeros(n, dtype=torch.int32, device=dev)
    npc = torch.zeros(n, dtype=torch.int32, device=dev)
    # |a_i| for the error-budget criterion while calibrating (in the timed
    # steps each step uses the previous step's accelerations)
    B.bh_forces(tree, 0.5, eps, acc, B.force_opts(order=order))
    anorm = acc.norm(dim=1).contiguous()

    # network operands of the learned criterion (fp16 where the workload asks)
    mlp_precision = B.BH_MLP_FP16 if cfg.get("mlp") == "fp16" else B.BH_MLP_BF16

    def opts_of(method, p, counters=False, for_sim=False):
        kw = dict(order=order_of(method), n_pp=npp if counters else None,
                  n_pc=npc if counters else None)
        floor = acc_floor_of(method, args.acc_floor)
        method = base_of(method)
        if method == "body-theta-guard":
            kw.update(mac=B.BH_MAC_THETA_GUARD)
        elif method in ("group-theta", "group-theta-o3"):
            kw.update(walk=B.BH_WALK_GROUP, walk_cap=args.walk_cap)
        elif method in ("group-budget", "group-budget-mono", "group-budget-mixed",
                        "group-learned"):
            kw.update(walk=B.BH_WALK_GROUP, walk_cap=args.walk_cap, mlp_precision=mlp_precision,
                      mac=B.BH_MAC_MLP if method == "group-learned" else B.BH_MAC_BUDGET,
                      mlp_log10_tau=p, mlp_theta_max=args.theta_max,
                      mlp_acc_norm=None if for_sim else anorm, mlp_acc_floor=floor)
        return B.force_opts(**kw)

    def walk(method, p, counters=False):
        theta = p if PARAM_NAME[method] == "theta" else 0.5
        B.bh_forces(tree_h if hilbert(method) else tree, theta, eps, acc,
                    opts_of(method, p, counters))

    def rms_at(method, p):
        walk(method, p)
        a = acc.index_select(0, tg_long).cpu().numpy().astype(np.float64)
        e = np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)
        return float(np.sqrt(np.mean(e * e)))

    def walk_ms(method, p, reps=10):
        for _ in range(3):
            walk(method, p)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            walk(method, p)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    names = list(METHODS) if args.method is None else args.method.split(",")
    for k in names:
        if k not in METHODS:
            raise SystemExit(f"unknown method {k!r}; choose from {', '.join(METHODS)}")
    # the same bodies sorted along the Peano-Hilbert curve
    tree_h = None
    if any(hilbert(k) for k in names):
        B.bh_ctx_set_curve(ctx, B.BH_CURVE_HILBERT)
        tree_h = B.bh_build(ctx, pos, mass, leaf)
        B.bh_ctx_set_curve(ctx, B.BH_CURVE_MORTON)
    # ---- the learned criterion: train the network on the library's own FP64
    # simulations of small Plummer spheres (bf16 MFMA inference afterwards)
    learned_info = None
    if "group-learned" in names or "group-learned-hilbert" in names:
        from paper_2203_08966_amd import learned as LM
        t0 = time.perf_counter()
        feat, label = LM.training_set(ctx)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = LM.train(ctx, feat, label)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        learned_info = {"pairs": int(feat.shape[0]), "epochs": len(loss),
                        "loss_first_last": [float(loss[0]), float(loss[-1])],
                        "label_var": float(label.double().var().item()),
                        "seconds": t2 - t0, "train_seconds": t2 - t1,
                        "inference": "fp16" if mlp_precision == B.BH_MLP_FP16 else "bf16"}
        learned_info["roofline"] = mlp_roofline(B, ctx, feat, len(loss), t2 - t1, mlp_precision)
        log(f"network roofline: {learned_info['roofline']}")
        del feat, label
        log(f"learned criterion: {learned_info}")

    # ---- per method: the cheapest parameter on its grid with rms <= target
    methods = {}
    for name in names:
        grid = METHODS[name]
        if name == "body-theta" and args.theta is not None:
            grid = [args.theta]
        sweep, best = [], None
        for p in grid:
            r = rms_at(name, p)
            sweep.append([p, r])
            if r <= args.target_err:
                best = p
            elif r > 1.5 * args.target_err:
                break
        if best is None:
            log(f"{name}: no grid value reaches rms {args.target_err}")
            continue
        walk(name, best, counters=True)
        torch.cuda.synchronize()
        s_pp = int(npp.to(torch.int64).sum().item())
        s_pc = int(npc.to(torch.int64).sum().item())
        methods[name] = {"param": best, "rms_rel_err": rms_at(name, best),
                         "walk_ms": walk_ms(name, best),
                         "interactions_per_eval": {"pp": s_pp, "pc": s_pc}, "sweep": sweep}
        log(f"{name}: param {best} rms {methods[name]['rms_rel_err']:.3e} "
            f"walk {methods[name]['walk_ms']:.3f} ms  pp/body {s_pp / n:.0f} pc/body {s_pc / n:.0f}")
    # ---- the paper's per-body walk at fixed angles and at the target error
    theta_points = {}
    if "body-theta" in names:
        for th in THETA_POINTS:
            walk("body-theta", th, counters=True)
            torch.cuda.synchronize()
            t_pp = int(npp.to(torch.int64).sum().item())
            t_pc = int(npc.to(torch.int64).sum().item())
            wm = walk_ms("body-theta", th)
            theta_points[str(th)] = {
                "rms_rel_err": rms_at("body-theta", th), "walk_ms": wm,
                "bodies_per_s": n / (wm * 1e-3),
                "interactions_per_s": (t_pp + t_pc) / (wm * 1e-3),
                "interactions_per_eval": {"pp": t_pp, "pc": t_pc}}
            log(f"body-theta at {th}: rms {theta_points[str(th)]['rms_rel_err']:.3e} "
                f"walk {wm:.3f} ms")
        th_t = interp_theta(methods.get("body-theta", {}).get("sweep", []), args.target_err)
        if th_t is not None:
            walk("body-theta", th_t, counters=True)
            torch.cuda.synchronize()
            t_pp = int(npp.to(torch.int64).sum().item())
            t_pc = int(npc.to(torch.int64).sum().item())
            wm = walk_ms("body-theta", th_t)
            theta_points["at_target"] = {
                "theta": th_t, "rms_rel_err": rms_at("body-theta", th_t), "walk_ms": wm,
                "bodies_per_s": n / (wm * 1e-3),
                "interactions_per_s": (t_pp + t_pc) / (wm * 1e-3),
                "interactions_per_eval": {"pp": t_pp, "pc": t_pc}}
            log(f"body-theta interpolated to rms {args.target_err}: theta {th_t:.4f} "
                f"walk {wm:.3f} ms")
    B.bh_tree_free(tree)
    if tree_h is not None:
        B.bh_tree_free(tree_h)
    chosen = min(methods, key=lambda k: methods[k]["walk_ms"])
    cp = methods[chosen]["param"]
    log(f"timed method: {chosen} ({PARAM_NAME[chosen]} = {cp})")

    # ---- timed simulation steps
    sim_theta = cp if PARAM_NAME[chosen] == "theta" else 0.5
    B.bh_ctx_set_curve(ctx, B.BH_CURVE_HILBERT if hilbert(chosen) else B.BH_CURVE_MORTON)
    B.bh_sim_init(ctx, pos, vel, mass, leaf, sim_theta, eps, opts_of(chosen, cp, for_sim=True))
    for _ in range(args.warmup):
        B.bh_leapfrog_step(ctx, dt)
    ek0, ep0 = B.bh_energy(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.bh_leapfrog_step(ctx, dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the phase breakdown (HIP events in every step) from further steps, so
    # that the events do not load the timed ones
    B.bh_sim_timing(ctx, True)
    for _ in range(min(args.steps, PHASE_STEPS)):
        B.bh_leapfrog_step(ctx, dt)
    phase_ms, nsteps = B.bh_sim_timing_get(ctx)
    sim_pp, sim_pc = B.bh_sim_counts_get(ctx)
    sim_pq = B.bh_sim_counts_pq_get(ctx)  # cell terms with the quadrupole
    # bodies the last rebuild's adaptive re-sort moved (-1: it sorted in full)
    movers = int(B.bh_tree_info_get(B.bh_sim_tree(ctx))["movers"])
    B.bh_sim_timing(ctx, False)
    ek, ep = B.bh_energy(ctx)
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_step * 1e-3)
    phases = {k: v / max(nsteps, 1) for k, v in
              zip(["kick_drift", "build", "walk", "kick", "walk_kernel"], phase_ms)}
    walk_step_ms = phases["walk"]
    walk_kernel_ms = phases["walk_kernel"]
    # accuracy of the timed method at the final state of the run
    xf, af = torch.empty_like(pos), torch.empty_like(pos)
    B.bh_sim_get(ctx, xf, None, af)
    ref_f = torch.empty((len(sample), 3), dtype=torch.float64, device=dev)
    B.bh_direct(ctx, xf, mass, tg, eps, ref_f)
    a_f = af.index_select(0, tg_long).cpu().numpy().astype(np.float64)
    r_f = ref_f.cpu().numpy()
    e_f = np.linalg.norm(a_f - r_f, axis=1) / np.linalg.norm(r_f, axis=1)
    rms_final = float(np.sqrt(np.mean(e_f * e_f)))
    err_final = {"rms": rms_final, "median": float(np.median(e_f)),
                 "p99": float(np.quantile(e_f, 0.99)), "max": float(e_f.max())}
    # interactions per walk of the recorded simulation steps (the walks the
    # walk kernel's event time is taken over)
    s_pp = sim_pp / max(nsteps, 1)
    s_pc = sim_pc / max(nsteps, 1)
    s_pq = sim_pq / max(nsteps, 1)
    inter = s_pp + s_pc
    if order_of(chosen) == 1:  # monopole and quadrupole cell terms
        flops = FLOP_PP * s_pp + FLOP_PC[0] * (s_pc - s_pq) + FLOP_PC[2] * s_pq
    else:
        flops = FLOP_PP * s_pp + FLOP_PC[order_of(chosen)] * s_pc
    achieved_tf = flops / (walk_kernel_ms * 1e-3) / 1e12
    log(f"step {ms_step:.3f} ms  phases {phases}  rms at the final state {rms_final:.3e}")

    kernel = "k_walk" if chosen.startswith("body-") else "k_gwalk"
    B.bh_ctx_set_curve(ctx, B.BH_CURVE_MORTON)
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "bodies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == torch.float32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": result_workload(cfg, n),
            "n": n, "eps": eps, "leaf": leaf, "order": order_of(chosen), "dt": dt,
            "curve": "hilbert" if hilbert(chosen) else "morton",
            "method": chosen, PARAM_NAME[chosen]: cp,
            **({"theta_max": args.theta_max, "acc_floor": acc_floor_of(chosen, args.acc_floor),
                "walk_cap": args.walk_cap or "library default"}
               if PARAM_NAME[chosen] == "log10_tau" else {}),
            **({"mlp": "fp16" if mlp_precision == B.BH_MLP_FP16 else "bf16"}
               if base_of(chosen) == "group-learned" else {}),
            "step": "KDK leapfrog step: kick+drift, rebuild, walk (accelerations), kick; "
                    "energy before and after the timed steps",
        },
        "rms_rel_err": methods[chosen]["rms_rel_err"],
        "rms_rel_err_final_state": rms_final,
        "rel_err_final_state": err_final,
        "interactions_per_s": inter / (walk_step_ms * 1e-3),
        # particle-cell terms weighted 2 (the paper's cost weights, Sec. 4.5)
        "weighted_interactions_per_s": (s_pp + 2 * s_pc) / (walk_step_ms * 1e-3),
        "interactions_per_eval": {"pp": s_pp, "pc": s_pc, "pc_quadrupole": s_pq,
                                  "source": f"mean over the {nsteps} recorded simulation steps"},
        "walk_bodies_per_s": n / (walk_step_ms * 1e-3),
        "body_theta_points": theta_points,
        "phases_ms": phases,
        "phase_steps": int(nsteps),
        "resort_movers_last_step": movers,
        "energy_rel_change": abs((ek + ep) - (ek0 + ep0)) / abs(ek0 + ep0),
        "methods": methods,
        "learned_training": learned_info,
        "roofline": {
            "bound": "alu",
            "kernel": f"{kernel} (FP32, "
                      f"{ {0: 'monopole', 1: 'mixed monopole/quadrupole', 2: 'quadrupole', 3: 'octopole'}[order_of(chosen)]})",
            "achieved": achieved_tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved_tf / PEAK_FP32_TFLOPS,
            "traffic": traffic_for(kernel, result_workload(cfg, n), chosen),
            "flop_per_launch": flops, "launch_ms": walk_kernel_ms,
            "valu_issue": valu_issue_for(kernel, result_workload(cfg, n), chosen, walk_kernel_ms),
        },
    }

    if n <= DIRECT_MAX_N:
        result["direct_method"] = direct_method(ctx, pos, vel, mass, leaf, eps, tg, ref,
                                                walk_step_ms)
    else:
        result["direct_method"] = {"skipped": f"N > {DIRECT_MAX_N}: one all-pairs evaluation "
                                              "would take minutes"}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(bodies, cfg, methods.get("body-theta", {}).get(
            "param", 0.6), order, args.cpu_sample)
    B.bh_ctx_destroy(ctx)
    print(json.dumps(result), flush=True)


def direct_method(ctx, pos, vel, mass, leaf, eps, tg, ref, walk_step_ms):
    """One force evaluation of the direct method (every pair, the
    simulation's dtype, no tree) on the timed workload's initial bodies:
    its kernel time, rate and error against the FP64 reference sum."""
    import torch
    from paper_2203_08966_amd import binding as B
    n = int(mass.shape[0])
    o = B.force_opts(walk=B.BH_WALK_DIRECT)
    B.bh_sim_init(ctx, pos, vel, mass, leaf, 0.5, eps, o)
    B.bh_sim_timing(ctx, True)
    B.bh_leapfrog_step(ctx, 0.0)  # dt 0: the same positions again
    ms, _ = B.bh_sim_timing_get(ctx)
    B.bh_sim_timing(ctx, False)
    a = torch.empty_like(pos)
    B.bh_sim_get(ctx, None, None, a)
    a = a.index_select(0, tg.to(torch.int64)).cpu().numpy().astype(np.float64)
    e = np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)
    t = ms[4]
    log(f"direct method: {t:.1f} ms per force evaluation, rms {np.sqrt(np.mean(e * e)):.2e}")
    return {"ms": t, "bodies_per_s": n / (t * 1e-3),
            "interactions_per_s": n * (n - 1) / (t * 1e-3),
            "rms_rel_err": float(np.sqrt(np.mean(e * e))),
            "tree_walk_speedup": t / walk_step_ms}


def energy_table(args):
    """Sec. 5's validation: |dE/E| (percent) after the run, per N and method."""
    import torch
    from paper_2203_08966_amd import binding as B
    from paper_2203_08966_amd import workloads as W
    ctx = B.bh_ctx_create(0)
    dev = torch.device("cuda:0")
    theta, dt, eps, steps, seed = 0.5, 0.01, args.table_eps, args.table_steps, 2203
    rows = []
    for n in [int(v) for v in args.table_n.split(",")]:
        b = W.two_clusters(n, seed)
        P, V, M = (torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
                   for a in (b.pos, b.vel, b.mass))
        B.bh_standard_units(ctx, P, V, M)
        for name, opts in (("direct", B.force_opts(walk=B.BH_WALK_DIRECT)),
                           ("tree", B.force_opts(order=2))):
            B.bh_sim_init(ctx, P, V, M, 1, theta, eps, opts)
            e0 = sum(B.bh_energy(ctx))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(steps):
                B.bh_leapfrog_step(ctx, dt)
                if (k + 1) % 100 == 0:
                    B.bh_energy(ctx)  # paces the queue; also a progress point
                    log(f"  N={n} {name}: step {k + 1}")
            e1 = sum(B.bh_energy(ctx))
            t1 = time.perf_counter()
            rows.append({"n": n, "method": name, "E0": e0, "E_end": e1,
                         "dE_over_E_percent": 100.0 * abs(e1 - e0) / abs(e0),
                         "ms_per_step": (t1 - t0) * 1e3 / steps})
            log(f"N={n} {name}: E0 {e0:.6f} |dE/E| {rows[-1]['dE_over_E_percent']:.4f} % "
                f"({rows[-1]['ms_per_step']:.2f} ms/step)")
    B.bh_ctx_destroy(ctx)
    print(json.dumps({"energy_table": rows, "config": {
        "workload": f"two Plummer clusters (offset +-2 (1,1,1), at rest), standard units, "
                    f"seed {seed}",
        "theta": theta, "dt": dt, "steps": steps, "eps": eps, "leaf": 1, "order": 2,
        "dtype": "f64"}}), flush=True)


def result_workload(cfg, n):
    what = {"plummer": "equal masses, G=M=a=1",
            "two_spheres": "radii 1 and 0.3, lognormal masses, approaching",
            "clumpy": "4096 Plummer clumps + 10% background, equal masses"}[cfg["workload"]]
    return f"{cfg['workload']} N={n} ({what}, seed {cfg['seed']})"


# the network 10 -> 32 -> 32 -> 1: FLOPs of one evaluation (two per
# multiply-add), and of one training sample (forward and backward, about
# three evaluations)
MLP_FLOP = 2 * (10 * 32 + 32 * 32 + 32)
MLP_TRAIN_FLOP = 3 * MLP_FLOP
PEAK_MFMA_16BIT_TFLOPS = 2500.0


def mlp_roofline(B, ctx, feat, epochs, train_s, precision):
    """The network's roofline figures: the batched MFMA inference kernel over
    the training features (10 FP32 features read per row: HBM-bound at
    2752 / 40 flop per byte, below the MFMA ridge), and the training pass
    (FP32 MFMA, whole bh_mlp_train call, against the FP32 peak)."""
    import torch
    n = int(feat.shape[0])
    B.bh_mlp_infer(ctx, feat, precision)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        B.bh_mlp_infer(ctx, feat, precision)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    inf_tf = n * MLP_FLOP / (ms * 1e-3) / 1e12
    gbs = n * 44 / (ms * 1e-3) / 1e9  # 40 B of features in, 4 B out per row
    tr_tf = n * epochs * MLP_TRAIN_FLOP / train_s / 1e12
    return {
        "infer": {"kernel": "k_mlp_infer (" + ("fp16" if precision else "bf16") + " MFMA)",
                  "rows": n, "ms": ms, "flop_per_row": MLP_FLOP, "achieved": inf_tf,
                  "peak": PEAK_MFMA_16BIT_TFLOPS, "unit": "TFLOP/s",
                  "frac": inf_tf / PEAK_MFMA_16BIT_TFLOPS, "bound": "hbm",
                  "hbm_gbs": gbs, "hbm_frac": gbs / PEAK_HBM_GBS},
        "train": {"kernel": "k_mlp_grad (FP32 MFMA) + k_mlp_adam", "samples": n,
                  "epochs": epochs, "seconds": train_s, "flop_per_sample": MLP_TRAIN_FLOP,
                  "achieved": tr_tf, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                  "frac": tr_tf / PEAK_FP32_TFLOPS},
    }


def traffic_for(kernel, workload, method):
    """HBM bytes per launch of the timed walk kernel from the committed
    rocprofv3 counter summary, if it was taken on this workload and method
    with the current walk source; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "walk_traffic.json")
    src = os.path.join(ROOT, "paper_2203_08966_amd", "csrc", "walk.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if (not k or rec.get("walk_hip_sha256") != sha or rec.get("workload") != workload
            or k.get("method") != method):
        return None
    return k["hbm_bytes_per_launch"]


def valu_issue_for(kernel, workload, method, launch_ms):
    """The walk kernel's wavefront VALU instructions per launch from the
    committed rocprofv3 counter summary (same workload, method and walk
    source, else None), and the time they take at one instruction per four
    cycles on every SIMD, against the launch's measured time."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "walk_valu.json")
    src = os.path.join(ROOT, "paper_2203_08966_amd", "csrc", "walk.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if (not k or rec.get("walk_hip_sha256") != sha or rec.get("workload") != workload
            or k.get("method") != method):
        return None
    v = k["valu_instr_per_launch"]
    ms = v * VALU_CYCLES_PER_INSTR / VALU_SIMDS / CLOCK_HZ * 1e3
    return {"valu_instr_per_launch": v, "ms_at_4_cycles_per_instr": ms,
            "launch_ms": launch_ms, "issue_frac": ms / launch_ms}


def cpu_model() -> str:
    """The host CPU's model name (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def interp_theta(sweep, target):
    """The theta at which the rms error reaches ``target``: log-log linear
    interpolation between the two swept angles that bracket it (rms grows
    with theta); None if no pair brackets it."""
    pts = sorted((float(t), float(r)) for t, r in sweep if r > 0)
    for (t0, r0), (t1, r1) in zip(pts, pts[1:]):
        if r0 <= target <= r1 and r1 > r0:
            f = (np.log(target) - np.log(r0)) / (np.log(r1) - np.log(r0))
            return float(np.exp(np.log(t0) + f * (np.log(t1) - np.log(t0))))
    return None


def cpu_baseline(bodies, cfg, theta, order, k):
    """The FP64 C oracle on the host cores: full tree build over all N bodies
    plus the walk of a seeded sample of k bodies; bodies/s extrapolated as
    N / (t_build + t_walk * N / k)."""
    import oracle
    from paper_2203_08966_amd import workloads as W
    oracle.build(force=False)
    p64 = bodies.pos.astype(np.float64)
    m64 = bodies.mass.astype(np.float64)
    n = len(m64)
    t0 = time.perf_counter()
    built = oracle.build_all(p64, m64, cfg["leaf"])
    t1 = time.perf_counter()
    sample = W.subsample(n, k, 4242)
    r = oracle.barnes_hut(None, None, theta, cfg["eps"], cfg["leaf"], order=order,
                          targets=sample, built=built)
    t2 = time.perf_counter()
    t_eval = (t1 - t0) + (t2 - t1) * n / len(sample)
    log(f"cpu oracle: build {t1 - t0:.2f} s, walk of {len(sample)} bodies {t2 - t1:.2f} s")
    # the oracle's FP64 direct sum over all N sources for a few targets
    dt_targets = W.subsample(n, 256, 4343)
    t3 = time.perf_counter()
    oracle.direct(p64, m64, cfg["eps"], dt_targets)
    t4 = time.perf_counter()
    log(f"cpu oracle: direct sum for {len(dt_targets)} targets {t4 - t3:.2f} s")
    return {
        "value": n / t_eval, "unit": "bodies/s", "cores": oracle.num_threads(),
        "cpu_model": cpu_model(), "kind": "oracle",
        "sample": f"full FP64 tree build of all {n} bodies ({t1 - t0:.2f} s) + walk of "
                  + (f"all {n} bodies ({t2 - t1:.2f} s)" if len(sample) == n else
                     f"{len(sample)} sampled bodies ({t2 - t1:.2f} s), extrapolated to N"),
        "interactions_per_s": float((r.npp.sum() + r.npc.sum()) / (t2 - t1)),
        "direct_sum": {"targets": int(len(dt_targets)), "seconds": t4 - t3,
                       "interactions_per_s": len(dt_targets) * (n - 1) / (t4 - t3)},
    }


if __name__ == "__main__":
    main()
