"""Charge solves per second of the CPM electrode charge solve on one MI355X.

    python bench.py [--steps K] [--warmup W] [--batch B] [--mode bf16r|f64|f32r]

Workload: the 2880-atom graphite capacitor (2 x 3 AB layers of 480 atoms,
34.08 x 36.89 A cell, 50 A gap, 2000 SPC/E-like waters + 64 NaCl pairs,
dV = 2 V, eta 1.979, alpha 0.3, r_c 12 A, k-space accuracy 1e-8, slab factor
3) with B Gaussian-jittered (sigma 0.1 A) electrolyte snapshots per step.

One step is one pass of the whole hot path over one batch: assemble A (FP64),
Cholesky-invert it and form S (FP64), set the applied potential, then for all
B snapshots compute b and solve q = S (b + v) with the neutrality projection
and electrode totals.  `value` = B * K / (timed seconds).  Inputs are
resident in HBM before the timed region; all work runs in libcpm's kernels.

The same line carries the metric's second point (the 20064-atom capacitor,
128 configurations per step, Ewald split retuned to alpha 0.19 / r_c 18.95 A
at the same truncation accuracy), the uneven eight-capacitor batch, the
batched FP64 matrix-core comparator, warm and cache-flushed matvec rates, the
real-space kernel's roofline and the FP64 oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MODES = {
    # name: (store flags, b in fp32, solve mode, dtype label).  The reduced-
    # precision modes keep b in FP32 (structure factors on FP16 matrix cores
    # with split operands) and refine q once against A in FP64.
    "f64": (1, False, 0x000, "f64"),
    "f32r": (1 | 2, True, 0x101, "b f32, S f32, f64 refine"),
    "bf16r": (1 | 4, True, 0x102, "b f32, S bf16x3 (f32 accumulation), f64 refine"),
    "bf16r64": (1 | 4, False, 0x102, "b f64, S bf16x3 (f32 accumulation), f64 refine"),
}
# dominant kernel families and their algorithmic work per launch
PEAK_FP64_VALU = 78.6e12     # FLOP/s, MI355X FP64 vector
PEAK_FP64_MFMA = 78.6e12     # FLOP/s, MI355X dense FP64 matrix cores
PEAK_FP32_VALU = 157.3e12
PEAK_FP16_MFMA = 2.5e15      # FLOP/s, MI355X dense FP16 matrix cores
PEAK_HBM = 8.0e12            # B/s
DOMINANT = "structure_factor"
# Ewald split of the 20064-atom capacitor: q does not depend on alpha; a
# smaller alpha moves work from the k-space sum (|K+| ~ alpha^3) to the real
# space (r_c^3 ~ alpha^-3); r_c = 3.6 / alpha keeps erfc(alpha r_c) at its
# alpha 0.3, r_c 12 A value and k_c = 2 alpha sqrt(ln 1e8) the k-space accuracy
ALPHA_20K = 0.19
REAL_SPACE_FLOP_PER_PAIR = 50.0   # one erfc-difference pair term (distance, g(r), accumulate)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=None,
                    help="snapshots per step (default 1000 at n=2880, 128 at n=20064)")
    ap.add_argument("--mode", default="bf16r", choices=sorted(MODES))
    ap.add_argument("--workload", default="graphite_capacitor_2880",
                    choices=["graphite_capacitor_2880", "graphite_capacitor_20064", "mixed8"])
    ap.add_argument("--no-20k", action="store_true",
                    help="skip the secondary one-step measurement at N = 20064")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the uneven eight-capacitor step")
    ap.add_argument("--alpha20k", type=float, default=ALPHA_20K,
                    help="Ewald alpha at N = 20064 (r_c = 3.6 / alpha keeps erfc(alpha r_c))")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device copy (for HBM counter scaling under rocprofv3)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; multi-GPU sharding is a "
                                   "design note, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2203_15461_amd import cpm
    from paper_2203_15461_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cpm.lib()
    if args.workload == "mixed8":
        out = run_mixed(args)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "graphite_capacitor_2880":
        w = I.graphite_capacitor()
        B = args.batch or 1000
    else:
        w = large_capacitor(args.alpha20k)
        B = args.batch or 128
    out = run_workload(args, w, B, args.workload, args.steps, args.warmup, args.calibrate_copy)
    if args.workload == "graphite_capacitor_2880":
        out["batched_comparator"] = batched_comparator(w)
    if args.workload == "graphite_capacitor_2880" and not args.no_20k:
        # the metric's second point: one step at N = 20064 with 128
        # configurations, the per-capacitor snapshot count of the uneven batch
        w20 = large_capacitor(args.alpha20k)
        r = run_workload(args, w20, 128, "graphite_capacitor_20064", 1, 1, False)
        out["workload_20064"] = {k: r[k] for k in ("value", "ms_per_step", "config", "roofline",
                                                   "roofline_real_space", "phase_s",
                                                   "solve_only_rate", "plain_fp64_per_step_rate",
                                                   "graph_fp64_per_step", "matvec_roofline",
                                                   "conjugate_gradient", "max_abs_sum_q")}
        out["workload_20064_factor"] = run_factor_step(w20, 128, 1, 1, True)
        out["workload_20064_factor_f64"] = run_factor_step(w20, 128, 1, 1, False)
    if args.workload == "graphite_capacitor_2880" and not args.no_mixed:
        margs = argparse.Namespace(**vars(args))
        margs.steps, margs.warmup, margs.batch = 1, 1, None
        out["mixed8"] = run_mixed(margs)
    if not args.no_cpu_baseline and w.n < 10000:
        out["cpu_baseline"], q_ref, Q_ref = cpu_baseline(w)
        out["accuracy_vs_oracle"] = accuracy_vs_oracle(w, q_ref, Q_ref)
    print(json.dumps(out), flush=True)


def run_factor_step(w, B, steps, warmup, b_f32):
    """The same step with the factor-only inverse (CPM_INVERT_FACTOR): A is
    assembled and Cholesky-factored on the second stream while b runs, and
    q = P A^-1 b + d comes from forward and back substitution with the
    factor for all B configurations (FP64 solve; no L^-1, A^-1 or S); b in
    FP64, or in FP32 from the FP32 structure factors (b_f32)."""
    import torch
    from paper_2203_15461_amd import cpm
    from paper_2203_15461_amd import inputs as I
    dev = torch.device("cuda:0")
    xyz = synthetic_configurations(w, B, I.BASE_SEED + 1, dev)
    R = torch.as_tensor(w.electrode_xyz, dtype=torch.float64, device=dev).contiguous()
    eid = torch.as_tensor(w.electrode_id, dtype=torch.int32, device=dev).contiguous()
    bvec = torch.empty((B, w.n), dtype=torch.float32 if b_f32 else torch.float64, device=dev)
    q = torch.empty((B, w.n), dtype=torch.float64, device=dev)
    Qe = torch.empty((B, 2), dtype=torch.float64, device=dev)
    ctx = cpm.Context(cpm.Params.of(w))
    ctx.set_electrolyte(w.electrolyte_q)
    flags = cpm.STORE_F64 | cpm.INVERT_FACTOR

    def step():
        ctx.build_elastance(R, eid, 2)
        ctx.invert(flags | cpm.INVERT_ASYNC)
        ctx.potential_vector(xyz, bvec)
        ctx.set_potential(w.v_electrode)
        ctx.solve_charges(bvec, 0x000, q, Qe)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # phases of one more step, serialised
    ts = time.perf_counter()
    ctx.build_elastance(R, eid, 2)
    ctx.invert(flags)
    ctx.set_potential(w.v_electrode)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - ts
    ts = time.perf_counter()
    ctx.potential_vector(xyz, bvec)
    torch.cuda.synchronize()
    b_s = time.perf_counter() - ts
    ts = time.perf_counter()
    ctx.solve_charges(bvec, 0x000, q, Qe)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - ts
    out = {"value": B * steps / elapsed, "ms_per_step": elapsed / steps * 1e3,
           "dtype": "b f32, f64 factor solve" if b_f32 else "f64",
           "solver": "Cholesky factor, forward and back substitution for all configurations",
           "phase_s": {"setup": setup_s, "b_all_snapshots": b_s, "solve_all_snapshots": solve_s},
           "max_abs_sum_q": float(q.sum(dim=1).abs().max().item())}
    ctx.close()
    return out


def large_capacitor(alpha):
    """The 20064-atom capacitor with the Ewald split at alpha, r_c = 3.6 / alpha."""
    from paper_2203_15461_amd import inputs as I
    return I.scaled_graphite_capacitor(20000).with_(alpha=alpha, rcut=3.6 / alpha)


def synthetic_configurations(w, B, seed, dev):
    """B Gaussian-jittered (sigma 0.1 A) copies of the electrolyte, x and y wrapped."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    base = w.electrolyte_xyz
    snaps = base[None] + rng.normal(0.0, 0.1, size=(B,) + base.shape)
    snaps[..., 0] %= w.Lx
    snaps[..., 1] %= w.Ly
    return torch.as_tensor(snaps, dtype=torch.float64, device=dev).contiguous()


def run_workload(args, w, B, name, steps, warmup, calibrate_copy):
    import torch
    from paper_2203_15461_amd import cpm
    from paper_2203_15461_amd import inputs as I
    dev = torch.device("cuda:0")
    store, b_f32, mode, dtype = MODES[args.mode]
    t0 = time.time()
    xyz = synthetic_configurations(w, B, I.BASE_SEED + 1, dev)
    R = torch.as_tensor(w.electrode_xyz, dtype=torch.float64, device=dev).contiguous()
    eid = torch.as_tensor(w.electrode_id, dtype=torch.int32, device=dev).contiguous()
    bvec = torch.empty((B, w.n), dtype=torch.float32 if b_f32 else torch.float64, device=dev)
    q = torch.empty((B, w.n), dtype=torch.float64, device=dev)
    Qe = torch.empty((B, 2), dtype=torch.float64, device=dev)
    if calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] {name}: inputs ready in {time.time() - t0:.1f}s: n={w.n} m={w.m} batch={B} "
          f"mode={args.mode}", file=sys.stderr, flush=True)

    ctx = cpm.Context(cpm.Params.of(w))
    ctx.set_electrolyte(w.electrolyte_q)

    def step():
        # the inversion runs on a second stream while b is computed (b does
        # not depend on A); set_potential joins it
        ctx.build_elastance(R, eid, 2)
        ctx.invert(store | cpm.INVERT_ASYNC)
        ctx.potential_vector(xyz, bvec)
        ctx.set_potential(w.v_electrode)
        ctx.solve_charges(bvec, mode, q, Qe)

    tune = None
    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        if i == 0 and store & cpm.STORE_BF16X2:
            tune = ctx.autotune(B, reps=3)      # tile shapes of the batched product
        print(f"[bench] {name}: warmup {i + 1}/{warmup} done", file=sys.stderr, flush=True)

    # timed region: HIP events bracket only the dominant kernel's launches
    ctx.enable_timing(DOMINANT)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    sf_ms, sf_cnt = ctx.timing(DOMINANT)
    print(f"[bench] {name}: {steps} steps in {elapsed:.3f}s", file=sys.stderr, flush=True)

    # per-family kernel breakdown from one more step with every launch timed
    ctx.enable_timing(True)
    step()
    fams = ["sf_tables", "structure_factor", "sf_reduce", "kspace_project", "projection", "real_space_b", "combine",
            "gemm_f64", "gemm_bf16x3", "matvec_f64", "matvec_f32", "finalize", "potrf_diag",
            "chol_update", "trtri", "lauum", "assemble_real", "assemble_kspace",
            "row_means", "pad_rows", "make_rhs", "center_rows"]
    timing = {f: ctx.timing(f) for f in fams}
    ctx.enable_timing(False)
    rs_roof = real_space_roofline(w, xyz, R, eid, bvec, int(ctx.info("group")), name)

    # per-phase split of one more (untimed) step, for the JSON context fields
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ctx.build_elastance(R, eid, 2)
    ctx.invert(store)
    ctx.set_potential(w.v_electrode)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - ts
    ts = time.perf_counter()
    ctx.potential_vector(xyz, bvec)
    torch.cuda.synchronize()
    b_s = time.perf_counter() - ts
    ts = time.perf_counter()
    ctx.solve_charges(bvec, mode, q, Qe)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - ts
    qsum = float(q.sum(dim=1).abs().max().item())

    # plain FP64 per-step path for comparison: one snapshot at a time,
    # b then q = S (b + v) as a streaming FP64 matvec (A and S already built)
    ctx.invert(1)
    ctx.set_potential(w.v_electrode)
    n_plain = min(B, 100 if w.n < 10000 else 8)
    b1 = torch.empty((1, w.n), dtype=torch.float64, device=dev)
    q1 = torch.empty((1, w.n), dtype=torch.float64, device=dev)
    Qe1 = torch.empty((1, 2), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for s_ in range(n_plain):
        ctx.potential_vector(xyz[s_:s_ + 1], b1)
        ctx.solve_charges(b1, 0x000, q1, Qe1)
    t_host = time.perf_counter()
    torch.cuda.synchronize()
    plain_rate = n_plain / (time.perf_counter() - ts)
    # host time to enqueue the loop: close to the wall time when the host,
    # not the GPU, bounds one configuration per step
    plain_host_us = (t_host - ts) / n_plain * 1e6
    # the same loop with b in FP32 (the split-FP16 structure factors), still
    # solved by the FP64 matvec: the reduced-precision single-configuration
    # step; its charges are compared with the FP64 loop's last ones
    b1f = torch.empty((1, w.n), dtype=torch.float32, device=dev)
    q1f = torch.empty_like(q1)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for s_ in range(n_plain):
        ctx.potential_vector(xyz[s_:s_ + 1], b1f)
        ctx.solve_charges(b1f, 0x000, q1f, Qe1)
    torch.cuda.synchronize()
    plain_f32b = {"steps_per_s": n_plain / (time.perf_counter() - ts),
                  "max_rel_diff_vs_fp64_last_step":
                      float(((q1f - q1).abs().max() / q1.abs().max()).item())}
    graph_step = graph_step_measure(w, xyz, dev, n_plain, q1)

    matvec = matvec_roofline(ctx, w, xyz, dev)
    cg = cg_measure(w, xyz, dev, ctx)

    # dominant kernel: the structure factors
    nk = int(ctx.info("nk"))
    sf_avg = sf_ms / max(sf_cnt, 1) * 1e-3
    # algorithmic work of one launch (it covers one launch group of
    # configurations): on matrix cores, 4 flop per (k, charge) pair (one
    # real 2 x 2 product of (Re C, Im C) with (Re Z, Im Z) serves k and its
    # mirror in k_z: 8 flop per 2 k); on the VALU kernel, 8 flop per pair (a
    # complex rotation and a complex accumulate)
    snaps_per_launch = B * steps / max(sf_cnt, 1)
    matrix = ctx.info("sf_matrix") == 1.0
    sf_prec = ctx.info("sf_fp32") if (b_f32 and matrix) else 0.0
    sf_fp32, sf_f16 = sf_prec == 1.0, sf_prec == 2.0
    flop_per_pair = 4.0 if matrix else 8.0
    flop_per_launch = flop_per_pair * nk * w.m * snaps_per_launch
    achieved = flop_per_launch / sf_avg if sf_avg > 0 else 0.0
    # FP64 MFMA and FP64 vector peaks are both 78.6 TFLOP/s; with b stored in
    # FP32 the structure factors run on FP16 matrix cores with split operands
    # (2.5 PFLOP/s dense; three products per algorithmic one) or, switched
    # to, on FP32 matrix cores (157.3 TFLOP/s)
    peak = PEAK_FP16_MFMA if sf_f16 else PEAK_FP32_VALU if sf_fp32 else PEAK_FP64_VALU
    sf_kernel = ("cpm::k_sf_mfma16<2>" if sf_f16 else "cpm::k_sf_mfma32" if sf_fp32
                 else "cpm::k_sf_mfma")
    traffic = stored_traffic(name, sf_kernel, snaps_per_launch)
    sf_bound = "mfma" if matrix else "alu"

    value = B * steps / elapsed
    out = {
        "metric": f"charge solves/sec (N_elec={w.n})",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": name, "n_elec": w.n, "m_elyt": w.m,
                   "snapshots_per_step": B, "n_k": nk, "alpha": w.alpha, "rcut": w.rcut,
                   "eta": w.eta, "mode": args.mode,
                   "step": "assemble A + invert + S + set v + b and q for every snapshot"},
        "roofline": {"kernel": "structure_factor", "bound": sf_bound,
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "flop_per_launch": flop_per_launch, "flop_per_k_charge_pair": flop_per_pair,
                     "avg_launch_us": sf_avg * 1e6,
                     "configurations_per_launch": snaps_per_launch,
                     "launch_group": int(ctx.info("group")),
                     "precision": "fp16 split pairs (3 products)" if sf_f16 else
                                  "fp32" if sf_fp32 else "fp64",
                     "matrix_core_frac_executed": achieved * (3.0 if sf_f16 else 1.0) / peak,
                     # the same algorithmic rate against the FP64 matrix peak
                     # (the ceiling of the FP64 structure factors it replaces)
                     "achieved_over_fp64_peak": achieved / PEAK_FP64_MFMA,
                     "sf_kernel": sf_kernel.split("::")[1]},
        "roofline_real_space": rs_roof,
        "phase_s": {"setup": setup_s, "b_all_snapshots": b_s, "solve_all_snapshots": solve_s},
        "solve_only_rate": B / (b_s + solve_s),
        "plain_fp64_per_step_rate": plain_rate,
        "plain_fp64_host_enqueue_us_per_step": plain_host_us,
        "plain_fp64_sample": f"{n_plain} snapshots, b + FP64 matvec solve one at a time, setup excluded",
        "plain_b_f32_per_step": plain_f32b,
        "graph_fp64_per_step": graph_step,
        "kernel_ms_per_step": {f: v[0] for f, v in timing.items() if v[1]},
        "matvec_roofline": matvec,
        "conjugate_gradient": cg,
        "autotune": tune,
        "max_abs_sum_q": qsum,
    }
    ctx.close()
    return out


def run_mixed(args):
    """Eight capacitors of uneven size (N from U{2000..20000}, snapped to whole
    graphene cells; electrolyte 10 N water charges + 1 M ions), 128
    configurations each: per step every A is assembled and inverted (on the
    context's second stream, beside the b of the instances), b is computed
    per instance (FP32, from the FP32 structure factors), and all instances
    are solved by cpm_solve_grouped (split-BF16, refined) in one persistent
    launch per S~ product."""
    import numpy as np
    import torch
    from paper_2203_15461_amd import cpm
    from paper_2203_15461_amd import inputs as I
    dev = torch.device("cuda:0")
    B = args.batch or 128
    rng = np.random.default_rng(5)
    targets = sorted(int(t) for t in rng.integers(2000, 20001, size=8))
    ws = [I.scaled_graphite_capacitor(t) for t in targets]
    s = torch.cuda.Stream()
    ctxs, data = [], []
    for k, w in enumerate(ws):
        c = cpm.Context(cpm.Params.of(w), stream=s)
        c.set_electrolyte(w.electrolyte_q)
        xyz = synthetic_configurations(w, B, I.BASE_SEED + 1 + k, dev)
        R = torch.as_tensor(w.electrode_xyz, dtype=torch.float64, device=dev).contiguous()
        eid = torch.as_tensor(w.electrode_id, dtype=torch.int32, device=dev).contiguous()
        data.append((xyz, R, eid, torch.empty((B, w.n), dtype=torch.float32, device=dev),
                     torch.empty((B, w.n), dtype=torch.float64, device=dev)))
        ctxs.append(c)
    torch.cuda.synchronize()
    print(f"[bench] mixed8: n = {[w.n for w in ws]}, m = {[w.m for w in ws]}", file=sys.stderr,
          flush=True)

    def step():
        with torch.cuda.stream(s):
            for c, w, (xyz, R, eid, b, q) in zip(ctxs, ws, data):
                c.build_elastance(R, eid, 2)
                c.invert(1 | 4 | cpm.INVERT_ASYNC)
                c.potential_vector(xyz, b)
                c.set_potential(w.v_electrode)
            cpm.solve_grouped(ctxs, [d[3] for d in data], 0x102, [d[4] for d in data])

    for i in range(args.warmup):
        step()
        s.synchronize()
        print(f"[bench] mixed8: warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    s.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step()
    s.synchronize()
    elapsed = time.perf_counter() - t_start
    qsum = max(float(d[4].sum(dim=1).abs().max().item()) for d in data)
    nconf = 8 * B
    # b of all instances and the grouped solve as one captured graph, replayed
    # (A and S kept from the last step: the fixed-electrode case)
    cpm.capture_grouped(ctxs, [d[0] for d in data], [d[3] for d in data], 0x102,
                        [d[4] for d in data])
    cpm.replay_grouped(ctxs)
    s.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        cpm.replay_grouped(ctxs)
    s.synchronize()
    replay_rate = nconf * reps / (time.perf_counter() - t0)
    for c in ctxs:
        c.close()
    return {"metric": "charge solves/sec (8 capacitors, N_elec 2000-20000)",
            "value": nconf * args.steps / elapsed, "unit": "solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "b f32, S bf16x3 (f32 accumulation), f64 refine",
            "graph_replay_rate": replay_rate,
            "graph_replay": "b of all instances + grouped split-BF16 solve replayed from one HIP graph, A and S fixed",
            "data": "synthetic",
            "config": {"workload": "mixed8", "n_elec": [w.n for w in ws],
                       "m_elyt": [w.m for w in ws], "snapshots_per_step_per_instance": B,
                       "step": "per instance: assemble A + invert + S + set v + b; then one "
                               "grouped split-BF16 solve of all instances"},
            "max_abs_sum_q": qsum}


def matvec_roofline(ctx, w, xyz, dev, reps=20):
    """HBM rate of the single-vector solve kernels: S streamed once per solve
    (FP64: 8 N^2 bytes, FP32: 4 N^2 bytes).  `warm`: back-to-back solves
    (below 256 MB, N < ~5800 in FP64, S can stay in the last-level cache);
    `cold`: each solve after a 1 GiB write that evicts it.  A and S must
    already be built; leaves the context with FP64 and FP32 copies of S."""
    import torch
    ctx.invert(1 | 2)
    ctx.set_potential(w.v_electrode)
    b1 = torch.empty((1, w.n), dtype=torch.float64, device=dev)
    ctx.potential_vector(xyz[:1], b1)
    q1 = torch.empty((1, w.n), dtype=torch.float64, device=dev)
    b32 = b1.float()
    flush = torch.empty(1 << 27, dtype=torch.float64, device=dev)       # 1 GiB
    out = {}
    for fam, mode, bb, bytes_per in (("matvec_f64", 0x000, b1, 8), ("matvec_f32", 0x001, b32, 4)):
        alg = bytes_per * float(w.n) ** 2
        rec = {"bound": "hbm", "peak": PEAK_HBM / 1e9, "unit": "GB/s", "bytes_per_launch": alg}
        for kind in ("warm", "cold"):
            ctx.solve_charges(bb, mode, q1)
            ctx.enable_timing(fam)
            for _ in range(reps if kind == "warm" else 5):
                if kind == "cold":
                    flush.fill_(1.0)
                    torch.cuda.synchronize()
                ctx.solve_charges(bb, mode, q1)
            ms, cnt = ctx.timing(fam)
            ctx.enable_timing(False)
            avg = ms / max(cnt, 1) * 1e-3
            rec[kind] = {"achieved": alg / avg / 1e9, "frac": alg / avg / PEAK_HBM,
                         "avg_launch_us": avg * 1e6, "launches": cnt}
        # top-level figures: the cold rate, i.e. S streamed from HBM
        rec.update(achieved=rec["cold"]["achieved"], frac=rec["cold"]["frac"],
                   avg_launch_us=rec["cold"]["avg_launch_us"])
        out[fam] = rec
    del flush
    out["note"] = ("cold: a 1 GiB write before every solve evicts S from the caches; warm: "
                   "back-to-back solves; nontemporal loads from 128 MiB of S on")
    return out


def count_pairs(w, xyz_one):
    """Electrode-electrolyte pairs closer than r_c in one configuration (all
    periodic images in x and y; the slab clearance keeps z images beyond r_c)."""
    import numpy as np
    from scipy.spatial import cKDTree
    R = np.array(w.electrode_xyz, dtype=np.float64)
    r = np.array(xyz_one, dtype=np.float64)
    z0 = min(R[:, 2].min(), r[:, 2].min()) - 1.0
    box = [w.Lx, w.Ly, 1e6]
    def wrap(a):
        a = a.copy()
        a[:, 0] %= w.Lx
        a[:, 1] %= w.Ly
        a[:, 2] -= z0
        return a
    ta, tb = cKDTree(wrap(R), boxsize=box), cKDTree(wrap(r), boxsize=box)
    return int(ta.count_neighbors(tb, w.rcut * (1 - 1e-12)))


def real_space_roofline(w, xyz, R, eid, bvec, group, name, reps=3):
    """FP64 rate of the real-space b kernel on its own: in the timed step it
    shares the chip with the structure factors (a stream of its own), so its
    event time there is not its speed.  A second context with the real-space
    pass on the context stream (CPM_RS_CONCURRENT=0, read when a context is
    created) forms b for `reps` launch groups of the step's size; rate =
    REAL_SPACE_FLOP_PER_PAIR per electrode-electrolyte pair inside r_c (pairs
    counted on the host for the first configuration) times the
    configurations of one launch, over the average launch time (HIP events on
    the context stream)."""
    import torch
    from paper_2203_15461_amd import cpm
    g = min(group, xyz.shape[0])
    old = os.environ.get("CPM_RS_CONCURRENT")
    os.environ["CPM_RS_CONCURRENT"] = "0"
    try:
        ctx = cpm.Context(cpm.Params.of(w))
    finally:
        if old is None:
            del os.environ["CPM_RS_CONCURRENT"]
        else:
            os.environ["CPM_RS_CONCURRENT"] = old
    try:
        ctx.set_electrolyte(w.electrolyte_q)
        ctx.build_elastance(R, eid, 2)
        ctx.potential_vector(xyz[:g], bvec[:g])            # warm-up: buffers, pair tables
        torch.cuda.synchronize()
        ctx.enable_timing(True)
        for _ in range(reps):
            ctx.potential_vector(xyz[:g], bvec[:g])
        torch.cuda.synchronize()
        total_ms, launches = ctx.timing("real_space_b")
        plane = bool(ctx.info("rs_plane"))
    finally:
        ctx.close()
    if not launches:
        return None
    pairs = count_pairs(w, xyz[0].cpu().numpy())
    per_launch_cfg = reps * g / launches
    flop = REAL_SPACE_FLOP_PER_PAIR * pairs * per_launch_cfg
    avg = total_ms / launches * 1e-3
    kernel = "cpm::k_real_space_plane" if plane else "cpm::k_real_space_b"
    return {"kernel": kernel.split("::")[1], "bound": "alu", "achieved": flop / avg / 1e12,
            "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s", "frac": flop / avg / PEAK_FP64_VALU,
            "traffic": stored_traffic(name, kernel, per_launch_cfg),
            "pairs_per_configuration": pairs,
            "flop_per_pair": REAL_SPACE_FLOP_PER_PAIR, "configurations_per_launch": per_launch_cfg,
            "avg_launch_us": avg * 1e6, "us_per_configuration": avg * 1e6 / per_launch_cfg,
            "measured": f"{reps} launch groups of {g} configurations, the real-space pass alone "
                        "on the context stream (in the timed step it overlaps the structure factors)"}


def batched_comparator(w, B=256, reps=5):
    """The batched solve Q = S B of 256 configurations (the 2880-atom
    capacitor, b computed beforehand): split-BF16 matrix-core product with one
    FP64 refinement, against the plain FP64 matrix-core product; solves/s of
    the solve alone, and the q difference between the two."""
    import torch
    from paper_2203_15461_amd import cpm
    from paper_2203_15461_amd import inputs as I
    dev = torch.device("cuda:0")
    ctx = cpm.setup(w, store=cpm.STORE_F64 | cpm.STORE_BF16X2)
    xyz = synthetic_configurations(w, B, I.BASE_SEED + 3, dev)
    b = torch.empty((B, w.n), dtype=torch.float64, device=dev)
    ctx.potential_vector(xyz, b)
    tune = ctx.autotune(B, reps=3)
    out = {"configurations": B, "autotune": tune}
    qs = {}
    for name, mode in (("bf16x3_refined", 0x102), ("f64_mfma", 0x000)):
        q = torch.empty_like(b)
        ctx.solve_charges(b, mode, q)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            ctx.solve_charges(b, mode, q)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / reps
        out[name] = {"solves_per_s": B / dt, "us_per_batch": dt * 1e6}
        qs[name] = q
    out["max_rel_diff_bf16x3_vs_f64"] = float(((qs["bf16x3_refined"] - qs["f64_mfma"]).abs().max()
                                               / qs["f64_mfma"].abs().max()).item())
    ctx.close()
    return out


def graph_step_measure(w, xyz, dev, n, q_last):
    """One configuration per step as a molecular-dynamics loop would run it:
    b and the FP64 matvec solve captured once as a HIP graph
    (cpm_capture_step) on a context with its own stream, then per step the
    coordinates copied into the captured input buffer and the graph
    replayed (S built beforehand).  The last step's configuration is the
    plain loop's last, so its charges are compared with q_last."""
    import torch
    from paper_2203_15461_amd import cpm
    stream = torch.cuda.Stream()
    ctx = cpm.setup(w, stream=stream)
    x1 = xyz[0:1].clone()
    b1 = torch.empty((1, w.n), dtype=torch.float64, device=dev)
    q1 = torch.empty_like(b1)
    Qe1 = torch.empty((1, 2), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    ctx.capture_step(x1, b1, 0x000, q1, Qe1)
    with torch.cuda.stream(stream):
        for s_ in range(2):                              # warm-up replays
            x1.copy_(xyz[s_:s_ + 1])
            ctx.replay_step()
    stream.synchronize()
    ts = time.perf_counter()
    with torch.cuda.stream(stream):
        for s_ in range(n):
            x1.copy_(xyz[s_:s_ + 1])
            ctx.replay_step()
    stream.synchronize()
    dt = (time.perf_counter() - ts) / n
    diff = float(((q1 - q_last).abs().max() / q_last.abs().max()).item())
    ctx.close()
    return {"steps_per_s": 1.0 / dt, "us_per_step": dt * 1e6, "steps": n,
            "max_rel_diff_vs_eager_last_step": diff,
            "note": "per step: coordinates copied into the captured buffer, then one graph replay"}


CG_FAMILIES = ("cg_plane_sums", "cg_plane_mix", "cg_tiles", "cg_apply", "cg_update", "cg_precond",
               "cg_dir", "cg_init", "cg_finish")


def cg_measure(w, xyz, dev, ctx_direct, B=64, tol=1e-13, reps=3):
    """The matrix-free conjugate-gradient solve on the same workload: operator
    set-up, then B = 64 configurations (one CG group) solved to |r| <= tol |r0|
    per call, with the two-level preconditioner (built by the first, untimed
    solve; its set-up time is reported on its own; the second untimed solve
    captures the 8-iteration graph) and, for comparison, the
    iteration count of plain CG.  Reports solves/s, iterations, the
    per-iteration kernel split
    with each family's algorithmic HBM bytes (and FP64 flops for the two
    matrix-core products), and the largest deviation from the direct FP64
    solve q = S (b + v) of ctx_direct on the same b."""
    import numpy as np
    import torch
    from paper_2203_15461_amd import cpm
    n = w.n
    ctx = cpm.Context(cpm.Params.of(w))
    ctx.set_electrolyte(w.electrolyte_q)
    R = torch.as_tensor(w.electrode_xyz, dtype=torch.float64, device=dev).contiguous()
    eid = torch.as_tensor(w.electrode_id, dtype=torch.int32, device=dev).contiguous()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ctx.build_operator(R, eid, 2)
    ctx.set_potential(w.v_electrode)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - ts
    if xyz.shape[0] < B:                             # one full CG group of configurations
        from paper_2203_15461_amd import inputs as I
        xyz = synthetic_configurations(w, B, I.BASE_SEED + 2, dev)
    b = torch.empty((B, n), dtype=torch.float64, device=dev)
    ctx.potential_vector(xyz[:B], b)
    q = torch.empty_like(b)
    Qe = torch.empty((B, 2), dtype=torch.float64, device=dev)
    ctx.enable_timing(True)
    iters, resid = ctx.solve_cg(b, q, Qe, tol=tol)       # builds the preconditioner
    pc_setup_ms = sum(ctx.timing(f)[0] for f in ("pc_blocks", "pc_coarse_matrix", "pc_balancing"))
    ctx.enable_timing(False)
    pc_tiles, pc_mode = int(ctx.info("pc_tiles")), int(ctx.info("pc_mode"))
    pc_coarse = int(ctx.info("pc_coarse"))
    ctx.solve_cg(b, q, Qe, tol=tol)                       # captures the iteration graph
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(reps):
        ctx.solve_cg(b, q, Qe, tol=tol)
    torch.cuda.synchronize()
    call_s = (time.perf_counter() - ts) / reps
    ctx.enable_timing(True)
    ctx.solve_cg(b, q, Qe, tol=tol)
    fam = {f: ctx.timing(f) for f in CG_FAMILIES}
    ctx.enable_timing(False)
    nc, nl, width = int(ctx.info("ncols")), int(ctx.info("nlayers")), int(ctx.info("ell_width"))
    nb = int(ctx.info("bsr_blocks"))
    workspace = ctx.info("workspace")
    ctx.close()
    # plain CG (no preconditioner) on the same b: iterations only
    was = os.environ.get("CPM_CG_PRECOND")
    os.environ["CPM_CG_PRECOND"] = "0"                # read when a context is created
    try:
        ctx0 = cpm.Context(cpm.Params.of(w))
    finally:
        if was is None:
            del os.environ["CPM_CG_PRECOND"]
        else:
            os.environ["CPM_CG_PRECOND"] = was
    ctx0.set_electrolyte(w.electrolyte_q)
    ctx0.build_operator(R, eid, 2)
    ctx0.set_potential(w.v_electrode)
    q0 = torch.empty_like(b)
    plain_iters, _ = ctx0.solve_cg(b, q0, tol=tol)
    ctx0.close()
    qd = torch.empty_like(b)
    ctx_direct.solve_charges(b, 0x000, qd)
    torch.cuda.synchronize()
    dev_rel = float(((q - qd).abs().max() / qd.abs().max()).item())

    m2 = 2 * ((nc + 31) // 32 * 32)                  # rows of the phase matrix
    nslot = int(sum(-(-c // 64) * 64 for c in np.bincount(
        np.searchsorted(np.unique(w.electrode_xyz[:, 2]), w.electrode_xyz[:, 2]))))
    vec = nslot * 64 * 8                             # one slot-major block of 64 vectors
    ld = -(-pc_coarse // 64) * 64                    # coarse row stride
    if pc_mode == 2:
        # balancing form: inverse tile blocks, DAZ (slots x ld) twice, the
        # two ld x ld coarse matrices; r read three times, z written
        pc_work = ((pc_tiles * 4096 + 2 * nslot * ld + 2 * ld * ld) * 8 + 4 * vec,
                   2.0 * pc_tiles * 64 ** 3 + 2 * 2.0 * nslot * ld * 64 + 3 * 2.0 * ld * ld * 64)
    else:
        # additive form: inverse tile blocks and the coarse inverse, r read
        # twice, z written, read and written again
        pc_work = ((pc_tiles * 4096 + pc_tiles * pc_tiles) * 8 + 5 * vec,
                   2.0 * pc_tiles * 64 ** 3 + 2.0 * pc_tiles ** 2 * 64)
    work = {   # (algorithmic HBM bytes, FP64 flops) per launch
        "cg_plane_sums": (m2 * nslot * 8 + vec + nl * m2 * 64 * 8, 2.0 * m2 * nslot * 64),
        # projection (phase matrix, T, output) + block-sparse real space
        # (64 x 64 FP64 blocks, the vector block): flops 2 K per output
        "cg_tiles": (m2 * nslot * 8 + nl * m2 * 64 * 8 + vec + nb * 4096 * 8 + vec,
                     2.0 * m2 * nslot * 64 + 2.0 * nb * 64 * 64 * 64),
        "cg_apply": (3 * vec, 0.0),
        "cg_update": (6 * vec, 0.0),
        "cg_dir": (3 * vec, 0.0),
        "cg_precond": pc_work,
    }
    per_iter = {}
    for f, (ms, cnt) in fam.items():
        if not cnt:
            continue
        us = ms / cnt * 1e3
        e = {"us": us, "launches": cnt}
        if f in work:
            by, fl = work[f]
            e["bytes"] = by
            e["hbm_frac"] = by / (us * 1e-6) / PEAK_HBM
            if fl:
                e["tflops"] = fl / (us * 1e-6) / 1e12
                e["fp64_frac"] = fl / (us * 1e-6) / PEAK_FP64_VALU
        per_iter[f] = e
    dom = max(per_iter, key=lambda f: per_iter[f]["us"] * per_iter[f]["launches"])
    out = {"solves_per_s": B / call_s, "ms_per_call": call_s * 1e3, "vectors_per_call": B,
           "tol": tol, "iterations": iters, "residual": resid, "operator_setup_s": setup_s,
           "preconditioner": {"form": {0: "none", 1: "additive", 2: "balancing"}[pc_mode],
                              "tiles": pc_tiles, "coarse_columns": pc_coarse,
                              "setup_s": pc_setup_ms * 1e-3,
                              "plain_cg_iterations": plain_iters},
           "ell_width": width, "bsr_blocks": nb, "columns": nc, "planes": nl, "slots": nslot,
           "max_rel_diff_vs_direct_fp64": dev_rel,
           "max_abs_sum_q": float(q.sum(dim=1).abs().max().item()),
           "per_launch": per_iter, "dominant": dom,
           "workspace_bytes": workspace,
           "note": "b computed once outside the timed calls; each call starts from q = 0"}
    return out


def stored_traffic(workload, kernel, configs_per_launch):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (each counter scaled by what it reads for
    a 1 GiB device copy), per configuration times the timed run's average
    configurations per launch (a step's last launch group can be partial);
    None when the kernel source changed since the counters were taken, when
    no record covers this kernel and workload, or when the average launch
    holds fewer than 3/4 (or more) of the profiled configurations."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "structure_factor_traffic.json")
    src = os.path.join(ROOT, "paper_2203_15461_amd", "csrc", "bvector.hip")
    try:
        rec = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    entry = rec.get("kernels", {}).get(kernel, {}).get(workload)
    if not entry or rec.get("bvector_sha256") != digest:
        return None
    per = entry.get("configurations_per_launch", 1)
    if configs_per_launch > per * 1.001 or configs_per_launch < 0.75 * per:
        return None
    # per configuration, times the timed run's average configurations per launch
    return entry["bytes_per_launch"] / per * configs_per_launch


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, snapshots=5):
    """The FP64 oracle on the host cores: b and q for `snapshots` snapshots of
    the same workload, median time per solve (A and S are built first and not
    timed: over a 1000-snapshot step they add < 0.1% per solve).  `cores` is
    the process CPU time over the wall time of the timed solves (numpy's
    elementwise work runs on one thread, its matrix products on the BLAS
    threads)."""
    import numpy as np
    from oracle import cpm_oracle as O
    from paper_2203_15461_amd import inputs as I
    p = O.params_for(w)
    S = O.capacitance(O.elastance(w.electrode_xyz, p)).S
    v = O.applied_potential(w.electrode_id, w.v_electrode)
    times, cpu, q0 = [], 0.0, None
    for s_ in range(snapshots):
        r = I.snapshot(w, s_)
        t, c = time.perf_counter(), time.process_time()
        b = O.potential_vector(w.electrode_xyz, r, w.electrolyte_q, p)
        q = O.charges(S, b, v)
        times.append(time.perf_counter() - t)
        cpu += time.process_time() - c
        assert abs(q.sum()) < 1e-10
        if s_ == 0:
            q0 = q
    med = float(np.median(times))
    try:
        from threadpoolctl import threadpool_info
        blas = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:
        blas = None
    Q = O.electrode_totals(q0, w.electrode_id, 2)
    return {"value": 1.0 / med, "unit": "solves/s", "cores": round(cpu / sum(times), 1),
            "kind": "oracle", "cpu_model": cpu_model(), "host_threads": os.cpu_count(),
            "blas_threads": blas, "median_s": med, "min_s": min(times), "max_s": max(times),
            "sample": f"{snapshots} snapshots of {w.name} (seeds 15461+1..{snapshots}): b "
                      "(Ewald real + k + slab) and q = S(b+v) in FP64 numpy, median time per "
                      "solve; A and S built beforehand, untimed"}, q0, Q


def accuracy_vs_oracle(w, q_ref, Q_ref):
    """Error of each solve path in q and in the electrode totals against the
    oracle's FP64 result for snapshot 0: the plain FP64 path (one vector,
    streaming matvec), and the batched FP32 and split-BF16 paths (a batch of 8
    snapshots, snapshot 0 first; b in FP32 from the FP32 structure factors,
    and for split-BF16 also b in FP64), each with one FP64 refinement step."""
    import numpy as np
    import torch
    from paper_2203_15461_amd import cpm
    from paper_2203_15461_amd import inputs as I
    dev = torch.device("cuda:0")
    ctx = cpm.setup(w, store=cpm.STORE_F64 | cpm.STORE_F32 | cpm.STORE_BF16X2)
    xyz = torch.as_tensor(np.stack([I.snapshot(w, s) for s in range(8)]), dtype=torch.float64,
                          device=dev).contiguous()
    b64 = torch.empty((8, w.n), dtype=torch.float64, device=dev)
    b32 = torch.empty((8, w.n), dtype=torch.float32, device=dev)
    ctx.potential_vector(xyz, b64)
    ctx.potential_vector(xyz, b32)
    out = {}
    for name, bb, mode, rows in (("f64_plain", b64, 0x000, 1), ("f32r_batched", b32, 0x101, 8),
                                 ("bf16r_batched", b32, 0x102, 8),
                                 ("bf16r_batched_b_f64", b64, 0x102, 8)):
        q = torch.empty((rows, w.n), dtype=torch.float64, device=dev)
        Qe = torch.empty((rows, 2), dtype=torch.float64, device=dev)
        ctx.solve_charges(bb[:rows], mode, q, Qe)
        ctx.synchronize()
        q0, Q0 = q[0].cpu().numpy(), Qe[0].cpu().numpy()
        out[name] = {"q_rel": float(np.abs(q0 - q_ref).max() / np.abs(q_ref).max()),
                     "Q_rel": float(np.abs(Q0 - Q_ref).max() / np.abs(Q_ref).max()),
                     "abs_sum_q": float(abs(q0.sum()))}
    ctx.close()
    return out


if __name__ == "__main__":
    main()
