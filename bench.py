"""Benchmark of the aSP-AMG solve phase on one MI355X.

Workload (default): the distorted layered block 128x128x64 Q1 hexes (3,244,995
DOF), interior nodes jittered by U[-0.3h, 0.3h], E = 1 and 1e4 in layers of 8
elements alternating in z, nu = 0.3, clamped at z = 0, body force, seed 3; the
paper's default test space (ten vectors: the six rigid-body modes and four
seeded random ones, ten SRQCG iterations per level).  A step is one PCG solve
to ||r|| <= 1e-10 ||f|| (at most 1000 iterations) with the FP32 V-cycle inside
FP64 PCG; the same number of solves with the FP64 V-cycle is timed beside it.
Inputs are resident in HBM before the timed region.

Prints one JSON line (rank 0): metric, value (FP32-cycle solve seconds), the
FP64-cycle solve time, V-cycle HBM GB/s for both precisions, the roofline of
the dominant kernel (PCG product q = K p, 3x3-block sliced-ELL SpMV) and the CPU
oracle measured on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG-AMG solve s and V-cycle HBM GB/s at 1e-10 rel-res, FP32 vs FP64 cycle"
HBM_PEAK_GBS = 8000.0


def kernel_source_hash():
    import hashlib
    path = os.path.join(ROOT, "paper_1902_01715_amd", "csrc", "kernels_solve.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def measured_traffic(workload):
    """HBM bytes per launch of q = K p from the committed counter runs
    (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel calibration), or
    None when the kernel source changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"k_sell_spmv_dot_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernels_solve_sha256") != kernel_source_hash():
        return None
    return rec["bytes_per_launch"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_problem(name):
    from paper_1902_01715_amd import problems as PR
    if name == "c2":
        return PR.c2_cantilever(), "cantilever 320x32x32 Q1 (1,048,707 DOF), aspect 10, E=10^U[-3,3], nu=U[.25,.45]"
    if name == "c3":
        return PR.c3_layered_distorted(), "layered distorted block 128x128x64 Q1 (3,244,995 DOF), E=1/1e4 layers"
    if name == "c4":
        return PR.c4_multiload(), "cube 96^3 Q1 (2,738,019 DOF), 32 load cases"
    if name == "c5":
        return PR.c5_simp(), "SIMP cube 48^3 Q1 (352,947 DOF), E=rho^3, compliance gradient"
    if name == "c1":
        return PR.c1_cube(), "unit cube 10^3 Q1 (3,993 DOF)"
    if name == "t1":
        return PR.t1_tet_elasticity(), "point-wise elasticity on 64^3 x 6 P1 tetrahedra (823,875 unknowns), scalar CSR"
    raise SystemExit(f"unknown config {name}")


def cpu_baseline(problem_name, gpu_iters, n_rq=0):
    """The CPU oracle, seconds per solve of the workload at the GPU's iteration
    count.  The full-size oracle was measured once per workload by
    oracle/fullsize_run.py (its hierarchy of the whole mesh; PCG iterations on
    one thread and on all cores of the recording host; profiles/).  Here the
    same bounded sample (oracle/baseline_sample.py: a small instance of the
    workload's recipe, about 15-30 s of CPU work) is timed on this host; the
    ratio of the two sample times carries the full-size figure over to this
    host."""
    import oracle
    from oracle.baseline_sample import time_sample
    oracle.build(force=False)
    tag = problem_name if n_rq == 0 else f"{problem_name}_srqcg"
    path = os.path.join(ROOT, "profiles", f"oracle_{tag}_fullsize.json")
    if not os.path.exists(path) or problem_name not in ("c2", "c3", "t1"):
        return None
    rec = json.load(open(path))
    if "sample" not in rec:
        return None
    live = time_sample(problem_name, n_rq)
    out = {}
    for key, rec_threads in (("one", "1"), ("all", str(rec["host"]["nproc"]))):
        live_threads = "1" if key == "one" else max(live["pcg"], key=int)
        ratio = live["pcg"][live_threads] / rec["sample"]["pcg"][rec_threads]
        full = rec["pcg"][rec_threads]["s_per_iter"]
        out[key] = {"value": full * ratio * gpu_iters, "s_per_iter": full * ratio, "threads": int(live_threads),
                    "host_ratio": ratio, "recorded_s_per_iter": full, "recorded_threads": int(rec_threads)}
    one, allc = out["one"], out["all"]
    return {"value": one["value"], "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"oracle PCG iteration on the full {problem_name} hierarchy, measured once "
                      f"({rec['pcg']['1']['iterations']} iterations) on {rec['host']['cpu']} ({rec['host']['nproc']} "
                      f"cores, git {rec['git']}) at {one['recorded_s_per_iter']:.3f} s/it on one thread; carried to "
                      f"this host by the {live['desc']} sample ({live['iterations']} iterations, "
                      f"{live['pcg']['1']:.4f} s/it here, host ratio {one['host_ratio']:.3f}); times the GPU's "
                      f"{gpu_iters} iterations",
            "all_cores": {"value": allc["value"], "unit": "s", "cores": allc["threads"],
                          "s_per_iter": allc["s_per_iter"], "host_ratio": allc["host_ratio"],
                          "recorded_s_per_iter": allc["recorded_s_per_iter"],
                          "recorded_threads": allc["recorded_threads"]},
            "recorded_setup_s": rec["setup_s"], "sample_setup_s_here": live["setup_s"]}


def test_space_label(args):
    if args.n_rq == 0:
        return "rigid-body modes (n_tv = 6)"
    return f"SRQCG, n_tv = 10 (rigid-body modes + 4 seeded random), n_rq = {args.n_rq}"


def scalar_config(name):
    """Block size and the parameters that differ for a scalar workload: one
    unknown per node, and 4 unknowns added to an FSAI row per step (the
    paper's rho_g = 4 scalar entries)."""
    return {"block_size": 1, "rho_blocks": 4} if name == "t1" else {}


def bench_batch(args, p, desc, S, t_setup):
    """32 load cases solved together (block SpMM V-cycle, tuned tile), FP32 and
    FP64 cycles, graph replay vs eager launches."""
    import numpy as np
    import torch
    F = torch.tensor(p.f, device="cuda")
    out = {}
    for prec in (32, 64):
        S.set_precision(prec)
        for _ in range(args.warmup):
            S.solve_batch(F)
        ts = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            U = S.solve_batch(F)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        st = S.last_stats
        its = [s["iterations"] for s in st]
        out[prec] = {"solve_s": float(np.median(ts)), "iterations_max": int(max(its)), "iterations_min": int(min(its)),
                     "status": [s["status"] for s in st], "relres_true_max": max(s["relres_true"] for s in st),
                     "spmm_tile": st[0]["spmm_tile"], "s_per_rhs": float(np.median(ts)) / F.shape[1]}
        log(f"batch fp{prec}: {out[prec]['solve_s']:.4f} s for {F.shape[1]} RHS, its {min(its)}..{max(its)}, "
            f"tile {st[0]['spmm_tile']}")
    # eager launches (no graph) for comparison, FP32 cycle
    S.params.use_graph = 0
    from paper_1902_01715_amd import aspamg
    prm = aspamg.default_params(max_it=args.max_it, use_graph=0)
    Se = aspamg.Solver(p.row_ptr, p.col, p.vals, p.V0, prm)
    Se.set_precision(32)
    Se.solve_batch(F)
    torch.cuda.synchronize()
    t = time.perf_counter()
    Se.solve_batch(F)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t
    Se.close()
    # single-RHS reference: FP32 solve of column 0
    S.set_precision(32)
    f0 = F[:, 0].contiguous()
    S.solve(f0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    S.solve(f0)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t
    t32, t64 = out[32]["solve_s"], out[64]["solve_s"]
    return {
        "metric": METRIC, "value": t32, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t32 * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 V-cycle in f64 PCG", "data": "synthetic",
        "config": {"workload": desc, "config": args.config, "rhs": int(F.shape[1]), "setup_s": t_setup,
                   "test_space": test_space_label(args)},
        "fp32_cycle": out[32], "fp64_cycle": out[64], "speedup_fp64_over_fp32": t64 / t32,
        "graph_vs_eager_fp32": {"graph_s": t32, "eager_s": t_eager},
        "single_rhs_fp32_s": t_single, "batch_speedup_per_rhs": t_single / out[32]["s_per_rhs"],
        "levels": [{k: li[k] for k in ("n", "n_coarse", "nnzb_A", "nnzb_G", "nnzb_P")}
                   for li in (S.level_info(l) for l in range(S.nlev))],
    }


def bench_adjoint(args, p, desc):
    """Compliance C = f.u with E = rho^3 and its gradient: forward (GPU
    assembly, setup, solve) and backward (adjoint solve, element gradient)."""
    import numpy as np
    import torch
    from paper_1902_01715_amd import aspamg
    from paper_1902_01715_amd.autograd import ElasticModel, elastic_solve
    model = ElasticModel.from_problem(p, aspamg.default_params(max_it=args.max_it))
    f = torch.tensor(p.f, device="cuda")
    res = []
    for it in range(args.warmup + args.steps):
        rho = torch.tensor(p.extra["rho"], device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = elastic_solve(rho ** 3, f, model)
        C = torch.dot(f, u)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        C.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if it >= args.warmup:
            res.append((t1 - t0, t2 - t1))
    g = rho.grad
    euler = float(((rho.detach() * g).sum() + 3 * C.detach()).abs() / C.detach())
    fw = float(np.median([r[0] for r in res]))
    bw = float(np.median([r[1] for r in res]))
    return {
        "metric": METRIC, "value": fw + bw, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": (fw + bw) * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "config": args.config},
        "forward_s": fw, "backward_s": bw, "euler_identity_rel_err": euler, "compliance": float(C.detach()),
    }


OP_NAMES = {0: "residual A", 1: "G", 2: "G^T", 3: "restriction R", 4: "merged G^T G", 5: "stacked [P; AP]",
            6: "dense", 7: "prolongation P"}


LEVEL_TABLE_REPS = 50


def level_table(S, levels, reps):
    """Every product of the V-cycle per level and precision: average launch
    time (HIP events, 50 launches), algorithmic bytes and GB/s, and how many
    times one cycle launches it (V(1,1): A once, G and G^T twice, R and the
    stacked product once, or P once and A twice on a level without the stacked
    product; merged G^T G twice where the FP32 cycle uses it)."""
    rows = []
    tail = S.last_stats["tail_level"]
    for l, li in enumerate(levels):
        dense = li["n_coarse"] == 0 or l == tail
        for prec in (32, 64):
            if dense:
                ops = [6]
            else:
                ops = [0, 4] if prec == 32 and li["nnzb_M"] > 0 else [0, 1, 2]
                ops += [3, 5] if li["sell_stacked"] != 0 else [3, 7]
            for op in ops:
                ms, by = S.time_operator(l, op, prec, reps)
                per_cycle = {0: 1 if li["sell_stacked"] != 0 else 2, 1: 2, 2: 2, 3: 1, 4: 2, 5: 1, 6: 1, 7: 1}[op]
                rows.append({"level": l, "prec": prec, "op": OP_NAMES[op], "per_cycle": per_cycle, "ms": ms,
                             "bytes": by, "GBps": by / (ms * 1e-3) / 1e9})
        if dense:
            break
    return rows


def stream_reference():
    """Streaming rates of PyTorch's own kernels on 2 GiB FP64 arrays (read-only
    sum, write-only fill, two-read-one-write add, copy): the practical HBM
    ceiling against which the solve kernels' GB/s are read."""
    import torch
    n = 1 << 28
    a = torch.empty(n, dtype=torch.float64, device="cuda").normal_()
    b = torch.empty_like(a)

    def rate(f, nbytes, reps=20):
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9

    out = {"stream_reference_GBps": {
        "sum": rate(lambda: a.sum(), 8 * n),
        "fill": rate(lambda: b.fill_(1.0), 8 * n),
        "add_2r1w": rate(lambda: torch.add(a, b, out=b), 24 * n),
        "copy": rate(lambda: b.copy_(a), 16 * n)}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-it", type=int, default=1000)
    ap.add_argument("--coarse-max-dof", type=int, default=1500,
                    help="factor the coarsest level densely once it has at most this many DOF")
    ap.add_argument("--n-rq", type=int, default=10,
                    help="SRQCG iterations on each level's test space, n_tv = 10 (the rigid-body modes and four "
                         "seeded random columns): the paper's defaults; 0 keeps the six rigid-body modes alone "
                         "(c2, c3, c4)")
    ap.add_argument("--layout", type=int, default=0,
                    help="operator layout policy (0 timed choice, 1 by stored slots, 2 sliced only, 3 row-packed in "
                         "workgroup units only, 4 row-packed in wavefront units only)")
    ap.add_argument("--level-table", action="store_true",
                    help="also time every V-cycle product per level and precision (aspamg_time_operator) and add "
                         "the table to the JSON line")
    ap.add_argument("--stream-ref", action="store_true",
                    help="only measure PyTorch's streaming rates on this device and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)
    if args.stream_ref:
        stream_reference()
        return

    import numpy as np
    import torch
    from paper_1902_01715_amd import aspamg

    from paper_1902_01715_amd import problems as PR

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    aspamg.lib()
    t0 = time.perf_counter()
    p, desc = make_problem(args.config)
    log(f"inputs {desc}: {time.perf_counter() - t0:.1f} s")
    if args.config == "c5":
        print(json.dumps(bench_adjoint(args, p, desc)), flush=True)
        return
    prm = aspamg.default_params(max_it=args.max_it, coarse_max_dof=args.coarse_max_dof, n_rq=args.n_rq,
                                layout=args.layout, **scalar_config(args.config))
    V0 = p.V0 if args.n_rq == 0 else PR.initial_test_space(p, 10, 11)
    t0 = time.perf_counter()
    S = aspamg.Solver(p.row_ptr, p.col, p.vals, V0, prm)
    t_setup = time.perf_counter() - t0
    levels = [S.level_info(l) for l in range(S.nlev)]
    log(f"setup {t_setup:.1f} s, {len(levels)} levels: " + ", ".join(str(li["n"]) for li in levels))
    if args.config == "c4":
        out = bench_batch(args, p, desc, S, t_setup)
        S.close()
        print(json.dumps(out), flush=True)
        return
    f = torch.tensor(p.f if p.f.ndim == 1 else p.f[:, 0], device="cuda")
    u = torch.empty_like(f)

    def run(prec, n):
        S.set_precision(prec)
        ts, st = [], None
        for _ in range(n):
            torch.cuda.synchronize()
            t = time.perf_counter()
            S.solve(f, u)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
            st = S.last_stats
        return ts, st

    for prec in (32, 64):
        run(prec, args.warmup)
    log("warmup done")
    ts32, st32 = run(32, args.steps)
    log(f"fp32 cycle: {st32['iterations']} it, relres {st32['relres_recursive']:.2e} (true {st32['relres_true']:.2e}),"
        f" {np.median(ts32):.4f} s")
    u32 = u.clone()
    ts64, st64 = run(64, args.steps)
    log(f"fp64 cycle: {st64['iterations']} it, relres {st64['relres_recursive']:.2e} (true {st64['relres_true']:.2e}),"
        f" {np.median(ts64):.4f} s")
    err32 = float(torch.linalg.norm(u32 - u) / torch.linalg.norm(u))

    # V-cycle bandwidth (M2) and the roofline of the dominant kernel
    vc32_ms, vc32_b = S.time_kernel(3, 50)
    vc64_ms, vc64_b = S.time_kernel(4, 50)
    kp_ms, kp_b = S.time_kernel(0, 50)
    r32_ms, r32_b = S.time_kernel(1, 50)
    r64_ms, r64_b = S.time_kernel(2, 50)
    kp_gbs = kp_b / (kp_ms * 1e-3) / 1e9
    t32 = float(np.median(ts32))
    t64 = float(np.median(ts64))
    out = {
        "metric": METRIC,
        "value": t32,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycle in f64 PCG",
        "data": "synthetic",
        "config": {"workload": desc, "config": args.config, "test_space": test_space_label(args),
                   "rtol": 1e-10, "max_it": args.max_it,
                   "cycle": "V(1,1)", "levels": len(levels), "c_gd": st32["c_gd"], "c_op": st32["c_op"],
                   "c_fs": st32["c_fs"], "setup_s": t_setup},
        "fp32_cycle": {"solve_s": t32, "iterations": st32["iterations"], "status": st32["status"],
                       "relres": st32["relres_recursive"], "relres_true": st32["relres_true"],
                       "relres_floor": st32["relres_floor"],
                       "s_per_iter": t32 / max(st32["iterations"], 1), "err_vs_fp64_cycle": err32},
        "fp64_cycle": {"solve_s": t64, "iterations": st64["iterations"], "status": st64["status"],
                       "relres": st64["relres_recursive"], "relres_true": st64["relres_true"],
                       "relres_floor": st64["relres_floor"],
                       "s_per_iter": t64 / max(st64["iterations"], 1)},
        "speedup_fp64_over_fp32": t64 / t32,
        "vcycle": {"fp32_ms": vc32_ms, "fp32_GBps": vc32_b / (vc32_ms * 1e-3) / 1e9,
                   "fp64_ms": vc64_ms, "fp64_GBps": vc64_b / (vc64_ms * 1e-3) / 1e9,
                   "fp32_bytes": vc32_b, "fp64_bytes": vc64_b},
        "kernels": {"residual_fp32_GBps": r32_b / (r32_ms * 1e-3) / 1e9,
                    "residual_fp64_GBps": r64_b / (r64_ms * 1e-3) / 1e9},
        "levels": [{k: li[k] for k in ("n", "n_coarse", "nnzb_A", "nnzb_G", "nnzb_P", "sell_slots_A", "sell_slots_G",
                                      "sell_slots_GT", "sell_lanes64", "sell_lanes32", "sell_stacked", "sell_index16",
                                      "sell_unit64", "sell_unit32", "sell_stacked32", "sell_stacked_unit64",
                                      "sell_stacked_unit32", "omega_s", "fsai_rounds")}
                   for li in levels],
        "roofline": {"bound": "hbm", "kernel": "k_sell_spmv_dot (q = K p, FP64, sliced ELL with one lane per row)",
                     "achieved": kp_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kp_gbs / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.config), "avg_launch_ms": kp_ms,
                     "alg_bytes_per_launch": kp_b},
    }
    if args.level_table:
        out["level_table"] = level_table(S, levels, LEVEL_TABLE_REPS)
        out["level_table_reps"] = LEVEL_TABLE_REPS
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args.config, st32["iterations"], args.n_rq)
    S.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
