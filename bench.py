#!/usr/bin/env python3
"""Per-time-step cost of the partial-reuse AMG step on one MI355X.

Workload: the two-fluid pressure Poisson series on a 128^3 grid (2,097,152 unknowns,
14,581,760 nonzeros, FP64), density ratio 1000, interface advancing one cell per step,
pattern fixed.  One *step* is the whole hot path for one time step: ingest the new
values, partial rebuild (Algorithm 4: numeric Galerkin products on the cached patterns,
smoothers, coarse inverse) and the V-cycle-preconditioned CG solve to a true relative
residual of 1e-8.  All inputs (values and right-hand sides of every step) are resident
in HBM before the timed region.

Also measured on the same steps: full rebuild every step (Algorithm 1), full reuse
(Algorithm 3, with a rebuild-and-retry when a solve does not converge in maxiter), the
mixed-precision form (FP32 hierarchy under FP64 CG), per-kernel HIP-event timings, and
the CPU oracle on a bounded sample of the same series.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "per-step setup+solve ms, partial vs full rebuild at 1e-8 rel res; RAP/SpMV GB/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed time steps")
    ap.add_argument("--warmup", type=int, default=3, help="untimed time steps before the timed ones")
    ap.add_argument("--config", type=int, default=2, choices=[2, 3, 5, 6, 7],
                    help="matrix series: 2 = two-fluid 7-point 128^3 FP64 (the headline), 3 = two-fluid "
                         "7-point 192^3, 5 = lognormal 27-point 160^3 with the FP32 hierarchy, 6 = non-symmetric "
                         "convection-diffusion 7-point 128^3 solved by BiCGStab, 7 = coupled system with 4x4 "
                         "blocks on 56^3 nodes (node aggregation, block Jacobi)")
    ap.add_argument("--n", type=int, default=0, help="grid size N (N^3 nodes); 0: the series' own")
    ap.add_argument("--no-compare", action="store_true", help="skip the full-rebuild/full-reuse/mixed runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=12, help="oracle partial steps in the CPU sample")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized FP64 buffer 3 times and exit: the known-size reference "
                         "that scales the FETCH_SIZE / WRITE_SIZE counters of the other kernels")
    return ap.parse_args()


def workload_name(cfg_id, N, n, nnz):
    series = {2: "two-fluid 7-point Poisson, rho ratio 1000, interface +1 cell/step",
              3: "two-fluid 7-point Poisson, rho ratio 1000, interface +1 cell/step",
              5: "27-point lognormal-coefficient Poisson (sigma 1.5) with smooth drift per step",
              6: "non-symmetric upwind convection-diffusion 7-point, flow turning 9 degrees per step",
              7: "coupled system, 4 unknowns per node in full 4x4 blocks on the 7-point node graph (two-fluid "
                 "face weights, SPD couplings turning 9 degrees per step, interface +1 cell/step)"}[cfg_id]
    form = ("FP32 hierarchy and V-cycle under FP64 CG" if cfg_id == 5 else "FP64")
    krylov = "BiCGStab" if cfg_id == 6 else "PCG"
    amg = ("plain aggregation of nodes on block norms, damped block Jacobi; " if cfg_id == 7 else "")
    return (f"{series}, {N}^3 {'nodes' if cfg_id == 7 else 'cells'} (n={n}, nnz={nnz}); {amg}partial reuse "
            f"(numeric-only cached RAP + smoother), {form}, {krylov} to 1e-8 true rel res")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_bandwidth(mib=1024, reps=5):
    """Measured device-copy bandwidth (read + write bytes over the copy's time, best of reps),
    the practical ceiling the HBM-bound kernels are compared with besides the 8 TB/s peak."""
    import torch

    x = torch.rand(mib * 131072, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        y.copy_(x)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del x, y
    torch.cuda.empty_cache()
    return 2 * mib * 2**20 / (best * 1e-3) / 1e9


def operator_timing(amg, n, reps=7, scrub_mib=512):
    """Median time (us) of the level-0 Krylov SpMV (its first-iteration form, through the
    library's operator entry point) back to back, and after a read of scrub_mib MiB that
    evicts the operator from the caches (L2 and the 256 MB MALL) without leaving dirty
    lines to write back."""
    import torch

    x = torch.rand(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    scrub = torch.ones(scrub_mib * 131072, dtype=torch.float64, device="cuda")
    amg.apply_operator(x, y)

    def once(cold, k):
        if cold:
            scrub.sum()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        amg.apply_operator(x, y)
        b.record()
        b.synchronize()
        return a.elapsed_time(b) * 1e3

    hot = sorted(once(False, k) for k in range(reps))
    cold = sorted(once(True, k) for k in range(reps))
    del scrub
    torch.cuda.empty_cache()
    return hot[reps // 2], cold[reps // 2]


def copy_probe(mib):
    """A plain device copy of known size (read mib MiB, write mib MiB), three launches."""
    import torch

    x = torch.rand(mib * 131072, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    log(f"copy probe: {mib} MiB read + {mib} MiB written per launch, 3 launches")


# ------------------------------------------------------------------ algorithmic bytes

def kernel_bytes(dims, sv_h, ndiag=0, sym=False, block=1):
    """Algorithmic bytes per launch of the level-0 kernels: each operand read once, each
    output written once, vector gathers counted once.  CSR: 4-byte indices; an operator
    in diagonal storage (ndiag > 0) needs no index arrays, so its bytes are its values,
    and with symmetric values (sym) only the main diagonal and the entries above it; an
    operator of full block x block blocks needs one index per block and one pointer per
    node.  sv_h is the value size of the hierarchy (8 FP64, 4 FP32); the CG kernels are
    FP64."""
    n, nnzA, nc, nnzP, nnzAP = dims[0]
    nnzAc = dims[1][1]
    ind = lambda rows, nnz: 4 * (rows + 1) + 4 * nnz  # noqa: E731
    if ndiag > 0:
        ind0 = lambda rows, nnz: 0  # noqa: E731
    elif block > 1:
        ind0 = lambda rows, nnz: 4 * (rows // block + 1) + 4 * (nnz // (block * block))  # noqa: E731
    else:
        ind0 = ind
    a0 = (nnzA + n) // 2 if (ndiag > 0 and sym) else nnzA  # level-0 matrix entries read
    b = {}
    # Krylov operator SpMV fused with p = z + beta p and p.q: A, z, p_old read; p_new, q written
    b["cg_pq"] = ind0(n, nnzA) + 8 * a0 + 8 * 4 * n
    b["krylov_spmv"] = ind0(n, nnzA) + 8 * a0 + 8 * 2 * n   # y = A x: A, x read, y written
    b["cg_update"] = 8 * 6 * n          # p, q, x, r read; x, r written
    b["cg_rz"] = 8 * 2 * n
    b["cg_init"] = ind(n, nnzA) + 8 * nnzA + 8 * 3 * n
    b["smooth0_res"] = ind0(n, nnzA) + sv_h * a0 + sv_h * 4 * n   # m, f read; u, r written
    b["jacobi"] = ind0(n, nnzA) + sv_h * a0 + sv_h * 4 * n        # m, f, u read; u' written
    b["restrict"] = ind(nc, nnzP) + sv_h * nnzP + sv_h * (n + nc)
    b["prolong"] = ind(n, nnzP) + sv_h * nnzP + sv_h * (nc + 2 * n)
    b["smoother"] = ind(n, nnzA) + sv_h * nnzA + sv_h * n
    # Galerkin product of level 0, per rebuild: A, P, R read once, A_1 written once with its
    # cached columns read once; the A P intermediate is an implementation cost, not counted
    rap = ind(n, nnzA) + sv_h * nnzA + 2 * (ind(n, nnzP) + sv_h * nnzP) + ind(nc, nnzAc) + sv_h * nnzAc
    b["galerkin"] = rap
    b["cast"] = 12 * n
    return b


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: runs on several GPUs "
              f"(row-block sharding of every level) are not implemented.", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return

    import numpy as np
    import torch

    from paper_2108_02054_amd import AMG, FULL, OPERATOR_ONLY
    from paper_2108_02054_amd.amg import PARTIAL, policy
    POLICY = policy(PARTIAL, every=10)  # an occasional full setup between partial updates (Section 3)
    # full reuse as the paper runs it: a solve that misses the iteration limit is not
    # repeated; the next update is a full setup (Algorithm 3, Section 3)
    POLICY_REUSE = policy(OPERATOR_ONLY)
    from workloads import CONFIGS, rhs_uniform, series_matrix

    dev = torch.device("cuda:0")
    cfg_id = args.config
    cfg = CONFIGS[cfg_id]
    N = args.n or cfg["N"]
    K, W = args.steps, args.warmup
    nsteps = W + K + 1
    # the series' own precision for the headline line: FP64, or the FP32 hierarchy under
    # FP64 CG for the 27-point series
    head_prec = 1 if cfg_id == 5 else 0
    bicg = cfg_id == 6  # the non-symmetric series: BiCGStab, the paper's Krylov method

    def solve(amg, f, x):
        return amg.solve_bicgstab(f, x) if bicg else amg.solve(f, x)
    amg_params = dict(eps_strong=cfg["eps_strong"])
    for key in ("block_size", "aggregation"):
        if key in cfg:
            amg_params[key] = cfg[key]

    # ---------------------------------------------------------------- inputs in HBM
    t0 = time.time()
    vals, rhs = [], []
    for t in range(nsteps):
        p, c, v = series_matrix(cfg_id, t, N)
        if t == 0:
            n = len(p) - 1
            ptr = torch.from_numpy(p).to(dev)
            col = torch.from_numpy(c).to(dev)
        vals.append(torch.from_numpy(v).to(dev))
        rhs.append(torch.from_numpy(rhs_uniform(n, cfg_id, t)).to(dev))
        del p, c, v
    torch.cuda.synchronize()
    nnz = int(col.numel())
    log(f"inputs: {nsteps} steps of {cfg['name']} at {N}^3 (n={n}, nnz={nnz}) generated and uploaded in "
        f"{time.time() - t0:.1f}s")

    u = torch.zeros(n, dtype=torch.float64, device=dev)

    def series(mode, precision=0, trace=None):
        """Setup at t=0 (untimed), W warm-up steps, K timed steps."""
        torch.cuda.synchronize()
        t_setup = time.perf_counter()
        amg = AMG(ptr, col, vals[0], precision=precision, **amg_params)
        torch.cuda.synchronize()
        info_log = {"iters": [], "rebuilds": 0, "converged": True, "rel_res_max": 0.0,
                    "setup_ms": (time.perf_counter() - t_setup) * 1e3}

        def step(t, record):
            if mode == "partial":
                amg.rebuild(vals[t])
            elif mode in ("policy", "reuse_paper"):
                pol = POLICY if mode == "policy" else POLICY_REUSE
                if amg.rebuild_auto(vals[t], pol) == FULL and record:
                    info_log["rebuilds"] += 1
            elif mode == "full":
                amg.rebuild_ex(vals[t], FULL)
            else:
                amg.rebuild_ex(vals[t], OPERATOR_ONLY)
            u.zero_()
            _, info = solve(amg, rhs[t], u)
            its = info["iters"]
            if mode == "reuse" and not info["converged"]:
                amg.rebuild_ex(vals[t], FULL)
                u.zero_()
                _, info = solve(amg, rhs[t], u)
                its += info["iters"]
                if record:
                    info_log["rebuilds"] += 1
            if record:
                info_log["iters"].append(its)
                info_log.setdefault("missed", 0)
                info_log["missed"] += 0 if info["converged"] else 1
                if mode != "reuse_paper":  # that series misses the limit by design
                    info_log["converged"] &= bool(info["converged"])
                info_log["rel_res_max"] = max(info_log["rel_res_max"], info["rel_res_true"])

        for t in range(1, W + 1):
            step(t, False)
        if trace:
            amg.trace(trace, level=0)
            amg.trace_read()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        marks = [ts]
        for t in range(W + 1, W + K + 1):
            step(t, True)
            marks.append(time.perf_counter())  # a solve returns once it has read its last residual
        torch.cuda.synchronize()
        te = time.perf_counter()
        per = sorted((b - a) * 1e3 for a, b in zip(marks, marks[1:]))
        info_log["step_ms"] = {"median": per[len(per) // 2], "min": per[0], "max": per[-1]}
        kt = amg.trace_read() if trace else {}
        amg.trace([], level=0)
        return amg, (te - ts) * 1e3 / K, info_log, kt

    # ---------------------------------------------------------------- partial reuse (headline)
    spmv_cls = "bicg_spmv" if bicg else "cg_pq"
    traced = [spmv_cls, "galerkin_ap", "galerkin_rap"]
    amg, ms_partial, info_p, kt = series("partial", precision=head_prec, trace=traced)
    L = amg.num_levels
    dims = [amg.dims(l) for l in range(L)]
    ndiag = amg.level_format(0)
    nread = amg.diagonals_read(0)
    plane = amg.march_plane(0)
    if plane:
        pq_kernel = "k_m7_cg_pq"
    elif ndiag:
        pq_kernel = "k_w_cg_pq" if ndiag != 7 else "k_dia_cg_pq"
    elif cfg.get("block_size", 1) > 1:
        pq_kernel = "k_rb_spmv" if bicg else "k_node_cg_pq"
    else:
        pq_kernel = "k_rb_spmv" if bicg else "k_cg_pq"
    log(f"levels: {[(d[0], d[1]) for d in dims]}")
    log(f"partial reuse: {ms_partial:.3f} ms/step, iters {info_p['iters']}")
    ph = amg.phase_times()

    # per-kernel breakdown of one partial step on every level (diagnostic pass, not timed)
    from paper_2108_02054_amd.amg import KERNEL_CLASSES
    amg.trace(KERNEL_CLASSES, level=-1)
    amg.trace_read()
    amg.rebuild(vals[W + 1])
    u.zero_()
    solve(amg, rhs[W + 1], u)
    breakdown_all = amg.trace_read()
    amg.trace(KERNEL_CLASSES, level=0)
    amg.rebuild(vals[W + 1])
    u.zero_()
    solve(amg, rhs[W + 1], u)
    breakdown_l0 = amg.trace_read()
    amg.trace([], level=0)
    spmv_hot_us, spmv_cold_us = operator_timing(amg, n)
    amg.close()

    kb = kernel_bytes(dims, 8, ndiag, sym=0 < nread < ndiag, block=cfg.get("block_size", 1))
    # live measurement over the timed region
    pq_ms, pq_cnt = kt.get(spmv_cls, (0.0, 0))
    n_solves = K
    block = cfg.get("block_size", 1) > 1
    if bicg:
        spmv_bytes = pq_cnt * kb["krylov_spmv"]
    elif block:  # the product after its own direction update: p read, q written
        spmv_bytes = pq_cnt * (kb["cg_pq"] - 16 * n)
    else:
        spmv_bytes = pq_cnt * kb["cg_pq"] - n_solves * 8 * n  # first iteration reads no p_old
    spmv_gbs = spmv_bytes / (pq_ms * 1e-3) / 1e9 if pq_ms > 0 else None
    # y = A x as the CG's first iteration forms it: no p_old read (block systems: the
    # direction update and the product together)
    spmv_first_bytes = kb["cg_pq"] - 8 * n
    first_kernel = pq_kernel if not pq_kernel.startswith("k_rb") else "k_cg_pq"
    g_ms = kt.get("galerkin_ap", (0.0, 0))[0] + kt.get("galerkin_rap", (0.0, 0))[0]
    g_cnt = kt.get("galerkin_rap", (0.0, 0))[1]
    rap_gbs = g_cnt * kb["galerkin"] / (g_ms * 1e-3) / 1e9 if g_ms > 0 else None

    copy_gbs = copy_bandwidth()
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write, 1 GiB, best of 5)")

    # dominant kernel class of a partial step (all levels), by total time
    dom = max(breakdown_all.items(), key=lambda kv: kv[1][0])[0] if breakdown_all else "cg_pq"
    log("kernel time per partial step (ms, launches), all levels: "
        + ", ".join(f"{k}={v[0]:.3f}/{v[1]}" for k, v in sorted(breakdown_all.items(), key=lambda kv: -kv[1][0])))

    def roof(name, ms, launches, alg_bytes, traffic_rec=None):
        """Roofline record of one kernel from its live HIP-event timing: algorithmic bytes per
        launch over the average launch duration; traffic = measured HBM bytes per launch
        (FETCH_SIZE + WRITE_SIZE, scaled by a known-size copy) when the stored counters were
        taken on the current kernel source, else null."""
        avg_us = ms * 1e3 / launches if launches else None
        achieved = alg_bytes / (avg_us * 1e-6) / 1e9 if avg_us else None
        return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                "traffic": traffic_rec["traffic_bytes_per_launch"] if traffic_rec else None,
                "algorithmic_bytes": alg_bytes, "avg_launch_us": avg_us, "launches": launches,
                "traffic_source": (f"profiles/{os.path.basename(traffic_rec['_path'])}" if traffic_rec else None)}

    from paper_2108_02054_amd.profiling import load_traffic
    pq_traffic = load_traffic(os.path.join(ROOT, "profiles", "cg_pq_two_fluid_128_traffic.json"))
    if pq_traffic is not None:
        pq_traffic["_path"] = "cg_pq_two_fluid_128_traffic.json"
    if cfg_id == 7:
        pq_traffic = load_traffic(os.path.join(ROOT, "profiles", "cg_pq_coupled4_56_traffic.json"))
        if pq_traffic is not None:
            pq_traffic["_path"] = "cg_pq_coupled4_56_traffic.json"
    rap_traffic = load_traffic(os.path.join(ROOT, "profiles", "galerkin_two_fluid_128_traffic.json"))
    if rap_traffic is not None:
        rap_traffic["_path"] = "galerkin_two_fluid_128_traffic.json"

    result = {
        "metric": METRIC,
        "value": ms_partial,
        "unit": "ms/step",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_partial,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head_prec == 0 else "f32 hierarchy and V-cycle, f64 CG",
        "data": "synthetic",
        "config": {"workload": workload_name(cfg_id, N, n, nnz),
                   "grid": N, "n": n, "nnz": nnz, "levels": L, "level_rows": [d[0] for d in dims],
                   "level_nnz": [d[1] for d in dims], "level0_storage": ((f"{ndiag} diagonals, {nread} read per row"
                                      + (f", marching planes of {plane} rows" if plane else "")) if ndiag else "CSR"),
                   "parallelism": "single GPU"},
        "iters_partial": info_p["iters"],
        "converged_all": info_p["converged"],
        "rel_res_max": info_p["rel_res_max"],
        "rebuild_phase_ms": ph,
        "setup_ms_step0": info_p["setup_ms"],
        "step_ms_spread": info_p["step_ms"],
        "copy_gbs_measured": copy_gbs,
        "krylov_spmv_first_iteration": {
            "kernel": first_kernel, "algorithmic_bytes": spmv_first_bytes,
            "hot_us": spmv_hot_us, "cold_us": spmv_cold_us,
            "hot_frac": spmv_first_bytes / (spmv_hot_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "cold_frac": spmv_first_bytes / (spmv_cold_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "note": "y = A x through amg_apply_operator (p = z, no p_old read), median of 7; cold: after a "
                    "512 MiB read that evicts L2 and the MALL"},
        "spmv_gbs": spmv_gbs,
        "rap_gbs": rap_gbs,
        "dominant_kernel": dom,
        "roofline": roof(pq_kernel + (" (BiCGStab Krylov operator products v = A p^, t = A s^, level 0)" if bicg
                                      else " (Krylov operator SpMV q = A p and p.q after the direction update, level 0)"
                                      if block else " (Krylov operator SpMV with p = z + beta p and p.q, level 0)"),
                         pq_ms, pq_cnt,
                         spmv_bytes / pq_cnt if pq_cnt else 0,
                         pq_traffic if (N == cfg["N"] and cfg_id in (2, 7) and pq_traffic is not None
                                        and pq_traffic["kernel"] == pq_kernel) else None),
        "roofline_rap": roof("k_galerkin_pos A_0 P_0 then R_0 (A_0 P_0), per rebuild (level 0)", g_ms, g_cnt,
                             kb["galerkin"],
                             rap_traffic if (cfg_id == 2 and N == 128 and head_prec == 0) else None),
        "kernels_level0_ms": {k: v for k, v in breakdown_l0.items()},
        "kernels_all_levels_ms": {k: v for k, v in breakdown_all.items()},
    }

    # ---------------------------------------------------------------- comparators
    if not args.no_compare:
        runs = {}
        if cfg_id == 5:
            plan = [("full", "full", 1), ("fp64_partial", "partial", 0)]
        elif cfg_id == 3:
            plan = [("mixed", "partial", 1), ("full", "full", 0)]
        elif cfg_id in (6, 7):
            plan = [("full", "full", 0), ("mixed", "partial", 1)]
        else:
            plan = [("full", "full", 0), ("reuse", "reuse", 0), ("mixed", "partial", 1), ("policy", "policy", 0),
                    ("reuse_paper", "reuse_paper", 0)]
        for name, mode, prec in plan:
            _, ms_x, info_x, _ = series(mode, precision=prec)
            runs[name] = (ms_x, info_x)
            extra = f", full setups {info_x['rebuilds']}" if mode in ("reuse", "policy", "reuse_paper") else ""
            if mode == "reuse_paper":
                extra += f", solves past the iteration limit {info_x.get('missed', 0)}"
            log(f"{name}: {ms_x:.3f} ms/step, iters {info_x['iters']}{extra}")
        conv = info_p["converged"]
        for name, (ms_x, info_x) in runs.items():
            conv = conv and bool(info_x["converged"])
        if "full" in runs:
            result["full_rebuild_ms_per_step"] = runs["full"][0]
            result["iters_full_rebuild"] = runs["full"][1]["iters"]
            # the paper's speedup form: (t_base / t - 1) * 100
            result["total_speedup_vs_full_rebuild_pct"] = (runs["full"][0] / ms_partial - 1.0) * 100.0
        if "reuse" in runs:
            result["full_reuse_ms_per_step"] = runs["reuse"][0]
            result["iters_full_reuse"] = runs["reuse"][1]["iters"]
            result["full_reuse_rebuilds"] = runs["reuse"][1]["rebuilds"]
        if "mixed" in runs:
            result["mixed_partial_ms_per_step"] = runs["mixed"][0]
            result["iters_mixed"] = runs["mixed"][1]["iters"]
            result["mixed_speedup_vs_fp64_pct"] = (ms_partial / runs["mixed"][0] - 1.0) * 100.0
        if "policy" in runs:
            result["policy_every_ms_per_step"] = runs["policy"][0]
            result["policy"] = f"partial reuse with a full setup every {POLICY.every}th step"
            result["iters_policy"] = runs["policy"][1]["iters"]
            result["policy_full_setups"] = runs["policy"][1]["rebuilds"]
        if "reuse_paper" in runs:
            result["full_reuse_paper_ms_per_step"] = runs["reuse_paper"][0]
            result["iters_full_reuse_paper"] = runs["reuse_paper"][1]["iters"]
            result["full_reuse_paper_full_setups"] = runs["reuse_paper"][1]["rebuilds"]
            result["full_reuse_paper_missed_solves"] = runs["reuse_paper"][1].get("missed", 0)
        if "fp64_partial" in runs:
            result["fp64_partial_ms_per_step"] = runs["fp64_partial"][0]
            result["iters_fp64"] = runs["fp64_partial"][1]["iters"]
            result["mixed_speedup_vs_fp64_pct"] = (runs["fp64_partial"][0] / ms_partial - 1.0) * 100.0
        result["converged_all"] = conv

    # ---------------------------------------------------------------- CPU oracle sample
    if not args.no_cpu:
        import oracle
        nthr = oracle.num_threads()
        p, c, v0 = series_matrix(cfg_id, 0, N)
        t0 = time.time()
        h = oracle.OracleHierarchy(p, c, v0, **amg_params)
        t_setup = time.time() - t0
        ks = max(1, args.cpu_steps if cfg_id == 2 else 1)
        elapsed = 0.0
        its = []
        for t in range(1, ks + 1):
            _, _, vt = series_matrix(cfg_id, t, N)
            ft = rhs_uniform(n, cfg_id, t)
            ts = time.perf_counter()  # the step's inputs are generated outside the timing
            h.rebuild(vt, 0)
            _, io = h.solve_bicgstab(ft) if bicg else h.solve(ft)
            elapsed += time.perf_counter() - ts
            its.append(io["iters"])
        cpu_ms = elapsed * 1e3 / ks
        # one more step on one thread (the oracle's results do not depend on the count)
        oracle.set_num_threads(1)
        _, _, vt = series_matrix(cfg_id, ks + 1, N)
        ft = rhs_uniform(n, cfg_id, ks + 1)
        ts = time.perf_counter()
        h.rebuild(vt, 0)
        _, io1 = h.solve_bicgstab(ft) if bicg else h.solve(ft)
        cpu1_ms = (time.perf_counter() - ts) * 1e3
        oracle.set_num_threads(nthr)
        h.close()
        log(f"oracle: setup {t_setup:.1f}s, partial step {cpu_ms:.0f} ms ({nthr} threads), iters {its}; "
            f"one thread {cpu1_ms:.0f} ms")
        result["cpu_baseline"] = {"value": cpu_ms, "unit": "ms/step", "cores": nthr, "kind": "oracle",
                                  "sample": f"oracle (FP64) partial rebuild + {'BiCGStab' if bicg else 'PCG'} solve "
                                            f"to 1e-8 of {cfg['name']} at "
                                            f"{N}^3, steps t=1..{ks} after an untimed setup at t=0 (full setup "
                                            f"took {t_setup:.1f}s); iterations {its}",
                                  "cpu_model": cpu_model(),
                                  "single_thread_ms_per_step": cpu1_ms}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
