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
(Algorithm 3, with a rebuild-and-retry when a solve does not converge in maxiter, and as
the paper runs it), an occasional-full-rebuild policy, the mixed-precision form (FP32
hierarchy under FP64 CG), the setup and solve time of each strategy (the paper's Table 2
form) and the phases of the full setup (its Table 1 form), per-kernel HIP-event timings on
every level, the roofline of the step's dominant kernel, of the Krylov SpMV and of the
level-0 Galerkin product, short legs of the 192^3 two-fluid and 160^3 27-point series
(working sets beyond the 256 MB MALL), and the CPU oracle on a bounded sample.

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
# the timed steps time every TRACE_EVERY-th launch of the dominant kernel class per level
TRACE_EVERY = 8
# untimed steps after the timed ones that time every launch of the Krylov SpMV and the
# Galerkin products
XSTEPS = 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed time steps")
    ap.add_argument("--warmup", type=int, default=3, help="untimed time steps before the timed ones")
    ap.add_argument("--config", type=int, default=2, choices=[2, 3, 4, 5, 6, 7],
                    help="matrix series: 2 = two-fluid 7-point 128^3 FP64 (the headline), 3 = two-fluid "
                         "7-point 192^3, 4 = the differentiable solve on the 7-point log-coefficient operator "
                         "(128^3; forward and adjoint solves on the reused hierarchy), 5 = lognormal 27-point "
                         "160^3 with the FP32 hierarchy, 6 = non-symmetric convection-diffusion 7-point 128^3 "
                         "solved by BiCGStab, 7 = coupled system with 4x4 blocks on 56^3 nodes (node "
                         "aggregation, block Jacobi)")
    ap.add_argument("--n", type=int, default=0, help="grid size N (N^3 nodes); 0: the series' own")
    ap.add_argument("--no-compare", action="store_true", help="skip the full-rebuild/full-reuse/mixed runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-legs", action="store_true", help="skip the short 192^3 and 160^3 legs")
    ap.add_argument("--leg-steps", type=int, default=2, help="timed steps of each short leg")
    ap.add_argument("--cpu-steps", type=int, default=12, help="oracle partial steps in the CPU sample")
    ap.add_argument("--aggregation", type=int, default=None, choices=[0, 1],
                    help="transfer operators: 0 = smoothed aggregation, 1 = plain aggregation (P = P_tent, the "
                         "paper's own form); default: the series' own")
    ap.add_argument("--allocator", default="torch", choices=["torch", "library"],
                    help="device memory of the hierarchy: PyTorch's caching allocator or the library's pool")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized FP64 buffer 3 times and exit: the known-size reference "
                         "that scales the FETCH_SIZE / WRITE_SIZE counters of the other kernels")
    return ap.parse_args()


def workload_name(cfg_id, N, n, nnz, prec, plain=False):
    series = {2: "two-fluid 7-point Poisson, rho ratio 1000, interface +1 cell/step",
              3: "two-fluid 7-point Poisson, rho ratio 1000, interface +1 cell/step",
              5: "27-point lognormal-coefficient Poisson (sigma 1.5) with smooth drift per step",
              6: "non-symmetric upwind convection-diffusion 7-point, flow turning 9 degrees per step",
              7: "coupled system, 4 unknowns per node in full 4x4 blocks on the 7-point node graph (two-fluid "
                 "face weights, SPD couplings turning 9 degrees per step, interface +1 cell/step)"}[cfg_id]
    form = "FP32 hierarchy and V-cycle under FP64 CG" if prec == 1 else "FP64"
    krylov = "BiCGStab" if cfg_id == 6 else "PCG"
    amg = ("plain aggregation of nodes on block norms, damped block Jacobi; " if cfg_id == 7
           else "plain aggregation (P = P_tent); " if plain else "")
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

    def once(cold):
        if cold:
            scrub.sum()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        amg.apply_operator(x, y)
        b.record()
        b.synchronize()
        return a.elapsed_time(b) * 1e3

    hot = sorted(once(False) for _ in range(reps))
    cold = sorted(once(True) for _ in range(reps))
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

class ByteModel:
    """Algorithmic bytes per launch of each kernel class on each level: every operand read
    once, every output written once, vector gathers counted once.  CSR operators count
    their row pointers (4 B), their columns as the kernels read them (4 B, or 2 B per
    entry plus one 4 B base per row block when the level keeps two-byte column offsets)
    and their values (8 B FP64, 4 B FP32); an operator in diagonal storage counts its
    values only, with symmetric values only the main and upper diagonals; an operator of
    full B x B blocks one index per block and one pointer per node (its Krylov SpMV)."""

    def __init__(self, dims, storage, ndiag=0, nread=0, block=1):
        self.L = len(dims)
        self.dims = dims
        self.st = storage
        self.ndiag = ndiag
        self.nread = nread
        self.block = block
        self.s = self.st[0]["value_bytes"]

    @classmethod
    def of(cls, amg, block=1):
        L = amg.num_levels
        return cls([amg.dims(l) for l in range(L)], [amg.level_storage(l) for l in range(L)],
                   amg.level_format(0), amg.diagonals_read(0), block)

    def _csr(self, rows, nnz, c16, rpb, s):
        cols = 2 * nnz + (4 * ((rows + rpb - 1) // rpb) if rpb > 0 else 0) if c16 else 4 * nnz
        return 4 * (rows + 1) + cols + s * nnz

    def a0_entries(self):
        n, nnz = self.dims[0][0], self.dims[0][1]
        return (nnz + n) // 2 if (self.ndiag > 0 and 0 < self.nread < self.ndiag) else nnz

    def A(self, l, s=None):
        s = self.s if s is None else s
        n, nnz = self.dims[l][0], self.dims[l][1]
        if l == 0 and self.ndiag > 0:
            return s * self.a0_entries()
        return self._csr(n, nnz, self.st[l]["A_c16"], self.st[l]["A_rpb"], s)

    def P(self, l):
        n, _, nc, nnzP, _ = self.dims[l]
        return self._csr(n, nnzP, self.st[l]["P_c16"], self.st[l]["P_rpb"], self.s)

    def R(self, l):
        n, _, nc, nnzP, _ = self.dims[l]
        return self._csr(nc, nnzP, self.st[l]["R_c16"], self.st[l]["R_rpb"], self.s)

    def krylov_A(self):
        """Level-0 operator as the FP64 Krylov SpMV reads it."""
        n, nnz = self.dims[0][0], self.dims[0][1]
        if self.ndiag > 0:
            return 8 * self.a0_entries()
        if self.block > 1:
            B = self.block
            return 4 * (n // B + 1) + 4 * (nnz // (B * B)) + 8 * nnz
        return 4 * (n + 1) + 4 * nnz + 8 * nnz

    def galerkin(self, l):
        """A_l, P_l, R_l read once, A_{l+1} written once with its cached columns read once
        (the A_l P_l intermediate and the cached plan are implementation costs).  The node
        form of a block system: A_l's values read and A_{l+1}'s written once, P_l and R_l as
        one aggregate index per node, A_{l+1}'s node pattern read once."""
        n, nnzA, nc, nnzP, _ = self.dims[l]
        nnzAc = self.dims[l + 1][1]
        s = self.s
        if self.st[l].get("node_galerkin"):
            B = self.block
            return s * (nnzA + nnzAc) + 8 * (n // B) + 4 * (nc // B + 1) + 4 * (nnzAc // (B * B))
        ind = lambda rows, nnz: 4 * (rows + 1) + 4 * nnz  # noqa: E731
        return (ind(n, nnzA) + s * nnzA + 2 * (ind(n, nnzP) + s * nnzP) - 4 * (n + 1) + 4 * (nc + 1)
                + ind(nc, nnzAc) + s * nnzAc)

    def bytes(self, cls, l):
        """Bytes per launch of class cls on level l, or None when the class has no model
        there."""
        s = self.s
        n = self.dims[l][0]
        nc = self.dims[l][2]
        last = self.L - 1
        if cls == "cg_pq" and l == 0:
            if self.block > 1:   # product after its own direction update: p read, q written
                return self.krylov_A() + 16 * n
            return self.krylov_A() + 32 * n      # z, p_old read; p_new, q written
        if cls == "cg_update" and l == 0:
            if self.ndiag > 0 and s == 8:        # fused with the first sweep and its residual
                return 8 * self.a0_entries() + 72 * n
            return 48 * n if s == 8 else None
        if cls == "cg_rz" and l == 0:
            return 16 * n
        if cls == "jacobi" and l < last:          # u' = u + m (f - A u); level 0: + r.z
            return self.A(l) + 4 * s * n
        if cls == "smooth0_res" and l < last:
            # level 0: u = m f and r = f - A u; below, the restriction formed u and the
            # kernel forms the residual (f, u read, r written)
            return self.A(l) + (4 if l == 0 else 3) * s * n
        if cls == "restrict" and l < last:
            smooths = (l + 2 < self.L) and not self.st[l + 1]["tail"]
            return self.R(l) + s * n + s * nc + (2 * s * nc if smooths else 0)
        if cls == "prolong" and l < last:
            return self.P(l) + s * nc + 2 * s * n
        if cls == "coarse_gemv" and l == last:
            return 8 * n * n + 2 * s * n
        return None


def roof(name, ms, launches, alg_bytes_total, traffic_rec=None):
    """Roofline record of one kernel from its live HIP-event timing: algorithmic bytes per
    launch over the average launch duration; traffic = measured HBM bytes per launch
    (FETCH_SIZE + WRITE_SIZE, scaled by a known-size copy) when the stored counters were
    taken on the current kernel source, else null."""
    avg_us = ms * 1e3 / launches if launches else None
    per = alg_bytes_total / launches if launches else 0.0
    achieved = per / (avg_us * 1e-6) / 1e9 if avg_us else None
    return {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic_rec["traffic_bytes_per_launch"] if traffic_rec else None,
            "algorithmic_bytes": per, "avg_launch_us": avg_us, "launches": launches,
            "traffic_source": (f"profiles/{os.path.basename(traffic_rec['_path'])}" if traffic_rec else None)}


def kernel_groups(L, bm, plane, block, bicg):
    """The kernels of a step as (name, class, levels): a traced class restricted to the
    levels on which one kernel function runs it, so that times compare with a kernel
    trace's per-kernel statistics."""
    up = set(range(1, L))
    if bicg:
        pq = "k_m7_cg_pq (BiCGStab products)" if plane else "k_rb_spmv (BiCGStab products)"
    elif plane:
        pq = "k_m7_cg_pq"
    elif bm.ndiag:
        pq = "k_w_cg_pq" if bm.ndiag != 7 else "k_dia_cg_pq"
    else:
        pq = "k_node_cg_pq" if block > 1 else "k_cg_pq"
    if plane:
        upd, post = "k_m7_update_smooth0", "k_m7_jacobi_rz"
    elif bm.ndiag:
        upd, post = "k_w_update_smooth0 / k_dia_update_smooth0", "k_w_jacobi_rz / k_dia_jacobi_rz"
    elif block > 1:
        upd, post = "k_cg_update", "k_node_sweep_rz"
    else:
        upd, post = "k_cg_update", "k_jacobi_rz"
    g = [(pq, "bicg_spmv" if bicg else "cg_pq", {0}), (upd, "cg_update", {0}),
         (post + " (level-0 post-sweep)", "jacobi", {0}),
         ("k_rb_jacobi" if block == 1 else "k_node_sweep / k_rb_jacobi", "jacobi", up),
         ("k_rb_residual", "smooth0_res", up), ("k_rb_spmv (restriction R_l)", "restrict", set(range(L))),
         ("k_rb_prolong_add (prolongation P_l)", "prolong", set(range(L))),
         ("k_vcycle_tail", "tail", set(range(L))), ("k_coarse_gemv", "coarse_gemv", set(range(L)))]
    return g


def load_traffic_rec(name):
    from paper_2108_02054_amd.profiling import load_traffic
    rec = load_traffic(os.path.join(ROOT, "profiles", name))
    if rec is not None:
        rec["_path"] = name
    return rec


# ------------------------------------------------------------------ one configuration

def run_config(cfg_id, N, K, W, args, headline_prec=None, compare=True, legs_mode=False):
    import numpy as np  # noqa: F401
    import torch

    from paper_2108_02054_amd import AMG, FULL, OPERATOR_ONLY
    from paper_2108_02054_amd.amg import KERNEL_CLASSES, PARTIAL, policy
    from workloads import CONFIGS, rhs_uniform, series_matrix

    POLICY = policy(PARTIAL, every=10)  # an occasional full setup between partial updates (Section 3)
    # full reuse as the paper runs it: a solve that misses the iteration limit is not
    # repeated; the next update is a full setup (Algorithm 3, Section 3)
    POLICY_REUSE = policy(OPERATOR_ONLY)
    dev = torch.device("cuda:0")
    cfg = CONFIGS[cfg_id]
    head_prec = (1 if cfg_id == 5 else 0) if headline_prec is None else headline_prec
    bicg = cfg_id == 6
    block = cfg.get("block_size", 1)
    nsteps = W + K + 1
    amg_params = dict(eps_strong=cfg["eps_strong"], allocator=args.allocator)
    for key in ("block_size", "aggregation"):
        if key in cfg:
            amg_params[key] = cfg[key]
    if args.aggregation is not None:
        amg_params["aggregation"] = args.aggregation

    def solve(amg, f, x):
        return amg.solve_bicgstab(f, x) if bicg else amg.solve(f, x)

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
    spmv_cls = "bicg_spmv" if bicg else "cg_pq"

    def groups_of(amg):
        bm_ = ByteModel.of(amg, block)
        return kernel_groups(bm_.L, bm_, amg.march_plane(0), block, bicg)

    def dominant(ktl, groups):
        """The kernel with the largest total time in one step (per-level table)."""
        def tot(gr):
            return sum(ktl[l].get(gr[1], (0.0, 0))[0] for l in gr[2] if l < len(ktl))
        return max(groups, key=tot)

    def series(mode, precision=0, diag=False, snap=False):
        """Setup at t=0 (untimed), W warm-up steps, optionally a per-level kernel table
        (untimed), K timed steps with the setup and solve of each step timed apart; with
        snap, host copies of the last step's level values, smoother and solution (untimed)."""
        torch.cuda.synchronize()
        t_setup = time.perf_counter()
        amg = AMG(ptr, col, vals[0], precision=precision, **amg_params)
        torch.cuda.synchronize()
        log_ = {"iters": [], "rebuilds": 0, "converged": True, "rel_res_max": 0.0, "missed": 0,
                "setup_ms": (time.perf_counter() - t_setup) * 1e3, "phases": []}

        def step(t, record, ev=None):
            if ev is not None:
                ev[0].record()
            full = False
            if mode == "partial":
                amg.rebuild(vals[t])
            elif mode in ("policy", "reuse_paper"):
                full = amg.rebuild_auto(vals[t], POLICY if mode == "policy" else POLICY_REUSE) == FULL
            elif mode == "full":
                amg.rebuild_ex(vals[t], FULL)
                full = True
            else:
                amg.rebuild_ex(vals[t], OPERATOR_ONLY)
            if full and record:
                log_["rebuilds"] += 1
                log_["phases"].append(amg.phase_times())
            if ev is not None:
                ev[1].record()
            u.zero_()
            _, info = solve(amg, rhs[t], u)
            its = info["iters"]
            if mode == "reuse" and not info["converged"]:
                if ev is not None:
                    ev[2].record()
                    ev[3].record()
                amg.rebuild_ex(vals[t], FULL)
                if ev is not None:
                    ev[4].record()
                u.zero_()
                _, info = solve(amg, rhs[t], u)
                its += info["iters"]
                if record:
                    log_["rebuilds"] += 1
            elif ev is not None:
                for e in ev[2:5]:
                    e.record()
            if ev is not None:
                ev[5].record()
            if record:
                log_["iters"].append(its)
                log_["last_rel_res"] = info["rel_res_true"]
                log_["missed"] += 0 if info["converged"] else 1
                if mode != "reuse_paper":  # that series misses the limit by design
                    log_["converged"] &= bool(info["converged"])
                log_["rel_res_max"] = max(log_["rel_res_max"], info["rel_res_true"])

        for t in range(1, W + 1):
            step(t, False)
        kt_levels = None
        if diag:
            # per-level kernel table of one step (repeats step W; untimed)
            L = amg.num_levels
            kt_levels = [dict() for _ in range(L)]
            for l in range(L):
                amg.trace(KERNEL_CLASSES, level=l)
                amg.trace_read()
                step(max(W, 1), False)
                got = amg.trace_read_levels()
                kt_levels[l] = got[l]
            amg.trace([], level=0)
        traced = None
        if diag:
            # the timed steps bracket only every TRACE_EVERY-th launch of the dominant
            # kernel class per level with events: each bracketed launch holds the stream for
            # its timestamps (tracing all launches of four classes cost 0.8 ms per 128^3 step)
            dom = dominant(kt_levels, groups_of(amg))
            traced = [dom[1]]
            amg.trace(traced, level=-1, every=TRACE_EVERY)
            amg.trace_read()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(K)]
        torch.cuda.synchronize()
        ts = time.perf_counter()
        marks = [ts]
        for i, t in enumerate(range(W + 1, W + K + 1)):
            step(t, True, evs[i])
            marks.append(time.perf_counter())  # a solve returns once it has read its last residual
        torch.cuda.synchronize()
        te = time.perf_counter()
        per = sorted((b - a) * 1e3 for a, b in zip(marks, marks[1:]))
        log_["step_ms"] = {"median": per[len(per) // 2], "min": per[0], "max": per[-1]}
        setup_ms = sum(e[0].elapsed_time(e[1]) + e[3].elapsed_time(e[4]) for e in evs) / K
        solve_ms = sum(e[1].elapsed_time(e[2]) + e[4].elapsed_time(e[5]) for e in evs) / K
        log_["setup_ms_per_step"], log_["solve_ms_per_step"] = setup_ms, solve_ms
        kt = amg.trace_read_levels() if traced else None
        amg.trace([], level=0)
        kx = None
        if diag:
            # untimed instrumented steps (the last step's values again): every launch of the
            # Krylov SpMV and of the Galerkin products bracketed
            amg.trace(sorted({spmv_cls, "galerkin_ap", "galerkin_rap"}), level=-1)
            amg.trace_read()
            for _ in range(XSTEPS):
                step(W + K, False)
            kx = amg.trace_read_levels()
            amg.trace([], level=0)
        log_["kt_levels"], log_["kt"], log_["kx"] = kt_levels, kt, kx
        if snap:
            lv = [amg.level(l) for l in range(amg.num_levels)]
            log_["snap"] = {"A": [x["A"][2] for x in lv], "m": [x["m"] for x in lv], "u": u.cpu().numpy()}
            del lv
        return amg, (te - ts) * 1e3 / K, log_

    # ---------------------------------------------------------------- partial reuse (headline)
    amg, ms_partial, info_p = series("partial", precision=head_prec, diag=True, snap=compare)
    bm = ByteModel.of(amg, block)
    L = bm.L
    dims = bm.dims
    plane = amg.march_plane(0)
    log(f"levels: {[(d[0], d[1]) for d in dims]}")
    log(f"partial reuse: {ms_partial:.3f} ms/step (setup {info_p['setup_ms_per_step']:.3f} + solve "
        f"{info_p['solve_ms_per_step']:.3f}), iters {info_p['iters']}")
    spmv_hot_us, spmv_cold_us = operator_timing(amg, n)
    amg.close()
    del amg
    torch.cuda.empty_cache()

    # kernel table of one partial step, per level and class
    ktl = info_p["kt_levels"]
    totals = {}
    for l, lv in enumerate(ktl):
        for k, (ms, cnt) in lv.items():
            a = totals.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] += cnt
    log("kernel time per partial step (ms, launches), all levels: "
        + ", ".join(f"{k}={v[0]:.3f}/{v[1]}" for k, v in sorted(totals.items(), key=lambda kv: -kv[1][0])))

    # live records: the dominant class over the timed region (sampled launches), the
    # Krylov SpMV and the Galerkin products over the instrumented steps after it
    kt = info_p["kt"]
    kx = info_p["kx"]

    def class_live(cls, levels=None, src=None):
        src = kt if src is None else src
        ms = cnt = 0
        byt = 0.0
        ok = True
        for l in (range(L) if levels is None else levels):
            m_, c_ = src[l].get(cls, (0.0, 0))
            if not c_:
                continue
            b = bm.bytes(cls, l)
            if b is None:
                ok = False
            else:
                byt += b * c_
            ms += m_
            cnt += c_
        return ms, cnt, (byt if ok else None)

    groups = kernel_groups(L, bm, plane, block, bicg)
    dom_name, dom, dom_levels = dominant(ktl, groups)
    d_ms, d_cnt, d_bytes = class_live(dom, sorted(dom_levels))
    by_kernel = {}
    for name, cls, lvls in groups:
        ms_ = sum(ktl[l].get(cls, (0.0, 0))[0] for l in lvls if l < L)
        cnt_ = sum(ktl[l].get(cls, (0.0, 0))[1] for l in lvls if l < L)
        if cnt_:
            by_kernel[name] = [round(ms_, 4), cnt_]
    pq_ms, pq_cnt, _ = class_live(spmv_cls, [0], kx)
    if bicg:
        spmv_bytes = pq_cnt * (bm.krylov_A() + 16 * n)
    elif block > 1:
        spmv_bytes = pq_cnt * bm.bytes("cg_pq", 0)
    else:
        spmv_bytes = pq_cnt * bm.bytes("cg_pq", 0) - XSTEPS * 8 * n  # first iteration reads no p_old

    def gal_cnt(l):  # products per level (the node form of a block system is one launch, traced as A P)
        return kx[l].get("galerkin_rap", (0.0, 0))[1] or kx[l].get("galerkin_ap", (0.0, 0))[1]

    g_ms = kx[0].get("galerkin_ap", (0.0, 0))[0] + kx[0].get("galerkin_rap", (0.0, 0))[0]
    g_cnt = gal_cnt(0)
    rap_all_ms = sum(kx[l].get("galerkin_ap", (0.0, 0))[0] + kx[l].get("galerkin_rap", (0.0, 0))[0]
                     for l in range(L))
    rap_all_bytes = sum(bm.galerkin(l) * gal_cnt(l) for l in range(L - 1))

    if plane:
        pq_kernel = "k_m7_cg_pq"
    elif bm.ndiag:
        pq_kernel = "k_w_cg_pq" if bm.ndiag != 7 else "k_dia_cg_pq"
    elif block > 1:
        pq_kernel = "k_rb_spmv" if bicg else "k_node_cg_pq"
    else:
        pq_kernel = "k_rb_spmv" if bicg else "k_cg_pq"
    first_kernel = pq_kernel if not pq_kernel.startswith("k_rb") else "k_cg_pq"
    spmv_first_bytes = (bm.bytes("cg_pq", 0) - 8 * n) if not block > 1 else bm.bytes("cg_pq", 0)

    plain = args.aggregation == 1 and cfg_id != 7
    work = workload_name(cfg_id, N, n, nnz, head_prec, plain)
    is_headline = cfg_id == 2 and N == 128 and head_prec == 0 and not plain
    dom_traffic = None
    pq_traffic = None
    rap_traffic = None
    dom_file = dom_name.split(" ")[0]
    if is_headline:
        dom_traffic = load_traffic_rec(f"{dom_file}_two_fluid_128_traffic.json")
        pq_traffic = load_traffic_rec("cg_pq_two_fluid_128_traffic.json")
        rap_traffic = load_traffic_rec("galerkin_two_fluid_128_traffic.json")
    elif cfg_id == 5 and N == 160:
        pq_traffic = load_traffic_rec("cg_pq_lognormal27_160_traffic.json")
    elif cfg_id == 7 and N == 56:
        pq_traffic = load_traffic_rec("cg_pq_coupled4_56_traffic.json")
        if bm.st[0].get("node_galerkin"):
            rap_traffic = load_traffic_rec("node_rap_coupled4_56_traffic.json")
    dom_rec = roof(f"{dom_name}: levels {sorted(dom_levels)} (the kernel with the step's largest time)",
                   d_ms, d_cnt, d_bytes or 0.0, dom_traffic)
    dom_rec["per_level"] = [{"level": l, "launches": kt[l].get(dom, (0, 0))[1],
                             "avg_us": (kt[l][dom][0] * 1e3 / kt[l][dom][1]) if kt[l].get(dom, (0, 0))[1] else None,
                             "algorithmic_bytes": bm.bytes(dom, l)}
                            for l in sorted(dom_levels) if l < L and kt[l].get(dom, (0, 0))[1]]
    spmv_rec = roof(pq_kernel + (" (BiCGStab Krylov operator products v = A p^, t = A s^, level 0)" if bicg
                                 else " (Krylov operator SpMV q = A p and p.q after the direction update, level 0)"
                                 if block > 1 else " (Krylov operator SpMV with p = z + beta p and p.q, level 0)"),
                    pq_ms, pq_cnt, spmv_bytes,
                    pq_traffic if (pq_traffic and pq_traffic["kernel"] == pq_kernel) else None)
    rap_name = ("k_node_rap R_0 A_0 P_0 in one pass over the BxB blocks" if bm.st[0].get("node_galerkin")
                else "k_galerkin_pos A_0 P_0 then R_0 (A_0 P_0)")
    rap_rec = roof(f"{rap_name}, per rebuild (level 0)", g_ms, g_cnt, g_cnt * bm.galerkin(0), rap_traffic)
    dom_rec["timing"] = (f"HIP events attached to every {TRACE_EVERY}th launch per level, on the library's "
                         f"stream, over the {K} timed steps")
    for r_ in (spmv_rec, rap_rec):
        r_["timing"] = (f"HIP events attached to every launch, on the library's stream, over {XSTEPS} untimed "
                        f"steps after the timed ones")

    res = {
        "ms_partial": ms_partial, "n": n, "nnz": nnz, "work": work, "head_prec": head_prec,
        "levels": L, "dims": dims, "ndiag": bm.ndiag, "nread": bm.nread, "plane": plane,
        "info_p": info_p, "dom": dom_name, "roofline_dominant": dom_rec, "by_kernel": by_kernel, "roofline_spmv": spmv_rec,
        "roofline_rap": rap_rec,
        "rap_all_levels": {"ms_per_rebuild": rap_all_ms / max(g_cnt, 1),
                           "algorithmic_bytes": rap_all_bytes / max(g_cnt, 1),
                           "frac": (rap_all_bytes / (rap_all_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if rap_all_ms else None},
        "krylov_spmv_first_iteration": {
            "kernel": first_kernel, "algorithmic_bytes": spmv_first_bytes,
            "hot_us": spmv_hot_us, "cold_us": spmv_cold_us,
            "hot_frac": spmv_first_bytes / (spmv_hot_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "cold_frac": spmv_first_bytes / (spmv_cold_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
            "note": "y = A x through amg_apply_operator (p = z, no p_old read), median of 7; cold: after a "
                    "512 MiB read that evicts L2 and the MALL"},
        "kernels_by_level": [{k: [round(v[0], 4), v[1]] for k, v in lv.items()} for lv in ktl],
        "kernels_all_levels_ms": {k: [round(v[0], 4), v[1]] for k, v in totals.items()},
    }
    if not compare:
        return res

    # ---------------------------------------------------------------- comparators
    runs = {}
    if legs_mode:
        plan = [("full", "full", head_prec)] + ([("mixed", "partial", 1)] if head_prec == 0 else
                                                [("fp64_partial", "partial", 0)])
    elif cfg_id == 5:
        plan = [("full", "full", 1), ("fp64_partial", "partial", 0)]
    elif cfg_id == 3:
        plan = [("mixed", "partial", 1), ("full", "full", 0)]
    elif cfg_id in (6, 7):
        plan = [("full", "full", 0), ("mixed", "partial", 1)]
    else:
        plan = [("full", "full", 0), ("reuse", "reuse", 0), ("mixed", "partial", 1), ("policy", "policy", 0),
                ("reuse_paper", "reuse_paper", 0)]
    for name, mode, prec in plan:
        a, ms_x, info_x = series(mode, precision=prec, snap=name in ("mixed", "fp64_partial"))
        a.close()
        del a
        runs[name] = (ms_x, info_x)
        extra = f", full setups {info_x['rebuilds']}" if mode in ("reuse", "policy", "reuse_paper") else ""
        if mode == "reuse_paper":
            extra += f", solves past the iteration limit {info_x['missed']}"
        log(f"{name}: {ms_x:.3f} ms/step (setup {info_x['setup_ms_per_step']:.3f} + solve "
            f"{info_x['solve_ms_per_step']:.3f}), iters {info_x['iters']}{extra}")
    for name in ("mixed", "fp64_partial"):
        if name in runs:
            mx, fp = (runs[name][1], info_p) if name == "mixed" else (info_p, runs[name][1])
            res["mixed_vs_fp64"] = mixed_errors(mx, fp)
            for r in (runs[name][1], info_p):
                r.pop("snap", None)
    res["runs"] = runs
    return res


def mixed_errors(mx, fp):
    """Error of every result of the mixed-precision form against the FP64 form over the
    same series, at its last step: per level ||dA_l||_F / ||A_l||_F and the largest
    relative error of the smoother's diagonal, the solution's largest error over its
    largest entry, the true relative residuals and the iterations of that step."""
    import numpy as np
    a, b = mx["snap"], fp["snap"]
    levels = []
    for l, (am, af) in enumerate(zip(a["A"], b["A"])):
        e = {"level": l, "A_rel_fro": float(np.linalg.norm(am - af) / np.linalg.norm(af))}
        if a["m"][l] is not None:
            e["smoother_rel_max"] = float(np.abs(a["m"][l] - b["m"][l]).max() / np.abs(b["m"][l]).max())
        levels.append(e)
    return {
        "reference": "the FP64 hierarchy on the device, which equals the FP64 oracle's bit for bit on the "
                     "7-point series and within 1e-10 on the 27-point one (parity tests at these sizes)",
        "step": "last timed step", "levels": levels,
        "u_max_err_over_max": float(np.abs(a["u"] - b["u"]).max() / np.abs(b["u"]).max()),
        "rel_res_true": {"mixed": mx["last_rel_res"], "fp64": fp["last_rel_res"]},
        "iters_last_step": {"mixed": mx["iters"][-1], "fp64": fp["iters"][-1]},
        "iters_mean": {"mixed": float(np.mean(mx["iters"])), "fp64": float(np.mean(fp["iters"]))},
    }


def table1(phases):
    """The paper's Table 1 form: share of each phase of the full setup (mean over the full
    setups of the series; host clock between the device synchronisations of the setup)."""
    if not phases:
        return None
    keys = ["aggregation", "prolongator", "symbolic", "galerkin", "smoother", "coarse", "total"]
    mean = {k: sum(p[k] for p in phases) / len(phases) for k in keys}
    tot = mean["total"]
    rows = {"transfer operators (strength, aggregation, P, R = P^T)": mean["aggregation"] + mean["prolongator"],
            "Galerkin operators (symbolic + numeric)": mean["symbolic"] + mean["galerkin"],
            "smoothers": mean["smoother"], "coarsest solver (dense inverse)": mean["coarse"],
            "hierarchy copied to the backend": 0.0}
    other = tot - sum(rows.values())
    out = {k: {"ms": v, "pct": 100.0 * v / tot} for k, v in rows.items()}
    out["other (allocation, vectors, diagonal storage, synchronisation)"] = {"ms": other, "pct": 100.0 * other / tot}
    out["total_ms"] = tot
    out["setups"] = len(phases)
    return out


def table2(ms_partial, info_p, runs):
    """The paper's Table 2 form per strategy: setup and solve ms per step (device events
    around the update and around the solve), iterations, full setups, and speedups over
    no reuse (a full setup every step) in the paper's form (t_base / t - 1) * 100."""
    rows = {"partial reuse": (ms_partial, info_p)}
    names = {"full": "no reuse (full setup every step)", "reuse": "full reuse (miss -> setup and re-solve)",
             "reuse_paper": "full reuse (miss -> setup at the next step)",
             "policy": "partial reuse + full setup every 10th step"}
    for k, v in runs.items():
        if k in names:
            rows[names[k]] = v
    base = rows.get("no reuse (full setup every step)")
    out = {}
    for k, (ms, info) in rows.items():
        r = {"ms_per_step": ms, "setup_ms_per_step": info["setup_ms_per_step"],
             "solve_ms_per_step": info["solve_ms_per_step"],
             "avg_iters": sum(info["iters"]) / len(info["iters"]), "full_setups": info["rebuilds"]}
        if base is not None:
            r["total_speedup_pct"] = (base[0] / ms - 1.0) * 100.0
            bs = base[1]["setup_ms_per_step"]
            r["setup_speedup_pct"] = (bs / info["setup_ms_per_step"] - 1.0) * 100.0 if info["setup_ms_per_step"] else None
        out[k] = r
    return out


def leg_record(res):
    info = res["info_p"]
    rec = {"workload": res["work"], "ms_per_step": res["ms_partial"],
           "setup_ms_per_step": info["setup_ms_per_step"], "solve_ms_per_step": info["solve_ms_per_step"],
           "iters": info["iters"], "converged_all": info["converged"], "rel_res_max": info["rel_res_max"],
           "levels": res["levels"], "level_rows": [d[0] for d in res["dims"]],
           "roofline_dominant": res["roofline_dominant"], "roofline_spmv": res["roofline_spmv"],
           "roofline_rap": res["roofline_rap"], "krylov_spmv_first_iteration": res["krylov_spmv_first_iteration"]}
    for name, (ms, inf) in res.get("runs", {}).items():
        rec[f"{name}_ms_per_step"] = ms
        rec[f"{name}_iters"] = inf["iters"]
    if "mixed_vs_fp64" in res:
        rec["mixed_vs_fp64"] = res["mixed_vs_fp64"]
    return rec


def run_grad(N, K, W, args):
    """Series 4, the differentiable solve: per step the log-coefficients theta_t move (an
    outer optimisation's update), u = A(theta_t)^{-1} f by AMGSolve (assembly of A(theta)
    on the device, the partial update of the hierarchy, PCG), the loss 0.5 ||u - u_t||^2
    and its gradient by the adjoint solve on the same hierarchy and the -lambda (dA/dtheta)
    u scatter.  Every theta_t is uploaded before the timed steps."""
    import numpy as np
    import torch

    from paper_2108_02054_amd import AMG, AMGSolve, logcoef7_assemble
    from workloads import logcoef_inputs, logcoef_theta, pattern_7pt

    dev = torch.device("cuda")

    def T(a):
        return torch.as_tensor(np.ascontiguousarray(a), device=dev)

    _, f, ut, _ = logcoef_inputs(N)
    p, c, _ = pattern_7pt(N)
    thetas = [T(logcoef_theta(N, t)) for t in range(W + K + 1)]
    F, UT = T(f), T(ut)
    amg = AMG(T(p), T(c), logcoef7_assemble(thetas[0], N, N, N), allocator=args.allocator, maxiter=300)
    grid = (N, N, N)
    dom_cls = "cg_pq"

    def step(t):
        theta = thetas[t].clone().requires_grad_(True)
        u = AMGSolve.apply(theta, F, amg, grid)
        loss = 0.5 * torch.sum((u - UT) ** 2)
        loss.backward()
        return theta.grad

    for t in range(1, W + 1):
        step(t)
    amg.trace([dom_cls], level=0, every=TRACE_EVERY)
    amg.trace_read()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ts = time.perf_counter()
    ev[0].record()
    for t in range(W + 1, W + K + 1):
        g = step(t)
    ev[1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - ts) * 1e3 / K
    ms = ev[0].elapsed_time(ev[1]) / K
    kt = amg.trace_read_levels()
    amg.trace([], level=0)
    pq_ms, pq_cnt = kt[0].get(dom_cls, (0.0, 0))
    n = N ** 3
    # the Krylov SpMV (7-point marching form, symmetric read): 4 diagonals, z and p_old read,
    # p_new and q written (the first iteration of each solve reads no p_old)
    nnz = int(p[-1])
    spmv_bytes = pq_cnt * (4.0 * (nnz + n) + 32.0 * n)
    rec = roof("k_m7_cg_pq (Krylov operator SpMV with p = z + beta p and p.q, level 0; forward and adjoint "
               "solves)", pq_ms, pq_cnt, spmv_bytes)
    rec["timing"] = (f"HIP events attached to every {TRACE_EVERY}th launch, on the library's stream, over "
                     f"the {K} timed steps")
    log(f"differentiable solve {N}^3: {ms:.3f} ms/step (events), {wall:.3f} ms/step (host clock); "
        f"gradient norm {float(torch.linalg.norm(g)):.4e}")
    result = {
        "metric": METRIC, "value": ms, "unit": "ms/step", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"differentiable solve on the 7-point log-coefficient Poisson operator, {N}^3 cells "
                               f"(n={n}, nnz={nnz}): theta_t = theta_0 + 0.02 t d (theta_0 ~ N(0, 0.5^2), d ~ "
                               f"N(0, 1)); per step the assembly of A(theta_t), the partial update, PCG to 1e-8, "
                               f"the loss 0.5||u - u_t||^2 and its gradient by the adjoint PCG on the same "
                               f"hierarchy", "grid": N, "n": n, "nnz": nnz, "levels": amg.num_levels,
                   "parallelism": "single GPU"},
        "host_ms_per_step": wall,
        "roofline": rec,
    }
    amg.close()
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: runs on several GPUs "
              f"(row-block sharding of every level) are not implemented.", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return

    from workloads import CONFIGS, rhs_uniform, series_matrix

    cfg_id = args.config
    if cfg_id == 4:
        run_grad(args.n or 128, args.steps, args.warmup, args)
        return
    cfg = CONFIGS[cfg_id]
    N = args.n or cfg["N"]
    K, W = args.steps, args.warmup
    res = run_config(cfg_id, N, K, W, args, compare=not args.no_compare)
    copy_gbs = copy_bandwidth()
    log(f"device copy: {copy_gbs:.0f} GB/s (read + write, 1 GiB, best of 5)")
    info_p = res["info_p"]
    dims = res["dims"]
    n, nnz = res["n"], res["nnz"]
    result = {
        "metric": METRIC,
        "value": res["ms_partial"],
        "unit": "ms/step",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": res["ms_partial"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if res["head_prec"] == 0 else "f32 hierarchy and V-cycle, f64 CG",
        "data": "synthetic",
        "config": {"workload": res["work"],
                   "grid": N, "n": n, "nnz": nnz, "levels": res["levels"], "level_rows": [d[0] for d in dims],
                   "level_nnz": [d[1] for d in dims],
                   "level0_storage": ((f"{res['ndiag']} diagonals, {res['nread']} read per row"
                                       + (f", marching planes of {res['plane']} rows" if res["plane"] else ""))
                                      if res["ndiag"] else "CSR"),
                   "parallelism": "single GPU"},
        "iters_partial": info_p["iters"],
        "converged_all": info_p["converged"],
        "rel_res_max": info_p["rel_res_max"],
        "partial_setup_ms_per_step": info_p["setup_ms_per_step"],
        "partial_solve_ms_per_step": info_p["solve_ms_per_step"],
        "setup_ms_step0": info_p["setup_ms"],
        "step_ms_spread": info_p["step_ms"],
        "copy_gbs_measured": copy_gbs,
        "roofline": res["roofline_dominant"],
        "roofline_spmv": res["roofline_spmv"],
        "roofline_rap": res["roofline_rap"],
        "rap_all_levels": res["rap_all_levels"],
        "krylov_spmv_first_iteration": res["krylov_spmv_first_iteration"],
        "dominant_kernel": res["dom"],
        "kernels_per_step_ms": res["by_kernel"],
        "mall_note": "MI355X has a 256 MB memory-side cache (MALL); at 128^3 part of a kernel's working set can "
                     "stay in it between kernels, so the 128^3 fractions can exceed what HBM alone gives; the "
                     "legs at 192^3 and 160^3 have working sets beyond it",
        "kernels_by_level_ms": res["kernels_by_level"],
        "kernels_all_levels_ms": res["kernels_all_levels_ms"],
        "allocator": args.allocator,
    }
    runs = res.get("runs", {})
    if runs:
        conv = info_p["converged"] and all(bool(v[1]["converged"]) for v in runs.values())
        result["converged_all"] = conv
        if "full" in runs:
            result["full_rebuild_ms_per_step"] = runs["full"][0]
            result["iters_full_rebuild"] = runs["full"][1]["iters"]
            result["total_speedup_vs_full_rebuild_pct"] = (runs["full"][0] / res["ms_partial"] - 1.0) * 100.0
            result["table1_full_setup_phases"] = table1(runs["full"][1]["phases"])
        if "reuse" in runs:
            result["full_reuse_ms_per_step"] = runs["reuse"][0]
            result["iters_full_reuse"] = runs["reuse"][1]["iters"]
            result["full_reuse_rebuilds"] = runs["reuse"][1]["rebuilds"]
        if "mixed" in runs:
            result["mixed_partial_ms_per_step"] = runs["mixed"][0]
            result["iters_mixed"] = runs["mixed"][1]["iters"]
            result["mixed_speedup_vs_fp64_pct"] = (res["ms_partial"] / runs["mixed"][0] - 1.0) * 100.0
        if "policy" in runs:
            result["policy_every_ms_per_step"] = runs["policy"][0]
            result["policy"] = "partial reuse with a full setup every 10th step"
            result["iters_policy"] = runs["policy"][1]["iters"]
            result["policy_full_setups"] = runs["policy"][1]["rebuilds"]
        if "reuse_paper" in runs:
            result["full_reuse_paper_ms_per_step"] = runs["reuse_paper"][0]
            result["iters_full_reuse_paper"] = runs["reuse_paper"][1]["iters"]
            result["full_reuse_paper_full_setups"] = runs["reuse_paper"][1]["rebuilds"]
            result["full_reuse_paper_missed_solves"] = runs["reuse_paper"][1]["missed"]
        if "fp64_partial" in runs:
            result["fp64_partial_ms_per_step"] = runs["fp64_partial"][0]
            result["iters_fp64"] = runs["fp64_partial"][1]["iters"]
            result["mixed_speedup_vs_fp64_pct"] = (runs["fp64_partial"][0] / res["ms_partial"] - 1.0) * 100.0
        result["table2_strategies"] = table2(res["ms_partial"], info_p, runs)
    if "mixed_vs_fp64" in res:
        result["mixed_vs_fp64"] = res["mixed_vs_fp64"]

    # ---------------------------------------------------------------- short legs beyond the MALL
    if cfg_id == 2 and not args.no_legs:
        import torch
        legs = {}
        for lid, prec in ((3, 0), (5, 1)):
            c = CONFIGS[lid]
            log(f"leg: {c['name']}")
            r = run_config(lid, c["N"], args.leg_steps, 1, args, headline_prec=prec, compare=True, legs_mode=True)
            legs[c["name"]] = leg_record(r)
            torch.cuda.empty_cache()
        result["legs"] = legs

    # ---------------------------------------------------------------- CPU oracle sample
    if not args.no_cpu:
        import oracle
        nthr = oracle.num_threads()
        bicg = cfg_id == 6
        amg_params = {k: cfg[k] for k in ("eps_strong", "block_size", "aggregation") if k in cfg}
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
