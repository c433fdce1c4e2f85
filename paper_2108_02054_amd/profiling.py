"""Summaries of rocprofv3 output for the committed profiles (host-side text processing).

Two products:
- a per-kernel table from a ``--kernel-trace --stats --output-format csv`` run
  (``*_kernel_stats.csv``), written as text with the command that produced it;
- the HBM traffic of one kernel from two ``--pmc`` runs (``FETCH_SIZE``, then
  ``WRITE_SIZE``, KiB per dispatch), each scaled by what the same counter reads for a
  device copy of known size, stored as JSON together with a hash of the kernel's source
  file so that a reader can tell whether the counters still describe the current kernel.

Usage (after the rocprofv3 runs):
  python -m paper_2108_02054_amd.profiling stats <kernel_stats.csv> <out.txt> --command "..." --workload "..."
  python -m paper_2108_02054_amd.profiling traffic --kernel k_cg_pq --source csrc/kernels_solve.hip \\
      --fetch <dir>/run_counter_collection.csv --write <dir>/run_counter_collection.csv \\
      --copy-fetch <dir> --copy-write <dir> --copy-mib 256 --command "..." --out profiles/x.json \\
      [--part REGEX:GRID[:K/M] ...]   (several kernels per unit, e.g. the Galerkin products of
      level 0; K/M keeps the K-th of every M matching dispatches, in dispatch order, for two
      products that share a kernel and a grid size)
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def short_name(name: str) -> str:
    """Kernel name without its parameter list (template arguments kept)."""
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i].replace("void ", "").strip()
    return name.replace("void ", "").strip()


def stats_table(csv_path: str, top: int = 30) -> list[dict]:
    rows = list(csv.DictReader(open(csv_path)))
    out = []
    for r in rows:
        out.append({
            "name": short_name(r["Name"]),
            "calls": int(r["Calls"]),
            "total_ms": float(r["TotalDurationNs"]) / 1e6,
            "avg_us": float(r["AverageNs"]) / 1e3,
            "min_us": float(r["MinNs"]) / 1e3,
            "max_us": float(r["MaxNs"]) / 1e3,
            "pct": float(r["Percentage"]),
        })
    out.sort(key=lambda d: -d["total_ms"])
    return out[:top]


def write_stats(csv_path: str, out_txt: str, command: str, workload: str, top: int = 30) -> None:
    table = stats_table(csv_path, top)
    lines = [f"workload: {workload}", f"command:  {command}", "",
             f"{'kernel':70s} {'calls':>6s} {'total ms':>9s} {'avg us':>9s} {'min us':>8s} {'max us':>8s} {'%':>6s}"]
    for d in table:
        lines.append(f"{d['name'][:70]:70s} {d['calls']:6d} {d['total_ms']:9.3f} {d['avg_us']:9.1f} "
                     f"{d['min_us']:8.1f} {d['max_us']:8.1f} {d['pct']:6.2f}")
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")


def counter_per_dispatch(csv_path: str, counter: str, kernel_re: str, grid: int | None = None,
                         every: tuple[int, int] | None = None) -> list[float]:
    """Counter value (KiB) of every dispatch whose kernel name matches kernel_re (and whose
    grid size is ``grid`` when given), in dispatch order; with every = (k, m) only the k-th
    of every m such dispatches (their count must be a multiple of m)."""
    rows = []
    for r in csv.DictReader(open(csv_path)):
        if r["Counter_Name"] == counter and re.search(kernel_re, r["Kernel_Name"]):
            if grid is None or int(r["Grid_Size"]) == grid:
                rows.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
    rows.sort()
    vals = [v for _, v in rows]
    if every is not None:
        k, m = every
        if len(vals) % m:
            raise ValueError(f"{len(vals)} dispatches of {kernel_re} (grid {grid}), not a multiple of {m}")
        vals = vals[k::m]
    return vals


def copy_kib(run_dir: str, counter: str) -> float:
    """Counter value of the copy probe's copies (the median of its dispatches)."""
    vals = sorted(counter_per_dispatch(os.path.join(run_dir, "run_counter_collection.csv"), counter, "copyBuffer"))
    if not vals:
        raise ValueError(f"no copy dispatches in {run_dir}")
    big = [v for v in vals if v >= 0.5 * vals[-1]]
    return big[len(big) // 2]


def traffic(kernel: str, source: str, fetch_csv: str, write_csv: str, copy_fetch_dir: str, copy_write_dir: str,
            copy_mib: int, command: str, parts: list[tuple] | None = None) -> dict:
    """HBM bytes per launch of ``kernel``; with ``parts`` (kernel regex, grid size) the
    per-dispatch averages of each part are added (one unit = one dispatch of every part,
    e.g. the two Galerkin products of one level per rebuild)."""
    known = copy_mib * 1024.0 * 1024.0
    f_scale = known / (copy_kib(copy_fetch_dir, "FETCH_SIZE") * 1024.0)
    w_scale = known / (copy_kib(copy_write_dir, "WRITE_SIZE") * 1024.0)
    fb = wb = 0.0
    nd = 0
    for part in (parts or [(kernel, None, None)]):
        rx, grid, every = part
        f = counter_per_dispatch(fetch_csv, "FETCH_SIZE", rx, grid, every)
        w = counter_per_dispatch(write_csv, "WRITE_SIZE", rx, grid, every)
        if not f or not w:
            raise ValueError(f"no dispatches of {rx} (grid {grid})")
        fb += sum(f) / len(f) * 1024.0 * f_scale
        wb += sum(w) / len(w) * 1024.0 * w_scale
        nd += len(f)
    return {
        "kernel": kernel,
        "source": os.path.relpath(source, os.path.dirname(HERE)),
        "source_sha256_16": source_hash(source),
        "dispatches": nd,
        "fetch_bytes_per_launch": fb,
        "write_bytes_per_launch": wb,
        "traffic_bytes_per_launch": fb + wb,
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "copy_probe_mib": copy_mib,
        "command": command,
    }


def load_traffic(json_path: str) -> dict | None:
    """The stored traffic record, or None when it is missing or its kernel source changed."""
    if not os.path.exists(json_path):
        return None
    rec = json.load(open(json_path))
    src = os.path.join(os.path.dirname(HERE), rec["source"])
    if not os.path.exists(src) or source_hash(src) != rec["source_sha256_16"]:
        return None
    return rec


def parse_part(spec: str) -> tuple:
    """REGEX:GRID or REGEX:GRID:K/M -> (regex, grid, (k, m) or None)."""
    head, last = spec.rsplit(":", 1)
    if "/" in last:
        rx, grid = head.rsplit(":", 1)
        k, m = last.split("/")
        return rx, int(grid), (int(k), int(m))
    return head, int(last), None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("out")
    a.add_argument("--command", required=True)
    a.add_argument("--workload", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("--kernel", required=True)
    b.add_argument("--source", required=True)
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--copy-fetch", required=True)
    b.add_argument("--copy-write", required=True)
    b.add_argument("--copy-mib", type=int, required=True)
    b.add_argument("--command", required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--part", action="append", default=[], metavar="REGEX:GRID[:K/M]",
                   help="add the per-dispatch traffic of the dispatches of REGEX with grid size GRID "
                        "(only the K-th of every M of them)")
    args = ap.parse_args()
    if args.cmd == "stats":
        write_stats(args.csv, args.out, args.command, args.workload)
    else:
        parts = [parse_part(p) for p in args.part] or None
        rec = traffic(args.kernel, args.source, args.fetch, args.write, args.copy_fetch, args.copy_write,
                      args.copy_mib, args.command, parts)
        with open(args.out, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
