"""Host-side summaries of rocprofv3 output (paper_2108_02054_amd/profiling.py) on
synthetic CSV files: per-dispatch counter selection (kernel, grid, every k-th of m in
dispatch order), the copy-probe scale and the traffic record."""
import csv
import json
import os

import pytest

from paper_2108_02054_amd import profiling

FIELDS = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(FIELDS, r)))


def test_parse_part():
    assert profiling.parse_part("k_galerkin_pos:1516544") == ("k_galerkin_pos", 1516544, None)
    assert profiling.parse_part("k_galerkin_pos:1516544:0/2") == ("k_galerkin_pos", 1516544, (0, 2))
    assert profiling.parse_part("k<a:b>:8:1/3") == ("k<a:b>", 8, (1, 3))


def test_counter_selection(tmp_path):
    p = str(tmp_path / "c.csv")
    # two products share kernel and grid, alternating per rebuild; dispatch ids out of file order
    rows = [(5, 64, "k_g<x>", "FETCH_SIZE", 20.0), (2, 64, "k_g<x>", "FETCH_SIZE", 10.0),
            (3, 64, "k_g<x>", "FETCH_SIZE", 1.0), (6, 64, "k_g<x>", "FETCH_SIZE", 2.0),
            (4, 32, "k_g<x>", "FETCH_SIZE", 7.0), (1, 64, "k_h", "FETCH_SIZE", 99.0)]
    _write(p, rows)
    assert profiling.counter_per_dispatch(p, "FETCH_SIZE", "k_g", 64) == [10.0, 1.0, 20.0, 2.0]
    assert profiling.counter_per_dispatch(p, "FETCH_SIZE", "k_g", 64, (0, 2)) == [10.0, 20.0]
    assert profiling.counter_per_dispatch(p, "FETCH_SIZE", "k_g", 64, (1, 2)) == [1.0, 2.0]
    assert profiling.counter_per_dispatch(p, "FETCH_SIZE", "k_g", 32) == [7.0]
    with pytest.raises(ValueError):
        profiling.counter_per_dispatch(p, "FETCH_SIZE", "k_g", 64, (0, 3))


def test_traffic_record(tmp_path):
    # copy probe: 256 MiB read reads as 128 MiB of FETCH_SIZE (scale 2), writes as written
    mib = 1024.0
    for c, v in (("FETCH_SIZE", 128 * mib), ("WRITE_SIZE", 256 * mib)):
        d = tmp_path / f"copy_{c}"
        d.mkdir()
        _write(str(d / "run_counter_collection.csv"), [(1, 1, "__amd_rocclr_copyBuffer", c, v)])
    fetch, write = str(tmp_path / "f.csv"), str(tmp_path / "w.csv")
    _write(fetch, [(1, 8, "k_a", "FETCH_SIZE", 100.0), (2, 4, "k_a", "FETCH_SIZE", 50.0),
                   (3, 4, "k_a", "FETCH_SIZE", 70.0)])
    _write(write, [(1, 8, "k_a", "WRITE_SIZE", 10.0), (2, 4, "k_a", "WRITE_SIZE", 5.0),
                   (3, 4, "k_a", "WRITE_SIZE", 6.0)])
    src = os.path.join(os.path.dirname(profiling.HERE), "bench.py")
    rec = profiling.traffic("k_a", src, fetch, write, str(tmp_path / "copy_FETCH_SIZE"),
                            str(tmp_path / "copy_WRITE_SIZE"), 256, "cmd",
                            [("k_a", 8, None), ("k_a", 4, (1, 2))])
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    # one unit = the grid-8 dispatch + the second of every two grid-4 dispatches
    assert rec["fetch_bytes_per_launch"] == pytest.approx((100.0 + 70.0) * 1024 * 2)
    assert rec["write_bytes_per_launch"] == pytest.approx((10.0 + 6.0) * 1024)
    assert rec["dispatches"] == 2
    out = str(tmp_path / "t.json")
    json.dump(rec, open(out, "w"))
    assert profiling.load_traffic(out)["traffic_bytes_per_launch"] == rec["traffic_bytes_per_launch"]
