"""The algorithmic-byte model behind bench.py's roofline figures, checked against the
counts written out by hand for the headline and block series (CPU only)."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_krylov_spmv_bytes_two_fluid_128():
    b = _bench()
    n, nnz = 128**3, 14_581_760
    dims = [(n, nnz, 189_568, 7_200_000, 17_000_000), (189_568, 6_277_188, 10_086, 0, 0)]
    kb = b.kernel_bytes(dims, 8, ndiag=7, sym=True)
    # symmetric diagonal storage: main diagonal and upper entries, 8 B each; z, p_old read,
    # p_new, q written
    assert kb["cg_pq"] == 8 * ((nnz + n) // 2) + 32 * n
    assert abs(kb["cg_pq"] / 1e6 - 133.8) < 0.1
    full = b.kernel_bytes(dims, 8, ndiag=7, sym=False)
    assert full["cg_pq"] == 8 * nnz + 32 * n
    csr = b.kernel_bytes(dims, 8)
    assert csr["cg_pq"] == 4 * (n + 1) + 12 * nnz + 32 * n


def test_krylov_spmv_bytes_blocks():
    b = _bench()
    B, nodes = 4, 56**3
    n = B * nodes
    nnz = 19_367_936
    dims = [(n, nnz, 64_656, n, 0), (64_656, 3_383_488, 3_752, 0, 0)]
    kb = b.kernel_bytes(dims, 8, block=B)
    # one 4-byte index per 4x4 block and one pointer per node
    assert kb["cg_pq"] == 4 * (nodes + 1) + 4 * (nnz // 16) + 8 * nnz + 32 * n
    assert abs((kb["cg_pq"] - 16 * n) / 1e6 - 171.7) < 0.1


def test_gpus_above_one_exit_with_a_message(capsys, monkeypatch):
    b = _bench()
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    try:
        b.main()
    except SystemExit as e:
        assert e.code == 2
    else:
        raise AssertionError("bench.py --gpus 2 did not exit")
    assert "one GPU" in capsys.readouterr().err
