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


def _st(c16=(0, 0, 0), rpb=(8, 256, 32), tail=0, s=8):
    return dict(A_c16=c16[0], P_c16=c16[1], R_c16=c16[2], A_rpb=rpb[0], P_rpb=rpb[1], R_rpb=rpb[2], tail=tail,
                value_bytes=s)


N0, NNZ0, N1, NNZP0 = 128**3, 14_581_760, 189_568, 7_224_490
DIMS = [[N0, NNZ0, N1, NNZP0, 17_000_000], [N1, 6_277_188, 10_086, 744_591, 0], [10_086, 616_480, 559, 35_605, 0],
        [559, 31_125, 37, 1_762, 0], [37, 1_073, 0, 0, 0]]


def test_krylov_spmv_bytes_two_fluid_128():
    b = _bench()
    n, nnz = N0, NNZ0
    st = [_st() for _ in DIMS]
    sym = b.ByteModel(DIMS, st, ndiag=7, nread=4)
    # symmetric diagonal storage: main diagonal and upper entries, 8 B each; z, p_old read,
    # p_new, q written
    assert sym.bytes("cg_pq", 0) == 8 * ((nnz + n) // 2) + 32 * n
    assert abs(sym.bytes("cg_pq", 0) / 1e6 - 133.8) < 0.1
    full = b.ByteModel(DIMS, st, ndiag=7, nread=7)
    assert full.bytes("cg_pq", 0) == 8 * nnz + 32 * n
    csr = b.ByteModel(DIMS, st)
    assert csr.bytes("cg_pq", 0) == 4 * (n + 1) + 12 * nnz + 32 * n


def test_transfer_and_level_bytes():
    b = _bench()
    st = [_st(c16=(1, 1, 0)) for _ in DIMS]
    st[3]["tail"] = st[4]["tail"] = 1
    m = b.ByteModel(DIMS, st, ndiag=7, nread=4)
    n, nc, nnzP = N0, N1, NNZP0
    # prolongation P_0 with two-byte columns (one 4-byte base per 256-row block): P read,
    # u_c gathered once, u read and written
    P = 4 * (n + 1) + 2 * nnzP + 4 * (n // 256) + 8 * nnzP
    assert m.bytes("prolong", 0) == P + 8 * nc + 16 * n
    # restriction R_0 (int32 columns) forming the coarse level's first sweep: R read, r
    # read, f_1 written, m_1 read, u_1 written
    R = 4 * (nc + 1) + 4 * nnzP + 8 * nnzP
    assert m.bytes("restrict", 0) == R + 8 * n + 8 * nc + 16 * nc
    # the restriction into the coarse tail forms no sweep
    assert m.bytes("restrict", 2) == (4 * (559 + 1) + 12 * 35_605) + 8 * 10_086 + 8 * 559
    # level-1 sweep on A_1 with two-byte columns (8-row blocks): m, f, u read, u' written
    n1, nnz1 = N1, 6_277_188
    A1 = 4 * (n1 + 1) + 2 * nnz1 + 4 * (n1 // 8) + 8 * nnz1
    assert m.bytes("jacobi", 1) == A1 + 32 * n1
    assert m.bytes("smooth0_res", 1) == A1 + 24 * n1
    # level 0 in diagonal storage: values only, main and upper diagonals
    a0 = (NNZ0 + N0) // 2
    assert m.bytes("jacobi", 0) == 8 * a0 + 32 * N0
    assert m.bytes("cg_update", 0) == 8 * a0 + 72 * N0
    assert m.bytes("tail", 3) is None


def test_galerkin_bytes():
    b = _bench()
    m = b.ByteModel(DIMS, [_st() for _ in DIMS], ndiag=7, nread=4)
    n, nnzA, nc, nnzP, _ = DIMS[0]
    nnzAc = DIMS[1][1]
    want = (4 * (n + 1) + 12 * nnzA) + (4 * (n + 1) + 12 * nnzP) + (4 * (nc + 1) + 12 * nnzP) + \
        (4 * (nc + 1) + 12 * nnzAc)
    assert m.galerkin(0) == want
    assert abs(want / 1e6 - 442.0) < 0.1


def test_krylov_spmv_bytes_blocks():
    b = _bench()
    B, nodes = 4, 56**3
    n = B * nodes
    nnz = 19_367_936
    dims = [[n, nnz, 64_656, n, 0], [64_656, 3_383_488, 3_752, 0, 0]]
    m = b.ByteModel(dims, [_st(), _st()], block=B)
    # one 4-byte index per 4x4 block and one pointer per node; p read, q written
    assert m.bytes("cg_pq", 0) == 4 * (nodes + 1) + 4 * (nnz // 16) + 8 * nnz + 16 * n
    assert abs(m.bytes("cg_pq", 0) / 1e6 - 171.7) < 0.1


def test_table_forms():
    b = _bench()
    ph = [dict(aggregation=4.0, prolongator=6.0, symbolic=8.0, galerkin=2.0, smoother=0.5, coarse=0.5, total=25.0)]
    t1 = b.table1(ph)
    assert abs(t1["transfer operators (strength, aggregation, P, R = P^T)"]["pct"] - 40.0) < 1e-12
    assert abs(t1["Galerkin operators (symbolic + numeric)"]["pct"] - 40.0) < 1e-12
    assert abs(sum(v["pct"] for k, v in t1.items() if isinstance(v, dict)) - 100.0) < 1e-9
    info = lambda s, v, it: dict(setup_ms_per_step=s, solve_ms_per_step=v, iters=[it], rebuilds=0)  # noqa: E731
    t2 = b.table2(12.0, info(1.0, 11.0, 36), {"full": (46.0, info(35.0, 11.0, 36))})
    assert abs(t2["partial reuse"]["total_speedup_pct"] - (46.0 / 12.0 - 1) * 100) < 1e-9
    assert abs(t2["partial reuse"]["setup_speedup_pct"] - 3400.0) < 1e-9


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
