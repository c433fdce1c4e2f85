"""The allocation-free operator entry point (GPU): amg_apply_operator_noalloc, called
through the C ABI, gives the bits of amg_apply_operator on the same input, on two calls in
a row whose second has a smaller input, for the diagonal-storage (7- and 27-point) and CSR
forms; it allocates nothing (counted through the caller's allocator) and leaves the CG's
work vectors alone."""
import ctypes as C

import numpy as np
import pytest
import torch

from tests.dense import random_spd_graph
from tests.gpu_util import T
from workloads import front_moving, lognormal_27pt, two_fluid_7pt

pytestmark = pytest.mark.gpu


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _counting():
    from paper_2108_02054_amd.amg import ALLOC_FN, FREE_FN
    st = {"alloc": 0, "free": 0}

    def a(nbytes, stream, user):
        st["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=0, stream=int(stream or 0))

    def f(ptr, nbytes, stream, user):
        st["free"] += 1
        torch.cuda.caching_allocator_delete(int(ptr))
    return st, (ALLOC_FN(a), FREE_FN(f))


CASES = [
    ("tf7 48^3 then 20^3", lambda: two_fluid_7pt(48, front_moving(48, 3)), lambda: two_fluid_7pt(20, 0.4), {}),
    ("27-point 24^3 then 12^3", lambda: lognormal_27pt(24, 2), lambda: lognormal_27pt(12, 1), {"eps_strong": 0.02}),
    ("csr 3000 then 700", lambda: random_spd_graph(3000, 5, 3), lambda: random_spd_graph(700, 4, 4), {}),
]


@pytest.mark.parametrize("name,big,small,kw", CASES)
def test_noalloc_operator_matches_operator(name, big, small, kw):
    from paper_2108_02054_amd import AMG, lib
    L = lib()
    print(f"case noalloc {name}", flush=True)
    outs = []
    for make in (big, small):
        p, c, v = make()
        st, cb = _counting()
        g = AMG(T(p), T(c), T(v), allocator=cb, coarse_enough=32, **kw)
        n = len(p) - 1
        x = T(np.random.default_rng(n).uniform(-1, 1, n))
        want = torch.empty_like(x)
        assert L.amg_apply_operator(g.ctx, _ptr(x), _ptr(want)) == 0
        # the CG work vectors: a solve before and after gives the same answer
        f = T(np.random.default_rng(n + 1).uniform(-1, 1, n))
        u0, _ = g.solve(f)
        torch.cuda.synchronize()
        n_alloc, n_free = st["alloc"], st["free"]
        y = torch.full_like(x, np.nan)
        assert L.amg_apply_operator_noalloc(g.ctx, _ptr(x), _ptr(y)) == 0, L.amg_last_error(g.ctx)
        torch.cuda.synchronize()
        assert (st["alloc"], st["free"]) == (n_alloc, n_free)
        assert torch.equal(y, want), (name, float((y - want).abs().max()))
        u1, _ = g.solve(f)
        assert torch.equal(u0, u1)
        outs.append(n)
        g.close()
    assert outs[1] < outs[0]


def test_noalloc_argument_errors():
    from paper_2108_02054_amd import AMG, lib
    L = lib()
    p, c, v = two_fluid_7pt(8, 0.5)
    g = AMG(T(p), T(c), T(v), coarse_enough=20)
    x = T(np.ones(len(p) - 1))
    assert L.amg_apply_operator_noalloc(None, _ptr(x), _ptr(x)) == -1
    assert L.amg_apply_operator_noalloc(g.ctx, _ptr(x), _ptr(x)) == -1
    assert L.amg_apply_operator_noalloc(g.ctx, None, _ptr(x)) == -1
    g.close()
