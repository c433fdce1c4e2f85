"""The C interface: header compiles as C, the library exports every declared entry point,
and argument checks that need no device reject bad input."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amg.h")
LIB = os.path.join(ROOT, "paper_2108_02054_amd", "libamgmi.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(amg_[a-z0-9_]+)\s*\(", src)))


def test_header_compiles_as_c(tmp_path):
    f = tmp_path / "t.c"
    f.write_text('#include "amg.h"\nint main(void){amg_params p; (void)p; return 0;}\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), "-c", str(f),
                    "-o", str(tmp_path / "t.o")], check=True)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libamgmi.so not built (run __graft_entry__.build())")
    L = C.CDLL(LIB)
    names = declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    from paper_2108_02054_amd import EXPORTED
    assert sorted(EXPORTED) == names


def test_host_side_argument_checks():
    """Calls that fail before touching a device."""
    from paper_2108_02054_amd import lib
    from paper_2108_02054_amd.amg import AmgParams
    L = lib()
    assert L.amg_params_default(None) == -1
    p = AmgParams()
    assert L.amg_params_default(C.byref(p)) == 0
    assert p.coarse_enough == 1024 and p.npre == 1 and p.rtol == 1e-8
    ctx = C.c_void_p()
    assert L.amg_setup(C.byref(ctx), 0, 10, None, None, None, None, None) == -1
    assert L.amg_setup(None, 10, 10, None, None, None, None, None) == -1
    assert L.amg_rebuild(None, None, 0) == -1
    assert L.amg_solve(None, None, None, None) == -1
    assert L.amg_destroy(None) == -1
    assert L.amg_logcoef7_assemble(0, 1, 1, None, None, None) == -1
    assert b"invalid" in L.amg_last_error(None) or L.amg_last_error(None) is not None


def test_rebuild_policy_decisions():
    """The rebuild policy's choice (host logic): an every-th full setup, iteration growth
    against the first solve after the last full setup, and a missed convergence under full
    reuse; invalid policies are rejected."""
    import math

    from paper_2108_02054_amd import lib
    from paper_2108_02054_amd.amg import FULL, OPERATOR_ONLY, PARTIAL, AmgError, policy, policy_pick

    every3 = policy(PARTIAL, every=3)
    assert [policy_pick(every3, u, 0, 0, 0) for u in range(6)] == [PARTIAL, PARTIAL, FULL, FULL, FULL, FULL]
    grow = policy(PARTIAL, growth=1.5)
    assert policy_pick(grow, 4, 10, 15, 1) == PARTIAL     # 15 is not more than 1.5 * 10
    assert policy_pick(grow, 4, 10, 16, 1) == FULL
    assert policy_pick(grow, 4, 0, 16, 1) == PARTIAL      # no reference solve yet
    assert policy_pick(grow, 4, 10, 0, 0) == PARTIAL      # no solve since the update
    reuse = policy(OPERATOR_ONLY)
    assert policy_pick(reuse, 7, 30, 100, 0) == FULL      # the last solve missed the limit
    assert policy_pick(reuse, 7, 30, 100, 1) == OPERATOR_ONLY
    assert policy_pick(reuse, 7, 30, 0, 0) == OPERATOR_ONLY
    plain = policy(PARTIAL)
    assert all(policy_pick(plain, u, 10, 99, 0) == PARTIAL for u in range(50))
    for bad in (policy(FULL), policy(PARTIAL, every=-1), policy(PARTIAL, growth=-1.0),
                policy(PARTIAL, growth=math.nan)):
        with pytest.raises(AmgError):
            policy_pick(bad, 0, 0, 0, 0)
    m = C.c_int()
    assert lib().amg_policy_pick(None, 0, 0, 0, 0, C.byref(m)) == -1
    assert lib().amg_policy_pick(C.byref(plain), 0, 0, 0, 0, None) == -1
    assert lib().amg_rebuild_auto(None, None, C.byref(plain), None) == -1


def test_params_struct_layout(tmp_path):
    """The binding's amg_params has the C struct's size and field offsets."""
    from paper_2108_02054_amd.amg import AmgParams
    fields = [f[0] for f in AmgParams._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "amg.h"', 'int main(void){',
           'printf("%zu\\n", sizeof(amg_params));']
    src += [f'printf("%zu\\n", offsetof(amg_params, {f}));' for f in fields]
    src += ['return 0;}']
    f = tmp_path / "layout.c"
    f.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(f), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out[0] == C.sizeof(AmgParams)
    assert out[1:] == [getattr(AmgParams, name).offset for name in fields]


def test_allocator_hooks_must_come_in_pairs():
    """alloc without dealloc is refused before any device work (the arrays are not read)."""
    from paper_2108_02054_amd import lib
    from paper_2108_02054_amd.amg import ALLOC_FN, AmgParams
    L = lib()
    p = AmgParams()
    L.amg_params_default(C.byref(p))
    assert not p.alloc and not p.dealloc
    p.alloc = ALLOC_FN(lambda n, s, u: None)
    ctx = C.c_void_p()
    dummy = C.c_void_p(8)
    assert L.amg_setup(C.byref(ctx), 4, 4, dummy, dummy, dummy, C.byref(p), None) == -1
    assert not ctx.value
