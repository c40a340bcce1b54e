"""C-ABI contract on the CPU: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before any device
work (no GPU needed for any of these calls)."""
import ctypes as C
import os
import re

import pytest

from paper_1206_6409_amd import gencd as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = ""
    for name in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if name.endswith(".h"):
            src += open(os.path.join(ROOT, "include", name)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gencd_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = G.lib()
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ but not exported"


def test_binding_covers_header():
    assert set(G.exported_symbols()) <= set(declared_functions())


def test_status_strings():
    assert G.status_string(0) == "ok"
    for s in (1, -1, -2, -3, -4, -5, -6, -7, -8):
        assert G.status_string(s) not in ("", "unknown status")
    assert G.status_string(12345) == "unknown status"


def _fake_matrix(n=10, k=5, nnz=7):
    # pointers are never dereferenced: host validation fails first
    return G.Csc(n, k, nnz, 0x1000, 0x2000, 0x3000)


def test_workspace_bytes_host_only():
    X = _fake_matrix(1000, 500, 4000)
    out = C.c_size_t()
    assert G.lib().gencd_workspace_bytes(C.byref(X), None, C.byref(out)) == 0
    small = out.value
    X2 = _fake_matrix(100000, 500000, 5000000)
    assert G.lib().gencd_workspace_bytes(C.byref(X2), None, C.byref(out)) == 0
    assert out.value > small
    bad = _fake_matrix(0, 5, 0)
    assert G.lib().gencd_workspace_bytes(C.byref(bad), None, C.byref(out)) == -1
    p = G.make_params(0, 0.1, group=12)
    assert G.lib().gencd_workspace_bytes(C.byref(X), C.byref(p), C.byref(out)) == -1
    p = G.make_params(0, 0.1, group=16, piece=24)
    assert G.lib().gencd_workspace_bytes(C.byref(X), C.byref(p), C.byref(out)) == -1
    assert G.lib().gencd_workspace_bytes(C.byref(X), None, None) == -1


@pytest.mark.parametrize("field,value", [
    ("loss", 7), ("lam", -1.0), ("lam", float("nan")), ("rule", 9),
    ("select_size", -1), ("max_epochs", -1), ("residual", 3), ("residual", -1),
    ("improve_steps", -1),
])
def test_solve_rejects_bad_params_before_device_work(field, value):
    X = _fake_matrix()
    p = G.make_params(1, 0.1, rule=G.SHOTGUN, select_size=4)
    setattr(p, field, value)
    rc = G.lib().gencd_solve(C.byref(X), C.c_void_p(0x4000), C.byref(p), C.c_void_p(0x5000), None,
                             C.c_void_p(0x6000), 1 << 30, None, None)
    assert rc == -1


def test_solve_rejects_null_and_bad_shapes():
    p = G.make_params(0, 0.1, rule=G.SHOTGUN, select_size=4)
    L = G.lib()
    assert L.gencd_solve(None, C.c_void_p(1), C.byref(p), C.c_void_p(1), None, C.c_void_p(1), 1,
                         None, None) == -1
    X = _fake_matrix(-3, 5, 0)
    assert L.gencd_solve(C.byref(X), C.c_void_p(1), C.byref(p), C.c_void_p(1), None, C.c_void_p(1),
                         1, None, None) == -1
    X = _fake_matrix()
    assert L.gencd_solve(C.byref(X), C.c_void_p(1), C.byref(p), None, None, C.c_void_p(1), 1, None,
                         None) == -1
    # workspace too small is reported before any device work
    assert L.gencd_solve(C.byref(X), C.c_void_p(1), C.byref(p), C.c_void_p(1), None, C.c_void_p(1),
                         16, None, None) == -4
    # coloring without colours
    pc = G.make_params(0, 0.1, rule=G.COLORING)
    assert L.gencd_solve(C.byref(X), C.c_void_p(1), C.byref(pc), C.c_void_p(1), None,
                         C.c_void_p(1), 1 << 30, None, None) == -1
    # thread-greedy without a block size
    pt = G.make_params(0, 0.1, rule=G.THREAD_GREEDY, select_size=8, block=0)
    assert L.gencd_solve(C.byref(X), C.c_void_p(1), C.byref(pt), C.c_void_p(1), None,
                         C.c_void_p(1), 1 << 30, None, None) == -1


def test_select_perm_rejects_bad_sizes():
    assert G.lib().gencd_select_perm(-1, 0, 0, None, None) == -1
    assert G.lib().gencd_select_perm(5, 0, 0, None, None) == -1


def test_rho_host_validation():
    X = _fake_matrix(1000, 500, 4000)
    out = C.c_size_t()
    base = C.c_size_t()
    assert G.lib().gencd_rho_workspace_bytes(C.byref(X), None, C.byref(out)) == 0
    assert G.lib().gencd_workspace_bytes(C.byref(X), None, C.byref(base)) == 0
    assert out.value >= base.value + 2 * 8 * 500  # 1/||X_j|| and the iterate
    # automatic |J| needs the same extra arrays in the solve workspace
    p = G.make_params(1, 0.1, rule=G.SHOTGUN, select_size=0)
    auto = C.c_size_t()
    assert G.lib().gencd_workspace_bytes(C.byref(X), C.byref(p), C.byref(auto)) == 0
    assert auto.value == out.value
    hist = (C.c_double * 4)()
    for iters in (0, 1025, -3):
        assert G.lib().gencd_estimate_rho(C.byref(X), None, iters, hist, None, None, None, 0,
                                          None) == -1
    assert G.lib().gencd_estimate_rho(C.byref(X), None, 4, None, None, None, None, 0, None) == -1
    bad = _fake_matrix(0, 5, 0)
    assert G.lib().gencd_rho_workspace_bytes(C.byref(bad), None, C.byref(out)) == -1


def test_block_rho_host_validation():
    X = _fake_matrix(1000, 500, 4000)
    out = C.c_size_t()
    base = C.c_size_t()
    assert G.lib().gencd_block_rho_workspace_bytes(C.byref(X), None, 8, C.byref(out)) == 0
    assert G.lib().gencd_workspace_bytes(C.byref(X), None, C.byref(base)) == 0
    assert out.value >= base.value + 8 * 1000 * 8  # one product vector per block
    p = G.make_params(1, 0.1, rule=G.BLOCK_SHOTGUN, block=8)
    solve_bytes = C.c_size_t()
    assert G.lib().gencd_workspace_bytes(C.byref(X), C.byref(p), C.byref(solve_bytes)) == 0
    assert solve_bytes.value >= out.value
    for nb in (0, -1, 4097):
        assert G.lib().gencd_block_rho_workspace_bytes(C.byref(X), None, nb, C.byref(out)) == -1
    rho = (C.c_double * 4)()
    ps = (C.c_int64 * 4)()
    for nb, it in ((0, 20), (4, 0), (4, 65)):
        assert G.lib().gencd_estimate_block_rho(C.byref(X), None, nb, it, rho, ps, None, 0, None) == -1
    bad = G.make_params(1, 0.1, rule=G.BLOCK_SHOTGUN, block=0)
    assert G.lib().gencd_solve(C.byref(X), None, C.byref(bad), None, None, None, 0, None, None) == -1


def test_balance_host_validation():
    X = _fake_matrix(1000, 500, 4000)
    out = C.c_size_t()
    assert G.lib().gencd_balance_workspace_bytes(C.byref(X), 40, C.byref(out)) == 0
    assert out.value >= 4 * 4 * 500
    assert G.lib().gencd_balance_workspace_bytes(C.byref(X), 0, C.byref(out)) == -1
    nc = C.c_int32()
    assert G.lib().gencd_balance_colors(C.byref(X), None, 4, 0, None, C.byref(nc), None, 0, None) == -1
    assert G.lib().gencd_balance_colors(C.byref(X), C.c_void_p(0x10), 0, 0, C.c_void_p(0x20),
                                        C.byref(nc), None, 0, None) == -1
