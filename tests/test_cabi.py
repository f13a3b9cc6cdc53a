"""The C-ABI library loads and exports every function include/ntf_admm.h
declares, and the ctypes mirrors of its structs have the C layout.  No GPU
work is done here (nothing is called that touches a device)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ntf_admm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ntf_[a-z0-9_]+)\s*\(", text)))


def _lib_path():
    from paper_1409_2383_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.LIB_PATH


def test_header_declares_the_solver_entry_points():
    names = _declared_functions()
    for n in ("ntf_admm_init", "ntf_admm_step", "ntf_admm_run", "ntf_admm_destroy",
              "ntf_admm_workspace_bytes", "ntf_inner_update", "ntf_gram"):
        assert n in names


def test_library_exports_every_declared_symbol():
    path = _lib_path()
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (ntf_[a-z0-9_]+)", out))
    assert set(_declared_functions()) <= exported


def test_ctypes_bindings_cover_the_header():
    from paper_1409_2383_amd import _lib
    bound = {name for name, _, _ in _lib.SIGNATURES}
    assert set(_declared_functions()) == bound


def _c_sizeof(struct_name):
    src = f'#include "{HEADER}"\n#include <stdio.h>\n#include <stddef.h>\nint main(){{printf("%zu\\n", sizeof({struct_name}));return 0;}}\n'
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.run(["gcc", c, "-o", exe], check=True)
        return int(subprocess.run([exe], capture_output=True, text=True).stdout)


@pytest.mark.parametrize("cname,pyname", [("ntf_problem", "Problem"), ("ntf_opts", "Opts"),
                                          ("ntf_stats", "Stats"), ("ntf_mlp", "Mlp"), ("ntf_constraints", "Constraints"),
                                          ("ntf_batch_tile", "BatchTile"),
                                          ("ntf_batch_info", "BatchInfo"),
                                          ("ntf_sparse_problem", "SparseProblem"),
                                          ("ntf_nway_problem", "NwayProblem"), ("ntf_nway_stats", "NwayStats")])
def test_struct_layouts_match(cname, pyname):
    from paper_1409_2383_amd import _lib
    assert _c_sizeof(cname) == ctypes.sizeof(getattr(_lib, pyname))


def test_status_strings_and_host_validation():
    # pure host paths: no device is touched
    from paper_1409_2383_amd import _lib
    L = _lib.lib()
    assert L.ntf_status_str(0) == b"ok"
    assert L.ntf_status_str(-2) == b"workspace too small"
    pr = _lib.Problem()
    op = _lib.Opts()
    pr.dims[0] = pr.dims[1] = pr.dims[2] = 10
    pr.F = 65                                  # out of range
    op.inner_iters = 1
    op.rho0 = 1.0
    assert L.ntf_admm_workspace_bytes(ctypes.byref(pr), ctypes.byref(op)) == 0
    assert L.ntf_inner_workspace_bytes(10, 0) == 0
    assert L.ntf_gram_workspace_bytes(10, 65) == 0


def test_sparse_host_validation():
    # workspace sizing of a sparse problem is host-only: valid problems get a
    # size, invalid ones 0 (mixed precision is not offered for sparse tensors)
    from paper_1409_2383_amd import _lib
    L = _lib.lib()
    pr = _lib.SparseProblem()
    op = _lib.Opts()
    pr.dims[0], pr.dims[1], pr.dims[2] = 1000, 500, 300
    pr.F = 16
    pr.nnz = 100000
    pr.idx = 4096
    pr.val = 8192
    for n in range(3):
        pr.H[n] = pr.U[n] = 16 * (n + 1)
    op.inner_iters = 1
    op.rho0 = 1.0
    ws = L.ntf_admm_sparse_workspace_bytes(ctypes.byref(pr), ctypes.byref(op))
    # three sorted copies of 16 bytes per non-zero and 24 bytes of sort scratch
    assert ws >= 100000 * (3 * 16 + 24)
    op.precision = 1
    assert L.ntf_admm_sparse_workspace_bytes(ctypes.byref(pr), ctypes.byref(op)) == 0
    op.precision = 0
    pr.dims[0] = 1 << 31
    pr.dims[1] = pr.dims[2] = 1 << 31
    assert L.ntf_admm_sparse_workspace_bytes(ctypes.byref(pr), ctypes.byref(op)) == 0   # key > 64 bits
