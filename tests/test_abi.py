"""The C-ABI library loads on the host, exports every declared entry point, and rejects
bad arguments before touching the device (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2509_11133_amd import _binding as B

pytestmark = pytest.mark.cpu

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "phfem.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(phfem_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    L = B.lib()
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTS)
    assert L.phfem_abi_version() == 2


def test_workspace_queries():
    L = B.lib()
    assert L.phfem_connect_workspace(8, 6, 7) > 0
    assert L.phfem_connect_workspace(0, 6, 7) == 0
    assert L.phfem_connect_workspace(10 ** 6, 10 ** 6, 1) > 10 ** 6 * 6 * 20
    assert L.phfem_condense_workspace(20, 50, 100, 1) > 0
    assert L.phfem_condense_workspace(20, 50, 100, 0) > L.phfem_condense_workspace(20, 50, 100, 1)
    # FP64 mode: a Jacobi-scaled FP64 copy of the 6 nF off-diagonal slots; the mixed mode holds an
    # FP32 copy besides (its FP64 polish iterates on the FP64 one) and the polish's FP64 vectors
    assert L.phfem_solve_workspace(100, 200, 0) >= 6 * 200 * 8
    assert L.phfem_solve_workspace(100, 200, 1) - L.phfem_solve_workspace(100, 200, 0) >= 6 * 200 * 4
    assert L.phfem_grad_workspace(100, 200, 0) > L.phfem_solve_workspace(100, 200, 0)
    assert L.phfem_refine_connected_levels_workspace(8, 6, 19, 18, 2) > L.phfem_refine_connected_workspace(72, 114)
    assert L.phfem_refine_connected_levels_workspace(8, 6, 19, 18, 0) == 0
    assert L.phfem_errors_workspace(0) == 0 and L.phfem_errors_workspace(1000) >= 3 * 8 * 4
    assert L.phfem_refine_workspace(0, 0) == 0 and L.phfem_refine_workspace(3, 0) > 0
    assert L.phfem_face_lookup_workspace(0) == 0 and L.phfem_face_lookup_workspace(100) >= 4 * (256 + 100)
    assert L.phfem_condense_batch_workspace(20, 50, 100, 1, 1) == L.phfem_condense_workspace(20, 50, 100, 1)
    # the cross pass keeps the records of up to four fields at once
    assert L.phfem_condense_batch_workspace(20, 50, 100, 1, 3) > L.phfem_condense_workspace(20, 50, 100, 1)
    assert L.phfem_condense_batch_workspace(20, 50, 100, 1, 9) == L.phfem_condense_batch_workspace(20, 50, 100, 1, 4)
    assert L.phfem_condense_batch_workspace(20, 50, 100, 1, 0) == 0
    # Kuhn cube: 6 tets, 19 edges, 18 faces -> Table-1-style counts by the recurrences
    assert B.phfem_refined_sizes(8, 6, 19, 18, 2) == (8 + 19 + 6 + 2 * 19 + 3 * 18 + 6 * 6 + 72, 864,
                                                   2 * (2 * 19 + 3 * 18 + 36) + 3 * (4 * 18 + 96) + 6 * 72,
                                                   4 * (4 * 18 + 96) + 16 * 72)


def test_validation_errors_on_host():
    L = B.lib()
    counts = np.zeros(3, np.int64)
    rc = L.phfem_connect(0, 6, None, 1, None, 0, *([None] * 12), counts.ctypes.data, None)
    assert rc == B.EINVAL and b"positive" in L.phfem_last_error()
    rc = L.phfem_connect(8, 6, 16, 1, 16, 0, *([16] * 4), *([None] * 8), counts.ctypes.data, None)
    assert rc == B.EWORKSPACE
    p = B.params(c=0.0)
    rc = L.phfem_assemble(8, 16, 6, 16, None, None, C.addressof(p), *([None] * 6), None)
    assert rc == B.ESINGULAR
    p = B.params(c=1.0)
    p.quad = 7
    rc = L.phfem_assemble(8, 16, 6, 16, None, None, C.addressof(p), *([None] * 6), None)
    assert rc == B.EINVAL
    st = B.SolveStats()
    p = B.params()
    rc = L.phfem_solve(8, 16, 6, 16, 18, *([16] * 4), None, C.addressof(p), *([16] * 5), 5, 1e-10, 1e-4, 10, 16, 0,
                       16, 16, C.addressof(st), None)
    assert rc == B.EINVAL  # bad mode
    rc = L.phfem_refine(8, 16, 6, 16, 0, *([16] * 3), None, None, None, 0, None, 0, None, None, 0, 16, 16, None, None,
                        None)
    assert rc == B.EINVAL
    # boundary faces need the refine workspace (its error word); triangles the lookup's
    rc = L.phfem_refine(8, 16, 6, 16, 19, *([16] * 3), 16, 16, 16, 2, 16, 0, None, None, 0, 16, 16, 16, None, None)
    assert rc == B.EWORKSPACE
    rc = L.phfem_face_lookup(8, 18, 16, 16, 3, 16, 16, 0, 16, None, None)
    assert rc == B.EWORKSPACE
    rc = L.phfem_face_lookup(8, 18, 16, 16, -1, 16, 16, 1 << 20, 16, None, None)
    assert rc == B.EINVAL
    par, out = (C.c_double * 4)(), (C.c_double * 3)()
    for nq, h in ((0, 0.5), (13, 0.5), (4, 0.0)):  # rule size / mesh size checked before any GPU work
        rc = L.phfem_errors(8, 16, 6, 16, 18, 16, 16, None, C.addressof(p), 16, 16, 4, C.addressof(par), h, nq, 16,
                            1 << 20, C.addressof(out), None)
        assert rc == B.EINVAL


def test_size_limits_on_host():
    """Sizes beyond the int32 index ranges are refused before anything is enqueued (the
    pointers below are never dereferenced)."""
    L = B.lib()
    counts = np.zeros(3, np.int64)
    big = 1 << 27
    rc = L.phfem_connect(8, big, 16, 3, 16, 1 << 40, *([16] * 12), counts.ctypes.data, None)
    assert rc == B.EINVAL and b"too large" in L.phfem_last_error()
    # one refinement of a 2^24-tet mesh: 6 nE' = 6 * 12 * 2^24 > 2^31
    nE = 1 << 24
    rc = L.phfem_refine_connected(4 * nE, 16, nE, 16, 2 * nE, 2 * nE, *([16] * 5), 16, 1 << 40, *([16] * 11),
                                  counts.ctypes.data, None, None)
    assert rc == B.EINVAL and b"index ranges" in L.phfem_last_error()
    rc = L.phfem_refine(1 << 30, 16, nE * 16, 16, nE, *([16] * 3), None, None, None, 0, None, 0, None, None, 0, 16, 16,
                        None, None, None)
    assert rc == B.EINVAL and b"int32" in L.phfem_last_error()
    p = B.params(c=1.0)
    nF = (1 << 31) // 6 + 1  # 6 nF >= 2^31
    rc = L.phfem_condense(8, 16, 6, 16, nF, *([16] * 6), C.addressof(p), 16, 1 << 40, *([16] * 5), None)
    assert rc == B.EINVAL and b"int32" in L.phfem_last_error()
    rc = L.phfem_condense_batch(8, 16, 6, 16, 18, *([16] * 5), 0, 16, C.addressof(p), 16, 1 << 40, None, None, 16,
                                16, 16, None)
    assert rc == B.EINVAL  # nk < 1
    rc = L.phfem_refine_connected_levels(8, 16, 6, 16, 19, 18, *([16] * 5), 17, 16, 1 << 40, *([16] * 11),
                                         counts.ctypes.data, None, None)
    assert rc == B.EINVAL and b"levels" in L.phfem_last_error()
    out = np.zeros(4, np.int64)
    assert L.phfem_refined_sizes(8, 6, 19, 18, -1, out.ctypes.data) == B.EINVAL
    assert L.phfem_refine_connected_levels_workspace(8, 6, 19, 18, 17) == 0


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and says so."""
    import json
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=root, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
