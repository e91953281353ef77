"""phfem_errors_noalloc (the error norms with the library's fixed scratch, for callers that
cannot allocate) against phfem_errors on the same inputs: two calls in a row, the second on
a smaller mesh, each equal to the workspace entry point's sums bit for bit (same kernels,
same reduction order)."""
import numpy as np
import pytest

import oracle as O
from paper_2509_11133_amd import meshes as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_11133_amd import _binding as B  # noqa: E402
from paper_2509_11133_amd import pipeline as P  # noqa: E402

DEV = torch.device("cuda:0")


def solved(L, precision):
    X0, T0 = M.kuhn_cube()
    X, T, c = P.refine_connected_levels(torch.tensor(X0, device=DEV), torch.tensor(T0, device=DEV), L)
    gp = P.params(c=1.0, f=(O.FUN_SIN3, (M.SIN3_AMPLITUDE,)), precision=precision)
    sysm = P.condense(X, T, c, None, gp)
    lam, U, _ = P.solve(X, T, c, sysm, None, gp, mode=precision, tol=1e-10)
    return X, T, c, gp, U, lam


def both(X, T, c, gp, U, lam, h, nq):
    nC, nE = X.shape[1], T.shape[1]
    work = B.workspace(B.lib().phfem_errors_workspace(nE), DEV)
    ref = B.phfem_errors(nC, X, nE, T, c["nF"], c["tet2face"], c["sigma"], None, gp, U, lam, O.FUN_SIN3, (1.0,), h,
                         nq, work)
    got = B.phfem_errors_noalloc(nC, X, nE, T, c["nF"], c["tet2face"], c["sigma"], None, gp, U, lam, O.FUN_SIN3,
                                 (1.0,), h, nq)
    return ref, got


def test_errors_noalloc_matches_workspace_entry():
    for L, prec, nq in ((4, 0, 6), (2, 1, 5)):  # the second call on a smaller mesh
        X, T, c, gp, U, lam = solved(L, prec)
        ref, got = both(X, T, c, gp, U, lam, 2.0 ** -L, nq)
        print(f"L{L}: nE={T.shape[1]} ref={ref} noalloc={got}", flush=True)
        assert all(np.isfinite(ref)) and ref[0] > 0
        assert got == ref


def test_errors_noalloc_refuses_beyond_its_scratch():
    L = B.lib()
    p = B.params(c=1.0)
    par, out = (B.C.c_double * 4)(), (B.C.c_double * 3)()
    rc = L.phfem_errors_noalloc(8, 16, B.ERRORS_NOALLOC_MAX_TETS + 1, 16, 18, 16, 16, None, B.C.addressof(p), 16, 16,
                                4, B.C.addressof(par), 0.5, 4, B.C.addressof(out), None)
    assert rc == B.EINVAL and b"MAX_TETS" in L.phfem_last_error()
