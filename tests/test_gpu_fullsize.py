"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

Kuhn cube refined 6 times (17,915,904 tets), built exactly as the benchmark builds it
(connect of level 0, then refine_connected_levels), and the Kuhn L5 jittered cube with
lognormal kappa and non-zero Dirichlet data (the gradient workload's mesh).

* Connectivity / refinement: properties that pin the first-appearance numberings at any
  size, checked exhaustively on the device (every tet, edge and face): ids ordered by their
  first position, endpoints / tuples equal to the tets' local entities, owner = lowest tet,
  sigma and face2tet consistent, neighbour symmetry, Euler characteristic, exact volume.
* Condensed system: sampled face rows (interior and boundary) against the oracle's element
  blocks of the two tets sharing the face, FP64 to 1e-12 and mixed to 1e-5 row-relative.
"""
import numpy as np
import pytest

import oracle as O
from paper_2509_11133_amd import meshes as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_11133_amd import pipeline as P  # noqa: E402

from tests.gpu_checks import DEV, check_rows, check_topology, refined_counts  # noqa: E402

KUHN0 = (8, 6, 19, 18, 12)  # level-0 (nC, nE, nEd, nF, nB) of the Kuhn cube


@pytest.fixture(scope="module")
def kuhn6():
    X0, T0 = M.kuhn_cube()
    X, T, conn = P.refine_connected_levels(torch.tensor(X0, device=DEV), torch.tensor(T0, device=DEV), 6)
    torch.cuda.synchronize()
    return X, T, conn


def test_fullsize_counts_topology(kuhn6):
    X, T, c = kuhn6
    check_topology(X, T, c, refined_counts(KUHN0, 6), volume=1.0)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_fullsize_condense_rows(kuhn6, precision, tol):
    X, T, c = kuhn6
    prm = (O.FUN_SIN3, (M.SIN3_AMPLITUDE,))
    sysm = P.condense(X, T, c, None, P.params(f=prm, precision=precision))
    oprm = O.params(c=1.0, kappa=1.0, f=prm)
    check_rows(X, T, c, sysm, None, oprm, tol, np.random.default_rng(6 + precision))
    del sysm


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_jittered_lognormal_L5_condense_rows(precision, tol):
    X0, T0 = M.kuhn_cube()
    Xd, Td, c = P.refine_connected_levels(torch.tensor(X0, device=DEV), torch.tensor(T0, device=DEV), 5)
    Xh = M.jitter_unit_cube(Xd.cpu().numpy(), Td.cpu().numpy(), 0.1)
    X = torch.tensor(Xh, device=DEV)
    kap = torch.tensor(M.lognormal_kappa(Td.shape[1], 1.0), device=DEV)
    f, ud = (O.FUN_SIN3, (2.0,)), (O.FUN_LINEAR, (0.1, 0.2, -0.3, 0.5))
    sysm = P.condense(X, Td, c, kap, P.params(c=0.7, f=f, ud=ud, precision=precision))
    oprm = O.params(c=0.7, kappa=1.0, f=f, ud=ud)
    check_rows(X, Td, c, sysm, kap, oprm, tol, np.random.default_rng(5 + precision))
