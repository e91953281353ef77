"""The library's stated contract on the GPU: bitwise reproducible solves and gradients,
device-side index and volume checks turned into status codes, ENOCONV when a solve stops
above its tolerance, and the boundary-face lookup (the Multiplier's Neumann-face search,
Section 4.4) against the oracle's."""
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


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def kuhn(L):
    X, T = M.kuhn_cube()
    for _ in range(L):
        X, T, _, _ = O.refine(X, T)
    return X, T


def gpu_case(L=3, seed=7, precision=0):
    X, T = kuhn(L)
    Xd, Td = dev(X), dev(T)
    gc = P.connect(Td, X.shape[1])
    kap = dev(M.lognormal_kappa(T.shape[1], 1.0, seed))
    gp = P.params(c=1.0, f=(O.FUN_SIN3, (M.SIN3_AMPLITUDE,)), precision=precision)
    sysm = P.condense(Xd, Td, gc, kap, gp)
    return Xd, Td, gc, kap, gp, sysm


@pytest.mark.parametrize("mode,precision", [(0, 0), (1, 1)])
def test_solve_and_grad_bitwise_reproducible(mode, precision):
    """Two runs of phfem_solve (and of phfem_grad's log-kappa gradient) give the same bits:
    every face residual is the owner's term then the neighbour's, every dot product a fixed
    reduction order."""
    Xd, Td, gc, kap, gp, sysm = gpu_case(3, precision=precision)
    runs = [P.solve(Xd, Td, gc, sysm, kap, gp, mode=mode, tol=1e-11) for _ in range(2)]
    (l1, U1, s1), (l2, U2, s2) = runs
    assert s1 == s2
    assert torch.equal(l1, l2) and torch.equal(U1, U2)
    g = [P.grad(Xd, Td, gc, sysm, kap, gp, U1, l1, U1, mode=mode, tol=1e-11, want_coord=False) for _ in range(2)]
    assert torch.equal(g[0][0], g[1][0]) and g[0][2] == g[1][2]


@pytest.mark.parametrize("mode", [0, 1])
def test_solve_zero_volume_tet(mode):
    """A flattened tet (four coplanar vertices) reaches phfem_solve as EDEGEN."""
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float).T.copy()
    T = np.array([[0, 1, 2, 3]], np.int32).T.copy()
    Xd, Td = dev(X), dev(T)
    gc = P.connect(Td, 4)
    gp = P.params(c=1.0, f=(O.FUN_CONST, (1.0,)), precision=mode)
    sysm = P.condense(Xd, Td, gc, None, gp)
    with pytest.raises(B.PhfemError) as e:
        P.solve(Xd, Td, gc, sysm, None, gp, mode=mode, tol=1e-10, max_iter=50)
    assert e.value.code == B.EDEGEN


@pytest.mark.parametrize("field", ["tet2face", "tetra", "face2tet"])
def test_solve_and_grad_index_checks(field):
    """A face, vertex or slot id out of range in the arrays phfem_solve and phfem_grad index
    is found by the kernels' range checks and returned as EINVAL (no access out of range)."""
    Xd, Td, gc, kap, gp, sysm = gpu_case(1)
    U0 = torch.zeros((4, Td.shape[1]), dtype=torch.float64, device=DEV)
    lam0 = torch.zeros(gc["nF"], dtype=torch.float64, device=DEV)
    bad = dict(gc)
    if field == "tetra":
        Tb = Td.clone()
        Tb[2, 5] = Xd.shape[1]
    else:
        Tb = Td
        a = gc[field].clone()
        a[1, 3] = gc["nF"] if field == "tet2face" else 4 * Td.shape[1] + 8
        bad[field] = a
    with pytest.raises(B.PhfemError) as e:
        P.solve(Xd, Tb, bad, sysm, kap, gp, mode=0, tol=1e-10, max_iter=50)
    assert e.value.code == B.EINVAL and "out of range" in str(e.value)
    with pytest.raises(B.PhfemError) as e:
        P.grad(Xd, Tb, bad, sysm, kap, gp, U0, lam0, U0, mode=0, tol=1e-10, max_iter=50)
    assert e.value.code == B.EINVAL


def test_fp64_solve_below_attainable_accuracy_is_enoconv():
    """The FP64 mode stops its correction solves once one no longer halves the true residual;
    above tol that is ENOCONV (stats filled), never a silent success."""
    Xd, Td, gc, kap, gp, sysm = gpu_case(3)
    lam, U, st = P.solve(Xd, Td, gc, sysm, kap, gp, mode=0, tol=1e-17, max_iter=100000, allow_noconv=True)
    assert not st["converged"]
    assert 0 < st["rel_res"] <= 1e-12 and st["iters"] < 100000 and st["ir_steps"] >= 1
    with pytest.raises(B.PhfemError) as e:
        P.solve(Xd, Td, gc, sysm, kap, gp, mode=0, tol=1e-17, max_iter=100000)
    assert e.value.code == B.ENOCONV


@pytest.mark.parametrize("L", [1, 2, 3])
def test_face_lookup_matches_oracle(L):
    """phfem_face_lookup flags exactly the faces the oracle's node-set search finds for the
    paper's refined Neumann list, and names each triangle's face."""
    X, T, Db, Nb = M.paper_cube()
    for _ in range(L):
        X, T, Db, Nb = O.refine(X, T, Db, Nb)
    oc = O.connect(X.shape[1], T)
    gc = P.connect(dev(T), X.shape[1])
    flags, face_of = P.neumann_flags(gc, dev(Nb), face_of=True)
    assert np.array_equal(host(flags), O.neumann_flags(oc, Nb))
    fo = host(face_of)
    assert np.array_equal(np.sort(oc["faces"][:, fo], axis=0), np.sort(Nb, axis=0))
    assert (oc["face2tet"][1][fo] < 0).all()
    # the Dirichlet list too, in a permuted node order per triangle
    rng = np.random.default_rng(L)
    Dp = np.array([Db[rng.permutation(3), j] for j in range(Db.shape[1])]).T.copy()
    fl2 = host(P.neumann_flags(gc, dev(Dp)))
    assert fl2.sum() == Db.shape[1] and not (fl2 & host(flags)).any()


def test_face_lookup_errors():
    X, T, Db, Nb = M.paper_cube()
    X, T, Db, Nb = O.refine(X, T, Db, Nb)
    gc = P.connect(dev(T), X.shape[1])
    f2t = host(gc["face2tet"])
    F = host(gc["faces"])
    inner = int(np.nonzero(f2t[1] >= 0)[0][0])
    for tris, msg in ((np.concatenate([Nb, F[:, inner:inner + 1]], axis=1), "not a boundary face"),
                      (np.array([[0], [0], [1]], np.int32), "repeated"),
                      (np.array([[0], [1], [X.shape[1]]], np.int32), "out of range")):
        with pytest.raises(B.PhfemError, match=msg):
            P.neumann_flags(gc, dev(tris.astype(np.int32)))
    assert int(P.neumann_flags(gc, dev(np.zeros((3, 0), np.int32))).sum()) == 0
