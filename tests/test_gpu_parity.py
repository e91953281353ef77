"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Connectivity and refinement bit-exact; FP64 local blocks and face system within 1e-12
(row-relative); mixed precision within 1e-5 on matrix entries; u_h within 1e-10 after the
solve (both paths); adjoint gradients within 1e-6 of the oracle's.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2509_11133_amd import meshes as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2509_11133_amd import pipeline as P  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def levels(make, L, with_faces=False):
    out = make()
    X, T = out[0], out[1]
    db = out[2] if with_faces else None
    nb = out[3] if with_faces else None
    for _ in range(L):
        X, T, db, nb = O.refine(X, T, db, nb)
    return X, T, db, nb


MESHES = [(M.kuhn_cube, 0), (M.kuhn_cube, 1), (M.kuhn_cube, 3), (M.fichera, 0), (M.fichera, 2)]


def single_tet():
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float).T.copy()
    return X, np.array([[0, 2, 1, 3]], np.int32).T.copy()


def disjoint_tets(n=700, seed=5):
    """n separate, positively oriented tets: every face is a boundary face owned by its tet
    (4 owned faces per tet, more than the record staging of one workgroup holds)."""
    rng = np.random.default_rng(seed)
    ref = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
    P4 = 0.3 * (ref[None] + 0.2 * rng.random((n, 4, 3))) + 3.0 * rng.random((n, 1, 3))
    X = P4.reshape(-1, 3).T.copy()
    T = np.arange(4 * n, dtype=np.int32).reshape(n, 4).T.copy()
    return X, T


# ------------------------------------------------------------------ connectivity (a1-a3)
@pytest.mark.parametrize("make,L", MESHES + [(single_tet, 0), (single_tet, 2)])
def test_connect_bitexact(make, L):
    X, T, _, _ = levels(make, L)
    oc = O.connect(X.shape[1], T)
    gc = P.connect(dev(T), X.shape[1], faces=True, n2e=True)
    assert gc["nEd"] == oc["nEd"] and gc["nF"] == oc["nF"] and gc["nB"] == oc["nB"]
    for k in ("edges", "tet2edge", "edge_first_tet", "tet_edge_prefix", "faces", "tet2face", "sigma", "face2tet",
              "nbr"):
        assert np.array_equal(host(gc[k]), oc[k]), k
    # Nodes2Edge: row i lists (j, e) for i < j with j ascending
    nEd = oc["nEd"]
    A = sp.csr_matrix((np.arange(nEd) + 1, (oc["edges"][0], oc["edges"][1])), shape=(X.shape[1], X.shape[1]))
    A.sort_indices()
    assert np.array_equal(host(gc["n2e_rowptr"]), A.indptr)
    assert np.array_equal(host(gc["n2e_col"]), A.indices)
    assert np.array_equal(host(gc["n2e_edge"]) + 1, A.data)


@pytest.mark.parametrize("seed", [0, 1])
def test_connect_permuted_relabelled(seed):
    """Random tet order and node labels (orientation kept): still the oracle's numbering."""
    rng = np.random.default_rng(seed)
    X, T, _, _ = levels(M.fichera, 1)
    T = T[:, rng.permutation(T.shape[1])]
    T = rng.permutation(X.shape[1])[T].astype(np.int32)
    oc = O.connect(X.shape[1], T)
    gc = P.connect(dev(T), X.shape[1])
    for k in ("edges", "tet2edge", "faces", "tet2face", "sigma", "face2tet", "nbr"):
        assert np.array_equal(host(gc[k]), oc[k]), k


CONN_KEYS = ("edges", "tet2edge", "edge_first_tet", "tet_edge_prefix", "faces", "tet2face", "sigma", "face2tet", "nbr")


def _permuted(X, T, seed):
    rng = np.random.default_rng(seed)
    T = T[:, rng.permutation(T.shape[1])]
    return X, rng.permutation(X.shape[1])[T].astype(np.int32)


@pytest.mark.parametrize("case", ["kuhn0", "kuhn1_perm", "fichera0_perm", "single2", "paper", "disjoint256",
                                  "disjoint257"])
def test_connect_small_path(case):
    """Meshes of at most 256 tets are connected in one workgroup (when Nodes2Edge is not asked
    for): the same numbering as the oracle and as the sort-based path (which a Nodes2Edge
    request takes), edges-only calls included; 257 tets take the sort-based path."""
    if case == "paper":
        X, T = M.paper_cube()[:2]
    elif case.startswith("disjoint"):
        X, T = disjoint_tets(int(case[8:]))
    else:
        make = {"kuhn": M.kuhn_cube, "fich": M.fichera, "sing": single_tet}[case[:4]]
        X, T, _, _ = levels(make, int(case.split("_")[0][-1]))
        if case.endswith("_perm"):
            X, T = _permuted(X, T, len(case))
    oc = O.connect(X.shape[1], T)
    small = P.connect(dev(T), X.shape[1])
    sort = P.connect(dev(T), X.shape[1], faces=True, n2e=True)
    edges_only = P.connect(dev(T), X.shape[1], faces=False)
    for g in (small, sort):
        assert g["nEd"] == oc["nEd"] and g["nF"] == oc["nF"] and g["nB"] == oc["nB"]
        for k in CONN_KEYS:
            assert np.array_equal(host(g[k]), oc[k]), k
    assert edges_only["nEd"] == oc["nEd"]
    for k in ("edges", "tet2edge", "edge_first_tet", "tet_edge_prefix"):
        assert np.array_equal(host(edges_only[k]), oc[k]), k


def test_connect_paper_mesh_example():
    """Listing 1 mesh on the GPU: 16 Faces rows, tet 5 -> [16 7 12 4] (Section 3.3)."""
    from tests import golden_io as G

    Fg, tet5 = G.faces_listing1()
    X, T, db, nb = M.paper_cube()
    gc = P.connect(dev(T), 8)
    assert np.array_equal(host(gc["faces"]).T + 1, Fg)
    assert np.array_equal(host(gc["tet2face"])[:, 4] + 1, tet5)


@pytest.mark.parametrize("n2e", [False, True])  # the one-workgroup path and the sort-based one
def test_connect_errors(n2e):
    X, T = M.kuhn_cube()
    flip = T.copy()
    flip[[2, 3], 1] = flip[[3, 2], 1]
    with pytest.raises(P.PhfemError) as e:
        P.connect(dev(flip), 8, n2e=n2e)
    assert e.value.code == P.B.EORIENT
    three = np.array([[0, 1, 2, 3], [0, 2, 1, 4], [0, 1, 2, 5]], np.int32).T.copy()  # one face in three tets
    with pytest.raises(P.PhfemError) as e:
        P.connect(dev(three), 6, n2e=n2e)
    assert e.value.code == P.B.EORIENT
    bad = T.copy()
    bad[0, 3] = 8
    with pytest.raises(P.PhfemError) as e:
        P.connect(dev(bad), 8, n2e=n2e)
    assert e.value.code == P.B.EINVAL
    rep = T.copy()
    rep[1, 2] = rep[0, 2]  # a repeated node in one tet
    with pytest.raises(P.PhfemError) as e:
        P.connect(dev(rep), 8, n2e=n2e)
    assert e.value.code == P.B.EINVAL


# ------------------------------------------------------------------ refinement (a4)
@pytest.mark.parametrize("make,L", [(M.kuhn_cube, 3), (M.fichera, 2), (single_tet, 3)])
def test_refine_bitexact(make, L):
    X, T = make()[:2]
    Xd, Td = dev(X), dev(T)
    for _ in range(L):
        X, T, _, _ = O.refine(X, T)
        conn = P.connect(Td, Xd.shape[1], faces=False)
        Xd, Td, _, _ = P.refine(Xd, Td, conn)
        assert np.array_equal(host(Td), T)
        assert np.array_equal(host(Xd), X)  # bitwise


def test_refine_worked_example_and_faces():
    """Section 3.4 example through the GPU, and refineFaces on Listing 1's Db/Nb."""
    from tests import golden_io as G

    Tg, Cg = G.refine_example()
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float).T.copy()
    T = np.array([[0, 2, 1, 3]], np.int32).T.copy()
    conn = P.connect(dev(T), 4, faces=False)
    Xo, To, _, _ = P.refine(dev(X), dev(T), conn)
    assert np.array_equal(host(To).T + 1, Tg) and np.array_equal(host(Xo).T, Cg)
    X, T, db, nb = M.paper_cube()
    Xd, Td, dbd, nbd = dev(X), dev(T), dev(db), dev(nb)
    for _ in range(3):
        X, T, db, nb = O.refine(X, T, db, nb)
        conn = P.connect(Td, Xd.shape[1], faces=False, n2e=True)
        Xd, Td, dbd, nbd = P.refine(Xd, Td, conn, dbd, nbd)
        for a, b in ((Xd, X), (Td, T), (dbd, db), (nbd, nb)):
            assert np.array_equal(host(a), b)


# ------------------------------------------------------------------ local blocks (a5, a6)
def problem(kind, nE, seed=3):
    if kind == "sin3":
        return dict(c=1.0, kappa=None, f=(O.FUN_SIN3, (M.SIN3_AMPLITUDE,)), ud=(O.FUN_ZERO, ()), quad=0)
    if kind == "rough":
        return dict(c=0.7, kappa=M.lognormal_kappa(nE, 1.0, seed), f=(O.FUN_SIN3, (2.0,)),
                    ud=(O.FUN_LINEAR, (0.1, 0.2, -0.3, 0.5)), quad=0)
    if kind == "p1":
        return dict(c=1.3, kappa=M.lognormal_kappa(nE, 0.5, seed), f=(O.FUN_X2Y2Z2_LOAD, (1.0, 1.3)),
                    ud=(O.FUN_X2Y2Z2, (1.0,)), quad=1)
    raise ValueError(kind)


def prm_pair(pb, precision=0):
    kc = 1.0
    op = O.params(c=pb["c"], kappa=kc, f=pb["f"], ud=pb["ud"], quad=pb["quad"])
    gp = P.params(c=pb["c"], kappa=kc, f=pb["f"], ud=pb["ud"], quad=pb["quad"], precision=precision)
    return op, gp


def rowrel(a, b):
    """max_ij |a_ij - b_ij| / max_j |b_ij| over rows (entries as [rows, n] blocks)."""
    scale = np.abs(b).max(axis=0)
    scale[scale == 0] = 1
    return (np.abs(a - b).max(axis=0) / scale).max()


def jittered(L, seed=1):
    X, T, _, _ = levels(M.kuhn_cube, L)
    return M.jitter_unit_cube(X, T, 0.1, seed=seed) if L else X, T


@pytest.mark.parametrize("kind", ["sin3", "rough", "p1"])
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_assemble_parity(kind, precision, tol):
    X, T = jittered(2)
    oc = O.connect(X.shape[1], T)
    pb = problem(kind, T.shape[1])
    op, gp = prm_pair(pb, precision)
    ref = O.local(X, T, oc["sigma"], pb["kappa"], op)
    kap = None if pb["kappa"] is None else dev(pb["kappa"])
    got = P.assemble(dev(X), dev(T), dev(oc["sigma"]), kap, gp)
    assert np.abs(host(got["vol"]) - ref["vol"]).max() <= 1e-15 * ref["vol"].max()
    for k in ("K", "d", "B", "S", "r"):
        g, r = host(got[k]), ref[k]
        nb = 4 if k in ("K", "S") else 1
        err = max(rowrel(g[i * nb:(i + 1) * nb], r[i * nb:(i + 1) * nb]) for i in range(g.shape[0] // nb))
        assert err <= tol, (k, err)


def full_csr(sysm, nF):
    rp, col, val, diag = (host(sysm[k]) for k in ("rowptr", "col", "val", "diag"))
    A = sp.csr_matrix((val, col, rp), shape=(nF, nF)) + sp.diags(diag)
    return A.tocsr()


@pytest.mark.parametrize("make,L,kind", [(M.kuhn_cube, 1, "sin3"), (M.kuhn_cube, 3, "sin3"), (M.fichera, 1, "rough"),
                                         (M.kuhn_cube, 2, "p1"), (disjoint_tets, 0, "rough")])
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_condense_parity(make, L, kind, precision, tol):
    X, T, _, _ = levels(make, L)
    oc = O.connect(X.shape[1], T)
    pb = problem(kind, T.shape[1])
    op, gp = prm_pair(pb, precision)
    A, rhs = O.condense(X, T, oc, pb["kappa"], op)
    gc = P.connect(dev(T), X.shape[1])
    kap = None if pb["kappa"] is None else dev(pb["kappa"])
    sysm = P.condense(dev(X), dev(T), gc, kap, gp)
    G = full_csr(sysm, oc["nF"])
    # pattern: 6 slots per row; the oracle's off-diagonals ascending, then (boundary rows) 3
    # explicit zeros in the row's own column
    nF = oc["nF"]
    assert sysm["nnz"] == 6 * nF and np.array_equal(host(sysm["rowptr"]), 6 * np.arange(nF + 1))
    Ad = (A - sp.diags(A.diagonal())).tocsr()
    Ad.eliminate_zeros()
    Ad.sort_indices()
    gcol, gval = host(sysm["col"]).reshape(nF, 6), host(sysm["val"]).reshape(nF, 6)
    cnt = np.diff(Ad.indptr)
    assert set(np.unique(cnt)) <= {3, 6} and (cnt == 3).sum() == oc["nB"]
    want = np.repeat(np.arange(nF)[:, None], 6, axis=1)
    for k in range(6):
        m = cnt > k
        want[m, k] = Ad.indices[Ad.indptr[:-1][m] + k]
    assert np.array_equal(gcol, want)
    assert np.all(gval[cnt == 3, 3:] == 0.0)
    D = abs(G - A).tocsr()
    rowmax = np.asarray(abs(A).max(axis=1).todense()).ravel()
    assert (np.asarray(D.max(axis=1).todense()).ravel() / rowmax).max() <= tol
    r = host(sysm["rhs"])
    assert np.abs(r - rhs).max() <= tol * np.abs(rhs).max()


def test_condense_deterministic():
    X, T, _, _ = levels(M.kuhn_cube, 3)
    gc = P.connect(dev(T), X.shape[1])
    gp = P.params(f=(O.FUN_SIN3, (M.SIN3_AMPLITUDE,)))
    a = P.condense(dev(X), dev(T), gc, None, gp)
    b = P.condense(dev(X), dev(T), gc, None, gp)
    for k in ("val", "diag", "rhs", "col"):
        assert torch.equal(a[k], b[k]), k


# ------------------------------------------------------------------ solve + recovery (a8, a9)
@pytest.mark.parametrize("make,L,kind", [(M.kuhn_cube, 2, "sin3"), (M.kuhn_cube, 3, "sin3"), (M.fichera, 1, "rough")])
@pytest.mark.parametrize("mode,precision", [(0, 0), (1, 1)])
def test_solve_parity(make, L, kind, mode, precision):
    X, T, _, _ = levels(make, L)
    pb = problem(kind, T.shape[1])
    op, gp = prm_pair(pb, precision)
    oc, A, rhs, olam, oU, _ = O.solve(X, T, pb["kappa"], op, tol=1e-14)
    gc = P.connect(dev(T), X.shape[1])
    kap = None if pb["kappa"] is None else dev(pb["kappa"])
    Xd, Td = dev(X), dev(T)
    sysm = P.condense(Xd, Td, gc, kap, gp)
    lam, U, st = P.solve(Xd, Td, gc, sysm, kap, gp, mode=mode, tol=1e-13, inner_tol=0.7, allow_noconv=True)
    assert st["rel_res"] <= 1e-12, st
    assert np.abs(host(U) - oU).max() <= 1e-10 * np.abs(oU).max(), st
    assert np.abs(host(lam) - olam).max() <= 1e-9 * np.abs(olam).max(), st


def test_linear_solution_gpu():
    """u = a + b.x, P1-interpolated load: U = nodal values to 1e-12 on the GPU path."""
    a = (0.3, 1.1, -0.7, 0.4)
    X, T, _, _ = levels(M.kuhn_cube, 2)
    gp = P.params(c=1.3, kappa=2.5, f=(O.FUN_LINEAR, tuple(1.3 * v for v in a)), ud=(O.FUN_LINEAR, a), quad=1)
    Xd, Td = dev(X), dev(T)
    gc = P.connect(Td, X.shape[1])
    sysm = P.condense(Xd, Td, gc, None, gp)
    lam, U, st = P.solve(Xd, Td, gc, sysm, None, gp, tol=1e-15, max_iter=20000, allow_noconv=True)
    nod = a[0] + a[1] * X[0] + a[2] * X[1] + a[3] * X[2]
    assert np.abs(host(U) - nod[T]).max() <= 1e-12


# ------------------------------------------------------------------ adjoint (a10)
@pytest.mark.parametrize("mode,precision", [(0, 0), (1, 1)])
def test_grad_parity(mode, precision):
    X, T = jittered(1, seed=11)
    pb = problem("rough", T.shape[1], seed=13)
    op, gp = prm_pair(pb, precision)
    oc, A, rhs, olam, oU, _ = O.solve(X, T, pb["kappa"], op, tol=1e-14)
    Ut = np.random.default_rng(17).standard_normal(oU.shape)
    og = O.adjoint(X, T, oc, pb["kappa"], op, oU, olam, oU - Ut, tol=1e-14)
    Xd, Td, kap = dev(X), dev(T), dev(pb["kappa"])
    gc = P.connect(Td, X.shape[1])
    sysm = P.condense(Xd, Td, gc, kap, gp)
    lam, U, st = P.solve(Xd, Td, gc, sysm, kap, gp, mode=mode, tol=1e-13, inner_tol=0.7, allow_noconv=True)
    dlogk, dX, st2 = P.grad(Xd, Td, gc, sysm, kap, gp, U, lam, U - dev(Ut), mode=mode, tol=1e-13, inner_tol=0.7,
                            allow_noconv=True)
    assert st["rel_res"] <= 1e-12 and st2["rel_res"] <= 1e-12, (st, st2)
    assert np.abs(host(dlogk) - og["dlogk"]).max() <= 1e-6 * np.abs(og["dlogk"]).max()
    assert np.abs(host(dX) - og["dX"]).max() <= 1e-6 * np.abs(og["dX"]).max()


def test_autograd_function():
    """torch.autograd through PrimalHybridSolve equals phfem_grad's VJP."""
    X, T = jittered(1, seed=5)
    kap = M.lognormal_kappa(T.shape[1], 1.0, 3)
    Xd, Td = dev(X), dev(T)
    gc = P.connect(Td, X.shape[1])
    gp = P.params(c=1.0, f=(O.FUN_SIN3, (M.SIN3_AMPLITUDE,)))
    logk = dev(np.log(kap)).requires_grad_(True)
    Xr = Xd.clone().requires_grad_(True)
    U = P.PrimalHybridSolve.apply(logk, Xr, Td, gc, gp, 0, 1e-12)
    Ut = torch.zeros_like(U)
    J = 0.5 * ((U - Ut) ** 2).sum()
    J.backward()
    oc = O.connect(X.shape[1], T)
    op = O.params(c=1.0, f=(O.FUN_SIN3, (M.SIN3_AMPLITUDE,)))
    _, _, _, olam, oU, _ = O.solve(X, T, kap, op, tol=1e-14)
    og = O.adjoint(X, T, oc, kap, op, oU, olam, oU, tol=1e-14)
    assert np.abs(host(logk.grad) - og["dlogk"]).max() <= 1e-6 * np.abs(og["dlogk"]).max()
    assert np.abs(host(Xr.grad) - og["dX"]).max() <= 1e-6 * np.abs(og["dX"]).max()


# ------------------------------------------------------------------ refinement with connectivity
def _perm_relabel(X, T, seed):
    rng = np.random.default_rng(seed)
    T = T[:, rng.permutation(T.shape[1])]
    perm = rng.permutation(X.shape[1])
    X2 = np.zeros_like(X)
    X2[:, perm] = X
    return X2, perm[T].astype(np.int32)


@pytest.mark.parametrize("case", ["kuhn", "fichera", "paper", "single_neg", "fichera_perm", "kuhn1_perm"])
def test_refine_connected_bitexact(case):
    """phfem_refine_connected = phfem_refine + oracle connect of the refined mesh, bit for bit,
    over two levels (the second consumes the first's derived connectivity)."""
    if case == "kuhn":
        X, T = M.kuhn_cube()
    elif case == "fichera":
        X, T = M.fichera()
    elif case == "paper":
        X, T = M.paper_cube()[:2]
    elif case == "single_neg":
        X, T = single_tet()
    elif case == "fichera_perm":
        X, T = _perm_relabel(*M.fichera(), seed=3)
    else:
        X, T, _, _ = O.refine(*M.kuhn_cube())
        X, T = _perm_relabel(X, T, seed=4)
    Xd, Td = dev(X), dev(T)
    conn = P.connect(Td, X.shape[1])
    for _ in range(2):
        X, T, _, _ = O.refine(X, T)
        Xd, Td, conn = P.refine_connected(Xd, Td, conn)
        assert np.array_equal(host(Td), T) and np.array_equal(host(Xd), X)
        oc = O.connect(X.shape[1], T)
        assert conn["nEd"] == oc["nEd"] and conn["nF"] == oc["nF"] and conn["nB"] == oc["nB"]
        for k in ("edges", "tet2edge", "edge_first_tet", "tet_edge_prefix", "faces", "tet2face", "sigma",
                  "face2tet", "nbr"):
            assert np.array_equal(host(conn[k]), oc[k]), k


def test_refine_connected_input_check():
    """An edge id outside [0, nEd) is caught (clamped in the kernels, reported): EINVAL when
    synchronous, status bit 1 when checked on the device; a valid level leaves status 0."""
    from paper_2509_11133_amd import _binding as B
    X, T, _, _ = levels(M.kuhn_cube, 1)
    Xd, Td = dev(X), dev(T)
    conn = P.connect(Td, X.shape[1], faces=True)
    bad = dict(conn)
    t2e = conn["tet2edge"].clone()
    t2e[2, 5] = conn["nEd"] + 7
    bad["tet2edge"] = t2e
    with pytest.raises(B.PhfemError):
        P.refine_connected(Xd, Td, bad)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    P.refine_connected(Xd, Td, bad, st)
    assert int(st.item()) & 1
    with pytest.raises(B.PhfemError):
        P.check_status(st)
    st.zero_()
    P.refine_connected(Xd, Td, conn, st)
    assert int(st.item()) == 0


def test_refine_connected_count_check():
    """Input ids all in range but not a consistent numbering: an interior face whose second tet
    claims no neighbour there, so that both tets take the face's children and the refined totals
    exceed the recurrences 2nEd+3nF+6nE, 4nF+16nE.  EINVAL when synchronous, status bit 2 (and
    only it) when checked on the device; the untouched input still passes."""
    from paper_2509_11133_amd import _binding as B
    X, T, _, _ = levels(M.kuhn_cube, 1)
    Xd, Td = dev(X), dev(T)
    conn = P.connect(Td, X.shape[1], faces=True)
    f2t = host(conn["face2tet"])
    f = int(np.nonzero(f2t[1] >= 0)[0][3])  # an interior face
    q1 = int(f2t[1, f])
    nb = conn["nbr"].clone()
    nb[q1 & 3, q1 >> 2] = -1  # its second tet (the higher index) loses its neighbour there
    bad = dict(conn)
    bad["nbr"] = nb
    print("face", f, "second slot", q1, flush=True)
    with pytest.raises(B.PhfemError) as e:
        P.refine_connected(Xd, Td, bad)
    assert e.value.code == B.EINVAL and "first-appearance" in str(e.value)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    P.refine_connected(Xd, Td, bad, st)
    assert int(st.item()) == 2
    st.zero_()
    P.refine_connected(Xd, Td, conn, st)
    assert int(st.item()) == 0


@pytest.mark.parametrize("make,L", [(M.kuhn_cube, 1), (M.kuhn_cube, 4), (M.fichera, 3), (single_tet, 3)])
def test_refine_connected_levels_equals_chained(make, L):
    """One multi-level call = L chained single-level calls, bit for bit."""
    X, T = make()[:2]
    Xd, Td = dev(X), dev(T)
    conn0 = P.connect(Td, X.shape[1], faces=True)
    Xa, Ta, ca = Xd, Td, conn0
    for _ in range(L):
        Xa, Ta, ca = P.refine_connected(Xa, Ta, ca)
    Xb, Tb, cb = P.refine_connected_levels(Xd, Td, L, conn=conn0)
    assert torch.equal(Xa, Xb) and torch.equal(Ta, Tb)
    for k in ("nEd", "nF", "nB"):
        assert ca[k] == cb[k], k
    for k in ("edges", "tet2edge", "edge_first_tet", "tet_edge_prefix", "faces", "tet2face", "sigma", "face2tet",
              "nbr"):
        assert torch.equal(ca[k], cb[k]), k
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    Xc, Tc, cc = P.refine_connected_levels(Xd, Td, L, conn=conn0, status=st)
    assert int(st.item()) == 0 and torch.equal(cc["face2tet"], cb["face2tet"])


def test_refine_connected_matches_sort_connect_L5():
    """At 1.49M tets (Kuhn, 5 levels): the derived connectivity equals phfem_connect of the
    same refined mesh, bit for bit, through the node buckets and through the radix sort (with
    Nodes2Edge as well: its rows against the derived edges' node pairs)."""
    X, T = M.kuhn_cube()
    Xd, Td, conn = P.refine_connected_levels(dev(X), dev(T), 5)
    for radix in (False, True):
        ref = P.connect(Td, Xd.shape[1], n2e=True, radix=radix)
        for k in ("edges", "tet2edge", "edge_first_tet", "tet_edge_prefix", "faces", "tet2face", "sigma",
                  "face2tet", "nbr"):
            assert torch.equal(conn[k], ref[k]), (radix, k)
        e = conn["edges"].cpu().numpy()
        rp, cl, ed = (ref[k].cpu().numpy() for k in ("n2e_rowptr", "n2e_col", "n2e_edge"))
        rows = np.repeat(np.arange(Xd.shape[1]), np.diff(rp))
        assert rp[-1] == conn["nEd"] and np.array_equal(np.sort(ed), np.arange(conn["nEd"])), radix
        assert np.array_equal(e[0][ed], rows) and np.array_equal(e[1][ed], cl), radix
        assert np.all(np.diff(cl)[np.diff(rows) == 0] > 0), radix  # ascending within each row
        del ref


# ------------------------------------------------------------------ mixed Dirichlet/Neumann (paper's example)
def paper_levels(L):
    X, T, Db, Nb = M.paper_cube()
    for _ in range(L):
        X, T, Db, Nb = O.refine(X, T, Db, Nb)
    return X, T, Db, Nb


EXAMPLE = dict(c=1.0, f=(O.FUN_X2Y2Z2_LOAD, (1.0, 1.0)), ud=(O.FUN_X2Y2Z2, (1.0,)), g=(O.FUN_X2Y2Z2, (1.0,)))


def owner_flux(X, T, conn, kap, gpar):
    """kappa grad(x^2 y^2 z^2 * p0) . nu (owner outward) at every face centroid"""
    f2t = np.asarray(conn["face2tet"])
    F = np.asarray(conn["faces"])
    local = [(0, 1, 2), (0, 2, 3), (0, 3, 1), (3, 2, 1)]
    out = np.zeros(F.shape[1])
    for f in range(F.shape[1]):
        t, k = divmod(int(f2t[0, f]), 4)
        a, b, c = (X[:, T[v, t]] for v in local[k])
        n = np.cross(b - a, c - a)
        n = (-n if n @ (X[:, T[6 - sum(local[k]), t]] - a) > 0 else n) / np.linalg.norm(n)
        x, y, z = (a + b + c) / 3
        gu = 2 * gpar * np.array([x * y * y * z * z, x * x * y * z * z, x * x * y * y * z])
        out[f] = kap * gu @ n
    return out


@pytest.mark.parametrize("L", [1, 2, 3])
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_neumann_condense_parity(L, precision, tol):
    """Listing 1's cube with its Db / Nb faces and the paper's example data: the rows of the
    faces left in the system equal the oracle's reduced system (RFaces) with LN in the load;
    Neumann rows are lambda_F = g(Ct_F) and their columns are zero."""
    X, T, Db, Nb = paper_levels(L)
    oc = O.connect(X.shape[1], T)
    nm = O.neumann_flags(oc, Nb)
    op = O.params(**EXAMPLE)
    A, rhs, rf = O.condense(X, T, oc, None, op, nm)
    gc = P.connect(dev(T), X.shape[1])
    nmd = P.neumann_flags(gc, dev(Nb))
    assert np.array_equal(host(nmd), nm)
    gp = P.params(**EXAMPLE, precision=precision, neumann=nmd)
    sysm = P.condense(dev(X), dev(T), gc, None, gp)
    G = full_csr(sysm, oc["nF"])
    free = np.flatnonzero(nm == 0)
    Gf = G[free][:, free]
    D = abs(Gf - A).tocsr()
    rowmax = np.asarray(abs(A).max(axis=1).todense()).ravel()
    assert (np.asarray(D.max(axis=1).todense()).ravel() / rowmax).max() <= tol
    r = host(sysm["rhs"])
    assert np.abs(r[free] - rhs).max() <= tol * np.abs(rhs).max()
    neu = np.flatnonzero(nm)
    assert np.all(G[free][:, neu].toarray() == 0) and np.all(G[neu][:, free].toarray() == 0)
    assert np.abs(G[neu][:, neu].toarray() - np.eye(len(neu))).max() == 0
    g = owner_flux(X, T, oc, 1.0, 1.0)
    assert np.abs(r[neu] - g[neu]).max() <= 1e-12 * np.abs(g).max() + (tol if precision else 0) * np.abs(g).max()


@pytest.mark.parametrize("mode,precision", [(0, 0), (1, 1)])
def test_neumann_solve_parity(mode, precision):
    """u_h of the paper's example with mixed boundaries against the oracle (1e-10), lambda on
    the faces left in the system (1e-9), lambda = g on the Neumann faces."""
    X, T, Db, Nb = paper_levels(3)
    op = O.params(**EXAMPLE)
    oc, A, rhs, lam, U, it = O.solve(X, T, None, op, tol=1e-14, neumann_faces=Nb)
    nm = O.neumann_flags(oc, Nb)
    gc = P.connect(dev(T), X.shape[1])
    gp = P.params(**EXAMPLE, precision=precision, neumann=P.neumann_flags(gc, dev(Nb)))
    sysm = P.condense(dev(X), dev(T), gc, None, gp)
    glam, gU, st = P.solve(dev(X), dev(T), gc, sysm, None, gp, mode=mode, tol=1e-13, allow_noconv=True)
    assert st["rel_res"] <= 1e-12, st
    assert np.abs(host(gU) - U).max() <= 1e-10 * np.abs(U).max()
    gl = host(glam)
    assert np.abs(gl - lam)[nm == 0].max() <= 1e-9 * np.abs(lam).max()
    g = owner_flux(X, T, oc, 1.0, 1.0)
    assert np.abs(gl - g)[nm == 1].max() <= 1e-9 * np.abs(g).max()


def test_neumann_linear_exact_gpu():
    """Linear exact solution with Listing 1's Db / Nb and the P1 load: U = nodal values."""
    X, T, Db, Nb = paper_levels(2)
    a = (0.3, 0.5, -0.2, 0.7)
    kap, cc = 0.8, 1.3
    par = dict(c=cc, kappa=kap, f=(O.FUN_LINEAR, tuple(cc * v for v in a)), ud=(O.FUN_LINEAR, a),
               g=(O.FUN_LINEAR, a), quad=1)
    gc = P.connect(dev(T), X.shape[1])
    gp = P.params(**par, neumann=P.neumann_flags(gc, dev(Nb)))
    sysm = P.condense(dev(X), dev(T), gc, None, gp)
    glam, gU, st = P.solve(dev(X), dev(T), gc, sysm, None, gp, mode=0, tol=1e-14, allow_noconv=True)
    u = a[0] + a[1] * X[0] + a[2] * X[1] + a[3] * X[2]
    assert np.abs(host(gU) - u[T]).max() <= 1e-12


def test_neumann_grad_rejected():
    X, T, Db, Nb = paper_levels(1)
    gc = P.connect(dev(T), X.shape[1])
    gp = P.params(**EXAMPLE, neumann=P.neumann_flags(gc, dev(Nb)))
    sysm = P.condense(dev(X), dev(T), gc, None, gp)
    glam, gU, st = P.solve(dev(X), dev(T), gc, sysm, None, gp, mode=0, tol=1e-12)
    from paper_2509_11133_amd import _binding as B
    with pytest.raises(B.PhfemError):
        P.grad(dev(X), dev(T), gc, sysm, None, gp, gU, glam, gU)


@pytest.mark.parametrize("mode,precision", [(0, 0), (1, 1)])
def test_solve_zero_data(mode, precision):
    """f = 0 and u_D = 0: lambda and U are exactly zero, reached without an iteration (both
    solvers start from zero and stop on a zero right-hand side)."""
    X, T, _, _ = levels(M.kuhn_cube, 1)
    gc = P.connect(dev(T), X.shape[1])
    gp = P.params(c=1.0, kappa=1.0, precision=precision)
    sysm = P.condense(dev(X), dev(T), gc, None, gp)
    lam, U, st = P.solve(dev(X), dev(T), gc, sysm, None, gp, mode=mode, tol=1e-12)
    assert st["converged"] and st["iters"] == 0
    assert float(lam.abs().max()) == 0.0 and float(U.abs().max()) == 0.0


def test_solve_pattern_check():
    """phfem_solve takes the 6-slot layout condense writes; another row pointer or a column id
    outside [0, nF) is found by the device-side check and refused before any iteration."""
    X, T = jittered(1, seed=2)
    gc = P.connect(dev(T), X.shape[1])
    gp = P.params(c=1.0, f=(O.FUN_SIN3, (M.SIN3_AMPLITUDE,)))
    sysm = P.condense(dev(X), dev(T), gc, None, gp)
    from paper_2509_11133_amd import _binding as B
    bad_rp = dict(sysm, rowptr=sysm["rowptr"].clone())
    bad_rp["rowptr"][5] += 1
    bad_col = dict(sysm, col=sysm["col"].clone())
    bad_col["col"][17] = gc["nF"]
    for bad in (bad_rp, bad_col):
        with pytest.raises(B.PhfemError, match="6-slot"):
            P.solve(dev(X), dev(T), gc, bad, None, gp, mode=0, tol=1e-10)
    lam, U, st = P.solve(dev(X), dev(T), gc, sysm, None, gp, mode=1, tol=1e-10)
    assert st["converged"]
