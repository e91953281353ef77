"""GPU: the three connect paths (one-workgroup, node buckets, radix sort) give the oracle's
numbering (Sections 3.1-3.3) on meshes that reach every branch of the bucket path: buckets
resolved in LDS, a workgroup whose buckets overflow LDS (resolved from global memory), and a
node that is the lowest node of more occurrences than the bucket path takes (the call falls
back to the radix sort).  Also the error flags on meshes above the one-workgroup size."""
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
KEYS = ("edges", "tet2edge", "edge_first_tet", "tet_edge_prefix", "faces", "tet2face", "sigma", "face2tet", "nbr")


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def refined(make, L):
    X, T = make()[:2]
    for _ in range(L):
        X, T, _, _ = O.refine(X, T)
    return X, T


def permuted(X, T, seed):
    rng = np.random.default_rng(seed)
    T = T[:, rng.permutation(T.shape[1])]
    return X, rng.permutation(X.shape[1])[T].astype(np.int32)


def uv_sphere_cone(m, k, center_first):
    """Cone from the centre over a latitude-longitude sphere (m meridians, k bands):
    2 m (k - 1) tets, every one holding the centre."""
    th = np.linspace(0, np.pi, k + 1)[1:-1]
    ph = 2 * np.pi * np.arange(m) / m
    ring = np.stack([np.outer(np.sin(th), np.cos(ph)).ravel(), np.outer(np.sin(th), np.sin(ph)).ravel(),
                     np.repeat(np.cos(th), m)])
    S = np.concatenate([[[0.0], [0.0], [1.0]], ring, [[0.0], [0.0], [-1.0]]], axis=1)
    nS = S.shape[1]
    r = lambda j, i: 1 + j * m + (i % m)  # noqa: E731
    tris = [(0, r(0, i), r(0, i + 1)) for i in range(m)]
    for j in range(k - 2):
        for i in range(m):
            tris += [(r(j, i), r(j + 1, i), r(j + 1, i + 1)), (r(j, i), r(j + 1, i + 1), r(j, i + 1))]
    tris += [(nS - 1, r(k - 2, i + 1), r(k - 2, i)) for i in range(m)]
    return _cone(S, np.array(tris, np.int64), center_first)


def icosphere_cone(n, center_first):
    """Cone from the centre over an icosphere subdivided n times (20 4^n tets)."""
    g = (1 + 5 ** 0.5) / 2
    V = [(-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0), (0, -1, g), (0, 1, g), (0, -1, -g), (0, 1, -g),
         (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6),
         (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
         (8, 6, 7), (9, 8, 1)]
    V = [np.array(v, float) / np.linalg.norm(v) for v in V]
    for _ in range(n):
        mid = {}

        def mp(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                p = V[a] + V[b]
                V.append(p / np.linalg.norm(p))
                mid[key] = len(V) - 1
            return mid[key]

        F2 = []
        for a, b, c in F:
            ab, bc, ca = mp(a, b), mp(b, c), mp(c, a)
            F2 += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = F2
    return _cone(np.array(V).T, np.array(F, np.int64), center_first)


def _cone(S, tris, center_first):
    nS = S.shape[1]
    if center_first:
        X = np.concatenate([np.zeros((3, 1)), S], axis=1)
        T = np.concatenate([np.zeros((1, len(tris)), np.int64), tris.T + 1])
    else:
        X = np.concatenate([S, np.zeros((3, 1))], axis=1)
        T = np.concatenate([np.full((1, len(tris)), nS, np.int64), tris.T])
    T = T.astype(np.int32)
    a, b, c, d = (X[:, T[i]] for i in range(4))
    det = np.einsum("in,in->n", b - a, np.cross(c - a, d - a, axis=0))
    neg = det < 0
    T[2, neg], T[3, neg] = T[3, neg].copy(), T[2, neg].copy()
    return np.ascontiguousarray(X), np.ascontiguousarray(T)


def check_all(X, T, paths=("bucket", "radix")):
    oc = O.connect(X.shape[1], T)
    nEd = oc["nEd"]
    A = sp.csr_matrix((np.arange(nEd) + 1, (oc["edges"][0], oc["edges"][1])), shape=(X.shape[1], X.shape[1]))
    A.sort_indices()
    for path in paths:
        radix = path == "radix"
        for n2e in (False, True):
            g = P.connect(dev(T), X.shape[1], faces=True, n2e=n2e, radix=radix)
            assert (g["nEd"], g["nF"], g["nB"]) == (oc["nEd"], oc["nF"], oc["nB"]), (path, n2e)
            for k in KEYS:
                assert np.array_equal(host(g[k]), oc[k]), (path, n2e, k)
            if n2e:
                assert np.array_equal(host(g["n2e_rowptr"]), A.indptr), path
                assert np.array_equal(host(g["n2e_col"]), A.indices), path
                assert np.array_equal(host(g["n2e_edge"]) + 1, A.data), path
        e = P.connect(dev(T), X.shape[1], faces=False, radix=radix)
        for k in ("edges", "tet2edge", "edge_first_tet", "tet_edge_prefix"):
            assert np.array_equal(host(e[k]), oc[k]), (path, "edges only", k)


@pytest.mark.parametrize("case", ["kuhn3", "fichera2_perm", "kuhn2_perm", "disjoint"])
def test_bucket_and_radix_paths_bitexact(case):
    """Refined, permuted-and-relabelled and disconnected meshes: both paths, with and without
    Nodes2Edge and faces, equal the oracle."""
    if case == "disjoint":
        rng = np.random.default_rng(3)
        n = 900
        ref = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float)
        X = (0.3 * (ref[None] + 0.2 * rng.random((n, 4, 3))) + 3.0 * rng.random((n, 1, 3))).reshape(-1, 3).T.copy()
        T = np.arange(4 * n, dtype=np.int32).reshape(n, 4).T.copy()
    else:
        make = M.kuhn_cube if case.startswith("kuhn") else M.fichera
        X, T = refined(make, int(case.split("_")[0][-1]))
        if case.endswith("_perm"):
            X, T = permuted(X, T, 11)
    print(case, T.shape[1], "tets", flush=True)
    check_all(X, T)


@pytest.mark.parametrize("case", ["uv_last", "uv_first", "uv600_first", "ico4_first", "ico3_first"])
def test_high_degree_node(case):
    """A node in every tet: numbered last, its buckets stay small on every node but itself as
    the highest node (LDS hash path); numbered first, it is the lowest node of 3 occurrences
    per tet -- 1800 (uv600, 600 tets: its workgroup's entries exceed the hash table and are
    staged in LDS, each scanning its bucket), 4800 (uv, 1600 tets) and 3840 (ico3, 1280 tets),
    where its workgroup's entries exceed LDS and are resolved from global memory, and 15360
    (ico4, 5120 tets), above the bucket path's limit, so that the call falls back to the radix
    sort."""
    if case.startswith("uv600"):
        X, T = uv_sphere_cone(20, 16, center_first=True)
    elif case.startswith("uv"):
        X, T = uv_sphere_cone(40, 21, center_first=case.endswith("first"))
    else:
        X, T = icosphere_cone(int(case[3]), center_first=case.endswith("first"))
    print(case, T.shape[1], "tets", X.shape[1], "nodes", flush=True)
    check_all(X, T, paths=("bucket",))


def _large_errors():
    X, T = refined(M.kuhn_cube, 2)  # 864 tets: above the one-workgroup size
    nC = X.shape[1]
    flip = T.copy()
    flip[[2, 3], 100] = flip[[3, 2], 100]
    oc = O.connect(nC, T)
    f = oc["face2tet"]
    q = int(f[0, np.nonzero(f[1] >= 0)[0][5]])  # an interior face, at its owner's slot
    t, k = q // 4, q % 4
    loc = [[0, 1, 2], [0, 2, 3], [0, 3, 1], [3, 2, 1]][k]
    tri = T[loc, t]
    three = np.concatenate([T, np.array([[tri[0]], [tri[2]], [tri[1]], [nC]], np.int32)], axis=1)
    bad = T.copy()
    bad[2, 500] = nC
    neg = T.copy()
    neg[1, 700] = -1
    rep = T.copy()
    rep[3, 300] = rep[0, 300]
    return [("flip", nC, flip, "EORIENT"), ("three", nC + 1, three, "EORIENT"), ("bad", nC, bad, "EINVAL"),
            ("neg", nC, neg, "EINVAL"), ("rep", nC, rep, "EINVAL")]


@pytest.mark.parametrize("radix", [False, True])
@pytest.mark.parametrize("n2e", [False, True])
def test_errors_above_one_workgroup(radix, n2e):
    """Flipped tet, a face in three tets, node ids out of range and a repeated node, on an
    864-tet mesh through the bucket and radix paths; then a good call on the same path."""
    for name, nC, T, code in _large_errors():
        print(name, "radix" if radix else "bucket", "n2e" if n2e else "", flush=True)
        with pytest.raises(P.PhfemError) as e:
            P.connect(dev(T), nC, faces=True, n2e=n2e, radix=radix)
        assert e.value.code == getattr(P.B, code), name
    X, T = refined(M.kuhn_cube, 2)
    g = P.connect(dev(T), X.shape[1], faces=True, n2e=n2e, radix=radix)
    oc = O.connect(X.shape[1], T)
    for k in KEYS:
        assert np.array_equal(host(g[k]), oc[k]), k


def test_bucket_path_deterministic():
    """Bucket entries land in an order set by atomics; every output is independent of it."""
    X, T = permuted(*refined(M.fichera, 2), 5)
    a = P.connect(dev(T), X.shape[1], faces=True, n2e=True)
    for _ in range(3):
        b = P.connect(dev(T), X.shape[1], faces=True, n2e=True)
        for k in KEYS + ("n2e_rowptr", "n2e_col", "n2e_edge"):
            assert torch.equal(a[k], b[k]), k
