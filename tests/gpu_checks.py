"""Full-size checks shared by the GPU tests of the benchmark meshes (a helper, not a test
module): exhaustive properties of a refined mesh's connectivity, sampled condensed rows
against the oracle's element blocks, and local conservation on sampled tets."""
import numpy as np
import torch

import oracle as O

DEV = torch.device("cuda:0")
EV = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]  # local edges IJ IK IL JK JL KL
FV = [(0, 1, 2), (0, 2, 3), (0, 3, 1), (3, 2, 1)]  # local faces [a b c] [a c d] [a d b] [d c b]


def refined_counts(level0, L):
    """(nC, nE, nEd, nF, nB) after L levels of the 12-subtet split, from the level-0 counts"""
    nC, nE, nEd, nF, nB = level0
    for _ in range(L):
        nC, nE, nEd, nF, nB = nC + nEd + nE, 12 * nE, 2 * nEd + 3 * nF + 6 * nE, 4 * nF + 16 * nE, 4 * nB
    return nC, nE, nEd, nF, nB


def _first_position_order(owner_pos):
    """ids numbered by first position <=> the first positions strictly increase with the id"""
    return bool(torch.all(owner_pos[1:] > owner_pos[:-1]).item())


def check_topology(X, T, c, counts, volume):
    """Properties that pin the first-appearance numberings at any size, on every tet, edge and
    face: ids ordered by their first position, endpoints / tuples equal to the tets' local
    entities, owner = lowest tet, sigma and face2tet consistent, neighbour symmetry, Euler
    characteristic, exact volume (dyadic coordinates)."""
    nC, nE, nEd, nF, nB = counts
    assert (X.shape[1], T.shape[1], c["nEd"], c["nF"], c["nB"]) == (nC, nE, nEd, nF, nB)
    assert nC - nEd + nF - nE == 1  # Euler characteristic of a contractible domain
    t = torch.arange(nE, device=DEV, dtype=torch.int64)
    T64 = T.long()
    # edges: endpoints = the tets' local edges; ids ordered by first position 6 t + j
    t2e = c["tet2edge"].long()
    E = c["edges"].long()
    first = torch.full((nEd,), 2 ** 62, dtype=torch.int64, device=DEV)
    for j, (a, b) in enumerate(EV):
        lo, hi = torch.minimum(T64[a], T64[b]), torch.maximum(T64[a], T64[b])
        assert torch.equal(E[0, t2e[j]], lo) and torch.equal(E[1, t2e[j]], hi)
        first.scatter_reduce_(0, t2e[j], 6 * t + j, reduce="amin")
    assert _first_position_order(first)
    assert torch.equal(c["edge_first_tet"].long(), first // 6)
    # tet_edge_prefix = number of edges first seen in earlier tets
    newcnt = torch.zeros(nE, dtype=torch.int64, device=DEV)
    newcnt.scatter_add_(0, first // 6, torch.ones_like(first))
    assert torch.equal(c["tet_edge_prefix"].long(), torch.cumsum(newcnt, 0) - newcnt)
    # faces: tuples = the owner's local face, ids ordered by owner slot 4 t + k, owner = lowest tet
    t2f = c["tet2face"].long()
    f2t = c["face2tet"].long()
    sig = c["sigma"].long()
    assert _first_position_order(f2t[0])
    interior = f2t[1] >= 0
    assert int((~interior).sum().item()) == nB
    assert torch.all(f2t[1][interior] > f2t[0][interior])
    Fc = c["faces"].long()
    for k, (a, b, d) in enumerate(FV):
        f = t2f[k]
        own = sig[k] > 0
        slot = 4 * t + k
        assert torch.equal(f2t[0, f[own]], slot[own]) and torch.equal(f2t[1, f[~own]], slot[~own])
        assert torch.all(sig[k][~own] == -1)
        for m, v in enumerate((a, b, d)):
            assert torch.equal(Fc[m, f[own]], T64[v][own])
        nb = c["nbr"].long()[k]
        assert torch.equal(nb >= 0, interior[f])
        other = torch.where(own, f2t[1, f], f2t[0, f])
        assert torch.equal(torch.where(nb >= 0, other // 4, nb), nb)
    # refinement: volume conserved exactly (dyadic coordinates), all tets positively oriented
    x = X[:, T64]  # (3, 4, nE)
    a, b, d = x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]
    det = (a[0] * (b[1] * d[2] - b[2] * d[1]) - a[1] * (b[0] * d[2] - b[2] * d[0]) +
           a[2] * (b[0] * d[1] - b[1] * d[0]))
    assert torch.all(det > 0)
    assert float(det.sum().item()) == 6.0 * volume  # dyadic coordinates: every partial sum is exact




def check_rows(X, T, c, sysm, kappa, prm, tol, rng, n_int=3000, n_bnd=600):
    nF = c["nF"]
    f2t = c["face2tet"].cpu().numpy()
    bnd = np.flatnonzero(f2t[1] < 0)
    faces = np.concatenate([rng.choice(np.flatnonzero(f2t[1] >= 0), n_int, replace=False),
                            rng.choice(bnd, min(n_bnd, len(bnd)), replace=False)])
    q0, q1 = f2t[0, faces], f2t[1, faces]
    tets = np.unique(np.concatenate([q0 // 4, q1[q1 >= 0] // 4]))
    tidx = torch.tensor(tets, device=DEV, dtype=torch.int64)
    # mini mesh of the sampled tets (their own coordinates), oracle element blocks
    Tt = T[:, tidx].cpu().numpy()
    Xt = X[:, torch.tensor(Tt.T.reshape(-1), device=DEV, dtype=torch.int64)].cpu().numpy()
    sig = c["sigma"][:, tidx].cpu().numpy()
    t2f = c["tet2face"][:, tidx].cpu().numpy()
    kap = None if kappa is None else kappa[tidx].cpu().numpy()
    Ts = np.arange(4 * len(tets), dtype=np.int32).reshape(-1, 4).T.copy()
    loc = O.local(Xt, Ts, sig, kap, prm)
    S, r = loc["S"].reshape(4, 4, -1), loc["r"]
    pos = {t: i for i, t in enumerate(tets)}
    fi = torch.tensor(faces, device=DEV, dtype=torch.int64)
    rows = (6 * fi[:, None] + torch.arange(6, device=DEV)[None, :])
    gcol, gval = sysm["col"][rows].cpu().numpy(), sysm["val"][rows].cpu().numpy()
    gdiag, grhs = sysm["diag"][fi].cpu().numpy(), sysm["rhs"][fi].cpu().numpy()
    assert np.array_equal(sysm["rowptr"][fi].cpu().numpy(), 6 * faces)
    bd = {}
    if prm.ud_kind != O.FUN_ZERO:  # b_D of sampled boundary faces: oracle condense of the owner alone
        for f in faces[q1 < 0]:
            i, k = pos[f2t[0, f] // 4], f2t[0, f] % 4
            A1, r1 = O.condense(Xt[:, 4 * i:4 * i + 4], np.arange(4, dtype=np.int32).reshape(4, 1),
                                O.connect(4, np.arange(4, dtype=np.int32).reshape(4, 1)), None if kap is None
                                else kap[i:i + 1], prm)
            bd[f] = r1[k] + r[k, i]  # rhs = b_D - r
    want_rhs, rscale = np.zeros(len(faces)), np.zeros(len(faces))
    for n, f in enumerate(faces):
        ent, dg, rh = {}, 0.0, bd.get(f, 0.0)
        rs = abs(rh)
        for q in (q0[n], q1[n]):
            if q < 0:
                continue
            i, k = pos[q // 4], q % 4
            dg += S[k, k, i]
            rh -= r[k, i]
            rs = max(rs, abs(r[k, i]))
            for l in range(4):
                if l != k:
                    ent[int(t2f[l, i])] = S[k, l, i]
        cols = sorted(ent)
        want_c = cols + [f] * (6 - len(cols))
        want_v = [ent[j] for j in cols] + [0.0] * (6 - len(cols))
        assert list(gcol[n]) == want_c, (f, gcol[n], want_c)
        scale = max(abs(dg), max(abs(v) for v in want_v))  # row-relative
        assert abs(gdiag[n] - dg) <= tol * scale and np.all(np.abs(gval[n] - want_v) <= tol * scale), f
        want_rhs[n], rscale[n] = rh, rs
    # rhs = b_D - r_owner - r_neighbour: the two element terms nearly cancel on interior faces,
    # so each rhs entry is compared relative to the largest term of its sum (row-relative)
    # In FP32 the load near the boundary (f ~ distance to it) carries the FP32 rounding of the
    # centroid coordinate relative to that distance; the mixed rhs is therefore bounded against
    # the vector's scale (it only seeds the FP32 correction solves; iterative refinement uses FP64
    # residuals), the FP64 rhs entry by entry.
    scale = rscale if tol < 1e-9 else np.full_like(rscale, np.abs(want_rhs).max())
    rel = np.abs(grhs - want_rhs) / scale
    worst = int(np.argmax(rel))
    assert rel[worst] <= tol, (rel[worst], faces[worst], q1[worst], grhs[worst], want_rhs[worst], rscale[worst])



def check_conservation(X, T, c, kappa, prm, U, lam, rng, n=2000, tol=1e-10):
    """Local conservation of the recovered solution on sampled tets (the mean identity of the
    element equations, Algorithm 1): (c|T|/4) sum_i U_T,i = 1'B_T + sum_k sigma_k |F_k|
    lambda_F(k), with |T|, B_T and sigma_k |F_k| from the oracle's element data."""
    tets = np.sort(rng.choice(T.shape[1], n, replace=False))
    tidx = torch.tensor(tets, device=DEV, dtype=torch.int64)
    Tt = T[:, tidx].cpu().numpy()
    Xt = X[:, torch.tensor(Tt.T.reshape(-1), device=DEV, dtype=torch.int64)].cpu().numpy()
    sig = c["sigma"][:, tidx].cpu().numpy()
    kap = None if kappa is None else kappa[tidx].cpu().numpy()
    Ts = np.arange(4 * n, dtype=np.int32).reshape(-1, 4).T.copy()
    loc = O.local(Xt, Ts, sig, kap, prm)
    Ut = U[:, tidx].cpu().numpy()
    lt = lam[c["tet2face"][:, tidx].long()].cpu().numpy()
    cc = prm.c
    lhs = cc * loc["vol"] / 4 * Ut.sum(axis=0)
    rhs = loc["B"].sum(axis=0) + (loc["d"] * lt).sum(axis=0)
    scale = np.abs(loc["B"]).sum(axis=0) + np.abs(loc["d"] * lt).sum(axis=0)
    assert np.all(np.abs(lhs - rhs) <= tol * scale), np.max(np.abs(lhs - rhs) / scale)
