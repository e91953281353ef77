"""Convenience layer over the C-ABI: allocates outputs and workspaces as torch tensors on
the mesh's device and calls the library.  No arithmetic of the method happens here.

Mesh arrays: coord float64 (3, nC), tetra int32 (4, nE), boundary face lists int32 (3, n),
all contiguous on a HIP device.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _binding as B
from ._binding import (CONNECT_EDGES, CONNECT_FACES, CONNECT_NODES2EDGE, CONNECT_RADIX, ENOCONV, FP64, MIXED,
                       OK, SOLVE_FP32_PCG_FP64_IR, SOLVE_FP64_PCG, PhfemError, SolveStats, params)

I32, F64 = torch.int32, torch.float64


def connect(tetra, nC, faces=True, n2e=False, radix=False):
    """Edges (+ Nodes2Edge CSR) and, with faces=True, the face numbering (a1-a3).
    radix=True takes the library's radix-sort path (same outputs)."""
    dev = tetra.device
    nE = tetra.shape[1]
    flags = (CONNECT_EDGES | (CONNECT_FACES if faces else 0) | (CONNECT_NODES2EDGE if n2e else 0)
             | (CONNECT_RADIX if radix else 0))
    work = B.workspace(B.lib().phfem_connect_workspace(nC, nE, flags), dev)
    e = torch.empty(12 * nE, dtype=I32, device=dev)
    t2e = torch.empty((6, nE), dtype=I32, device=dev)
    eft = torch.empty(6 * nE, dtype=I32, device=dev)
    pre = torch.empty(nE, dtype=I32, device=dev)
    rp = torch.empty(nC + 1, dtype=I32, device=dev) if n2e else None
    nc = torch.empty(6 * nE, dtype=I32, device=dev) if n2e else None
    ne = torch.empty(6 * nE, dtype=I32, device=dev) if n2e else None
    fa = torch.empty(12 * nE, dtype=I32, device=dev) if faces else None
    t2f = torch.empty((4, nE), dtype=I32, device=dev) if faces else None
    sig = torch.empty((4, nE), dtype=torch.int8, device=dev) if faces else None
    f2t = torch.empty(8 * nE, dtype=I32, device=dev) if faces else None
    nbr = torch.empty((4, nE), dtype=I32, device=dev) if faces else None
    counts = np.zeros(3, np.int64)
    B.phfem_connect(nC, nE, tetra, flags, work, e, t2e, eft, pre, rp, nc, ne, fa, t2f, sig, f2t, nbr, counts)
    nEd, nF, nB = (int(v) for v in counts)
    out = dict(nC=nC, nE=nE, nEd=nEd, edges=e[: 2 * nEd].view(2, nEd), tet2edge=t2e, edge_first_tet=eft[:nEd],
               tet_edge_prefix=pre)
    if n2e:
        out.update(n2e_rowptr=rp, n2e_col=nc[:nEd], n2e_edge=ne[:nEd])
    if faces:
        out.update(nF=nF, nB=nB, faces=fa[: 3 * nF].view(3, nF), tet2face=t2f, sigma=sig,
                   face2tet=f2t[: 2 * nF].view(2, nF), nbr=nbr)
    return out


def refine(coord, tetra, conn, db=None, nb=None):
    """One level of the 12-subtet refinement (a4).  Needs connect(..., n2e=True) when
    boundary face lists are given.  Returns (coord, tetra, db, nb)."""
    dev = coord.device
    nC, nE, nEd = coord.shape[1], tetra.shape[1], conn["nEd"]
    nCo = nC + nEd + nE
    Xo = torch.empty((3, nCo), dtype=F64, device=dev)
    To = torch.empty((4, 12 * nE), dtype=I32, device=dev)
    nDb = 0 if db is None else db.shape[1]
    nNb = 0 if nb is None else nb.shape[1]
    dbo = torch.empty((3, 4 * nDb), dtype=I32, device=dev) if nDb else None
    nbo = torch.empty((3, 4 * nNb), dtype=I32, device=dev) if nNb else None
    wb = B.lib().phfem_refine_workspace(nDb, nNb)
    work = B.workspace(wb, dev) if wb else None
    B.phfem_refine(nC, coord, nE, tetra, nEd, conn["tet2edge"], conn["edge_first_tet"], conn["tet_edge_prefix"],
                   conn.get("n2e_rowptr"), conn.get("n2e_col"), conn.get("n2e_edge"), nDb, db if nDb else None, nNb,
                   nb if nNb else None, work, Xo, To, dbo, nbo)
    return Xo, To, dbo, nbo


def neumann_flags(conn, tris, face_of=False):
    """Device uint8 flags [nF] (1 = Neumann face) for the boundary triangles tris [3][n] (node
    triples in any order, e.g. a refined Nb list), matched to the face numbering by
    phfem_face_lookup; every triangle must be a boundary face.  face_of=True also returns each
    triangle's face id."""
    dev = conn["faces"].device
    tris = torch.as_tensor(tris, dtype=I32).to(dev).contiguous()
    n = tris.shape[1]
    nF = conn["nF"]
    flags = torch.empty(nF, dtype=torch.uint8, device=dev)
    fo = torch.empty(max(n, 1), dtype=I32, device=dev)
    wb = B.lib().phfem_face_lookup_workspace(n)
    work = B.workspace(wb, dev) if wb else None
    nC = conn["nC"]
    B.phfem_face_lookup(nC, nF, conn["faces"].contiguous(), conn["face2tet"].contiguous(), n, tris if n else None,
                        work, flags, fo if n else None)
    return (flags, fo[:n]) if face_of else flags


def refine_connected(coord, tetra, conn, status=None):
    """One refinement level that also returns the refined mesh's full connectivity (same
    numbering as connect() on it), derived from `conn` (full connectivity of the coarse
    mesh) without sorting.  Returns (coord, tetra, conn).  With `status` (a zeroed device
    int32 tensor) the input check is left on the device (nothing synchronizes): read it
    with check_status()."""
    dev = coord.device
    nC, nE, nEd, nF = coord.shape[1], tetra.shape[1], conn["nEd"], conn["nF"]
    nC2, nE2 = nC + nEd + nE, 12 * nE
    nEd2, nF2 = 2 * nEd + 3 * nF + 6 * nE, 4 * nF + 16 * nE
    work = B.workspace(B.lib().phfem_refine_connected_workspace(nE, nEd), dev)
    Xo = torch.empty((3, nC2), dtype=F64, device=dev)
    To = torch.empty((4, nE2), dtype=I32, device=dev)
    e = torch.empty((2, nEd2), dtype=I32, device=dev)
    t2e = torch.empty((6, nE2), dtype=I32, device=dev)
    eft = torch.empty(nEd2, dtype=I32, device=dev)
    pre = torch.empty(nE2, dtype=I32, device=dev)
    fa = torch.empty((3, nF2), dtype=I32, device=dev)
    t2f = torch.empty((4, nE2), dtype=I32, device=dev)
    sig = torch.empty((4, nE2), dtype=torch.int8, device=dev)
    f2t = torch.empty((2, nF2), dtype=I32, device=dev)
    nbr = torch.empty((4, nE2), dtype=I32, device=dev)
    counts = np.zeros(3, np.int64)
    B.phfem_refine_connected(nC, coord, nE, tetra, nEd, nF, conn["tet2edge"], conn["edge_first_tet"],
                             conn["tet_edge_prefix"], conn["tet2face"], conn["nbr"], work, Xo, To, e, t2e, eft, pre,
                             fa, t2f, sig, f2t, nbr, counts, status)
    out = dict(nC=nC2, nE=nE2, nEd=int(counts[0]), edges=e, tet2edge=t2e, edge_first_tet=eft, tet_edge_prefix=pre,
               nF=int(counts[1]), nB=int(counts[2]), faces=fa, tet2face=t2f, sigma=sig, face2tet=f2t, nbr=nbr)
    return Xo, To, out


def check_status(status):
    """Raise if a device-side refine_connected check failed (one synchronization)."""
    code = int(status.item())
    if code:
        raise B.PhfemError(B.EINVAL, "refine_connected input check failed (code %d: %s)" % (
            code, "edge id out of range" if code & 1 else "refined totals differ from the recurrences"))


def refine_connected_levels(coord, tetra, levels, conn=None, status=None):
    """connect() on the input mesh (unless `conn` is given), then `levels` refinements with
    derived connectivity in one library call (phfem_refine_connected_levels).  Without
    `status` the call checks its input and synchronizes once; with a zeroed device int32
    `status` nothing synchronizes (read it with check_status).  Returns (coord, tetra, conn)."""
    if conn is None:
        conn = connect(tetra, coord.shape[1], faces=True)
    if levels == 0:
        return coord, tetra, conn
    dev = coord.device
    nC, nE, nEd, nF = coord.shape[1], tetra.shape[1], conn["nEd"], conn["nF"]
    nC2, nE2, nEd2, nF2 = B.phfem_refined_sizes(nC, nE, nEd, nF, levels)
    work = B.workspace(B.lib().phfem_refine_connected_levels_workspace(nC, nE, nEd, nF, levels), dev)
    Xo = torch.empty((3, nC2), dtype=F64, device=dev)
    To = torch.empty((4, nE2), dtype=I32, device=dev)
    e = torch.empty((2, nEd2), dtype=I32, device=dev)
    t2e = torch.empty((6, nE2), dtype=I32, device=dev)
    eft = torch.empty(nEd2, dtype=I32, device=dev)
    pre = torch.empty(nE2, dtype=I32, device=dev)
    fa = torch.empty((3, nF2), dtype=I32, device=dev)
    t2f = torch.empty((4, nE2), dtype=I32, device=dev)
    sig = torch.empty((4, nE2), dtype=torch.int8, device=dev)
    f2t = torch.empty((2, nF2), dtype=I32, device=dev)
    nbr = torch.empty((4, nE2), dtype=I32, device=dev)
    counts = np.zeros(3, np.int64)
    B.phfem_refine_connected_levels(nC, coord, nE, tetra, nEd, nF, conn["tet2edge"], conn["edge_first_tet"],
                                    conn["tet_edge_prefix"], conn["tet2face"], conn["nbr"], levels, work, Xo, To, e,
                                    t2e, eft, pre, fa, t2f, sig, f2t, nbr, counts, status)
    out = dict(nC=nC2, nE=nE2, nEd=int(counts[0]), edges=e, tet2edge=t2e, edge_first_tet=eft, tet_edge_prefix=pre,
               nF=int(counts[1]), nB=int(counts[2]), faces=fa, tet2face=t2f, sigma=sig, face2tet=f2t, nbr=nbr)
    return Xo, To, out


def assemble(coord, tetra, sigma, kappa, prm):
    """Per-tet blocks: vol, kappa K (16), sigma|F| (4), B (4), S (16), r (4)."""
    dev = coord.device
    nC, nE = coord.shape[1], tetra.shape[1]
    out = dict(vol=torch.empty(nE, dtype=F64, device=dev), K=torch.empty((16, nE), dtype=F64, device=dev),
               d=torch.empty((4, nE), dtype=F64, device=dev), B=torch.empty((4, nE), dtype=F64, device=dev),
               S=torch.empty((16, nE), dtype=F64, device=dev), r=torch.empty((4, nE), dtype=F64, device=dev))
    B.phfem_assemble(nC, coord, nE, tetra, sigma, kappa, prm, out["vol"], out["K"], out["d"], out["B"], out["S"],
                     out["r"])
    return out


def condense(coord, tetra, conn, kappa, prm):
    """Condensed face system (a5-a7): diag, off-diagonal CSR (rowptr, col, val), rhs."""
    dev = coord.device
    nC, nE, nF, nB = coord.shape[1], tetra.shape[1], conn["nF"], conn["nB"]
    work = B.workspace(B.lib().phfem_condense_workspace(nC, nE, nF, prm.precision), dev)
    nnz = 6 * nF  # fixed 6 slots per row (boundary rows padded with explicit zeros)
    rowptr = torch.empty(nF + 1, dtype=I32, device=dev)
    col = torch.empty(max(nnz, 1), dtype=I32, device=dev)
    val = torch.empty(max(nnz, 1), dtype=F64, device=dev)
    diag = torch.empty(nF, dtype=F64, device=dev)
    rhs = torch.empty(nF, dtype=F64, device=dev)
    B.phfem_condense(nC, coord, nE, tetra, nF, conn["faces"], conn["tet2face"], conn["sigma"], conn["nbr"],
                     conn["face2tet"], kappa, prm, work, rowptr, col, val, diag, rhs)
    return dict(rowptr=rowptr, col=col[:nnz], val=val[:nnz], diag=diag, rhs=rhs, nnz=nnz)


def condense_batch(coord, tetra, conn, kappas, prm, pattern=None):
    """Face systems of several kappa fields kappas [nk, nE] on one mesh in one call (NEXT
    item: pattern reuse and batched coefficients).  pattern = (rowptr, col) of an earlier
    condense on the same connectivity: only values are written; None: the pattern is built too.
    Returns a list of nk systems (dicts as condense returns; they share rowptr and col)."""
    dev = coord.device
    nC, nE, nF = coord.shape[1], tetra.shape[1], conn["nF"]
    kappas = kappas.contiguous()
    nk = kappas.shape[0]
    work = B.workspace(B.lib().phfem_condense_batch_workspace(nC, nE, nF, prm.precision, nk), dev)
    nnz = 6 * nF
    if pattern is None:
        rowptr = torch.empty(nF + 1, dtype=I32, device=dev)
        col = torch.empty(nnz, dtype=I32, device=dev)
        rp, cl = rowptr, col
    else:
        rowptr, col = pattern
        rp = cl = None
    val = torch.empty((nk, nnz), dtype=F64, device=dev)
    diag = torch.empty((nk, nF), dtype=F64, device=dev)
    rhs = torch.empty((nk, nF), dtype=F64, device=dev)
    B.phfem_condense_batch(nC, coord, nE, tetra, nF, conn["faces"], conn["tet2face"], conn["sigma"], conn["nbr"],
                           conn["face2tet"], nk, kappas, prm, work, rp, cl, val, diag, rhs)
    return [dict(rowptr=rowptr, col=col, val=val[j], diag=diag[j], rhs=rhs[j], nnz=nnz) for j in range(nk)]


def condense_reuse(coord, tetra, conn, kappa, prm):
    """condense with the pattern kept in conn["pattern"]: the first call builds it, later calls
    on the same connectivity write values only (the pattern depends on the connectivity alone)."""
    if "pattern" not in conn:
        sysm = condense(coord, tetra, conn, kappa, prm)
        conn["pattern"] = (sysm["rowptr"], sysm["col"])
        return sysm
    nE = tetra.shape[1]
    k = (torch.full((1, nE), prm.kappa_const, dtype=F64, device=coord.device) if kappa is None
         else kappa.reshape(1, nE))
    return condense_batch(coord, tetra, conn, k, prm, pattern=conn["pattern"])[0]


def solve(coord, tetra, conn, sysm, kappa, prm, mode=SOLVE_FP64_PCG, tol=1e-10, inner_tol=0.9, max_iter=200000,
          allow_noconv=False):
    """Face solve + recovery (a8-a9).  Returns (lambda, U, stats)."""
    dev = coord.device
    nC, nE, nF = coord.shape[1], tetra.shape[1], conn["nF"]
    work = B.workspace(B.lib().phfem_solve_workspace(nE, nF, mode), dev)
    lam = torch.empty(nF, dtype=F64, device=dev)
    U = torch.empty((4, nE), dtype=F64, device=dev)
    st = SolveStats()
    rc = B.phfem_solve(nC, coord, nE, tetra, nF, conn["faces"], conn["tet2face"], conn["sigma"], conn["face2tet"],
                       kappa, prm, sysm["rowptr"], sysm["col"], sysm["val"], sysm["diag"], sysm["rhs"], mode, tol,
                       inner_tol, max_iter, work, lam, U, st, check=False)
    stats = st.as_dict()
    stats["converged"] = rc == OK
    if rc != OK and not (rc == ENOCONV and allow_noconv):
        raise PhfemError(rc, B.lib().phfem_last_error().decode())
    return lam, U, stats


def solve_multi(coord, tetra, conn, sysm, kappa, prms, rhs=None, tol=1e-10, max_iter=200000, allow_noconv=False):
    """Several loads on one face system (FP64 lockstep PCG): prms = one params per load (same c
    and kappa), rhs = [nk, nF] tensor or None (formed matrix-free).  Returns (lambda [nk, nF],
    U [nk, 4, nE], list of stats)."""
    dev = coord.device
    nC, nE, nF = coord.shape[1], tetra.shape[1], conn["nF"]
    nk = len(prms)
    work = B.workspace(B.lib().phfem_solve_multi_workspace(nE, nF, nk), dev)
    lam = torch.empty((nk, nF), dtype=F64, device=dev)
    U = torch.empty((nk, 4, nE), dtype=F64, device=dev)
    st = (SolveStats * nk)()
    rc = B.phfem_solve_multi(nC, coord, nE, tetra, nF, conn["faces"], conn["tet2face"], conn["sigma"],
                             conn["face2tet"], kappa, prms, sysm["rowptr"], sysm["col"], sysm["val"], sysm["diag"],
                             None if rhs is None else rhs.contiguous(), tol, max_iter, work, lam, U, st, check=False)
    stats = [s_.as_dict() for s_ in st]
    for s_ in stats:
        s_["converged"] = rc == OK and s_["rel_res"] <= tol
    if rc != OK and not (rc == ENOCONV and allow_noconv):
        raise PhfemError(rc, B.lib().phfem_last_error().decode())
    return lam, U, stats


def grad(coord, tetra, conn, sysm, kappa, prm, U, lam, dJdU, mode=SOLVE_FP64_PCG, tol=1e-10, inner_tol=0.9,
         max_iter=200000, want_coord=True, allow_noconv=False):
    """Adjoint gradient (a10): (dJ/dlog kappa [nE], dJ/dX [3, nC], stats).  With allow_noconv an
    adjoint solve that stopped above tol (ENOCONV: the last iterate) still returns its
    gradient; stats["converged"] says which."""
    dev = coord.device
    nC, nE, nF = coord.shape[1], tetra.shape[1], conn["nF"]
    work = B.workspace(B.lib().phfem_grad_workspace(nE, nF, mode), dev)
    dlogk = torch.empty(nE, dtype=F64, device=dev)
    dX = torch.empty((3, nC), dtype=F64, device=dev) if want_coord else None
    st = SolveStats()
    rc = B.phfem_grad(nC, coord, nE, tetra, nF, conn["faces"], conn["tet2face"], conn["sigma"], conn["face2tet"],
                      conn["nbr"], kappa, prm, sysm["rowptr"], sysm["col"], sysm["val"], sysm["diag"], U, lam,
                      dJdU.contiguous(), mode, tol, inner_tol, max_iter, work, dlogk, dX, st, check=False)
    stats = st.as_dict()
    stats["converged"] = rc == OK
    if rc != OK and not (rc == ENOCONV and allow_noconv):
        raise PhfemError(rc, B.lib().phfem_last_error().decode())
    return dlogk, dX, stats


def errors(coord, tetra, conn, kappa, prm, U, lam, u_kind, u_par, h, nq=8):
    """Error norms of (U, lambda) against the exact solution u (Section 5, Table 4's norms):
    dict(grad2, l22, lam_h2, Y, h_norm) with Y = sqrt(grad2 + l22 / h^2), h_norm = sqrt(lam_h2).
    Neumann faces (prm.neumann) are left out of the multiplier norm."""
    nC, nE = coord.shape[1], tetra.shape[1]
    work = B.workspace(B.lib().phfem_errors_workspace(nE), coord.device)
    g2, l2, lh = B.phfem_errors(nC, coord, nE, tetra, conn["nF"], conn["tet2face"], conn["sigma"], kappa, prm, U, lam,
                                u_kind, u_par, h, nq, work)
    return dict(grad2=g2, l22=l2, lam_h2=lh, Y=(g2 + l2 / h ** 2) ** 0.5, h_norm=lh ** 0.5)


def refine_levels(coord, tetra, levels, db=None):
    """Pipeline of the paper's uniform refinement: [connect edges -> refine] per level."""
    for _ in range(levels):
        conn = connect(tetra, coord.shape[1], faces=False, n2e=db is not None)
        coord, tetra, db, _ = refine(coord, tetra, conn, db)
    return coord, tetra, db


class PrimalHybridSolve(torch.autograd.Function):
    """U = solution of the primal hybrid system for per-tet log-diffusivity and vertex
    coordinates; backward = one adjoint face solve + per-tet VJP kernels (phfem_grad).
    Mesh connectivity (from connect) and params are fixed inputs; the face-system pattern is
    built by the first call and reused (values-only re-assembly) by later ones."""

    @staticmethod
    def forward(ctx, log_kappa, coord, tetra, conn, prm, mode, tol):
        kappa = torch.exp(log_kappa.detach()).contiguous()
        X = coord.detach().contiguous()
        sysm = condense_reuse(X, tetra, conn, kappa, prm)
        lam, U, st = solve(X, tetra, conn, sysm, kappa, prm, mode=mode, tol=tol)
        ctx.save_for_backward(X, kappa, U, lam)
        ctx.tetra, ctx.conn, ctx.prm, ctx.mode, ctx.tol, ctx.sysm = tetra, conn, prm, mode, tol, sysm
        ctx.need_X = coord.requires_grad
        return U

    @staticmethod
    def backward(ctx, gU):
        X, kappa, U, lam = ctx.saved_tensors
        dlogk, dX, _ = grad(X, ctx.tetra, ctx.conn, ctx.sysm, kappa, ctx.prm, U, lam, gU.contiguous(), mode=ctx.mode,
                            tol=ctx.tol, want_coord=ctx.need_X)
        return dlogk, dX, None, None, None, None, None
