"""Oracle of the primal hybrid FEM hot path (arXiv 2509.11133) — TEST INFRASTRUCTURE ONLY.

ctypes front end of ``liboracle.so`` (built from ``phfem_oracle.cpp`` with g++).  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import this
package; the GPU library never does.  Arrays are numpy, SoA, 0-based:
``tet`` int32 (4, nE), ``coord`` float64 (3, nC), per-slot arrays (k, nE).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "phfem_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EORIENT, EDEGEN, ESINGULAR, ENOCONV = 0, 1, 2, 3, 4, 5

# data-function kinds (f, u_D, exact solutions)
FUN_ZERO, FUN_CONST, FUN_SIN3, FUN_LINEAR, FUN_X2Y2Z2, FUN_X2Y2Z2_LOAD = 0, 1, 2, 3, 4, 5
QUAD_FACE_CENTROID, QUAD_P1_INTERP = 0, 1


# PHFEM_ORACLE_SANITIZE=1: an AddressSanitizer + UndefinedBehaviorSanitizer build (its own file),
# for a process started with gcc's libasan preloaded (tests/test_sanitizers.py)
_SAN = os.environ.get("PHFEM_ORACLE_SANITIZE") == "1"
if _SAN:
    _LIB = os.path.join(_HERE, "liboracle_san.so")


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (single-threaded, -O2, no fast-math), or the sanitizer build."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        opt = (["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                "-fno-omit-frame-pointer"] if _SAN else ["-O2"])
        subprocess.check_call(["g++", *opt, "-std=c++17", "-fPIC", "-shared", _SRC, "-o", _LIB])
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("c", C.c_double),
        ("kappa_const", C.c_double),
        ("f_kind", C.c_int32),
        ("f_par", C.c_double * 4),
        ("ud_kind", C.c_int32),
        ("ud_par", C.c_double * 4),
        ("quad", C.c_int32),
        ("g_kind", C.c_int32),
        ("g_par", C.c_double * 4),
    ]


def params(c=1.0, kappa=1.0, f=(FUN_ZERO, ()), ud=(FUN_ZERO, ()), quad=QUAD_FACE_CENTROID, g=(FUN_ZERO, ())) -> Params:
    """g: on Neumann faces the flux kappa grad(u_g) . nu of u_g = fun(g) (nu outward)."""
    p = Params()
    p.c = c
    p.kappa_const = kappa
    p.f_kind = f[0]
    for i, v in enumerate(f[1]):
        p.f_par[i] = v
    p.ud_kind = ud[0]
    for i, v in enumerate(ud[1]):
        p.ud_par[i] = v
    p.quad = quad
    p.g_kind = g[0]
    for i, v in enumerate(g[1]):
        p.g_par[i] = v
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB)
        _lib.orc_last_error.restype = C.c_char_p
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _chk(rc):
    if rc != 0:
        raise OracleError(rc, lib().orc_last_error().decode())


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


I64 = C.c_int64


def edges(nC, tet):
    tet = _i32(tet)
    nE = tet.shape[1]
    e = np.zeros(12 * nE, np.int32)
    t2e = np.zeros((6, nE), np.int32)
    eft = np.zeros(6 * nE, np.int32)
    pre = np.zeros(nE, np.int32)
    n = I64()
    _chk(lib().orc_edges(I64(nC), I64(nE), _p(tet), _p(e), _p(t2e), _p(eft), _p(pre), C.byref(n)))
    nEd = n.value
    return dict(nEd=nEd, edges=e[: 2 * nEd].reshape(2, nEd), tet2edge=t2e, edge_first_tet=eft[:nEd],
                tet_edge_prefix=pre)


def edges2tetra(nC, tet):
    tet = _i32(tet)
    nE = tet.shape[1]
    r = np.zeros(12 * nE, np.int32)
    c = np.zeros(12 * nE, np.int32)
    t = np.zeros(12 * nE, np.int32)
    n = I64()
    _chk(lib().orc_edges2tetra(I64(nC), I64(nE), _p(tet), _p(r), _p(c), _p(t), C.byref(n)))
    n = n.value
    return r[:n], c[:n], t[:n]


def faces(nC, tet):
    tet = _i32(tet)
    nE = tet.shape[1]
    f = np.zeros(12 * nE, np.int32)
    t2f = np.zeros((4, nE), np.int32)
    sig = np.zeros((4, nE), np.int8)
    f2t = np.zeros(8 * nE, np.int32)
    nbr = np.zeros((4, nE), np.int32)
    cnt = np.zeros(2, np.int64)
    _chk(lib().orc_faces(I64(nC), I64(nE), _p(tet), _p(f), _p(t2f), _p(sig), _p(f2t), _p(nbr), _p(cnt)))
    nF, nB = int(cnt[0]), int(cnt[1])
    return dict(nF=nF, nB=nB, faces=f[: 3 * nF].reshape(3, nF), tet2face=t2f, sigma=sig,
                face2tet=f2t[: 2 * nF].reshape(2, nF), nbr=nbr)


def refine(coord, tet, db=None, nb=None):
    coord = _f64(coord)
    tet = _i32(tet)
    nC, nE = coord.shape[1], tet.shape[1]
    db = np.zeros((3, 0), np.int32) if db is None else _i32(db)
    nb = np.zeros((3, 0), np.int32) if nb is None else _i32(nb)
    Xo = np.zeros(3 * (nC + 7 * nE), np.float64)
    To = np.zeros((4, 12 * nE), np.int32)
    dbo = np.zeros((3, 4 * db.shape[1]), np.int32)
    nbo = np.zeros((3, 4 * nb.shape[1]), np.int32)
    n = I64()
    _chk(lib().orc_refine(I64(nC), _p(coord), I64(nE), _p(tet), I64(db.shape[1]), _p(db), I64(nb.shape[1]),
                          _p(nb), _p(Xo), _p(To), _p(dbo), _p(nbo), C.byref(n)))
    nCo = n.value
    return Xo[: 3 * nCo].reshape(3, nCo), To, dbo, nbo


def local(coord, tet, sigma, kappa, prm):
    coord, tet = _f64(coord), _i32(tet)
    nC, nE = coord.shape[1], tet.shape[1]
    sigma = None if sigma is None else np.ascontiguousarray(sigma, np.int8)
    kappa = None if kappa is None else _f64(kappa)
    out = dict(vol=np.zeros(nE), K=np.zeros((16, nE)), d=np.zeros((4, nE)), B=np.zeros((4, nE)),
               S=np.zeros((16, nE)), r=np.zeros((4, nE)))
    _chk(lib().orc_local(I64(nC), _p(coord), I64(nE), _p(tet), _p(sigma), _p(kappa), C.byref(prm),
                         _p(out["vol"]), _p(out["K"]), _p(out["d"]), _p(out["B"]), _p(out["S"]), _p(out["r"])))
    return out


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def condense(coord, tet, conn, kappa, prm, neumann=None):
    """CSR of S+ (diagonal included) as scipy.sparse.csr_matrix, and rhs.  With `neumann`
    (nF flags, 1 = face on Gamma_N) the system is the paper's reduced one over the other faces
    (RFaces, face order) and (A, rhs, rfaces) is returned, rfaces[f] = row of face f or -1."""
    coord, tet = _f64(coord), _i32(tet)
    nC, nE = coord.shape[1], tet.shape[1]
    nF = conn["nF"]
    kappa = None if kappa is None else _f64(kappa)
    nm = _u8(neumann)
    rowptr = np.zeros(nF + 1, np.int32)
    col = np.zeros(7 * nF, np.int32)
    val = np.zeros(7 * nF)
    rhs = np.zeros(nF)
    rfaces = np.zeros(nF, np.int32)
    n, L = I64(), I64()
    _chk(lib().orc_condense(I64(nC), _p(coord), I64(nE), _p(tet), I64(nF), _p(_i32(conn["tet2face"])),
                            _p(np.ascontiguousarray(conn["sigma"], np.int8)), _p(_i32(conn["face2tet"])),
                            _p(_i32(conn["faces"])), _p(kappa), C.byref(prm), _p(nm), _p(rowptr), _p(col), _p(val),
                            _p(rhs), _p(rfaces), C.byref(n), C.byref(L)))
    nnz, L = n.value, L.value
    A = sp.csr_matrix((val[:nnz].copy(), col[:nnz].copy(), rowptr[:L + 1].copy()), shape=(L, L))
    if neumann is None:
        return A, rhs[:L]
    return A, rhs[:L].copy(), rfaces


def pcg(A, b, tol=1e-13, maxit=100000):
    A = A.tocsr()
    n = A.shape[0]
    x = np.zeros(n)
    it = C.c_int32()
    rr = C.c_double()
    rc = lib().orc_pcg(I64(n), _p(_i32(A.indptr)), _p(_i32(A.indices)), _p(_f64(A.data)), _p(_f64(b)),
                       C.c_double(tol), C.c_int32(maxit), _p(x), C.byref(it), C.byref(rr))
    _chk(rc)
    return x, it.value, rr.value


def recover(coord, tet, conn, kappa, prm, lam, neumann=None):
    """U(T) = A^-1 (B + LN + C' lambda) with lambda [nF] (entries on Gamma_N are not read)."""
    coord, tet = _f64(coord), _i32(tet)
    nC, nE = coord.shape[1], tet.shape[1]
    kappa = None if kappa is None else _f64(kappa)
    U = np.zeros((4, nE))
    _chk(lib().orc_recover(I64(nC), _p(coord), I64(nE), _p(tet), _p(_i32(conn["tet2face"])),
                           _p(np.ascontiguousarray(conn["sigma"], np.int8)), _p(kappa), C.byref(prm),
                           _p(_u8(neumann)), _p(None if lam is None else _f64(lam)), _p(U)))
    return U


def dense_solve(coord, tet, conn, kappa, prm, neumann=None):
    coord, tet = _f64(coord), _i32(tet)
    nC, nE = coord.shape[1], tet.shape[1]
    nF = conn["nF"]
    kappa = None if kappa is None else _f64(kappa)
    U = np.zeros((4, nE))
    lam = np.zeros(nF)
    _chk(lib().orc_dense_solve(I64(nC), _p(coord), I64(nE), _p(tet), I64(nF), _p(_i32(conn["tet2face"])),
                               _p(np.ascontiguousarray(conn["sigma"], np.int8)), _p(_i32(conn["face2tet"])),
                               _p(_i32(conn["faces"])), _p(kappa), C.byref(prm), _p(_u8(neumann)), _p(U),
                               _p(lam)))
    return U, lam


def adjoint(coord, tet, conn, kappa, prm, U, lam, gbar, tol=1e-13, maxit=100000):
    coord, tet = _f64(coord), _i32(tet)
    nC, nE = coord.shape[1], tet.shape[1]
    nF = conn["nF"]
    kappa = None if kappa is None else _f64(kappa)
    dlogk = np.zeros(nE)
    dX = np.zeros((3, nC))
    Q = np.zeros(nF)
    P = np.zeros((4, nE))
    it = C.c_int32()
    _chk(lib().orc_adjoint(I64(nC), _p(coord), I64(nE), _p(tet), I64(nF), _p(_i32(conn["tet2face"])),
                           _p(np.ascontiguousarray(conn["sigma"], np.int8)), _p(_i32(conn["face2tet"])),
                           _p(_i32(conn["faces"])), _p(kappa), C.byref(prm), _p(_f64(U)), _p(_f64(lam)),
                           _p(_f64(gbar)), C.c_double(tol), C.c_int32(maxit), _p(dlogk), _p(dX), _p(Q), _p(P),
                           C.byref(it)))
    return dict(dlogk=dlogk, dX=dX, Q=Q, P=P, iters=it.value)


def errors(coord, tet, conn, kappa, prm, U, lam, u_kind, u_par, h, nq=6, neumann=None):
    coord, tet = _f64(coord), _i32(tet)
    nC, nE = coord.shape[1], tet.shape[1]
    kappa = None if kappa is None else _f64(kappa)
    par = np.zeros(4)
    par[: len(u_par)] = u_par
    out = np.zeros(3)
    _chk(lib().orc_errors(I64(nC), _p(coord), I64(nE), _p(tet), _p(_i32(conn["tet2face"])),
                          _p(np.ascontiguousarray(conn["sigma"], np.int8)), _p(kappa), C.byref(prm),
                          _p(_u8(neumann)), _p(_f64(U)), _p(_f64(lam)), C.c_int32(u_kind), _p(par), C.c_double(h),
                          C.c_int32(nq), _p(out)))
    return dict(grad2=out[0], l22=out[1], lam_h2=out[2])


def tet_rule(n):
    m = n ** 3
    pts = np.zeros((3, m))
    w = np.zeros(m)
    _chk(lib().orc_tet_rule(C.c_int32(n), _p(pts), _p(w)))
    return pts, w


def tri_rule(n):
    m = n ** 2
    pts = np.zeros((2, m))
    w = np.zeros(m)
    _chk(lib().orc_tri_rule(C.c_int32(n), _p(pts), _p(w)))
    return pts, w


def connect(nC, tet):
    """Edges + faces of a mesh in one dict (oracle numbering)."""
    d = edges(nC, tet)
    d.update(faces(nC, tet))
    return d


def solve(coord, tet, kappa, prm, tol=1e-13, maxit=100000, neumann_faces=None):
    """Connect, condense, PCG, recover.  Returns (conn, A, rhs, lam, U, iters).  neumann_faces:
    optional boundary face list [3][n] (node triples, any orientation) on Gamma_N; lam [nF]
    then holds the solved multipliers on the other faces and 0 on Gamma_N."""
    conn = connect(coord.shape[1], tet)
    nm = None if neumann_faces is None else neumann_flags(conn, neumann_faces)
    if nm is None:
        A, rhs = condense(coord, tet, conn, kappa, prm)
        lam, it, _ = pcg(A, rhs, tol, maxit)
    else:
        A, rhs, rf = condense(coord, tet, conn, kappa, prm, nm)
        lr, it, _ = pcg(A, rhs, tol, maxit)
        lam = np.zeros(conn["nF"])
        lam[rf >= 0] = lr[rf[rf >= 0]]
    U = recover(coord, tet, conn, kappa, prm, lam, nm)
    return conn, A, rhs, lam, U, it


def neumann_flags(conn, tris):
    """nF flags (uint8): 1 for the faces whose node sets appear in tris [3][n]."""
    F = np.asarray(conn["faces"])
    key = {tuple(sorted(F[:, f])): f for f in range(F.shape[1])}
    nm = np.zeros(F.shape[1], np.uint8)
    for j in range(np.asarray(tris).shape[1]):
        nm[key[tuple(sorted(np.asarray(tris)[:, j]))]] = 1
    return nm
