#!/usr/bin/env python3
"""Throughput of the primal hybrid FEM hot path on one MI355X.

Headline (one JSON line on stdout): tets/s of refine + connect + condensed assembly
(12-subtet refinement per level with edge connectivity, full connectivity at the final
level, local matrices + element Schur + FP64 face system) on the Kuhn cube refined 6 times
(17,915,904 tets), mixed precision, inputs resident on the GPU.  One step = the whole
pipeline from the 6-tet level-0 mesh.  The same pipeline in FP64 is timed beside it, and
the face solve, recovery and adjoint (timed separately, not in the headline) on the 5-level
cube.  The roofline object is computed from HIP events around every launch of the
dominant kernel in the timed region; cpu_baseline times the CPU oracle on a smaller mesh.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kuhn_counts(L):
    """(nE, nC, nEd, nF, nB) of the Kuhn cube after L levels (size recurrences of the split)."""
    nE, nC, nEd, nF, nB = 6, 8, 19, 18, 12
    for _ in range(L):
        nE, nC, nEd, nF, nB = 12 * nE, nC + nEd + nE, 2 * nEd + 3 * nF + 6 * nE, 4 * nF + 16 * nE, 4 * nB
    return nE, nC, nEd, nF, nB


def section8d_rows(L):
    """Compulsory bytes of the pipeline by stage, each input read once and each output written
    once, with the arrays' own sizes (the per-tet figures of the hot-path measurement plan,
    evaluated with the exact counts of the Kuhn cube at level L; kappa constant, so no kappa
    array is read).  Returns {stage: bytes}."""
    nE, nC, nEd, nF, nB = kuhn_counts(L)
    cE, cC, cEd, cF, cB = kuhn_counts(L - 1)
    rows = {}
    # refinement of level L-1 to L: coarse tets, tet->edge, coordinates, edge/tet prefix in;
    # refined tets and the new coordinates out
    rows["refine"] = 16 * cE + 24 * cE + 24 * cC + 4 * cEd + 4 * cE + 16 * nE + 24 * (cEd + cE)
    # connectivity of level L: tets in; edges, tet->edge, tet->face + sigma (4 bits), faces,
    # face->tet out
    rows["connect"] = 16 * nE + 8 * nEd + 24 * nE + 16.5 * nE + 12 * nF + 8 * nF
    # edge connectivity of the levels below L (tets in, edges and tet->edge out)
    rows["connect_lower"] = sum(16 * e + 24 * e + 8 * ed for e, _, ed, _, _ in (kuhn_counts(l) for l in range(L)))
    # assembly + condensation: tets, coordinates, tet->face + sigma in; the face system out
    # (values and column ids of nnz = 7 nI + 4 nB entries with the diagonal, row pointers, rhs)
    nnz = 7 * (nF - nB) + 4 * nB
    rows["condense"] = 16 * nE + 24 * nC + 16.5 * nE + 8 * nnz + 4 * nnz + 4 * (nF + 1) + 8 * nF
    return rows


def compulsory_bytes(L):
    return sum(section8d_rows(L).values())


# The dominant kernels' share of those compulsory bytes per launch at the final level: the
# tile pass of the condensation reads the mesh and writes the whole face system (the
# "condense" row); the second refinement-connectivity pass writes the refined mesh's
# connectivity (the "connect" row less its tet reads, which the derived path does not make).
def kernel_8d_bytes(name, L):
    rows = section8d_rows(L)
    nE = kuhn_counts(L)[0]
    if name.startswith("cond_tile"):
        return rows["condense"]
    if name == "refconn_pass2":
        return rows["connect"] - 16 * nE
    if name == "refine":
        return rows["refine"]
    return None


def run_pipeline(P, X0, T0, db0, L, prm, kappa=None, sort_connect=False, status=None):
    """One step.  Default: the level-0 mesh is connected by the general sort-based connect,
    every refinement level derives the refined mesh's connectivity in closed form
    (phfem_refine_connected), then assemble + condense.  sort_connect=True: per level
    connect-edges (sort) -> refine (with the Dirichlet face list), then a sort-based full
    connect of the final mesh.  status: a zeroed device int32 that the refinement's input
    check ORs its code into (every step still runs the check; the host reads the flag after
    the timed steps instead of synchronizing inside each one)."""
    if sort_connect:
        X, T, db = X0, T0, db0
        for _ in range(L):
            conn = P.connect(T, X.shape[1], faces=False, n2e=True)
            X, T, db, _ = P.refine(X, T, conn, db)
        conn = P.connect(T, X.shape[1], faces=True)
    else:
        X, T, conn = P.refine_connected_levels(X0, T0, L, status=status)
    sysm = P.condense(X, T, conn, kappa, prm)
    return X, T, conn, sysm


def time_pipeline(torch, P, B, X0, T0, db0, L, prm, steps, warmup, profile, sort_connect=False):
    """ms per step (HIP events around `steps` steps, profiler off), the median of the steps'
    own event times, host wall ms per step, and -- from a second, separately run set of
    `steps` steps with the per-launch event profiler on -- per-kernel launches / ms /
    algorithmic bytes."""
    st = torch.zeros(1, dtype=torch.int32, device=X0.device)
    for _ in range(warmup):
        run_pipeline(P, X0, T0, db0, L, prm, sort_connect=sort_connect, status=st)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        out = run_pipeline(P, X0, T0, db0, L, prm, sort_connect=sort_connect, status=st)
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev[0].elapsed_time(ev[-1]) / steps
    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    med = per[len(per) // 2] if steps % 2 else 0.5 * (per[len(per) // 2 - 1] + per[len(per) // 2])
    P.check_status(st)  # every step's refinement input check, read once
    kern = {}
    if profile:
        del out
        B.phfem_profile_reset()
        B.phfem_profile_enable(True)
        for _ in range(steps):
            out = run_pipeline(P, X0, T0, db0, L, prm, sort_connect=sort_connect, status=st)
        torch.cuda.synchronize()
        B.phfem_profile_enable(False)
        P.check_status(st)
        for name in B.phfem_profile_names():
            n, tms, by = B.phfem_profile_query(name)
            kern[name] = dict(launches=n, ms=tms, bytes=by)
    return ms, med, wall / steps * 1e3, kern, out


def stages(kern, steps):
    """Per-stage ms per step from the profiled kernels: the condensation (AoS coordinates and
    both condensation passes) and everything before it (refinement, connectivity, scans)."""
    out = {"refine_connect": 0.0, "assemble_condense": 0.0}
    for k, v in kern.items():
        key = "assemble_condense" if k.startswith("cond_") or k == "coords_aos" else "refine_connect"
        out[key] += v["ms"] / steps
    return {k: round(v, 4) for k, v in out.items()}


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from the
    committed rocprofv3 summary, or None when the kernel's source changed since then."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        t = json.load(open(os.path.join(here, "profiles", "traffic_kuhn_L6.json")))
        k = t["kernels"][kernel]
        src = os.path.join(here, "paper_2509_11133_amd", "csrc", k["source"])
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != t["source_sha256"][k["source"]]:
            return None
        return round(k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def pipeline_traffic(kern, steps):
    """Measured HBM bytes per step of the whole pipeline: each kernel's launches per step x
    its measured bytes per launch.  None unless every kernel with >= 1 % of the step time has a
    current measurement (the small rest is left out, so the figure is a lower bound)."""
    total_ms = sum(v["ms"] for v in kern.values())
    tot = 0.0
    for name, v in kern.items():
        b = measured_traffic(name)
        if b is None:
            if v["ms"] >= 0.01 * total_ms:
                return None
            continue
        tot += b * v["launches"] / max(steps, 1)
    return tot


def roofline(kern, steps, L):
    """The dominant kernel (largest summed HIP-event time in the profiled pass) against HBM
    peak: achieved = its compulsory bytes per launch at the final level (kernel_8d_bytes) / its
    average launch time (of the final-level launches: the kernels that run once per step)."""
    name, k = max(kern.items(), key=lambda kv: kv[1]["ms"])
    b8 = kernel_8d_bytes(name, L)
    per_step = k["launches"] // max(steps, 1)
    avg = k["ms"] / max(k["launches"], 1)
    if b8 is None or per_step != 1:
        return name, None
    gbs = b8 / (avg * 1e-3) / 1e9
    return name, dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(gbs / HBM_PEAK_GBS, 4), traffic=measured_traffic(name), kernel=name,
                      launches_per_step=per_step, avg_launch_ms=round(avg, 5), algorithmic_bytes_per_launch=b8,
                      kernel_bytes_per_launch=k["bytes"] / max(k["launches"], 1),
                      note="algorithmic bytes: the compulsory reads and writes of what the kernel produces "
                           "(mesh in, face system out); kernel_bytes_per_launch adds its own intermediates; "
                           "traffic: rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, scaled by the "
                           "library's calibration streams")


def cpu_baseline(levels, runs=3):
    """The oracle (single-threaded FP64 C++) on the same pipeline at a smaller level: the median
    of `runs` runs."""
    import numpy as np

    import oracle as O
    from paper_2509_11133_amd import meshes as M

    O.build()
    X, T = M.kuhn_cube()
    db = M.boundary_faces_box(X, T)
    prm = O.params(c=1.0, kappa=1.0, f=(O.FUN_SIN3, (M.SIN3_AMPLITUDE,)))
    # one thread pinned to one core (this process's affinity, restored afterwards)
    aff = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    core = min(aff) if aff else None
    if aff:
        os.sched_setaffinity(0, {core})
    X0, T0, db0 = X, T, db
    times = []
    try:
        for _ in range(runs):
            X, T, db = X0, T0, db0
            t0 = time.perf_counter()
            for _ in range(levels):
                O.edges(X.shape[1], T)
                X, T, db, _ = O.refine(X, T, db)
            conn = O.connect(X.shape[1], T)
            O.condense(X, T, conn, None, prm)
            times.append(time.perf_counter() - t0)
            del conn
    finally:
        if aff:
            os.sched_setaffinity(0, aff)
    dt = sorted(times)[len(times) // 2]
    nE = T.shape[1]
    del np
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=round(nE / dt, 1), unit="tets/s", cores=1, kind="oracle",
                host_cpu=cpu, host_cores=os.cpu_count(), pinned_core=core,
                runs_s=[round(t, 3) for t in times],
                sample=f"Kuhn cube, {levels} levels ({nE} tets): edges+refine per level, full connectivity, "
                       f"condensed assembly; FP64, 1 thread pinned to one core; median of {runs} runs {dt:.2f} s")


def solve_block(torch, P, B, M, Ls):
    """a8-a10 time-to-solution on the Kuhn cube at Ls levels (FP64 PCG, mixed IR, adjoint)."""
    dev = torch.device("cuda:0")
    X0, T0 = M.kuhn_cube()
    X, T, _ = P.refine_levels(torch.tensor(X0, device=dev), torch.tensor(T0, device=dev), Ls)
    conn = P.connect(T, X.shape[1])
    out = {"workload": f"Kuhn cube, {Ls} levels ({T.shape[1]} tets, {conn['nF']} faces), tol 1e-10"}
    for label, prec, mode in (("fp64_pcg", B.FP64, B.SOLVE_FP64_PCG), ("mixed_ir", B.MIXED, B.SOLVE_FP32_PCG_FP64_IR)):
        prm = P.params(c=1.0, kappa=1.0, f=(B.FUN_SIN3, (M.SIN3_AMPLITUDE,)), precision=prec)
        sysm = P.condense(X, T, conn, None, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, U, st = P.solve(X, T, conn, sysm, None, prm, mode=mode, tol=1e-10, inner_tol=0.9, max_iter=400000,
                             allow_noconv=True)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        t0 = time.perf_counter()
        dlogk, dX, st2 = P.grad(X, T, conn, sysm, None, prm, U, lam, U, mode=mode, tol=1e-10, inner_tol=0.9,
                                max_iter=400000)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        out[label] = dict(solve_ms=round(ts * 1e3, 1), iters=st["iters"], ir_steps=st["ir_steps"],
                          rel_res=st["rel_res"], converged=st["converged"], grad_ms=round(tg * 1e3, 1),
                          grad_iters=st2["iters"])
        log(label, out[label])
    return out


def reassembly_block(torch, P, B, M, X0d, T0d, L, reps=5, nk=4):
    """Pattern reuse and batched coefficients on the final mesh (mixed precision): a full
    condense (pattern + values), values-only re-assembly of one lognormal kappa field, and a
    values-only batch of nk fields; ms per call (HIP events, mean of reps) and tets/s per field."""
    X, T, conn = P.refine_connected_levels(X0d, T0d, L)
    nE = T.shape[1]
    K = torch.tensor(M.lognormal_kappa_fields(nE, nk, 1.0), device=X.device)
    prm = P.params(c=1.0, kappa=1.0, f=(B.FUN_SIN3, (M.SIN3_AMPLITUDE,)), precision=B.MIXED)
    first = P.condense(X, T, conn, K[0].contiguous(), prm)
    pat = (first["rowptr"], first["col"])
    k1 = K[:1].contiguous()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        del out
        return e0.elapsed_time(e1) / reps

    full = timed(lambda: P.condense(X, T, conn, K[0].contiguous(), prm))
    vals = timed(lambda: P.condense_batch(X, T, conn, k1, prm, pattern=pat))
    batch = timed(lambda: P.condense_batch(X, T, conn, K, prm, pattern=pat))
    out = {"workload": f"Kuhn cube, {L} levels ({nE} tets), mixed precision, lognormal kappa (sigma 1)",
           "condense_ms": round(full, 4), "values_only_ms": round(vals, 4), f"batch{nk}_values_only_ms": round(batch, 4),
           "condense_tets_per_s": round(nE / (full * 1e-3), 1),
           "values_only_tets_per_s": round(nE / (vals * 1e-3), 1),
           f"batch{nk}_tets_per_s_per_field": round(nk * nE / (batch * 1e-3), 1)}
    log("reassembly", out)
    return out


def general_connect_block(torch, P, X0d, T0d, L, reps=3):
    """phfem_connect (edges + faces) on the final mesh, which the benchmark step connects in
    closed form instead: ms per call through the node buckets and through the radix sort
    (HIP events, mean of reps after one untimed call); both outputs checked against the
    derived connectivity."""
    X, T, conn = P.refine_connected_levels(X0d, T0d, L)
    nC, nE = X.shape[1], T.shape[1]
    out = {"workload": f"Kuhn cube, {L} levels ({nE} tets), edges + faces"}
    for radix in (False, True):
        g = P.connect(T, nC, faces=True, radix=radix)
        for k in ("edges", "tet2edge", "faces", "tet2face", "sigma", "face2tet", "nbr"):
            assert torch.equal(g[k], conn[k]), k
        del g
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            P.connect(T, nC, faces=True, radix=radix)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out["radix_ms" if radix else "bucket_ms"] = round(ms, 4)
        if not radix:
            out["bucket_tets_per_s"] = round(nE / (ms * 1e-3), 1)
    log("general connect", out)
    return out


def rows_block(torch, P, B, M, X0d, T0d, L, reps=3, iters=300):
    """Each stage of the path on its own at the final level, against HBM peak on its compulsory
    bytes: the last refinement with derived connectivity (level L-1 -> L), the condensation in
    both precisions, one PCG iteration of each solver on the L face system (mean over `iters`
    iterations of its two kernels) and the recovery of u_h.  Per stage: the kernels' HIP-event
    ms (profiler on), the compulsory bytes and bytes / time / 8 TB/s."""
    nE, nC, nEd, nF, nB = kuhn_counts(L)
    rows8 = section8d_rows(L)
    out = {"workload": f"Kuhn cube, level {L} ({nE} tets, {nF} faces); kernel times from the library's event "
                       f"profiler, mean of {reps} calls (PCG: of {iters} iterations)"}

    def profiled(fn, n):
        B.phfem_profile_reset()
        B.phfem_profile_enable(True)
        for _ in range(n):
            r = fn()
        torch.cuda.synchronize()
        B.phfem_profile_enable(False)
        return r, {k: B.phfem_profile_query(k) for k in B.phfem_profile_names()}

    def row(kern, names, nbytes, calls):
        ms = sum(kern[k][1] for k in kern if k in names) / calls
        return {"kernels": sorted(k for k in kern if k in names), "ms": round(ms, 4), "compulsory_bytes": round(nbytes),
                "frac": round(nbytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}

    Xc, Tc, cc = P.refine_connected_levels(X0d, T0d, L - 1)
    (X, T, conn), kern = profiled(lambda: P.refine_connected(Xc, Tc, cc), reps)
    out["refine_connect"] = row(kern, set(kern), rows8["refine"] + rows8["connect"], reps)
    out["refine_connect"]["note"] = "refine + connect rows (the derived path reads no refined tets: an upper bound)"
    del Xc, Tc, cc
    f = (B.FUN_SIN3, (M.SIN3_AMPLITUDE,))
    for label, prec, mode, bpf in (("mixed", B.MIXED, B.SOLVE_FP32_PCG_FP64_IR, 92.0),
                                   ("fp64", B.FP64, B.SOLVE_FP64_PCG, 168.0)):
        prm = P.params(c=1.0, kappa=1.0, f=f, precision=prec)
        sysm, kern = profiled(lambda: P.condense(X, T, conn, None, prm), reps)
        out[f"condense_{label}"] = row(kern, set(kern), rows8["condense"], reps)
        torch.cuda.synchronize()
        B.phfem_profile_reset()
        B.phfem_profile_enable(True)
        P.solve(X, T, conn, sysm, None, prm, mode=mode, tol=1e-30, max_iter=iters, allow_noconv=True)
        torch.cuda.synchronize()
        B.phfem_profile_enable(False)
        kern = {k: B.phfem_profile_query(k) for k in B.phfem_profile_names()}
        it = {k: kern[k][1] / kern[k][0] for k in ("spmv_dir", "pcg_update") if k in kern and kern[k][0]}
        ms = sum(it.values())
        out[f"pcg_iteration_{label}"] = {"kernels": sorted(it), "ms": round(ms, 4), "bytes_per_face": bpf,
                                         "compulsory_bytes": round(bpf * nF),
                                         "frac": round(bpf * nF / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
        if label == "fp64" and "recover" in kern:
            rb = 16 * nE + 16 * nE + 4 * nE + 24 * nC + 8 * nF + 32 * nE  # tets, faces, sigma, coords, lambda in; U out
            rms = kern["recover"][1] / kern["recover"][0]
            out["recover"] = {"kernels": ["recover"], "ms": round(rms, 4), "compulsory_bytes": rb,
                              "frac": round(rb / (rms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
        del sysm
        torch.cuda.empty_cache()
    log("rows", out)
    return out


# The paper's own timings (MATLAB R2025a, vectorized, FP64, on an Intel Core i5-10210U), level
# 5 of its 5-tet cube (1,244,160 tets): Table 1 (connectivity and refinement) and Table 2
# (local matrices), in seconds.  Another machine and another program: context, not a target.
PAPER_L5 = {"cpu": "Intel Core i5-10210U, MATLAB R2025a (vectorized, FP64)", "tets": 1244160,
            "FacesUp_s": 3.7920, "NumEdges_s": 1.0248, "EdgeNum2Tetra_s": 2.7785, "RedRefine_s": 0.5407,
            "StiffMassPH_s": 4.2434, "Multiplier_s": 4.5835}


def paper_mesh_block(torch, P, B, M, L=5, reps=5):
    """The paper's 5-tet cube refined to its Table 1/2 level 5 (1,244,160 tets), through the
    same GPU pipeline as the headline (connect of level 0, refined connectivity per level,
    condense), FP64 and mixed, beside the paper's level-5 MATLAB timings (context only: the
    paper's times cover one level's connectivity / refinement and the local matrices)."""
    dev = torch.device("cuda:0")
    X0, T0, _, _ = M.paper_cube()
    X0d, T0d = torch.tensor(X0, device=dev), torch.tensor(T0, device=dev)
    out = {"workload": f"the paper's 5-tet cube (Section 2.3), {L} levels, sin^3 load, all faces Dirichlet"}
    for label, prec in (("fp64", B.FP64), ("mixed", B.MIXED)):
        prm = P.params(c=1.0, kappa=1.0, f=(B.FUN_SIN3, (M.SIN3_AMPLITUDE,)), precision=prec)
        st = torch.zeros(1, dtype=torch.int32, device=dev)
        run_pipeline(P, X0d, T0d, None, L, prm, status=st)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            res = run_pipeline(P, X0d, T0d, None, L, prm, status=st)
        e1.record()
        torch.cuda.synchronize()
        P.check_status(st)
        nE = res[1].shape[1]
        ms = e0.elapsed_time(e1) / reps
        out[label] = {"ms": round(ms, 4), "tets_per_s": round(nE / (ms * 1e-3), 1)}
        del res
    out["nE"] = nE
    paper_s = sum(v for k, v in PAPER_L5.items() if k.endswith("_s"))
    out["paper_matlab_level5"] = dict(PAPER_L5, sum_s=round(paper_s, 4),
                                      note="one level's connectivity + refinement + local matrices; other machine")
    log("paper mesh", out)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--solve-levels", type=int, default=5)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-levels", type=int, default=5)
    ap.add_argument("--no-profile", action="store_true", help="skip the profiled pass (per-kernel HIP events)")
    ap.add_argument("--no-sort-variant", action="store_true",
                    help="skip the general-connect comparisons (pipeline with phfem_connect at every level, "
                         "connect of the final mesh)")
    ap.add_argument("--no-reassembly", action="store_true", help="skip the pattern-reuse / batched-kappa timings")
    ap.add_argument("--no-rows", action="store_true", help="skip the per-stage roofline table at the final level")
    ap.add_argument("--no-paper-mesh", action="store_true", help="skip the paper's 5-tet cube timings")
    ap.add_argument("--connect-only", action="store_true",
                    help="only the general connect of the final mesh (node buckets, then radix sort); one JSON line")
    ap.add_argument("--calibrate", action="store_true",
                    help="only run the library's calibration streams (1 GiB read, 1 GiB write, 1 GiB copy, "
                         "2^25 scattered 32-byte records gathered from a 2 GiB array), each twice, and exit: "
                         "profiled with FETCH_SIZE / WRITE_SIZE they give the counters' scale")
    args = ap.parse_args()
    if args.calibrate:
        import torch

        from paper_2509_11133_amd import _binding as B
        n = 1 << 27  # doubles: 1 GiB
        a = torch.ones(2 * n, dtype=torch.float64, device="cuda")  # 2 GiB (2^26 records of 32 B)
        b = torch.empty(n, dtype=torch.float64, device="cuda")
        part = torch.empty(4096, dtype=torch.float64, device="cuda")
        for _ in range(2):
            B.phfem_profile_stream(0, a, part, n)
            B.phfem_profile_stream(1, None, b, n)
            B.phfem_profile_stream(2, a, b, n)
            B.phfem_profile_stream(3, a, part, 1 << 25, 1 << 26)
        torch.cuda.synchronize()
        print(json.dumps({"cal_read": 8 * n, "cal_write": 8 * n, "cal_copy_read": 8 * n, "cal_copy_write": 8 * n,
                          "cal_gather_requested": 32 << 25, "repeats": 2}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only: the hot path runs on a single MI355X; "
                                   "run with --gpus 1"}))
        sys.exit(2)

    import torch

    from paper_2509_11133_amd import _binding as B
    from paper_2509_11133_amd import meshes as M
    from paper_2509_11133_amd import pipeline as P

    B.lib()
    dev = torch.device("cuda:0")
    X0, T0 = M.kuhn_cube()
    db0 = M.boundary_faces_box(X0, T0)
    X0d, T0d, db0d = (torch.tensor(a, device=dev) for a in (X0, T0, db0))
    L = args.levels
    if args.connect_only:
        print(json.dumps(general_connect_block(torch, P, X0d, T0d, L)), flush=True)
        return
    nE, nC, nEd, nF, nB = kuhn_counts(L)
    f = (B.FUN_SIN3, (M.SIN3_AMPLITUDE,))
    res = {}
    for label, prec, sortc in (("mixed", B.MIXED, False), ("fp64", B.FP64, False), ("mixed_sort", B.MIXED, True)):
        if sortc and args.no_sort_variant:
            continue
        prm = P.params(c=1.0, kappa=1.0, f=f, precision=prec)
        ms, med, wall_ms, kern, out = time_pipeline(torch, P, B, X0d, T0d, db0d, L, prm, args.steps, args.warmup,
                                                    not args.no_profile, sort_connect=sortc)
        assert out[1].shape[1] == nE and out[2]["nF"] == nF
        res[label] = dict(ms=ms, med=med, wall_ms=wall_ms, kern=kern)
        log(f"{label}: {ms:.3f} ms/step, {nE / ms * 1e3:.4g} tets/s")
        del out
        torch.cuda.empty_cache()

    mixed, fp64 = res["mixed"], res["fp64"]
    value = nE / (mixed["ms"] * 1e-3)
    comp = compulsory_bytes(L)
    line = {
        "metric": "tets/s refine+connect+condensed assembly, mixed vs FP64 on 1 GPU; % HBM peak",
        "value": round(value, 1),
        "unit": "tets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["ms"], 4),
        "ms_per_step_median": round(mixed["med"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"Kuhn cube (6 tets) refined {L} times by the 12-subtet split -> {nE} tets, "
                               f"{nF} faces; general connect of level 0 (one workgroup), refine with derived connectivity per "
                               f"level, assemble + condense at the last level; mixed precision (FP32 local/Schur, "
                               f"FP64 dets and face system)",
                   "levels": L, "nE": nE, "nC": nC, "nEd": nEd, "nF": nF, "nnz_offdiag": 6 * nF - 3 * nB,
                   "stored_offdiag": 6 * nF},
        "fp64": {"value": round(nE / (fp64["ms"] * 1e-3), 1), "ms_per_step": round(fp64["ms"], 4),
                 "ms_per_step_median": round(fp64["med"], 4), "mixed_speedup": round(fp64["ms"] / mixed["ms"], 3)},
        "useful_hbm_frac": round(comp / (mixed["ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "compulsory_bytes_per_step": comp,
    }
    if "mixed_sort" in res:
        ms_ = res["mixed_sort"]
        line["sort_connect_pipeline"] = {
            "value": round(nE / (ms_["ms"] * 1e-3), 1), "ms_per_step": round(ms_["ms"], 4),
            "ms_per_step_median": round(ms_["med"], 4),
            "note": "same workload with the general connect (phfem_connect) at every level instead of the "
                    "derived connectivity",
            "kernels_ms_per_step": {k: round(v["ms"] / args.steps, 4)
                                    for k, v in sorted(ms_["kern"].items(), key=lambda kv: -kv[1]["ms"])[:8]}}
    if mixed["kern"]:
        name, rl = roofline(mixed["kern"], args.steps, L)
        line["roofline"] = rl
        line["compulsory_bytes_by_stage"] = {k: round(v) for k, v in section8d_rows(L).items()}
        pt = pipeline_traffic(mixed["kern"], args.steps)
        line["achieved_hbm_frac"] = None if pt is None else round(pt / (mixed["ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
        line["measured_bytes_per_step"] = None if pt is None else round(pt)
        line["stages_ms_per_step"] = stages(mixed["kern"], args.steps)
        line["fp64"]["stages_ms_per_step"] = stages(fp64["kern"], args.steps)
        line["kernels_ms_per_step"] = {k: round(v["ms"] / args.steps, 4)
                                       for k, v in sorted(mixed["kern"].items(), key=lambda kv: -kv[1]["ms"])}
        line["fp64"]["kernels_ms_per_step"] = {k: round(v["ms"] / args.steps, 4)
                                               for k, v in sorted(fp64["kern"].items(), key=lambda kv: -kv[1]["ms"])}
    if not args.no_sort_variant:
        line["general_connect"] = general_connect_block(torch, P, X0d, T0d, L)
        gc = line["general_connect"]
        gc["frac"] = round(section8d_rows(L)["connect"] / (gc["bucket_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
        torch.cuda.empty_cache()
    if not args.no_rows:
        line["rows_roofline"] = rows_block(torch, P, B, M, X0d, T0d, L)
        torch.cuda.empty_cache()
    if not args.no_reassembly:
        line["reassembly"] = reassembly_block(torch, P, B, M, X0d, T0d, L)
        torch.cuda.empty_cache()
    if not args.no_paper_mesh:
        line["paper_mesh"] = paper_mesh_block(torch, P, B, M)
        torch.cuda.empty_cache()
    if not args.no_solve:
        line["solve"] = solve_block(torch, P, B, M, args.solve_levels)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_levels)
        line["cpu_baseline"]["speedup_gpu_over_cpu"] = round(value / line["cpu_baseline"]["value"], 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
