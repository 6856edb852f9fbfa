#!/usr/bin/env python
"""Benchmark of the EFIE hot path on one MI355X.

Workload (default): PEC unit sphere, icosphere level 5 (T = 20480 triangles,
N = 30720 RWG unknowns), k = 10 rad/m, 512 plane waves on the uniform
16 (theta) x 32 (phi) grid, incidence from rhat with theta-hat polarisation,
monostatic observation.  Mixed precision: complex64 operator (far pairs in
FP32, near pairs in FP64), COCG with Z X on FP32 matrix cores, FP64 outer
refinement to ||V - Z J|| <= 1e-6 ||V|| per right-hand side.

One step = the whole hot path on inputs already resident in HBM:
assembly (far + near), excitation of the 512 right-hand sides, the Calderon
preconditioner P = T_BC(k~) G_mix^-1 (barycentric second operator at the complex
wavenumber, mixed Gram inverse), the preconditioned multi-RHS solve (CGS on
P Z J = P V, complex64 Z and P on FP32 matrix cores, FP64 true-residual
refinement; --solver cocg: unpreconditioned COCG instead), and the far field in
the 512 monostatic directions.

Printed JSON line: `value` is the complex Z.X throughput (8 M N K real flops per
launch / mean launch time, HIP events around every launch inside the timed
steps), plus assembly Mentries/s and the time-to-solve; `roofline` describes
the dominant kernel (the matrix-core GEMM); `cpu_baseline` times the FP64
oracle's own Z.X (numpy) on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3      # TFLOP/s, MI355X dense FP32 matrix
PEAK_HBM = 8000.0           # GB/s
PEAK_FP32_VALU = 78.6       # TFLOP/s with FMA = 2 flops, packed FP32 disabled (256 CU x 64 lanes x 2.4 GHz x 2)
VALU_LANE_SLOTS = 256 * 64 * 2.4e9   # vector-ALU lane-instructions per second
# Algorithmic cost model of the assembly (vector ALU): 7 x 7 Green's-function
# evaluations per triangle pair, every ordered pair counted, i.e. 49 T^2 / N^2 per Z
# entry (21.8 on a closed surface, T = 2N/3); one evaluation costs about 46 FP32
# issue slots (4 transcendentals at quarter rate, about 30 FMA-class operations for
# R^2, the kernel and the moment sums) or about 110 in FP64 (no hardware sine and
# cosine).  The bound does not credit the symmetry Z = Z^T that the kernels use.
EVAL_SLOTS = {"c64": 46.0, "c128": 110.0}


def assembly_alu_peak(n, t, dtype):
    """Mentries/s at which the vector ALUs would finish the model's work."""
    return VALU_LANE_SLOTS / (49.0 * t * t / (n * n) * EVAL_SLOTS[dtype]) / 1e6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(level, n_sample_rows, nrhs, k, seconds):
    """FP64 oracle on the host: its Z.X product (numpy) on a row sample of the same
    shape, and its assembly on a few rows of the same mesh."""
    import numpy as np

    try:
        from threadpoolctl import threadpool_info

        threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    import synth
    from oracle import efie, rwg

    v, f = synth.icosphere(level)
    om = rwg.build(v, f)
    N = om.n
    rng = np.random.default_rng(0)
    rows = n_sample_rows
    Zs = rng.standard_normal((rows, N)) + 1j * rng.standard_normal((rows, N))
    X = rng.standard_normal((N, nrhs)) + 1j * rng.standard_normal((N, nrhs))
    t0 = time.perf_counter()
    reps = 0
    while True:
        Y = Zs @ X                       # the oracle's product (numpy/BLAS, complex128)
        reps += 1
        if time.perf_counter() - t0 > seconds * 0.6:
            break
    tz = (time.perf_counter() - t0) / reps
    gflops = 8.0 * rows * N * nrhs / tz / 1e9
    geo = efie.Geometry(om)
    t1 = time.perf_counter()
    nrow = 0
    while True:
        efie.z_rows(om, k, [nrow * 997 % N], geo=geo)
        nrow += 1
        if time.perf_counter() - t1 > seconds * 0.4:
            break
    ta = time.perf_counter() - t1
    phases = oracle_phases(np, k, nrhs)
    return {
        "value": round(gflops, 3),
        "unit": "GFLOP/s",
        "cores": int(threads),
        "cpu_model": cpu_model(),
        "cores_available": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count(),
        "phases": phases,
        "kind": "oracle",
        "sample": (f"oracle Z.X (numpy complex128) of a {rows} x {N} row block of Z times {N} x {nrhs}, "
                   f"{reps} repetitions; oracle assembly of {nrow} rows of the level-{level} Z at k={k}: "
                   f"{nrow * N / ta / 1e6:.4f} Mentries/s on 1 core"),
        "assembly_mentries_per_s": round(nrow * N / ta / 1e6, 5),
    }


TRAFFIC_FILES = {False: os.path.join(ROOT, "profiles", "cgemm_planar_fp32acc_l5_k10_512rhs_hbm_traffic.md"),
                 True: os.path.join(ROOT, "profiles", "cgemm_planar_flush64_l5_k10_512rhs_hbm_traffic.md")}
GEMM_SOURCE = os.path.join(ROOT, "paper_2310_15644_amd", "csrc", "gemm_mfma.hip")


def gemm_code_sha256(path=None):
    """SHA-256 of the GEMM source with its // comments and all whitespace removed:
    the counters stay attached to the kernel code, not to the wording of its comments."""
    import hashlib
    import re

    text = open(path or GEMM_SOURCE).read()
    code = re.sub(r"//[^\n]*", "", text)
    code = re.sub(r"\s+", "", code)
    return hashlib.sha256(code.encode()).hexdigest()


def measured_traffic(tiles, acc64, n, nrhs, solver):
    """HBM bytes per launch of the in-solve matrix-core GEMM, from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE per dispatch, each divided
    by the factor the same counter reads for a plain 1 GiB copy).  The summary may
    hold one entry per tile; None when no entry is for the selected tile and this
    workload, or the GEMM code has changed since the counters were taken."""
    path = TRAFFIC_FILES[bool(acc64)]
    if tiles is None or not os.path.exists(path):
        return None, None
    from paper_2310_15644_amd import gemm_kernel_name

    entries = []
    for line in open(path):
        if line.startswith("- kernel:"):
            entries.append({})
        if entries and line.startswith("- ") and ": " in line:
            key, val = line[2:].split(": ", 1)
            entries[-1][key.strip()] = val.strip().strip("`")
    sha = gemm_code_sha256()
    want = gemm_kernel_name(tiles, acc64)
    for kv in entries:
        if (kv.get("gemm_code_sha256") == sha and kv.get("kernel") == want
                and kv.get("workload") == f"n={n} nrhs={nrhs} solver={solver}"):
            return float(kv["hbm_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


ASSEMBLY_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "assembly_tiles_l5_k10_hbm_traffic.md")
TILE_SOURCES = [os.path.join(ROOT, "paper_2310_15644_amd", "csrc", f)
                for f in ("tile_kernels.h", "pair_kernels.h", "rows_kernels.h")]
TILE_WRAPPER = os.path.join(ROOT, "paper_2310_15644_amd", "csrc", "assemble.hip")


def tile_code_sha256():
    """SHA-256 of the tile assembly's device code (comments and whitespace removed)."""
    import hashlib
    import re

    h = hashlib.sha256()
    codes = [open(path).read() for path in TILE_SOURCES]
    # the tile kernel's own definition (its launch bounds) in assemble.hip
    src = open(TILE_WRAPPER).read()
    i = src.index("void tile_kernel(")
    codes.append(src[src.rindex("template", 0, i):src.index("\n}\n", i) + 3])
    for code in codes:
        code = re.sub(r"//[^\n]*", "", code)
        h.update(re.sub(r"\s+", "", code).encode())
    return h.hexdigest()


def _assembly_entry(n, k, dtype, far_rule):
    """The entry of the committed assembly counter summary, or None when it is for
    another workload or the device code has changed since."""
    if not os.path.exists(ASSEMBLY_TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(ASSEMBLY_TRAFFIC_FILE):
        if line.startswith("- ") and ": " in line:
            key, val = line[2:].split(": ", 1)
            kv[key.strip()] = val.strip().strip("`")
    if (kv.get("tile_code_sha256") == tile_code_sha256()
            and kv.get("workload") == f"n={n} k={float(k)} dtype={dtype} far_rule={float(far_rule)}"):
        return kv
    return None


def assembly_traffic(n, k, dtype, far_rule):
    """HBM bytes of one tile assembly from the committed counter summary (and that
    file), or (None, None)."""
    kv = _assembly_entry(n, k, dtype, far_rule)
    if kv is None:
        return None, None
    return float(kv["hbm_bytes_per_assembly"]), os.path.relpath(ASSEMBLY_TRAFFIC_FILE, ROOT)


def assembly_valu_issue(n, k, dtype, far_rule):
    """Fraction of the VALU issue rate the tile kernel used (SQ counters), or None."""
    kv = _assembly_entry(n, k, dtype, far_rule)
    return None if kv is None or "valu_issue_frac" not in kv else float(kv["valu_issue_frac"])


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_phases(np, k, nrhs):
    """Per-phase timings of the oracle on the level-3 sphere (N = 1920) on the host
    cores: its LU solve of the dense system for nrhs right-hand sides (numpy/LAPACK,
    all BLAS threads; the values of Z do not change the LU's cost, so a seeded
    matrix of the same shape stands in for the assembled one) and its far field of
    nrhs currents in nrhs directions (numpy, one thread's loops)."""
    import synth
    from oracle import efie, krylov, rwg

    v, f = synth.icosphere(3)
    om = rwg.build(v, f)
    N = om.n
    rng = np.random.default_rng(1)
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) + N * np.eye(N)
    B = rng.standard_normal((N, nrhs)) + 1j * rng.standard_normal((N, nrhs))
    t0 = time.perf_counter()
    krylov.lu_solve(A, B)
    t_lu = time.perf_counter() - t0
    rhat, _, _, _, _ = synth.monostatic_grid(16, 32)
    J = (rng.standard_normal((nrhs, N)) + 1j * rng.standard_normal((nrhs, N)))[:nrhs]
    t0 = time.perf_counter()
    efie.farfield(om, k, J, rhat[:nrhs])
    t_ff = time.perf_counter() - t0
    return {"mesh": f"icosphere level 3 (N={N})", "lu_solve_s": round(t_lu, 3),
            "lu_rhs": nrhs, "farfield_s": round(t_ff, 3), "farfield_currents_x_dirs": [nrhs, min(nrhs, len(rhat))]}


def copy_calibration(torch):
    """A plain elementwise kernel that reads 1 GiB and writes 1 GiB, three times:
    the reference reading of the HBM byte counters."""
    log("bench: copy calibration (3 x 1 GiB read + 1 GiB write)")
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    del x, y


def bench_ellipsoids(args, P, synth, torch, np, dev):
    """64 seeded ellipsoids (geodesic frequency 6..16, semi-axes U[0.5, 1.5]), k = 2,
    x-polarised plane wave along -z: the near-pair blocks of all meshes in one launch,
    their tiles of Z in one persistent launch (complex64, FP32 far pairs), and one
    grouped COCG solve to rel.res 1e-6 per step."""
    batch = synth.ellipsoid_batch(64, seed=0)
    meshes = [P.Mesh(v, f).upload(dev) for v, f, _, _ in batch]
    ns = np.array([m.n for m in meshes])
    B = P.Batch(meshes)
    k = 2.0
    kh, pol = synth.planewave_x_along_minus_z()
    Z = torch.empty(B.z_elems, dtype=torch.complex64, device=dev)
    V = torch.empty(B.v_elems, dtype=torch.complex128, device=dev)
    log(f"bench: 64 ellipsoids, N {ns.min()}..{ns.max()}, sum N^2 {int((ns ** 2).sum())}, {B.items} work items")

    def step(rec):
        t0 = time.perf_counter()
        B.assemble(k, dtype=P.C64, out=Z)
        for i, m in enumerate(meshes):
            P.excite_planewave(m, k, kh, pol, out=V[B.voff[i]:B.voff[i + 1]].view(1, -1))
        J, st = B.solve(Z, V, tol=args.tol, maxit=args.maxit)
        torch.cuda.synchronize()
        rec.append({"t": time.perf_counter() - t0, "st": st})

    for _ in range(args.warmup):
        step([])
    P.prof_reset()
    P.prof_enable(True)
    rec = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        log(f"bench: timed step {i + 1}/{args.steps}")
        step(rec)
    wall = time.perf_counter() - t0
    prof = P.prof_read(with_work=True)
    P.prof_enable(False)
    asm_ms = (prof["far"][1] + prof["near"][1]) / args.steps   # tiles + near blocks
    st = rec[-1]["st"]
    out = {
        "metric": "assembly Mentries/s (one persistent tile launch over 64 uneven meshes); time-to-solve @ rel.res 1e-6",
        "value": round(float((ns ** 2).sum()) / (asm_ms * 1e-3) / 1e6, 1),
        "unit": "Mentries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "64 ellipsoids, geodesic frequency U{6..16}, semi-axes U[0.5,1.5] (seed 0), k=2, "
                               "one plane wave each; complex64 storage, FP32 far pairs, FP64 near pairs, "
                               "FP64-accumulated grouped COCG",
                   "n_meshes": 64, "n_min": int(ns.min()), "n_max": int(ns.max()), "sum_n2": int((ns ** 2).sum())},
        "assembly_ms": round(asm_ms, 3),
        "time_to_solve_s": round(float(np.mean([r["t"] for r in rec])), 3),
        "iters_min": int(st.iters.min()), "iters_max": int(st.iters.max()),
        "relres_true_max": float(st.relres_true.max()), "all_converged": bool(np.all(st.status == 0)),
        "kernel_ms": {kname: [n, round(ms, 3)] for kname, (n, ms, _) in prof.items()},
    }
    print(json.dumps(out), flush=True)


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def bench_calderon(args, P, synth, torch, np, dev):
    """Level-4 sphere (N = 7680), x-polarised plane wave along -z, k = 0.1 and 5:
    unpreconditioned CGS against CGS on the Calderon product P Z J = P V with
    P = T_BC(k~) G_mix^-1 (everything FP64), stopping at a relative (preconditioned)
    residual of 1e-6; the reported residual is the unpreconditioned true one."""
    v, f = synth.icosphere(4)
    m = P.Mesh(v, f).upload(dev)
    kh, pol = synth.planewave_x_along_minus_z()
    cal = P.Calderon(m).upload(dev)
    res = {}
    for k in (0.1, 5.0):
        Z, t_asm = _timed(torch, lambda: P.assemble(m, k))
        V = P.excite_planewave(m, k, kh, pol)
        (_, st0), t_plain = _timed(torch, lambda: P.solve(Z, V, solver=P.CGS, tol=1e-6, maxit=4000))
        Pm, t_build = _timed(torch, lambda: cal.assemble(P.ktilde(k)))
        (_, st1), t_prec = _timed(torch, lambda: P.solve_precond(Z, Pm, V, tol=1e-6, maxit=2000))
        res[str(k)] = {
            "ktilde": [P.ktilde(k).real, P.ktilde(k).imag], "assembly_s": round(t_asm, 4),
            "cgs_iters": int(st0.iters[0]), "cgs_converged": bool(st0.status[0] == 0), "cgs_s": round(t_plain, 4),
            "cgs_relres_true": float(st0.relres_true[0]),
            "calderon_build_s": round(t_build, 4), "calderon_cgs_iters": int(st1.iters[0]),
            "calderon_cgs_s": round(t_prec, 4), "calderon_relres_true": float(st1.relres_true[0]),
            "gram_relres": cal.gram_relres,
        }
        log(f"bench: k={k} {res[str(k)]}")
        del Z, Pm
    tot = res["5.0"]["calderon_build_s"] + res["5.0"]["calderon_cgs_s"]
    out = {
        "metric": "Calderon-preconditioned CGS vs unpreconditioned CGS: iterations and time-to-solve @ 1e-6",
        "value": round(tot, 4), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * tot, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": "PEC unit sphere icosphere level 4 (N=7680 RWG), x-polarised plane wave along -z, "
                               "k=0.1 and k=5, FP64; value = Calderon build + solve at k=5",
                   "n_unknowns": m.n, "n_bary_rwg": cal.n_bary},
        "results": res,
    }
    print(json.dumps(out), flush=True)


def bench_cfie(args, P, synth, torch, np, dev):
    """The 3-D Calderon-stabilized CFIE against the Calderon-EFIE on the sphere of
    --cfie-level (default 4, N = 7680) at wavenumbers --cfie-ks (default: 4.9734
    and 9.9675, zeros of (x j_3(x))' and of (x j_7(x))' where the EFIE has interior
    resonances, and 5 and 10 beside them), --cfie-nrhs plane waves along the
    monostatic grid: build times (Z, P, M and Q), CGS iterations and time to 1e-6,
    and the RCS difference between the two solutions.  Everything FP64."""
    v, f = synth.icosphere(args.cfie_level)
    m = P.Mesh(v, f).upload(dev)
    cal = P.Calderon(m).upload(dev)
    rhat, khat, pol, _, _ = synth.monostatic_grid(4, 8)
    S = min(args.cfie_nrhs, len(khat))
    kh, po = khat[:S], pol[:S]
    res = {}
    for k in args.cfie_ks:
        kt = P.ktilde(k)
        Z, t_z = _timed(torch, lambda: P.assemble(m, k))
        Pm, t_p = _timed(torch, lambda: cal.assemble(kt, tol=1e-10))
        (M, Q), t_mq = _timed(torch, lambda: cal.cfie(k, kt, tol=1e-10))
        V = P.excite_planewave(m, k, kh, po)
        H = cal.mfie_rhs(k, kh, po)
        (J, st), t_c = _timed(torch, lambda: P.solve_cfie(Z, Pm, M, Q, V, H, tol=1e-6, maxit=1000))
        (Je, se), t_e = _timed(torch, lambda: P.solve_precond(Z, Pm, V, tol=1e-6, maxit=3000))
        Fc = P.farfield(m, k, J, rhat[:S]).cpu().numpy()
        Fe = P.farfield(m, k, Je, rhat[:S]).cpu().numpy()
        sc = np.sum(np.abs(Fc) ** 2, axis=-1)          # (rhs, direction) bistatic
        sv = np.sum(np.abs(Fe) ** 2, axis=-1)
        db = np.abs(10 * np.log10(sc / sv))
        db30 = db[sv >= 1e-3 * sv.max(axis=1, keepdims=True)]
        row = {"ktilde": [kt.real, kt.imag], "Z_s": round(t_z, 3), "P_s": round(t_p, 3), "M_Q_s": round(t_mq, 3),
               "cfie_iters_max": int(st.iters.max()), "cfie_iters_mean": round(float(st.iters.mean()), 1),
               "cfie_solve_s": round(t_c, 3), "cfie_relres_true_max": float(st.relres_true.max()),
               "efie_iters_max": int(se.iters.max()), "efie_iters_mean": round(float(se.iters.mean()), 1),
               "efie_solve_s": round(t_e, 3), "efie_relres_true_max": float(se.relres_true.max()),
               "bistatic_rcs_db_diff_max": float(db.max()), "bistatic_rcs_db_diff_max_within_30db": float(db30.max()),
               "q_gram_relres": cal.cfie_gram_relres}
        log(f"bench: cfie k={k} {row}")
        res[str(k)] = row
        del Z, Pm, M, Q
        torch.cuda.empty_cache()
    key = str(args.cfie_ks[0])
    tot = res[key]["M_Q_s"] + res[key]["cfie_solve_s"]
    out = {
        "metric": "Calderon-stabilized CFIE vs Calderon-EFIE: CGS iterations and time-to-solve @ 1e-6",
        "value": round(tot, 3), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * tot, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"PEC unit sphere icosphere level {args.cfie_level} (N={m.n} RWG), {S} plane waves, "
                               f"k in {list(args.cfie_ks)}, FP64; value = M, Q build + CFIE solve at k={key}",
                   "n_unknowns": m.n, "nrhs": S},
        "results": res,
    }
    print(json.dumps(out), flush=True)


def bench_gradient(args, P, synth, torch, np, dev):
    """Adjoint vertex gradient of J = sum_d |F(rhat_d)|^2 (32 seeded directions) on the
    level-4 perturbed sphere (N = 7680), k = 3, x-polarised plane wave along -z:
    forward (assembly, excitation, COCG to 1e-13, far field) and backward (adjoint
    source, adjoint solve with the same Z, vertex-gradient kernels) through the torch
    autograd function; HIP-event times of the three gradient kernels."""
    from paper_2310_15644_amd.objective import far_field_objective

    v, f = synth.perturbed_sphere(4, seed=0)
    kh, pol = synth.planewave_x_along_minus_z()
    dirs = synth.uniform_directions(32, seed=1)

    def run():
        x = torch.tensor(v, dtype=torch.float64, device=dev, requires_grad=True)
        J = far_field_objective(x, f, 3.0, kh[0], pol[0], dirs, tol=1e-13)
        J.backward()
        return float(J), x.grad

    run()   # warm-up
    P.prof_reset()
    P.prof_enable(True)
    (J, g), t = _timed(torch, run)
    prof = P.prof_read(with_work=True)
    P.prof_enable(False)
    gk = {name: {"launches": prof[name][0], "ms": round(prof[name][1], 3), "units": prof[name][2]}
          for name in ("grad_far", "grad_near", "grad_tri")}
    g_ms = sum(x["ms"] for x in gk.values())
    far_pairs = prof["grad_far"][2]
    out = {
        "metric": "adjoint vertex gradient: forward + backward time and gradient-kernel time",
        "value": round(t, 4), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * t, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": "perturbed unit sphere (icosphere level 4, radial spherical-harmonic perturbation "
                               "degree <= 6, max 5 %, seed 0), k=3, 32 uniform directions (seed 1), x-polarised "
                               "plane wave along -z; value = forward + backward wall time", "n_vertices": len(v)},
        "objective": J,
        "grad_norm": float(torch.linalg.norm(g)),
        "grad_kernels": gk,
        "grad_kernels_ms": round(g_ms, 3),
        "grad_far_pairs_per_s": round(far_pairs / (gk["grad_far"]["ms"] * 1e-3), 1) if gk["grad_far"]["ms"] else None,
    }
    print(json.dumps(out), flush=True)


def bench_mixed_fp64(args, P, synth, torch, np, dev):
    """Level-5 sphere (N = 30720), k = 10, x-polarised plane wave along -z: the mixed
    form (complex64 Z, FP32 far pairs, FP32 matrix-core products, FP64 refinement)
    against the FP64 GPU path on the same input; current difference, RCS difference
    over the 512 monostatic-grid directions, and both times-to-solve @ 1e-6
    (assembly + excitation + solve)."""
    v, f = synth.icosphere(5)
    m = P.Mesh(v, f).upload(dev)
    k = 10.0
    kh, pol = synth.planewave_x_along_minus_z()
    rhat, _, _, _, _ = synth.monostatic_grid(16, 32)

    def run(dt):
        Z = P.assemble(m, k, dtype=dt)
        V = P.excite_planewave(m, k, kh, pol)
        J, st = P.solve(Z, V, solver=P.COCG, tol=1e-6, maxit=5000, max_refine=8, inner_tol=1e-3)
        return J, st

    run(P.C64)   # warm-up (library load, first launches)
    (J32, st32), t32 = _timed(torch, lambda: run(P.C64))
    (J64, st64), t64 = _timed(torch, lambda: run(P.C128))
    dj = float(torch.linalg.norm(J32 - J64) / torch.linalg.norm(J64))
    F32 = P.farfield(m, k, J32, rhat).cpu().numpy()[0]
    F64 = P.farfield(m, k, J64, rhat).cpu().numpy()[0]
    r32 = 10 * np.log10(4 * math.pi * np.sum(np.abs(F32) ** 2, axis=1))
    r64 = 10 * np.log10(4 * math.pi * np.sum(np.abs(F64) ** 2, axis=1))
    keep = r64 >= r64.max() - 40.0
    out = {
        "metric": "mixed precision vs FP64: time-to-solve @ rel.res 1e-6 and solution difference",
        "value": round(t32, 4), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * t32, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": "PEC unit sphere icosphere level 5 (N=30720 RWG), k=10, x-polarised plane wave "
                               "along -z; value = mixed-path time-to-solve (assembly + excitation + solve)",
                   "n_unknowns": m.n},
        "fp64_time_to_solve_s": round(t64, 4),
        "mixed_iters": int(st32.iters[0]), "fp64_iters": int(st64.iters[0]),
        "mixed_relres_true": float(st32.relres_true[0]), "fp64_relres_true": float(st64.relres_true[0]),
        "current_rel_diff": dj,
        "rcs_db_max_abs_diff": float(np.abs(r32 - r64).max()),
        "rcs_db_max_abs_diff_within_40db": float(np.abs(r32 - r64)[keep].max()),
    }
    print(json.dumps(out), flush=True)


def far3_fraction(v, f, ratio, near_factor=2.0):
    """Fraction of the ordered triangle pairs beyond the near distance (D >= near_factor h;
    the shared-vertex test is left out) that take the 3x3 rule, D >= ratio h, h the
    larger longest edge of the two."""
    import numpy as np

    x = v[f]                                              # (T, 3, 3)
    c = x.mean(axis=1)
    e = np.stack([np.linalg.norm(x[:, 1] - x[:, 0], axis=1), np.linalg.norm(x[:, 2] - x[:, 1], axis=1),
                  np.linalg.norm(x[:, 0] - x[:, 2], axis=1)], 1)
    h = e.max(axis=1)
    n3 = nfar = 0
    for a in range(0, len(c), 1024):
        d2 = ((c[a:a + 1024, None, :] - c[None, :, :]) ** 2).sum(-1)
        hm = np.maximum(h[a:a + 1024, None], h[None, :])
        far = d2 >= (near_factor * hm) ** 2
        n3 += int(np.count_nonzero(d2 >= (ratio * hm) ** 2))
        nfar += int(np.count_nonzero(far))
    return n3 / max(nfar, 1)


def bench_far_rule(args, P, synth, torch, np, dev):
    """Level-5 sphere (N = 30720), k = 10: the distance-adaptive far rule (the 3x3
    product of the interior 3-point rule on pairs with D >= r h; r = --far-rule, 4 if
    unset) against the 7x7 rule everywhere.  Complex64 tile assembly (kernel time,
    mean of 3), the Calderon P build (Gram solve to 1e-3, FP32 barycentric pairs, whose
    operator follows the same rule), and one x-polarised plane wave along -z solved
    by the Calderon-preconditioned mixed CGS to 1e-6 with each: currents and RCS over
    the 512 monostatic-grid directions compared."""
    r = args.far_rule if args.far_rule > 0 else 4.0
    v, f = synth.icosphere(5)
    m = P.Mesh(v, f).upload(dev)
    k = 10.0
    N = m.n
    kh, pol = synth.planewave_x_along_minus_z()
    rhat, _, _, _, _ = synth.monostatic_grid(16, 32)
    cal = P.Calderon(m).upload(dev)
    Z = torch.empty((N, N), dtype=torch.complex64, device=dev)
    res = {}
    for name, ratio in (("seven_point", 0.0), ("adaptive", r)):
        log(f"bench: far rule {ratio}")
        m.set_far_rule(ratio)
        P.assemble(m, k, dtype=P.C64, out=Z)
        torch.cuda.synchronize()
        P.prof_reset()
        P.prof_enable(True)
        for _ in range(3):
            P.assemble(m, k, dtype=P.C64, out=Z)
        torch.cuda.synchronize()
        prof = P.prof_read()
        P.prof_enable(False)
        asm_ms = (prof["far"][1] + prof["near"][1]) / 3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Pm = P.convert(cal.assemble(P.ktilde(k), tol=1e-3, bary_dtype=P.C64), P.C64)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        V = P.excite_planewave(m, k, kh, pol)
        J, st = P.solve_precond(Z, Pm, V, tol=1e-6, maxit=3000, inner_tol=1e-3)
        F = P.farfield(m, k, J, rhat).cpu().numpy()[0]
        res[name] = {"asm_ms": asm_ms, "build_s": tb, "J": J.clone(), "F": F, "iters": int(st.iters[0]),
                     "relres": float(st.relres_true[0])}
        del Pm
    m.set_far_rule(0.0)
    a, s7 = res["adaptive"], res["seven_point"]
    me = N * N / (a["asm_ms"] * 1e-3) / 1e6
    me7 = N * N / (s7["asm_ms"] * 1e-3) / 1e6
    dj = float(torch.linalg.norm(a["J"] - s7["J"]) / torch.linalg.norm(s7["J"]))
    ra = 10 * np.log10(4 * math.pi * np.sum(np.abs(a["F"]) ** 2, axis=1))
    r7 = 10 * np.log10(4 * math.pi * np.sum(np.abs(s7["F"]) ** 2, axis=1))
    keep = r7 >= r7.max() - 40.0
    zbytes = N * N * 8
    out = {
        "metric": "distance-adaptive far rule: complex64 assembly Mentries/s (kernel time)",
        "value": round(me, 1), "unit": "Mentries/s", "n_gpus": 1, "steps": 3, "warmup": 1,
        "ms_per_step": round(a["asm_ms"], 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": "PEC unit sphere icosphere level 5 (N=30720 RWG), k=10; far pairs with centroid "
                               f"distance >= {r} x the larger longest edge by the 3x3 interior 3-point rule, "
                               "the others by the 7x7 rule; one x-polarised plane wave along -z for the accuracy",
                   "n_unknowns": N, "far_rule": r},
        "seven_point_mentries_per_s": round(me7, 1),
        "assembly_speedup": round(me / me7, 3),
        "pair_fraction_3x3": round(far3_fraction(np.asarray(v, dtype=np.float64), np.asarray(f), r), 4),
        "z_write_gbs": round(zbytes / (a["asm_ms"] * 1e-3) / 1e9, 1),
        "hbm_roofline": {"bound": "hbm", "achieved": round(zbytes / (a["asm_ms"] * 1e-3) / 1e9, 1),
                         "peak": 8000.0, "unit": "GB/s",
                         "frac": round(zbytes / (a["asm_ms"] * 1e-3) / 1e9 / 8000.0, 4),
                         "note": "bytes of Z written once (complex64) over the tile and near-block kernel "
                                 "time; the tiles are bound by the vector ALU, not by HBM"},
        "calderon_build_s": {"adaptive": round(a["build_s"], 3), "seven_point": round(s7["build_s"], 3)},
        "iters": {"adaptive": a["iters"], "seven_point": s7["iters"]},
        "relres_true": {"adaptive": a["relres"], "seven_point": s7["relres"]},
        "current_rel_diff": dj,
        "rcs_db_max_abs_diff": float(np.abs(ra - r7).max()),
        "rcs_db_max_abs_diff_within_40db": float(np.abs(ra - r7)[keep].max()),
    }
    print(json.dumps(out), flush=True)


# the paper's Table I: skeleton compression time of the ellipse (aspect ratio 1.5,
# perimeter 2 pi) on 25 parallel processes (hardware not stated)
PAPER_TABLE1 = {15011: (833.91, 59.33), 30021: (1667.8, 129.6), 45032: (2501.7, 210.2)}


def bench_bie2d(args, P, synth, torch, np, dev):
    """The paper's 2-D fast direct solver (Sec. III-IV): for each ellipse of the
    paper's Table I (or --bie2d-n / --bie2d-k), assemble S_k, D*_k, N_k~, D*_k~ and
    the circular counterpart, compress C_p - C_p,c by the randomized skeleton to
    --bie2d-tol, factor the Woodbury inverse, and solve for --bie2d-nrhs plane waves;
    the stabilized system's residual ||C_p x - b_p|| / ||b_p|| checks the solve.
    Times are wall clock around each phase (device synchronised)."""
    import math

    cases = [(n, kk) for n, (kk, _) in sorted(PAPER_TABLE1.items())]
    if args.bie2d_n:
        cases = [(int(n), float(kk)) for n, kk in zip(args.bie2d_n, args.bie2d_k)]
    geom = {"ellipse": synth.contour_ellipse, "airfoil": synth.contour_joukowsky}[args.bie2d_geom]
    pols = args.bie2d_pol or ["TM"]
    rows = []
    for (n, k), pol in [(c, p) for c in cases for p in pols]:
        nodes, circ = geom(n), synth.contour_circle(n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = P.Bie2d(nodes, circ, device=dev)
        rmax = min(n, args.bie2d_rmax)
        h.setup(k, rmax=rmax, block=64, nvec=max(64, args.bie2d_nrhs), pol=pol)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        g = torch.Generator(device=dev).manual_seed(0)
        om = torch.randn((rmax + 64, n), dtype=torch.complex128, device=dev, generator=g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rank, est, ref = h.skeleton(om, args.bie2d_tol)
        torch.cuda.synchronize()
        t_skel = time.perf_counter() - t0
        del om
        phis = 2.0 * math.pi * np.arange(args.bie2d_nrhs) / args.bie2d_nrhs
        e, hv, bp = h.rhs(phis)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = h.solve(bp)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        res = (h.apply("cp", x) - bp).norm(dim=1) / bp.norm(dim=1)
        paper = PAPER_TABLE1.get(n)
        row = {"n": n, "k0": k, "pol": pol, "nodes_per_wavelength": round(n * 2.0 * math.pi / (k * h.perimeter()), 2),
               "rank": rank, "tol": args.bie2d_tol, "est_rel": est / ref if ref else 0.0,
               "setup_s": round(t_setup, 3), "skeleton_s": round(t_skel, 3), "solve_s": round(t_solve, 4),
               "nrhs": args.bie2d_nrhs, "residual_max": float(res.max()),
               "paper_skeleton_s": None if paper is None or abs(paper[0] - k) > 1e-6 else paper[1]}
        log(f"bench: bie2d {row}")
        rows.append(row)
        del h, e, hv, bp, x
        torch.cuda.empty_cache()
    main = rows[-1]
    out = {
        "metric": "skeleton compression time of C_p - C_p,c (paper Table I)",
        "value": main["skeleton_s"],
        "unit": "s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * (main["setup_s"] + main["skeleton_s"]), 1),
        "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None if main["paper_skeleton_s"] is None else round(main["skeleton_s"] / main["paper_skeleton_s"], 5),
        "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"2-D PEC {args.bie2d_geom} (aspect 1.5, perimeter 2 pi), {main['pol']}, "
                               f"Calderon-stabilized CFIE "
                               f"C_p (eq. 16), randomized skeleton of C_p - C_p,c to {args.bie2d_tol:g} and Woodbury "
                               f"inverse (eqs. 17-18); N and k0 of the paper's Table I",
                   "cases": [[r["n"], r["k0"], r["pol"]] for r in rows]},
        "cases": rows,
    }
    print(json.dumps(out), flush=True)


def bench_bie2d_rank(args, P, synth, torch, np, dev):
    """Skeleton rank of C_p - C_p,c against k0 (the paper's Figs. 1-2, whose data
    are not in the text) for the ellipse and the airfoil at a fixed number of nodes
    per wavelength."""
    import math

    out = {"metric": "skeleton rank of C_p - C_p,c vs k0", "unit": "rank", "tol": args.bie2d_tol,
           "nodes_per_wavelength": args.bie2d_ppw, "curves": {}}
    curves = [(g, m, p) for g, m in (("ellipse", synth.contour_ellipse), ("airfoil", synth.contour_joukowsky))
              for p in (args.bie2d_pol or ["TM", "TE"])]
    for geom, make, pol in curves:
        pts = []
        for k in args.bie2d_ks:
            n = int(round(args.bie2d_ppw * k))          # perimeter 2 pi: k0 wavelengths
            h = P.Bie2d(make(n), synth.contour_circle(n), device=dev)
            rmax = min(n, args.bie2d_rmax)
            h.setup(k, rmax=rmax, block=32, nvec=32, pol=pol)
            g = torch.Generator(device=dev).manual_seed(0)
            om = torch.randn((rmax + 32, n), dtype=torch.complex128, device=dev, generator=g)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rank, est, ref = h.skeleton(om, args.bie2d_tol)
            torch.cuda.synchronize()
            pts.append({"k0": k, "n": n, "rank": rank, "skeleton_s": round(time.perf_counter() - t0, 3)})
            log(f"bench: bie2d rank {geom} {pol} {pts[-1]}")
            del h, om
            torch.cuda.empty_cache()
        ks = np.array([p["k0"] for p in pts])
        rk = np.array([max(p["rank"], 1) for p in pts], dtype=float)
        slope = np.polyfit(np.log(ks[-3:]), np.log(rk[-3:]), 1)[0] if len(ks) >= 3 else None
        out["curves"][f"{geom}_{pol}"] = {"points": pts, "loglog_slope_last3": None if slope is None else round(float(slope), 3)}
    print(json.dumps(out), flush=True)


def fp64_leg(args, P, torch, np, m, kh_d, po_d, V, J, cal):
    """The plain FP64 path on the same inputs, timed like a step (after the mixed
    steps, --fp64-steps of them, no warm-up): complex128 Z, complex128 P (the same
    build), CGS on P Z J = P V with FP64 products to the same true residual."""
    log(f"bench: FP64 path, {args.fp64_steps} step(s)")
    Z = torch.empty((m.n, m.n), dtype=torch.complex128, device=V.device)
    times, st = [], None
    for _ in range(args.fp64_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.assemble(m, args.k, dtype=P.C128, out=Z)
        P.excite_planewave(m, args.k, kh_d, po_d, out=V)
        Pm = cal.assemble(P.ktilde(args.k), tol=1e-3, bary_dtype=P.C64)
        _, st = P.solve_precond(Z, Pm, V, tol=args.tol, maxit=args.maxit, out=J)
        del Pm
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    del Z
    torch.cuda.empty_cache()
    return {"time_to_solve_s": round(float(np.mean(times)), 3), "steps": args.fp64_steps,
            "iters_max": int(np.max(st.iters)), "iters_mean": round(float(np.mean(st.iters)), 1),
            "relres_true_max": float(np.max(st.relres_true)), "all_converged": bool(np.all(st.status == 0)),
            "dtype": "c128"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=5)
    ap.add_argument("--k", type=float, default=10.0)
    ap.add_argument("--ntheta", type=int, default=16)
    ap.add_argument("--nphi", type=int, default=32)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--maxit", type=int, default=3000)
    ap.add_argument("--dtype", choices=["c64", "c128"], default="c64")
    ap.add_argument("--solver", choices=["calderon", "cocg"], default="calderon",
                    help="calderon: CGS on P Z J = P V with P = T_BC(k~) G_mix^-1 built in the step (default); "
                         "cocg: unpreconditioned COCG")
    ap.add_argument("--workload", choices=["sphere", "ellipsoids", "calderon", "mixed-fp64", "gradient",
                                           "far-rule", "bie2d", "bie2d-rank", "cfie"],
                    default="sphere",
                    help="sphere: the 512-RHS level-5 sphere (default); ellipsoids: 64 uneven ellipsoids; "
                         "calderon: level-4 Calderon vs plain CGS; mixed-fp64: level-5 mixed vs FP64 path; "
                         "gradient: level-4 adjoint vertex gradient; far-rule: level-5 assembly, P build and "
                         "accuracy with the distance-adaptive far rule against the 7x7 rule")
    ap.add_argument("--cal-far-rule", type=float, default=4.0,
                    help="far rule of the Calderon preconditioner's barycentric operator alone: its pairs with "
                         "centroid distance >= this times the larger longest edge take the 3x3 rule (default 4; "
                         "< 0: follow --far-rule).  P only preconditions: Z and the true residual keep their rule")
    ap.add_argument("--far-rule", type=float, default=0.0,
                    help="distance-adaptive far rule: far pairs with centroid distance >= this times the larger "
                         "longest edge take the 3x3 rule (0: the 7x7 rule everywhere, the default)")
    ap.add_argument("--fp32-acc", action="store_true",
                    help="mixed solve: accumulate the matrix-core products in FP32 instead of flushing "
                         "the partial sums into FP64 every K chunk")
    ap.add_argument("--fp64-steps", type=int, default=1,
                    help="after the timed mixed steps, time this many steps of the plain FP64 path "
                         "(complex128 Z and P, FP64 products; Calderon solver only; 0: skip)")
    ap.add_argument("--bie2d-n", type=int, nargs="*", help="2-D workload: node counts (default: the paper's Table I)")
    ap.add_argument("--bie2d-k", type=float, nargs="*", help="2-D workload: wavenumbers, one per --bie2d-n")
    ap.add_argument("--bie2d-geom", choices=["ellipse", "airfoil"], default="ellipse")
    ap.add_argument("--bie2d-tol", type=float, default=1e-4)
    ap.add_argument("--bie2d-rmax", type=int, default=4096)
    ap.add_argument("--bie2d-nrhs", type=int, default=64)
    ap.add_argument("--bie2d-ks", type=float, nargs="*", default=[25, 50, 100, 200, 400, 834])
    ap.add_argument("--bie2d-ppw", type=float, default=18.0, help="bie2d-rank: nodes per wavelength")
    ap.add_argument("--bie2d-pol", choices=["TM", "TE"], nargs="*",
                    help="2-D polarizations (default: TM for bie2d, TM and TE for bie2d-rank)")
    ap.add_argument("--cfie-level", type=int, default=4)
    ap.add_argument("--cfie-ks", type=float, nargs="*", default=[4.9734, 5.0, 9.9675, 10.0])
    ap.add_argument("--cfie-nrhs", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy 1 GiB three times with a plain elementwise kernel (for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library drives one GPU per "
              "process and has no sharded path (rows of Z split by test RWG across GPUs is the intended "
              "extension, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2310_15644_amd as P
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.workload == "ellipsoids":
        bench_ellipsoids(args, P, synth, torch, np, dev)
        return
    if args.workload == "calderon":
        bench_calderon(args, P, synth, torch, np, dev)
        return
    if args.workload == "mixed-fp64":
        bench_mixed_fp64(args, P, synth, torch, np, dev)
        return
    if args.workload == "gradient":
        bench_gradient(args, P, synth, torch, np, dev)
        return
    if args.workload == "far-rule":
        bench_far_rule(args, P, synth, torch, np, dev)
        return
    if args.workload == "bie2d":
        bench_bie2d(args, P, synth, torch, np, dev)
        return
    if args.workload == "bie2d-rank":
        bench_bie2d_rank(args, P, synth, torch, np, dev)
        return
    if args.workload == "cfie":
        bench_cfie(args, P, synth, torch, np, dev)
        return
    v, f = synth.icosphere(args.level)
    m = P.Mesh(v, f).upload(dev)
    if args.far_rule > 0:
        m.set_far_rule(args.far_rule)
    N = m.n
    rhat, khat, pol, _, _ = synth.monostatic_grid(args.ntheta, args.nphi)
    S = len(khat)
    dt = P.C64 if args.dtype == "c64" else P.C128
    tdt = torch.complex64 if dt == P.C64 else torch.complex128
    log(f"bench: level {args.level} N={N} T={m.t} near={m.n_near} k={args.k} nrhs={S} dtype={args.dtype}")
    # inputs resident in HBM before the timed region
    kh_d = torch.as_tensor(khat, dtype=torch.float64, device=dev).contiguous()
    po_d = torch.as_tensor(pol, dtype=torch.float64, device=dev).contiguous()
    rh_d = torch.as_tensor(rhat, dtype=torch.float64, device=dev).contiguous()
    Z = torch.empty((N, N), dtype=tdt, device=dev)
    V = torch.empty((S, N), dtype=torch.complex128, device=dev)
    J = torch.empty((S, N), dtype=torch.complex128, device=dev)
    tuning = None
    if dt == P.C64:
        P.assemble(m, args.k, dtype=dt, out=Z)
        tuning = P.gemm_autotune(Z, S, reps=2)
        log(f"bench: GEMM tiles {tuning}")

    def sync():
        torch.cuda.synchronize()

    cal = None
    cal_host_s = None
    if args.solver == "calderon":
        t_c = time.perf_counter()
        cal = P.Calderon(m).upload(dev)        # host refinement and BC tables: mesh preprocessing
        cal.set_far_rule(args.cal_far_rule)
        sync()
        cal_host_s = time.perf_counter() - t_c
        log(f"bench: Calderon tables: {cal.n_bary} barycentric RWGs, host setup and upload {cal_host_s:.2f} s")

    def step(rec):
        t0 = time.perf_counter()
        P.assemble(m, args.k, dtype=dt, out=Z)
        P.excite_planewave(m, args.k, kh_d, po_d, out=V)
        tb = 0.0
        if cal is not None:
            # P only has to be a fixed approximation of T_BC G_mix^-1: the Gram solve to 1e-3
            Pm = cal.assemble(P.ktilde(args.k), tol=1e-3, bary_dtype=P.C64)
            if dt == P.C64:
                Pm = P.convert(Pm, P.C64)
            sync()
            tb = time.perf_counter() - t0
            _, st = P.solve_precond(Z, Pm, V, tol=args.tol, maxit=args.maxit, inner_tol=1e-3, fp32_acc=args.fp32_acc,
                                    out=J)
            del Pm
        else:
            _, st = P.solve(Z, V, solver=P.COCG, tol=args.tol, maxit=args.maxit, max_refine=6, inner_tol=1e-3,
                            fp32_acc=args.fp32_acc, out=J)
        sync()
        t1 = time.perf_counter()
        F = P.farfield(m, args.k, J, rh_d)
        sync()
        t2 = time.perf_counter()
        rec.append({"solve_s": t1 - t0, "step_s": t2 - t0, "build_s": tb, "iters": st.iters,
                    "relres": st.relres_true, "status": st.status, "F": F})

    warm = []
    for i in range(args.warmup):
        log(f"bench: warmup step {i + 1}/{args.warmup}")
        step(warm)
    P.prof_reset()
    P.prof_enable(True)
    rec = []
    sync()
    t0 = time.perf_counter()
    for i in range(args.steps):
        log(f"bench: timed step {i + 1}/{args.steps}")
        step(rec)
    sync()
    wall = time.perf_counter() - t0
    prof = P.prof_read(with_work=True)
    P.prof_enable(False)

    ms_step = 1e3 * wall / args.steps
    fp64 = None
    if args.fp64_steps > 0 and dt == P.C64 and args.solver == "calderon":
        fp64 = fp64_leg(args, P, torch, np, m, kh_d, po_d, V, J, cal)
    gemm_key = "mfma" if dt == P.C64 else "zgemm"
    # Z.X launches inside the solve run over the active (unconverged) columns only:
    # the algorithmic flops 8 M N N are summed per launch with its own M.  The
    # roofline is that of the selected tile ("mfma"); the metric's value counts
    # every matrix-core launch, those of <= 32 columns on the 32-row tile too.
    n_mm, ms_mm, fl_mm = prof[gemm_key]
    n_sm, ms_sm, fl_sm = prof["mfma_small"] if dt == P.C64 else (0, 0.0, 0.0)
    avg_mm = ms_mm / max(n_mm, 1)
    flops = fl_mm / max(n_mm, 1)                 # mean algorithmic flops per launch
    zx_gflops = (fl_mm + fl_sm) / ((ms_mm + ms_sm) * 1e-3) / 1e9 if n_mm + n_sm else float("nan")
    n_far, ms_far, _ = prof["far"]
    n_near, ms_near, _ = prof["near"]
    asm_ms = (ms_far + ms_near) / args.steps
    mentries = N * N / (asm_ms * 1e-3) / 1e6
    alu_peak = assembly_alu_peak(N, m.t, args.dtype) if args.far_rule <= 0 else None
    last = rec[-1]
    F = last["F"]
    # reciprocity of the bistatic matrix S_ij = theta_j . F_i(rhat_j)
    Sm = F[:, :, 0].cpu().numpy()
    recip = float(np.abs(Sm - Sm.T).max() / np.abs(Sm).max())
    tts = float(np.mean([r["solve_s"] for r in rec]))
    out = {
        "metric": "Z·X complex GFLOP/s + assembly Mentries/s; time-to-solve @ rel.res 1e-6",
        "value": round(zx_gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64" if dt == P.C64 else "c128",
        "data": "synthetic",
        "config": {
            "workload": f"PEC unit sphere icosphere level {args.level} (N={N} RWG), k={args.k}, "
                        f"{S} plane waves on a {args.ntheta}x{args.nphi} (theta,phi) grid, monostatic; "
                        + ((f"mixed precision (complex64 Z, FP32 MFMA with "
                            f"{'FP32 accumulation' if args.fp32_acc else 'FP64 flushes'}, FP64 refinement)")
                           if dt == P.C64 else "FP64") + "; "
                        + ("Calderon-preconditioned CGS (P = T_BC(k~) G_mix^-1 built in the step"
                           + (f", its barycentric far pairs beyond {args.cal_far_rule} h by the 3x3 rule)"
                              if args.cal_far_rule >= 0 else ")")
                           if args.solver == "calderon" else "unpreconditioned COCG"),
            "solver": args.solver,
            "far_rule": args.far_rule if args.far_rule > 0 else None,
            "calderon_far_rule": args.cal_far_rule if args.cal_far_rule >= 0 else None,
            "accumulation": ("fp32" if args.fp32_acc else "fp64-flush") if dt == P.C64 else "fp64",
            "n_unknowns": N,
            "nrhs": S,
            "k": args.k,
            "tol": args.tol,
        },
        "zx_gflops": round(zx_gflops, 2),
        "zx_launches": n_mm,
        "zx_ms_per_launch": round(avg_mm, 4),
        "zx_small_launches": n_sm,
        "zx_small_ms_per_launch": round(ms_sm / n_sm, 4) if n_sm else None,
        "assembly_mentries_per_s": round(mentries, 1),
        "assembly_ms": round(asm_ms, 3),
        "time_to_solve_s": round(tts, 3),
        "calderon_build_s": round(float(np.mean([r["build_s"] for r in rec])), 3) if args.solver == "calderon"
        else None,
        "calderon_host_s": None if cal_host_s is None else round(cal_host_s, 3),
        "time_to_solve_fp64_s": None if fp64 is None else fp64["time_to_solve_s"],
        "fp64_path": fp64,
        "mixed_speedup_vs_fp64": None if fp64 is None else round(fp64["time_to_solve_s"] / tts, 3),
        "iters_max": int(np.max(last["iters"])),
        "iters_mean": round(float(np.mean(last["iters"])), 1),
        "relres_true_max": float(np.max(last["relres"])),
        "all_converged": bool(np.all(last["status"] == 0)),
        "reciprocity_rel": recip,
        "roofline": {
            "bound": "mfma",
            "achieved": round(flops / (avg_mm * 1e-3) / 1e12, 3),
            "peak": PEAK_FP32_MFMA if dt == P.C64 else 78.6,
            "unit": "TFLOP/s",
            "frac": round(flops / (avg_mm * 1e-3) / 1e12 / (PEAK_FP32_MFMA if dt == P.C64 else 78.6), 4),
            "traffic": None,
            # the FP64-flush GEMM forms each complex product from three real ones (3M):
            # the matrix cores execute 6 M N n_cols of the 8 M N n_cols algorithmic flops
            "executed_flop_fraction": 0.75 if (dt == P.C64 and not args.fp32_acc) else 1.0,
        },
        "assembly_roofline": {
            "bound": "alu",
            "kernel": "near_blocks_kernel + tile_kernel (owner-computes tiles, Z written once)",
            "achieved": round(mentries, 1),
            # the cost model of the 7x7 rule; with the far rule on it does not apply
            "peak": round(alu_peak, 1) if alu_peak else None,
            "unit": "Mentries/s",
            "frac": round(mentries / alu_peak, 4) if alu_peak else None,
            "model": "49 T^2/N^2 Green's-function evaluations per entry x %g issue slots" % EVAL_SLOTS[args.dtype],
            "z_write_gbs": round(N * N * (8 if dt == P.C64 else 16) / (asm_ms * 1e-3) / 1e9, 1),
        },
        "kernel_ms": {kname: [n, round(ms, 3)] for kname, (n, ms, _) in prof.items()},
        "gemm_tiles": None if tuning is None else {"acc32": tuning["tiles"][tuning["acc32"]],
                                                   "acc64": tuning["tiles"][tuning["acc64"]], "ms": tuning["ms"]},
    }
    tiles = None if tuning is None else tuning["tiles"][tuning["acc32" if args.fp32_acc else "acc64"]]
    out["roofline"]["kernel"] = None if tiles is None else P.gemm_kernel_name(tiles, not args.fp32_acc)
    out["roofline"]["traffic"], out["roofline"]["traffic_source"] = measured_traffic(
        tiles, not args.fp32_acc, out["config"]["n_unknowns"], S, args.solver)
    # the assembly's HBM bytes (rocprofv3 counters) against Z's and the 8 TB/s peak
    a_tr, a_src = assembly_traffic(N, args.k, args.dtype, args.far_rule)
    zb = N * N * (8 if dt == P.C64 else 16)
    out["assembly_roofline"]["traffic"] = a_tr
    out["assembly_roofline"]["traffic_source"] = a_src
    out["assembly_roofline"]["traffic_over_z"] = None if a_tr is None else round(a_tr / zb, 3)
    out["assembly_roofline"]["hbm_frac"] = None if a_tr is None else round(a_tr / (asm_ms * 1e-3) / 8e12, 4)
    out["assembly_roofline"]["valu_issue_frac"] = assembly_valu_issue(N, args.k, args.dtype, args.far_rule)
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.level, 2048, S, args.k, args.cpu_seconds)
    if args.copy_calibration:
        copy_calibration(torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
