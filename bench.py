#!/usr/bin/env python3
"""Benchmark of the adaptive-MG hot path on one MI355X.

Workload (the precision configuration): 256x256 lattice, quenched U(1) fields at
beta = 6 (500 Metropolis sweeps, 4 fields, seeds 2000-2003), 5 masses per field at
lambda_min(A)/lambda_max(A) = 1e-2, 3e-3, 1e-3, 3e-4, 1e-4 (tuned offline, stored in
workloads/masses_256_beta6.json), 3 levels of 4x4 aggregates with Nv = 12, nu = 4 MR
smoother (omega 0.8), 5 setup iterations, dense FP64 coarsest inverse, one Gaussian
right-hand side per field (rhs = D^H b), true residual 1e-10.

The adaptive setup runs once per field at its lightest mass; the heavier masses
reuse its near-null vectors (their coarse operators are rebuilt) -- both are timed
separately as setup.  One step solves all 20 (field, mass) systems.  `value` is
mixed-precision (FP32 inner MG-CG with FP16-stored operators, FP64 defect
correction) solves/s; the plain FP64
GPU MG is timed on the same hierarchies and reported beside it.

Prints one JSON line.  `--gpus N` with N > 1 exits: this build uses one GPU.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

L = 256
BETA = 6.0
SWEEPS = 500
SEEDS = [2000, 2001, 2002, 2003]
BLOCKS = [(4, 4), (4, 4)]
NV = [12, 12]
SPLIT_NV = [6, 6]   # chirality-split comparison: 2 x 6 = 12 coarse variables per site, as above
NU = 4
OMEGA = 0.8
SETUP_ITERS = 5
SA_SCALE = 4.0 / 3.0     # smoothed aggregation weight scale
TOL = 1e-10
DSLASH_L = 2048          # fine D^H D bandwidth lattice (working set far beyond the caches)
# The 20 systems of the precision workload (4 fields x 5 masses) solve as 5 grouped
# solves of 4: group k holds the four fields at their k-th mass, whose solves take
# alike many iterations, so no column of a group runs on masked while a slower one
# finishes (group_parts; measured on MI355X with that grouping: 5 x 4 1711-1731
# solves/s, 10 x 2 1680; with masses mixed in a group: 4 x 5 1506, 3 groups 1415,
# 6-8 uneven groups 1383-1540).
GROUPS = 5
GROUP_SIZE = 4

# Serving workload: Poisson streams of requests over 8 seeded fields per (lattice size,
# beta), sizes 64..512^2, beta 3, 6, 10 (500 sweeps, beta 10: 1000), masses
# m_c + {0.1, 0.05, 0.02, 0.01} with m_c = 0, the critical mass of the free field
# (for m > 0 every singular value of D is at least m, so every request is solvable;
# with m_c(beta) the median m_crit of sampled 128^2 fields, the two lightest masses
# fall below the critical point of some 256^2 and 512^2 fields), 1-16 Gaussian
# right-hand sides per request, 4x4 aggregates with Nv = 12 down to a coarsest
# lattice of at most 16^2, admission under a 200 GB HBM budget.
SERVE_SIZES = [64, 128, 256, 512]
SERVE_BETAS = [3.0, 6.0, 10.0]
SERVE_FIELDS = 8                       # per (size, beta)
SERVE_SWEEPS = {3.0: 500, 6.0: 500, 10.0: 1000}
SERVE_GAPS = [0.1, 0.05, 0.02, 0.01]
SERVE_NV = 12
SERVE_LOADS = [0.7]                    # offered load / saturation (--serve-full: 0.5, 0.7, 0.9 and a cold run)
# Mixed solves of the serving and chirality legs store the FP32 V-cycle's operators
# (coarse links on the vector-ALU path, prolongators, coarsest dense inverse) in FP16
# (smg.STORE_F16).
OPERATOR_STORAGE = 2
# Mixed-precision variants of the headline, on the same systems:
# (name, operator_storage, coarsest_fp64).  The first gives `value`.
VARIANTS = [
    ("f16_ops_f16_coarsest", 2, False),   # FP16 copies of links, P and the coarsest inverse
    ("f16_ops_fp64_coarsest", 2, True),   # FP16 links and P, the coarsest inverse applied in FP64
    ("f32_ops_fp64_coarsest", 0, True),   # FP32 operators, FP64 coarsest solve (the configuration as stated)
]
SERVE_BUDGET = 200 * 10**9
SERVE_CAPACITY = 16

# Multi-RHS workload: 32 Z2-noise sources on one 512x512 field at beta = 6 (500
# sweeps, seed 3000) at the mass where lambda_min(A)/lambda_max(A) = 1e-4, 3 levels of
# 4x4 aggregates with Nv = 16 (coarse links 16x16 on the matrix cores, dense inverse
# of the 16384-variable coarsest operator applied in FP64, BF16 storage of the fine
# smoother iterates and FP16 storage of the prolongators in the mixed solve).
MRHS_L = 512
MRHS_SEED = 3000
MRHS_NRHS = 32
MRHS_NV = [16, 16]

# Large single field: 2048x2048 at beta = 10 (1000 sweeps, seed 5000), 4 levels
# 2048^2 -> (4x4) 512^2 -> (2x2) 256^2 -> (2x2) 128^2 with Nv = 16, the coarsest
# level (262144 variables, a dense inverse would take 1.1 TB) solved by CG, 64
# Gaussian right-hand sides; the mass puts lambda_min(A)/lambda_max(A) near 1e-5 on
# this field (measured in the run by block inverse iteration).
C5_L = 2048
C5_BETA = 10.0
C5_SWEEPS = 1000
C5_SEED = 5000
C5_NRHS = 64
C5_MASS = -0.027
C5_BLOCKS = [(4, 4), (2, 2), (2, 2)]
C5_NV = [16, 16, 16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_masses():
    with open(os.path.join(ROOT, "workloads", "masses_256_beta6.json")) as f:
        data = json.load(f)
    out = {}
    for fld in data["fields"]:
        assert fld["L"] == L and fld["beta"] == BETA and fld["sweeps"] == SWEEPS
        out[fld["seed"]] = [m["mass"] for m in fld["masses"]]
    return out


def make_field(seed):
    import synth

    return synth.links_from_angles(synth.metropolis_u1(L, L, BETA, SWEEPS, seed))


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample (child process, one thread)
# ---------------------------------------------------------------------------

C1 = dict(L=32, beta=3.0, sweeps=200, seed=1000, mass=0.1, b_seed=0, blocks=[(4, 4)], nv=[8], rnd_seed=1)


def cpu_baseline_leg():
    """The FP64 oracle on the host (child process; it waits for "go" on stdin so that
    it does not share the host with the GPU legs timed before it).

    * The precision configuration, one field in full (field 2000): the adaptive setup
      at its lightest mass, then for each of its 5 masses the re-mass (set_mass) and the
      MG-CG solve, with BLAS on every host core; then the same 5 solves again with BLAS
      on one thread (threadpoolctl).  The sparse products are single-threaded either way.
    * The plain-method configuration (32^2, beta 3, m 0.1, 2 levels, CG coarsest):
      setup and solve.
    Returns None at end of input without "go"."""
    if sys.stdin.readline().strip() != "go":
        return None
    from threadpoolctl import threadpool_info, threadpool_limits

    import synth
    from oracle import multigrid as mg
    from oracle.wilson import dirac_matrix, normal_matrix

    out = {}
    # plain method (c1)
    U1 = synth.links_from_angles(synth.metropolis_u1(C1["L"], C1["L"], C1["beta"], C1["sweeps"], C1["seed"]))
    R1 = synth.setup_randoms(C1["L"], C1["L"], C1["blocks"], C1["nv"], C1["rnd_seed"])
    A1 = normal_matrix(U1, C1["mass"])
    t0 = time.perf_counter()
    h1 = mg.adaptive_setup(A1, (C1["L"], C1["L"], 2), C1["blocks"], C1["nv"], R1, nu=NU, omega=OMEGA,
                           setup_iters=SETUP_ITERS, coarsest="cg", sa_scale=SA_SCALE)
    s1 = time.perf_counter() - t0
    rhs1 = dirac_matrix(U1, C1["mass"]).conj().T @ synth.gaussian(2 * C1["L"] ** 2, C1["b_seed"])
    t0 = time.perf_counter()
    _, info1 = mg.mg_cg(h1, rhs1, TOL)
    out["c1"] = dict(setup_s=s1, solve_s=time.perf_counter() - t0, iterations=info1.iterations,
                     relres=info1.relres)
    # precision configuration, field SEEDS[0] in full
    seed = SEEDS[0]
    masses = sorted(load_masses()[seed])
    U = make_field(seed)
    m_light = masses[0]
    R = synth.setup_randoms(L, L, BLOCKS, NV, seed)
    t0 = time.perf_counter()
    h = mg.adaptive_setup(normal_matrix(U, m_light), (L, L, 2), BLOCKS, NV, R, nu=NU, omega=OMEGA,
                          setup_iters=SETUP_ITERS, sa_scale=SA_SCALE)
    setup_s = time.perf_counter() - t0
    b = synth.gaussian(2 * L * L, 10000 * 2 + 0)
    hs, rhss, remass_s, solve_all, iters, res = [], [], [], [], [], []
    for m in masses:
        t0 = time.perf_counter()
        hm = h if m == m_light else mg.set_mass(h, normal_matrix(U, m), [r[0] for r in R], NU, OMEGA)
        if m != m_light:
            remass_s.append(time.perf_counter() - t0)
        rhs = dirac_matrix(U, m).conj().T @ b
        t0 = time.perf_counter()
        _, info = mg.mg_cg(hm, rhs, TOL)
        solve_all.append(time.perf_counter() - t0)
        iters.append(info.iterations)
        res.append(info.relres)
        hs.append(hm)
        rhss.append(rhs)
    solve_one = []
    with threadpool_limits(limits=1):
        for hm, rhs in zip(hs, rhss):
            t0 = time.perf_counter()
            mg.mg_cg(hm, rhs, TOL)
            solve_one.append(time.perf_counter() - t0)
    blas_threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    out.update(setup_s=setup_s, remass_s=remass_s, solve_s=solve_all, solve_s_1thread=solve_one, iterations=iters,
               relres=res, masses=masses, blas_threads=blas_threads, cores=len(os.sched_getaffinity(0)))
    return out


def start_cpu_baseline():
    # started before anything touches the GPU (a GPU process does not start programs);
    # it waits for "go" on stdin.  BLAS may use every core the process may run on.
    ncores = str(len(os.sched_getaffinity(0)))
    env = dict(os.environ, OMP_NUM_THREADS=ncores, OPENBLAS_NUM_THREADS=ncores, MKL_NUM_THREADS=ncores)
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-leg"], env=env,
                            stdin=subprocess.PIPE, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# GPU
# ---------------------------------------------------------------------------

def serve_mcrit(beta):
    """Median m_crit (the mass minimising lambda_min(A)) of the sampled 128^2 fields of
    this beta (workloads/masses_128_beta*.json, found offline with the oracle)."""
    import statistics

    with open(os.path.join(ROOT, "workloads", f"masses_128_beta{int(beta)}.json")) as f:
        data = json.load(f)
    return statistics.median(fld["m_star"] for fld in data["fields"])


def mrhs_field(_=None):
    import synth

    return synth.links_from_angles(synth.metropolis_u1(MRHS_L, MRHS_L, BETA, SWEEPS, MRHS_SEED))


def mrhs_mass():
    with open(os.path.join(ROOT, "workloads", "masses_512_beta6_s3000.json")) as f:
        data = json.load(f)
    fld = data["fields"][0]
    assert fld["L"] == MRHS_L and fld["seed"] == MRHS_SEED and fld["sweeps"] == SWEEPS
    return fld["masses"][0]["mass"], fld["masses"][0]["ratio"]


def mrhs_leg(args, torch, smg, dev, U):
    """32 right-hand sides on one 512^2 field: mixed (FP32 MG-CG with the matrix-core
    coarse operator, FP64 defect correction) against plain FP64 MG-CG."""
    import ctypes

    import numpy as np

    import synth

    mass, ratio = mrhs_mass()
    n = 2 * MRHS_L * MRHS_L
    p = smg.make_params(MRHS_L, MRHS_L, mass, levels=3, blocks=[(4, 4), (4, 4)], nv=MRHS_NV,
                        setup_iters=SETUP_ITERS, smoother_steps=NU, smoother_omega=OMEGA, seed=MRHS_SEED,
                        sa_scale=SA_SCALE, mfma_min_rhs=16, smoother_storage=smg.STORE_BF16,
                        operator_storage=OPERATOR_STORAGE)
    g = torch.from_numpy(np.ascontiguousarray(U)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = smg.Solver(g, p)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    eta = torch.from_numpy(synth.z2_noise((MRHS_NRHS, n), 10 * MRHS_SEED)).to(dev)
    rhs = s.apply_D(eta, dagger=True)
    x = torch.empty_like(rhs)
    torch.cuda.synchronize()
    time.sleep(1.0)  # an idle gap that separates the setup from the solves in a kernel trace
    out = {}
    for name, prec in (("mixed", smg.MIXED), ("fp64", smg.FP64)):
        _, st, code = s.solve(rhs, tol=TOL, maxiter=2000, precision=prec, out=x)
        if code != 0 or max(q["true_relres"] for q in st) > TOL:
            raise RuntimeError(f"multi-RHS {name} solve did not converge: {st[0]}")
        torch.cuda.synchronize()
        reps = max(1, args.mrhs_steps)
        t0 = time.perf_counter()
        for _ in range(reps):
            s.solve(rhs, tol=TOL, maxiter=2000, precision=prec, out=x)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = dict(solves_per_s=MRHS_NRHS / dt, seconds_per_batch=dt,
                         mean_iterations=float(np.mean([q["iterations"] for q in st])),
                         max_relres=max(q["true_relres"] for q in st))
        log(f"multi-RHS {name}: {MRHS_NRHS / dt:.1f} solves/s ({dt * 1e3:.1f} ms per {MRHS_NRHS} RHS)")
    # matrix-core utilisation of the level-1 coarse operator (128^2 sites, nc = 16, 32 RHS),
    # HIP events on the stream the kernel runs on
    cx, ct, nc = s.level_info(1)
    nl = cx * ct * nc
    v32 = torch.randn(MRHS_NRHS * nl, dtype=torch.complex64, device=dev)
    y32 = torch.empty_like(v32)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    lib = smg.load_library()
    h = s.handle
    px, py = ctypes.c_void_p(v32.data_ptr()), ctypes.c_void_p(y32.data_ptr())
    nul = ctypes.c_void_p()
    dur = timed_events(lambda: lib.smg_level_op_f32(h, 1, 0, 0.0, px, py, nul, nul, MRHS_NRHS, sp), 100, stream)
    flops = 72.0 * nc * nc * MRHS_NRHS * cx * ct
    mfma = dict(kernel=f"coarse operator on the matrix cores (k_coarse_mfma_tw: strips of 4 sites, rows of V staged "
                       f"under the MFMAs), {cx}x{ct} sites, nc={nc}, "
                       f"{MRHS_NRHS} RHS, FP32 arithmetic on the FP16 copy of the links (power-of-two scale)",
                bound="mfma", achieved=flops / dur / 1e12, peak=157.3,
                unit="TFLOP/s", frac=flops / dur / 1e12 / 157.3, avg_launch_us=dur * 1e6, flops_per_launch=flops)
    # the same operator in FP64 (the plain solve's) on the FP64 matrix cores
    v64 = torch.randn(MRHS_NRHS * nl, dtype=torch.complex128, device=dev)
    y64 = torch.empty_like(v64)
    qx, qy = ctypes.c_void_p(v64.data_ptr()), ctypes.c_void_p(y64.data_ptr())
    dur64 = timed_events(lambda: lib.smg_level_op(h, 1, 0, 0.0, qx, qy, nul, nul, MRHS_NRHS, sp), 50, stream)
    mfma64 = dict(kernel=f"k_coarse_mfma64, {cx}x{ct} sites, nc={nc}, {MRHS_NRHS} RHS, FP64", bound="mfma",
                  achieved=flops / dur64 / 1e12, peak=78.6, unit="TFLOP/s", frac=flops / dur64 / 1e12 / 78.6,
                  avg_launch_us=dur64 * 1e6)
    del v64, y64
    s.close()
    del g, eta, rhs, x, v32, y32
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return dict(workload=(f"{MRHS_L}x{MRHS_L} U(1) beta={BETA:g} ({SWEEPS} sweeps, seed {MRHS_SEED}), mass {mass:.5f} "
                          f"(lambda_min/lambda_max {ratio:.1e}), {MRHS_NRHS} Z2-noise sources (rhs = D^H eta), "
                          f"3 levels 4x4, Nv=16, nu={NU}, dense coarsest inverse, tol {TOL:g}; mixed: FP32 inner "
                          f"MG-CG, BF16 storage of the fine smoother iterates, FP16 storage of the prolongators, "
                          f"FP16-stored coarse links on the FP32 matrix cores, the coarsest inverse applied in FP64; FP64: "
                          f"coarse links and the coarsest inverse on the FP64 matrix cores"),
                setup_s=setup_s, mixed=out["mixed"], fp64=out["fp64"],
                mixed_over_fp64=out["mixed"]["solves_per_s"] / out["fp64"]["solves_per_s"], mfma=mfma,
                mfma64=mfma64)


def c5_leg(args, torch, smg, dev):
    """The large single field: adaptive setup at 2048^2, then 64 right-hand sides
    solved by plain FP64 MG-CG and by the mixed solver (FP32 MG-CG with BF16 storage
    of the fine smoother iterates and the coarse links on the FP32 matrix cores,
    coarsest CG in FP32 inside the V-cycle, FP64 defect correction) to 1e-10."""
    import ctypes

    import numpy as np

    import synth

    t_start = time.perf_counter()
    last = [0.0]
    coarse_its = []  # iterations of every coarsest CG solve of the current timed solve

    def progress(stage, level, step, total, value):
        now = time.perf_counter()
        if stage == "coarsest-cg":
            coarse_its.append(step)
        if stage in ("calibrate", "coarsest", "refinement") or now - last[0] > 10.0:
            last[0] = now
            log(f"c5 {stage} level {level}: {step}/{total} ({value:.2e}) at {now - t_start:.0f} s")

    smg.set_progress(progress)
    n = 2 * C5_L * C5_L
    th = synth.metropolis_u1_device(C5_L, C5_L, C5_BETA, C5_SWEEPS, C5_SEED, device=dev)[0]
    plaq = torch.cos(th[0] + torch.roll(th[1], -1, 1) - torch.roll(th[0], -1, 0) - th[1]).mean().item()
    U = torch.exp(1j * th).contiguous()
    del th
    torch.cuda.synchronize()
    field_s = time.perf_counter() - t_start
    log(f"c5 field {C5_L}^2 beta {C5_BETA:g}: {field_s:.1f} s, plaquette {plaq:.5f}")
    p = smg.make_params(C5_L, C5_L, C5_MASS, levels=4, blocks=C5_BLOCKS, nv=C5_NV, setup_iters=SETUP_ITERS,
                        smoother_steps=NU, smoother_omega=OMEGA, seed=C5_SEED, sa_scale=SA_SCALE,
                        coarsest=smg.COARSEST_CG, mfma_min_rhs=16, smoother_storage=smg.STORE_BF16)
    plan = {name: smg.query_bytes(p, C5_NRHS, prec) for name, prec in (("fp64", smg.FP64), ("mixed", smg.MIXED))}
    t0 = time.perf_counter()
    s = smg.Solver(U, p)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"c5 setup {setup_s:.1f} s, {s.memory_bytes() / 1e9:.1f} GB")
    b = synth.gaussian_device(n, 10000 * 5, device=dev, count=C5_NRHS)
    rhs = s.apply_D(b, dagger=True)
    del b
    x = torch.empty_like(rhs)
    out = {}

    def run(solver, name, prec):
        # a first pass of one iteration allocates the solve's work vectors
        solver.solve(rhs, tol=TOL, maxiter=1, precision=prec, out=x)
        torch.cuda.synchronize()
        coarse_its.clear()
        t0 = time.perf_counter()
        _, st, code = solver.solve(rhs, tol=TOL, maxiter=2000, precision=prec, out=x)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cits = list(coarse_its)
        worst = max(q["true_relres"] for q in st)
        if code != 0 or worst > TOL:
            raise RuntimeError(f"2048^2 {name} solve did not converge: {st[0]}")
        out[name] = dict(solves_per_s=C5_NRHS / dt, seconds=dt,
                         mean_iterations=float(np.mean([q["iterations"] for q in st])),
                         max_relres=worst, vcycles=int(st[0]["vcycles"]), memory_gb=solver.memory_bytes() / 1e9,
                         coarsest_cg_solves=len(cits), coarsest_cg_iterations=sum(cits),
                         coarsest_cg_mean=float(np.mean(cits)) if cits else 0.0)
        log(f"c5 {name}: {dt:.2f} s for {C5_NRHS} RHS ({C5_NRHS / dt:.2f} solves/s), "
            f"{out[name]['mean_iterations']:.1f} iterations, max relres {worst:.2e}, "
            f"{len(cits)} coarsest CG solves of {out[name]['coarsest_cg_mean']:.0f} iterations on average")

    # FP64 on a second handle with the same hierarchy (smg_derive at the same mass), so
    # that the two solves' work vectors are not held at once
    d = s.derive(C5_MASS)
    run(d, "fp64", smg.FP64)
    # fine A = D^H D on the 64 right-hand sides (FP64; 64 B per site and RHS plus the links)
    stream = torch.cuda.current_stream()
    lib = smg.load_library()
    px, py = ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(x.data_ptr())
    sp = ctypes.c_void_p(stream.cuda_stream)
    dur = timed_events(lambda: lib.smg_apply_level(d.handle, 0, px, py, C5_NRHS, sp), 10, stream)
    abytes = C5_L * C5_L * (64.0 * C5_NRHS + 32.0)
    fineA = dict(kernel=f"k_normal_fused, {C5_L}^2, {C5_NRHS} RHS, FP64", avg_launch_ms=dur * 1e3,
                 algorithmic_gb=abytes / 1e9, achieved_tb_s=abytes / dur / 1e12, frac=abytes / dur / 8e12)
    log(f"c5 fine A, {C5_NRHS} RHS: {dur * 1e3:.2f} ms, {abytes / dur / 1e12:.2f} TB/s")
    # the coarse operators of 64 right-hand sides on the FP64 matrix cores (levels 1 and 3)
    coarse = {}
    for lev in (1, 3):
        cx, ct, nc = d.level_info(lev)
        nl = cx * ct * nc
        vl = synth.gaussian_device(nl, 13, device=dev, count=C5_NRHS)
        yl = torch.empty_like(vl)
        pv, pw = ctypes.c_void_p(vl.data_ptr()), ctypes.c_void_p(yl.data_ptr())
        nul = ctypes.c_void_p()
        dl = timed_events(lambda: lib.smg_level_op(d.handle, lev, 0, 0.0, pv, pw, nul, nul, C5_NRHS, sp), 10, stream)
        fl = 72.0 * nc * nc * C5_NRHS * cx * ct
        coarse[f"level{lev}"] = dict(kernel=f"k_coarse_mfma64, {cx}x{ct} sites, nc={nc}, {C5_NRHS} RHS, FP64",
                                     avg_launch_ms=dl * 1e3, tflops=fl / dl / 1e12, frac=fl / dl / 1e12 / 78.6)
        log(f"c5 level {lev} coarse operator, {C5_NRHS} RHS, FP64 matrix cores: {dl * 1e3:.3f} ms, "
            f"{fl / dl / 1e12:.1f} TFLOP/s")
        del vl, yl
    # spectral ratio: lambda_max by power iteration, lambda_min (an upper bound) by
    # block inverse iteration with Rayleigh-Ritz on 8 vectors
    v = synth.gaussian_device(n, 7, device=dev)
    for _ in range(50):
        w = d.apply_A(v)
        lmax = (torch.vdot(v[0], w[0]).real / torch.vdot(v[0], v[0]).real).item()
        v = w / torch.linalg.vector_norm(w)
    k = 8
    X = synth.gaussian_device(n, 11, device=dev, count=k)

    def orth(X):
        for i in range(k):
            for _ in range(2):
                for j in range(i):
                    X[i] -= torch.vdot(X[j], X[i]) * X[j]
            X[i] /= torch.linalg.vector_norm(X[i])
        return X

    X = orth(X)
    ritz, Y = [], None
    for _ in range(args.c5_inverse_iters):
        Y, _, _ = d.solve(X, tol=1e-8, maxiter=2000, precision=smg.FP64)
        X = orth(Y)
        H = (X.conj() @ d.apply_A(X).T).cpu().numpy()
        ritz = np.linalg.eigvalsh(0.5 * (H + H.conj().T)).tolist()
        log(f"c5 lowest Ritz values {ritz[0]:.4e} .. {ritz[-1]:.4e}, ratio {ritz[0] / lmax:.2e}")
    d.close()
    del X, Y, v, w
    run(s, "mixed", smg.MIXED)
    s.close()
    smg.set_progress(None)
    del U, rhs, x
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return dict(workload=(f"{C5_L}x{C5_L} U(1) beta={C5_BETA:g} ({C5_SWEEPS} sweeps, seed {C5_SEED}, torch device "
                          f"generator), mass {C5_MASS:g}, {C5_NRHS} Gaussian right-hand sides (rhs = D^H b), 4 levels "
                          f"4x4, 2x2, 2x2, Nv=16, nu={NU}, coarsest (128^2 x 16 = 262144 variables) by CG to 1e-12 "
                          f"(FP64) / 1e-6 (inside the FP32 V-cycle), tol {TOL:g}; mixed: FP32 inner MG-CG, BF16 "
                          f"storage of the fine smoother iterates, coarse links on the FP32 matrix cores; FP64: coarse "
                          f"links on the FP64 matrix cores"),
                plaquette=plaq, field_s=field_s, setup_s=setup_s, setup_gb=plan["fp64"][0] / 1e9,
                solve_gb={k_: v_[1] / 1e9 for k_, v_ in plan.items()}, lambda_max=lmax,
                lambda_min_ritz=ritz[0] if ritz else None,
                ratio_upper_bound=(ritz[0] / lmax) if ritz else None, lowest_ritz=ritz,
                fp64=out["fp64"], mixed=out["mixed"],
                mixed_over_fp64=out["mixed"]["solves_per_s"] / out["fp64"]["solves_per_s"], fine_A=fineA,
                coarse_fp64=coarse,
                seconds=time.perf_counter() - t_start)


def group_parts(syss, ng):
    """Indices of the systems of each of ng groups.  A group's solve runs until its
    slowest system converges, so systems that take alike many iterations share a
    group: the k-th mass of every field (each field's masses target the same spectral
    ratios), in consecutive chunks of near-equal size."""
    seen, rank = {}, []
    for _, _, seed, _ in syss:
        rank.append(seen.get(seed, 0))
        seen[seed] = rank[-1] + 1
    order = sorted(range(len(syss)), key=lambda j: (rank[j], j))
    base, extra = divmod(len(syss), ng)
    parts, at = [], 0
    for k in range(ng):
        size = base + (1 if k < extra else 0)
        parts.append(order[at:at + size])
        at += size
    return parts


def grouped_leg(args, torch, smg, syss, xs_single, streams):
    """The same mixed solves as grouped solves (smg_group_solve): the systems split
    into args.groups groups of one hierarchy shape, each group on its own stream and
    host thread, every launch serving all systems of its group.  The solutions are
    compared bit for bit with the single solves' (xs_single)."""
    from concurrent.futures import ThreadPoolExecutor

    ng = max(1, min(args.groups, len(syss), len(streams)))
    parts = group_parts(syss, ng)
    groups = [smg.Group([syss[j][0] for j in part], stream=streams[k]) for k, part in enumerate(parts)]
    rhs = [torch.stack([syss[j][1].reshape(-1) for j in part]) for part in parts]
    outs = [torch.empty_like(r) for r in rhs]
    recs = []

    def run(k, rec):
        with torch.cuda.stream(streams[k]):
            _, st, code = groups[k].solve(rhs[k], tol=TOL, maxiter=2000, out=outs[k], stream=streams[k])
            if code != 0 or max(q["true_relres"] for q in st) > TOL:
                raise RuntimeError(f"grouped solve did not converge: {st}")
            if rec is not None:
                rec.extend(q["iterations"] for q in st)

    pool = ThreadPoolExecutor(max_workers=ng)
    for f in [pool.submit(run, k, recs) for k in range(ng)]:
        f.result()
    torch.cuda.synchronize()
    equal = None if xs_single is None else all(torch.equal(outs[k][i], xs_single[j].reshape(-1))
                                               for k, part in enumerate(parts) for i, j in enumerate(part))
    time.sleep(1.0)  # an idle gap that separates the warm-up from the timed solves in a kernel trace
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for f in [pool.submit(run, k, None) for k in range(ng)]:
            f.result()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pool.shutdown()
    for g in groups:
        g.close()
    return dict(solves_per_s=len(syss) * args.steps / dt, groups=ng, systems_per_group=[len(p) for p in parts],
                members=parts, mean_iterations=sum(recs) / len(recs),
                equal_to_single=None if equal is None else bool(equal))


def legs_summary(dslash_2048, dslash_4096, c1, mrhs, serving, split, cpu):
    """The other legs' headline figures in a few numbers (their full records follow
    the config in the same line)."""
    def r(x, nd=4):
        return None if x is None else float(f"{x:.{nd}g}")

    out = {"fine_A_fp64_tb_s": {"2048": r(dslash_2048["achieved"] / 1e3), "4096": r(dslash_4096["achieved"] / 1e3)},
           "fine_A_fp64_frac": {"2048": r(dslash_2048["frac"], 3), "4096": r(dslash_4096["frac"], 3)}}
    if c1:
        out["plain_32"] = {"gpu_solve_s": r(c1["gpu_solve_s"]), "iterations": c1["iterations"],
                           "relres": r(c1["relres"], 3)}
    if mrhs:
        out["multi_rhs_512"] = {"mixed_solves_per_s": r(mrhs["mixed"]["solves_per_s"]),
                                "fp64_solves_per_s": r(mrhs["fp64"]["solves_per_s"]),
                                "mixed_over_fp64": r(mrhs["mixed_over_fp64"], 3),
                                "mfma_fp32_frac": r(mrhs["mfma"]["frac"], 3),
                                "mfma_fp64_frac": r(mrhs.get("mfma64", {}).get("frac"), 3)}
    if serving:
        out["serving"] = {"saturation_solves_per_s": r(serving["saturation_solves_per_s"]),
                          "solves_per_s_0.7": r(serving["solves_per_s"]), "p50_ms_0.7": r(serving["p50_ms"]),
                          "p99_ms_0.7": r(serving["p99_ms"])}
    if split:
        out["chirality_split_solves_per_s"] = r(split["mixed_solves_per_s"])
    if cpu:
        out["cpu_oracle_solves_per_s"] = r(cpu.get("value"))
    return out


def c1_leg(torch, smg, dev):
    """The plain-method configuration on the GPU: 32^2, beta 3 (200 sweeps, seed 1000),
    m = 0.1, b Gaussian (seed 0), rhs = D^H b, 2 levels of 4x4 with Nv = 8 from 5
    adaptive setup iterations, nu = 4, coarsest CG to 1e-12, FP64 MG-CG to 1e-10.
    Wall times of the setup and of the solve (the first call of each, and the median
    of 5 after it)."""
    import numpy as np

    import synth

    U = synth.links_from_angles(synth.metropolis_u1(C1["L"], C1["L"], C1["beta"], C1["sweeps"], C1["seed"]))
    R = synth.setup_randoms(C1["L"], C1["L"], C1["blocks"], C1["nv"], C1["rnd_seed"])
    p = smg.make_params(C1["L"], C1["L"], C1["mass"], levels=2, blocks=C1["blocks"], nv=C1["nv"],
                        setup_iters=SETUP_ITERS, smoother_steps=NU, smoother_omega=OMEGA, coarsest=smg.COARSEST_CG,
                        sa_scale=SA_SCALE)
    g = torch.from_numpy(U).to(dev)
    rnd = torch.from_numpy(np.concatenate([r.ravel() for r in R])).to(dev)
    b = torch.from_numpy(synth.gaussian(2 * C1["L"] ** 2, C1["b_seed"])).to(dev)
    setups, solves, st = [], [], None
    for _ in range(6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = smg.Solver(g, p, randoms=rnd)
        torch.cuda.synchronize()
        setups.append(time.perf_counter() - t0)
        rhs = s.apply_D(b, dagger=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st, code = s.solve(rhs, tol=TOL, maxiter=500, precision=smg.FP64)
        torch.cuda.synchronize()
        solves.append(time.perf_counter() - t0)
        if code != 0:
            raise RuntimeError(f"c1 solve did not converge: {st[0]}")
        s.close()
    return dict(workload="32x32 U(1) beta=3 (200 sweeps, seed 1000), m=0.1, 2 levels 4x4, Nv=8, nu=4, coarsest CG "
                         "1e-12, FP64 MG-CG to 1e-10, one Gaussian RHS",
                gpu_setup_s_first=setups[0], gpu_setup_s=sorted(setups[1:])[2], gpu_solve_s_first=solves[0],
                gpu_solve_s=sorted(solves[1:])[2], iterations=st[0]["iterations"], relres=st[0]["true_relres"])


def serving_leg(args, torch, smg, dev):
    """The request loop (continuous batching over a setup cache): fields drawn on the
    GPU, then a warm cache (every key that fits the budget built before the trace), the
    saturation throughput (all requests arriving at once), the offered loads of
    SERVE_LOADS times it, and with --serve-full a cold run (empty cache, setups inside
    the trace) at 0.7 x saturation."""
    import numpy as np

    import synth
    from paper_0710_3612_amd import serve

    t0 = time.perf_counter()
    fields, masses, sizes = {}, {}, {}
    mc = {b: 0.0 for b in SERVE_BETAS}  # sampled medians, for the record: serve_mcrit(beta)
    for si, Ls in enumerate(SERVE_SIZES):
        for bi, beta in enumerate(SERVE_BETAS):
            th = synth.metropolis_u1_device(Ls, Ls, beta, SERVE_SWEEPS[beta], 4000 + 100 * si + 10 * bi,
                                            count=SERVE_FIELDS, device=dev)
            for i in range(SERVE_FIELDS):
                key = f"L{Ls}_b{int(beta)}_{i}"
                ms = [round(mc[beta] + g, 6) for g in SERVE_GAPS]
                lv = serve.levels_for(Ls, 4, 16)  # coarsest lattice at most 16^2
                p = smg.make_params(Ls, Ls, min(ms), levels=lv, blocks=[(4, 4)] * (lv - 1), nv=[SERVE_NV] * (lv - 1),
                                    setup_iters=SETUP_ITERS, smoother_steps=NU, smoother_omega=OMEGA,
                                    seed=4000 + i, sa_scale=SA_SCALE, operator_storage=OPERATOR_STORAGE,
                                    remass_affine=True)
                fields[key] = (torch.polar(torch.ones_like(th[i]), th[i]).contiguous(), p)
                masses[key] = ms
                sizes[key] = Ls
            del th
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    log(f"serving: {len(fields)} fields on the GPU in {gen_s:.1f}s; m_c = {mc}")
    backend = serve.DeviceBackend(fields, mixed=True)
    keys = [(f, m) for f in fields for m in masses[f]]

    def run(srv, rate, seed, nreq):
        trace = serve.poisson_trace(nreq, rate, list(fields), masses, (1, 16), seed=seed)
        reqs = []
        for i, (t, f, m, k, sd) in enumerate(trace):
            n = 2 * sizes[f] ** 2
            reqs.append(serve.Request(seed * 100000 + i, f, m,
                                      (lambda n=n, sd=sd, k=k: synth.gaussian_device(n, sd, "cuda", k)), k, t))
        if rate == math.inf:
            for r in reqs:
                r.arrival = 0.0
        c0 = dict(setups=srv.cache.setups, derives=srv.cache.derives, evictions=srv.cache.evictions)
        ph0 = srv.phase_times()
        results = srv.run_trace(reqs, timeout=1800,
                                progress=lambda o, n: log(f"serving: {n - o} of {n} requests done"))
        summ = serve.latency_summary(results)
        bad = [r for r in results if not r.ok or max(r.true_relres) > TOL]
        by_size = {}
        for r in results:
            by_size.setdefault(sizes[r.field], []).append(r)
        ph1 = srv.phase_times()
        summ.update(phase_s={k: round(ph1[k] - ph0.get(k, 0.0), 3) for k in sorted(ph1)})
        summ.update(offered_rps=None if rate == math.inf else rate, failed=len(bad),
                    first_failure=(None if not bad else f"{bad[0].error} {bad[0].status} {bad[0].true_relres}"),
                    setups=srv.cache.setups - c0["setups"], derives=srv.cache.derives - c0["derives"],
                    evictions=srv.cache.evictions - c0["evictions"], resident_gb=srv.cache.used / 1e9,
                    mean_iterations=float(np.mean([i for r in results if r.ok for i in r.iterations])),
                    max_relres=max((max(r.true_relres) for r in results if r.ok), default=None),
                    p50_ms_by_size={str(k): serve.latency_summary(v)["p50_ms"] for k, v in sorted(by_size.items())},
                    p99_ms_by_size={str(k): serve.latency_summary(v)["p99_ms"] for k, v in sorted(by_size.items())})
        return summ

    def server():
        return serve.Server(backend, SERVE_BUDGET, capacity=SERVE_CAPACITY, tol=TOL, maxiter=2000,
                            precision=smg.MIXED, max_lanes=args.serve_lanes, keep_solutions=False,
                            fit_capacity=not args.serve_fixed_batches)

    # warm: every field's full setup at its lightest mass (the expensive part), then
    # the other masses, small lattices first, while 90% of the budget holds them
    srv = server()
    lightest = [(f, min(masses[f])) for f in fields]
    others = sorted([k for k in keys if k not in lightest], key=lambda k: (sizes[k[0]], k[0], k[1]))
    warm_keys, used = [], 0
    # room for every lane's batch of the largest lattice stays free
    room = 0.9 * SERVE_BUDGET - args.serve_lanes * max(backend.batch_estimate(f, SERVE_CAPACITY) for f in fields)
    for f, m in sorted(lightest, key=lambda k: sizes[k[0]]) + others:
        need = backend.estimate(f, 0)
        if used + need > room:
            continue
        warm_keys.append((f, m))
        used += need
    # one field of each lattice size first, built alone (every kernel instantiation a
    # size uses is launched once before eight threads build the others)
    firsts = []
    for f, m in warm_keys:
        if sizes[f] not in {sizes[g] for g in firsts}:
            firsts.append(f)
    warm_keys = [k for f in firsts for k in warm_keys if k[0] == f] + [k for k in warm_keys if k[0] not in firsts]
    t0 = time.perf_counter()
    srv.warm(warm_keys, workers=8, serial=len(firsts))
    torch.cuda.synchronize()
    warm_s = time.perf_counter() - t0
    log(f"serving: warmed {len(warm_keys)} of {len(keys)} keys in {warm_s:.1f}s ({srv.cache.used / 1e9:.1f} GB)")
    nreq = max(args.serve_requests, 2000) if args.serve_full else args.serve_requests
    out = dict(workload=(f"{nreq} Poisson requests per run over {len(fields)} fields "
                         f"({'/'.join(map(str, SERVE_SIZES))}^2 x beta 3/6/10 x {SERVE_FIELDS}, 500 sweeps, beta 10: "
                         f"1000, drawn on the GPU), masses {SERVE_GAPS} (above the free-field critical mass 0), "
                         f"1-16 Gaussian RHS each, 4x4 "
                         f"aggregates down to a coarsest lattice of at most 16^2 (2/3/3/4 levels), "
                         f"Nv={SERVE_NV}, mixed precision (FP64 flexible CG, FP32 V-cycle, FP16 operator copies), "
                         f"{'' if args.serve_fixed_batches else '4-'}{SERVE_CAPACITY}-slot batches, {args.serve_lanes} lanes, "
                         f"budget {SERVE_BUDGET / 1e9:.0f} GB, "
                         f"tol {TOL:g}"),
               keys=len(keys), warm_keys=len(warm_keys), warm_s=warm_s, field_generation_s=gen_s)
    sat = run(srv, math.inf, 11, nreq)
    sat_rps = sat["requests"] / sat["span_s"]
    out["saturation"] = sat
    log(f"serving: saturation {sat['solves_per_s']:.1f} solves/s, {sat_rps:.1f} requests/s")
    loads = [0.5, 0.7, 0.9] if args.serve_full else SERVE_LOADS
    for j, frac in enumerate(loads):
        out[f"load_{frac:g}"] = run(srv, frac * sat_rps, 12 + j, nreq)
        q = out[f"load_{frac:g}"]
        log(f"serving: load {frac:g} x saturation: p50 {q['p50_ms']:.1f} ms, p99 {q['p99_ms']:.1f} ms, "
            f"{q['solves_per_s']:.1f} solves/s")
    srv.close()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if args.serve_full:
        srv = server()
        out["cold_0.7"] = run(srv, 0.7 * sat_rps, 13, nreq)
        q = out["cold_0.7"]
        log(f"serving: cold at 0.7 x saturation: p50 {q['p50_ms']:.1f} ms, p99 {q['p99_ms']:.1f} ms")
        srv.close()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    main_pt = out[f"load_{0.7:g}"]
    out.update(p50_ms=main_pt["p50_ms"], p99_ms=main_pt["p99_ms"], solves_per_s=main_pt["solves_per_s"],
               saturation_solves_per_s=sat["solves_per_s"], saturation_requests_per_s=sat_rps)
    return out

def timed_graph(fn, reps, stream, per_graph=20):
    """Average duration of fn() with the launches replayed from a HIP graph of
    per_graph calls, HIP events on `stream`: for kernels of a few microseconds the
    host cannot enqueue single launches as fast as the GPU retires them, and the
    graph removes that host time from the measurement.  fn must only launch kernels
    on `stream` (no allocation, copy or synchronisation)."""
    import torch

    with torch.cuda.stream(stream):
        fn()
    stream.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for _ in range(per_graph):
            fn()
    n = max(1, reps // per_graph)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        g.replay()
        start.record(stream)
        for _ in range(n):
            g.replay()
        stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) * 1e-3 / (n * per_graph)


def timed_events(fn, reps, stream):
    """Average duration of fn() over reps launches, HIP events on `stream`."""
    import torch

    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        fn()
        start.record(stream)
        for _ in range(reps):
            fn()
        stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) * 1e-3 / reps


COUNTERS_MD = os.path.join(ROOT, "profiles", "coarse_f16_level1_256_counters.md")
COUNTERS_MD_GROUP = os.path.join(ROOT, "profiles", "coarse_f16_level1_256_group4_counters.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_0710_3612_amd", "csrc", "multigrid.hip")


def kernel_source_digest():
    """sha256 of the roofline kernel's own source: the single-RHS coarse kernel
    (k_coarse_sv) and the launch functions that reach it (edits elsewhere in the file
    leave its counters valid)."""
    import hashlib

    text = open(KERNEL_SOURCE).read()
    parts = []
    for start in ("template <typename R, int MODE, int Q, typename TL, bool GRP = false>\n"
                  "__global__ void __launch_bounds__(kThreads) k_coarse_sv(",
                  "void launch_coarse_t(", "void launch_coarse_h16("):
        i = text.index(start)
        parts.append(text[i:text.index("\n}\n", i) + 3])
    return hashlib.sha256("".join(parts).encode()).hexdigest()


def measured_traffic(path):
    """HBM bytes per launch of a roofline kernel from its committed counter runs
    (FETCH_SIZE and WRITE_SIZE, calibrated on a copy of known size), or None when
    the kernel source changed since they were taken."""
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = dict(line.split(" = ", 1) for line in text.splitlines() if " = " in line and line[:1].isalpha())
    if vals.get("kernel_source_sha256", "").strip() != kernel_source_digest():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def coarse_roofline(smg, lib, s, sp, stream, reps, torch, dev, group=None):
    """Average launch time of the FP32 coarse operator on level 1 (the kernel that
    dominates the mixed-precision V-cycle), and its algorithmic bytes: 9 link
    blocks of nc x nc complex values per coarse site (4 bytes each in FP16 operator
    storage, 8 in FP32) plus the input and output vector (complex64), per system.
    With a group (smg.Group) one launch applies every system's operator to its own
    column, as inside the grouped solves."""
    import ctypes

    cx, ct, nc = s.level_info(1)
    G = 1 if group is None else len(group.solvers)
    v = torch.randn(G * cx * ct * nc, dtype=torch.complex64, device=dev)
    y = torch.empty_like(v)
    px, py = ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(y.data_ptr())
    if group is None:
        dur = timed_graph(lambda: lib.smg_apply_level_f32(s.handle, 1, px, py, 1, sp), reps, stream)
    else:
        gh, nul = group.handle, ctypes.c_void_p()
        dur = timed_graph(lambda: lib.smg_group_level_op_f32(gh, 1, 0, px, py, nul, sp), reps, stream)
    h16 = s.params.operator_storage == smg.STORE_F16
    nbytes = G * (9 * nc * nc * (4 if h16 else 8) * cx * ct + 2 * cx * ct * nc * 8)
    gbs = nbytes / dur / 1e9
    q = (nc + 3) // 4
    if 4 <= nc <= 16:  # the LDS-staged kernel, one pass of q columns per wave
        name = f"k_coarse_sv<float,0,{q},{'hfc' if h16 else 'cpx<float>'}{',true' if group is not None else ''}>"
    else:
        cols = 2 if q <= 2 else min(q, 4)  # columns per pass, as the launcher picks them
        name = f"k_coarse<float,0,1,{cols}{',hfc' if h16 else ''}>"
    what = "FP16 links (scaled), FP32 arithmetic" if h16 else "FP32"
    per = "single RHS" if group is None else f"{G} systems per launch (each its own links), one RHS each"
    # context: a plain device copy moving the same bytes (half read, half written), timed the same way
    src = torch.ones(nbytes // 8, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dcopy = timed_graph(lambda: dst.copy_(src), reps, stream)
    return dict(kernel=f"{name}: coarse 9-point operator, {what}, level 1 ({cx}x{ct} sites, nc={nc}), {per}",
                bound="hbm", achieved=gbs, peak=8000.0, unit="GB/s", frac=gbs / 8000.0,
                traffic=measured_traffic(COUNTERS_MD if group is None else COUNTERS_MD_GROUP),
                avg_launch_us=dur * 1e6, bytes_per_launch=nbytes,
                same_bytes_copy_us=dcopy * 1e6, same_bytes_copy_GBps=nbytes / dcopy / 1e9)


def kernel_probe(reps):
    """Launch only the roofline kernel and a plain copy of known size (for PMC runs)."""
    import ctypes

    import numpy as np
    import torch

    import paper_0710_3612_amd as smg
    import synth

    dev = torch.device("cuda:0")
    U = synth.links_from_angles(synth.metropolis_u1(L, L, BETA, 20, SEEDS[0]))
    p = smg.make_params(L, L, 0.0, levels=3, blocks=BLOCKS, nv=NV, setup_iters=0, smoother_steps=NU,
                        smoother_omega=OMEGA, seed=SEEDS[0], sa_scale=SA_SCALE, operator_storage=OPERATOR_STORAGE)
    s = smg.Solver(torch.from_numpy(U).to(dev), p)
    lib = smg.load_library()
    stream = torch.cuda.Stream(dev)  # graphs are not captured on the null stream
    sp = ctypes.c_void_p(stream.cuda_stream)
    single = coarse_roofline(smg, lib, s, sp, stream, reps, torch, dev)
    # a group of GROUP_SIZE systems of the benchmark's shape, as the grouped solves launch
    # them (here one field at further masses; the kernel's work does not depend on which)
    sys_ = [s] + [s.derive(0.01 * k) for k in range(1, GROUP_SIZE)]
    with smg.Group(sys_, stream=stream) as g:
        roof = coarse_roofline(smg, lib, s, sp, stream, reps, torch, dev, group=g)
    for d in sys_[1:]:
        d.close()
    # calibration: an elementwise FP32 kernel that reads and writes 64 MiB each
    a = torch.ones(16 << 20, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.add(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps(dict(roofline=roof, roofline_single=single, copy_read_bytes=a.numel() * 4,
                          copy_write_bytes=b.numel() * 4)))


def dslash_probe(Ld, reps):
    """Launch only the fine FP64 A = D^H D at Ld^2 (single RHS) and a plain FP32
    elementwise kernel reading and writing 64 MiB each (the counters' calibration),
    for kernel-trace and counter runs; prints the event-timed rate."""
    import ctypes

    import numpy as np
    import torch

    import paper_0710_3612_amd as smg
    import synth

    dev = torch.device("cuda:0")
    th = np.random.default_rng(5000 + Ld).uniform(-math.pi, math.pi, size=(2, Ld, Ld))
    s = smg.Solver(torch.from_numpy(np.exp(1j * th)).to(dev), smg.make_params(Ld, Ld, 0.01, levels=1))
    x = torch.from_numpy(synth.gaussian(2 * Ld * Ld, 6)).to(dev)
    y = torch.empty_like(x)
    lib = smg.load_library()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    px, py = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    dur = timed_events(lambda: lib.smg_apply_A(s.handle, px, py, 1, sp), reps, stream)
    nbytes = Ld * Ld * 96
    a = torch.ones(16 << 20, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.add(a, 1.0, out=b)
    torch.cuda.synchronize()
    print(json.dumps(dict(kernel="k_normal_fused FP64", L=Ld, avg_launch_us=dur * 1e6, bytes_per_launch=nbytes,
                          achieved_GBps=nbytes / dur / 1e9, copy_read_bytes=a.numel() * 4,
                          copy_write_bytes=b.numel() * 4)))


def mfma_probe(reps, f16=False):
    """Launch only the matrix-core coarse operator (512^2 hierarchy, level 1: 128^2 sites,
    nc = 16, 32 RHS; FP32 links, or with f16 the FP16 copy of the links) for profiler
    runs; prints its event-timed rate."""
    import ctypes

    import numpy as np
    import torch

    import paper_0710_3612_amd as smg
    import synth

    dev = torch.device("cuda:0")
    U = synth.links_from_angles(synth.metropolis_u1(MRHS_L, MRHS_L, BETA, 20, MRHS_SEED))
    p = smg.make_params(MRHS_L, MRHS_L, 0.0, levels=3, blocks=[(4, 4), (4, 4)], nv=MRHS_NV, setup_iters=0,
                        smoother_steps=NU, smoother_omega=OMEGA, seed=MRHS_SEED, sa_scale=SA_SCALE,
                        coarsest=smg.COARSEST_CG, mfma_min_rhs=16,
                        operator_storage=smg.STORE_F16 if f16 else smg.STORE_F32)
    s = smg.Solver(torch.from_numpy(np.ascontiguousarray(U)).to(dev), p)
    cx, ct, nc = s.level_info(1)
    v = torch.randn(MRHS_NRHS * cx * ct * nc, dtype=torch.complex64, device=dev)
    y = torch.empty_like(v)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    lib = smg.load_library()
    h = s.handle
    px, py, nul = ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p()
    dur = timed_events(lambda: lib.smg_level_op_f32(h, 1, 0, 0.0, px, py, nul, nul, MRHS_NRHS, sp), reps, stream)
    flops = 72.0 * nc * nc * MRHS_NRHS * cx * ct
    print(json.dumps(dict(kernel="k_coarse_mfma_tw", links="FP16 (scaled)" if f16 else "FP32", sites=cx * ct, nc=nc,
                          nrhs=MRHS_NRHS, avg_launch_us=dur * 1e6,
                          tflops=flops / dur / 1e12, frac=flops / dur / 1e12 / 157.3,
                          link_bytes=9 * nc * nc * (4 if f16 else 8) * cx * ct)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-leg", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--dslash-reps", type=int, default=200)
    ap.add_argument("--streams", type=int, default=16, help="concurrent solve streams")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests per serving run (--serve-full: 2000)")
    ap.add_argument("--serve-lanes", type=int, default=8, help="concurrent (field, mass) lanes")
    ap.add_argument("--serve-fixed-batches", action="store_true",
                    help="every lane's batch has 16 slots (default: sized to the right-hand sides queued for its "
                         "key, 4-16 slots)")
    ap.add_argument("--serve-full", action="store_true",
                    help="serving at 0.5, 0.7 and 0.9 x saturation and a cold run (longer)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-only", action="store_true", help="only the serving leg (prints its summary)")
    ap.add_argument("--no-mrhs", action="store_true")
    ap.add_argument("--no-group", action="store_true", help="skip the grouped solves of the headline systems")
    ap.add_argument("--groups", type=int, default=GROUPS, help="groups (streams) of the grouped headline solves")
    ap.add_argument("--group-only", action="store_true",
                    help="with --solves-only: time only the grouped solves (an idle second before the timed steps)")
    ap.add_argument("--no-split", action="store_true", help="skip the chirality-split comparison")
    ap.add_argument("--mrhs-only", action="store_true", help="only the multi-RHS leg (prints its summary)")
    ap.add_argument("--mrhs-steps", type=int, default=3)
    ap.add_argument("--c5", action="store_true",
                    help="only the 2048^2 four-level leg, 64 right-hand sides (prints its summary)")
    ap.add_argument("--c5-inverse-iters", type=int, default=6,
                    help="block inverse iterations for the 2048^2 leg's spectral ratio")
    ap.add_argument("--mfma-probe", action="store_true", help="only launch the matrix-core coarse operator")
    ap.add_argument("--probe-f16", action="store_true", help="--mfma-probe on the FP16 copy of the links")
    ap.add_argument("--dslash-probe", type=int, default=0, metavar="L",
                    help="only launch the fine FP64 A at L x L and a 64 MiB copy (for profiler runs)")
    ap.add_argument("--solves-only", action="store_true",
                    help="set up the precision workload, pause 1 s, run --steps mixed steps (for kernel traces)")
    ap.add_argument("--kernel-probe", action="store_true",
                    help="only launch the roofline kernel and a 64 MiB copy (for counter runs)")
    args = ap.parse_args()
    if args.kernel_probe:
        kernel_probe(args.dslash_reps)
        return 0
    if args.mfma_probe:
        mfma_probe(args.dslash_reps, args.probe_f16)
        return 0
    if args.dslash_probe:
        dslash_probe(args.dslash_probe, args.dslash_reps)
        return 0

    if args.cpu_baseline_leg:
        print(json.dumps(cpu_baseline_leg()))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        return 2

    if args.serve_only:
        import torch

        import paper_0710_3612_amd as smg

        print(json.dumps(serving_leg(args, torch, smg, torch.device("cuda:0"))))
        return 0

    if args.c5:
        import torch

        import paper_0710_3612_amd as smg

        print(json.dumps(c5_leg(args, torch, smg, torch.device("cuda:0"))))
        return 0

    if args.mrhs_only:
        import torch

        import paper_0710_3612_amd as smg

        U = mrhs_field()
        print(json.dumps(mrhs_leg(args, torch, smg, torch.device("cuda:0"), U)))
        return 0

    cpu_proc = None if args.no_cpu_baseline else start_cpu_baseline()

    import numpy as np
    from concurrent.futures import ProcessPoolExecutor

    import synth

    masses = load_masses()
    log("generating gauge fields")
    with ProcessPoolExecutor(max_workers=len(SEEDS) + 1) as ex:
        mrhs_future = None if args.no_mrhs else ex.submit(mrhs_field)
        fields = list(ex.map(make_field, SEEDS))
        mrhs_U = None if mrhs_future is None else mrhs_future.result()

    import torch

    import paper_0710_3612_amd as smg

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    torch.cuda.set_stream(stream)

    def T(a):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(dev)

    # ---- setup (timed separately) ---------------------------------------------
    # One hierarchy per field at its lightest mass (adaptive setup, mass coefficients
    # kept), the heavier masses derived from it.  Every storage variant gets its own
    # handles from the same random starts: the FP64 hierarchy is the same.
    def build_systems(opst, c64, timing):
        systems, keep = [], []
        for seed, U in zip(SEEDS, fields):
            ms = masses[seed]
            m_light = min(ms)
            p = smg.make_params(L, L, m_light, levels=3, blocks=BLOCKS, nv=NV, setup_iters=SETUP_ITERS,
                                smoother_steps=NU, smoother_omega=OMEGA, seed=seed, sa_scale=SA_SCALE,
                                operator_storage=opst, coarsest_fp64=c64, remass_affine=True)
            R = synth.setup_randoms(L, L, BLOCKS, NV, seed)
            g = T(U)
            rnd = T(np.concatenate([r.ravel() for r in R]))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s0 = smg.Solver(g, p, randoms=rnd)
            torch.cuda.synchronize()
            if timing is not None:
                timing["setup"].append(time.perf_counter() - t0)
            b = T(synth.gaussian(2 * L * L, 10000 * 2 + SEEDS.index(seed)))
            keep.append(s0)
            for m in ms:
                t0 = time.perf_counter()
                s = s0 if m == m_light else s0.derive(m)
                torch.cuda.synchronize()
                if m != m_light and timing is not None:
                    timing["remass"].append(time.perf_counter() - t0)
                rhs = s.apply_D(b, dagger=True)
                systems.append((s, rhs, seed, m))
                if s is not s0:
                    keep.append(s)
        return systems, keep

    timing = dict(setup=[], remass=[])
    variant_systems = {}
    for name, opst, c64 in VARIANTS:
        variant_systems[name] = build_systems(opst, c64, timing if not variant_systems else None)
        log(f"variant {name}: {len(variant_systems[name][0])} systems")
    systems = variant_systems[VARIANTS[0][0]][0]
    setup_s, remass_s = timing["setup"], timing["remass"]
    xs = [torch.empty_like(rhs) for _, rhs, _, _ in systems]

    # The systems are independent: worker threads, each with its own stream, keep
    # several solves in flight (ctypes releases the GIL during library calls).
    from concurrent.futures import ThreadPoolExecutor

    nwork = max(1, min(args.streams, len(systems)))
    streams = [torch.cuda.Stream(dev) for _ in range(nwork)]
    torch.cuda.synchronize()

    def run_share(w, syss, prec, rec):
        with torch.cuda.stream(streams[w]):
            for k in range(w, len(syss), nwork):
                s, rhs, seed, m = syss[k]
                x, st, code = s.solve(rhs, tol=TOL, maxiter=2000, precision=prec, out=xs[k], stream=streams[w])
                if code != 0 or st[0]["true_relres"] > TOL:
                    raise RuntimeError(f"solve did not converge: field {seed} mass {m} {st[0]}")
                if rec is not None:
                    rec.append(dict(seed=seed, mass=m, iterations=st[0]["iterations"],
                                    refinements=st[0]["refinements"], fine_applies=st[0]["fine_applies"],
                                    relres=st[0]["true_relres"], seconds=st[0]["seconds"]))

    pool = ThreadPoolExecutor(max_workers=nwork)

    def step(syss, prec, rec=None):
        futs = [pool.submit(run_share, w, syss, prec, rec) for w in range(nwork)]
        for f in futs:
            f.result()

    if args.solves_only and args.group_only:
        res = grouped_leg(args, torch, smg, systems, None, streams)
        print(json.dumps(dict(res, steps=args.steps)))
        return 0
    if args.solves_only:
        step(systems, smg.MIXED)
        torch.cuda.synchronize()
        time.sleep(1.0)  # an idle gap that separates setup from the steps in a kernel trace
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(systems, smg.MIXED)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pool.shutdown()
        print(json.dumps(dict(solves_per_s=len(systems) * args.steps / dt, steps=args.steps, streams=nwork)))
        return 0

    def timed(syss, prec):
        rec = []
        step(syss, prec, rec)                       # also the first warmup
        for _ in range(max(args.warmup - 1, 0)):
            step(syss, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(syss, prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dict(seconds=dt, solves=len(syss) * args.steps, records=rec)

    results = {}
    grouped = None
    for vi, (name, _opst, _c64) in enumerate(VARIANTS):
        results[name] = timed(variant_systems[name][0], smg.MIXED)
        log(f"mixed {name}: {results[name]['solves'] / results[name]['seconds']:.1f} solves/s")
        if vi == 0 and not args.no_group:
            grouped = grouped_leg(args, torch, smg, variant_systems[name][0], xs, streams)
            log(f"grouped {name}: {grouped['solves_per_s']:.1f} solves/s ({grouped['groups']} groups, "
                f"bitwise equal to the single solves: {grouped['equal_to_single']})")
    results["fp64"] = timed(systems, smg.FP64)
    log(f"fp64: {results['fp64']['solves'] / results['fp64']['seconds']:.1f} solves/s")
    for name, _opst, _c64 in VARIANTS[1:]:
        for s_ in variant_systems[name][1]:
            s_.close()
        variant_systems[name] = None
    results["mixed"] = results[VARIANTS[0][0]]

    # ---- chirality-split aggregates on the same systems: Nv = 6 candidates per level, each
    # block split by chirality, so the coarse levels carry 12 variables per site as above
    split = None
    if not args.no_split:
        ssys, ssetup = [], []
        rhs_of = {(seed, m): rhs for _, rhs, seed, m in systems}
        for seed, U in zip(SEEDS, fields):
            ms = masses[seed]
            m_light = min(ms)
            p = smg.make_params(L, L, m_light, levels=3, blocks=BLOCKS, nv=SPLIT_NV, setup_iters=SETUP_ITERS,
                                smoother_steps=NU, smoother_omega=OMEGA, seed=seed, sa_scale=SA_SCALE,
                                operator_storage=OPERATOR_STORAGE, split_chirality=True)
            R = synth.setup_randoms(L, L, BLOCKS, SPLIT_NV, seed, split=True)
            g, rnd = T(U), T(np.concatenate([r.ravel() for r in R]))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s0 = smg.Solver(g, p, randoms=rnd)
            torch.cuda.synchronize()
            ssetup.append(time.perf_counter() - t0)
            for m in ms:
                ssys.append((s0 if m == m_light else s0.derive(m), rhs_of[(seed, m)]))

        def run_split(w, rec):
            with torch.cuda.stream(streams[w]):
                for k in range(w, len(ssys), nwork):
                    s, rhs = ssys[k]
                    x, st, code = s.solve(rhs, tol=TOL, maxiter=2000, precision=smg.MIXED, out=xs[k],
                                          stream=streams[w])
                    if code != 0 or st[0]["true_relres"] > TOL:
                        raise RuntimeError(f"split solve did not converge: system {k} {st[0]}")
                    if rec is not None:
                        rec.append(st[0]["iterations"])

        srec = []
        for f in [pool.submit(run_split, w, srec) for w in range(nwork)]:
            f.result()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for f in [pool.submit(run_split, w, None) for w in range(nwork)]:
                f.result()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        split = dict(nv=SPLIT_NV, coarse_dof=[2 * k for k in SPLIT_NV],
                     mixed_solves_per_s=len(ssys) * args.steps / dt,
                     mean_iterations_mixed=sum(srec) / len(srec),
                     unsplit_mean_iterations_mixed=sum(r["iterations"] for r in results["mixed"]["records"])
                     / len(results["mixed"]["records"]),
                     setup_s_per_field=ssetup)
        log(f"chirality split: {split['mixed_solves_per_s']:.1f} solves/s, "
            f"{split['mean_iterations_mixed']:.2f} iterations")
        for s, _ in ssys:
            s.close()
        del ssys
    pool.shutdown()

    # ---- dominant-kernel roofline: the FP32 level-1 coarse operator of the mixed solve
    # (64x64 coarse sites, nc = 12) as the grouped solves launch it (the systems of the
    # first group, each its own links, one launch), and for one system alone; HIP events
    # on the launching stream
    import ctypes

    lib = smg.load_library()
    sp = ctypes.c_void_p(stream.cuda_stream)
    s = systems[0][0]
    roof_single = coarse_roofline(smg, lib, s, sp, stream, args.dslash_reps, torch, dev)
    roof = roof_single
    if grouped is not None:
        first = [systems[j][0] for j in grouped["members"][0]]
        with smg.Group(first, stream=stream) as g:
            roof = coarse_roofline(smg, lib, s, sp, stream, args.dslash_reps, torch, dev, group=g)

    # ---- fine D^H D at 2048^2 and 4096^2 (working sets beyond the caches) ------------
    def dslash(Ld):
        th = np.random.default_rng(5000 + Ld).uniform(-math.pi, math.pi, size=(2, Ld, Ld))
        sbig = smg.Solver(T(np.exp(1j * th)), smg.make_params(Ld, Ld, 0.01, levels=1))
        xb = T(synth.gaussian(2 * Ld * Ld, 6))
        yb = torch.empty_like(xb)
        hb = sbig.handle
        pxb, pyb = ctypes.c_void_p(xb.data_ptr()), ctypes.c_void_p(yb.data_ptr())
        dur = timed_events(lambda: lib.smg_apply_A(hb, pxb, pyb, 1, sp), args.dslash_reps, stream)
        nbytes = Ld * Ld * (32 + 32 + 32)     # psi in, A psi out, 2 links per site (FP64)
        sbig.close()
        del xb, yb
        torch.cuda.empty_cache()
        return dict(kernel=f"fine A = D^H D, {Ld}x{Ld}, FP64, single RHS", bound="hbm",
                    achieved=nbytes / dur / 1e9, peak=8000.0, unit="GB/s", frac=nbytes / dur / 1e9 / 8000.0,
                    avg_launch_us=dur * 1e6, bytes_per_launch=nbytes)

    dslash_2048 = dslash(DSLASH_L)
    dslash_4096 = dslash(2 * DSLASH_L)
    n_systems = len(systems)
    del systems, xs, s
    for s_ in variant_systems[VARIANTS[0][0]][1]:
        s_.close()
    variant_systems.clear()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    c1 = c1_leg(torch, smg, dev)
    mrhs = None if args.no_mrhs else mrhs_leg(args, torch, smg, dev, mrhs_U)

    cpu = None
    if cpu_proc is not None:
        # every GPU leg that times host-driven solves is done: the oracle may use the host
        # now, and the serving leg waits for it
        cpu_proc.stdin.write("go\n")
        cpu_proc.stdin.flush()
        out, err = cpu_proc.communicate(timeout=1800)  # also closes its stdin
        if cpu_proc.returncode == 0:
            leg = json.loads(out.strip().splitlines()[-1])
            n_s = len(leg["solve_s"])
            cpu = dict(value=n_s / sum(leg["solve_s"]), unit="solves/s", cores=leg["cores"], kind="oracle",
                       sample=(f"FP64 oracle (numpy/scipy; sparse products single-threaded, BLAS on "
                               f"{leg['blas_threads']} threads; {cpu_model()}, {leg['cores']} cores): field "
                               f"{SEEDS[0]} of the precision workload in full, MG-CG at its {n_s} masses "
                               f"({sum(leg['solve_s']):.1f}s of solves, iterations {leg['iterations']}); the adaptive "
                               f"setup ({leg['setup_s']:.1f}s) and the {len(leg['remass_s'])} re-masses "
                               f"({sum(leg['remass_s']):.1f}s) are not in the rate"),
                       single_thread_solves_per_s=n_s / sum(leg["solve_s_1thread"]),
                       setup_s=leg["setup_s"], remass_s=leg["remass_s"],
                       field_s=leg["setup_s"] + sum(leg["remass_s"]) + sum(leg["solve_s"]),
                       max_relres=max(leg["relres"]), cpu_model=cpu_model(), c1=leg["c1"])
            if c1 is not None:
                c1["oracle"] = leg["c1"]
        else:
            log("cpu baseline failed: " + err[-2000:])
    serving = None if args.no_serve else serving_leg(args, torch, smg, dev)

    mixed = results["mixed"]
    fp64 = results["fp64"]
    single_rate = mixed["solves"] / mixed["seconds"]
    # the job's throughput: the grouped solves, when their solutions equal the single
    # solves' bit for bit (checked in this run); otherwise the single solves
    use_grouped = grouped is not None and grouped["equal_to_single"] is True
    if grouped is not None and not use_grouped:
        log("grouped solutions differ from the single solves: the value is the single-solve rate")
    value = grouped["solves_per_s"] if use_grouped else single_rate

    def rate(r):
        return r["solves"] / r["seconds"]

    variants = {name: dict(operator_storage="f16" if opst == 2 else "f32",
                           coarsest="fp64 inverse" if c64 else ("fp16 copy" if opst == 2 else "fp32 copy"),
                           solves_per_s=rate(results[name]), over_fp64=rate(results[name]) / rate(fp64),
                           mean_iterations=sum(q["iterations"] for q in results[name]["records"])
                           / len(results[name]["records"]),
                           max_relres=max(q["relres"] for q in results[name]["records"]))
                for name, opst, c64 in VARIANTS}
    line = {
        "metric": "MG solves/s to 1e-10 residual (mixed vs FP64); D†D HBM GB/s; p99 latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": n_systems / value * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"f32 inner ({variants[VARIANTS[0][0]]['operator_storage']} operator storage, coarsest "
                 f"{variants[VARIANTS[0][0]]['coarsest']}) / f64 outer",
        "data": "synthetic",
        "config": {
            "workload": "256x256 U(1) beta=6, 4 fields x 5 masses (lambda_min/lambda_max 1e-2..1e-4), "
                        "3 levels 4x4, Nv=12, nu=4, 1 Gaussian RHS per system, tol 1e-10; mixed: FP32 MG-CG inside "
                        f"FP64 defect correction, variant {VARIANTS[0][0]} (others in mixed_variants); "
                        + (f"value: the {n_systems} systems as {grouped['groups']} grouped solves of "
                           f"{max(grouped['systems_per_group'])} (systems of like mass together) on "
                           f"{grouped['groups']} streams (grouped)"
                           if use_grouped else f"value: one solve per system on {nwork} streams"),
            "mixed_variants": variants,
            "systems_per_step": n_systems,
            "concurrent_streams": nwork,
            "single_solves_per_s": single_rate,
            "fp64_solves_per_s": fp64["solves"] / fp64["seconds"],
            "mixed_over_fp64": single_rate / (fp64["solves"] / fp64["seconds"]),
            "value_over_fp64": value / (fp64["solves"] / fp64["seconds"]),
            "setup_s_per_field": setup_s,
            "remass_s_mean": sum(remass_s) / max(len(remass_s), 1),
            "mean_iterations_mixed": sum(r["iterations"] for r in mixed["records"]) / len(mixed["records"]),
            "mean_iterations_fp64": sum(r["iterations"] for r in fp64["records"]) / len(fp64["records"]),
            "max_relres": max(r["relres"] for r in mixed["records"] + fp64["records"]),
            "grouped": grouped,
            "legs": legs_summary(dslash_2048, dslash_4096, c1, mrhs, serving, split, cpu),
        },
        "roofline": roof,
        "roofline_single": roof_single,
        "dslash": dslash_2048,
        "dslash_4096": dslash_4096,
        "cpu_baseline": cpu,
        "plain_method_c1": c1,
        "multi_rhs": mrhs,
        "serving": serving,
        "chirality_split": split,
    }
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
