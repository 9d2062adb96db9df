"""Write masses at prescribed spectral ratios lambda_min(A)/lambda_max(A) (offline).

The paper sweeps the mass gap m - m_crit towards zero (Results section) but does
not give m_crit.  The benchmark instead fixes, per gauge field, the masses at which
the condition number of A = D^H D reaches given ratios.  This script finds them
with the FP64 oracle's sparse D and A:

  * lambda_min(A(m)) = sigma_min(D(m))^2 by shift-invert Lanczos, with
    A^{-1} = D^{-1} D^{-H} from a sparse LU of D;
  * lambda_max(A(m)) by 60 power iterations (about 1% accurate, enough for a ratio);
  1. scan lambda_min on a grid, refine the minimiser m* by golden section;
  2. for each target ratio r, bisect on m > m* for lambda_min/lambda_max = r; if
     the field is gapped and r is out of reach, m* is used and the reached ratio
     is recorded.

For the 512^2 lattice (one field, one target) a full scan is too slow (each LU of
D takes most of a minute and some near-critical ones far longer), so the target is
reached from a starting mass by secant steps on sigma_min(D) = sqrt(lambda_min(A)),
which moves almost linearly with m away from m_crit; m* is not searched there.

Usage: python -m workloads.make_masses [256_beta6 | 512_beta6 | 512_beta6_s3000 | 128_beta3 | 128_beta6 |
       128_beta10 | 128_beta6_cold | 128_beta10_cold]
       (writes workloads/masses_<name>.json)
"""

from __future__ import annotations

import json
import math
import os
import sys

# one BLAS thread per worker process: the pool already fills the cores
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import scipy.sparse.linalg as spla

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.wilson import dirac_matrix  # noqa: E402

CONFIGS = {
    "256_beta6": dict(L=256, beta=6.0, sweeps=500, seeds=[2000, 2001, 2002, 2003],
                      ratios=[1e-2, 3e-3, 1e-3, 3e-4, 1e-4]),
    "512_beta6": dict(L=512, beta=6.0, sweeps=500, seeds=[5000], ratios=[1e-3], start=0.065),
    # the multi-RHS configuration as stated: field seed 3000, ratio 1e-4
    "512_beta6_s3000": dict(L=512, beta=6.0, sweeps=500, seeds=[3000], ratios=[1e-4], start=0.0),
    # the paper's 128^2 experiment: m_crit (= m*) of candidate fields, picked by topological charge
    "128_beta6": dict(L=128, beta=6.0, sweeps=1000, seeds=list(range(7000, 7008)), ratios=[]),
    "128_beta10": dict(L=128, beta=10.0, sweeps=1000, seeds=list(range(7100, 7108)), ratios=[]),
    # the serving workload's beta = 3 fields: m_crit (= m*) of 8 fields, 500 sweeps
    "128_beta3": dict(L=128, beta=3.0, sweeps=500, seeds=list(range(7200, 7208)), ratios=[]),
    # cold starts; the first seeds whose field keeps topological charge 0 after 1000 sweeps
    "128_beta6_cold": dict(L=128, beta=6.0, sweeps=1000, seeds=[7014], ratios=[], cold=True),
    "128_beta10_cold": dict(L=128, beta=10.0, sweeps=1000, seeds=[7110], ratios=[], cold=True),
}

_FIELDS = {}


def field(L, beta, sweeps, seed, cold=False):
    key = (L, beta, sweeps, seed, cold)
    if key not in _FIELDS:
        _FIELDS[key] = synth.metropolis_u1(L, L, beta, sweeps, seed, cold=cold)
    return _FIELDS[key]


def extremes(U, m):
    """(lambda_min, lambda_max) of A(m) = D(m)^H D(m)."""
    D = dirac_matrix(U, m).tocsc()
    A = (D.conj().T @ D).tocsr()
    n = D.shape[0]
    lu = spla.splu(D, permc_spec="MMD_AT_PLUS_A")
    op = spla.LinearOperator((n, n), dtype=np.complex128,
                             matvec=lambda v: lu.solve(lu.solve(np.asarray(v, np.complex128), trans="H")))
    lmin = spla.eigsh(A, k=1, sigma=0.0, which="LM", OPinv=op, tol=1e-6, return_eigenvectors=False)[0]
    v = np.random.default_rng(0).standard_normal(n) + 0j
    lmax = 0.0
    for _ in range(60):
        w = A @ v
        lmax = np.vdot(v, w).real / np.vdot(v, v).real
        v = w / np.linalg.norm(w)
    return float(lmin), float(lmax)


def find_mstar(args):
    L, beta, sweeps, seed = args[:4]
    cold = len(args) > 4 and args[4]
    th = field(L, beta, sweeps, seed, cold)
    U = synth.links_from_angles(th)
    cache = {}

    def lmin(m):
        if m not in cache:
            cache[m] = extremes(U, m)[0]
        return cache[m]

    grid = np.linspace(-0.3, 0.1, 9)
    vals = [lmin(float(m)) for m in grid]
    i = int(np.argmin(vals))
    a, b = float(grid[max(i - 1, 0)]), float(grid[min(i + 1, len(grid) - 1)])
    g = (math.sqrt(5) - 1) / 2
    c, d = b - g * (b - a), a + g * (b - a)
    for _ in range(12):
        if lmin(c) < lmin(d):
            b = d
        else:
            a = c
        c, d = b - g * (b - a), a + g * (b - a)
    mstar = 0.5 * (a + b)
    lo_min, lo_max = extremes(U, mstar)
    return dict(seed=seed, cold=bool(cold), m_star=mstar, lambda_min=lo_min, lambda_max=lo_max,
                plaquette=synth.mean_plaquette(th), topological_charge=round(synth.topological_charge(th)))


def bisect_target(args):
    L, beta, sweeps, seed, mstar, r0, target = args
    U = synth.links_from_angles(field(L, beta, sweeps, seed))
    if r0 >= target:
        return dict(target=target, mass=mstar, ratio=r0, reached=False)
    lo, hi = mstar, mstar + 0.05
    while True:
        mn, mx = extremes(U, hi)
        if mn / mx > target:
            break
        lo, hi = hi, hi + 0.05
    for _ in range(14):
        mid = 0.5 * (lo + hi)
        mn, mx = extremes(U, mid)
        if mn / mx > target:
            hi = mid
        else:
            lo = mid
    mn, mx = extremes(U, hi)
    return dict(target=target, mass=hi, ratio=mn / mx, reached=True)


def _lmin_job(args):
    L, beta, sweeps, seed, m = args
    U = synth.links_from_angles(field(L, beta, sweeps, seed))
    return extremes(U, m)


def parallel_field(cfg, seed, ex, width=8):
    """m* by nested 8-point grids, then each target ratio by 8-ary search."""
    L, beta, sweeps = cfg["L"], cfg["beta"], cfg["sweeps"]
    lo, hi = -0.3, 0.1
    best = None
    for _ in range(3):
        grid = list(np.linspace(lo, hi, width))
        vals = list(ex.map(_lmin_job, [(L, beta, sweeps, seed, float(m)) for m in grid]))
        i = int(np.argmin([v[0] for v in vals]))
        best = (grid[i], vals[i])
        step = grid[1] - grid[0]
        lo, hi = grid[i] - step, grid[i] + step
    mstar, (mn0, mx0) = best
    th = field(L, beta, sweeps, seed)
    out = dict(seed=seed, m_star=mstar, lambda_min=mn0, lambda_max=mx0, plaquette=synth.mean_plaquette(th),
               topological_charge=round(synth.topological_charge(th)), masses=[])
    for target in cfg["ratios"]:
        if mn0 / mx0 >= target:
            out["masses"].append(dict(target=target, mass=mstar, ratio=mn0 / mx0, reached=False))
            continue
        lo, hi = mstar, mstar + 0.2
        res = None
        for _ in range(3):
            grid = list(np.linspace(lo, hi, width + 2))[1:-1]
            vals = list(ex.map(_lmin_job, [(L, beta, sweeps, seed, float(m)) for m in grid]))
            above = [k for k, v in enumerate(vals) if v[0] / v[1] > target]
            k = above[0] if above else len(grid) - 1
            res = (grid[k], vals[k])
            lo, hi = (grid[k - 1] if k > 0 else lo), grid[k]
        m, (mn, mx) = res
        out["masses"].append(dict(target=target, mass=m, ratio=mn / mx, reached=mn / mx > target))
    return out


def secant_field(cfg, seed, ex):
    """Each target ratio by secant steps on sigma_min from cfg['start'] (3 evaluations)."""
    L, beta, sweeps = cfg["L"], cfg["beta"], cfg["sweeps"]
    th = field(L, beta, sweeps, seed)
    out = dict(seed=seed, m_star=None, plaquette=synth.mean_plaquette(th),
               topological_charge=round(synth.topological_charge(th)), masses=[])
    for target in cfg["ratios"]:
        m0 = cfg["start"]
        mn, mx = _lmin_job((L, beta, sweeps, seed, m0))
        pts = [(m0, mn, mx)]
        m1 = m0 + (math.sqrt(target * mx) - math.sqrt(mn))
        for _ in range(2):
            mn, mx = _lmin_job((L, beta, sweeps, seed, m1))
            pts.append((m1, mn, mx))
            (ma, na, xa), (mb, nb, xb) = pts[-2], pts[-1]
            sa, sb = math.sqrt(na) - math.sqrt(target * xa), math.sqrt(nb) - math.sqrt(target * xb)
            m1 = mb - sb * (mb - ma) / (sb - sa) if sb != sa else mb
        m, mn, mx = min(pts, key=lambda t: abs(math.log(t[1] / t[2] / target)))
        out["masses"].append(dict(target=target, mass=m, ratio=mn / mx, reached=abs(mn / mx / target - 1) < 0.1,
                                  evaluations=[dict(mass=a, lambda_min=b, lambda_max=c) for a, b, c in pts]))
    return out


def main():
    name = sys.argv[1] if len(sys.argv) > 1 else "256_beta6"
    cfg = CONFIGS[name]
    t0 = time.time()
    base = [(cfg["L"], cfg["beta"], cfg["sweeps"], s, cfg.get("cold", False)) for s in cfg["seeds"]]
    with ProcessPoolExecutor(max_workers=8) as ex:
        if cfg["L"] <= 256:
            stars = list(ex.map(find_mstar, base))
            jobs = [(cfg["L"], cfg["beta"], cfg["sweeps"], st["seed"], st["m_star"],
                     st["lambda_min"] / st["lambda_max"], r) for st in stars for r in cfg["ratios"]]
            res = list(ex.map(bisect_target, jobs))
            fields = []
            for k, st in enumerate(stars):
                fld = dict(st, L=cfg["L"], beta=cfg["beta"], sweeps=cfg["sweeps"])
                fld["masses"] = res[k * len(cfg["ratios"]):(k + 1) * len(cfg["ratios"])]
                fields.append(fld)
        elif "start" in cfg:
            fields = [dict(secant_field(cfg, s, ex), L=cfg["L"], beta=cfg["beta"], sweeps=cfg["sweeps"])
                      for s in cfg["seeds"]]
        else:
            fields = [dict(parallel_field(cfg, s, ex), L=cfg["L"], beta=cfg["beta"], sweeps=cfg["sweeps"])
                      for s in cfg["seeds"]]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"masses_{name}.json")
    with open(path, "w") as f:
        json.dump(dict(config=cfg, fields=fields, seconds=time.time() - t0), f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
