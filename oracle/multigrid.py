"""Adaptive multigrid for A = D^H D, written out step by step in FP64 (oracle).

Every function cites the passage of the paper it follows.  The operators are scipy
sparse matrices, so each level's operator is literally the matrix the paper
writes down: the fine A = D^H D (Introduction), the coarse A^(l+1) = P^H A^(l) P
(Eq. 2).  Nothing here is blocked, fused or reordered for speed.

Readings of the paper taken here (the paper is silent or garbled at these points):

* Eq. (3) is printed with "+ R A R^dagger"; only "- R A R^dagger" reproduces the
  five V-cycle steps listed above it, so the V-cycle follows the steps.
* Step 5 of the V-cycle is read as x <- x + R (b - A x) (the correction is added).
* The relaxation used inside the setup (Eq. 4) is the solve smoother itself:
  the frozen minimal-residual polynomial, so I - R A = prod_k (I - c_k A).
* An aggregate is all degrees of freedom of a bx x bt block of sites (4x4 in the
  paper), so a coarse site carries M = Nv degrees of freedom.  The alternative
  reading, aggregates split by chirality (the paper's aggregates are subsets of
  variables), is the `split` option: each block holds two aggregates, the
  variables d with d % 2 = 0 and those with d % 2 = 1.  On the fine lattice d is
  the spin index and gamma5 = sigma3, so the two halves are the chiralities +1
  and -1; a coarse site then carries 2 Nv degrees of freedom, ordered 2k + chi
  (candidate k, chirality chi), so the same parity rule holds on every level and
  the tentative P maps chirality to chirality.
* The setup's V-cycle on level l is the two-level cycle on the current P with the
  coarse system solved exactly (sparse direct solve here).
* Smoothed aggregation (Adaptive Multigrid section): the block-orthonormal
  tentative prolongator P_t is smoothed by one Richardson step, P = (I - w A) P_t.
  The paper picks w to minimise the coarse condition number without a formula;
  here w = s / lambda_max with s = 4/3 (the usual smoothed-aggregation weight) and
  lambda_max the Rayleigh quotient after 20 power iterations of A from the level's
  calibration start vector.  Smoothing is applied only where both block extents
  are >= 4 and both coarse extents >= 2 (then A_c stays a 9-point stencil), and
  the smoothed P is kept when the mass changes.

Vectors at level l are complex128, index ((t*lx_l + x)*dof_l + d).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class SetupError(RuntimeError):
    """Raised when an aggregate's candidate vectors are linearly dependent."""


def dot(a: np.ndarray, b: np.ndarray) -> complex:
    """<a, b> = sum conj(a_i) b_i."""
    return complex(np.vdot(a, b))


def norm(a: np.ndarray) -> float:
    return float(np.linalg.norm(a))


# ---------------------------------------------------------------------------
# Smoother (Results section: degree-nu polynomial from nu under-relaxed minimal
# residual steps, coefficients then frozen, so R = R^dagger).
# ---------------------------------------------------------------------------

def mr_coefficients(A, b: np.ndarray, nu: int, omega: float) -> List[float]:
    """Run nu minimal-residual steps on A x = b from x = 0, damping each by omega.

    The MR step length is alpha = <A r, r> / <A r, A r> (real for Hermitian A); the
    frozen coefficient is c_k = omega * alpha_k.
    """
    r = np.array(b, dtype=np.complex128, copy=True)
    coefs = []
    for _ in range(nu):
        q = A @ r
        alpha = dot(q, r).real / dot(q, q).real
        ck = omega * alpha
        coefs.append(ck)
        r = r - ck * q
    return coefs


def smoother_apply(A, coefs: Sequence[float], b: np.ndarray) -> np.ndarray:
    """R b for the frozen polynomial: the nu MR updates replayed with fixed c_k from x = 0.

    x_k = x_{k-1} + c_k r_{k-1},  r_k = r_{k-1} - c_k A r_{k-1}.
    """
    x = np.zeros_like(b)
    r = np.array(b, copy=True)
    for k, ck in enumerate(coefs):
        x = x + ck * r
        if k + 1 < len(coefs):
            r = r - ck * (A @ r)
    return x


def smoother_matrix(A_dense: np.ndarray, coefs: Sequence[float]) -> np.ndarray:
    """Dense R, built from the identity I - R A = prod_k (I - c_k A) (test helper)."""
    n = A_dense.shape[0]
    E = np.eye(n, dtype=np.complex128)
    for ck in coefs:
        E = (np.eye(n) - ck * A_dense) @ E
    # R A = I - E  =>  R = (I - E) A^{-1}
    return np.linalg.solve(A_dense.T, (np.eye(n) - E).T).T


# ---------------------------------------------------------------------------
# Aggregates S_j and the prolongator (Adaptive Multigrid section, Eqs. 5 and the
# M-vector form that follows it).
# ---------------------------------------------------------------------------

def aggregate_gather(shape, block, split: bool = False) -> np.ndarray:
    """G[J, i]: fine-vector index of the i-th variable of aggregate J.

    shape = (lx, lt, dof) of the fine side, block = (bx, bt).  Aggregate J =
    Jt*(lx/bx) + Jx holds the sites x in [Jx*bx, Jx*bx+bx), t in [Jt*bt, Jt*bt+bt)
    with all dof components; within it i = ((t % bt)*bx + (x % bx))*dof + d.
    With split, row 2J + chi keeps only the variables with d % 2 = chi (chirality
    split; the order within the row is unchanged).
    """
    lx, lt, dof = shape
    bx, bt = block
    if lx % bx or lt % bt:
        raise ValueError("lattice extent not divisible by the block extent")
    cx, ct = lx // bx, lt // bt
    Jt, Jx, ty, tx, d = np.meshgrid(
        np.arange(ct), np.arange(cx), np.arange(bt), np.arange(bx), np.arange(dof), indexing="ij"
    )
    fine = ((Jt * bt + ty) * lx + (Jx * bx + tx)) * dof + d
    G = fine.reshape(ct * cx, bt * bx * dof)
    if not split:
        return G
    if dof % 2:
        raise ValueError("a chirality split needs an even number of components per site")
    chi = np.arange(bt * bx * dof) % dof % 2
    return np.stack([G[:, chi == 0], G[:, chi == 1]], axis=1).reshape(2 * ct * cx, -1)


def block_gram_schmidt(vectors: np.ndarray, gather: np.ndarray, tol: float = 1e-12) -> np.ndarray:
    """Block-orthonormalise candidate vectors (Adaptive Multigrid section).

    vectors[k] is the k-th near-null candidate on the fine side.  For every
    aggregate J the restrictions v_k|_J are taken in order, made orthogonal to the
    earlier ones (modified Gram-Schmidt, two passes) and normalised to 1.
    Returns U[J, k, i], the columns of P on aggregate J.
    """
    nv = vectors.shape[0]
    nJ, nagg = gather.shape
    U = np.zeros((nJ, nv, nagg), dtype=np.complex128)
    # The same arithmetic is done for every aggregate, so the aggregates form the
    # leading array axis; the loops over k and j are the Gram-Schmidt order itself.
    for k in range(nv):
        w = vectors[k][gather]                                  # [J, i]
        ref = np.linalg.norm(w, axis=1)
        for _ in range(2):
            for j in range(k):
                proj = np.sum(np.conj(U[:, j, :]) * w, axis=1)  # <u_j, w> per aggregate
                w = w - proj[:, None] * U[:, j, :]
        nw = np.linalg.norm(w, axis=1)
        bad = ~(nw > tol * ref)
        if np.any(bad):
            raise SetupError(f"aggregate {int(np.argmax(bad))}: candidate {k} is linearly dependent")
        U[:, k, :] = w / nw[:, None]
    return U


def prolongator(U: np.ndarray, gather: np.ndarray, n_fine: int, split: bool = False) -> sp.csr_matrix:
    """P with P[gather[J, i], J*Nv + k] = U[J, k, i] (coarse index (K*Nv + k)).

    With split (gather rows 2K + chi), P[gather[2K + chi, i], K*2Nv + 2k + chi] =
    U[2K + chi, k, i]: coarse site K carries 2 Nv variables, candidate-major."""
    nJ, nv, nagg = U.shape
    rows = np.broadcast_to(gather[:, None, :], (nJ, nv, nagg)).ravel()
    R, k = np.arange(nJ)[:, None], np.arange(nv)[None, :]
    col = (R // 2) * 2 * nv + 2 * k + R % 2 if split else R * nv + k
    cols = np.broadcast_to(col[:, :, None], (nJ, nv, nagg)).ravel()
    return sp.coo_matrix((U.ravel(), (rows, cols)), shape=(n_fine, nJ * nv)).tocsr()


def galerkin(A, P) -> sp.csr_matrix:
    """Eq. (2): A^(l+1) = P^H A^(l) P."""
    return (P.conj().T @ (A @ P)).tocsr()


# ---------------------------------------------------------------------------
# Krylov solvers (Multigrid section: the V-cycle preconditions conjugate gradients).
# ---------------------------------------------------------------------------

@dataclass
class SolveInfo:
    converged: bool
    iterations: int
    fine_applies: int          # applications of A on the level solved (2 D/D^H each)
    relres: float              # true relative residual ||rhs - A x|| / ||rhs||
    history: List[float] = field(default_factory=list)


def cg(A, rhs: np.ndarray, tol: float, maxiter: int = 100000) -> (np.ndarray, SolveInfo):
    """Plain conjugate gradients on HPD A from x = 0, stopping on the true residual."""
    return pcg(A, rhs, None, tol, maxiter)


def pcg(A, rhs: np.ndarray, precond: Optional[Callable], tol: float, maxiter: int = 100000):
    """Preconditioned CG, z = M r with M = precond (identity when None).

    Stops when the recursive residual reaches tol and the recomputed true residual
    ||rhs - A x|| / ||rhs|| also does; otherwise the residual is replaced by the
    true one and the iteration continues.
    """
    bnorm = norm(rhs)
    x = np.zeros_like(rhs)
    if bnorm == 0.0:
        return x, SolveInfo(True, 0, 0, 0.0)
    applies = 0
    r = np.array(rhs, copy=True)
    z = precond(r) if precond else r.copy()
    p = z.copy()
    rz = dot(r, z).real
    hist = []
    for it in range(1, maxiter + 1):
        q = A @ p
        applies += 1
        pq = dot(p, q).real
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        rel = norm(r) / bnorm
        hist.append(rel)
        if rel <= tol:
            rt = rhs - A @ x
            applies += 1
            true_rel = norm(rt) / bnorm
            if true_rel <= tol:
                return x, SolveInfo(True, it, applies, true_rel, hist)
            r = rt
        z = precond(r) if precond else r.copy()
        rz_new = dot(r, z).real
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    true_rel = norm(rhs - A @ x) / bnorm
    return x, SolveInfo(False, maxiter, applies + 1, true_rel, hist)


# ---------------------------------------------------------------------------
# Hierarchy and V-cycle (Multigrid section, steps 1-5; Eq. 3 with the sign reading).
# ---------------------------------------------------------------------------

@dataclass
class Level:
    A: sp.csr_matrix
    shape: tuple                    # (lx, lt, dof)
    coefs: List[float] = field(default_factory=list)
    block: Optional[tuple] = None   # (bx, bt) towards the next level
    U: Optional[np.ndarray] = None  # [J, k, i] tentative (block-orthonormal) columns
    P: Optional[sp.csr_matrix] = None  # prolongator used by the V-cycle (smoothed or tentative)
    P_t: Optional[sp.csr_matrix] = None
    gather: Optional[np.ndarray] = None
    sa_weight: float = 0.0
    split: bool = False             # chirality-split aggregates towards the next level


@dataclass
class Hierarchy:
    levels: List[Level]
    coarsest: str = "cholesky"      # "cholesky" (exact) or "cg"
    coarsest_tol: float = 1e-12
    _chol: object = None

    def factor_coarsest(self):
        if self.coarsest == "cholesky":
            Ad = self.levels[-1].A.toarray()
            self._chol = sla.cho_factor(Ad, lower=True)
        return self

    def coarse_solve(self, b: np.ndarray) -> np.ndarray:
        """Exact solve on the coarsest level (Results: 'solved exactly')."""
        A = self.levels[-1].A
        if self.coarsest == "cholesky":
            if self._chol is None:
                self.factor_coarsest()
            return sla.cho_solve(self._chol, b)
        x, _ = cg(A, b, self.coarsest_tol)
        return x


def vcycle(h: Hierarchy, l: int, b: np.ndarray, counter: Optional[list] = None) -> np.ndarray:
    """One V-cycle V^(l) b, following steps 1-5 of the Multigrid section.

    1. x = R^H b                       (pre-relaxation; R^H = R here)
    2. r_c = P^H (b - A x)             (restrict the residual)
    3. e = V^(l+1) r_c                 (recurse; the coarsest level is exact)
    4. x = x + P e                     (coarse-grid correction)
    5. x = x + R (b - A x)             (post-relaxation)
    """
    lev = h.levels[l]
    if l == len(h.levels) - 1:
        return h.coarse_solve(b)
    A = lev.A
    x = smoother_apply(A, lev.coefs, b)
    rc = lev.P.conj().T @ (b - A @ x)
    e = vcycle(h, l + 1, rc, counter)
    x = x + lev.P @ e
    x = x + smoother_apply(A, lev.coefs, b - A @ x)
    if counter is not None and l == 0:
        counter[0] += 1
    return x


def mg_cg(h: Hierarchy, rhs: np.ndarray, tol: float, maxiter: int = 10000):
    """MG-CG: CG on the fine A with the V-cycle as preconditioner (Results section)."""
    return pcg(h.levels[0].A, rhs, lambda r: vcycle(h, 0, r), tol, maxiter)


# ---------------------------------------------------------------------------
# Building a hierarchy.
# ---------------------------------------------------------------------------

def power_lambda_max(A, start: np.ndarray, iters: int = 20) -> float:
    """Rayleigh quotient after `iters` power iterations of A from `start`."""
    v = np.array(start, dtype=np.complex128, copy=True)
    lam = 0.0
    for _ in range(iters):
        w = A @ v
        lam = dot(v, w).real / dot(v, v).real
        v = w / norm(w)
    return lam


def sa_applies(shape, block) -> bool:
    lx, lt, _ = shape
    bx, bt = block
    return bx >= 4 and bt >= 4 and lx // bx >= 2 and lt // bt >= 2


def coarsen(level: Level, vectors: np.ndarray, block, sa_weight: float = 0.0,
            split: bool = False) -> (Level, Level):
    """Given candidate vectors on `level`, form P (block Gram-Schmidt, then the
    smoothed-aggregation step when sa_weight > 0) and A_c = P^H A P (Eq. 2).
    With split the aggregates are the two chirality halves of each block."""
    gather = aggregate_gather(level.shape, block, split)
    U = block_gram_schmidt(vectors, gather)
    P_t = prolongator(U, gather, level.A.shape[0], split)
    P = P_t
    if sa_weight > 0:
        P = (P_t - sa_weight * (level.A @ P_t)).tocsr()
    level.block, level.U, level.P, level.P_t, level.gather = tuple(block), U, P, P_t, gather
    level.sa_weight, level.split = sa_weight, split
    lx, lt, _ = level.shape
    nc = vectors.shape[0] * (2 if split else 1)
    nxt = Level(A=galerkin(level.A, P), shape=(lx // block[0], lt // block[1], nc))
    return level, nxt


def level_sa_weight(level: Level, block, calib: np.ndarray, sa_scale: float) -> float:
    if sa_scale <= 0 or not sa_applies(level.shape, block):
        return 0.0
    return sa_scale / power_lambda_max(level.A, calib)


def hierarchy_from_vectors(A, shape, blocks, vectors_per_level, calib_per_level, nu, omega,
                           coarsest="cholesky", coarsest_tol=1e-12, sa_scale: float = 0.0,
                           split: bool = False) -> Hierarchy:
    """Hierarchy from given near-null vectors (no adaptive iteration).

    vectors_per_level[l] is [Nv_l, n_l]; calib_per_level[l] starts the MR
    calibration (and the lambda_max estimate) of level l.  split: chirality-split
    aggregates on every coarsening.
    """
    levels = [Level(A=A, shape=tuple(shape))]
    for l, block in enumerate(blocks):
        cur = levels[-1]
        cur.coefs = mr_coefficients(cur.A, calib_per_level[l], nu, omega)
        wsa = level_sa_weight(cur, block, calib_per_level[l], sa_scale)
        cur, nxt = coarsen(cur, np.asarray(vectors_per_level[l]), block, wsa, split)
        levels.append(nxt)
    return Hierarchy(levels, coarsest, coarsest_tol).factor_coarsest()


def _two_level_exact(level: Level, Ac) -> Callable:
    """Two-level V-cycle on `level` with the coarse system solved by a sparse direct solve."""
    # Symmetric fill-reducing ordering; Ac is Hermitian positive definite.
    lu = spla.splu(Ac.tocsc(), permc_spec="MMD_AT_PLUS_A", options=dict(SymmetricMode=True))
    A, P, c = level.A, level.P, level.coefs

    def V(b):
        x = smoother_apply(A, c, b)
        e = lu.solve(P.conj().T @ (b - A @ x))
        x = x + P @ e
        return x + smoother_apply(A, c, b - A @ x)

    return V


def two_level_factor(level: Level, Ac, e0: np.ndarray, iters: int) -> float:
    """Convergence factor of the current two-level cycle on a start error e0
    (Adaptive Multigrid section: vectors are added until the V-cycle reduces a random
    error sufficiently): iters passes of e <- (I - V A) e, then the geometric mean of
    the A-norm reduction, (||e_iters||_A / ||e_0||_A)^(1 / iters)."""
    V = _two_level_exact(level, Ac)
    A = level.A
    e = np.array(e0, dtype=np.complex128, copy=True)
    q = A @ e
    n0 = math.sqrt(dot(e, q).real)
    for _ in range(iters):
        e = e - V(q)
        q = A @ e
    return (math.sqrt(max(dot(e, q).real, 0.0)) / n0) ** (1.0 / iters)


def adaptive_setup(A, shape, blocks, nvs, randoms, nu: int, omega: float, setup_iters: int,
                   coarsest="cholesky", coarsest_tol=1e-12, log: Optional[list] = None,
                   sa_scale: float = 0.0, split: bool = False, nv_stop_rho: float = 0.0,
                   nv_stop_iters: int = 3) -> Hierarchy:
    """Adaptive setup (Adaptive Multigrid section), level by level.

    For each coarsening l with random starts randoms[l] ([1 + Nv, n_l]):
      * freeze the smoother from MR steps on randoms[l][0];
      * candidate 1: relax A e = 0 from randoms[l][1], e <- (I - R A) e, setup_iters
        times (Eq. 4 with the frozen polynomial), renormalising each pass;
      * candidates k = 2..Nv: from randoms[l][k], apply the current two-level V-cycle
        as an error propagator, e <- (I - V A) e, setup_iters times; the surviving
        error is restricted to the aggregates, orthonormalised against the earlier
        vectors and appended, and A_c is rebuilt;
      * the finished A_c is the next level's operator (the procedure recurses).
    With sa_scale > 0 every prolongator is the smoothed one (see the module notes);
    with split every coarsening uses chirality-split aggregates.

    nv_stop_rho > 0 stops adding vectors early ("repeated as necessary"): after each
    appended vector (the first included) the two-level cycle's convergence factor on
    the level's calibration start randoms[l][0] (two_level_factor, nv_stop_iters
    passes) is measured, and the level keeps the vectors it has once the factor is
    <= nv_stop_rho; Nv_l is then the most it takes.  The next level's vectors are
    shorter then: its random rows are still given at full length and their first
    n_{l+1} entries are used.  Each level's factors go to log[l]["factors"].
    """
    levels = [Level(A=A, shape=tuple(shape))]
    for l, block in enumerate(blocks):
        cur = levels[-1]
        n = cur.A.shape[0]
        R = np.asarray(randoms[l])[:, :n]
        cur.coefs = mr_coefficients(cur.A, R[0], nu, omega)
        wsa = level_sa_weight(cur, block, R[0], sa_scale)
        e = np.array(R[1], copy=True)
        for _ in range(setup_iters):
            e = e - smoother_apply(cur.A, cur.coefs, cur.A @ e)
            e = e / norm(e)
        vecs = [e]
        cur, nxt = coarsen(cur, np.array(vecs), block, wsa, split)
        factors = []
        # at most the variables of an aggregate (the next level may have fewer per site)
        nmax = min(nvs[l], block[0] * block[1] * cur.shape[2] // (2 if split else 1))
        for k in range(1, nmax + 1):
            if nv_stop_rho > 0:
                factors.append(two_level_factor(cur, nxt.A, R[0], nv_stop_iters))
                if factors[-1] <= nv_stop_rho:
                    break
            if k == nmax:
                break
            V = _two_level_exact(cur, nxt.A)
            e = np.array(R[1 + k], copy=True)
            for _ in range(setup_iters):
                e = e - V(cur.A @ e)
                e = e / norm(e)
            vecs.append(e)
            cur, nxt = coarsen(cur, np.array(vecs), block, wsa, split)
        if log is not None:
            log.append({"level": l, "coefs": list(cur.coefs), "factors": factors, "nv": len(vecs)})
        levels.append(nxt)
    return Hierarchy(levels, coarsest, coarsest_tol).factor_coarsest()


def set_mass(h: Hierarchy, A_fine, calib_per_level, nu: int, omega: float) -> Hierarchy:
    """Reuse the prolongators at a new mass (Results: setup at the lightest mass,
    vectors reused for heavier masses): rebuild every A^(l) by Eq. (2) and
    recalibrate the smoothers."""
    levels = []
    A = A_fine
    for l, lev in enumerate(h.levels):
        new = Level(A=A, shape=lev.shape, block=lev.block, U=lev.U, P=lev.P, P_t=lev.P_t, gather=lev.gather,
                    sa_weight=lev.sa_weight, split=lev.split)
        if lev.P is not None:
            new.coefs = mr_coefficients(A, calib_per_level[l], nu, omega)
            A = galerkin(A, lev.P)
        levels.append(new)
    return Hierarchy(levels, h.coarsest, h.coarsest_tol).factor_coarsest()
