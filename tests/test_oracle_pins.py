"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed form,
a value the paper prints, an invariant, a special case that reduces to a library
routine, or a dense brute-force computation on a tiny lattice.  They run on CPU.
"""

import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import multigrid as mg
from oracle.wilson import SIGMA1, SIGMA2, SIGMA3, dirac_matrix, fermion_links, gamma5_matrix, normal_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


def hot_field(lx, lt, seed, sweeps=0, beta=3.0):
    return synth.links_from_angles(synth.metropolis_u1(lx, lt, beta, sweeps, seed))


# ---------------------------------------------------------------------------
# P1: free field (U = 1) closed forms
# ---------------------------------------------------------------------------

def test_free_field_plane_wave_action():
    """D e^{ipx} u = [(2 + m - sum cos p) + i sum sigma_mu sin p_mu] e^{ipx} u.

    p_x = 2 pi n / lx (periodic), p_t = (2n+1) pi / lt (antiperiodic).  The sign of
    the i sigma sin p term fixes the sign convention of the hopping projectors."""
    lx, lt, m = 6, 4, 0.37
    U = np.ones((2, lt, lx), dtype=np.complex128)
    D = dirac_matrix(U, m, antiperiodic_t=True)
    rng = np.random.default_rng(5)
    t, x = np.meshgrid(np.arange(lt), np.arange(lx), indexing="ij")
    for nx in range(lx):
        for nt in range(lt):
            px, pt = 2 * math.pi * nx / lx, (2 * nt + 1) * math.pi / lt
            u = rng.standard_normal(2) + 1j * rng.standard_normal(2)
            phase = np.exp(1j * (px * x + pt * t)).ravel()
            psi = np.kron(phase, u)
            Dp = (2 + m - math.cos(px) - math.cos(pt)) * np.eye(2) + 1j * (SIGMA1 * math.sin(px) + SIGMA2 * math.sin(pt))
            np.testing.assert_allclose(D @ psi, np.kron(phase, Dp @ u), atol=1e-13)


def test_free_field_spectrum_of_A():
    """spec(A) = {(m + sum(1 - cos p))^2 + sum sin^2 p}, each twice (8x8, antiperiodic t)."""
    lx = lt = 8
    m = 0.05
    U = np.ones((2, lt, lx), dtype=np.complex128)
    A = normal_matrix(U, m).toarray()
    ev = np.sort(np.linalg.eigvalsh(A))
    ref = []
    for nx in range(lx):
        for nt in range(lt):
            px, pt = 2 * math.pi * nx / lx, (2 * nt + 1) * math.pi / lt
            lam = (m + (1 - math.cos(px)) + (1 - math.cos(pt))) ** 2 + math.sin(px) ** 2 + math.sin(pt) ** 2
            ref += [lam, lam]
    np.testing.assert_allclose(ev, np.sort(ref), atol=1e-13)


def test_free_field_periodic_zero_mode_mass():
    """With periodic BC the constant spinor is an eigenvector of D with eigenvalue m
    (reading (d + m) of the diagonal: the free operator at zero momentum is m)."""
    lx, lt, m = 4, 6, 0.123
    U = np.ones((2, lt, lx), dtype=np.complex128)
    D = dirac_matrix(U, m, antiperiodic_t=False)
    for spin in range(2):
        v = np.zeros(2 * lx * lt, dtype=np.complex128)
        v[spin::2] = 1.0
        np.testing.assert_allclose(D @ v, m * v, atol=1e-14)


# ---------------------------------------------------------------------------
# P2, P3: gamma5-hermiticity and gauge covariance on random fields
# ---------------------------------------------------------------------------

def test_gamma5_hermiticity():
    lx, lt = 6, 8
    U = hot_field(lx, lt, seed=11)
    D = dirac_matrix(U, 0.2)
    G5 = gamma5_matrix(lx * lt)
    diff = (D.conj().T - G5 @ D @ G5).toarray()
    assert np.max(np.abs(diff)) <= 1e-14


def test_gauge_covariance():
    """U'_x^mu = g_x U_x^mu g*_{x+mu}  =>  D[U'] = G D[U] G^H."""
    lx, lt = 6, 4
    theta = synth.metropolis_u1(lx, lt, 2.0, 0, 12)
    U = synth.links_from_angles(theta)
    rng = np.random.default_rng(3)
    g = np.exp(1j * rng.uniform(-math.pi, math.pi, size=(lt, lx)))
    Up = np.empty_like(U)
    Up[0] = g * U[0] * np.conj(np.roll(g, -1, axis=1))
    Up[1] = g * U[1] * np.conj(np.roll(g, -1, axis=0))
    G = np.kron(np.diag(g.ravel()), np.eye(2))
    D = dirac_matrix(U, 0.3).toarray()
    Dp = dirac_matrix(Up, 0.3).toarray()
    np.testing.assert_allclose(Dp, G @ D @ G.conj().T, atol=1e-14)


def test_antiperiodic_sign_only_on_last_slice():
    lx, lt = 4, 6
    U = hot_field(lx, lt, seed=4)
    Ut = fermion_links(U, True)
    np.testing.assert_array_equal(Ut[0], U[0])
    np.testing.assert_array_equal(Ut[1, :-1], U[1, :-1])
    np.testing.assert_array_equal(Ut[1, -1], -U[1, -1])


# ---------------------------------------------------------------------------
# P4: A = D^H D is a 9-point box stencil and HPD
# ---------------------------------------------------------------------------

def test_normal_operator_box_support_and_hpd():
    lx, lt = 8, 8
    U = hot_field(lx, lt, seed=21)
    A = normal_matrix(U, 0.1).toarray()
    n = A.shape[0]
    assert np.allclose(A, A.conj().T, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0
    for s in range(lx * lt):
        t0, x0 = divmod(s, lx)
        for col in range(2 * s, 2 * s + 2):
            for row in np.nonzero(np.abs(A[:, col]) > 1e-14)[0]:
                t1, x1 = divmod(row // 2, lx)
                dx = min((x1 - x0) % lx, (x0 - x1) % lx)
                dt = min((t1 - t0) % lt, (t0 - t1) % lt)
                assert dx <= 1 and dt <= 1, "A couples sites outside the 3x3 box"
        # the straight distance-2 couplings cancel: (1 + gamma)(1 - gamma) = 0
        for dx, dt in ((2, 0), (0, 2)):
            t1, x1 = (t0 + dt) % lt, (x0 + dx) % lx
            blk = A[2 * (t1 * lx + x1): 2 * (t1 * lx + x1) + 2, 2 * s: 2 * s + 2]
            assert np.max(np.abs(blk)) <= 1e-14


# ---------------------------------------------------------------------------
# Aggregates, P, Galerkin
# ---------------------------------------------------------------------------

def _tiny_hierarchy(lx=8, lt=8, block=(2, 2), nv=4, seed=7, mass=0.2, sweeps=20, beta=3.0, levels=2,
                    coarsest="cholesky"):
    U = hot_field(lx, lt, seed, sweeps=sweeps, beta=beta)
    A = normal_matrix(U, mass)
    blocks = [tuple(block)] * (levels - 1)
    nvs = [nv] * (levels - 1)
    R = synth.setup_randoms(lx, lt, blocks, nvs, seed)
    h = mg.adaptive_setup(A, (lx, lt, 2), blocks, nvs, R, nu=2, omega=0.8, setup_iters=3, coarsest=coarsest)
    return U, A, h


def test_aggregate_gather_partitions_lattice():
    G = mg.aggregate_gather((8, 4, 3), (2, 2))
    assert G.shape == (4 * 2, 2 * 2 * 3)
    assert np.array_equal(np.sort(G.ravel()), np.arange(8 * 4 * 3))
    # aggregate 0 is the block x in {0,1}, t in {0,1}, all dof
    assert set(G[0].tolist()) == {((t * 8 + x) * 3 + d) for t in (0, 1) for x in (0, 1) for d in range(3)}


def test_prolongator_is_block_orthonormal():
    _, A, h = _tiny_hierarchy()
    P = h.levels[0].P.toarray()
    np.testing.assert_allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-14)
    Pi = P @ P.conj().T
    np.testing.assert_allclose(Pi @ Pi, Pi, atol=1e-14)
    # column (J, k) is supported on aggregate J only
    G = h.levels[0].gather
    for J in range(G.shape[0]):
        mask = np.ones(P.shape[0], dtype=bool)
        mask[G[J]] = False
        assert np.max(np.abs(P[mask][:, J * 4:(J + 1) * 4])) == 0.0


def test_gram_schmidt_spans_candidates():
    """Each aggregate's span{u_1..u_k} equals span{v_1|_J..v_k|_J} (k = 1..Nv)."""
    rng = np.random.default_rng(2)
    G = mg.aggregate_gather((4, 4, 2), (2, 2))
    V = rng.standard_normal((3, 32)) + 1j * rng.standard_normal((3, 32))
    U = mg.block_gram_schmidt(V, G)
    for J in range(G.shape[0]):
        for k in range(1, 4):
            B = V[:k, G[J]].T                      # candidates restricted to J
            Q = U[J, :k].T                          # orthonormal basis
            np.testing.assert_allclose(Q @ (Q.conj().T @ B), B, atol=1e-13)


def test_gram_schmidt_degenerate_raises():
    G = mg.aggregate_gather((4, 4, 2), (2, 2))
    v = np.ones(32, dtype=np.complex128)
    with pytest.raises(mg.SetupError):
        mg.block_gram_schmidt(np.stack([v, 2 * v]), G)


def test_galerkin_links_nine_point_and_hermitian():
    """A_c couples only the 3x3 box of coarse sites, and L_{K,D} = L_{K+D,-D}^H."""
    lx = lt = 12
    _, A, h = _tiny_hierarchy(lx=lx, lt=lt, block=(4, 4), nv=4)
    Ac = h.levels[1].A.toarray()
    assert np.allclose(Ac, Ac.conj().T, atol=1e-14)
    cx = ct = 3
    nc = 4
    for K in range(cx * ct):
        for Kn in range(cx * ct):
            blk = Ac[K * nc:(K + 1) * nc, Kn * nc:(Kn + 1) * nc]
            kt, kx = divmod(K, cx)
            nt, nx = divmod(Kn, cx)
            near = min((nx - kx) % cx, (kx - nx) % cx) <= 1 and min((nt - kt) % ct, (kt - nt) % ct) <= 1
            if not near:
                assert np.max(np.abs(blk)) == 0.0
    # the coarsest Cholesky exists (HPD)
    sla.cho_factor(Ac)


def test_galerkin_free_field_constant_vectors():
    """Free field, periodic BC, candidates = the two constant spinors: A 1 = m^2 1, so
    the coarse operator maps the coarse constant to m^2 times itself."""
    lx, lt, m = 8, 8, 0.3
    U = np.ones((2, lt, lx), dtype=np.complex128)
    A = normal_matrix(U, m, antiperiodic_t=False)
    V = np.zeros((2, 2 * lx * lt), dtype=np.complex128)
    V[0, 0::2] = 1.0
    V[1, 1::2] = 1.0
    lev = mg.Level(A=A, shape=(lx, lt, 2))
    lev, nxt = mg.coarsen(lev, V, (4, 4))
    e = np.ones(nxt.A.shape[0], dtype=np.complex128)
    np.testing.assert_allclose(nxt.A @ e, m * m * e, atol=1e-13)


def test_coarse_grid_correction_is_A_orthogonal_projector():
    """E = I - P A_c^{-1} P^H A is an A-orthogonal projector exactly when A_c = P^H A P
    (the variational property behind Eq. 2)."""
    _, A, h = _tiny_hierarchy(lx=8, lt=8, block=(2, 2), nv=3)
    Ad = A.toarray()
    P = h.levels[0].P.toarray()
    Ac = h.levels[1].A.toarray()
    E = np.eye(Ad.shape[0]) - P @ np.linalg.solve(Ac, P.conj().T @ Ad)
    np.testing.assert_allclose(E @ E, E, atol=1e-11)
    AE = Ad @ E
    np.testing.assert_allclose(AE, AE.conj().T, atol=1e-11)
    # and it removes the coarse space exactly
    np.testing.assert_allclose(E @ P, 0, atol=1e-11)


def test_mass_affinity_of_coarse_operator():
    """A(m) = D0^H D0 + m (D0 + D0^H) + m^2 and P^H P = I give
    A_c(m) = C2 + m C1 + m^2 I with C2, C1 independent of m."""
    lx = lt = 8
    U = hot_field(lx, lt, seed=9, sweeps=10)
    _, _, h = _tiny_hierarchy(lx=lx, lt=lt, seed=9, sweeps=10)
    P = h.levels[0].P
    D0 = dirac_matrix(U, 0.0)
    C2 = (P.conj().T @ (D0.conj().T @ D0) @ P).toarray()
    C1 = (P.conj().T @ (D0 + D0.conj().T) @ P).toarray()
    for m in (0.0, 0.05, -0.2, 0.7):
        Ac = mg.galerkin(normal_matrix(U, m), P).toarray()
        np.testing.assert_allclose(Ac, C2 + m * C1 + m * m * np.eye(Ac.shape[0]), atol=1e-13)


def test_set_mass_rebuilds_every_level_from_the_new_mass():
    """set_mass on a 3-level hierarchy (smoothed P on the first coarsening): with
    D(m) = D0 + m and P, P2 kept, level 1 is C2 + m C1 + m^2 C0 (C0 = P^H P, which
    is not I for a smoothed P) and level 2 is P2^H (C2 + m C1 + m^2 C0) P2.  The C
    are formed here from D0 at mass 0, never from set_mass's own operators, so a
    level rebuilt from the old mass, or level 2 from the old level 1, fails."""
    lx = lt = 16
    m0, m1 = 0.2, -0.05
    U = hot_field(lx, lt, seed=71, sweeps=10)
    blocks, nvs = [(4, 4), (2, 2)], [3, 3]
    R = synth.setup_randoms(lx, lt, blocks, nvs, 12)
    h = mg.adaptive_setup(normal_matrix(U, m0), (lx, lt, 2), blocks, nvs, R, nu=2, omega=0.8, setup_iters=2,
                          sa_scale=4 / 3)
    assert h.levels[0].sa_weight > 0 and h.levels[1].sa_weight == 0
    calib = [r[0] for r in R]
    h1 = mg.set_mass(h, normal_matrix(U, m1), calib, nu=2, omega=0.8)
    P, P2 = h.levels[0].P.toarray(), h.levels[1].P.toarray()
    D0 = dirac_matrix(U, 0.0).toarray()
    C0 = P.conj().T @ P
    C1 = P.conj().T @ (D0 + D0.conj().T) @ P
    C2 = P.conj().T @ (D0.conj().T @ D0) @ P
    assert np.max(np.abs(C0 - np.eye(C0.shape[0]))) > 1e-3  # smoothed: P^H P differs from I
    A1 = C2 + m1 * C1 + m1 * m1 * C0
    scale = np.max(np.abs(A1))
    assert np.max(np.abs(h1.levels[1].A.toarray() - A1)) <= 1e-13 * scale
    A2 = P2.conj().T @ A1 @ P2
    assert np.max(np.abs(h1.levels[2].A.toarray() - A2)) <= 1e-13 * scale
    # the old operators differ by far more than that
    assert np.max(np.abs(h.levels[1].A.toarray() - A1)) > 1e-3 * scale
    # prolongators are kept as they are (Results section: vectors reused)
    assert (h1.levels[0].P != h.levels[0].P).nnz == 0 and (h1.levels[1].P != h.levels[1].P).nnz == 0


def test_set_mass_recalibrates_from_closed_form_eigenvectors():
    """Free field, periodic BC, constant candidates, plain aggregation.  set_mass to m1
    with the fine calibration start a plane wave (an eigenvector of A(m1) with
    eigenvalue lam) and the coarse start the coarse constant (A_c(m1) 1 = m1^2 1):
    every frozen coefficient is then omega / lam on level 0 and omega / m1^2 on
    level 1 (MR on an eigenvector), and A_c(m1) 1 = m1^2 1."""
    lx = lt = 16
    m0, m1, omega, nu = 0.4, 0.25, 0.8, 3
    U = np.ones((2, lt, lx), dtype=np.complex128)
    blocks = [(4, 4), (2, 2)]
    V0 = np.zeros((2, 2 * lx * lt), dtype=np.complex128)
    V0[0, 0::2] = 1.0
    V0[1, 1::2] = 1.0
    n1 = (lx // 4) * (lt // 4) * 2
    V1 = np.zeros((2, n1), dtype=np.complex128)
    V1[0, 0::2] = 1.0
    V1[1, 1::2] = 1.0
    t, x = np.meshgrid(np.arange(lt), np.arange(lx), indexing="ij")
    px, pt = 2 * math.pi * 2 / lx, 2 * math.pi * 3 / lt
    Dp = (2 + m1 - math.cos(px) - math.cos(pt)) * np.eye(2) + 1j * (SIGMA1 * math.sin(px) + SIGMA2 * math.sin(pt))
    w, vecs = np.linalg.eigh(Dp.conj().T @ Dp)
    wave = np.kron(np.exp(1j * (px * x + pt * t)).ravel(), vecs[:, 1])
    ones1 = np.ones(n1, dtype=np.complex128)
    rnd = [synth.gaussian(2 * lx * lt, 1), synth.gaussian(n1, 2)]
    h = mg.hierarchy_from_vectors(normal_matrix(U, m0, antiperiodic_t=False), (lx, lt, 2), blocks, [V0, V1], rnd,
                                  nu, omega)
    h1 = mg.set_mass(h, normal_matrix(U, m1, antiperiodic_t=False), [wave, ones1], nu, omega)
    np.testing.assert_allclose(h1.levels[0].coefs, [omega / w[1]] * nu, rtol=1e-12)
    np.testing.assert_allclose(h1.levels[1].coefs, [omega / m1 ** 2] * nu, rtol=1e-12)
    np.testing.assert_allclose(h1.levels[1].A @ ones1, m1 ** 2 * ones1, atol=1e-13)
    n2 = (lx // 8) * (lt // 8) * 2
    np.testing.assert_allclose(h1.levels[2].A @ np.ones(n2), m1 ** 2 * np.ones(n2), atol=1e-13)


# ---------------------------------------------------------------------------
# Smoother (P11) and V-cycle (P9, P10)
# ---------------------------------------------------------------------------

def test_mr_on_plane_wave_closed_form():
    """For an eigenvector b of A with eigenvalue lam, every MR step length is 1/lam,
    so c_k = omega/lam and the residual shrinks by exactly 1 - omega per step."""
    lx, lt, m = 8, 8, 0.1
    U = np.ones((2, lt, lx), dtype=np.complex128)
    A = normal_matrix(U, m)
    t, x = np.meshgrid(np.arange(lt), np.arange(lx), indexing="ij")
    px, pt = 2 * math.pi * 3 / lx, 5 * math.pi / lt
    Dp = (2 + m - math.cos(px) - math.cos(pt)) * np.eye(2) + 1j * (SIGMA1 * math.sin(px) + SIGMA2 * math.sin(pt))
    w, vecs = np.linalg.eigh(Dp.conj().T @ Dp)
    b = np.kron(np.exp(1j * (px * x + pt * t)).ravel(), vecs[:, 0])
    lam = w[0]
    c = mg.mr_coefficients(A, b, 4, 0.8)
    np.testing.assert_allclose(c, [0.8 / lam] * 4, rtol=1e-13)
    x1 = mg.smoother_apply(A, c[:1], b)
    np.testing.assert_allclose(b - A @ x1, 0.2 * b, atol=1e-13)


def test_smoother_is_polynomial_identity():
    """R b from the replayed MR updates satisfies I - R A = prod_k (I - c_k A)."""
    _, A, h = _tiny_hierarchy(lx=6, lt=6)
    Ad = A.toarray()
    c = h.levels[0].coefs
    n = Ad.shape[0]
    Rm = np.column_stack([mg.smoother_apply(A, c, e) for e in np.eye(n, dtype=np.complex128)])
    E = np.eye(n, dtype=np.complex128)
    for ck in c:
        E = (np.eye(n) - ck * Ad) @ E
    np.testing.assert_allclose(np.eye(n) - Rm @ Ad, E, atol=1e-12)
    np.testing.assert_allclose(Rm, Rm.conj().T, atol=1e-13)


def _dense_of(f, n):
    return np.column_stack([f(e) for e in np.eye(n, dtype=np.complex128)])


@pytest.mark.parametrize("levels", [2, 3])
def test_vcycle_error_propagator(levels):
    """I - V A = (I - R A)(I - P V_c P^H A)(I - R A) with V_c the next level's cycle
    (exact inverse on the coarsest level).  This is Eq. 3 with -R A R^H; the printed
    +R A R^H would not give this product.  V is Hermitian positive definite."""
    lx = lt = 8
    _, A, h = _tiny_hierarchy(lx=lx, lt=lt, block=(2, 2), nv=3, levels=levels)
    Ad = A.toarray()
    n = Ad.shape[0]
    V = _dense_of(lambda e: mg.vcycle(h, 0, e), n)
    lev = h.levels[0]
    Rm = _dense_of(lambda e: mg.smoother_apply(A, lev.coefs, e), n)
    P = lev.P.toarray()
    nc = P.shape[1]
    Vc = _dense_of(lambda e: mg.vcycle(h, 1, e), nc)
    I = np.eye(n)
    lhs = I - V @ Ad
    rhs = (I - Rm @ Ad) @ (I - P @ Vc @ P.conj().T @ Ad) @ (I - Rm @ Ad)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)
    np.testing.assert_allclose(V, V.conj().T, atol=1e-12)
    assert np.linalg.eigvalsh(0.5 * (V + V.conj().T)).min() > 0
    # the printed sign (+R A R^H) gives a different operator
    Vplus = Rm + Rm.conj().T + Rm @ Ad @ Rm.conj().T + (I - Rm @ Ad) @ P @ Vc @ P.conj().T @ (I - Ad @ Rm.conj().T)
    assert np.max(np.abs(Vplus - V)) > 1e-3


def test_full_coarse_space_vcycle_is_exact():
    """1x1 aggregates with Nv = 2 make P unitary, so one V-cycle inverts A."""
    lx = lt = 4
    U = hot_field(lx, lt, seed=31, sweeps=5)
    A = normal_matrix(U, 0.3)
    R = synth.setup_randoms(lx, lt, [(1, 1)], [2], 31)
    h = mg.adaptive_setup(A, (lx, lt, 2), [(1, 1)], [2], R, nu=2, omega=0.8, setup_iters=2)
    P = h.levels[0].P.toarray()
    np.testing.assert_allclose(P.conj().T @ P, np.eye(P.shape[0]), atol=1e-14)
    b = synth.gaussian(A.shape[0], 1)
    x = mg.vcycle(h, 0, b)
    np.testing.assert_allclose(A @ x, b, atol=1e-12)


def test_single_level_mgcg_is_cg():
    lx = lt = 8
    U = hot_field(lx, lt, seed=41, sweeps=5)
    A = normal_matrix(U, 0.2)
    h = mg.Hierarchy([mg.Level(A=A, shape=(lx, lt, 2))], coarsest="cg")
    b = synth.gaussian(A.shape[0], 2)
    x1, i1 = mg.cg(A, b, 1e-10)
    # a one-level "V-cycle" is the coarsest solve itself: preconditioner = A^{-1}
    h2 = mg.Hierarchy([mg.Level(A=A, shape=(lx, lt, 2))], coarsest="cholesky").factor_coarsest()
    x2, i2 = mg.mg_cg(h2, b, 1e-10)
    assert i2.iterations == 1
    np.testing.assert_allclose(x1, x2, atol=1e-9 * np.linalg.norm(x2))


# ---------------------------------------------------------------------------
# P5: solves against dense LAPACK
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lx,lt,block,nv,levels", [(4, 4, (2, 2), 4, 2), (8, 8, (2, 2), 4, 3),
                                                    (8, 6, (2, 2), 3, 2), (6, 6, (3, 3), 4, 2)])
def test_solves_match_dense_lu(lx, lt, block, nv, levels):
    U = hot_field(lx, lt, seed=lx * 10 + lt, sweeps=10)
    A = normal_matrix(U, 0.15)
    blocks = [block] * (levels - 1)
    nvs = [nv] * (levels - 1)
    R = synth.setup_randoms(lx, lt, blocks, nvs, 3)
    h = mg.adaptive_setup(A, (lx, lt, 2), blocks, nvs, R, nu=2, omega=0.8, setup_iters=3)
    b = synth.gaussian(A.shape[0], 9)
    ref = np.linalg.solve(A.toarray(), b)
    cond = np.linalg.cond(A.toarray())
    for x, info in (mg.mg_cg(h, b, 1e-10), mg.cg(A, b, 1e-10)):
        assert info.converged and info.relres <= 1e-10
        assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= cond * 1e-10


# ---------------------------------------------------------------------------
# Adaptive setup behaviour
# ---------------------------------------------------------------------------

def test_adaptive_vectors_are_near_null_and_help():
    """The adaptive vectors have small Rayleigh quotients compared with the spectrum
    of A, and MG-CG needs far fewer iterations than CG (Results section)."""
    lx = lt = 32
    U = hot_field(lx, lt, seed=1000, sweeps=200, beta=3.0)
    A = normal_matrix(U, 0.1)
    R = synth.setup_randoms(lx, lt, [(4, 4)], [8], 1)
    h = mg.adaptive_setup(A, (lx, lt, 2), [(4, 4)], [8], R, nu=4, omega=0.8, setup_iters=5, coarsest="cg")
    b = synth.gaussian(A.shape[0], 0)
    rhs = dirac_matrix(U, 0.1).conj().T @ b
    _, info_mg = mg.mg_cg(h, rhs, 1e-10)
    _, info_cg = mg.cg(A, rhs, 1e-10)
    assert info_mg.converged and info_cg.converged
    assert info_mg.iterations * 5 < info_cg.iterations
    # random vectors instead of adaptive ones give a much weaker preconditioner
    hr = mg.hierarchy_from_vectors(A, (lx, lt, 2), [(4, 4)], [R[0][1:]], [R[0][0]], 4, 0.8)
    _, info_r = mg.mg_cg(hr, rhs, 1e-10)
    assert info_mg.iterations < info_r.iterations


# ---------------------------------------------------------------------------
# P12: gauge generator
# ---------------------------------------------------------------------------

def test_string_length_matches_paper():
    """1/sqrt(-ln(I1/I0)) (area law W ~ exp(-A/l^2) with W = (I1/I0)^A) reproduces the
    correlation lengths the paper prints; this fixes the sign of the action in the
    Boltzmann weight, since the opposite sign has no area law of that size."""
    g = json.load(open(GOLDEN))["string_length"]
    for beta in ("6", "10"):
        assert abs(synth.gauge.string_length(float(beta)) - g[beta]) < 0.006


@pytest.mark.parametrize("beta", [3.0, 6.0, 10.0])
def test_metropolis_plaquette_matches_bessel_ratio(beta):
    """<cos theta_p> = I1(beta)/I0(beta) for 2D U(1) (independent plaquettes)."""
    from scipy.special import i0, i1

    means = []
    for seed in range(6):
        th = synth.metropolis_u1(16, 16, beta, 150, 500 + seed)
        means.append(synth.mean_plaquette(th))
    means = np.array(means)
    err = means.std(ddof=1) / math.sqrt(len(means))
    target = i1(beta) / i0(beta)
    assert abs(means.mean() - target) < 3.5 * err + 2e-3


def test_topological_charge_is_integer_and_gauge_invariant():
    th = synth.metropolis_u1(16, 16, 3.0, 50, 77)
    q = synth.topological_charge(th)
    assert abs(q - round(q)) < 1e-9
    rng = np.random.default_rng(1)
    a = rng.uniform(-math.pi, math.pi, size=(16, 16))
    th2 = th.copy()
    th2[0] = th[0] + a - np.roll(a, -1, axis=1)
    th2[1] = th[1] + a - np.roll(a, -1, axis=0)
    assert abs(synth.topological_charge(th2) - q) < 1e-9
    np.testing.assert_allclose(synth.mean_plaquette(th2), synth.mean_plaquette(th), atol=1e-12)


# ---------------------------------------------------------------------------
# Smoothed aggregation (Adaptive Multigrid section)
# ---------------------------------------------------------------------------

def test_sa_free_field_closed_form():
    """Free field, periodic BC, constant candidates: A 1 = m^2 1, so the smoothed
    prolongator maps the coarse constant to (1 - w m^2) times the fine constant
    and the coarse operator has eigenvalue m^2 (1 - w m^2)^2 on it."""
    lx, lt, m, w = 8, 8, 0.3, 0.07
    U = np.ones((2, lt, lx), dtype=np.complex128)
    A = normal_matrix(U, m, antiperiodic_t=False)
    V = np.zeros((2, 2 * lx * lt), dtype=np.complex128)
    V[0, 0::2] = 1.0
    V[1, 1::2] = 1.0
    lev = mg.Level(A=A, shape=(lx, lt, 2))
    lev, nxt = mg.coarsen(lev, V, (4, 4), sa_weight=w)
    e = np.ones(nxt.A.shape[0], dtype=np.complex128)
    np.testing.assert_allclose(nxt.A @ e, m * m * (1 - w * m * m) ** 2 * e, atol=1e-13)
    np.testing.assert_allclose(lev.P @ e, (1 - w * m * m) * (lev.P_t @ e), atol=1e-14)


def test_sa_columns_live_on_block_plus_ring_and_stencil_stays_nine_point():
    lx = lt = 16
    U = hot_field(lx, lt, seed=51, sweeps=10)
    A = normal_matrix(U, 0.1)
    R = synth.setup_randoms(lx, lt, [(4, 4)], [3], 5)
    h = mg.adaptive_setup(A, (lx, lt, 2), [(4, 4)], [3], R, nu=2, omega=0.8, setup_iters=2, sa_scale=4 / 3)
    lev = h.levels[0]
    assert lev.sa_weight > 0
    P = lev.P.toarray()
    for J in range(16):
        jt, jx = divmod(J, 4)
        rows = np.nonzero(np.abs(P[:, J * 3:(J + 1) * 3]).sum(axis=1))[0]
        for row in rows:
            t, x = divmod(row // 2, lx)
            dx = (x - jx * 4 + 1) % lx
            dt = (t - jt * 4 + 1) % lt
            assert dx <= 5 and dt <= 5, "smoothed column leaves the block plus one ring"
    Ac = h.levels[1].A.toarray()
    assert np.allclose(Ac, Ac.conj().T, atol=1e-14)
    for K in range(16):
        kt, kx = divmod(K, 4)
        for Kn in range(16):
            nt, nx = divmod(Kn, 4)
            near = min((nx - kx) % 4, (kx - nx) % 4) <= 1 and min((nt - kt) % 4, (kt - nt) % 4) <= 1
            if not near:
                assert np.max(np.abs(Ac[K * 3:(K + 1) * 3, Kn * 3:(Kn + 1) * 3])) == 0.0


def test_sa_weight_from_power_iteration_and_applicability():
    lx = lt = 16
    U = hot_field(lx, lt, seed=52, sweeps=10)
    A = normal_matrix(U, 0.1)
    start = synth.gaussian(2 * lx * lt, 3)
    lam = mg.power_lambda_max(A, start, 200)
    ev = np.linalg.eigvalsh(A.toarray())
    assert ev[-1] * 0.97 <= lam <= ev[-1] * (1 + 1e-12)
    assert mg.sa_applies((16, 16, 2), (4, 4))
    assert not mg.sa_applies((16, 16, 2), (2, 4))
    assert not mg.sa_applies((4, 16, 2), (4, 4))


@pytest.mark.parametrize("levels", [2, 3])
def test_sa_vcycle_error_propagator_and_projector(levels):
    """The V-cycle identity and the A-orthogonal coarse projector hold with the
    smoothed prolongator (Galerkin with any full-rank P)."""
    lx = lt = 16 if levels == 2 else 32
    U = hot_field(lx, lt, seed=53, sweeps=10)
    A = normal_matrix(U, 0.2)
    blocks = [(4, 4)] * (levels - 1)
    nvs = [3] * (levels - 1)
    R = synth.setup_randoms(lx, lt, blocks, nvs, 6)
    h = mg.adaptive_setup(A, (lx, lt, 2), blocks, nvs, R, nu=2, omega=0.8, setup_iters=2, sa_scale=4 / 3)
    assert h.levels[0].sa_weight > 0
    Ad = A.toarray()
    n = Ad.shape[0]
    lev = h.levels[0]
    P = lev.P.toarray()
    if levels == 2:
        Ac = h.levels[1].A.toarray()
        E = np.eye(n) - P @ np.linalg.solve(Ac, P.conj().T @ Ad)
        np.testing.assert_allclose(E @ E, E, atol=1e-10)
        np.testing.assert_allclose(Ad @ E, (Ad @ E).conj().T, atol=1e-10)
    nc = P.shape[1]
    b = synth.gaussian(n, 8)
    # apply both sides of I - V A = (I - R A)(I - P V_c P^H A)(I - R A) to one vector
    def R_(v):
        return mg.smoother_apply(A, lev.coefs, v)
    lhs = b - mg.vcycle(h, 0, A @ b)
    v1 = b - R_(A @ b)
    v2 = v1 - P @ mg.vcycle(h, 1, P.conj().T @ (A @ v1))
    rhs = v2 - R_(A @ v2)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11 * np.linalg.norm(b))


# ---------------------------------------------------------------------------
# Chirality-split aggregates (the alternative reading of the aggregates S_j as
# subsets of variables: each block split by chirality, gamma5 = sigma3)
# ---------------------------------------------------------------------------

def _split_hierarchy(levels=3, lx=16, lt=16, nv=3, sa_scale=0.0, seed=61):
    U = hot_field(lx, lt, seed, sweeps=10)
    A = normal_matrix(U, 0.15)
    blocks = [(2, 2)] * (levels - 1)
    nvs = [nv] * (levels - 1)
    R = synth.setup_randoms(lx, lt, blocks, nvs, seed, split=True)
    h = mg.adaptive_setup(A, (lx, lt, 2), blocks, nvs, R, nu=2, omega=0.8, setup_iters=2, sa_scale=sa_scale,
                          split=True)
    return A, h


def test_split_gather_partitions_by_component_parity():
    G = mg.aggregate_gather((8, 4, 2), (2, 2), split=True)
    assert G.shape == (2 * 4 * 2, 2 * 2)
    assert np.array_equal(np.sort(G.ravel()), np.arange(8 * 4 * 2))
    # row 2J + chi: block J, spin chi, sites in the unsplit order
    assert G[0].tolist() == [0, 2, 16, 18] and G[1].tolist() == [1, 3, 17, 19]
    Gc = mg.aggregate_gather((4, 4, 6), (2, 2), split=True)
    assert all(int(i) % 6 % 2 == 0 for i in Gc[0]) and all(int(i) % 6 % 2 == 1 for i in Gc[1])


def test_split_tentative_prolongator_commutes_with_gamma5():
    """gamma5 P_t = P_t gamma5_c with gamma5_c = diag((-1)^c) on every coarse site: on the
    fine level gamma5 = sigma3, on a coarse level the parity of the variable."""
    _, h = _split_hierarchy()
    for l in range(2):
        lev = h.levels[l]
        P = lev.P_t.toarray()
        n, nc_tot = P.shape
        g_f = np.where(np.arange(n) % lev.shape[2] % 2 == 0, 1.0, -1.0)
        g_c = np.where(np.arange(nc_tot) % 2 == 0, 1.0, -1.0)
        if l == 0:
            np.testing.assert_array_equal(g_f, np.diag(gamma5_matrix(16 * 16).toarray()))
        assert np.max(np.abs(g_f[:, None] * P - P * g_c[None, :])) == 0.0
        np.testing.assert_allclose(P.conj().T @ P, np.eye(nc_tot), atol=1e-14)
        assert h.levels[l + 1].shape[2] == 2 * 3


def test_split_columns_equal_qr_of_restricted_candidates():
    """Column 2k + chi on block K is the k-th column of the QR factor (positive real
    diagonal of R) of the candidates restricted to the chi-variables of K."""
    rng = np.random.default_rng(12)
    lx, lt, nv = 4, 4, 3
    V = rng.standard_normal((nv, 2 * lx * lt)) + 1j * rng.standard_normal((nv, 2 * lx * lt))
    lev = mg.Level(A=normal_matrix(hot_field(lx, lt, 3, sweeps=2), 0.3), shape=(lx, lt, 2))
    lev, nxt = mg.coarsen(lev, V, (2, 2), split=True)
    P = lev.P_t.toarray()
    Gb = mg.aggregate_gather((lx, lt, 2), (2, 2))
    for K in range(Gb.shape[0]):
        for chi in (0, 1):
            rows = [int(i) for i in Gb[K] if i % 2 == chi]
            Q, Rr = np.linalg.qr(V[:, rows].T)
            ph = np.diag(Rr) / np.abs(np.diag(Rr))   # Q R = (Q ph)(ph^* R), diag(ph^* R) > 0
            cols = [K * 2 * nv + 2 * k + chi for k in range(nv)]
            np.testing.assert_allclose(P[np.ix_(rows, cols)], Q * ph[None, :], atol=1e-13)
    assert nxt.shape == (2, 2, 2 * nv)


def test_split_range_contains_unsplit_range():
    """Every unsplit column lies in the span of the split columns of its block."""
    rng = np.random.default_rng(13)
    V = rng.standard_normal((3, 2 * 8 * 8)) + 1j * rng.standard_normal((3, 2 * 8 * 8))
    A = normal_matrix(hot_field(8, 8, 4, sweeps=2), 0.3)
    Pu = mg.coarsen(mg.Level(A=A, shape=(8, 8, 2)), V, (2, 2))[0].P_t.toarray()
    Ps = mg.coarsen(mg.Level(A=A, shape=(8, 8, 2)), V, (2, 2), split=True)[0].P_t.toarray()
    np.testing.assert_allclose(Ps @ (Ps.conj().T @ Pu), Pu, atol=1e-13)
    assert np.linalg.matrix_rank(Ps) == 2 * np.linalg.matrix_rank(Pu)


@pytest.mark.parametrize("sa_scale", [0.0, 4 / 3])
def test_split_hierarchy_vcycle_identity_and_mgcg(sa_scale):
    """With split aggregates the V-cycle keeps I - V A = (I - R A)(I - P V_c P^H A)(I - R A)
    and MG-CG converges to the direct solution."""
    lx = lt = 16
    U = hot_field(lx, lt, 62, sweeps=10)
    A = normal_matrix(U, 0.15)
    blocks = [(4, 4)]
    R = synth.setup_randoms(lx, lt, blocks, [3], 62, split=True)
    h = mg.adaptive_setup(A, (lx, lt, 2), blocks, [3], R, nu=2, omega=0.8, setup_iters=2, sa_scale=sa_scale,
                          split=True)
    assert h.levels[1].shape == (4, 4, 6) and (h.levels[0].sa_weight > 0) == (sa_scale > 0)
    lev = h.levels[0]
    P = lev.P.toarray()
    Ad = A.toarray()
    b = synth.gaussian(A.shape[0], 9)
    lhs = b - mg.vcycle(h, 0, A @ b)
    v1 = b - mg.smoother_apply(A, lev.coefs, A @ b)
    v2 = v1 - P @ np.linalg.solve(h.levels[1].A.toarray(), P.conj().T @ (A @ v1))
    rhs = v2 - mg.smoother_apply(A, lev.coefs, A @ v2)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11 * np.linalg.norm(b))
    x, info = mg.mg_cg(h, b, 1e-12)
    assert info.converged
    np.testing.assert_allclose(x, np.linalg.solve(Ad, b), atol=1e-9 * np.linalg.norm(np.linalg.solve(Ad, b)))


# ---------------------------------------------------------------------------
# Adaptive number of vectors (Adaptive Multigrid section: the procedure is repeated
# until a V-cycle reduces a random error sufficiently)
# ---------------------------------------------------------------------------

def test_two_level_factor_matches_dense_error_propagator():
    """two_level_factor = (||E^s e0||_A / ||e0||_A)^(1/s) with the dense two-level
    error propagator E = (I - R A)(I - P A_c^{-1} P^H A)(I - R A)."""
    lx = lt = 8
    U = hot_field(lx, lt, seed=91, sweeps=10)
    A = normal_matrix(U, 0.1)
    R = synth.setup_randoms(lx, lt, [(2, 2)], [3], 4)
    h = mg.adaptive_setup(A, (lx, lt, 2), [(2, 2)], [3], R, nu=2, omega=0.8, setup_iters=2)
    lev = h.levels[0]
    Ad = A.toarray()
    n = Ad.shape[0]
    P = lev.P.toarray()
    Ac = h.levels[1].A.toarray()
    Rd = mg.smoother_matrix(Ad, lev.coefs)
    I = np.eye(n)
    E = (I - Rd @ Ad) @ (I - P @ np.linalg.solve(Ac, P.conj().T @ Ad)) @ (I - Rd @ Ad)
    e0 = R[0][0]
    for s in (1, 3):
        e = np.linalg.matrix_power(E, s) @ e0
        want = (math.sqrt(np.vdot(e, Ad @ e).real) / math.sqrt(np.vdot(e0, Ad @ e0).real)) ** (1 / s)
        got = mg.two_level_factor(lev, h.levels[1].A, e0, s)
        assert abs(got - want) <= 1e-10 * want
        assert 0 < got < 1


def test_nv_stop_off_and_at_one():
    """nv_stop_rho = 0 keeps Nv vectors and measures nothing; a threshold of 1 stops
    after the first vector, since a two-level cycle with an exact coarse solve and a
    convergent smoother contracts the A-norm (factor < 1)."""
    lx = lt = 16
    U = hot_field(lx, lt, seed=92, sweeps=10)
    A = normal_matrix(U, 0.1)
    R = synth.setup_randoms(lx, lt, [(4, 4)], [5], 5)
    log = []
    h = mg.adaptive_setup(A, (lx, lt, 2), [(4, 4)], [5], R, nu=2, omega=0.8, setup_iters=2, log=log)
    assert log[0]["nv"] == 5 and log[0]["factors"] == [] and h.levels[1].shape[2] == 5
    log = []
    h = mg.adaptive_setup(A, (lx, lt, 2), [(4, 4)], [5], R, nu=2, omega=0.8, setup_iters=2, log=log,
                          nv_stop_rho=1.0)
    assert log[0]["nv"] == 1 and h.levels[1].shape[2] == 1 and 0 < log[0]["factors"][0] < 1


def test_nv_stop_full_coarse_space_is_exact():
    """1x1 aggregates with both spin vectors make P unitary, so the coarse correction
    is exact and the two-level factor is 0 (to rounding) after the second vector,
    while one vector leaves a factor in (0, 1)."""
    lx = lt = 8
    U = hot_field(lx, lt, seed=93, sweeps=10)
    A = normal_matrix(U, 0.2)
    R = synth.setup_randoms(lx, lt, [(1, 1)], [2], 6)
    log = []
    mg.adaptive_setup(A, (lx, lt, 2), [(1, 1)], [2], R, nu=2, omega=0.8, setup_iters=2, log=log,
                      nv_stop_rho=1e-300)
    f1, f2 = log[0]["factors"]
    assert 0 < f1 < 1 and f2 <= 1e-7 * f1


def test_nv_stop_is_a_prefix_of_the_full_setup_and_shortens_the_next_level():
    """With a threshold between two consecutive factors of the full setup, the setup
    keeps exactly the vectors up to the first factor below it: the same vectors and
    factors as the full run up to there (the rule only truncates), the next level has
    that many variables per site and is built from the leading part of its random
    rows, and the resulting 3-level hierarchy satisfies the V-cycle identity."""
    lx = lt = 32
    U = hot_field(lx, lt, seed=94, sweeps=20)
    A = normal_matrix(U, 0.05)
    blocks, nvs = [(4, 4), (2, 2)], [8, 4]
    R = synth.setup_randoms(lx, lt, blocks, nvs, 7)
    full = []
    mg.adaptive_setup(A, (lx, lt, 2), blocks, nvs, R, nu=2, omega=0.8, setup_iters=3, log=full, nv_stop_rho=1e-300)
    f = full[0]["factors"]
    assert len(f) == 8
    # a threshold halfway (geometrically) across the largest relative drop between vector counts 2..7
    i = max(range(1, 6), key=lambda j: f[j - 1] / f[j])
    k = i + 1  # vectors kept: the factor after k vectors is the first below the threshold
    thr = math.sqrt(f[i] * f[i - 1])
    assert f[i - 1] / f[i] > 1.01 and all(x > thr for x in f[:i]) and f[i] < thr
    log = []
    h = mg.adaptive_setup(A, (lx, lt, 2), blocks, nvs, R, nu=2, omega=0.8, setup_iters=3, log=log, nv_stop_rho=thr)
    assert log[0]["nv"] == k and h.levels[1].shape == (8, 8, k)
    np.testing.assert_allclose(log[0]["factors"], f[:k], rtol=1e-12)
    Rk = [R[0], R[1][:, :8 * 8 * k]]
    ref = mg.adaptive_setup(A, (lx, lt, 2), blocks, [k, 4], Rk, nu=2, omega=0.8, setup_iters=3)
    np.testing.assert_allclose(h.levels[2].A.toarray(), ref.levels[2].A.toarray(), atol=1e-12)
    b = synth.gaussian(2 * lx * lt, 9)
    lev = h.levels[0]
    lhs = b - mg.vcycle(h, 0, A @ b)
    v1 = b - mg.smoother_apply(A, lev.coefs, A @ b)
    v2 = v1 - lev.P @ mg.vcycle(h, 1, lev.P.conj().T @ (A @ v1))
    rhs = v2 - mg.smoother_apply(A, lev.coefs, A @ v2)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11 * np.linalg.norm(b))


@pytest.mark.parametrize("beta", [3.0, 10.0])
def test_device_metropolis_plaquette_and_charge(beta):
    """The torch copy of the Metropolis update (run here on the CPU) thermalises to the
    same plaquette, I1(beta)/I0(beta), and gives integer charges, for a batch of fields."""
    from scipy.special import i0, i1

    th = synth.metropolis_u1_device(32, 32, beta, 300, 5, count=4, device="cpu").numpy()
    plaq = [synth.mean_plaquette(t) for t in th]
    target = i1(beta) / i0(beta)
    # four 32^2 fields: 4096 plaquettes; the spread of cos is below 0.5 at these couplings
    assert abs(np.mean(plaq) - target) < 3 * 0.5 / math.sqrt(4096)
    for t in th:
        q = synth.topological_charge(t)
        assert abs(q - round(q)) < 1e-9
