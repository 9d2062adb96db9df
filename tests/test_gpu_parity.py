"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

FP64 operator applications must agree to 1e-12 relative (max-norm over the
output); solves must reach a true residual <= 1e-10 recomputed by the oracle's own
sparse A on the downloaded solution.  Lattices are small enough for the oracle to
finish in seconds but span several thread blocks and end on a ragged tail.
"""

import math

import numpy as np
import pytest

import synth
from oracle import multigrid as mg
from oracle.wilson import dirac_matrix, normal_matrix

pytestmark = pytest.mark.gpu

TOL_APPLY = 1e-12


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def field(lx, lt, seed, beta=3.0, sweeps=20):
    return synth.links_from_angles(synth.metropolis_u1(lx, lt, beta, sweeps, seed))


def smg_mod():
    import paper_0710_3612_amd as smg

    return smg


def hierarchy_inputs(lx, lt, blocks, nvs, seed, split=False):
    """Near-null vectors and calibration starts per level, shared by both sides."""
    shapes = synth.level_shapes(lx, lt, blocks, nvs, split)
    vecs, calib = [], []
    for l, nv in enumerate(nvs):
        cx, ct, dof = shapes[l]
        n = cx * ct * dof
        vecs.append(synth.gaussian((nv, n), seed * 100 + l))
        calib.append(synth.gaussian(n, seed * 100 + 50 + l))
    return vecs, calib


def links_from_sparse(Ac, cx, ct, nc):
    """Oracle coarse matrix -> [K, 9, nc, nc] link blocks (coarse extents >= 3)."""
    A = Ac.toarray()
    out = np.zeros((cx * ct, 9, nc, nc), dtype=np.complex128)
    for K in range(cx * ct):
        kt, kx = divmod(K, cx)
        for D in range(9):
            dt, dx = D // 3 - 1, D % 3 - 1
            Kn = ((kt + dt) % ct) * cx + (kx + dx) % cx
            out[K, D] = A[K * nc:(K + 1) * nc, Kn * nc:(Kn + 1) * nc]
    return out


# ---------------------------------------------------------------------------
# Fine operators
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("lx,lt,nrhs", [(30, 26, 3), (64, 48, 1), (8, 4, 2), (128, 64, 2), (32, 32, 1),
                                        (16, 64, 3), (192, 40, 1), (64, 12, 2), (256, 128, 1),
                                        (96, 24, 1)])
def test_apply_D_and_A(cuda, lx, lt, nrhs):
    smg = smg_mod()
    U = field(lx, lt, seed=lx + lt)
    m = 0.07
    p = smg.make_params(lx, lt, m, levels=1)
    s = smg.Solver(dev(U), p)
    x = synth.gaussian((nrhs, 2 * lx * lt), 3)
    D = dirac_matrix(U, m)
    A = normal_matrix(U, m)
    yd = host(s.apply_D(dev(x))).reshape(nrhs, -1)
    yh = host(s.apply_D(dev(x), dagger=True)).reshape(nrhs, -1)
    ya = host(s.apply_A(dev(x))).reshape(nrhs, -1)
    for j in range(nrhs):
        assert rel_err(yd[j], D @ x[j]) <= TOL_APPLY
        assert rel_err(yh[j], D.conj().T @ x[j]) <= TOL_APPLY
        assert rel_err(ya[j], A @ x[j]) <= TOL_APPLY
    s.close()


def test_apply_periodic_bc(cuda):
    smg = smg_mod()
    lx, lt = 16, 12
    U = field(lx, lt, seed=5)
    p = smg.make_params(lx, lt, -0.3, levels=1, t_antiperiodic=False)
    s = smg.Solver(dev(U), p)
    x = synth.gaussian(2 * lx * lt, 4)
    assert rel_err(host(s.apply_D(dev(x))), dirac_matrix(U, -0.3, antiperiodic_t=False) @ x) <= TOL_APPLY


# ---------------------------------------------------------------------------
# Hierarchy from given vectors: every step of the V-cycle
# ---------------------------------------------------------------------------

SA = 4.0 / 3.0
CASES = [
    # lx, lt, blocks, nvs, mass, sa_scale
    (32, 24, [(4, 4), (2, 2)], [6, 5], 0.05, SA),   # smoothed level 1, plain level 2
    (24, 24, [(4, 4)], [8], 0.1, 0.0),              # plain aggregation
    (40, 24, [(4, 2), (2, 3)], [4, 4], 0.2, SA),    # blocks too small to smooth
    (64, 64, [(4, 4), (4, 4)], [6, 6], 0.03, SA),   # fused fine kernel, smoothed on both levels
    (32, 32, [(4, 4), (4, 4)], [4, 4], 0.1, SA),    # coarse extents 8 -> 2 (two colours)
    (20, 20, [(4, 4)], [5], 0.1, SA),               # odd coarse vector length (5 x 5 x 5)
    (64, 64, [(4, 4)], [8], 0.1, SA),               # coarsest 2048: blocked Gauss-Jordan, 4 blocks
    (48, 48, [(4, 4)], [7], 0.1, SA),               # coarsest 1008: blocked, ragged last block
    (64, 64, [(2, 2)], [5], 0.1, SA),               # coarsest 5120: blocked inverse, tiled multi-RHS apply
    # chirality-split aggregates: 2 Nv coarse variables per site
    (32, 32, [(4, 4), (2, 2)], [4, 3], 0.05, SA, True),  # split on both levels (dof 8, then 6)
    (64, 64, [(4, 4)], [6], 0.1, SA, True),              # nc = 12 on 16^2 coarse sites, fused fine kernel
    (24, 24, [(4, 4)], [8], 0.1, 0.0, True),             # plain aggregation, nc = 16
]


def windowed(P, shape, block, nv, halo):
    """Oracle sparse P -> [J, k, nw] over the (bx+2h) x (bt+2h) windows."""
    lx, lt, dof = shape
    bx, bt = block
    cx, ct = lx // bx, lt // bt
    wx, wy = bx + 2 * halo, bt + 2 * halo
    Pd = P.tocsc()
    out = np.zeros((cx * ct, nv, wx * wy * dof), dtype=np.complex128)
    for J in range(cx * ct):
        jt, jx = divmod(J, cx)
        for a in range(wy):
            for b in range(wx):
                t = (jt * bt + a - halo) % lt
                x = (jx * bx + b - halo) % lx
                for d in range(dof):
                    f = (t * lx + x) * dof + d
                    i = (a * wx + b) * dof + d
                    for k in range(nv):
                        out[J, k, i] = Pd[f, J * nv + k]
    return out


@pytest.fixture(scope="module", params=range(len(CASES)))
def pair(request):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    smg = smg_mod()
    lx, lt, blocks, nvs, m, sa = CASES[request.param][:6]
    split = CASES[request.param][6] if len(CASES[request.param]) > 6 else False
    U = field(lx, lt, seed=request.param + 1)
    vecs, calib = hierarchy_inputs(lx, lt, blocks, nvs, request.param + 7, split)
    A = normal_matrix(U, m)
    h = mg.hierarchy_from_vectors(A, (lx, lt, 2), blocks, vecs, calib, nu=4, omega=0.8, sa_scale=sa, split=split)
    p = smg.make_params(lx, lt, m, levels=len(blocks) + 1, blocks=blocks, nv=nvs, sa_scale=sa,
                        split_chirality=split)
    s = smg.Solver(dev(U), p, vectors=dev(np.concatenate([v.ravel() for v in vecs])),
                   calib=dev(np.concatenate(calib)))
    yield dict(U=U, A=A, h=h, s=s, lx=lx, lt=lt, blocks=blocks, nvs=nvs, m=m, calib=calib)
    s.close()


def test_smoother_coefficients(pair):
    h, s = pair["h"], pair["s"]
    for l in range(len(pair["blocks"])):
        np.testing.assert_allclose(s.smoother_coefs(l), h.levels[l].coefs, rtol=1e-12)


def test_prolongator(pair):
    """Tentative P_t (block Gram-Schmidt) and the smoothed P = (I - w A) P_t."""
    h, s = pair["h"], pair["s"]
    for l in range(len(pair["blocks"])):
        lev = h.levels[l]
        nc = s.level_info(l + 1)[2]
        if lev.split:
            assert rel_err(host(s.prolongator(l)), windowed(lev.P_t, lev.shape, lev.block, nc, 0)) <= 1e-12
        else:
            assert rel_err(host(s.prolongator(l)), lev.U) <= 1e-12
        halo, w = s.transfer_info(l)
        assert halo == (1 if lev.sa_weight > 0 else 0)
        if halo:
            assert abs(w - lev.sa_weight) <= 1e-12 * lev.sa_weight
        ref = windowed(lev.P, lev.shape, lev.block, nc, halo)
        assert rel_err(host(s.prolongator(l, smoothed=True)), ref) <= 1e-12


def dense_from_links(Lk, cx, ct, nc):
    """[K, 9, nc, nc] link blocks -> dense coarse matrix (offsets naming the same
    neighbour on extents <= 2 are summed, as the coarse apply does)."""
    A = np.zeros((cx * ct * nc, cx * ct * nc), dtype=np.complex128)
    for K in range(cx * ct):
        kt, kx = divmod(K, cx)
        for D in range(9):
            dt, dx = D // 3 - 1, D % 3 - 1
            Kn = ((kt + dt) % ct) * cx + (kx + dx) % cx
            A[K * nc:(K + 1) * nc, Kn * nc:(Kn + 1) * nc] += Lk[K, D]
    return A


def test_coarse_links(pair):
    h, s = pair["h"], pair["s"]
    for l in range(1, len(pair["blocks"]) + 1):
        cx, ct, nc = s.level_info(l)
        links = host(s.coarse_links(l))
        if min(cx, ct) >= 3:
            assert rel_err(links, links_from_sparse(h.levels[l].A, cx, ct, nc)) <= 1e-12
        assert rel_err(dense_from_links(links, cx, ct, nc), h.levels[l].A.toarray()) <= 1e-12


@pytest.mark.parametrize("nrhs", [16, 20, 33])
def test_transfer_many_rhs_matrix_cores(pair, nrhs):
    """FP64 restriction and prolongation of at least mfma_min_rhs right-hand sides
    (the FP64 matrix-core kernels, 16, 32 or 64 columns per wave with masked columns)
    equal P^H x and P e of the oracle's sparse P column by column, on every case's
    levels (smoothed windows, blocks of unequal extents, odd and chirality-split nc)."""
    h, s = pair["h"], pair["s"]
    for l in range(len(pair["blocks"])):
        n = s.level_size(l)
        nc = s.level_size(l + 1)
        P = h.levels[l].P
        x = synth.gaussian((nrhs, n), 17 + l + nrhs)
        e = synth.gaussian((nrhs, nc), 19 + l + nrhs)
        r = host(s.restrict(l, dev(x))).reshape(nrhs, -1)
        pe = host(s.prolong(l, dev(e))).reshape(nrhs, -1)
        for j in range(nrhs):
            assert rel_err(r[j], P.conj().T @ x[j]) <= 1e-12, (l, j)
            assert rel_err(pe[j], P @ e[j]) <= 1e-12, (l, j)


def test_transfer_and_coarse_apply(pair):
    h, s = pair["h"], pair["s"]
    for l in range(len(pair["blocks"])):
        n = s.level_size(l)
        nc = s.level_size(l + 1)
        P = h.levels[l].P
        x = synth.gaussian((2, n), 11 + l)
        e = synth.gaussian((2, nc), 13 + l)
        r = host(s.restrict(l, dev(x))).reshape(2, -1)
        pe = host(s.prolong(l, dev(e))).reshape(2, -1)
        Al = h.levels[l].A
        ya = host(s.apply_level(l, dev(x))).reshape(2, -1)
        rb = host(s.smooth(l, dev(x))).reshape(2, -1)
        for j in range(2):
            assert rel_err(r[j], P.conj().T @ x[j]) <= 1e-12
            assert rel_err(pe[j], P @ e[j]) <= 1e-12
            assert rel_err(ya[j], Al @ x[j]) <= 1e-12
            assert rel_err(rb[j], mg.smoother_apply(Al, h.levels[l].coefs, x[j])) <= 1e-11
        Ac = h.levels[l + 1].A
        yc = host(s.apply_level(l + 1, dev(e))).reshape(2, -1)
        for j in range(2):
            assert rel_err(yc[j], Ac @ e[j]) <= 1e-12


def test_vcycle(pair):
    h, s = pair["h"], pair["s"]
    n = s.level_size(0)
    b = synth.gaussian((3, n), 17)
    x = host(s.vcycle(dev(b))).reshape(3, -1)
    for j in range(3):
        assert rel_err(x[j], mg.vcycle(h, 0, b[j])) <= 1e-11


def test_mgcg_solve_fp64_and_mixed(pair):
    smg = smg_mod()
    U, A, s, m = pair["U"], pair["A"], pair["s"], pair["m"]
    n = s.level_size(0)
    b = synth.gaussian((2, n), 19)
    Dm = dirac_matrix(U, m)
    rhs = np.stack([Dm.conj().T @ b[j] for j in range(2)])
    xo = [mg.mg_cg(pair["h"], rhs[j], 1e-10)[0] for j in range(2)]
    for prec in (smg.FP64, smg.MIXED):
        x, stats, code = s.solve(dev(rhs), tol=1e-10, maxiter=500, precision=prec)
        assert code == 0
        xh = host(x).reshape(2, -1)
        for j in range(2):
            res = np.linalg.norm(rhs[j] - A @ xh[j]) / np.linalg.norm(rhs[j])
            assert res <= 1e-10, (prec, j, res)
            assert stats[j]["true_relres"] <= 1e-10
            # forward error vs the oracle's MG-CG solution
            assert np.linalg.norm(xh[j] - xo[j]) / np.linalg.norm(xo[j]) < 1e-6


def test_set_mass_rebuilds_coarse_operators(pair):
    """Setup reuse across masses: P kept, A_c(m) rebuilt by Eq. 2, smoothers recalibrated."""
    U, h, s = pair["U"], pair["h"], pair["s"]
    m2 = pair["m"] + 0.13
    s.set_mass(m2)
    try:
        h2 = mg.set_mass(h, normal_matrix(U, m2), pair["calib"], 4, 0.8)
        for l in range(1, len(pair["blocks"]) + 1):
            cx, ct, nc = s.level_info(l)
            assert rel_err(dense_from_links(host(s.coarse_links(l)), cx, ct, nc), h2.levels[l].A.toarray()) <= 1e-12
        for l in range(len(pair["blocks"])):
            np.testing.assert_allclose(s.smoother_coefs(l), h2.levels[l].coefs, rtol=1e-12)
    finally:
        s.set_mass(pair["m"])


@pytest.mark.parametrize("split", [False, True])
def test_affine_remass_equals_galerkin(cuda, split):
    """remass_affine: the setup keeps the mass coefficients C0, C1, C2 of every coarse
    operator (C0 = P^H P is not I for the smoothed P), and smg_derive / smg_set_mass
    form A^(l)(m) = C2 + m C1 + m^2 C0 in one pass.  Every level equals the oracle's
    Galerkin rebuild at the new mass (set_mass) and the GPU's own Eq. 2 rebuild within
    1e-12; the smoothers match; the setup handle's own links are those of a setup
    without coefficients, bit for bit; MG-CG on the derived handle reaches 1e-10."""
    smg = smg_mod()
    lx = lt = 32
    blocks, nvs, m, m2 = [(4, 4), (2, 2)], [4, 3], 0.05, 0.21
    U = field(lx, lt, seed=81)
    vecs, calib = hierarchy_inputs(lx, lt, blocks, nvs, 82, split)
    A = normal_matrix(U, m)
    h = mg.hierarchy_from_vectors(A, (lx, lt, 2), blocks, vecs, calib, nu=4, omega=0.8, sa_scale=SA, split=split)
    h2 = mg.set_mass(h, normal_matrix(U, m2), calib, 4, 0.8)
    vv, cc = dev(np.concatenate([v.ravel() for v in vecs])), dev(np.concatenate(calib))
    out = {}
    for aff in (True, False):
        p = smg.make_params(lx, lt, m, levels=3, blocks=blocks, nv=nvs, sa_scale=SA, split_chirality=split,
                            remass_affine=aff)
        out[aff] = smg.Solver(dev(U), p, vectors=vv, calib=cc)
    try:
        for l in (1, 2):
            assert np.array_equal(host(out[True].coarse_links(l)), host(out[False].coarse_links(l)))
        d_aff, d_gal = out[True].derive(m2), out[False].derive(m2)
        try:
            for l in (1, 2):
                cx, ct, nc = d_aff.level_info(l)
                la, lg = host(d_aff.coarse_links(l)), host(d_gal.coarse_links(l))
                assert rel_err(la, lg) <= 1e-12
                assert rel_err(dense_from_links(la, cx, ct, nc), h2.levels[l].A.toarray()) <= 1e-12
            for l in (0, 1):
                np.testing.assert_allclose(d_aff.smoother_coefs(l), h2.levels[l].coefs, rtol=1e-12)
            rhs = dirac_matrix(U, m2).conj().T @ synth.gaussian(2 * lx * lt, 83)
            x, st, code = d_aff.solve(dev(rhs), tol=1e-10, precision=smg.MIXED)
            assert code == 0
            assert np.linalg.norm(rhs - normal_matrix(U, m2) @ host(x)) / np.linalg.norm(rhs) <= 1e-10
        finally:
            d_aff.close()
            d_gal.close()
        out[True].set_mass(m2)
        for l in (1, 2):
            cx, ct, nc = out[True].level_info(l)
            assert rel_err(dense_from_links(host(out[True].coarse_links(l)), cx, ct, nc),
                           h2.levels[l].A.toarray()) <= 1e-12
    finally:
        for s in out.values():
            s.close()


# ---------------------------------------------------------------------------
# Adaptive setup and the c1 workload (32^2, beta 3, m 0.1, 2 levels, Nv 8)
# ---------------------------------------------------------------------------

def c1_inputs():
    lx = lt = 32
    U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 200, 1000))
    R = synth.setup_randoms(lx, lt, [(4, 4)], [8], 1)
    b = synth.gaussian(2 * lx * lt, 0)
    return U, R, b


def test_adaptive_setup_and_solve_c1(cuda):
    smg = smg_mod()
    U, R, b = c1_inputs()
    lx = lt = 32
    m = 0.1
    A = normal_matrix(U, m)
    rhs = dirac_matrix(U, m).conj().T @ b
    h = mg.adaptive_setup(A, (lx, lt, 2), [(4, 4)], [8], R, nu=4, omega=0.8, setup_iters=5, coarsest="cg",
                          sa_scale=4 / 3)
    xo, io = mg.mg_cg(h, rhs, 1e-10)
    p = smg.make_params(lx, lt, m, levels=2, blocks=[(4, 4)], nv=[8], coarsest=smg.COARSEST_CG, sa_scale=4 / 3)
    s = smg.Solver(dev(U), p, randoms=dev(np.concatenate([r.ravel() for r in R])))
    # setup parity: smoother exactly, prolongator up to rounding amplified by the
    # setup iterations, compared through the per-aggregate projectors P_J P_J^H
    np.testing.assert_allclose(s.smoother_coefs(0), h.levels[0].coefs, rtol=1e-12)
    Pg = host(s.prolongator(0))
    Po = h.levels[0].U
    proj_g = np.einsum("jki,jkl->jil", Pg, Pg.conj())
    proj_o = np.einsum("jki,jkl->jil", Po, Po.conj())
    assert np.max(np.abs(proj_g - proj_o)) <= 1e-8
    assert abs(s.transfer_info(0)[1] - h.levels[0].sa_weight) <= 1e-12 * h.levels[0].sa_weight
    for prec in (smg.FP64, smg.MIXED):
        x, st, code = s.solve(dev(rhs), tol=1e-10, maxiter=500, precision=prec)
        assert code == 0
        xh = host(x)
        res = np.linalg.norm(rhs - A @ xh) / np.linalg.norm(rhs)
        assert res <= 1e-10
        assert np.linalg.norm(xh - xo) / np.linalg.norm(xo) < 1e-7
        if prec == smg.FP64:
            assert abs(st[0]["iterations"] - io.iterations) <= 1
    # plain CG agrees with the oracle's CG iteration count
    xc, stc, code = s.cg(dev(rhs), tol=1e-10)
    _, ic = mg.cg(A, rhs, 1e-10)
    assert code == 0 and abs(stc[0]["iterations"] - ic.iterations) <= 2
    s.close()


def test_adaptive_setup_split_chirality(cuda):
    """Adaptive setup with chirality-split aggregates (3 levels, 2 Nv coarse variables
    per site): smoothers, the per-block projectors of P and the solves against the oracle."""
    smg = smg_mod()
    lx = lt = 32
    m = 0.08
    blocks, nvs = [(4, 4), (2, 2)], [4, 3]
    U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 50, 1001))
    R = synth.setup_randoms(lx, lt, blocks, nvs, 2, split=True)
    A = normal_matrix(U, m)
    rhs = dirac_matrix(U, m).conj().T @ synth.gaussian(2 * lx * lt, 1)
    h = mg.adaptive_setup(A, (lx, lt, 2), blocks, nvs, R, nu=4, omega=0.8, setup_iters=4, sa_scale=4 / 3,
                          split=True)
    xo, io = mg.mg_cg(h, rhs, 1e-10)
    p = smg.make_params(lx, lt, m, levels=3, blocks=blocks, nv=nvs, setup_iters=4, sa_scale=4 / 3,
                        split_chirality=True)
    s = smg.Solver(dev(U), p, randoms=dev(np.concatenate([r.ravel() for r in R])))
    assert s.level_info(1) == (8, 8, 8) and s.level_info(2) == (4, 4, 6)
    np.testing.assert_allclose(s.smoother_coefs(0), h.levels[0].coefs, rtol=1e-12)
    for l in range(2):
        Pg = host(s.prolongator(l))
        Po = windowed(h.levels[l].P_t, h.levels[l].shape, h.levels[l].block, Pg.shape[1], 0)
        proj_g = np.einsum("jki,jkl->jil", Pg, Pg.conj())
        proj_o = np.einsum("jki,jkl->jil", Po, Po.conj())
        assert np.max(np.abs(proj_g - proj_o)) <= 1e-7, l
        # chirality: column 2k + chi vanishes on the variables of the other chirality
        dof = h.levels[l].shape[2]
        chi_var = np.arange(Pg.shape[2]) % dof % 2
        for c in range(Pg.shape[1]):
            assert np.max(np.abs(Pg[:, c, chi_var != c % 2])) == 0.0
    for prec in (smg.FP64, smg.MIXED):
        x, st, code = s.solve(dev(rhs), tol=1e-10, maxiter=500, precision=prec)
        assert code == 0
        xh = host(x)
        assert np.linalg.norm(rhs - A @ xh) / np.linalg.norm(rhs) <= 1e-10
        assert np.linalg.norm(xh - xo) / np.linalg.norm(xo) < 1e-7
        if prec == smg.FP64:
            assert abs(st[0]["iterations"] - io.iterations) <= 1
    s.close()


def test_adaptive_nv_stop_matches_oracle(cuda):
    """Adaptive number of vectors: the oracle's full setup gives the two-level factor
    per vector count; with a threshold across its largest drop, the GPU's setup and the
    oracle's stop at the same count (the next level's variables per site), measure the
    same factors (within 1e-8: the GPU's coarse solve is CG to 1e-12), build the same
    per-aggregate projectors on both coarsenings (1e-8), and the MG-CG solve on the
    shortened hierarchy reaches 1e-10 within one iteration of the oracle's."""
    smg = smg_mod()
    lx = lt = 32
    m = 0.05
    blocks, nvs = [(4, 4), (2, 2)], [8, 4]
    U = field(lx, lt, seed=94, sweeps=20)
    A = normal_matrix(U, m)
    R = synth.setup_randoms(lx, lt, blocks, nvs, 7)
    kw = dict(nu=2, omega=0.8, setup_iters=3, sa_scale=SA)
    full = []
    mg.adaptive_setup(A, (lx, lt, 2), blocks, nvs, R, log=full, nv_stop_rho=1e-300, **kw)
    f = full[0]["factors"]
    i = max(range(1, 6), key=lambda j: f[j - 1] / f[j])
    thr = math.sqrt(f[i] * f[i - 1])
    log = []
    h = mg.adaptive_setup(A, (lx, lt, 2), blocks, nvs, R, log=log, nv_stop_rho=thr, **kw)
    k = log[0]["nv"]
    assert k == i + 1 < nvs[0]
    p = smg.make_params(lx, lt, m, levels=3, blocks=blocks, nv=nvs, setup_iters=3, smoother_steps=2,
                        sa_scale=SA, nv_stop_rho=thr)
    with smg.Solver(dev(U), p, randoms=dev(np.concatenate([r.ravel() for r in R]))) as s:
        assert s.level_info(1) == (8, 8, k)
        assert s.level_info(2) == h.levels[2].shape
        for l in range(2):
            np.testing.assert_allclose(s.setup_factors(l), log[l]["factors"], rtol=1e-8)
            Pg = host(s.prolongator(l))
            Po = h.levels[l].U
            assert Pg.shape == Po.shape
            proj_g = np.einsum("jki,jkl->jil", Pg, Pg.conj())
            proj_o = np.einsum("jki,jkl->jil", Po, Po.conj())
            assert np.max(np.abs(proj_g - proj_o)) <= 1e-8, l
        rhs = dirac_matrix(U, m).conj().T @ synth.gaussian(2 * lx * lt, 95)
        _, io = mg.mg_cg(h, rhs, 1e-10)
        x, st, code = s.solve(dev(rhs), tol=1e-10, precision=smg.FP64)
        assert code == 0
        assert np.linalg.norm(rhs - A @ host(x)) / np.linalg.norm(rhs) <= 1e-10
        assert abs(st[0]["iterations"] - io.iterations) <= 1
        # a mass derived from the shortened hierarchy keeps its shape
        with s.derive(m + 0.1) as d:
            assert d.level_info(1) == (8, 8, k)
            x, st, code = d.solve(dev(rhs), tol=1e-10, precision=smg.MIXED)
            assert code == 0


def test_batch_invariance_and_edge_cases(cuda):
    """A column's result is bitwise the same alone and in a batch; a zero column
    returns zero; NaN input is reported as a breakdown; maxiter too small is
    reported as not converged."""
    smg = smg_mod()
    lx = lt = 24
    U = field(lx, lt, seed=3, sweeps=50)
    p = smg.make_params(lx, lt, 0.05, levels=2, blocks=[(4, 4)], nv=[6], seed=9)
    s = smg.Solver(dev(U), p)
    n = 2 * lx * lt
    B = synth.gaussian((4, n), 23)
    B[2] = 0.0
    xb, stb, code = s.solve(dev(B), tol=1e-10)
    assert code == 0
    xb = host(xb).reshape(4, -1)
    assert np.all(xb[2] == 0)
    for j in (0, 1, 3):
        xa, _, _ = s.solve(dev(B[j]), tol=1e-10)
        assert np.array_equal(host(xa), xb[j])
    _, st, code = s.solve(dev(B[0]), tol=1e-10, maxiter=1)
    assert code == smg.NOTCONV and st[0]["status"] == smg.NOTCONV
    bad = B[0].copy()
    bad[5] = np.nan
    with pytest.raises(smg.SmgError) as ei:
        s.solve(dev(bad), tol=1e-10)
    assert ei.value.code == -5
    s.close()


def test_batch_invariance_many_columns(cuda):
    """Nine columns take the kernels that share operator loads across right-hand sides
    (coarse links for 8, P rows for 4 and 8 columns); each column still equals its
    single-column solve bit for bit, in FP64 and in mixed precision."""
    smg = smg_mod()
    lx = lt = 32
    U = field(lx, lt, seed=4, sweeps=50)
    p = smg.make_params(lx, lt, 0.05, levels=3, blocks=[(4, 4), (2, 2)], nv=[6, 4], seed=11)
    s = smg.Solver(dev(U), p)
    n = 2 * lx * lt
    B = synth.gaussian((9, n), 29)
    for prec in (smg.FP64, smg.MIXED):
        xb, _, code = s.solve(dev(B), tol=1e-10, precision=prec)
        assert code == 0
        xb = host(xb).reshape(9, -1)
        for j in (0, 5, 8):
            xa, _, _ = s.solve(dev(B[j]), tol=1e-10, precision=prec)
            assert np.array_equal(host(xa), xb[j]), (prec, j)
    s.close()


def test_fp32_operators(pair):
    """The FP32 copies of every level's operator (used inside the mixed-precision
    solves) against the FP64 oracle.  Inputs and links are rounded to FP32 (unit
    roundoff 6e-8) and each output sums at most 9 * nc * 4 products, so 2e-5 of the
    output max-norm bounds the error with a wide margin."""
    import torch

    h, s = pair["h"], pair["s"]
    for l in range(len(pair["blocks"]) + 1):
        n = s.level_size(l)
        x = synth.gaussian((2, n), 29 + l)
        y = s.apply_level_f32(l, torch.from_numpy(x.astype(np.complex64)).to("cuda")).cpu().numpy()
        y = y.reshape(2, -1).astype(np.complex128)
        Al = h.levels[l].A
        for j in range(2):
            assert rel_err(y[j], Al @ x[j]) <= 2e-5


def test_stop_on_recursive_residual(cuda):
    """stop_recursive: MG-CG and CG stop when the recursive residual reaches tol
    (the paper's stopping rule); the recomputed residual is still reported and,
    for a well-conditioned system, agrees with the oracle's to rounding."""
    smg = smg_mod()
    lx = lt = 24
    U = field(lx, lt, seed=12, sweeps=30)
    A = normal_matrix(U, 0.1)
    b = synth.gaussian(2 * lx * lt, 31)
    out = {}
    for flag in (False, True):
        p = smg.make_params(lx, lt, 0.1, levels=2, blocks=[(4, 4)], nv=[6], seed=4, stop_recursive=flag)
        with smg.Solver(dev(U), p) as s:
            x, st, code = s.solve(dev(b), tol=1e-10, maxiter=500, precision=smg.FP64)
            xc, stc, codec = s.cg(dev(b), tol=1e-10, maxiter=5000)
            assert code == 0 and codec == 0
            for xx, ss in ((x, st), (xc, stc)):
                res = np.linalg.norm(b - A @ host(xx)) / np.linalg.norm(b)
                assert abs(res - ss[0]["true_relres"]) <= 1e-3 * res + 1e-15
                assert res <= 1e-9
            out[flag] = (st[0]["iterations"], stc[0]["iterations"])
    assert out[True][0] <= out[False][0] and out[True][1] <= out[False][1]


@pytest.mark.parametrize("nu", [1, 2, 3])
def test_smoother_degrees(nu):
    """Smoother and V-cycle with nu = 1, 2 (the degree of the paper's experiment) and
    3 MR steps, which take the one-step, two-step-from-zero and first/last-step
    epilogues of the operator kernels: FP64 against the oracle to 1e-11, the FP32
    V-cycle to 1e-4 (FP32 rounding, as in the mixed-precision tests)."""
    smg = smg_mod()
    lx, lt, blocks, nvs, m = 32, 32, [(4, 4), (2, 2)], [6, 6], 0.07
    U = field(lx, lt, seed=41 + nu)
    vecs, calib = hierarchy_inputs(lx, lt, blocks, nvs, 43 + nu)
    A = normal_matrix(U, m)
    h = mg.hierarchy_from_vectors(A, (lx, lt, 2), blocks, vecs, calib, nu=nu, omega=0.8, sa_scale=4 / 3)
    p = smg.make_params(lx, lt, m, levels=3, blocks=blocks, nv=nvs, smoother_steps=nu)
    s = smg.Solver(dev(U), p, vectors=dev(np.concatenate([v.ravel() for v in vecs])), calib=dev(np.concatenate(calib)))
    try:
        n = s.level_size(0)
        b = synth.gaussian((2, n), 47 + nu)
        x = host(s.vcycle(dev(b))).reshape(2, -1)
        for l in range(2):
            bl = synth.gaussian((2, s.level_size(l)), 53 + l)
            rb = host(s.smooth(l, dev(bl))).reshape(2, -1)
            for j in range(2):
                assert rel_err(rb[j], mg.smoother_apply(h.levels[l].A, h.levels[l].coefs, bl[j])) <= 1e-11, (l, j)
        import torch

        x32 = host(s.vcycle_f32(torch.from_numpy(b.astype(np.complex64)).to("cuda"))).reshape(2, -1)
        for j in range(2):
            ref = mg.vcycle(h, 0, b[j])
            assert rel_err(x[j], ref) <= 1e-11, j
            assert rel_err(x32[j], ref) <= 1e-4, j
    finally:
        s.close()


@pytest.mark.parametrize("opst,c64", [(0, False), (2, False), (2, True)])
def test_fp32_vcycle_large_coarsest_matrix_cores(opst, c64):
    """FP32 V-cycle whose 5120-variable coarsest inverse is applied on the matrix
    cores from an FP32 or FP16 copy (n above the row-kernel limit), or in FP64 by
    the tiled kernel (coarsest_fp64), with FP32 or FP16 operator storage: within
    1e-4 (FP32) or 1e-3 (FP16, unit roundoff 2^-11 times 2) of the oracle's FP64
    V-cycle, for 1 and 33 right-hand sides (two column tiles, the second ragged);
    a column's result is bitwise the same alone and inside the batch."""
    import torch

    smg = smg_mod()
    lx, lt, blocks, nvs, m = 64, 64, [(2, 2)], [5], 0.1
    U = field(lx, lt, seed=61)
    vecs, calib = hierarchy_inputs(lx, lt, blocks, nvs, 63)
    A = normal_matrix(U, m)
    h = mg.hierarchy_from_vectors(A, (lx, lt, 2), blocks, vecs, calib, nu=4, omega=0.8, sa_scale=4 / 3)
    p = smg.make_params(lx, lt, m, levels=2, blocks=blocks, nv=nvs, operator_storage=opst, coarsest_fp64=c64)
    s = smg.Solver(dev(U), p, vectors=dev(np.concatenate([v.ravel() for v in vecs])), calib=dev(np.concatenate(calib)))
    try:
        assert s.level_size(1) == 5120
        n = s.level_size(0)
        b = synth.gaussian((33, n), 67).astype(np.complex64)
        xa = host(s.vcycle_f32(torch.from_numpy(b[:1].copy()).to("cuda"))).reshape(1, -1)
        xb = host(s.vcycle_f32(torch.from_numpy(b).to("cuda"))).reshape(33, -1)
        assert np.array_equal(xa[0], xb[0])
        bound = 1e-4 if opst == 0 else 1e-3
        for j in (0, 17, 32):
            ref = mg.vcycle(h, 0, b[j].astype(np.complex128))
            assert rel_err(xb[j], ref) <= bound, (j, rel_err(xb[j], ref))
    finally:
        s.close()


def test_fp64_vcycle_large_coarsest_matrix_cores():
    """FP64 V-cycle whose 5120-variable coarsest inverse is applied on the FP64
    matrix cores (n above the row-kernel limit): within 1e-11 of the oracle's
    V-cycle for 1, 16 and 33 right-hand sides (two column tiles, the second ragged).
    A column's result is bitwise the same in a call of 16 and of 33 columns (both at
    or above mfma_min_rhs, so the transfers also run on the matrix cores; below it
    they take the vector-ALU kernels, which round differently)."""
    import torch

    smg = smg_mod()
    lx, lt, blocks, nvs, m = 64, 64, [(2, 2)], [5], 0.1
    U = field(lx, lt, seed=61)
    vecs, calib = hierarchy_inputs(lx, lt, blocks, nvs, 63)
    A = normal_matrix(U, m)
    h = mg.hierarchy_from_vectors(A, (lx, lt, 2), blocks, vecs, calib, nu=4, omega=0.8, sa_scale=4 / 3)
    p = smg.make_params(lx, lt, m, levels=2, blocks=blocks, nv=nvs)
    s = smg.Solver(dev(U), p, vectors=dev(np.concatenate([v.ravel() for v in vecs])), calib=dev(np.concatenate(calib)))
    try:
        assert s.level_size(1) == 5120
        n = s.level_size(0)
        b = synth.gaussian((33, n), 68)
        x1 = host(s.vcycle(torch.from_numpy(b[:1].copy()).to("cuda"))).reshape(1, -1)
        xa = host(s.vcycle(torch.from_numpy(b[:16].copy()).to("cuda"))).reshape(16, -1)
        xb = host(s.vcycle(torch.from_numpy(b).to("cuda"))).reshape(33, -1)
        assert np.array_equal(xa[0], xb[0]) and np.array_equal(xa[15], xb[15])
        assert rel_err(x1[0], mg.vcycle(h, 0, b[0])) <= 1e-11
        for j in (0, 17, 32):
            ref = mg.vcycle(h, 0, b[j])
            assert rel_err(xb[j], ref) <= 1e-11, (j, rel_err(xb[j], ref))
    finally:
        s.close()
