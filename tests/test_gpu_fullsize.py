"""GPU parity on the kernel paths that only large lattices and the benchmark's
hierarchy shapes reach, against the FP64 oracle.

* The fused A = D^H D kernel picks its tile by lattice size: 64x8 (non-temporal
  stores), 32x16 (non-temporal), 64x4 or 32x8 once the lattice holds at least 256
  (FP64) or 1024 (FP32) tiles of 512 sites, 16x16 below.  Every large-tile shape
  is compared here in both precisions, with every epilogue the V-cycle and the
  mixed solve use on it (MR steps from zero and accumulating, residual, last two
  steps, the fused CG step and the V-cycle end).
* The headline hierarchy shape (256^2, 4x4 blocks twice, Nv = 12, smoothed
  aggregation) runs the FP32 restriction kernels for 16-column windows of <= 128
  and of 432 variables, the nc = 12 prolongation, the 3072-variable coarsest
  inverse, and the matrix-core coarse operator at >= 16 right-hand sides.
* Mixed solves must not hide a weak FP32 preconditioner behind the FP64 defect
  correction: their iteration counts are bounded by the FP64 ones.
* The paper's experiment setting (nu = 2, M = 8, 3 levels down to an exact 8^2).

Tolerances: FP64 applies 1e-12 (max-norm relative), FP64 smoother and V-cycle
1e-11, FP32 operators 2e-5, FP32 V-cycles 1e-4 with FP32 storage, 1e-3 with FP16
operator storage, the smoother-storage bounds of test_gpu_lowprec.
"""

import json
import os

import numpy as np
import pytest

import synth
from oracle import multigrid as mg
from oracle.wilson import dirac_matrix, normal_matrix

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def dev32(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex64)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def field(lx, lt, seed, beta=3.0, sweeps=2):
    return synth.links_from_angles(synth.metropolis_u1(lx, lt, beta, sweeps, seed))


def smg_mod():
    import paper_0710_3612_amd as smg

    return smg


def vectors_for(lx, lt, blocks, nvs, seed):
    shapes = synth.level_shapes(lx, lt, blocks, nvs)
    vecs = [synth.gaussian((nv, shapes[l][0] * shapes[l][1] * shapes[l][2]), seed * 100 + l)
            for l, nv in enumerate(nvs)]
    calib = [synth.gaussian(shapes[l][0] * shapes[l][1] * shapes[l][2], seed * 100 + 50 + l) for l in range(len(nvs))]
    return vecs, calib


def build_pair(U, lx, lt, m, blocks, nvs, seed, nu=4, **kw):
    smg = smg_mod()
    vecs, calib = vectors_for(lx, lt, blocks, nvs, seed)
    A = normal_matrix(U, m)
    h = mg.hierarchy_from_vectors(A, (lx, lt, 2), blocks, vecs, calib, nu=nu, omega=0.8, sa_scale=4 / 3)
    p = smg.make_params(lx, lt, m, levels=len(blocks) + 1, blocks=blocks, nv=nvs, smoother_steps=nu, **kw)
    s = smg.Solver(dev(U), p, vectors=dev(np.concatenate([v.ravel() for v in vecs])),
                   calib=dev(np.concatenate(calib)))
    return A, h, s


# ---------------------------------------------------------------------------
# FP64 large tiles: >= 131072 sites
# ---------------------------------------------------------------------------

FP64_TILES = [
    # lx, lt, the tile the size selects, blocks with a small coarsest level
    (512, 256, "64x8 non-temporal", [(8, 8), (4, 4)]),
    (160, 832, "32x16 non-temporal", [(8, 8), (4, 4)]),
    (512, 260, "64x4", [(4, 4), (4, 5)]),
    (480, 280, "32x8", [(8, 8), (4, 5)]),
]


@pytest.mark.parametrize("lx,lt,tile,blocks", FP64_TILES, ids=[t[2] for t in FP64_TILES])
def test_fp64_large_tiles(cuda, lx, lt, tile, blocks):
    """D, D^H, A (2 right-hand sides), the nu = 4 and nu = 2 smoothers (first step
    from zero, accumulating steps, the last two steps fused, both steps of nu = 2
    fused) and the FP64 V-cycle (residual epilogue) on the large-tile fine kernel."""
    assert lx * lt >= 256 * 512
    m = 0.08
    U = field(lx, lt, seed=lx + 7 * lt)
    nvs = [3, 3]
    A, h, s = build_pair(U, lx, lt, m, blocks, nvs, seed=5)
    try:
        n = 2 * lx * lt
        D = dirac_matrix(U, m)
        x = synth.gaussian((2, n), 71)
        yd = host(s.apply_D(dev(x))).reshape(2, -1)
        yh = host(s.apply_D(dev(x), dagger=True)).reshape(2, -1)
        ya = host(s.apply_A(dev(x))).reshape(2, -1)
        for j in range(2):
            assert rel_err(yd[j], D @ x[j]) <= 1e-12
            assert rel_err(yh[j], D.conj().T @ x[j]) <= 1e-12
            assert rel_err(ya[j], A @ x[j]) <= 1e-12
        np.testing.assert_allclose(s.smoother_coefs(0), h.levels[0].coefs, rtol=1e-12)
        rb = host(s.smooth(0, dev(x))).reshape(2, -1)
        vb = host(s.vcycle(dev(x))).reshape(2, -1)
        for j in range(2):
            assert rel_err(rb[j], mg.smoother_apply(A, h.levels[0].coefs, x[j])) <= 1e-11
            assert rel_err(vb[j], mg.vcycle(h, 0, x[j])) <= 1e-11
    finally:
        s.close()
    # nu = 2: both steps from zero in one launch
    A2, h2, s2 = build_pair(U, lx, lt, m, blocks, nvs, seed=6, nu=2)
    try:
        x = synth.gaussian(2 * lx * lt, 72)
        assert rel_err(host(s2.smooth(0, dev(x))), mg.smoother_apply(A2, h2.levels[0].coefs, x)) <= 1e-11
        assert rel_err(host(s2.vcycle(dev(x))), mg.vcycle(h2, 0, x)) <= 1e-11
    finally:
        s2.close()


def test_fp64_large_tile_mgcg_solve(cuda):
    """FP64 MG-CG on the 64x8 tile (every fine apply of the solve on it): the true
    residual, recomputed by the oracle's A, reaches 1e-10, and the iteration count
    equals the oracle's MG-CG on the same hierarchy within one."""
    smg = smg_mod()
    lx, lt, m = 512, 256, 0.06
    U = field(lx, lt, seed=91, sweeps=5)
    A, h, s = build_pair(U, lx, lt, m, [(8, 8), (4, 4)], [3, 3], seed=9)
    try:
        b = synth.gaussian(2 * lx * lt, 92)
        rhs = dirac_matrix(U, m).conj().T @ b
        x, st, code = s.solve(dev(rhs), tol=1e-10, maxiter=1000, precision=smg.FP64)
        assert code == 0
        res = np.linalg.norm(rhs - A @ host(x)) / np.linalg.norm(rhs)
        assert res <= 1e-10
        _, info = mg.mg_cg(h, rhs, 1e-10)
        assert abs(st[0]["iterations"] - info.iterations) <= 1, (st[0]["iterations"], info.iterations)
    finally:
        s.close()


# ---------------------------------------------------------------------------
# FP32 large tiles: >= 524288 sites
# ---------------------------------------------------------------------------

FP32_TILES = [
    (1024, 512, "64x8 non-temporal"),
    (992, 544, "32x16 non-temporal"),
    (1024, 516, "64x4"),
    (992, 536, "32x8"),
]


@pytest.mark.parametrize("lx,lt,tile", FP32_TILES, ids=[t[2] for t in FP32_TILES])
def test_fp32_large_tiles_epilogues(cuda, lx, lt, tile):
    """The FP32 fine operator with the epilogues of smg_level_op_f32 (plain, one MR
    step, residual, first MR step) on each large FP32 tile, element by element
    against the oracle's A in FP64: inputs rounded to FP32, each output a sum of
    at most 13 products per spin, so 2e-5 of the output max-norm bounds it."""
    import torch

    smg = smg_mod()
    assert lx * lt >= 1024 * 512
    m = 0.08
    U = field(lx, lt, seed=lx + 3 * lt)
    A = normal_matrix(U, m)
    p = smg.make_params(lx, lt, m, levels=1)
    with smg.Solver(dev(U), p) as s:
        n = 2 * lx * lt
        x = synth.gaussian(n, 81).astype(np.complex64)
        aux = synth.gaussian(n, 82).astype(np.complex64)
        acc0 = synth.gaussian(n, 83).astype(np.complex64)
        xd = x.astype(np.complex128)
        Ax = A @ xd
        c = 0.37
        # mode 0: y = A x
        y = host(s.level_op_f32(0, dev32(x), mode=0)).astype(np.complex128)
        assert rel_err(y, Ax) <= 2e-5
        # mode 1: xacc += c x, y = x - c A x
        acc = dev32(acc0)
        y = host(s.level_op_f32(0, dev32(x), mode=1, coef=c, xacc=acc)).astype(np.complex128)
        assert rel_err(y, xd - c * Ax) <= 2e-5
        assert rel_err(host(acc).astype(np.complex128), acc0.astype(np.complex128) + c * xd) <= 2e-6
        # mode 2: y = aux - A x
        y = host(s.level_op_f32(0, dev32(x), mode=2, aux=dev32(aux))).astype(np.complex128)
        assert rel_err(y, aux.astype(np.complex128) - Ax) <= 2e-5
        # mode 3: xacc = c x, y = x - c A x
        acc = dev32(acc0)
        y = host(s.level_op_f32(0, dev32(x), mode=3, coef=c, xacc=acc)).astype(np.complex128)
        assert rel_err(y, xd - c * Ax) <= 2e-5
        assert rel_err(host(acc).astype(np.complex128), c * xd) <= 2e-6
        torch.cuda.synchronize()


def test_fp32_large_tile_vcycle_and_mixed_solve(cuda):
    """1024 x 512 (the FP32 64x8 tile): the FP32 V-cycle against the oracle's
    V-cycle within 1e-4 (fine MR steps from zero and accumulating, residual, last
    two steps fused), and mixed MG-CG, whose FP32 outer CG takes every step in the
    fused CG-step kernel and ends each V-cycle in the V-cycle-end kernel on that
    tile: true residual <= 1e-10 by the oracle's A, iterations bounded by FP64's."""
    smg = smg_mod()
    lx, lt, m = 1024, 512, 0.08
    U = field(lx, lt, seed=101)
    A, h, s = build_pair(U, lx, lt, m, [(8, 8), (4, 4)], [4, 4], seed=10)
    try:
        n = 2 * lx * lt
        b = synth.gaussian((2, n), 102)
        x32 = host(s.vcycle_f32(dev32(b))).reshape(2, -1)
        for j in range(2):
            assert rel_err(x32[j], mg.vcycle(h, 0, b[j])) <= 1e-4
        rhs = dirac_matrix(U, m).conj().T @ b[0]
        its = {}
        for prec in (smg.FP64, smg.MIXED):
            x, st, code = s.solve(dev(rhs), tol=1e-10, maxiter=1000, precision=prec)
            assert code == 0
            assert np.linalg.norm(rhs - A @ host(x)) / np.linalg.norm(rhs) <= 1e-10
            its[prec] = st[0]["iterations"]
        assert its[smg.MIXED] <= its[smg.FP64] + max(2, its[smg.FP64] // 4), its
    finally:
        s.close()


# ---------------------------------------------------------------------------
# The headline hierarchy shape: 256^2, 4x4 blocks twice, Nv = 12
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def headline():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L, m = 256, 0.07
    U = synth.links_from_angles(synth.metropolis_u1(L, L, 6.0, 30, 2000))
    blocks, nvs = [(4, 4), (4, 4)], [12, 12]
    vecs, calib = vectors_for(L, L, blocks, nvs, 21)
    A = normal_matrix(U, m)
    h = mg.hierarchy_from_vectors(A, (L, L, 2), blocks, vecs, calib, nu=4, omega=0.8, sa_scale=4 / 3)
    b = synth.gaussian((17, 2 * L * L), 23).astype(np.complex64)
    refs = {j: mg.vcycle(h, 0, b[j].astype(np.complex128)) for j in (0, 8, 16)}
    return dict(L=L, m=m, U=U, blocks=blocks, nvs=nvs, vecs=vecs, calib=calib, A=A, h=h, b=b, refs=refs)


HEADLINE_VARIANTS = [
    # operator storage, FP64 coarsest apply, smoother storage, bound
    (0, True, 0, 1e-4),
    (0, False, 0, 1e-4),
    (2, True, 0, 1e-3),
    (2, False, 0, 1e-3),
    (2, True, 1, 5e-2),
    (2, False, 2, 6e-3),
]


@pytest.mark.parametrize("opst,c64,smst,bound", HEADLINE_VARIANTS)
def test_headline_shape_fp32_vcycle(headline, opst, c64, smst, bound):
    """FP32 V-cycle of the headline hierarchy (nc = 12 on both coarse levels, 3072-
    variable coarsest inverse) against the oracle's FP64 V-cycle, for 1, 9 and 17
    right-hand sides (17 takes the matrix-core coarse operator); the first column is
    the same alone and in every batch, and columns 8 and 16 meet the bound too."""
    smg = smg_mod()
    H = headline
    L = H["L"]
    p = smg.make_params(L, L, H["m"], levels=3, blocks=H["blocks"], nv=H["nvs"], operator_storage=opst,
                        coarsest_fp64=c64, smoother_storage=smst)
    s = smg.Solver(dev(H["U"]), p, vectors=dev(np.concatenate([v.ravel() for v in H["vecs"]])),
                   calib=dev(np.concatenate(H["calib"])))
    try:
        assert s.level_info(1) == (64, 64, 12) and s.level_info(2) == (16, 16, 12)
        b = H["b"]
        x1 = host(s.vcycle_f32(dev32(b[:1]))).reshape(1, -1)
        x9 = host(s.vcycle_f32(dev32(b[:9]))).reshape(9, -1)
        x17 = host(s.vcycle_f32(dev32(b))).reshape(17, -1)
        assert rel_err(x1[0], H["refs"][0]) <= bound, rel_err(x1[0], H["refs"][0])
        assert np.array_equal(x1[0], x9[0])
        assert rel_err(x9[8], H["refs"][8]) <= bound
        assert rel_err(x17[0], H["refs"][0]) <= bound
        assert rel_err(x17[16], H["refs"][16]) <= bound
    finally:
        s.close()


def test_headline_shape_mixed_iterations_bounded_by_fp64(cuda):
    """Adaptive setup on the headline shape (256^2 beta = 6, Nv = 12 twice, 5 setup
    iterations) at a light mass; mixed solves with every storage variant reach the
    oracle's 1e-10 and take at most FP64's iterations plus max(2, FP64 / 4), so a
    broken FP32 kernel cannot hide behind the FP64 defect correction."""
    smg = smg_mod()
    L, m = 256, 0.02
    U = synth.links_from_angles(synth.metropolis_u1(L, L, 6.0, 100, 2001))
    A = normal_matrix(U, m)
    rhs = dirac_matrix(U, m).conj().T @ synth.gaussian(2 * L * L, 24)
    R = synth.setup_randoms(L, L, [(4, 4), (4, 4)], [12, 12], 2001)
    rnd = dev(np.concatenate([r.ravel() for r in R]))
    its = {}
    for opst, c64, smst in ((0, True, 0), (2, True, 0), (2, False, 0), (2, False, 1)):
        p = smg.make_params(L, L, m, levels=3, blocks=[(4, 4), (4, 4)], nv=[12, 12], operator_storage=opst,
                            coarsest_fp64=c64, smoother_storage=smst)
        with smg.Solver(dev(U), p, randoms=rnd) as s:
            if not its:
                x, st, code = s.solve(dev(rhs), tol=1e-10, maxiter=500, precision=smg.FP64)
                assert code == 0
                assert np.linalg.norm(rhs - A @ host(x)) / np.linalg.norm(rhs) <= 1e-10
                its["fp64"] = st[0]["iterations"]
            x, st, code = s.solve(dev(rhs), tol=1e-10, maxiter=500, precision=smg.MIXED)
            assert code == 0
            assert np.linalg.norm(rhs - A @ host(x)) / np.linalg.norm(rhs) <= 1e-10
            its[(opst, c64, smst)] = st[0]["iterations"]
    f = its["fp64"]
    for k, v in its.items():
        assert v <= f + max(2, f // 4), its


# ---------------------------------------------------------------------------
# The paper's experiment setting
# ---------------------------------------------------------------------------

def test_paper_experiment_setting(cuda):
    """Results section: 128^2 beta = 6 (Q = 0 field), 4x4 blocks twice with M = 8
    down to an 8^2 lattice solved exactly, nu = 2 MR smoother with omega = 0.8,
    point source, at mass gap 0.01 above the field's m_crit.  The GPU's adaptive
    setup (same random starts as the oracle's, 5 setup iterations) and FP64 MG-CG
    to 1e-12: the same smoother, the per-aggregate projectors within 1e-7, the true
    residual by the oracle's A, and the iteration count within 10% of the oracle's."""
    smg = smg_mod()
    L = 128
    with open(os.path.join(ROOT, "workloads", "masses_128_beta6_cold.json")) as f:
        fld = json.load(f)["fields"][0]
    th = synth.metropolis_u1(L, L, 6.0, fld["sweeps"], fld["seed"], cold=True)
    assert synth.topological_charge(th) == pytest.approx(0.0, abs=1e-9)
    U = synth.links_from_angles(th)
    m = fld["m_star"] + 0.01
    blocks, nvs = [(4, 4), (4, 4)], [8, 8]
    R = synth.setup_randoms(L, L, blocks, nvs, 7)
    A = normal_matrix(U, m)
    h = mg.adaptive_setup(A, (L, L, 2), blocks, nvs, R, nu=2, omega=0.8, setup_iters=5, sa_scale=4 / 3)
    rhs = dirac_matrix(U, m).conj().T @ synth.point_source(L, L)
    _, io = mg.mg_cg(h, rhs, 1e-12)
    p = smg.make_params(L, L, m, levels=3, blocks=blocks, nv=nvs, setup_iters=5, smoother_steps=2)
    with smg.Solver(dev(U), p, randoms=dev(np.concatenate([r.ravel() for r in R]))) as s:
        assert s.level_info(2) == (8, 8, 8)
        np.testing.assert_allclose(s.smoother_coefs(0), h.levels[0].coefs, rtol=1e-12)
        Pg = host(s.prolongator(0))
        Po = h.levels[0].U
        proj_g = np.einsum("jki,jkl->jil", Pg, Pg.conj())
        proj_o = np.einsum("jki,jkl->jil", Po, Po.conj())
        assert np.max(np.abs(proj_g - proj_o)) <= 1e-7
        x, st, code = s.solve(dev(rhs), tol=1e-12, maxiter=5000, precision=smg.FP64)
        assert code == 0
        assert np.linalg.norm(rhs - A @ host(x)) / np.linalg.norm(rhs) <= 1e-12
        assert abs(st[0]["iterations"] - io.iterations) <= max(1, io.iterations // 10), (st[0], io.iterations)


# ---------------------------------------------------------------------------
# Several right-hand sides per workgroup (lattices of at least 2^20 sites)
# ---------------------------------------------------------------------------

def test_fused_rhs_groups_equal_single_columns(cuda):
    """On a 1024x1024 lattice a fused-A workgroup takes four right-hand sides in turn
    (the links loaded once for them). Every column of a 6-column call (a group of 4
    and a ragged group of 2) equals the same column applied alone, bit for bit, for
    the plain operator, the MR steps from zero and accumulating, the residual (FP64
    and FP32), and the fused smoother; one column of A x matches the oracle's D^H D."""
    import torch

    smg = smg_mod()
    lx = lt = 1024
    m = 0.07
    U = field(lx, lt, seed=1024)
    n = 2 * lx * lt
    vecs, calib = vectors_for(lx, lt, [(8, 8)], [2], 3)
    p = smg.make_params(lx, lt, m, levels=2, blocks=[(8, 8)], nv=[2], coarsest=smg.COARSEST_CG)
    s = smg.Solver(dev(U), p, vectors=dev(np.concatenate([v.ravel() for v in vecs])), calib=dev(np.concatenate(calib)))
    try:
        nr = 6
        x = synth.gaussian((nr, n), 1025)
        aux = synth.gaussian((nr, n), 1026)
        acc = synth.gaussian((nr, n), 1027)
        coef = 0.31

        def ops(level_op, conv, cols):
            xt = conv(x[cols])
            out = [host(level_op(0, xt, mode=0))]
            xa = conv(acc[cols])
            out.append(host(level_op(0, xt, mode=1, coef=coef, xacc=xa)))
            out.append(host(xa))
            out.append(host(level_op(0, xt, mode=2, aux=conv(aux[cols]))))
            xa3 = conv(acc[cols])
            out.append(host(level_op(0, xt, mode=3, coef=coef, xacc=xa3)))
            out.append(host(xa3))
            torch.cuda.synchronize()
            return [o.reshape(-1, n) for o in out]

        for level_op, conv in ((s.level_op, dev), (s.level_op_f32, dev32)):
            many = ops(level_op, conv, slice(0, nr))
            for j in range(nr):
                one = ops(level_op, conv, slice(j, j + 1))
                for a, b in zip(many, one):
                    assert np.array_equal(a[j], b[0]), j
        sm = host(s.smooth(0, dev(x))).reshape(nr, n)
        for j in (0, 5):
            assert np.array_equal(sm[j], host(s.smooth(0, dev(x[j:j + 1]))).reshape(n))
        D = dirac_matrix(U, m)
        assert rel_err(host(s.apply_A(dev(x))).reshape(nr, n)[5], D.conj().T @ (D @ x[5])) <= 1e-12
    finally:
        s.close()
