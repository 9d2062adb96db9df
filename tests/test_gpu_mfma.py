"""GPU: the matrix-core coarse operators (MFMA FP32 and FP64) against the FP64 oracle.

The coarse operator of Eq. 2 applied to many right-hand sides runs on
v_mfma_f32_32x32x2f32 for levels with nc <= 16.  Each mode (plain apply, one
frozen MR smoother step, residual, first smoother step from a zero iterate) is compared with the oracle's sparse coarse
matrix in FP64 on the same FP32-rounded inputs, and with the vector-ALU path.
Inputs and links are rounded to FP32 (unit roundoff 6e-8) and an output sums at
most 9 * 16 complex products, so 2e-5 of the column's largest entry bounds the
difference with a wide margin.  Cases cover nc = 16, 12 and an odd nc = 5, tiles
cut by the lattice edge (coarse extents not multiples of the tile), both tile
shapes (2x2 on small coarse lattices, 4x4 from 64x64 sites), and right-hand-side
counts that are not multiples of 32.  The FP64 operator of many right-hand sides
runs on v_mfma_f64_16x16x4f64; its modes are held to 1e-12 of the column's largest
entry (FP64 inputs and links, the same sums).
"""

import numpy as np
import pytest

import synth
from oracle import multigrid as mg
from oracle.wilson import normal_matrix

pytestmark = pytest.mark.gpu

TOL32 = 2e-5
TOL16 = 2e-3  # FP16 unit roundoff 2^-11 per link entry, times 4 for cancellation in sums of random terms

CASES = [
    # lx, lt, blocks, nvs, mass
    (32, 32, [(4, 4), (2, 2)], [16, 16], 0.05),   # levels 8x8x16 and 4x4x16
    (40, 24, [(4, 4)], [12], 0.1),                # 10x6x12: tiles cut at both edges
    (20, 20, [(4, 4)], [5], 0.2),                 # 5x5x5: odd nc
    (24, 24, [(4, 4)], [16], 0.03),               # 6x6x16: tiles cut at both edges
    (16, 16, [(4, 4), (2, 2)], [8, 16], 0.1),     # 2x2x16: the ring wraps more than once
    (256, 256, [(4, 4), (4, 4)], [16, 4], 0.05),  # 64x64x16: the 4x4-tile path (>= 256 tiles)
]


def dev(x, dtype=np.complex128):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def colerr(a, b):
    """Largest per-column max-norm difference relative to the column's max |b|."""
    a = a.reshape(b.shape)
    return max(float(np.max(np.abs(a[j] - b[j])) / np.max(np.abs(b[j]))) for j in range(b.shape[0]))


@pytest.fixture(scope="module", params=range(len(CASES)))
def hier(request):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0710_3612_amd as smg

    lx, lt, blocks, nvs, m = CASES[request.param]
    U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 20, 70 + request.param))
    shapes = synth.level_shapes(lx, lt, blocks, nvs)
    vecs, calib = [], []
    for l, nv in enumerate(nvs):
        cx, ct, dof = shapes[l]
        n = cx * ct * dof
        vecs.append(synth.gaussian((nv, n), 900 + 10 * request.param + l))
        calib.append(synth.gaussian(n, 950 + 10 * request.param + l))
    A = normal_matrix(U, m)
    h = mg.hierarchy_from_vectors(A, (lx, lt, 2), blocks, vecs, calib, nu=4, omega=0.8, sa_scale=4 / 3)
    vv = dev(np.concatenate([v.ravel() for v in vecs]))
    cc = dev(np.concatenate(calib))
    out = {}
    for name, mmin in (("mfma", 1), ("valu", 0)):
        p = smg.make_params(lx, lt, m, levels=len(blocks) + 1, blocks=blocks, nv=nvs, mfma_min_rhs=mmin)
        out[name] = smg.Solver(dev(U), p, vectors=vv, calib=cc)
    p = smg.make_params(lx, lt, m, levels=len(blocks) + 1, blocks=blocks, nv=nvs, mfma_min_rhs=0,
                        operator_storage=smg.STORE_F16)
    out["h16"] = smg.Solver(dev(U), p, vectors=vv, calib=cc)
    p = smg.make_params(lx, lt, m, levels=len(blocks) + 1, blocks=blocks, nv=nvs, mfma_min_rhs=1,
                        operator_storage=smg.STORE_F16)
    out["mfma16"] = smg.Solver(dev(U), p, vectors=vv, calib=cc)
    yield dict(h=h, A=A, U=U, m=m, nlev=len(blocks) + 1, **out)
    for s in out.values():
        s.close()


@pytest.mark.parametrize("nrhs", [32, 45, 1])
def test_mfma_coarse_modes(hier, nrhs):
    import torch

    for level in range(1, hier["nlev"]):
        Ac = hier["h"].levels[level].A
        n = Ac.shape[0]
        rng = np.random.default_rng(level * 100 + nrhs)
        x = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
        aux = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
        acc0 = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
        coef = 0.37
        x64 = x.astype(np.complex128)
        Ax = np.stack([Ac @ x64[j] for j in range(nrhs)])
        got = {}
        for name in ("mfma", "valu"):
            s = hier[name]
            xt = dev(x, np.complex64)
            y0 = host(s.level_op_f32(level, xt, mode=0)).reshape(nrhs, n)
            xacc = dev(acc0, np.complex64)
            y1 = host(s.level_op_f32(level, xt, mode=1, coef=coef, xacc=xacc)).reshape(nrhs, n)
            a1 = host(xacc).reshape(nrhs, n)
            y2 = host(s.level_op_f32(level, xt, mode=2, aux=dev(aux, np.complex64))).reshape(nrhs, n)
            xacc3 = dev(acc0, np.complex64)
            y3 = host(s.level_op_f32(level, xt, mode=3, coef=coef, xacc=xacc3)).reshape(nrhs, n)
            a3 = host(xacc3).reshape(nrhs, n)
            torch.cuda.synchronize()
            assert colerr(y0, Ax) <= TOL32, (name, level, "mode 0")
            assert colerr(y1, x64 - coef * Ax) <= TOL32, (name, level, "mode 1")
            assert colerr(a1, acc0.astype(np.complex128) + coef * x64) <= TOL32, (name, level, "mode 1 acc")
            assert colerr(y2, aux.astype(np.complex128) - Ax) <= TOL32, (name, level, "mode 2")
            assert colerr(y3, x64 - coef * Ax) <= TOL32, (name, level, "mode 3")
            assert colerr(a3, coef * x64) <= TOL32, (name, level, "mode 3 acc")
            got[name] = y0
        assert colerr(got["mfma"], got["valu"].astype(np.complex128)) <= TOL32


def test_mfma_mixed_solve_many_rhs(hier):
    """Mixed-precision MG-CG of 40 right-hand sides with the matrix-core coarse
    operator: every column reaches 1e-10 against the oracle's A, and the solution
    agrees with the vector-ALU path to the accuracy both reached."""
    import paper_0710_3612_amd as smg

    A = hier["A"]
    n = A.shape[0]
    B = synth.gaussian((40, n), 4242)
    xs = {}
    for name in ("mfma", "valu"):
        x, st, code = hier[name].solve(dev(B), tol=1e-10, maxiter=500, precision=smg.MIXED)
        assert code == 0
        xh = host(x).reshape(40, n)
        for j in range(0, 40, 7):
            assert np.linalg.norm(B[j] - A @ xh[j]) / np.linalg.norm(B[j]) <= 1e-10
        xs[name] = xh
    d = np.linalg.norm(xs["mfma"] - xs["valu"], axis=1) / np.linalg.norm(xs["valu"], axis=1)
    assert d.max() < 1e-6


@pytest.mark.parametrize("nrhs", [1, 5])
def test_fp16_link_coarse_modes(hier, nrhs):
    """Vector-ALU coarse operator with FP16 links (scaled by a power of two): every
    mode within TOL16 of the oracle's FP64 operator."""
    import torch

    for level in range(1, hier["nlev"]):
        Ac = hier["h"].levels[level].A
        n = Ac.shape[0]
        rng = np.random.default_rng(level * 1000 + nrhs)
        x = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
        aux = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
        acc0 = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
        coef = 0.37
        x64 = x.astype(np.complex128)
        Ax = np.stack([Ac @ x64[j] for j in range(nrhs)])
        s = hier["h16"]
        xt = dev(x, np.complex64)
        y0 = host(s.level_op_f32(level, xt, mode=0)).reshape(nrhs, n)
        xacc = dev(acc0, np.complex64)
        y1 = host(s.level_op_f32(level, xt, mode=1, coef=coef, xacc=xacc)).reshape(nrhs, n)
        a1 = host(xacc).reshape(nrhs, n)
        y2 = host(s.level_op_f32(level, xt, mode=2, aux=dev(aux, np.complex64))).reshape(nrhs, n)
        torch.cuda.synchronize()
        print("fp16 links level", level, "mode 0 error", colerr(y0, Ax))
        assert colerr(y0, Ax) <= TOL16, (level, "mode 0")
        assert colerr(y1, x64 - coef * Ax) <= TOL16, (level, "mode 1")
        assert colerr(a1, acc0.astype(np.complex128) + coef * x64) <= TOL32, (level, "mode 1 acc")
        assert colerr(y2, aux.astype(np.complex128) - Ax) <= TOL16, (level, "mode 2")


@pytest.mark.parametrize("nrhs", [32, 45])
def test_fp16_link_mfma_coarse_modes(hier, nrhs):
    """Matrix-core coarse operator reading the FP16 links (scaled by a power of two,
    FP32 arithmetic): every mode within TOL16 of the oracle's FP64 operator, and
    within TOL32 of the vector-ALU kernel that reads the same FP16 links (so a wrong
    scale, layout or column pairing of the FP16 stream cannot hide in TOL16)."""
    import torch

    for level in range(1, hier["nlev"]):
        Ac = hier["h"].levels[level].A
        n = Ac.shape[0]
        rng = np.random.default_rng(level * 2000 + nrhs)
        x = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
        aux = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
        acc0 = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
        coef = 0.37
        x64 = x.astype(np.complex128)
        Ax = np.stack([Ac @ x64[j] for j in range(nrhs)])
        s = hier["mfma16"]
        xt = dev(x, np.complex64)
        y0 = host(s.level_op_f32(level, xt, mode=0)).reshape(nrhs, n)
        xacc = dev(acc0, np.complex64)
        y1 = host(s.level_op_f32(level, xt, mode=1, coef=coef, xacc=xacc)).reshape(nrhs, n)
        a1 = host(xacc).reshape(nrhs, n)
        y2 = host(s.level_op_f32(level, xt, mode=2, aux=dev(aux, np.complex64))).reshape(nrhs, n)
        xacc3 = dev(acc0, np.complex64)
        y3 = host(s.level_op_f32(level, xt, mode=3, coef=coef, xacc=xacc3)).reshape(nrhs, n)
        a3 = host(xacc3).reshape(nrhs, n)
        v0 = host(hier["h16"].level_op_f32(level, xt, mode=0)).reshape(nrhs, n)
        torch.cuda.synchronize()
        assert colerr(y0, Ax) <= TOL16, (level, "mode 0")
        assert colerr(y1, x64 - coef * Ax) <= TOL16, (level, "mode 1")
        assert colerr(a1, acc0.astype(np.complex128) + coef * x64) <= TOL32, (level, "mode 1 acc")
        assert colerr(y2, aux.astype(np.complex128) - Ax) <= TOL16, (level, "mode 2")
        assert colerr(y3, x64 - coef * Ax) <= TOL16, (level, "mode 3")
        assert colerr(a3, coef * x64) <= TOL32, (level, "mode 3 acc")
        assert colerr(y0, v0.astype(np.complex128)) <= TOL32, (level, "against the vector-ALU FP16 kernel")


TOL64 = 1e-12  # FP64 inputs and links; sums of at most 9 * 16 complex products


@pytest.mark.parametrize("nrhs", [16, 33, 64, 70, 1])
def test_mfma64_coarse_modes(hier, nrhs):
    """FP64 coarse operator on the matrix cores (v_mfma_f64_16x16x4f64, 16, 32 or
    64 right-hand sides per wave) against the oracle's sparse coarse matrix for
    every mode, and against the vector-ALU FP64 kernel; counts that are not
    multiples of 16 leave masked columns in the last wave."""
    import torch

    for level in range(1, hier["nlev"]):
        Ac = hier["h"].levels[level].A
        n = Ac.shape[0]
        rng = np.random.default_rng(level * 300 + nrhs)
        x = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
        aux = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
        acc0 = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
        coef = 0.37
        Ax = np.stack([Ac @ x[j] for j in range(nrhs)])
        got = {}
        for name in ("mfma", "valu"):
            s = hier[name]
            xt = dev(x)
            y0 = host(s.level_op(level, xt, mode=0)).reshape(nrhs, n)
            xacc = dev(acc0)
            y1 = host(s.level_op(level, xt, mode=1, coef=coef, xacc=xacc)).reshape(nrhs, n)
            a1 = host(xacc).reshape(nrhs, n)
            y2 = host(s.level_op(level, xt, mode=2, aux=dev(aux))).reshape(nrhs, n)
            xacc3 = dev(acc0)
            y3 = host(s.level_op(level, xt, mode=3, coef=coef, xacc=xacc3)).reshape(nrhs, n)
            a3 = host(xacc3).reshape(nrhs, n)
            torch.cuda.synchronize()
            assert colerr(y0, Ax) <= TOL64, (name, level, "mode 0")
            assert colerr(y1, x - coef * Ax) <= TOL64, (name, level, "mode 1")
            assert colerr(a1, acc0 + coef * x) <= TOL64, (name, level, "mode 1 acc")
            assert colerr(y2, aux - Ax) <= TOL64, (name, level, "mode 2")
            assert colerr(y3, x - coef * Ax) <= TOL64, (name, level, "mode 3")
            assert colerr(a3, coef * x) <= TOL64, (name, level, "mode 3 acc")
            got[name] = y0
        assert colerr(got["mfma"], got["valu"]) <= TOL64


def test_mfma64_fp64_solve_many_rhs(hier):
    """FP64 MG-CG of 40 right-hand sides whose coarse levels run on the FP64 matrix
    cores: every sampled column reaches 1e-10 against the oracle's A, and the
    solutions agree with the vector-ALU path to the accuracy both reached."""
    import paper_0710_3612_amd as smg

    A = hier["A"]
    n = A.shape[0]
    B = synth.gaussian((40, n), 4343)
    xs = {}
    for name in ("mfma", "valu"):
        x, st, code = hier[name].solve(dev(B), tol=1e-10, maxiter=500, precision=smg.FP64)
        assert code == 0
        xh = host(x).reshape(40, n)
        for j in range(0, 40, 7):
            assert np.linalg.norm(B[j] - A @ xh[j]) / np.linalg.norm(B[j]) <= 1e-10
        xs[name] = xh
    d = np.linalg.norm(xs["mfma"] - xs["valu"], axis=1) / np.linalg.norm(xs["valu"], axis=1)
    assert d.max() < 1e-6


TW_CASES = [
    # lx, lt, blocks, nvs, mass: level 1 large enough for the strip-walking kernel
    (512, 256, [(4, 4)], [16], 0.05),  # 128x64x16: 32 strips, segments of 8 rows
    (520, 264, [(4, 4)], [16], 0.05),  # 130x66x16: a last strip of 2 columns, segments of 10 rows, the last of 6
]


@pytest.mark.parametrize("case", range(len(TW_CASES)))
def test_strip_walking_mfma_coarse_modes(case):
    """The strip-walking matrix-core kernel (coarse lattices with at least 8 rows per
    workgroup, rows of V staged under the MFMAs of the rows before) in every mode, on
    FP32 and on FP16 links, against the oracle's Galerkin operator, and against the
    vector-ALU kernels on the same links; 32 and 40 right-hand sides (a partial
    second block of columns)."""
    import torch

    import paper_0710_3612_amd as smg

    lx, lt, blocks, nvs, m = TW_CASES[case]
    U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 5, 170 + case))
    shapes = synth.level_shapes(lx, lt, blocks, nvs)
    n0 = shapes[0][0] * shapes[0][1] * shapes[0][2]
    vecs = synth.gaussian((nvs[0], n0), 1900 + case)
    calib = synth.gaussian(n0, 1950 + case)
    A = normal_matrix(U, m)
    h = mg.hierarchy_from_vectors(A, (lx, lt, 2), blocks, [vecs], [calib], nu=4, omega=0.8, sa_scale=4 / 3,
                                  coarsest="cg")
    Ac = h.levels[1].A
    n = Ac.shape[0]
    sol = {}
    try:
        for name, mmin, store in (("tw", 1, smg.STORE_F32), ("tw16", 1, smg.STORE_F16), ("valu", 0, smg.STORE_F32),
                                  ("valu16", 0, smg.STORE_F16)):
            p = smg.make_params(lx, lt, m, levels=2, blocks=blocks, nv=nvs, mfma_min_rhs=mmin, operator_storage=store,
                                coarsest=smg.COARSEST_CG)
            sol[name] = smg.Solver(dev(U), p, vectors=dev(vecs.ravel()), calib=dev(calib))
        for nrhs in (32, 40):
            rng = np.random.default_rng(7000 + 10 * case + nrhs)
            x = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
            aux = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
            acc0 = (rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))).astype(np.complex64)
            coef = 0.37
            x64 = x.astype(np.complex128)
            Ax = (Ac @ x64.T).T
            y0 = {}
            for name in sol:
                y0[name] = host(sol[name].level_op_f32(1, dev(x, np.complex64), mode=0)).reshape(nrhs, n)
            for name, tol in (("tw", TOL32), ("tw16", TOL16)):
                s = sol[name]
                xt = dev(x, np.complex64)
                xacc = dev(acc0, np.complex64)
                y1 = host(s.level_op_f32(1, xt, mode=1, coef=coef, xacc=xacc)).reshape(nrhs, n)
                a1 = host(xacc).reshape(nrhs, n)
                y2 = host(s.level_op_f32(1, xt, mode=2, aux=dev(aux, np.complex64))).reshape(nrhs, n)
                xacc3 = dev(acc0, np.complex64)
                y3 = host(s.level_op_f32(1, xt, mode=3, coef=coef, xacc=xacc3)).reshape(nrhs, n)
                a3 = host(xacc3).reshape(nrhs, n)
                torch.cuda.synchronize()
                assert colerr(y0[name], Ax) <= tol, (name, nrhs, "mode 0")
                assert colerr(y1, x64 - coef * Ax) <= tol, (name, nrhs, "mode 1")
                assert colerr(a1, acc0.astype(np.complex128) + coef * x64) <= TOL32, (name, nrhs, "mode 1 acc")
                assert colerr(y2, aux.astype(np.complex128) - Ax) <= tol, (name, nrhs, "mode 2")
                assert colerr(y3, x64 - coef * Ax) <= tol, (name, nrhs, "mode 3")
                assert colerr(a3, coef * x64) <= TOL32, (name, nrhs, "mode 3 acc")
            assert colerr(y0["tw"], y0["valu"].astype(np.complex128)) <= TOL32, nrhs
            assert colerr(y0["tw16"], y0["valu16"].astype(np.complex128)) <= TOL32, nrhs
    finally:
        for s in sol.values():
            s.close()
