"""GPU: grouped solves (smg_group_*).  Several independent systems of one hierarchy
shape (different fields and masses) run as the columns of every launch of the
mixed-precision solve.  Each column's arithmetic is that of the system solved alone,
so the solutions, iteration counts and residuals must equal one-column smg_solve
calls on the same handles bit for bit, also after a re-mass of one handle; the
solutions reach 1e-10 against the oracle's A."""

import numpy as np
import pytest

import synth
from oracle.wilson import normal_matrix

pytestmark = pytest.mark.gpu


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


CASES = [
    # lx, lt, blocks, nv, operator_storage, coarsest_fp64
    (64, 64, [(4, 4), (4, 4)], [6, 6], 0, True),
    (128, 128, [(4, 4), (4, 4)], [12, 12], 2, False),   # the benchmark's hierarchy shape and storage
    (64, 32, [(4, 4), (2, 2)], [5, 8], 2, True),
]


@pytest.mark.parametrize("lx,lt,blocks,nv,opst,c64", CASES)
def test_group_equals_single_solves(cuda, lx, lt, blocks, nv, opst, c64):
    import paper_0710_3612_amd as smg

    n = 2 * lx * lt
    masses = [0.05, 0.12]
    solvers, systems = [], []
    for f in range(2):
        U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 10, 300 + f))
        p = smg.make_params(lx, lt, masses[0], levels=len(blocks) + 1, blocks=blocks, nv=nv, operator_storage=opst,
                            coarsest_fp64=c64, seed=7 + f)
        s0 = smg.Solver(dev(U), p)
        solvers.append(s0)
        systems.append((U, masses[0]))
        d = s0.derive(masses[1])
        solvers.append(d)
        systems.append((U, masses[1]))
    B = synth.gaussian((len(solvers), n), 4711)
    try:
        alone = [s.solve(dev(B[j:j + 1]), tol=1e-10, maxiter=400, precision=smg.MIXED) for j, s in enumerate(solvers)]
        with smg.Group(solvers) as g:
            X, st, code = g.solve(dev(B), tol=1e-10, maxiter=400)
            assert code == 0
            X = host(X)
            for j, (x1, st1, c1) in enumerate(alone):
                assert c1 == 0
                assert np.array_equal(X[j], host(x1)[0]), j
                assert st[j]["iterations"] == st1[0]["iterations"]
                assert st[j]["true_relres"] == st1[0]["true_relres"]
            U, m = systems[1]
            A = normal_matrix(U, m)
            assert np.linalg.norm(B[1] - A @ X[1]) / np.linalg.norm(B[1]) <= 1e-10
            # a re-mass of one handle reaches the group's tables
            solvers[2].set_mass(0.2)
            X2, st2, code = g.solve(dev(B), tol=1e-10, maxiter=400)
            assert code == 0
            x2, _, _ = solvers[2].solve(dev(B[2:3]), tol=1e-10, maxiter=400, precision=smg.MIXED)
            assert np.array_equal(host(X2)[2], host(x2)[0])
            assert np.array_equal(host(X2)[0], X[0])
    finally:
        for s in solvers:
            s.close()


def test_group_rejects_mismatched_shapes(cuda):
    import paper_0710_3612_amd as smg

    U = dev(synth.links_from_angles(synth.metropolis_u1(32, 32, 3.0, 5, 1)))
    a = smg.Solver(U, smg.make_params(32, 32, 0.1, levels=2, blocks=[(4, 4)], nv=[6]))
    b = smg.Solver(U, smg.make_params(32, 32, 0.1, levels=2, blocks=[(4, 4)], nv=[5]))
    c = smg.Solver(U, smg.make_params(32, 32, 0.1, levels=2, blocks=[(4, 4)], nv=[6], coarsest=smg.COARSEST_CG))
    try:
        with pytest.raises(smg.SmgError):
            smg.Group([a, b])
        with pytest.raises(smg.SmgError):
            smg.Group([c, c])
    finally:
        for s in (a, b, c):
            s.close()


@pytest.mark.parametrize("lx,lt,blocks,nv,opst", [(128, 128, [(4, 4), (4, 4)], [12, 12], 2),
                                                 (64, 64, [(4, 4), (4, 4)], [6, 6], 0)])
def test_group_level_op_equals_single(cuda, lx, lt, blocks, nv, opst):
    """smg_group_level_op_f32: column j is handle j's own FP32 level operator (fine A,
    the coarse operators, modes 0 and 2) bit for bit, also after a re-mass of one
    handle (the tables are filled again)."""
    import torch

    import paper_0710_3612_amd as smg

    solvers = []
    for f in range(2):
        U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 10, 400 + f))
        p = smg.make_params(lx, lt, 0.05, levels=len(blocks) + 1, blocks=blocks, nv=nv, operator_storage=opst,
                            coarsest_fp64=False, seed=17 + f)
        s0 = smg.Solver(dev(U), p)
        solvers += [s0, s0.derive(0.11)]
    G = len(solvers)
    try:
        with smg.Group(solvers) as g:
            for remass in (False, True):
                if remass:
                    solvers[1].set_mass(0.2)
                for level in range(len(blocks) + 1):
                    n = solvers[0].level_size(level)
                    rng = np.random.default_rng(31 + level)
                    X = torch.from_numpy((rng.standard_normal((G, n)) + 1j * rng.standard_normal((G, n)))
                                         .astype(np.complex64)).to("cuda")
                    Aux = torch.from_numpy((rng.standard_normal((G, n)) + 1j * rng.standard_normal((G, n)))
                                           .astype(np.complex64)).to("cuda")
                    Y0 = host(g.level_op_f32(level, X))
                    Y2 = host(g.level_op_f32(level, X, mode=2, aux=Aux))
                    for j, s in enumerate(solvers):
                        y0 = host(s.level_op_f32(level, X[j:j + 1].contiguous()))
                        y2 = host(s.level_op_f32(level, X[j:j + 1].contiguous(), mode=2,
                                                 aux=Aux[j:j + 1].contiguous()))
                        assert np.array_equal(Y0[j], y0.reshape(-1)), (remass, level, j)
                        assert np.array_equal(Y2[j], y2.reshape(-1)), (remass, level, j)
            X1 = torch.zeros((G, solvers[0].level_size(1)), dtype=torch.complex64, device="cuda")
            with pytest.raises(smg.SmgError):
                g.level_op_f32(1, X1, mode=1)
            with pytest.raises(ValueError):
                g.level_op_f32(1, X1[:, 1:].contiguous())
    finally:
        for s in solvers:
            s.close()
