"""GPU: continuous batching (smg_batch_*) and the serving loop.

A right-hand side's solution must be bitwise the same whether it is solved alone
or admitted into a batch that other right-hand sides enter and leave; FP64
batches must reproduce smg_solve's MG-CG bitwise; every converged solution must
reach a true residual <= 1e-10 recomputed with the oracle's sparse A.
"""

import numpy as np
import pytest

import synth
from oracle import multigrid as mg
from oracle.wilson import dirac_matrix, normal_matrix

pytestmark = pytest.mark.gpu


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def smg_mod():
    import paper_0710_3612_amd as smg

    return smg


def relres(A, b, x):
    return np.linalg.norm(b - A @ x) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def setup32():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    smg = smg_mod()
    lx, lt, m = 32, 24, 0.04
    U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 30, 41))
    p = smg.make_params(lx, lt, m, levels=3, blocks=[(4, 4), (2, 2)], nv=[6, 6], seed=5)
    s = smg.Solver(dev(U), p)
    A = normal_matrix(U, m)
    n = 2 * lx * lt
    D = dirac_matrix(U, m)
    B = np.stack([D.conj().T @ v for v in synth.gaussian((6, n), 77)])
    yield dict(s=s, A=A, B=B, n=n, U=U, p=p)
    s.close()


def run_to_end(bt, slots, max_steps=2000):
    """Step until none of `slots` is running; returns {slot: stats}."""
    out = {}
    for _ in range(max_steps):
        for j, st in bt.poll():
            if j in slots and j not in out:
                out[j] = st
        if all(j in out for j in slots):
            return out
        bt.step(1)
    raise AssertionError("batch did not finish")


def test_fp64_batch_reproduces_solve_bitwise(setup32):
    smg = smg_mod()
    s, A, B = setup32["s"], setup32["A"], setup32["B"]
    ref = []
    for j in range(3):
        x, st, code = s.solve(dev(B[j]), tol=1e-10, maxiter=500, precision=smg.FP64)
        assert code == 0
        ref.append((host(x), st[0]["iterations"]))
    with smg.Batch(s, 4, tol=1e-10, maxiter=500, precision=smg.FP64) as bt:
        a = bt.admit(dev(B[0]))
        bt.step(2)
        b = bt.admit(dev(B[1]))
        bt.step(1)
        c = bt.admit(dev(B[2]))
        done = run_to_end(bt, [a, b, c])
        for j, slot in enumerate((a, b, c)):
            st = done[slot]
            assert st["status"] == 0
            x = host(bt.harvest(slot))
            assert np.array_equal(x, ref[j][0]), j
            assert st["iterations"] == ref[j][1]
            assert relres(A, B[j], x) <= 1e-10
            assert st["true_relres"] <= 1e-10


def test_mixed_batch_alone_vs_mix_bitwise(setup32):
    """Continuous batching: slots enter, leave (harvest, cancel) and are refilled;
    each solution equals the one from a batch where it runs alone."""
    smg = smg_mod()
    s, A, B = setup32["s"], setup32["A"], setup32["B"]
    alone = {}
    for j in range(5):
        with smg.Batch(s, 1, tol=1e-10, maxiter=500, precision=smg.MIXED) as bt:
            slot = bt.admit(dev(B[j]))
            st = run_to_end(bt, [slot])[slot]
            assert st["status"] == 0
            alone[j] = (host(bt.harvest(slot)), st["iterations"])
            assert relres(A, B[j], alone[j][0]) <= 1e-10
    with smg.Batch(s, 3, tol=1e-10, maxiter=500, precision=smg.MIXED) as bt:
        s0 = bt.admit(dev(B[0]))
        s1 = bt.admit(dev(B[1]))
        s2 = bt.admit(dev(B[5]))  # cancelled below
        assert bt.admit(dev(B[2])) is None  # full
        assert bt.counts() == (3, 3)
        bt.step(2)
        bt.cancel(s2)
        assert bt.counts() == (2, 2)
        s3 = bt.admit(dev(B[2]))  # refills the freed slot
        assert s3 == s2
        got = {}
        pending = {s0: 0, s1: 1, s3: 2}
        queue = [3, 4]
        for _ in range(2000):
            for slot, st in bt.poll():
                j = pending.pop(slot)
                assert st["status"] == 0
                got[j] = (host(bt.harvest(slot)), st["iterations"])
                if queue:
                    k = queue.pop(0)
                    pending[bt.admit(dev(B[k]))] = k
            if not pending:
                break
            bt.step(1)
        assert sorted(got) == [0, 1, 2, 3, 4]
        for j in range(5):
            assert np.array_equal(got[j][0], alone[j][0]), j
            assert got[j][1] == alone[j][1]


def test_batch_matches_oracle_solution(setup32):
    """Flexible CG with the FP32 V-cycle reaches the oracle's solution."""
    smg = smg_mod()
    s, A, B = setup32["s"], setup32["A"], setup32["B"]
    Ad = A.tocsc()
    import scipy.sparse.linalg as sla

    lu = sla.splu(Ad)
    with smg.Batch(s, 2, tol=1e-10, maxiter=500, precision=smg.MIXED) as bt:
        slot = bt.admit(dev(B[4]))
        run_to_end(bt, [slot])
        x = host(bt.harvest(slot))
    xo = lu.solve(B[4])
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-7


def test_batch_edge_cases(setup32):
    smg = smg_mod()
    s, B, n = setup32["s"], setup32["B"], setup32["n"]
    with smg.Batch(s, 2, tol=1e-10, maxiter=3, precision=smg.FP64) as bt:
        z = bt.admit(dev(np.zeros(n)))
        done = dict(bt.poll())
        assert z in done and done[z]["status"] == 0 and done[z]["iterations"] == 0
        assert np.all(host(bt.harvest(z)) == 0)
        bad = B[0].copy()
        bad[7] = np.nan
        with pytest.raises(smg.SmgError) as ei:
            bt.admit(dev(bad))
        assert ei.value.code == -5
        assert bt.counts() == (0, 0)
        a = bt.admit(dev(B[0]))
        with pytest.raises(smg.SmgError) as ei:
            bt.harvest(a)  # still running
        assert ei.value.code == -1
        st = run_to_end(bt, [a])[a]
        assert st["status"] == smg.NOTCONV and st["iterations"] == 3
        bt.harvest(a)
        with pytest.raises(smg.SmgError):
            bt.harvest(a)  # slot no longer in use
        assert bt.memory_bytes() > 0
    with pytest.raises(smg.SmgError):
        smg.Batch(s, 0)
    with pytest.raises(smg.SmgError):
        smg.Batch(s, 4, precision=7)


def test_server_results_equal_alone(cuda):
    """The request loop on two fields and three masses with Poisson arrivals:
    every result reaches 1e-10 against the oracle and equals the same right-hand
    side solved alone in a batch of the same hierarchy."""
    import torch

    smg = smg_mod()
    from paper_0710_3612_amd import serve

    fields = {}
    ops = {}
    for f, (L, beta) in enumerate([(32, 3.0), (16, 6.0)]):
        U = synth.links_from_angles(synth.metropolis_u1(L, L, beta, 30, 500 + f))
        p = smg.make_params(L, L, 0.0, levels=serve.levels_for(L), blocks=[(4, 4)] * 3, nv=[6, 6, 6], seed=11 + f)
        fields[f] = (dev(U), p)
        ops[f] = U
    masses = {0: [0.05, 0.1], 1: [0.2]}

    class Recording(serve.DeviceBackend):
        """Remembers how each key's hierarchy was made (setup, or derived from
        which mass) so that the test can rebuild it the same way."""

        def __init__(self, *a, **k):
            super().__init__(*a, **k)
            self.made = {}
            self.key_of = {}

        def setup(self, field, mass, stream):
            s = super().setup(field, mass, stream)
            self.made[(field, mass)] = None
            self.key_of[id(s)] = (field, mass)
            return s

        def derive(self, solver, mass, stream):
            f, m0 = self.key_of[id(solver)]
            s = super().derive(solver, mass, stream)
            self.made[(f, mass)] = m0
            self.key_of[id(s)] = (f, mass)
            return s

    be = Recording(fields, mixed=True)
    trace = serve.poisson_trace(14, rate=400.0, fields=[0, 1], masses=masses, k_range=(1, 3), seed=8)
    reqs = []
    for i, (t, f, m, k, sd) in enumerate(trace):
        n = fields[f][0].shape[1] * fields[f][0].shape[2] * 2
        rhs = synth.gaussian_device(n, sd, "cuda", count=k)
        reqs.append(serve.Request(i, f, m, rhs, k, t))
    torch.cuda.synchronize()
    with serve.Server(be, budget_bytes=8 << 30, capacity=4, tol=1e-10, maxiter=500, precision=smg.MIXED,
                      max_lanes=3) as srv:
        results = srv.run_trace(reqs, timeout=120)
        summ = serve.latency_summary(results)
        assert summ["ok"] == len(reqs)
        # rebuild each key the way the server did and solve alone
        ref_solvers = {}

        def ref_solver(f, m):
            key = (f, m)
            if key not in ref_solvers:
                src = be.made[key]
                g, p = fields[f]
                if src is None:
                    q = type(p)()
                    serve.ctypes_copy(q, p)
                    q.mass = m
                    ref_solvers[key] = smg.Solver(g, q)
                else:
                    ref_solvers[key] = ref_solver(f, src).derive(m)
            return ref_solvers[key]

        try:
            for req, res in zip(reqs, results):
                s = ref_solver(req.field, req.mass)
                A = normal_matrix(ops[req.field], req.mass)
                xs = host(res.x)
                bs = host(req.rhs)
                with smg.Batch(s, 1, tol=1e-10, maxiter=500, precision=smg.MIXED) as bt:
                    for j in range(req.k):
                        slot = bt.admit(req.rhs[j])
                        run_to_end(bt, [slot])
                        xa = host(bt.harvest(slot))
                        assert np.array_equal(xa, xs[j]), (req.rid, j)
                        assert relres(A, bs[j], xs[j]) <= 1e-10
                assert res.latency >= 0 and res.finished >= res.admitted >= res.arrival - 1e-6
        finally:
            for v in ref_solvers.values():
                v.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_equal_eager_launches(setup32, precision):
    """Each iteration's device work replayed from a captured graph gives bitwise
    the results of launching it kernel by kernel, over many replays and with slots
    entering and leaving (different leading-slot counts, eager work in between)."""
    smg = smg_mod()
    s, B = setup32["s"], setup32["B"]

    def run(graphs):
        out = {}
        with smg.Batch(s, 4, tol=1e-10, maxiter=500, precision=precision) as bt:
            bt.use_graphs(graphs)
            a = bt.admit(dev(B[0]))
            bt.step(3)
            b = bt.admit(dev(B[1]))
            c = bt.admit(dev(B[2]))
            bt.step(2)
            bt.cancel(b)
            d = bt.admit(dev(B[3]))
            done = run_to_end(bt, [a, c, d])
            for name, slot in (("a", a), ("c", c), ("d", d)):
                out[name] = (host(bt.harvest(slot)), done[slot]["iterations"], done[slot]["status"])
        return out

    g, e = run(True), run(False)
    for k in g:
        assert g[k][2] == 0 and e[k][2] == 0
        assert g[k][1] == e[k][1], k
        assert np.array_equal(g[k][0], e[k][0]), k
