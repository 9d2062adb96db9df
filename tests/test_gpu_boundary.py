"""GPU checks of the boundary's memory contract: smg_query_bytes equals what the
calls allocate, and the library's device memory comes from PyTorch's caching
allocator (smg_set_allocator, installed by the binding) so that torch accounts
for it."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def smg_mod():
    import paper_0710_3612_amd as smg

    return smg


CONFIGS = [
    # lx, lt, extra make_params arguments
    (64, 64, dict(levels=3, blocks=[(4, 4), (4, 4)], nv=[6, 6])),
    (64, 64, dict(levels=3, blocks=[(4, 4), (4, 4)], nv=[6, 6], operator_storage=2, coarsest_fp64=False)),
    (64, 32, dict(levels=2, blocks=[(4, 4)], nv=[5], coarsest=1, smoother_storage=1)),
    (32, 32, dict(levels=3, blocks=[(4, 4), (2, 2)], nv=[4, 3], split_chirality=True, sa_scale=0.0)),
    (48, 40, dict(levels=1)),
    (64, 64, dict(levels=3, blocks=[(4, 4), (4, 4)], nv=[6, 6], remass_affine=True)),
]


@pytest.mark.parametrize("lx,lt,kw", CONFIGS)
@pytest.mark.parametrize("prec", [0, 1])
def test_query_bytes_equals_allocations(cuda, lx, lt, kw, prec):
    """setup_bytes = the handle's bytes after smg_setup and after smg_derive;
    solve_bytes = what its first solve of nrhs columns adds (a second, smaller
    solve adds nothing); batch_bytes = what smg_batch_create adds (batch plus
    handle growth)."""
    smg = smg_mod()
    if kw.get("levels", 2) == 1 and prec == 1:
        pytest.skip("one level: no mixed-precision V-cycle")
    U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 5, lx + lt))
    p = smg.make_params(lx, lt, 0.1, **kw)
    nrhs = 3
    setup, solve, batch = smg.query_bytes(p, nrhs, prec)
    n = 2 * lx * lt
    b = dev(synth.gaussian((nrhs, n), 5))
    with smg.Solver(dev(U), p) as s:
        assert s.memory_bytes() == setup
        # a derived handle keeps no mass coefficients (three link-sized arrays per coarse level)
        coef = 0
        if p.remass_affine:
            for l in range(1, p.levels):
                cx, ct, nc = s.level_info(l)
                coef += 3 * 9 * cx * ct * nc * nc * 16
        d = s.derive(0.2)
        try:
            assert d.memory_bytes() == setup - coef
        finally:
            d.close()
        s.solve(b, tol=1e-8, maxiter=200, precision=prec)
        assert s.memory_bytes() == setup + solve
        s.solve(b[:1], tol=1e-8, maxiter=200, precision=prec)
        assert s.memory_bytes() == setup + solve
    with smg.Solver(dev(U), p) as s:
        with smg.Batch(s, nrhs, tol=1e-8, maxiter=200, precision=prec) as bt:
            assert s.memory_bytes() + bt.memory_bytes() == setup + batch
            for j in range(nrhs):
                assert bt.admit(b[j]) is not None
            for _ in range(300):
                bt.step(1)
                if bt.counts()[1] == 0:
                    break
            assert s.memory_bytes() + bt.memory_bytes() == setup + batch


def test_library_memory_is_torch_memory(cuda):
    """A handle's device arrays are torch caching-allocator blocks: torch's
    allocated bytes grow by at least the handle's bytes while it lives and fall
    back when it is destroyed; hipMalloc is restored for later handles when the
    binding turns the allocator off, and the handles made before keep theirs."""
    import gc

    import torch

    smg = smg_mod()
    lx = lt = 64
    U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 5, 3))
    p = smg.make_params(lx, lt, 0.1, levels=3, blocks=[(4, 4), (4, 4)], nv=[6, 6])
    g = dev(U)
    # no collection of earlier tests' tensors may free memory inside the measurement
    gc.collect()
    gc.disable()
    try:
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        s = smg.Solver(g, p)
        used = torch.cuda.memory_allocated() - base
    finally:
        gc.enable()
    assert used >= s.memory_bytes() > 0
    smg.use_torch_allocator(False)
    try:
        before = torch.cuda.memory_allocated()
        s2 = smg.Solver(g, p)
        assert torch.cuda.memory_allocated() - before < s2.memory_bytes() // 2
        x = dev(synth.gaussian(2 * lx * lt, 4))
        y1, y2 = s.apply_A(x), s2.apply_A(x)
        assert torch.equal(y1, y2)
        s2.close()
    finally:
        smg.use_torch_allocator(True)
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base < used // 2


def test_progress_reports_setup_and_solve(cuda):
    """The progress callback sees every level's calibration, each near-null vector as
    it is added (1..nv in order), the end of the setup, the outer iterations with
    their largest relative residual, and the defect-correction passes of a mixed
    solve; with reporting off it sees nothing."""
    smg = smg_mod()
    lx = lt = 64
    U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 5, 9))
    p = smg.make_params(lx, lt, 0.1, levels=3, blocks=[(4, 4), (4, 4)], nv=[5, 4])
    ev = []
    smg.set_progress(lambda *a: ev.append(a))
    try:
        with smg.Solver(dev(U), p) as s:
            setup = list(ev)
            ev.clear()
            b = dev(synth.gaussian((2, 2 * lx * lt), 6))
            _, st, _ = s.solve(b, tol=1e-10, maxiter=200, precision=0)
            fp64 = list(ev)
            ev.clear()
            s.solve(b, tol=1e-10, maxiter=200, precision=1)
            mixed = list(ev)
            ev.clear()
            smg.set_progress(None)
            s.solve(b, tol=1e-10, maxiter=200, precision=0)
            assert ev == []
    finally:
        smg.set_progress(None)
    for l, nv in enumerate([5, 4]):
        assert ("calibrate", l, 0, nv, 0.0) in setup
        assert [e[2] for e in setup if e[0] == "candidate" and e[1] == l] == list(range(1, nv + 1))
    assert setup[-1][0] == "coarsest"
    its = [e for e in fp64 if e[0] == "iteration"]
    assert [e[2] for e in its] == list(range(1, len(its) + 1))
    assert len(its) == max(int(x["iterations"]) for x in st)
    assert its[-1][4] < its[0][4]
    ref = [e for e in mixed if e[0] == "refinement"]
    assert ref and [e[2] for e in ref] == list(range(1, len(ref) + 1))
    assert ref[-1][4] <= 1e-10


def test_open_handles_at_exit(cuda, tmp_path):
    """A program that ends with a handle and a batch still open exits cleanly: the
    binding closes them at exit, while the allocator callbacks that release their
    memory are still alive (module teardown would free those callbacks first)."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    prog = (
        "import numpy as np, torch, synth, paper_0710_3612_amd as smg\n"
        "U = synth.links_from_angles(synth.metropolis_u1(32, 32, 3.0, 5, 1))\n"
        "p = smg.make_params(32, 32, 0.1, levels=2, blocks=[(4, 4)], nv=[4])\n"
        "s = smg.Solver(torch.from_numpy(U).to('cuda'), p)\n"
        "d = s.derive(0.2)\n"
        "b = smg.Batch(s, 2)\n"
        "smg.set_progress(lambda *a: None)\n"
        "print('ok', flush=True)\n"
    )
    r = subprocess.run([sys.executable, "-c", prog], cwd=root, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip() == "ok"
