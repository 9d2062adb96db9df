"""smg_vcycle_noalloc, the V-cycle entry point that allocates nothing: its work
vectors live in the library's static scratch array.  Called through the C ABI and
compared with smg_vcycle, which runs the same kernels on the handle's own work
vectors: equal bit for bit (and so within the FP64 parity bound), on two calls in
a row, the second with fewer columns."""

import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def test_noalloc_vcycle_equals_vcycle(cuda):
    import torch

    import paper_0710_3612_amd as smg

    lib = smg.load_library()
    lx, lt = 64, 48
    U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 10, 77))
    p = smg.make_params(lx, lt, 0.07, levels=3, blocks=[(4, 4), (2, 2)], nv=[6, 5], seed=3)
    n = 2 * lx * lt
    with smg.Solver(dev(U), p) as s:
        stream = torch.cuda.current_stream()
        sp = ctypes.c_void_p(stream.cuda_stream)
        for nrhs, seed in ((4, 11), (1, 12)):
            b = dev(synth.gaussian((nrhs, n), seed))
            ref = s.vcycle(b)
            x = torch.full_like(b, complex("nan"))
            mem_lib, mem_torch = s.memory_bytes(), torch.cuda.memory_allocated()
            code = lib.smg_vcycle_noalloc(s.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                          nrhs, sp)
            assert code == 0, lib.smg_last_error().decode()
            torch.cuda.synchronize()
            # nothing was allocated, by the library or through its allocator callback
            assert s.memory_bytes() == mem_lib and torch.cuda.memory_allocated() == mem_torch
            assert torch.equal(x, ref), (nrhs, float((x - ref).abs().max()))
        # too many columns for the scratch array: a clear error before any launch
        code = lib.smg_vcycle_noalloc(s.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                      4096, sp)
        assert code == -1 and "scratch" in lib.smg_last_error().decode()


def test_noalloc_vcycle_rejects_cg_coarsest(cuda):
    import paper_0710_3612_amd as smg

    lx = lt = 32
    U = synth.links_from_angles(synth.metropolis_u1(lx, lt, 3.0, 5, 78))
    p = smg.make_params(lx, lt, 0.1, levels=2, blocks=[(4, 4)], nv=[4], coarsest=smg.COARSEST_CG)
    with smg.Solver(dev(U), p) as s:
        b = dev(synth.gaussian(2 * lx * lt, 13))
        out = dev(np.zeros(2 * lx * lt))
        with pytest.raises(smg.SmgError) as e:
            s.vcycle_noalloc(b, out)
        assert e.value.code == -1
