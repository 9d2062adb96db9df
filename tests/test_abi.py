"""Host-side checks of the C ABI (no GPU needed): the shared library loads and
exports every entry point that include/smg.h declares, the ctypes mirrors of the
parameter and statistics structs have the C layout, and error codes map to text."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smg.h")


def declared_functions():
    text = open(HEADER).read()
    return re.findall(r"^(?:int|void|const char\*)\s+(smg_\w+)\s*\(", text, re.M)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("smg_setup", "smg_solve", "smg_apply_A", "smg_apply_D", "smg_set_mass", "smg_vcycle",
                     "smg_restrict", "smg_prolong", "smg_smooth", "smg_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_0710_3612_amd as smg

    lib = smg.load_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"missing exports: {missing}"


def c_layout():
    """Offsets and sizes of the ABI structs as the C compiler lays them out."""
    import json
    import subprocess
    import tempfile

    fields = {
        "smg_params": ["lx", "lt", "mass", "levels", "block", "nv", "setup_iters", "smoother_steps",
                       "smoother_omega", "t_antiperiodic", "coarsest", "coarsest_tol", "coarsest_maxiter",
                       "inner_tol", "seed", "sa_scale", "smoother_storage", "stop_recursive", "mfma_min_rhs",
                       "operator_storage", "split_chirality", "coarsest_fp64", "remass_affine",
                       "nv_stop_rho", "nv_stop_iters"],
        "smg_stats": ["status", "iterations", "refinements", "vcycles", "fine_applies", "true_relres", "seconds"],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {", 'printf("{");']
    first = True
    for st, fs in fields.items():
        for f in fs:
            sep = "" if first else ","
            first = False
            lines.append(f'printf("{sep}\\"{st}.{f}\\": %zu", offsetof({st}, {f}));')
        lines.append(f'printf(",\\"{st}\\": %zu", sizeof({st}));')
    lines += ['printf("}\\n");', "return 0; }"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c99", src, "-o", exe], check=True)
        return json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout), fields


def test_struct_layouts_match_c():
    """Offsets and sizes of the ctypes mirrors equal the C compiler's."""
    import paper_0710_3612_amd as smg

    lay, fields = c_layout()
    for st, cls in (("smg_params", smg.Params), ("smg_stats", smg.Stats)):
        assert [f for f, _ in cls._fields_] == fields[st]
        for f in fields[st]:
            assert getattr(cls, f).offset == lay[f"{st}.{f}"], (st, f)
        assert ctypes.sizeof(cls) == lay[st]


def test_default_params_and_strerror():
    import paper_0710_3612_amd as smg

    lib = smg.load_library()
    p = smg.Params()
    lib.smg_default_params(ctypes.byref(p))
    assert (p.levels, p.smoother_steps, p.setup_iters) == (2, 4, 5)
    assert abs(p.smoother_omega - 0.8) < 1e-15
    assert p.block[0][0] == 4 and p.nv[0] == 8
    assert abs(p.sa_scale - 4.0 / 3.0) < 1e-15
    assert p.mfma_min_rhs == 16
    assert lib.smg_strerror(-2).decode().startswith("lattice extents")
    assert lib.smg_strerror(1).decode().startswith("not converged")


def test_setup_rejects_bad_shapes_without_touching_the_device():
    """Parameter validation happens before any device call."""
    import paper_0710_3612_amd as smg

    lib = smg.load_library()
    p = smg.make_params(30, 32, 0.1, levels=2, blocks=[(4, 4)], nv=[8])
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    assert lib.smg_setup(fake, ctypes.byref(p), None, None, ctypes.byref(h)) == -2
    assert "divisible" in lib.smg_last_error().decode()
    p = smg.make_params(32, 32, 0.1, levels=2, blocks=[(2, 2)], nv=[9])
    assert lib.smg_setup(fake, ctypes.byref(p), None, None, ctypes.byref(h)) == -1
    p = smg.make_params(32, 32, float("nan"))
    assert lib.smg_setup(fake, ctypes.byref(p), None, None, ctypes.byref(h)) == -1
    assert lib.smg_setup(None, ctypes.byref(p), None, None, ctypes.byref(h)) == -1


def test_reduced_smoother_storage_rejected_where_no_tile_fits():
    import paper_0710_3612_amd as smg

    lib = smg.load_library()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    p = smg.make_params(48, 32, 0.1, levels=2, blocks=[(4, 4)], nv=[4], smoother_storage=smg.STORE_BF16)
    assert lib.smg_setup(fake, ctypes.byref(p), None, None, ctypes.byref(h)) == -1
    assert "lx % 32" in lib.smg_last_error().decode()
    p = smg.make_params(64, 32, 0.1, levels=2, blocks=[(4, 4)], nv=[4], smoother_storage=7)
    assert lib.smg_setup(fake, ctypes.byref(p), None, None, ctypes.byref(h)) == -1


def test_operator_storage_validation():
    """operator_storage takes FP32 (default) or FP16 only; anything else is rejected
    before any device call."""
    import paper_0710_3612_amd as smg

    lib = smg.load_library()
    p = smg.Params()
    lib.smg_default_params(ctypes.byref(p))
    assert p.operator_storage == smg.STORE_F32
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    for bad in (smg.STORE_BF16, 7, -1):
        p = smg.make_params(64, 32, 0.1, levels=2, blocks=[(4, 4)], nv=[4], operator_storage=bad)
        assert lib.smg_setup(fake, ctypes.byref(p), None, None, ctypes.byref(h)) == -1
        assert "operator_storage" in lib.smg_last_error().decode()


def test_query_bytes_plans_without_a_device():
    """smg_query_bytes runs the allocation plan on the host: it answers without a
    GPU, grows with the columns and the precision's extra copies, counts the
    FP16 operator copies, and rejects what smg_setup rejects."""
    import paper_0710_3612_amd as smg

    p = smg.make_params(64, 64, 0.1, levels=3, blocks=[(4, 4), (4, 4)], nv=[8, 8])
    s1, f1, b1 = smg.query_bytes(p, 1, smg.FP64)
    s8, f8, b8 = smg.query_bytes(p, 8, smg.FP64)
    assert s1 == s8 > 0 and f8 > f1 > 0 and b8 > b1 > 0
    _, m8, bm8 = smg.query_bytes(p, 8, smg.MIXED)
    assert m8 > f8 and bm8 > b8  # FP32 copies of the hierarchy and FP32 work vectors
    # the fine links (32 B per site) and the coarsest inverse (n^2 16 B) are in the setup
    n_c = 4 * 4 * 8
    assert s1 > 64 * 64 * 32 + n_c * n_c * 16
    q = smg.make_params(64, 64, 0.1, levels=3, blocks=[(4, 4), (4, 4)], nv=[8, 8], operator_storage=smg.STORE_F16,
                        coarsest_fp64=False)
    _, m16, _ = smg.query_bytes(q, 8, smg.MIXED)
    assert m16 > m8  # FP16 copies of links, P and the inverse, plus the FP32 inverse
    bad = smg.make_params(30, 32, 0.1, levels=2, blocks=[(4, 4)], nv=[8])
    with pytest.raises(smg.SmgError) as e:
        smg.query_bytes(bad, 1, smg.FP64)
    assert e.value.code == -2
    assert smg.query_bytes(p, 300, smg.FP64)[2] is None  # a batch has at most 256 slots
    with pytest.raises(smg.SmgError):
        smg.query_bytes(p, 5000, smg.FP64)
    lib = smg.load_library()
    a = ctypes.c_size_t()
    assert lib.smg_query_bytes(ctypes.byref(p), 300, 0, None, None, ctypes.byref(a)) == -1


def test_set_allocator_needs_both_callbacks():
    import paper_0710_3612_amd as smg

    lib = smg.load_library()
    fn = smg._ALLOC_FN(lambda n, s, c: None)
    assert lib.smg_set_allocator(fn, smg._RELEASE_FN(), None) == -1
    smg.use_torch_allocator(True)


def test_set_progress_installs_and_clears():
    """smg_set_progress takes a callback and NULL; installing one calls nothing."""
    import paper_0710_3612_amd as smg

    seen = []
    smg.set_progress(lambda *a: seen.append(a))
    smg.set_progress(None)
    assert seen == []
