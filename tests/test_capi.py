"""CPU checks of the C ABI library: it loads and exports every entry point the header declares."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vsr.h")
LIB = os.path.join(ROOT, "paper_2107_14758_amd", "libvsr.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vsr_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("vsr_setup", "vsr_apply_operator", "vsr_apply_relaxation", "vsr_pcg_solve", "vsr_destroy",
              "vsr_load_vector", "vsr_num_dofs", "vsr_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvsr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvsr.so not built")
def test_error_text_and_defaults_without_gpu_work():
    from paper_2107_14758_amd import vsr
    L = vsr.lib()
    opt = vsr.Options()
    L.vsr_default_options(ctypes.byref(opt))
    assert opt.lanczos_steps == 20 and opt.max_iterations == 1000 and opt.relax_fp32 == 0
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    mesh = vsr.Mesh(2, 2, 2, None)
    st = L.vsr_setup(ctypes.byref(mesh), 3, None, None, ctypes.byref(h))
    assert st == vsr.VSR_EINVAL and b"NULL" in L.vsr_last_error()
    assert L.vsr_num_dofs(None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvsr.so not built")
def test_batch_and_tuning_argument_checks_without_gpu_work():
    from paper_2107_14758_amd import vsr
    L = vsr.lib()
    h = ctypes.c_void_p()
    opt = vsr.Options()
    L.vsr_default_options(ctypes.byref(opt))
    assert opt.autotune == 0 and opt.batch_streams == 0 and opt.batch_eager == 0 and opt.tune_cache is None
    assert L.vsr_setup_batch(0, None, None, None, ctypes.byref(opt), ctypes.byref(h)) == vsr.VSR_EINVAL
    meshes = (vsr.Mesh * 1)(vsr.Mesh(2, 2, 2, None))
    ps = (ctypes.c_int32 * 1)(3)
    st = L.vsr_setup_batch(1, meshes, ps, None, ctypes.byref(opt), ctypes.byref(h))
    assert st == vsr.VSR_EINVAL and b"member 0" in L.vsr_last_error()
    assert L.vsr_batch_size(None) == -1 and L.vsr_batch_member(None, 0) is None
    shapes = (ctypes.c_int32 * 6)(1, 1, 8, 0, 0, 256)
    assert L.vsr_set_tuning(None, shapes) == vsr.VSR_EINVAL
    assert L.vsr_pcg_solve_batch(None, None, None, 1e-8, None) == vsr.VSR_EINVAL
    # the options record keeps the C layout: the new fields follow the stream pointer
    assert vsr.Options.autotune.offset == vsr.Options.stream.offset + 8
    assert vsr.Options.tune_cache.offset == vsr.Options.autotune.offset + 16
    assert vsr.Options.share_factors.offset == vsr.Options.tune_cache.offset + 8 and opt.share_factors == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="libvsr.so not built")
def test_batch_create_argument_checks_without_gpu_work():
    from paper_2107_14758_amd import vsr
    L = vsr.lib()
    h = ctypes.c_void_p()
    assert L.vsr_batch_create(0, None, None, ctypes.byref(h)) == vsr.VSR_EINVAL
    null_members = (ctypes.c_void_p * 2)(None, None)
    st = L.vsr_batch_create(2, null_members, None, ctypes.byref(h))
    assert st == vsr.VSR_EINVAL and b"NULL member 0" in L.vsr_last_error()


def test_binding_rejects_wrong_lengths_and_shapes_before_any_device_call():
    """The kernels read and write exactly n entries through each vector pointer, so the
    binding checks every length (and the host arrays' shapes) before calling the library."""
    torch = pytest.importorskip("torch")
    from paper_2107_14758_amd import inputs, vsr
    V = inputs.cube_vertices(2, 3, 2)
    with pytest.raises(ValueError):
        vsr._Inputs(V[..., :2])                       # two coordinates per vertex
    with pytest.raises(ValueError):
        vsr._Inputs(V, kappa=np.ones(11))              # 12 cells
    with pytest.raises(ValueError):
        vsr._Inputs(V, mu_override=np.ones(35))
    ok = vsr._Inputs(V, kappa=np.ones(12), mu_override=np.ones((12, 3)))
    assert ok.shape == (2, 3, 2)
    # a problem handle stand-in: only the sizes are read before the length checks fire
    prob = object.__new__(vsr.Problem)
    prob._h, prob._owned, prob.p, prob.q = ctypes.c_void_p(), False, 3, 6
    prob.n, prob.ncell = 5 * 8 * 5, 12
    short, right = torch.zeros(prob.n - 1, dtype=torch.float64), torch.zeros(prob.n, dtype=torch.float64)
    for call in (lambda: prob.apply_operator(short, right), lambda: prob.apply_relaxation(short, right, 1),
                 lambda: prob.pcg_solve(short, right),
                 lambda: prob.load_vector(torch.zeros(12 * 6 ** 3 - 1, dtype=torch.float64), right),
                 lambda: vsr._ptr(short, prob.n)):
        with pytest.raises(ValueError):
            call()
    with pytest.raises(TypeError):                      # right length, but host memory
        prob.apply_operator(right, right.clone())
    with pytest.raises(ValueError):
        vsr._rows(torch.zeros(4, 73), 74, "X")
    with pytest.raises(ValueError):
        vsr._cells(np.zeros((3, 23)))
