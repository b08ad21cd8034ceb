"""Host-only checks of the C ABI: the library loads, exports every function declared in
include/*.h, and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2404_03313_amd import native as nt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(s3ttv_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    declared = _declared_functions()
    assert len(declared) >= 9
    L = nt.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(nt.EXPORTS) == declared


def test_strerror_and_workspace_queries():
    assert nt.strerror(0) == "ok"
    assert "workspace" in nt.strerror(nt.EWORKSPACE)
    b1 = nt.workspace_bytes(32, 32, 16, 3, 3)
    b2 = nt.workspace_bytes(256, 256, 128, 4, 4)
    # dominant term: one 16 x 2*Bp dual block per pixel
    assert b2 > 256 * 256 * 16 * 256 * 4
    assert b1 < b2


@pytest.mark.parametrize("K,ncols,code", [(16, 64, 0), (17, 45, 0), (100, 396, 0),
                                           (101, 396, nt.EUNSUPPORTED), (0, 8, nt.EINVAL)])
def test_clip_workspace_query(K, ncols, code):
    """Spectral clip of K x ncols blocks: K <= 100 is served (K > 16 by the large-block
    kernel, whose workspace holds K x ncols rows padded to 32 columns and a K x K basis per
    block)."""
    sz = ctypes.c_size_t()
    sh = nt.Shape(1, 1, ncols, K, 1)
    assert nt.lib().s3ttv_op_workspace_bytes(nt.OP_CLIP, ctypes.byref(sh), 7, ctypes.byref(sz)) == code
    if code == 0 and K > 16:
        ncolp = (ncols + 31) // 32 * 32
        assert sz.value >= 7 * K * ncolp * 4 + 7 * K * K * 4


@pytest.mark.parametrize("k,code", [((4, 4), 0), ((5, 4), 0), ((10, 10), 0), ((11, 10), nt.EUNSUPPORTED)])
def test_dual_blocks_workspace_query(k, code):
    # the operator covers the same block sizes as the solver (K = k1 k2 up to 100)
    sz, sz_solve = ctypes.c_size_t(), ctypes.c_size_t()
    sh = nt.Shape(12, 12, 20, *k)
    assert nt.lib().s3ttv_op_workspace_bytes(nt.OP_DUAL_BLOCKS, ctypes.byref(sh), 0,
                                             ctypes.byref(sz)) == code
    if code == 0:
        assert nt.lib().s3ttv_workspace_bytes(ctypes.byref(sh), None, ctypes.byref(sz_solve)) == 0
        K = k[0] * k[1]
        assert sz.value >= 144 * max(K, 16) * 2 * 32 * 4


@pytest.mark.parametrize("shape,code", [((1, 8, 4, 1, 1), nt.EINVAL), ((8, 8, 1, 1, 1), nt.EINVAL),
                                        ((8, 8, 4, 9, 1), nt.EINVAL), ((8, 8, 4, 0, 2), nt.EINVAL),
                                        ((12, 12, 4, 11, 10), nt.EUNSUPPORTED),
                                        # 4 x 4 blocks: the 1 x 1 anchor tile's overlap-add
                                        # accumulators hold 16 (2 Bp + 16) floats <= 152 KiB
                                        # (Bp = N3 rounded up to 16): N3 <= 1200
                                        ((8, 8, 1200, 4, 4), 0),
                                        ((8, 8, 1201, 4, 4), nt.EUNSUPPORTED),
                                        ((8, 8, 3000, 2, 2), 0),
                                        # more rows: one workgroup per block, any band count
                                        ((12, 12, 3000, 5, 4), 0),
                                        # ... while the gradient field (n1 n2 x 2 Bp) has
                                        # fewer than 2^32 entries: 11000^2 x 64 does not,
                                        # the fused path (4 x 4) takes it
                                        ((11000, 11000, 17, 5, 5), nt.EUNSUPPORTED),
                                        ((11000, 11000, 17, 4, 4), 0)])
def test_shape_validation(shape, code):
    sz = ctypes.c_size_t()
    sh = nt.Shape(*shape)
    assert nt.lib().s3ttv_workspace_bytes(ctypes.byref(sh), None, ctypes.byref(sz)) == code


@pytest.mark.parametrize("bad", [dict(eps=0.0), dict(alpha=-1.0), dict(beta=float("nan")),
                                 dict(mu_min=1.0, mu_max=0.0), dict(max_iter=0),
                                 dict(gammas=dict(gamma_u=0.1)), dict(eig_max_steps=256),
                                 dict(regularizer=5), dict(regularizer=-1), dict(omega=-0.1),
                                 dict(omega=float("nan"))])
def test_param_validation_before_any_gpu_call(bad):
    kw = dict(eps=1.0, alpha=1.0, beta=1.0, max_iter=10)
    kw.update(bad)
    p = nt.make_params(**kw)
    dummy = ctypes.c_void_p(16)   # never dereferenced: validation fails first
    rc = nt.lib().s3ttv_solve(ctypes.byref(nt.Shape(8, 8, 4, 2, 2)), ctypes.byref(p), dummy, None,
                              dummy, dummy, dummy, dummy, 1 << 30, None, None)
    assert rc == nt.EINVAL


def test_continue_rejects_invalid_arguments_before_any_gpu_call():
    """s3ttv_solve_continue validates shape, parameters and pointers like s3ttv_solve before it
    reads the workspace's state."""
    p = nt.make_params(1.0, 1.0, 1.0, 10)
    dummy = ctypes.c_void_p(16)
    L = nt.lib()
    rc = L.s3ttv_solve_continue(ctypes.byref(nt.Shape(8, 8, 4, 2, 2)), ctypes.byref(p), None,
                                None, None, None, None, 0, None, None)
    assert rc == nt.EINVAL
    bad = nt.make_params(1.0, 1.0, 1.0, 0)
    rc = L.s3ttv_solve_continue(ctypes.byref(nt.Shape(8, 8, 4, 2, 2)), ctypes.byref(bad), dummy,
                                dummy, dummy, dummy, dummy, 1 << 30, None, None)
    assert rc == nt.EINVAL
    rc = L.s3ttv_solve_continue(ctypes.byref(nt.Shape(12, 12, 4, 11, 10)), ctypes.byref(p), dummy,
                                dummy, dummy, dummy, dummy, 1 << 30, None, None)
    assert rc == nt.EUNSUPPORTED
    rc = L.s3ttv_solve_continue(ctypes.byref(nt.Shape(8, 8, 4, 2, 2)), ctypes.byref(p), dummy,
                                dummy, dummy, dummy, dummy, 16, None, None)
    assert rc == nt.EWORKSPACE


def test_l1_noalloc_validates_before_any_gpu_call():
    """The allocation-free l1 projection rejects sizes beyond its static scratch (2^24
    elements) and invalid arguments on the host."""
    L = nt.lib()
    dummy = ctypes.c_void_p(16)
    assert L.s3ttv_op_l1_project_noalloc((1 << 24) + 1, dummy, 1.0, dummy, None, None) == nt.EUNSUPPORTED
    assert L.s3ttv_op_l1_project_noalloc(0, dummy, 1.0, dummy, None, None) == nt.EINVAL
    assert L.s3ttv_op_l1_project_noalloc(10, None, 1.0, dummy, None, None) == nt.EINVAL
    assert L.s3ttv_op_l1_project_noalloc(10, dummy, 0.0, dummy, None, None) == nt.EINVAL
    assert L.s3ttv_op_l1_project_noalloc(10, dummy, float("inf"), dummy, None, None) == nt.EINVAL


def test_null_pointers_rejected():
    p = nt.make_params(1.0, 1.0, 1.0, 10)
    rc = nt.lib().s3ttv_solve(ctypes.byref(nt.Shape(8, 8, 4, 2, 2)), ctypes.byref(p), None, None,
                              None, None, None, None, 0, None, None)
    assert rc == nt.EINVAL


@pytest.mark.parametrize("cname,pyty", [("s3ttv_shape", "Shape"), ("s3ttv_params", "Params"),
                                        ("s3ttv_stats", "Stats"), ("s3ttv_cnn_shape", "CnnShape")])
def test_struct_layouts_match_header(tmp_path, cname, pyty):
    """ctypes mirrors of the public structs agree with the C header field by field (offsets
    and total size, as gcc lays them out)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    cls = getattr(nt, pyty)
    lines = [f'printf("size %zu\\n", sizeof({cname}));']
    for name, *_ in cls._fields_:
        lines.append(f'printf("{name} %zu\\n", offsetof({cname}, {name}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"s3ttv.h\"\n"
                   "#include \"s3ttv_cnn.h\"\n"
                   "int main(void) {\n" + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], check=True, capture_output=True,
                                                        text=True).stdout.splitlines())
    assert int(out["size"]) == ctypes.sizeof(cls)
    for name, *_ in cls._fields_:
        assert int(out[name]) == getattr(cls, name).offset, name


# ---------------------------------------------------------------- learned initial estimate

def test_cnn_param_count_and_workspace():
    assert nt.cnn_param_count() == 84801
    small = nt.cnn_workspace_bytes((8, 8, 8), False)
    train = nt.cnn_workspace_bytes((8, 8, 8), True)
    assert train > small > 2 * 8 ** 3 * 32 * 2
    # inference keeps two BF16 activation buffers of 32 channels per voxel
    big = nt.cnn_workspace_bytes((512, 512, 191), False)
    assert 2 * 512 * 512 * 191 * 64 <= big < 2 * 512 * 512 * 191 * 64 + (1 << 20)
    assert nt.cnn_workspace_bytes((4, 8, 8, 8), True) > train


@pytest.mark.parametrize("shape,code", [((0, 4, 4, 1), nt.EINVAL), ((4, 4, 4, 0), nt.EINVAL),
                                        ((4, -1, 4, 1), nt.EINVAL),
                                        ((1024, 1024, 1024, 2), nt.EUNSUPPORTED)])
def test_cnn_shape_validation(shape, code):
    sz = ctypes.c_size_t()
    sh = nt.CnnShape(*shape)
    assert nt.lib().s3ttv_cnn_workspace_bytes(ctypes.byref(sh), 0, ctypes.byref(sz)) == code
    assert nt.lib().s3ttv_cnn_workspace_bytes(None, 0, ctypes.byref(sz)) == nt.EINVAL


def test_cnn_arguments_rejected_before_any_gpu_call():
    L = nt.lib()
    sh = ctypes.byref(nt.CnnShape(4, 4, 4, 1))
    d = ctypes.c_void_p(256)   # never dereferenced: validation fails first
    odd = ctypes.c_void_p(258)
    big = 1 << 40
    loss = ctypes.c_double()
    assert L.s3ttv_cnn_forward(sh, None, d, d, d, big, None) == nt.EINVAL
    assert L.s3ttv_cnn_forward(sh, d, d, d, d, big, None) == nt.EINVAL       # v aliases u0
    assert L.s3ttv_cnn_forward(sh, d, odd, ctypes.c_void_p(512), d, big, None) == nt.EINVAL
    assert L.s3ttv_cnn_forward(sh, d, ctypes.c_void_p(512), ctypes.c_void_p(768), d, 16,
                               None) == nt.EWORKSPACE
    assert L.s3ttv_cnn_forward(sh, d, ctypes.c_void_p(512), ctypes.c_void_p(768), None, big,
                               None) == nt.EINVAL
    assert L.s3ttv_cnn_grad(sh, d, d, None, d, ctypes.byref(loss), d, big, None) == nt.EINVAL
    assert L.s3ttv_cnn_grad(sh, d, d, d, d, None, d, 16, None) == nt.EWORKSPACE
    for step, lr in ((0, 1e-3), (1, 0.0), (1, -1e-3), (1, float("nan")), (1, float("inf"))):
        assert L.s3ttv_cnn_train_step(sh, d, d, d, step, lr, d, d, None, d, big, None) == nt.EINVAL
    assert L.s3ttv_cnn_train_step(sh, d, d, None, 1, 1e-3, d, d, None, d, big, None) == nt.EINVAL
    assert L.s3ttv_cnn_train_step(sh, d, d, d, 1, 1e-3, d, d, None, d, 16, None) == nt.EWORKSPACE
