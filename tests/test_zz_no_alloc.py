"""The allocation-free weight gradient of the warm-start network (GPU), through the C ABI.

ivx_nn_conv3x3_grad_weight_noalloc keeps its split partials in a static device array
instead of a per-call allocation.  Its results must be those of the allocating
ivx_nn_conv3x3_grad_weight bit for bit (same kernels, same summation order), on calls in a
row that reuse the array with shrinking shapes: a large tiled layer, a smaller tiled layer,
then a small layer on the direct-load path (cout not a multiple of 4).
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2609_17636_amd import load_library  # noqa: E402

SHAPES = [(2, 40, 51, 96, 64), (1, 23, 33, 16, 32), (1, 9, 11, 8, 18)]


def _lib():
    lib = load_library("f32")
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    for name in ("ivx_nn_conv3x3_grad_weight", "ivx_nn_conv3x3_grad_weight_noalloc"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp, vp]
        f.restype = ctypes.c_int
    lib.ivx_nn_conv3x3_grad_weight_noalloc_capacity.argtypes = []
    lib.ivx_nn_conv3x3_grad_weight_noalloc_capacity.restype = ctypes.c_int64
    lib.ivx_nn_conv3x3_grad_weight_scratch_floats.argtypes = [i32] * 5
    lib.ivx_nn_conv3x3_grad_weight_scratch_floats.restype = ctypes.c_int64
    lib.ivx_last_error.restype = ctypes.c_char_p
    return lib


def _call(lib, name, x, dy, shape):
    n, h, w, cin, cout = shape
    dw = torch.full((cout, 9 * cin), float("nan"), device="cuda")
    db = torch.full((cout,), float("nan"), device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = getattr(lib, name)(x.data_ptr(), dy.data_ptr(), n, h, w, cin, cout, dw.data_ptr(), db.data_ptr(), stream)
    assert rc == 0, lib.ivx_last_error().decode()
    torch.cuda.synchronize()
    return dw.cpu(), db.cpu()


def test_noalloc_weight_gradient_matches_the_allocating_call():
    lib = _lib()
    cap = lib.ivx_nn_conv3x3_grad_weight_noalloc_capacity()
    print(f"[noalloc] capacity {cap} floats", flush=True)
    for i, shape in enumerate(SHAPES):
        need = lib.ivx_nn_conv3x3_grad_weight_scratch_floats(*shape)
        assert 0 < need <= cap, (shape, need, cap)
        if i > 0:
            assert need < lib.ivx_nn_conv3x3_grad_weight_scratch_floats(*SHAPES[i - 1])
        n, h, w, cin, cout = shape
        rng = np.random.default_rng(100 + i)
        x = torch.tensor(rng.standard_normal((n, h, w, cin)), dtype=torch.float32, device="cuda")
        dy = torch.tensor(rng.standard_normal((n, h, w, cout)), dtype=torch.float32, device="cuda")
        want_dw, want_db = _call(lib, "ivx_nn_conv3x3_grad_weight", x, dy, shape)
        got_dw, got_db = _call(lib, "ivx_nn_conv3x3_grad_weight_noalloc", x, dy, shape)
        print(f"[noalloc] shape {shape}: {need} floats of partials, max |d dw| "
              f"{float((got_dw - want_dw).abs().max()):.3e}", flush=True)
        assert torch.isfinite(got_dw).all() and torch.isfinite(got_db).all()
        assert torch.equal(got_dw, want_dw), shape
        assert torch.equal(got_db, want_db), shape
