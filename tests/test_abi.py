"""The C ABI on the CPU: the library loads, exports every symbol include/ivx.h declares,
its descriptor matches the header's layout, and argument checking happens before any
device call (no kernel runs here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2609_17636_amd as ivx
from paper_2609_17636_amd import IvxError, Plan, load_library

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ivx.h")


def _declared():
    import glob

    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(ivx_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_library_exports_every_declared_symbol(precision):
    lib = load_library(precision)
    names = _declared()
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
    assert lib.ivx_version() == 5
    assert lib.ivx_real_size() == (4 if precision == "f32" else 8)


@pytest.mark.parametrize("real_double", [False, True])
def test_descriptor_layout_matches_header(tmp_path, real_double):
    c = tmp_path / "probe.c"
    c.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ivx.h"\n'
                 'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(ivx_problem),'
                 ' offsetof(ivx_problem, sd_fwhm_rad), offsetof(ivx_problem, reserved), sizeof(ivx_real));'
                 'return 0;}\n')
    exe = tmp_path / "probe"
    cmd = ["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)]
    if real_double:
        cmd.insert(1, "-DIVX_REAL_DOUBLE")
    subprocess.run(cmd, check=True)
    size, off_fwhm, off_res, rs = map(int, subprocess.run([str(exe)], capture_output=True, text=True,
                                                           check=True).stdout.split())
    assert size == ctypes.sizeof(ivx._Problem)
    assert off_fwhm == ivx._Problem.sd_fwhm_rad.offset
    assert off_res == ivx._Problem.reserved.offset
    assert rs == (8 if real_double else 4)


def test_solver_structs_match_header(tmp_path):
    """The solver's options and result as the ctypes binding lays them out."""
    from paper_2609_17636_amd.solver import _LbOptions, _LbResult

    c = tmp_path / "probe_lb.c"
    c.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ivx_lbfgsb.h"\n'
                 'int main(void){printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(ivx_lbfgsb_options),'
                 ' offsetof(ivx_lbfgsb_options, stream_wait), offsetof(ivx_lbfgsb_options, ftol),'
                 ' offsetof(ivx_lbfgsb_options, target), sizeof(ivx_lbfgsb_result),'
                 ' offsetof(ivx_lbfgsb_result, n_walks));return 0;}\n')
    exe = tmp_path / "probe_lb"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()))
    assert got == [ctypes.sizeof(_LbOptions), _LbOptions.stream_wait.offset, _LbOptions.ftol.offset,
                   _LbOptions.target.offset, ctypes.sizeof(_LbResult), _LbResult.n_walks.offset]


def _args(**over):
    a = dict(n_chan=1, n_sky=64, pixel_rad=1e-4, n_point=1, n_sub=64,
             vis_offsets=np.array([0, 10], dtype=np.int64), flux_scale=np.array([1.0]))
    a.update(over)
    return a


@pytest.mark.parametrize("bad", [
    dict(n_sub=63), dict(n_sub=2), dict(n_chan=0), dict(pixel_rad=-1.0), dict(pixel_rad=float("nan")),
    dict(vis_offsets=np.array([0, 10, 5], dtype=np.int64), n_chan=2, flux_scale=np.array([1.0, 1.0])),
    dict(vis_offsets=np.array([3, 10], dtype=np.int64)), dict(lambda_r=-1.0), dict(kernel_width=3),
    dict(kernel_width=17), dict(fine_size=100), dict(fine_size=64, n_sub=64), dict(tile=4),
    dict(sd_n=64, sd_stride=2, sd_offset=1, sd_fwhm_rad=1e-3, sd_sigma=1.0),
    dict(sd_n=8, sd_stride=8, sd_offset=4, sd_fwhm_rad=0.0, sd_sigma=1.0),
    dict(flux_scale=np.array([np.inf])),
])
def test_plan_create_rejects_bad_descriptors(bad):
    with pytest.raises(IvxError) as e:
        Plan(**_args(**bad))
    assert e.value.code == -1
    assert ivx.load_library().ivx_last_error().decode()


def test_plan_create_chooses_parameters():
    p = Plan(**_args())
    info = p.info()
    assert info["n_fine"] == 128 and info["kernel_width"] == 8
    assert info["tile"] >= info["kernel_width"]
    assert info["window"] == info["tile"] + info["kernel_width"] - 1
    p64 = Plan(**_args(), precision="f64")
    assert p64.info()["kernel_width"] >= 12
    explicit = Plan(**_args(kernel_width=6, fine_size=256, tile=16))
    assert (explicit.info()["n_fine"], explicit.info()["kernel_width"], explicit.info()["tile"]) == (256, 6, 16)


def test_evaluation_before_data_is_a_state_error():
    lib = load_library()
    p = Plan(**_args())
    terms = np.zeros(4)
    code = lib.ivx_objective_grad(p._h, ctypes.c_void_p(16), ctypes.c_void_p(16), terms.ctypes.data, None)
    assert code == -5
    assert "set_data" in lib.ivx_last_error().decode()
    assert lib.ivx_forward(p._h, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == -5
    assert lib.ivx_adjoint(p._h, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == -5


def test_null_handling():
    lib = load_library()
    assert lib.ivx_plan_destroy(None) == 0
    out = ctypes.c_void_p()
    assert lib.ivx_plan_create(None, ctypes.byref(out)) == -1
    assert out.value is None
    assert lib.ivx_objective_grad(None, None, None, None, None) == -1


def test_shared_uv_arguments_are_checked_before_any_device_call():
    """ivx_plan_set_data_shared needs equal counts in every channel of a pointing and
    finite, positive channel scales; both are checked on the host."""
    offs = np.array([0, 10, 20, 35, 50], dtype=np.int64)  # 2 pointings x 2 channels
    plan = Plan(2, 32, 1e-4, 2, 32, offs, np.ones(2))
    uv = np.zeros((25, 2), np.float32)
    w = np.ones(25, np.float32)
    vis = np.zeros((50, 2), np.float32)
    beams = np.ones((2, 32, 32), np.float32)
    interp = np.zeros((2, 32, 32, 2), np.float32)
    for scale in ([1.0, 0.0], [1.0, -1.0], [1.0, float("nan")]):
        with pytest.raises(IvxError) as e:
            plan.set_data_shared(uv, w, scale, vis, beams, interp)
        assert e.value.code == -1 and "uv_scale" in str(e.value)
    bad = np.array([0, 10, 21, 35, 50], dtype=np.int64)  # pointing 0: 10 and 11 samples
    plan2 = Plan(2, 32, 1e-4, 2, 32, bad, np.ones(2))
    with pytest.raises(IvxError) as e:
        plan2.set_data_shared(uv, w, [1.0, 1.01], vis, beams, interp)
    assert e.value.code == -1 and "same visibility count" in str(e.value)


def test_noalloc_weight_gradient_rejects_shapes_beyond_its_scratch():
    """The allocation-free weight gradient refuses, before any device work, a shape whose
    split partials exceed its static array (CPU: the check precedes every HIP call)."""
    import ctypes

    import paper_2609_17636_amd as ivx

    lib = ivx.load_library("f32")
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    f = lib.ivx_nn_conv3x3_grad_weight_noalloc
    f.argtypes = [vp, vp, i32, i32, i32, i32, i32, vp, vp, vp]
    f.restype = ctypes.c_int
    lib.ivx_nn_conv3x3_grad_weight_noalloc_capacity.restype = ctypes.c_int64
    lib.ivx_nn_conv3x3_grad_weight_scratch_floats.argtypes = [i32] * 5
    lib.ivx_nn_conv3x3_grad_weight_scratch_floats.restype = ctypes.c_int64
    cap = lib.ivx_nn_conv3x3_grad_weight_noalloc_capacity()
    shape = (1, 64, 64, 256, 256)
    assert lib.ivx_nn_conv3x3_grad_weight_scratch_floats(*shape) > cap
    code = f(ctypes.c_void_p(16), ctypes.c_void_p(16), *shape, ctypes.c_void_p(16), ctypes.c_void_p(16), None)
    assert code == -1
    msg = lib.ivx_last_error().decode()
    assert "static scratch" in msg and str(cap) in msg
    assert f(None, None, *shape, None, None, None) == -1


def test_nufft_probe_is_monotone_and_brackets_the_widths():
    """The accuracy probe of the autotuner falls with the kernel width and with the
    oversampling factor, and places the widths the library uses on the right side of its
    accuracy targets (sigma = 2: W = 8 below 1e-6, W = 6 above 1e-5)."""
    import paper_2609_17636_amd as ivx

    for nk, nf in ((64, 128), (384, 1024), (384, 512)):
        e = [ivx.nufft_probe(nk, nf, W) for W in range(4, 13)]
        assert all(a > b for a, b in zip(e, e[1:])), (nk, nf, e)
    assert ivx.nufft_probe(64, 256, 7) < ivx.nufft_probe(64, 128, 7) < ivx.nufft_probe(96, 128, 7)
    assert ivx.nufft_probe(64, 128, 8) < 1e-6 < 1e-5 < ivx.nufft_probe(64, 128, 6)


def test_full_model_needs_data_and_checks_its_arguments():
    """ivx_plan_set_w before set_data is a state error; the plan stays coplanar."""
    p = Plan(**_args())
    with pytest.raises(IvxError) as e:
        p.set_w(np.zeros(10, np.float32))
    assert e.value.code == -5 and "set_data" in str(e.value)
    assert p.w_info()["enabled"] is False
    lib = load_library()
    assert lib.ivx_plan_set_w(None, None, 0, 0.0, None) == -1
    assert lib.ivx_plan_w_info(None, None) == -1


@pytest.mark.parametrize("n,end_bit", [(-1, 64), (2 ** 31, 64), (10, 0), (10, 65)])
def test_sort_rejects_bad_sizes_before_any_device_call(n, end_bit):
    lib = load_library()
    assert lib.ivx_sort_u64(None, None, None, None, n, end_bit, None) == -1
    assert "ivx_sort_u64" in lib.ivx_last_error().decode()


def test_sort_of_nothing_is_a_no_op():
    lib = load_library()
    assert lib.ivx_sort_u64(None, None, None, None, 0, 64, None) == 0
    # a non-empty sort without arrays is refused, still before any device call
    assert lib.ivx_sort_u64(None, None, None, None, 5, 64, None) == -1
