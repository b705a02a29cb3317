"""The C-ABI library loads, exports every symbol include/n2f.h declares, and
its host-only entry points behave (no GPU needed for any of these)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2108_10209_amd import n2f, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "n2f.h")

pytestmark = pytest.mark.skipif(not os.path.exists(n2f.LIB_PATH), reason="libn2f.so not built")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(n2f_[a-z_]+)\s*\(", text)))


def test_header_declares_binding_symbols():
    assert _declared() == sorted(n2f.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(n2f.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_config_default_is_the_papers():
    c = n2f.default_config()
    assert (c.n_layers, c.width, c.patience) == (8, 64, 100)
    assert abs(c.lr - 1e-3) < 1e-9 and abs(c.beta1 - 0.9) < 1e-7 and abs(c.beta2 - 0.999) < 1e-7
    assert abs(c.eps - 1e-8) < 1e-15
    assert list(c.pair_order) == [0, 1, 2, 3] and c.precision == n2f.FP32 and c.fixed_epochs == 0


@pytest.mark.parametrize("C", [1, 3])
def test_param_count(C):
    assert n2f.param_count(C) == synth.n_params(C)


@pytest.mark.parametrize("C,seed", [(1, 0), (3, 12345), (1, 2 ** 63 + 7)])
def test_library_init_equals_generator(C, seed):
    """The library's built-in initial weights are the generator's, bit for
    bit: both implement SplitMix64 from its published definition."""
    a = n2f.init_params(C, seed)
    b = synth.init_params(C, seed)
    assert a.dtype == b.dtype == np.float32
    np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))


def test_workspace_bytes_scales_and_rejects():
    small = n2f.workspace_bytes(64, 64, 1)
    big = n2f.workspace_bytes(512, 512, 1)
    assert 0 < small < big
    assert n2f.workspace_bytes(512, 512, 3) > big
    # activation stash of 8 layers x 64 channels x P pixels dominates
    assert big >= 8 * 64 * (512 * 256) * 4
    for H, W, C in [(1, 8, 1), (8, 1, 1), (8, 8, 0), (8, 8, 4)]:
        with pytest.raises(n2f.N2FError) as e:
            n2f.workspace_bytes(H, W, C)
        assert e.value.code == n2f.EINVAL


def test_config_validation():
    for kw in [dict(n_layers=7), dict(width=40), dict(width=512), dict(lr=0.0), dict(beta1=1.0), dict(patience=0),
               dict(max_epochs=0), dict(pair_order=(0, 0, 1, 2)), dict(precision=7), dict(downsample=2),
               dict(exact_targets=2), dict(wgrad_splits=-1), dict(wgrad_splits=257)]:
        with pytest.raises(n2f.N2FError) as e:
            n2f.workspace_bytes(8, 8, 1, n2f.default_config(**kw))
        assert e.value.code == n2f.EINVAL


def test_wgrad_splits_shrink_the_partials():
    """Fewer weight-gradient splits need less workspace: the partial rows of
    the seven 64->64 layers (9 * 64 * 64 + 64 floats each per split)."""
    base = n2f.workspace_bytes(1024, 1024, 1, n2f.default_config(precision=n2f.BF16))
    assert n2f.default_config().wgrad_splits == 0
    for k in (16, 32):
        b = n2f.workspace_bytes(1024, 1024, 1, n2f.default_config(precision=n2f.BF16, wgrad_splits=k))
        assert b < base
        assert base - b >= 7 * (64 - k) * (9 * 64 * 64 + 64) * 4


def test_null_arguments_rejected_without_device():
    L = n2f.lib()
    cfg = n2f.default_config()
    run = ctypes.c_void_p()
    st = L.n2f_run_create(ctypes.byref(run), None, 8, 8, 1, ctypes.byref(cfg), None, 0, None)
    assert st == n2f.EINVAL and b"NULL" in L.n2f_last_error()
    assert L.n2f_train_step(None, 0, 0) == n2f.EINVAL
    assert L.n2f_result(None, None) == n2f.EINVAL


def test_ablation_workspaces():
    """2x2 blocks halve the training pixels (so the stash); exact targets add
    four target images of C x P floats."""
    base = n2f.workspace_bytes(512, 512, 1)
    quad = n2f.workspace_bytes(512, 512, 1, n2f.default_config(downsample=n2f.DS_QUAD))
    assert quad < base and quad >= 8 * 64 * (256 * 256) * 4
    ex = n2f.workspace_bytes(512, 512, 3, n2f.default_config(exact_targets=1))
    assert ex - n2f.workspace_bytes(512, 512, 3) >= 4 * 3 * (512 * 256) * 4
    # smallest images still plan: 2x2 gives 1x1 block images
    assert n2f.workspace_bytes(2, 2, 1, n2f.default_config(downsample=n2f.DS_QUAD)) > 0
    assert n2f.workspace_bytes(3, 3, 2, n2f.default_config(downsample=n2f.DS_QUAD, exact_targets=1)) > 0


def test_exact_targets_refused_where_no_clean_image_fits():
    L = n2f.lib()
    cfg = n2f.default_config(exact_targets=1)
    assert L.n2f_denoise(None, None, 8, 8, 1, ctypes.byref(cfg), None, 0, None) == n2f.EINVAL
    assert b"clean" in L.n2f_last_error()
    srv = ctypes.c_void_p()
    assert L.n2f_server_create(ctypes.byref(srv), ctypes.byref(cfg), None, 1 << 30, 1, 4,
                               n2f.SERVER_SIMULATE) == n2f.EINVAL
    b = ctypes.c_void_p()
    one = (ctypes.c_int * 1)(8)
    ptrs = (ctypes.c_void_p * 1)(None)
    assert L.n2f_batch_create(ctypes.byref(b), 1, ptrs, one, one, (ctypes.c_int * 1)(1), ctypes.byref(cfg),
                              ctypes.c_void_p(256), 1 << 20, 1, None) == n2f.EINVAL
    assert L.n2f_run_set_clean(None, None) == n2f.EINVAL


def test_max_project_argument_checks_without_device():
    L = n2f.lib()
    assert L.n2f_max_project(None, 3, 16, None, None) == n2f.EINVAL
    p = ctypes.c_void_p(1 << 20)
    assert L.n2f_max_project(p, 0, 16, ctypes.c_void_p(1 << 24), None) == n2f.EINVAL
    assert L.n2f_max_project(p, 2, 0, ctypes.c_void_p(1 << 24), None) == n2f.EINVAL
    # output inside the stack
    assert L.n2f_max_project(p, 2, 16, ctypes.c_void_p((1 << 20) + 64), None) == n2f.EINVAL
    assert b"overlaps" in L.n2f_last_error()


def test_noalloc_rejects_before_touching_the_device():
    """The allocation-free entry point checks its arguments and the fixed
    workspace's size on the host first: a NULL pointer is N2F_EINVAL and an
    image whose workspace exceeds N2F_NOALLOC_MAX_BYTES is N2F_ENOMEM."""
    L = n2f.lib()
    cfg = n2f.default_config(precision=n2f.BF16)
    fake = ctypes.c_void_p(256)
    assert L.n2f_denoise_noalloc(None, fake, 64, 64, 1, ctypes.byref(cfg), None) == n2f.EINVAL
    assert n2f.workspace_bytes(1024, 1024, 1, cfg) > n2f.NOALLOC_MAX_BYTES
    assert L.n2f_denoise_noalloc(fake, fake, 1024, 1024, 1, ctypes.byref(cfg), None) == n2f.ENOMEM
    assert b"fixed device array" in L.n2f_last_error()
    assert n2f.workspace_bytes(256, 256, 1, cfg) <= n2f.NOALLOC_MAX_BYTES


@pytest.mark.parametrize("C", [1, 3])
def test_literal_widths_parameters(C):
    """Per-layer widths (the Methods' 32, ..., 256): the library's parameter
    count and initial weights equal the generator's for that net, and its
    workspace grows accordingly."""
    cfg = n2f.default_config(widths=n2f.LITERAL_WIDTHS)
    assert n2f.param_count(C, cfg) == synth.n_params(C, synth.LITERAL_WIDTHS)
    a = n2f.init_params(C, 11, cfg)
    b = synth.init_params(C, 11, synth.LITERAL_WIDTHS)
    np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
    assert n2f.workspace_bytes(64, 64, C, cfg) > n2f.workspace_bytes(64, 64, C)


def test_widths_are_checked():
    for bad in [(32, 32, 64, 64, 128, 128, 256, 512), (24,) * 8, (32, 32, 64, 64, 128, 128, 256, 0)]:
        cfg = n2f.default_config(widths=bad)
        with pytest.raises(n2f.N2FError) as e:
            n2f.workspace_bytes(64, 64, 1, cfg)
        assert e.value.code == n2f.EINVAL
    assert n2f.param_count(1, n2f.default_config(width=32)) == synth.n_params(1, 32)
