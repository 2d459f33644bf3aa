"""C ABI checks that need no GPU: every function declared in include/rbfs.h
is exported by librbfs.so and bound in the Python layer, and argument
validation / no-device paths return the documented codes."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2012_10026_amd as rb

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "rbfs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbfs_[a-z_0-9]+)\s*\(", text)))


def test_header_functions_exported_and_bound():
    names = declared_functions()
    assert len(names) >= 19
    L = rb.lib()
    for name in names:
        assert hasattr(L, name), name
        assert name in rb.SIGNATURES, name


def gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_argument_validation_without_device():
    L = rb.lib()
    out = ctypes.c_void_p()
    off = np.array([0, 1, 2], np.int64)
    cols = np.array([1, 0], np.int32)
    p_off = off.ctypes.data_as(ctypes.c_void_p)
    p_cols = cols.ctypes.data_as(ctypes.c_void_p)
    assert L.rbfs_graph_create(-1, 2, p_off, p_cols, rb.HOST_PTRS, None,
                               ctypes.byref(out)) == -2
    assert L.rbfs_graph_create(2, 2, None, p_cols, rb.HOST_PTRS, None, ctypes.byref(out)) == -1
    assert L.rbfs_graph_create(2, 2, p_off, p_cols, rb.HOST_PTRS, None, None) == -1
    assert L.rbfs_graph_create(2, 2, p_off, p_cols, 1 << 7, None, ctypes.byref(out)) == -1
    bad = np.array([0, 1, 3], np.int64)  # offsets do not end at nnz
    assert L.rbfs_graph_create(2, 2, bad.ctypes.data_as(ctypes.c_void_p), p_cols,
                               rb.HOST_PTRS, None, ctypes.byref(out)) == -1
    assert L.rbfs_bfs(None, 0, None, None, None, None, None) == -1
    assert L.rbfs_bfs_batch(None, None, 0, None, None, None, None, None) == -1
    assert L.rbfs_rcm_reorder(None, None, None, None) == -1
    assert L.rbfs_graph_destroy(None) == 0
    assert L.rbfs_multi_destroy(None) == 0
    assert L.rbfs_switch_load(None, 3) == -1
    assert L.rbfs_mlp_train(None, 0, None, None, 0, 0, ctypes.c_float(0.0), None, None,
                            None) == -1
    assert rb.lib().rbfs_last_error()  # message set


@pytest.mark.skipif(gpu_present(), reason="checks the no-device path")
def test_no_device_codes():
    L = rb.lib()
    out = ctypes.c_void_p()
    off = np.array([0, 1, 2], np.int64)
    cols = np.array([1, 0], np.int32)
    rc = L.rbfs_graph_create(2, 2, off.ctypes.data_as(ctypes.c_void_p),
                             cols.ctypes.data_as(ctypes.c_void_p), rb.HOST_PTRS, None,
                             ctypes.byref(out))
    assert rc == -6
    d = rb.DeviceInfo()
    assert L.rbfs_device_info(ctypes.byref(d)) == -6
    with pytest.raises(rb.RbfsError) as e:
        rb.device_info()
    assert e.value.code == -6


def test_struct_sizes_match_header():
    """rbfs_opts_t layout the binding assumes: 4 x int32, pointer, 3 x int32."""
    assert ctypes.sizeof(rb.Opts) == 40
    assert rb.Opts.schedule.offset == 16 and rb.Opts.flags.offset == 32


def test_set_allocator_arguments_without_device():
    L = rb.lib()
    cb = ctypes.cast(rb._torch_alloc_cb, ctypes.c_void_p)
    # one function without the other
    assert L.rbfs_set_allocator(cb, None, None) == -1
    assert L.rbfs_set_allocator(None, cb, None) == -1
    before = rb.allocator()
    rb.set_allocator("hip")
    assert rb.allocator() == "hip"
    rb.set_allocator("torch")
    assert rb.allocator() == "torch"
    rb.set_allocator(before)
    with pytest.raises(ValueError):
        rb.set_allocator("cuda")


def test_switch_blob_layout_matches_the_oracle():
    """make_switch_blob writes the weights, the training feature range, the
    largest training level and the margin where the oracle's decision reads
    them (both follow the 1428-float layout of rbfs_switch_load)."""
    from oracle import mlp
    assert rb.SWITCH_BLOB == mlp.BLOB == 1428 and rb.MLP_PARAMS == mlp.NPARAMS == 1410
    rng = np.random.default_rng(3)
    w = rng.standard_normal(rb.MLP_PARAMS).astype(np.float32)
    rows = rng.uniform(-1, 1, size=(50, 11)).astype(np.float32)
    rows[:, 10] = rng.integers(1, 9, size=50)
    blob = rb.make_switch_blob(w, rows, margin=0.3)
    assert np.array_equal(blob[:mlp.NPARAMS], w)
    assert np.array_equal(blob[mlp.NPARAMS:mlp.NPARAMS + 8], rows[:, :8].min(axis=0))
    assert np.array_equal(blob[mlp.NPARAMS + 8:mlp.NPARAMS + 16], rows[:, :8].max(axis=0))
    assert blob[mlp.NPARAMS + 16] == rows[:, 10].max()
    assert blob[mlp.BLOB - 1] == np.float32(0.3)
    assert rb.make_switch_blob(w, rows)[mlp.BLOB - 1] == np.float32(0.1)  # the default
