"""C-ABI checks that need no GPU: the library loads, exports every function
that include/spiir.h declares, and rejects bad arguments on the host before
anything reaches a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1602_05573_amd as pkg
from paper_1602_05573_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "spiir.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spiir_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libspiir.so missing: run __graft_entry__.build() first")
    return _lib.load()


def test_exports_match_header(lib):
    declared = header_functions()
    assert len(declared) >= 20
    assert sorted(_lib.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name), name


def test_version_and_empty_error(lib):
    assert b"gfx950" in lib.spiir_version()
    assert isinstance(lib.spiir_last_error(), bytes)


def test_opts_default(lib):
    o = _lib.default_opts()
    assert o.chunk_len == 256 and o.precision == 0 and o.device == -1 and o.max_block == 16384
    assert o.time_split == 0 and o.autotune == 0 and o.waves_per_group == 0


def _create(lib, T, off, a, b, d, **kw):
    o = _lib.default_opts()
    for k, v in kw.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    off = np.ascontiguousarray(off, np.int64)
    a = np.ascontiguousarray(a, np.complex128)
    b = np.ascontiguousarray(b, np.complex128)
    d = np.ascontiguousarray(d, np.int32)
    rc = lib.spiir_bank_create(ctypes.byref(h), T, off.ctypes.data_as(ctypes.c_void_p),
                               a.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p),
                               d.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o))
    return rc, h


GOOD = dict(T=2, off=[0, 2, 3], a=[0.5, 0.9j, -0.3 + 0.1j], b=[1, 1j, 0.5], d=[0, 3, 7])


@pytest.mark.parametrize("change,needle", [
    (dict(T=0), "n_templates"),
    (dict(off=[1, 2, 3]), "offsets[0]"),
    (dict(off=[0, 2, 2]), "no filters"),
    (dict(a=[0.5, 1.0, 0.1]), "not stable"),
    (dict(a=[0.5, 0.6 + 0.8j, 0.1]), "not stable"),
    (dict(a=[0.5, np.nan, 0.1]), "non-finite"),
    (dict(b=[1, np.inf, 0.5]), "non-finite"),
    (dict(d=[0, -1, 7]), "negative delay"),
    (dict(max_delay=5), "exceeds max_delay"),
    (dict(chunk_len=12), "chunk_len"),
    (dict(chunk_len=8192), "chunk_len"),
    (dict(filters_per_lane=5), "filters_per_lane"),
    (dict(precision=3), "precision"),
    (dict(waves_per_group=17), "waves_per_group"),
    (dict(time_split=33), "time_split"),
])
def test_create_rejects_bad_arguments(lib, change, needle):
    args = dict(GOOD)
    opts = {}
    for k, v in change.items():
        if k in args:
            args[k] = v
        else:
            opts[k] = v
    rc, h = _create(lib, args["T"], args["off"], args["a"], args["b"], args["d"], **opts)
    assert rc == _lib.SPIIR_EINVAL
    assert not h.value
    assert needle in lib.spiir_last_error().decode()


def test_null_arguments(lib):
    assert lib.spiir_bank_create(None, 1, None, None, None, None, None) == _lib.SPIIR_EINVAL
    h = ctypes.c_void_p()
    assert lib.spiir_bank_create(ctypes.byref(h), 1, None, None, None, None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_bank_destroy(None) == 0
    assert lib.spiir_tape_destroy(None) == 0
    assert lib.spiir_batch_destroy(None) == 0
    assert lib.spiir_filter_block(None, None, 0, None, 0, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_trigger_max(None, None, 0, None, None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_backward(None, None, None, None, None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_bank_get_info(None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_bank_time_kernels(None, 1) == _lib.SPIIR_EINVAL
    assert lib.spiir_batch_set_time_split(None, 0) == _lib.SPIIR_EINVAL
    assert lib.spiir_bank_kernel_time(None, None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_filter_block_z(None, None, 0, None, 0, None) == _lib.SPIIR_EINVAL
    mh = ctypes.c_void_p()
    assert lib.spiir_multirate_create(None, 2, 1, None, None, None, None, None, 4, None, 4, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_multirate_create(ctypes.byref(mh), 0, 1, None, None, None, None, None, 4, None, 4,
                                      None) == _lib.SPIIR_EINVAL
    assert "n_levels" in lib.spiir_last_error().decode()
    assert not mh.value
    assert lib.spiir_multirate_destroy(None) == 0
    assert lib.spiir_multirate_reset(None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_multirate_filter_block_z(None, None, 0, None, 0, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_multirate_trigger_max(None, None, 0, None, None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_multirate_level_bank(None, 0, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_multirate_set_graph(None, 1) == _lib.SPIIR_EINVAL
    wh = ctypes.c_void_p()
    assert lib.spiir_whitener_create(None, 64, 0, -1) == _lib.SPIIR_EINVAL
    for bad in (0, 8, 100, 16384):
        assert lib.spiir_whitener_create(ctypes.byref(wh), bad, 0, -1) == _lib.SPIIR_EINVAL
        assert "power of two" in lib.spiir_last_error().decode()
    assert lib.spiir_whitener_create(ctypes.byref(wh), 64, -1, -1) == _lib.SPIIR_EINVAL
    assert not wh.value
    assert lib.spiir_whitener_destroy(None) == 0
    assert lib.spiir_whitener_estimate_psd(None, None, 0, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_whitener_set_psd(None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_whitener_get_psd(None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_whitener_process(None, None, 0, None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_whitener_reset(None, None) == _lib.SPIIR_EINVAL
    th = ctypes.c_void_p()
    assert lib.spiir_trigger_stream_create(None, 1.0, 4, 16, -1) == _lib.SPIIR_EINVAL
    assert lib.spiir_trigger_stream_create(ctypes.byref(th), 1.0, -1, 16, -1) == _lib.SPIIR_EINVAL
    assert lib.spiir_trigger_stream_create(ctypes.byref(th), 1.0, 4, 0, -1) == _lib.SPIIR_EINVAL
    assert not th.value
    assert lib.spiir_trigger_stream_destroy(None) == 0
    assert lib.spiir_trigger_stream_reset(None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_trigger_stream_push(None, None, None, 0, None, None, None, 0, None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_trigger_stream_flush(None, None, None, None, 0, None, None) == _lib.SPIIR_EINVAL
    assert lib.spiir_batch_create(None, 1, None, None, None, None, None, 4096, None) == _lib.SPIIR_EINVAL
    bh = ctypes.c_void_p()
    assert lib.spiir_batch_create(ctypes.byref(bh), 0, None, None, None, None, None, 4096, None) == _lib.SPIIR_EINVAL
    L, F = ctypes.c_int32(), ctypes.c_int32()
    assert lib.spiir_autotune(0, None, None, None, None, None, 0, 4096, -1, ctypes.byref(L),
                              ctypes.byref(F), None) == _lib.SPIIR_EINVAL


def test_cluster_arguments(lib):
    """Clustering rejects bad sizes and null buffers on the host, and reports
    a workspace that grows with n."""
    nb = ctypes.c_size_t()
    assert lib.spiir_cluster_workspace_size(-1, ctypes.byref(nb)) == _lib.SPIIR_EINVAL
    assert lib.spiir_cluster_workspace_size(1 << 41, ctypes.byref(nb)) == _lib.SPIIR_EINVAL
    assert lib.spiir_cluster_workspace_size(10, None) == _lib.SPIIR_EINVAL
    sizes = []
    for n in (0, 1, 4096, 4097, 1 << 22):
        assert lib.spiir_cluster_workspace_size(n, ctypes.byref(nb)) == 0
        sizes.append(nb.value)
    assert sizes == sorted(sizes) and sizes[1] > 0
    # (1<<22)/64 block maxima + masks and (1<<22)/4096 counts and offsets
    assert sizes[-1] >= (1 << 16) * 12 + (1 << 10) * 16
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails on the host
    C = lib.spiir_cluster_triggers
    assert C(fake, fake, 10, 1.0, 4, fake, 1 << 20, fake, fake, fake, 4, None, -1, None) == _lib.SPIIR_EINVAL
    assert "count" in lib.spiir_last_error().decode()
    assert C(fake, fake, -1, 1.0, 4, fake, 1 << 20, fake, fake, fake, 4, fake, -1, None) == _lib.SPIIR_EINVAL
    assert C(fake, fake, 10, 1.0, -1, fake, 1 << 20, fake, fake, fake, 4, fake, -1, None) == _lib.SPIIR_EINVAL
    assert "window" in lib.spiir_last_error().decode()
    assert C(fake, fake, 10, 1.0, 4, fake, 1 << 20, fake, fake, fake, -1, fake, -1, None) == _lib.SPIIR_EINVAL
    assert C(fake, fake, 10, 1.0, 4, fake, 1 << 20, None, fake, fake, 4, fake, -1, None) == _lib.SPIIR_EINVAL
    assert C(None, fake, 10, 1.0, 4, fake, 1 << 20, fake, fake, fake, 4, fake, -1, None) == _lib.SPIIR_EINVAL
    assert C(fake, fake, 10, 1.0, 4, None, 1 << 20, fake, fake, fake, 4, fake, -1, None) == _lib.SPIIR_EINVAL
    lib.spiir_cluster_workspace_size(10000, ctypes.byref(nb))
    assert C(fake, fake, 10000, 1.0, 4, fake, nb.value - 1, fake, fake, fake, 4, fake, -1,
             None) == _lib.SPIIR_EINVAL
    assert "workspace" in lib.spiir_last_error().decode()


def test_multirate_create_arguments(lib):
    """Argument errors of the multi-rate bank are found on the host."""
    T = 2
    off0 = np.array([0, 1, 2], np.int64)
    off1 = np.array([0, 0, 1], np.int64)
    a = np.array([0.5, 0.3j, 0.1], np.complex128)
    b = np.ones(3, np.complex128)
    d = np.zeros(3, np.int32)
    h = np.ones(4) / 4
    VP = ctypes.c_void_p * 2
    offs = VP(off0.ctypes.data, off1.ctypes.data)
    aa = VP(a.ctypes.data, a.ctypes.data)
    bb = VP(b.ctypes.data, b.ctypes.data)
    dd = VP(d.ctypes.data, d.ctypes.data)
    hp = h.ctypes.data_as(ctypes.c_void_p)
    mh = ctypes.c_void_p()
    C = lib.spiir_multirate_create
    assert C(ctypes.byref(mh), 2, T, offs, aa, bb, dd, hp, 0, hp, 4, None) == _lib.SPIIR_EINVAL
    assert "taps" in lib.spiir_last_error().decode()
    assert C(ctypes.byref(mh), 2, T, offs, aa, bb, dd, hp, 4, hp, 65, None) == _lib.SPIIR_EINVAL
    hn = np.array([1.0, np.nan, 0.0, 0.0])
    assert C(ctypes.byref(mh), 2, T, offs, aa, bb, dd, hn.ctypes.data_as(ctypes.c_void_p), 4, hp, 4,
             None) == _lib.SPIIR_EINVAL
    assert "non-finite" in lib.spiir_last_error().decode()
    bad = np.array([0, 2, 1], np.int64)
    assert C(ctypes.byref(mh), 2, T, VP(off0.ctypes.data, bad.ctypes.data), aa, bb, dd, hp, 4, hp, 4,
             None) == _lib.SPIIR_EINVAL
    assert "decrease" in lib.spiir_last_error().decode()
    zero = np.zeros(3, np.int64)
    assert C(ctypes.byref(mh), 2, T, VP(zero.ctypes.data, zero.ctypes.data), aa, bb, dd, hp, 4, hp, 4,
             None) == _lib.SPIIR_EINVAL
    assert "no level" in lib.spiir_last_error().decode()
    assert C(ctypes.byref(mh), 2, T, offs, VP(a.ctypes.data, None), bb, dd, hp, 4, hp, 4,
             None) == _lib.SPIIR_EINVAL
    assert not mh.value


def test_no_device_reported_cleanly(lib):
    """With valid arguments and no GPU, creation fails with ENODEV (never a fallback)."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    rc, h = _create(lib, GOOD["T"], GOOD["off"], GOOD["a"], GOOD["b"], GOOD["d"])
    assert rc == _lib.SPIIR_ENODEV
    assert not h.value
    fake = ctypes.c_void_p(0x1000)
    assert lib.spiir_cluster_triggers(None, None, 0, 1.0, 4, None, 0, None, None, None, 0, fake, -1,
                                      None) == _lib.SPIIR_ENODEV


def test_package_has_no_cpu_fallback():
    # the binding holds only marshalling code: no oracle import, no numpy recursion
    pkgdir = os.path.dirname(pkg.__file__)
    for fn in os.listdir(pkgdir):
        if fn.endswith(".py"):
            src = open(os.path.join(pkgdir, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn
