"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point include/dtb.h declares, and host-side validation rejects bad
inputs with DTB_ERR_INVALID (validation runs before any device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

import netgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "dtb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dtb_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2308_01241_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2308_01241_amd import build
        build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert "dtb_create" in names and "dtb_step" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in include/dtb.h but not exported"
    from paper_2308_01241_amd._lib import SIGNATURES
    assert set(SIGNATURES) == set(names), "binding and header disagree"


def test_abi_version_and_bitmap_words(lib):
    assert lib.dtb_abi_version() == 14
    assert [lib.dtb_bitmap_words(n) for n in (0, 1, 32, 33, 64)] == [0, 1, 1, 2, 2]
    assert isinstance(lib.dtb_last_error(), bytes)


def test_null_handles_are_rejected(lib):
    assert lib.dtb_step(None, 1) == -1
    assert lib.dtb_sync(None) == -1
    lib.dtb_destroy(None)  # NULL-safe


def _base():
    return netgen.make_network(netgen.small_net(n=40, k_in=7, k_cross=3))


def _mutations():
    def col_oob(n):
        n.col[5] = n.n
    def delay_zero(n):
        n.delay[3] = 0
    def delay_big(n):
        n.delay[3] = n.max_delay + 1
    def w_neg(n):
        n.w[7] = -0.1
    def w_nan(n):
        n.w[7] = np.nan
    def v0_inf(n):
        n.V0[2] = np.inf
    def region_oob(n):
        n.region[1] = n.n_regions
    def rowptr_dec(n):
        n.row_ptr[3], n.row_ptr[4] = n.row_ptr[4], n.row_ptr[3]
    def reset_above(n):
        n.ptypes[0, 4] = n.ptypes[0, 3] + 1.0
    def cap_zero(n):
        n.ptypes[0, 0] = 0.0
    def maxdelay_32(n):
        n.max_delay = 32
    def lam_big(n):
        n.bg_lambda = 1000.0
    def tau_zero(n):
        n.tau_ms[1] = 0.0
    def inh_two(n):
        n.is_inh[0] = 2
    def ptype_oob(n):
        n.ptype[0] = 1
    return [col_oob, delay_zero, delay_big, w_neg, w_nan, v0_inf, region_oob, rowptr_dec,
            reset_above, cap_zero, maxdelay_32, lam_big, tau_zero, inh_two, ptype_oob]


@pytest.mark.parametrize("kw", [{"unroll": 4}, {"unroll": -1}, {"bundle_syn": 100}, {"bundle_syn": 1 << 20},
                                {"fuse": 3}, {"fuse": -1}, {"events": 3}, {"events": -1}],
                         ids=lambda k: "_".join(f"{a}{b}" for a, b in k.items()))
def test_invalid_launch_shapes_are_rejected(lib, kw):
    from paper_2308_01241_amd import DtbError, Net
    with pytest.raises(DtbError) as ei:
        Net(_base(), **kw)
    assert ei.value.status == -1


@pytest.mark.parametrize("mut", _mutations(), ids=lambda f: f.__name__)
def test_invalid_inputs_are_rejected(lib, mut):
    from paper_2308_01241_amd import DtbError, Net
    net = _base()
    mut(net)
    with pytest.raises(DtbError) as ei:
        Net(net)
    assert ei.value.status == -1
    assert len(str(ei.value)) > len("DTB_ERR_INVALID: ")


def test_record_steps_zero_is_rejected(lib):
    from paper_2308_01241_amd import DtbError, Net
    with pytest.raises(DtbError) as ei:
        Net(_base(), record_steps=0)
    assert ei.value.status == -1


def test_validation_message_names_the_index(lib):
    from paper_2308_01241_amd import DtbError, Net
    net = _base()
    net.col[123] = -4
    with pytest.raises(DtbError, match="synapse 123"):
        Net(net)


def test_bit_packing_roundtrip():
    from paper_2308_01241_amd import pack_bits, unpack_bits
    rng = np.random.default_rng(1)
    for n in (1, 31, 32, 33, 1000):
        r = (rng.random((5, n)) < 0.2).astype(np.uint8)
        words = (n + 31) // 32
        b = pack_bits(r, words)
        np.testing.assert_array_equal(unpack_bits(b, n), r)
        i = int(np.argmax(r[0])) if r[0].any() else None
        if i is not None:
            assert (int(b[0, i >> 5]) >> (i & 31)) & 1 == 1


def test_remote_and_enkf_validation_without_a_gpu(lib):
    P = ctypes.c_void_p
    assert lib.dtb_set_remote_block(None, 10, 0, None, None, None, None, None) == -1
    assert lib.dtb_push_remote_spikes(None, None, 1) == -1
    fake = P(16)            # never dereferenced: validation fails first
    r = np.ones(65, np.float32)
    rp = P(r.ctypes.data)
    # null arrays, too many observations, one member, inflation below 1, r <= 0
    assert lib.dtb_enkf_analysis(4, 3, 2, None, fake, fake, rp, 1.0, 0, 0, 0.0, 1.0, None) == -1
    assert lib.dtb_enkf_analysis(4, 3, 65, fake, fake, fake, rp, 1.0, 0, 0, 0.0, 1.0, None) == -1
    assert lib.dtb_enkf_analysis(1, 3, 2, fake, fake, fake, rp, 1.0, 0, 0, 0.0, 1.0, None) == -1
    assert lib.dtb_enkf_analysis(4, 3, 2, fake, fake, fake, rp, 0.5, 0, 0, 0.0, 1.0, None) == -1
    assert lib.dtb_enkf_analysis(4, 3, 2, fake, fake, fake, rp, 1.0, 0, 0, 2.0, 1.0, None) == -1
    bad = np.array([1.0, 0.0], np.float32)
    assert lib.dtb_enkf_analysis(4, 3, 2, fake, fake, fake, P(bad.ctypes.data), 1.0, 0, 0, 0.0, 1.0, None) == -1
    # LDS beyond 160 KB is unsupported, before any launch
    assert lib.dtb_enkf_analysis(4096, 8, 64, fake, fake, fake, rp, 1.0, 0, 0, 0.0, 1.0, None) == -6


def test_checkpoint_validation_without_a_gpu(lib):
    used = ctypes.c_size_t(0)
    assert lib.dtb_save(None, None, 0, ctypes.byref(used)) == -1
    assert lib.dtb_load(None, None, 0) == -1


def test_autotune_rejects_bad_arguments_before_any_device_call(lib):
    from paper_2308_01241_amd._lib import Desc, TuneResult
    res = TuneResult()
    d = (Desc * 1)()
    cands = (ctypes.c_int32 * 9)(*([65536] * 9))
    assert lib.dtb_autotune(None, 1, None, None, None, 0, 0, 10, ctypes.byref(res)) == -1
    assert lib.dtb_autotune(d, 0, None, None, None, 0, 0, 10, ctypes.byref(res)) == -1
    assert lib.dtb_autotune(d, 1, None, None, cands, 9, 0, 10, ctypes.byref(res)) == -1   # > 8 candidates
    bad = (ctypes.c_int32 * 1)(100)
    assert lib.dtb_autotune(d, 1, None, None, bad, 1, 0, 10, ctypes.byref(res)) == -1     # below 4096
    assert lib.dtb_autotune(d, 1, None, None, None, 0, 0, 0, ctypes.byref(res)) == -1     # no timed step
    assert lib.dtb_autotune(d, 1, None, None, None, 0, -1, 10, ctypes.byref(res)) == -1   # negative burn-in
    assert lib.dtb_autotune(d, 1, None, None, None, 0, 0, 10, None) == -1
    assert b"candidate" in lib.dtb_last_error() or b"burnin" in lib.dtb_last_error() or lib.dtb_last_error()


def test_topk_noalloc_validates_before_any_device_call(lib):
    s = np.zeros(4097, np.float32)
    idx = np.zeros(8, np.int32)
    assert lib.dtb_topk_noalloc(s.ctypes.data, 4097, 1, idx.ctypes.data, None) == -1
    assert b"4096" in lib.dtb_last_error()
    assert lib.dtb_topk_noalloc(None, 4, 1, idx.ctypes.data, None) == -1
    assert lib.dtb_topk_noalloc(s.ctypes.data, 4, 5, idx.ctypes.data, None) == -1
    assert lib.dtb_topk_noalloc(s.ctypes.data, 0, 0, idx.ctypes.data, None) == -1
