"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/phmm.h declares, and validates inputs on the host."""
import ctypes
import os
import re
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import paper_2606_25738_amd as phmm  # noqa: E402
import synth  # noqa: E402

HEADER = os.path.join(ROOT, "include", "phmm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phmm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = phmm.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), "libphmm.so does not export %s" % n


def test_exports_are_c_symbols():
    # extern "C": plain names, no C++ mangling
    out = os.popen("nm -D --defined-only %s" % phmm.lib_path()).read()
    for n in declared_functions():
        assert re.search(r"\bT %s\b" % n, out), n


def test_classes():
    assert phmm.phmm_num_classes() == 21
    ns = [phmm.phmm_class_n(c) for c in range(phmm.phmm_num_classes())]
    assert ns == list(range(4, 25))
    assert phmm.phmm_class_n(-1) == -1 and phmm.phmm_class_n(21) == -1


def test_default_options():
    from paper_2606_25738_amd._binding import _Options
    o = _Options()
    phmm.lib().phmm_default_options(ctypes.byref(o))
    assert o.precision == phmm.PHMM_FP32_RERUN
    assert o.accept_min_sum == 1e-28
    assert o.force_class == -1 and o.one_pair_per_wave == 0
    assert o.fp32_max_rows == 1024 and o.long_fp32_max_rows == 0 and o.timing == 0
    assert o.route_diverse_fp64 == 1


def small_batch():
    return synth.generate("one_region")


def expect(code, batch, match):
    with pytest.raises(phmm.PhmmError) as e:
        phmm.phmm_validate_batch(batch)
    assert e.value.code == code
    assert match in str(e.value)


def test_validate_ok():
    b = small_batch()
    assert phmm.phmm_validate_batch(b) == (100, 200)


def test_validate_bad_read_base():
    b = small_batch()
    b["reads"] = b["reads"].copy()
    b["reads"][1234] = ord("X")
    expect(phmm.PHMM_EINVAL, b, "read base 1234")


def test_validate_lowercase_hap_base():
    b = small_batch()
    b["haplotypes"] = b["haplotypes"].copy()
    b["haplotypes"][77] = ord("a")
    expect(phmm.PHMM_EINVAL, b, "haplotype base 77")


def test_validate_pair_index():
    b = small_batch()
    b["pair_list"] = b["pair_list"].copy()
    b["pair_list"][40, 1] = 8
    expect(phmm.PHMM_EINVAL, b, "pair 40")
    b = small_batch()
    b["pair_list"] = b["pair_list"].copy()
    b["pair_list"][3, 0] = 64
    expect(phmm.PHMM_EINVAL, b, "pair 3")


def test_validate_offsets():
    b = small_batch()
    b["read_offsets"] = b["read_offsets"].copy()
    b["read_offsets"][5] = b["read_offsets"][4]  # empty read 4
    expect(phmm.PHMM_EINVAL, b, "read 4")
    b = small_batch()
    b["hap_offsets"] = b["hap_offsets"].copy()
    b["hap_offsets"][0] = 1
    expect(phmm.PHMM_EINVAL, b, "hap_offsets[0]")


def test_validate_ranges():
    n = 131073
    b = dict(reads=np.full(n, ord("A"), np.uint8), base_quals=np.full(n, 30, np.uint8),
             ins_quals=np.full(n, 45, np.uint8), del_quals=np.full(n, 45, np.uint8),
             gcp=np.full(n, 10, np.uint8), read_offsets=np.array([0, n], np.uint64),
             haplotypes=np.full(10, ord("A"), np.uint8), hap_offsets=np.array([0, 10], np.uint64),
             pair_list=np.array([[0, 0]], np.uint32))
    expect(phmm.PHMM_ERANGE, b, "read 0")


def test_validate_large_batch_reports_first_error():
    """Arrays large enough to be checked in parallel blocks (2^26 read bases,
    2^25 pairs, 2^25 reads): each error is reported at the first offending
    index, as a sequential scan would, whichever block finds it first."""
    nr = 1 << 25  # reads of 2 bases
    nb = 2 * nr
    b = dict(reads=np.full(nb, ord("A"), np.uint8), base_quals=np.full(nb, 30, np.uint8),
             ins_quals=np.full(nb, 45, np.uint8), del_quals=np.full(nb, 45, np.uint8),
             gcp=np.full(nb, 10, np.uint8),
             read_offsets=np.arange(0, nb + 1, 2, dtype=np.uint64),
             haplotypes=np.full(8, ord("C"), np.uint8), hap_offsets=np.array([0, 8], np.uint64),
             pair_list=np.zeros((nr, 2), np.uint32))
    b["pair_list"][:, 0] = np.arange(nr, dtype=np.uint32)
    assert phmm.phmm_validate_batch(b) == (2, 8)
    b["reads"][nb - 3] = ord("x")
    b["reads"][nb // 2 + 5] = ord("Z")
    b["reads"][12345678] = ord("U")
    expect(phmm.PHMM_EINVAL, b, "read base 12345678 ")
    b["reads"][[12345678, nb // 2 + 5, nb - 3]] = ord("G")
    b["pair_list"][nr - 1, 1] = 1
    b["pair_list"][20000000, 1] = 5
    expect(phmm.PHMM_EINVAL, b, "pair 20000000:")
    b["pair_list"][[nr - 1, 20000000], 1] = 0
    ro = b["read_offsets"]
    ro[30000001] = ro[30000000]  # read 30000000 is empty
    ro[nr - 1] = ro[nr - 2]
    expect(phmm.PHMM_EINVAL, b, "read 30000000 ")


def test_validate_empty_batch_is_fine():
    b = small_batch()
    b["pair_list"] = np.zeros((0, 2), np.uint32)
    assert phmm.phmm_validate_batch(b) == (0, 0)


def test_null_context_rejected():
    L = phmm.lib()
    rc = L.phmm_forward_batch(None, *([None] * 5), None, 0, None, None, 0, None, 0, None, None)
    assert rc == phmm.PHMM_EINVAL
    assert b"ctx" in L.phmm_last_error()


def test_bad_options_rejected():
    with pytest.raises(phmm.PhmmError) as e:
        phmm.Context(precision=7)
    assert e.value.code == phmm.PHMM_EINVAL
    with pytest.raises(phmm.PhmmError) as e:
        phmm.Context(force_class=21)
    assert e.value.code == phmm.PHMM_EINVAL


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device error path")
def test_no_device_fails_loudly():
    with pytest.raises(phmm.PhmmError) as e:
        phmm.Context()
    assert e.value.code == phmm.PHMM_EDEVICE
    with pytest.raises(phmm.PhmmError) as e:
        phmm.Server()
    assert e.value.code == phmm.PHMM_EDEVICE


def test_server_rejects_bad_options():
    for kw in (dict(lanes=0), dict(lanes=2, long_lanes=2), dict(hbm_budget_bytes=1 << 20),
               dict(short_cu_percent=101), dict(precision=7), dict(long_read_min=0),
               dict(long_grid_percent=0), dict(long_grid_percent=101)):
        with pytest.raises(phmm.PhmmError) as e:
            phmm.Server(**kw)
        assert e.value.code == phmm.PHMM_EINVAL, kw


@pytest.mark.parametrize("value", [0.0, 1e-45, 1e-38, 9.9e-31, float("nan"), 1e39])
def test_accept_threshold_outside_range_rejected(value):
    """The FP32 acceptance threshold is held as a float in the kernels: values
    under the 1e-30 floor (near FP32's smallest normals, or 0 after rounding)
    and values a float cannot hold are refused before any device work."""
    with pytest.raises(phmm.PhmmError) as e:
        phmm.Context(accept_min_sum=value)
    assert e.value.code == phmm.PHMM_EINVAL and "accept_min_sum" in str(e.value)


def test_forward_one_argument_errors():
    """phmm_forward_one checks its arguments before touching a device."""
    q = np.full(4, 30, np.uint8)
    with pytest.raises(phmm.PhmmError) as e:
        phmm.phmm_forward_one(b"", q[:0], q[:0], q[:0], q[:0], b"ACGT")
    assert e.value.code == phmm.PHMM_EINVAL and "empty" in str(e.value)
    with pytest.raises(phmm.PhmmError) as e:
        phmm.phmm_forward_one(b"ACGT", q, q, q, q, b"")
    assert e.value.code == phmm.PHMM_EINVAL
