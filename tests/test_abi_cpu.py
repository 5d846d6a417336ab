"""Host-side checks of the C ABI (no GPU needed): every function declared in
include/mbl.h is exported by libmbl.so, argument validation rejects bad input
before touching a device, and the footprint (admission) model."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbl.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mbl_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2012_00217_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header(lib):
    from paper_2012_00217_amd import _lib
    assert set(_declared()) <= set(_lib.PROTOTYPES)


def test_validation_without_device(lib):
    from paper_2012_00217_amd import _lib
    h = (C.c_double * 40)()
    out = C.c_void_p()
    for L, Sz in [(1, 0.0), (40, 0.0), (13, 0.0), (12, 0.5), (4, 3.0)]:
        st = lib.mbl_hamiltonian_create(L, Sz, 1.0, 1.0, C.cast(h, _lib.dptr), None, C.byref(out))
        assert st == _lib.MBL_EINVAL, (L, Sz)
        assert lib.mbl_last_error()
    nanh = (C.c_double * 4)(0.0, float("nan"), 0.0, 0.0)
    assert lib.mbl_hamiltonian_create(4, 0.0, 1.0, 1.0, C.cast(nanh, _lib.dptr), None,
                                      C.byref(out)) == _lib.MBL_EINVAL
    assert lib.mbl_apply_block(None, 0.0, 0, None, 1, None, 1, 1, None) == _lib.MBL_EINVAL
    assert lib.mbl_lobpcg_solve(None, 0.0, 1, 2, 1e-10, None, None, None, 1, None, None,
                                None) == _lib.MBL_EINVAL
    assert lib.mbl_small_eigh(0, None, 1, None, None, 1, None) == _lib.MBL_EINVAL
    assert lib.mbl_batch_solve(-1, None, None, 1) == _lib.MBL_EINVAL
    assert lib.mbl_server_create(0, 0, 0, C.byref(out)) == _lib.MBL_EINVAL  # no slots
    assert lib.mbl_server_cancel(None, 1) == _lib.MBL_EINVAL


def test_allocator_callbacks_install_and_restore(lib):
    """Installing and removing callbacks needs no device; both callbacks or
    neither."""
    from paper_2012_00217_amd import _lib, api
    api.use_allocator(lambda n, s: 0, lambda p, s: None)
    assert api._allocator is not None
    api.use_allocator(None)
    assert api._allocator is None
    assert lib.mbl_set_allocator(_lib.AllocFn(lambda n, s, c: 0), _lib.FreeFn(), None) == \
        _lib.MBL_EINVAL
    api.use_torch_allocator()
    assert api._allocator is not None


def test_footprint_model():
    from paper_2012_00217_amd import api
    n20, n24, n28 = 184756, 2704156, 40116600
    f64 = api.footprint_bytes(20, 64, "f64")
    # 14 FP64 block columns of LOBPCG, 3 of PCG, 2 of vectors per block column
    assert f64 >= n20 * 64 * 8 * (14 + 3 + 2)
    assert api.footprint_bytes(20, 64, "pcg32") < f64
    mixed24 = api.footprint_bytes(24, 128, "mixed")
    assert mixed24 > api.footprint_bytes(24, 128, "pcg32") * 0.99
    # the L=28, block 32 FP64 solve fits one 288 GB MI355X
    big = api.footprint_bytes(28, 32, "f64")
    assert n28 * 32 * 8 * 17 < big < 288e9
    with pytest.raises(api.MblError):
        api.footprint_bytes(13, 64, "f64", Sz=0.0)


def test_gap_ratio_host_routine():
    import numpy as np
    from paper_2012_00217_amd import api
    assert api.gap_ratio([0.0, 1.0, 3.0, 3.5]) == 0.375
    assert api.gap_ratio(np.arange(12.0)[::-1]) == 1.0
    with pytest.raises(api.MblError):
        api.gap_ratio([1.0, 2.0])
