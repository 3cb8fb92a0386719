"""CPU checks of the C ABI: the library loads, exports every function that
include/ssp.h declares, and validates configurations on the host (no GPU
call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1106_2899_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libssp.so not built")
    return _lib


def test_header_declarations_are_exported():
    L = _lib()
    with open(os.path.join(ROOT, "include", "ssp.h")) as f:
        text = f.read()
    declared = set(re.findall(r"^(?:int|const char\*)\s+(ssp_\w+)\s*\(", text, flags=re.M))
    assert declared, "no declarations parsed"
    assert declared == set(L.EXPORTS)
    lib = L.lib()
    for name in declared:
        assert hasattr(lib, name)


def _cfg(L, **kw):
    c = L.SspConfig()
    assert L.lib().ssp_config_init(ctypes.byref(c)) == 0
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _query(L, c):
    sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    rc = L.lib().ssp_query_sizes(ctypes.byref(c), ctypes.byref(sb), ctypes.byref(wb))
    return rc, sb.value, wb.value, (L.lib().ssp_last_error(None) or b"").decode()


def test_defaults_are_the_paper_parameters():
    L = _lib()
    c = _cfg(L)
    assert (c.n0, c.ns, c.zeta_s, c.dt) == (4.0, 0.5, 0.1, 0.01)
    assert c.precision == L.SSP_FP32 and c.corr_levels == 16 and c.corr_lags == 16
    assert c.construct_rule == 0  # K = C - Z, the GPU rule of Sec. 3.2


def test_query_sizes_valid_and_scaling():
    L = _lib()
    rc, s1, w1, _ = _query(L, _cfg(L, n_chains=1000, n_beads=32, sample_every=10))
    assert rc == 0 and s1 >= 1000 * 32 * (4 * 16 + 4) and w1 > 0
    rc, s2, _, _ = _query(L, _cfg(L, n_chains=2000, n_beads=32, sample_every=10))
    assert rc == 0 and s2 >= 2 * s1 - 1024
    rc, s3, _, _ = _query(L, _cfg(L, n_chains=1000, n_beads=32, precision=L.SSP_FP64))
    assert rc == 0 and s3 >= 1000 * 32 * (2 * 32 + 4)


@pytest.mark.parametrize("field,value,msg", [
    ("n_chains", 0, "n_chains"),
    ("n_beads", 1, "N <= 128"),
    ("n_beads", 129, "N <= 128"),
    ("precision", 7, "precision"),
    ("dt", 0.0, "positive"),
    ("ns", -1.0, "positive"),
    ("zeta_s", float("nan"), "positive"),
    ("sample_every", 0, "sample_every"),
    ("corr_levels", 17, "corr_levels"),
    ("corr_lags", 8, "corr_lags"),
    ("series_capacity", -1, "series_capacity"),
    ("construct_rule", 2, "construct_rule"),
    ("n_elements", 0, "n_elements"),
])
def test_invalid_configs_are_rejected(field, value, msg):
    L = _lib()
    c = _cfg(L, n_chains=64, n_beads=8)
    setattr(c, field, value)
    rc, _, _, err = _query(L, c)
    assert rc == L.SSP_EINVAL
    assert msg in err


def test_element_offsets_are_validated():
    L = _lib()
    c = _cfg(L, n_chains=10, n_beads=8, n_elements=2, corr_batches=2)
    bad = (ctypes.c_int32 * 3)(0, 5, 9)
    c.element_offsets_host = ctypes.cast(bad, ctypes.POINTER(ctypes.c_int32))
    rc, _, _, err = _query(L, c)
    assert rc == L.SSP_EINVAL and "element_offsets" in err
    good = (ctypes.c_int32 * 3)(0, 5, 10)
    c.element_offsets_host = ctypes.cast(good, ctypes.POINTER(ctypes.c_int32))
    assert _query(L, c)[0] == 0


def test_create_rejects_null_and_misaligned_buffers():
    L = _lib()
    c = _cfg(L, n_chains=4, n_beads=8, corr_batches=2)
    h = ctypes.c_void_p()
    assert L.lib().ssp_create(ctypes.byref(c), None, None, ctypes.byref(h)) == L.SSP_EINVAL
    assert L.lib().ssp_create(ctypes.byref(c), ctypes.c_void_p(0x1001), ctypes.c_void_p(0x2000),
                              ctypes.byref(h)) == L.SSP_EINVAL
    assert b"aligned" in L.lib().ssp_last_error(None)


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_1106_2899_amd")
    for dp, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".h")):
                with open(os.path.join(dp, fn)) as f:
                    src = f.read()
                assert "import oracle" not in src and "ssp_oracle" not in src, fn


@pytest.mark.parametrize("zeta_s,n0,want", [
    (0.1, 4.0, None),                                    # the paper's dt / zeta_s = 0.1: no cap binds
    (0.04, 4.0, None),                                   # 0.25 exactly: still below
    (0.02, 4.0, "hop probabilities bind"),               # 0.5
    (0.0025, 1.0, "construction probability and the destruction"),  # 4: every cap can bind
])
def test_warning_when_the_half_caps_can_bind(zeta_s, n0, want):
    """dt / zeta_s > 1/4 is accepted with a warning naming the caps of the
    Sec. 3.1 step map that can bind; none at the paper's parameters."""
    L = _lib()
    rc, *_ = _query(L, _cfg(L, n_chains=8, n_beads=8, corr_batches=4, zeta_s=zeta_s, n0=n0))
    assert rc == 0
    msg = L.lib().ssp_warning(None)
    if want is None:
        assert msg is None
    else:
        assert msg is not None and want in msg.decode() and "dt/zeta_s" in msg.decode(), msg
