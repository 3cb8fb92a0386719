"""The allocation-free reverse pass (ssp_adjoint_elements_noalloc) against the
workspace form (ssp_adjoint_elements), both called through the C ABI: the
element means must be bit-identical (same kernels, same fixed-order
reductions), on two calls in a row, the second on a smaller ensemble (the
static scratch keeps the first call's contents), and a third call on the first
ensemble again.  An ensemble beyond the scratch's capacity is refused."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _elements_both_ways(e, comp=3):
    from paper_1106_2899_amd._lib import check, lib
    L = lib()
    chain = torch.empty((e.M, 10), dtype=torch.float64, device=e.device)
    ref = torch.empty((e.n_elements, 10), dtype=torch.float64, device=e.device)
    got = torch.full((e.n_elements, 10), float("nan"), dtype=torch.float64, device=e.device)
    rec, kap = ctypes.c_void_p(e._rec_p), e._rec_kappa_p
    check(L.ssp_adjoint_elements(e._h, rec, kap, comp, 1, ctypes.c_void_p(chain.data_ptr()),
                                 ctypes.c_void_p(ref.data_ptr()), e._s), e._h)
    check(L.ssp_adjoint_elements_noalloc(e._h, rec, kap, comp, 1, ctypes.c_void_p(got.data_ptr()), e._s), e._h)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def _recorded(M, E, N, T, ckpt, seed, precision):
    from paper_1106_2899_amd.ensemble import Ensemble
    e = Ensemble(N, M, n_elements=E, precision=precision, seed=seed, corr_levels=0).init()
    kap = np.zeros((E, 9))
    kap[:, 1] = np.linspace(0.05, 0.5, E)
    e.forward_record(T, ckpt, kap)
    return e


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_matches_workspace_form_on_two_calls(precision):
    _need_gpu()
    big = _recorded(600, 3, 16, 80, 20, 41, precision)
    small = _recorded(96, 2, 12, 50, 50, 42, precision)  # stored window, fewer chains
    for e in (big, small, big):
        ref, got = _elements_both_ways(e)
        assert np.isfinite(ref).all()
        assert np.array_equal(ref, got), np.abs(ref - got).max()
    big.close()
    small.close()


def test_noalloc_refuses_more_chains_than_its_scratch_holds():
    _need_gpu()
    from paper_1106_2899_amd._lib import SSP_ESIZE, lib
    from paper_1106_2899_amd.ensemble import Ensemble
    e = Ensemble(2, (1 << 18) + 1, precision="fp32", seed=3, corr_levels=0).init()
    out = torch.empty((1, 10), dtype=torch.float64, device=e.device)
    rc = lib().ssp_adjoint_elements_noalloc(e._h, ctypes.c_void_p(0), ctypes.c_void_p(0), 3, 1,
                                           ctypes.c_void_p(out.data_ptr()), e._s)
    assert rc == SSP_ESIZE
    assert b"262144" in lib().ssp_last_error(e._h)
    e.close()
