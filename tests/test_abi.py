"""CPU-side checks of the C ABI: the library loads, exports every declared symbol, and its host
logic (time coupling, argument validation) agrees with the oracle.  No device compute here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import timecoupling as otc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bkts.h")
LIB = os.path.join(ROOT, "paper_2504_02117_amd", "libbkts.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libbkts.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(bkts_\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if not n.endswith("_cb")))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    from paper_2504_02117_amd import bkts
    assert set(declared_functions()) <= set(bkts.EXPORTED)


def test_no_gpu_context_fails_cleanly():
    import torch
    from paper_2504_02117_amd import bkts
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(bkts.BktsError) as e:
        bkts.bkts_ctx_create(0)
    assert e.value.status in (bkts.BKTS_EDEVICE, bkts.BKTS_EINVAL)
    assert bkts.bkts_last_error()


@pytest.mark.parametrize("method,name,theta", [(0, "ie", 1.0), (1, "theta", 0.5), (1, "theta", 0.3), (2, "sdirk2", 0.5)])
@pytest.mark.parametrize("k", [1, 2, 5, 8])
def test_time_coupling_matches_oracle(method, name, theta, k):
    from paper_2504_02117_amd import bkts
    tau = 0.125
    tc = bkts.bkts_tc_create(None, method, k, tau, theta=theta)
    try:
        A, _, c = otc.tableau(name, theta)
        mi = otc.implicit_part(A, c)[0].shape[0]
        for phase in range(mi):
            A1, A2, beta, m_impl = bkts.bkts_tc_get(tc, phase)
            oA1, oA2, obeta = otc.window_matrices(A, c, k, phase, tau)
            assert m_impl == mi
            np.testing.assert_allclose(A1, oA1, rtol=0, atol=1e-15)
            np.testing.assert_allclose(A2, oA2, rtol=0, atol=1e-15)
            assert beta == obeta
    finally:
        bkts.bkts_tc_destroy(tc)


def test_custom_tableau_and_validation():
    from paper_2504_02117_amd import bkts
    g = 1 - 1 / np.sqrt(2)
    A = np.array([[g, 0.0], [1 - g, g]])
    tc = bkts.bkts_tc_create(None, bkts.BKTS_DIRK_CUSTOM, 4, 0.1, A=A, c=np.array([g, 1.0]))
    A1, A2, beta, mi = bkts.bkts_tc_get(tc, 1)
    oA1, oA2, _ = otc.window_matrices(A, np.array([g, 1.0]), 4, 1, 0.1)
    np.testing.assert_allclose(A2, oA2, atol=1e-15)
    bkts.bkts_tc_destroy(tc)
    for bad in [dict(k=0), dict(k=33), dict(tau=-1.0)]:
        kw = dict(k=4, tau=0.1)
        kw.update(bad)
        with pytest.raises(bkts.BktsError) as e:
            bkts.bkts_tc_create(None, bkts.BKTS_IE, kw["k"], kw["tau"])
        assert e.value.status == bkts.BKTS_EINVAL
    with pytest.raises(bkts.BktsError):  # fully implicit but singular: no averaged coefficient
        bkts.bkts_tc_create(None, bkts.BKTS_DIRK_CUSTOM, 2, 0.1, A=np.array([[1.0, 0.5], [2.0, 1.0]]),
                            c=np.array([1.5, 3.0]))
    with pytest.raises(bkts.BktsError):  # fully implicit: k must hold whole steps
        bkts.bkts_tc_create(None, bkts.BKTS_RADAU2, 3, 0.1)
    for A_bad, c_bad in (([[0.5, 0.0], [0.5, 0.5]], [0.4, 1.0]),      # c is not the row sums of A
                         ([[0.5, 0.0], [0.25, 0.5]], [0.5, 0.75])):   # the last stage does not end at 1
        with pytest.raises(bkts.BktsError) as e:
            bkts.bkts_tc_create(None, bkts.BKTS_DIRK_CUSTOM, 2, 0.1, A=np.array(A_bad), c=np.array(c_bad))
        assert e.value.status == bkts.BKTS_EINVAL
    with pytest.raises(bkts.BktsError):
        bkts.bkts_tc_get(tc := bkts.bkts_tc_create(None, bkts.BKTS_IE, 2, 0.1), 1)
    bkts.bkts_tc_destroy(tc)


def test_null_handles_rejected():
    from paper_2504_02117_amd import bkts
    lib = bkts._lib
    assert lib.bkts_spmm(None, None, 0, 4, 0.0, 1.0, None, 4, None, 4) == bkts.BKTS_EINVAL
    assert lib.bkts_ctx_synchronize(None) == bkts.BKTS_EINVAL
    assert "ctx" in bkts.bkts_last_error()


def test_server_null_handles_rejected():
    import ctypes as C
    from paper_2504_02117_amd import bkts
    lib = bkts._lib
    out = C.c_void_p()
    assert lib.bkts_server_create(None, 1 << 30, 8, C.byref(out)) == bkts.BKTS_EINVAL
    req = bkts.bkts_request()
    t = C.c_uint64()
    assert lib.bkts_server_submit(None, C.byref(req), C.byref(t)) == bkts.BKTS_EINVAL
    n = C.c_int()
    assert lib.bkts_server_poll(None, None, 0, C.byref(n)) == bkts.BKTS_EINVAL
    assert lib.bkts_server_clock(None) == 0.0
    lib.bkts_server_destroy(None)
    assert lib.bkts_nlop_create(None, None, None, C.byref(out)) == bkts.BKTS_EINVAL
    assert lib.bkts_richards_create(None, None, None, None, C.byref(out)) == bkts.BKTS_EINVAL
    assert lib.bkts_nl_mass(None, None, 1, None, 1, None, 1) == bkts.BKTS_EINVAL


@pytest.mark.parametrize("k", [2, 4, 6])
def test_fully_implicit_time_coupling_matches_oracle(k):
    """2-stage Radau IIA (named and as a custom full tableau): full diagonal blocks in A2, the
    averaged splitting coefficient, and whole-step windows."""
    from paper_2504_02117_amd import bkts
    tau = 0.2
    A, _, c = otc.tableau("radau2")
    oA1, oA2, _ = otc.window_matrices(A, c, k, 0, tau)
    for tc in (bkts.bkts_tc_create(None, bkts.BKTS_RADAU2, k, tau),
               bkts.bkts_tc_create(None, bkts.BKTS_DIRK_CUSTOM, k, tau, A=A, c=c)):
        try:
            A1, A2, beta, mi = bkts.bkts_tc_get(tc, 0)
            assert mi == 2
            np.testing.assert_allclose(A1, oA1, rtol=0, atol=1e-15)
            np.testing.assert_allclose(A2, oA2, rtol=0, atol=1e-15)
            assert beta == pytest.approx(otc.averaged_beta(A), rel=1e-14)
        finally:
            bkts.bkts_tc_destroy(tc)


def test_binding_constants_match_header():
    """Every enum constant the binding names has the header's value, and the profiling categories
    cover every kernel id the header declares."""
    import re
    from pathlib import Path
    from paper_2504_02117_amd import bkts
    hdr = (Path(__file__).resolve().parents[1] / "include" / "bkts.h").read_text()
    vals = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(BKTS_[A-Z0-9_]+)\s*=\s*(-?\d+)", hdr)}
    checked = 0
    for name, v in vars(bkts).items():
        if name.startswith("BKTS_") and isinstance(v, int) and name in vals:
            assert v == vals[name], name
            checked += 1
    assert checked >= 20
    for name in ("BKTS_FMT_STENCIL", "BKTS_PREC_MG", "BKTS_RADAU2"):
        assert getattr(bkts, name) == vals[name]
    assert len(bkts.KERNELS) == vals["BKTS_K_COUNT"]
