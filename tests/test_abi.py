"""The C ABI library on the CPU: it loads, exports every declared symbol,
its host-side FP64 tables agree with the oracle's independent kernel
mathematics, and host-side argument errors come back as status codes.
No test here launches device work."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2408_02367_amd as sdn
from oracle import kernel as okernel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stodip_nufft.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SDN_API[^;(]*?\b(sdn_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = sdn.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert sorted(sdn.API) == names


@pytest.mark.parametrize("W", [4, 6, 8])
def test_kernel_tables_match_oracle(W):
    t = sdn.kernel_tables(W, 2.0, 48)
    assert abs(t["beta"] - okernel.beta(W, 2.0)) < 1e-12
    assert t["nf"] == okernel.fine_size(48, 2.0, W)
    # the piecewise polynomial against the oracle's kernel, normalised to peak 1
    b = okernel.beta(W, 2.0)
    peak = okernel.phi(np.array([0.0]), W, b)[0]
    tt = np.linspace(0.0, 1.0, 4001)[:-1]
    z = 2 * tt - 1
    for i in range(W):
        c = t["coef"][i, :t["ncoef"]].astype(np.float64)
        val = np.polyval(c[::-1], z)
        ref = okernel.phi(tt + W / 2 - 1 - i, W, b) / peak
        assert np.max(np.abs(val - ref)) < 5e-7, (W, i)
    # deapodisation factors on the same normalisation
    n = np.arange(48) - 24
    ref = peak / okernel.phi_hat(n / t["nf"], W, b)
    assert np.max(np.abs(t["deapod_inv"] / ref - 1)) < 1e-6


def test_fine_sizes_match_oracle():
    for N in (1, 5, 11, 32, 100, 160, 192, 224, 333):
        assert sdn.kernel_tables(6, 2.0, N)["nf"] == okernel.fine_size(N, 2.0, 6)
    assert sdn.kernel_tables(6, 1.5, 100)["nf"] == okernel.fine_size(100, 1.5, 6)


def test_host_side_errors():
    L = sdn.lib()
    assert L.sdn_plan_destroy(None) == 0
    h = ctypes.c_void_p()
    sh = (ctypes.c_int64 * 3)(8, 8, 8)
    assert L.sdn_plan_create(None, sh, None, 0, None, 0, None, None) == -1
    bad = (ctypes.c_int64 * 3)(0, 8, 8)
    assert L.sdn_plan_create(ctypes.byref(h), bad, None, 0, None, 0, None, None) == -1
    assert b"shape" in L.sdn_last_error() or b"sizes" in L.sdn_last_error()
    o = sdn.Opts()
    L.sdn_default_opts(ctypes.byref(o))
    assert (o.W, o.sigma) == (6, 2.0)
    o.W = 5
    assert L.sdn_plan_create(ctypes.byref(h), sh, None, 0, None, 0, ctypes.byref(o), None) == -4
    info = sdn.PlanInfo()
    assert L.sdn_plan_get_info(None, ctypes.byref(info)) == -6
    with pytest.raises(sdn.SdnError):
        sdn.kernel_tables(7, 2.0, 8)


def _header_struct_fields(name):
    """Field names of `typedef struct { ... } name;` in the public header,
    comments stripped, in declaration order."""
    import re
    src = open(os.path.join(os.path.dirname(__file__), "..", "include", "stodip_nufft.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", src).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            fields += [re.sub(r"\[.*\]", "", f).strip().split()[-1] for f in decl.split(",")]
    return fields


def test_binding_structs_mirror_the_header():
    assert [f for f, _ in sdn.Opts._fields_] == _header_struct_fields("sdn_opts")
    info = [f for f, _ in sdn.PlanInfo._fields_]
    hdr = _header_struct_fields("sdn_plan_info")
    assert info == hdr


def test_point_order_option_is_checked_on_the_host():
    L = sdn.lib()
    o = sdn.Opts()
    L.sdn_default_opts(ctypes.byref(o))
    assert (o.spread_engine, o.point_order) == (0, 0)
    assert sdn.POINT_ORDERS == {"auto": 0, "cell": 1}
    h = ctypes.c_void_p()
    sh = (ctypes.c_int64 * 3)(8, 8, 8)
    o.point_order = 7
    assert L.sdn_plan_create(ctypes.byref(h), sh, None, 0, None, 0, ctypes.byref(o), None) == -1
    assert b"point_order" in L.sdn_last_error()
