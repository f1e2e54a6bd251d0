"""The C-ABI library loads on a machine without a GPU, exports every symbol
that include/iga2l.h declares, and rejects invalid input on the host side
(before any device call)."""
import ctypes
import math

import numpy as np
import pytest

import paper_2009_01499_amd as G


def test_library_exports_every_declared_symbol():
    L = G.lib()
    names = G.header_functions()
    assert len(names) >= 14
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_default_opts_match_python_mirror():
    o = G.CIgaOpts()
    G.lib().iga2l_default_opts(ctypes.byref(o))
    py = G.Opts()
    for f, _ in G.CIgaOpts._fields_:
        assert getattr(o, f) == getattr(py, f), f


def _assemble(dim, knots, p, kappa=None):
    arrs = [np.ascontiguousarray(k, dtype=np.float64) for k in knots]
    kp = (ctypes.c_void_p * dim)(*[a.ctypes.data for a in arrs])
    nk = (ctypes.c_int * dim)(*[len(a) for a in arrs])
    kap = None
    if kappa is not None:
        kappa = np.ascontiguousarray(kappa, dtype=np.float64)
        kap = ctypes.c_void_p(kappa.ctypes.data)
    h = ctypes.c_void_p()
    code = G.lib().iga2l_assemble(dim, ctypes.cast(kp, ctypes.POINTER(ctypes.c_void_p)), nk, p, kap, 0,
                                  ctypes.byref(h))
    return code, G.lib().iga2l_last_error().decode()


def test_invalid_inputs_are_rejected_on_host():
    t = G.open_uniform_knots(3, 8)
    assert _assemble(4, [t] * 4, 3)[0] == G.EINVAL                    # dimension
    assert _assemble(2, [t, t], 0)[0] == G.EINVAL                     # degree
    assert _assemble(2, [t, t], 9)[0] == G.EINVAL
    bad = t.copy(); bad[5] += 0.01                                    # not uniform
    assert _assemble(2, [bad, t], 3)[0] == G.EINVAL
    notopen = t.copy(); notopen[0] = -0.1                             # not open
    assert _assemble(2, [notopen, t], 3)[0] == G.EINVAL
    assert _assemble(2, [t, G.open_uniform_knots(3, 9)], 3)[0] == G.EUNSUPPORTED
    assert _assemble(2, [G.open_uniform_knots(3, 1)] * 2, 3)[0] == G.EINVAL   # m < 2
    k = np.ones(64); k[3] = -1.0
    code, msg = _assemble(2, [t, t], 3, k)
    assert code == G.EINVAL and "kappa" in msg
    k[3] = math.nan
    assert _assemble(2, [t, t], 3, k)[0] == G.EINVAL
    assert _assemble(3, [G.open_uniform_knots(5, 4)] * 3, 5)[0] == G.EUNSUPPORTED


def test_null_problem_is_rejected():
    assert G.lib().iga2l_setup_blocks(None, 0, None) == G.EINVAL
    assert G.lib().iga2l_sizes(None, None, None, None) == G.EINVAL
    G.lib().iga2l_destroy(None)
