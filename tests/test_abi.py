"""The C-ABI boundary without a GPU: the shared library loads, exports every
function include/dgx.h declares (C linkage, unmangled), and the Python
binding wraps each of them under the same name; unsupported configurations
are rejected (DGX_E_INVAL) before any device work.  No compute call is made.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgx.h")
LIB = os.path.join(ROOT, "paper_2511_17551_amd", "libdgx.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dgx_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2511_17551_amd import build
        build.build()
    return LIB


def test_header_declares_the_boundary():
    names = declared()
    for required in ("dgx_create", "dgx_set_mesh", "dgx_rhs", "dgx_ssprk3_step", "dgx_thermo",
                     "dgx_chem_step", "dgx_check", "dgx_last_error", "dgx_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (dgx_[a-z0-9_]+)$", out, flags=re.M))
    assert set(declared()) <= exported


def test_binding_wraps_every_symbol(lib_path):
    from paper_2511_17551_amd import dgx
    assert set(dgx.EXPORTED) == set(declared())
    for n in declared():
        assert callable(getattr(dgx, n, None)), n


def test_errors_without_a_context(lib_path):
    """Argument checks run before any device work: NULL contexts are rejected."""
    lib = ctypes.CDLL(lib_path)
    lib.dgx_rhs.restype = ctypes.c_int
    lib.dgx_rhs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.dgx_rhs(None, None, 0.0, None, None) < 0
    lib.dgx_create.restype = ctypes.c_int
    lib.dgx_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.dgx_create(None, None) < 0


def bad_configs():
    """Unsupported configurations; each must be rejected before any device
    work, so the check runs without a GPU."""
    from paper_2511_17551_amd import workloads as W
    pg = W.case_c2(n=1).cfg
    mix = W.base_cfg(3, 4, W.EQ_EULER_MIX, volume_flux=W.VF_DUCROS)
    react = W.base_cfg(2, 3, W.EQ_REACT_MIX, volume_flux=W.VF_DUCROS)
    sp = W.Species()
    rx = W.park17_reactions(4)

    def table(A=None, rows=None):
        r = rows if rows is not None else np.arange(rx.nreactions)
        return W.Reactions(A=rx.A[r] if A is None else A, b=rx.b[r], theta_a=rx.theta_a[r], nu=rx.nu[r], nup=rx.nup[r])

    bad_A = rx.A.copy()
    bad_A[3] = 0.0
    inf_A = rx.A.copy()
    inf_A[0] = np.inf
    return [
        ("dim 1", dict(pg, dim=1), None, None),
        ("N 2", dict(pg, N=2), None, None),
        ("N 5", dict(pg, N=5), None, None),
        ("equation 7", dict(pg, eq=7), None, None),
        ("gamma 1", dict(pg, gamma=1.0), None, None),
        ("negative viscosity", dict(pg, mu=-1.0), None, None),
        ("mixture without species", mix, None, None),
        ("mixture at N = 3 with the entropy-conservative flux (not built)",
         dict(mix, N=3, volume_flux=W.VF_RANOCHA), sp, None),
        ("mixture with the Morinishi flux", dict(mix, volume_flux=W.VF_MORINISHI), sp, None),
        ("mixture at N = 3 with the Kennedy-Gruber flux (not built)",
         dict(mix, N=3, volume_flux=W.VF_KENNEDY_GRUBER), sp, None),
        ("reacting mixture with the HLL flux (not built)", dict(react, surface_flux=W.SF_HLL), sp, table()),
        ("Navier-Stokes at N = 4 with the Pirozzoli flux (not built)", dict(pg, N=4, volume_flux=W.VF_PIROZZOLI), None, None),
        ("volume flux 6", dict(pg, eq=W.EQ_EULER, volume_flux=6), None, None),
        ("surface flux 4", dict(pg, eq=W.EQ_EULER, surface_flux=4), None, None),
        ("mixture at N = 3 with the HLLC flux (not built)", dict(mix, N=3, surface_flux=W.SF_HLLC), sp, None),
        ("negative Sutherland constant", dict(pg, sutherland_S=-1.0), None, None),
        ("Sutherland law without a reference temperature", dict(pg, sutherland_S=110.0, sutherland_T0=0.0), None, None),
        ("reacting mixture without reactions", react, sp, None),
        ("A = 0", react, sp, table(A=bad_A)),
        ("A = inf", react, sp, table(A=inf_A)),
        ("no reactions", react, sp, table(rows=np.arange(0))),
        ("33 reactions", react, sp, table(rows=np.concatenate([np.arange(17), np.arange(16)]))),
    ]


def test_create_rejects_unsupported_configurations(lib_path):
    from paper_2511_17551_amd import dgx
    for name, cfg, sp, rx in bad_configs():
        with pytest.raises(dgx.DgxError) as ei:
            dgx.dgx_create(cfg, sp, rx)
        assert dgx.ERRORS[ei.value.code] == "DGX_E_INVAL", name
