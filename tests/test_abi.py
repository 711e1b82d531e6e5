"""CPU checks of the boundary: the shared library loads without a GPU and
exports every function include/megapf.h declares; the binding knows them all."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^MP_API\s+[\w\s\*]+?\b(mp_\w+)\s*\(", txt, re.M))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2404_16370_amd import megapf
    names = _declared()
    assert len(names) >= 17
    L = ctypes.CDLL(megapf.LIB_PATH)
    for n in sorted(names):
        assert hasattr(L, n), n
    assert names == set(megapf.EXPORTS)


def test_default_params_and_errors_without_gpu():
    from paper_2404_16370_amd import megapf as M
    p = M.mp_filter_default_params()
    assert p.k == 16 and p.sigma_r == 5.0 and p.sigma_t == 2.5 and p.post_iters == 10
    mp = M.mp_map_default_params()
    assert mp.voxel == 0.5 and mp.nnf_radius == 2
    # argument errors are detected before any device work
    L = M.lib()
    h = ctypes.c_void_p()
    st = L.mp_map_build(None, -1, ctypes.byref(mp), None, ctypes.byref(h))
    assert st == M.MP_E_ARG
    assert b"n < 0" in L.mp_last_error()
