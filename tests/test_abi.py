"""The C-ABI library loads and exports every entry point declared in include/lensfield.h
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lensfield.h")).read()
    decl = re.compile(r"^(?:lf_status|const char\*|size_t|int32_t|void)\s+(lf_[a-z0-9_]+)\s*\(", re.M)
    return sorted(set(decl.findall(txt)))


def test_header_declares_the_four_hot_path_calls():
    names = _declared()
    for n in ("lf_lens_maps", "lf_chi2_batch", "lf_find_images", "lf_multiplane_trace"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2609_08649_amd import build
    path = build.ensure_built()
    lib = ctypes.CDLL(path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import torch  # noqa: F401  (the binding loads the library after torch)
    from paper_2609_08649_amd import lensfield as lf
    assert lf.header_symbols() == _declared()
    L = lf.lib()
    for n in _declared():
        assert getattr(L, n).restype is not None or n == "lf_shutdown"


def test_host_cosmology_helpers_match_oracle_without_gpu(orc):
    """Host-side helpers of the library (no device needed) agree with the oracle."""
    import ctypes as C
    import torch  # noqa: F401
    from paper_2609_08649_amd import lensfield as lf
    L = lf.lib()
    c = lf.lf_cosmo(70.0, 0.3)
    out = C.c_double()
    for z1, z2 in ((0.0, 0.5), (0.3, 1.2), (0.6, 9.0)):
        assert L.lf_cosmo_dist(C.byref(c), z1, z2, C.byref(out)) == 0
        assert abs(out.value / orc.dist(z1, z2) - 1) < 1e-11
    assert L.lf_cosmo_adis(C.byref(c), 0.5, 2.0, C.byref(out)) == 0
    assert abs(out.value / orc.adis(0.5, 2.0) - 1) < 1e-11
    ks, rs = C.c_double(), C.c_double()
    assert L.lf_nfw_params(C.byref(c), 0.3, 8e14, 5.0, C.byref(ks), C.byref(rs)) == 0
    oks, ors = orc.nfw_params(70.0, 0.3, 0.3, 8e14, 5.0)
    assert abs(ks.value / oks - 1) < 1e-10 and abs(rs.value / ors - 1) < 1e-10
    assert L.lf_cosmo_adis(C.byref(c), 2.0, 1.0, C.byref(out)) == lf.LF_E_INVALID_ARG
    for zd, zs, H0 in ((0.5, 2.0, 70.0), (0.3, 1.2, 67.0), (0.6, 9.0, 73.0)):
        c = lf.lf_cosmo(H0, 0.3)
        assert L.lf_cosmo_tdscale(C.byref(c), zd, zs, C.byref(out)) == 0
        assert abs(out.value / orc.tdscale(zd, zs, H0=H0) - 1) < 1e-11
    assert L.lf_cosmo_tdscale(C.byref(c), 2.0, 1.0, C.byref(out)) == lf.LF_E_INVALID_ARG
