"""The C ABI library loads, exports every entry point include/xc.h declares,
and rejects bad input before touching the device (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "xc.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(xc_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    import paper_2007_03143_amd as pkg
    lib = ctypes.CDLL(pkg.LIB_PATH)
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_messages():
    import paper_2007_03143_amd as pkg
    assert pkg.xc_abi_version() == 3
    assert pkg.xc_strerror(0) == "ok"
    assert pkg.xc_strerror(pkg.XC_ERR_NOMEM) == "out of device memory"
    assert pkg.xc_strerror(pkg.XC_ERR_BUSY) == "busy"
    assert pkg.xc_strerror(-99) == "unknown error"


def _water():
    from workloads import cfg_water, grid_spec_dict
    w = cfg_water()
    return w, grid_spec_dict(w)


@pytest.mark.parametrize("override,code", [
    (dict(batch_max=8), -1), (dict(batch_max=4096), -1), (dict(ssf_a=1.0), -1),
    (dict(screen_eta=-1.0), -1), (dict(rho_thresh=0.0), -1), (dict(n_rad=0), -1),
    (dict(partition=5), -1), (dict(partition="becke", becke_radius=[0.6, -0.35, 0.35]), -1),
])
def test_invalid_grid_rejected(override, code):
    import paper_2007_03143_amd as pkg
    w, g = _water()
    with pytest.raises(pkg.XcError) as e:
        pkg.xc_integrate(w.coords, w.mk_alpha, w.basis, dict(g, **override), "lda", w.P)
    assert e.value.code == code


def test_invalid_basis_and_functional_rejected():
    import paper_2007_03143_amd as pkg
    from workloads.basis import BasisSet
    w, g = _water()
    b = w.basis
    bad_L = BasisSet(b.shell_atom, np.where(b.shell_L == 2, 4, b.shell_L).astype(np.int32),
                     b.shell_nprim, b.prim_alpha, b.prim_coef)
    with pytest.raises(pkg.XcError) as e:
        pkg.xc_integrate(w.coords, w.mk_alpha, bad_L, g, "lda", w.P)
    assert e.value.code == pkg.XC_ERR_UNSUPPORTED
    bad_atom = BasisSet(np.where(b.shell_atom == 2, 7, b.shell_atom).astype(np.int32),
                        b.shell_L, b.shell_nprim, b.prim_alpha, b.prim_coef)
    with pytest.raises(pkg.XcError) as e:
        pkg.xc_integrate(w.coords, w.mk_alpha, bad_atom, g, "lda", w.P)
    assert e.value.code == pkg.XC_ERR_INVALID_ARG
    neg = BasisSet(b.shell_atom, b.shell_L, b.shell_nprim, -b.prim_alpha, b.prim_coef)
    with pytest.raises(pkg.XcError) as e:
        pkg.xc_integrate(w.coords, w.mk_alpha, neg, g, "pbe", w.P)
    assert e.value.code == pkg.XC_ERR_INVALID_ARG
    with pytest.raises(pkg.XcError) as e:
        pkg.xc_integrate(w.coords, w.mk_alpha, b, g, 7, w.P)
    assert e.value.code == pkg.XC_ERR_UNSUPPORTED
    with pytest.raises(pkg.XcError) as e:
        pkg.xc_integrate(w.coords, w.mk_alpha, b, g, "lda", w.P[:24, :24])
    assert e.value.code == pkg.XC_ERR_INVALID_ARG
    with pytest.raises(pkg.XcError) as e:
        pkg.xc_integrate(w.coords, -w.mk_alpha, b, g, "lda", w.P)
    assert e.value.code == pkg.XC_ERR_INVALID_ARG


def test_spherical_flags_and_becke_size_limits_rejected():
    import paper_2007_03143_amd as pkg
    from workloads import make_basis
    from workloads.basis import BasisSet
    w, g = _water()
    b = w.basis
    bad = BasisSet(b.shell_atom, b.shell_L, b.shell_nprim, b.prim_alpha, b.prim_coef,
                   np.full(b.nshells, 2, dtype=np.int32))
    with pytest.raises(pkg.XcError) as e:
        pkg.xc_integrate(w.coords, w.mk_alpha, bad, g, "lda", w.P)
    assert e.value.code == pkg.XC_ERR_INVALID_ARG
    # 1200 hydrogen atoms on a lattice: above the Becke kernel's atom limit
    Z = np.ones(1200, dtype=np.int32)
    X = 3.0 * np.stack(np.meshgrid(np.arange(12), np.arange(10), np.arange(10),
                                   indexing="ij"), -1).reshape(-1, 3).astype(float)
    hb = make_basis(Z)
    grid = dict(g, partition="becke", atom_mask=None)
    with pytest.raises(pkg.XcError) as e:
        pkg.xc_integrate(X, np.full(1200, 5.0), hb, grid, "lda", np.zeros((hb.nbf, hb.nbf)))
    assert e.value.code == pkg.XC_ERR_UNSUPPORTED


def test_allocator_needs_both_callbacks():
    """A device allocator with alloc but no free (or the reverse) is refused
    before any device call."""
    import paper_2007_03143_amd.binding as b
    w, g = _water()
    alloc = b.XC_ALLOC_FN(lambda n, user: None)
    free = b.XC_FREE_FN(lambda p, user: None)
    for a, f in ((alloc, None), (None, free)):
        with pytest.raises(b.XcError) as e:
            b.xc_context_create(w.coords, w.mk_alpha, w.basis, g, 0, 0, a, f)
        assert e.value.code == b.XC_ERR_INVALID_ARG
        assert "alloc" in str(e.value)
