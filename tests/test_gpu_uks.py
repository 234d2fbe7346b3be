"""Spin-unrestricted integration on the HIP path (the two-density extension
of Sec. 2.1) against the oracle's spin-unrestricted quadrature, through the
C ABI. Same bar as the restricted parity tests: |dE_xc|, |dN_e| and
max|dV^s| at most 1e-10 in FP64."""
import numpy as np
import pytest

from gpu_util import say
from oracle.spin import integrate_uks
from workloads import cfg_water, cfg_water_cluster, grid_spec_dict

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _open_shell(w, n_beta_drop=1):
    """P^a from the n_occ leading natural orbitals of P/2, P^b without the
    first n_beta_drop of them (an open-shell density pair)."""
    ev, U = np.linalg.eigh(w.P)
    k = w.n_occ
    C = U[:, -k:] * np.sqrt(np.maximum(ev[-k:], 0) / 2)
    return C @ C.T, C[:, n_beta_drop:] @ C[:, n_beta_drop:].T


def _gpu_uks(w, Pa, Pb, functional, wave_bytes=0, also_rks=None, **over):
    import torch
    from paper_2007_03143_amd import XcContext
    ctx = XcContext(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w, **over),
                    wave_bytes=wave_bytes)
    try:
        a = torch.from_numpy(np.ascontiguousarray(Pa)).cuda()
        b = torch.from_numpy(np.ascontiguousarray(Pb)).cuda()
        Va, Vb, EN = ctx.integrate_uks(a, b, functional)
        torch.cuda.synchronize()
        out = [float(EN[0]), float(EN[1]), Va.cpu().numpy(), Vb.cpu().numpy(), ctx.stats()]
        if also_rks is not None:
            V, EN = ctx.integrate(torch.from_numpy(np.ascontiguousarray(also_rks)).cuda(),
                                  functional)
            torch.cuda.synchronize()
            out.append((float(EN[0]), float(EN[1]), V.cpu().numpy()))
        return out
    finally:
        ctx.close()


def _oracle_uks(w, Pa, Pb, functional, **over):
    return integrate_uks(w.coords, w.mk_alpha, w.basis, Pa, Pb, functional,
                         over.get("n_rad", w.n_rad), w.ang, ssf_a=w.ssf_a,
                         screen_eta=w.screen_eta, rho_thresh=w.rho_thresh)


def _compare(tag, gpu, ref):
    E, N, Va, Vb = gpu[:4]
    Eo, No, Vao, Vbo = ref
    dVa, dVb = np.abs(Va - Vao).max(), np.abs(Vb - Vbo).max()
    say(f"  {tag}: E gpu {E!r} oracle {Eo!r} dE {E - Eo:.3e} dN {N - No:.3e} "
        f"max dVa {dVa:.3e} max dVb {dVb:.3e}")
    assert abs(E - Eo) <= TOL and abs(N - No) <= TOL
    assert dVa <= TOL and dVb <= TOL
    assert np.array_equal(Va, Va.T) and np.array_equal(Vb, Vb.T)


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_open_shell_water_parity(functional):
    w = cfg_water(n_rad=50, n_ang=194)
    Pa, Pb = _open_shell(w)
    say(f"case uks water open shell {functional}")
    _compare(functional, _gpu_uks(w, Pa, Pb, functional),
             _oracle_uks(w, Pa, Pb, functional))


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_open_shell_spherical_parity(functional):
    """Spherical f and d shells (41 functions) through the two-spin Z pass."""
    w = cfg_water(polarisation=True, pure=True, n_rad=40, n_ang=146)
    Pa, Pb = _open_shell(w, n_beta_drop=2)
    say(f"case uks spherical water {functional}")
    _compare(functional, _gpu_uks(w, Pa, Pb, functional),
             _oracle_uks(w, Pa, Pb, functional))


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_closed_shell_uks_equals_rks(functional):
    """P^a = P^b = P/2: E and N equal the restricted integration's, and
    V^a = V^b = V to rounding, on the same context (the restricted call after the
    spin-unrestricted one runs on the re-planned waves)."""
    w = cfg_water()
    say(f"case uks closed shell {functional}")
    E, N, Va, Vb, st, (Er, Nr, Vr) = _gpu_uks(w, w.P / 2, w.P / 2, functional, also_rks=w.P)
    say(f"  dE {E - Er:.3e} dN {N - Nr:.3e} max dVa {np.abs(Va - Vr).max():.3e} "
        f"max dVb {np.abs(Vb - Vr).max():.3e}")
    assert abs(E - Er) <= 1e-12 * abs(Er) and abs(N - Nr) <= 1e-12 * abs(Nr)
    # V is accumulated with atomic adds across batches, so V^a and V^b agree
    # to rounding, not bit for bit
    assert np.abs(Va - Vb).max() <= 1e-13 * np.abs(Vr).max()
    assert np.abs(Va - Vr).max() <= 1e-13 * np.abs(Vr).max()


def test_closed_shell_uks_equals_rks_on_wide_tiles():
    """The 600-atom chain on two parent atoms of a reduced grid: its batches
    screen in several hundred functions, so every wave's FP64 density
    contraction runs on 64 x 128 tiles, for both spins. P^a = P^b = P/2
    gives the restricted E, N and V."""
    from gpu_util import chain600
    w = chain600(n_rad=30, n_ang=50)
    mask = np.zeros(w.natoms, np.uint8)
    mask[[int(np.nonzero(w.mol.Z == 6)[0][3]), int(np.nonzero(w.mol.Z == 1)[0][7])]] = 1
    say("case uks closed shell chain600 two atoms, 64 x 128 tiles")
    E, N, Va, Vb, st, (Er, Nr, Vr) = _gpu_uks(w, w.P / 2, w.P / 2, "pbe", also_rks=w.P,
                                               atom_mask=mask)
    say(f"  waves {st['n_waves']} wide {st['n_wide_waves']} dE {E - Er:.3e} dN {N - Nr:.3e} "
        f"max dVa {np.abs(Va - Vr).max():.3e}")
    assert st["n_wide_waves"] == st["n_waves"] > 0
    assert abs(E - Er) <= 1e-12 * abs(Er) and abs(N - Nr) <= 1e-12 * abs(Nr)
    assert np.abs(Va - Vr).max() <= 1e-13 * np.abs(Vr).max()
    assert np.abs(Vb - Vr).max() <= 1e-13 * np.abs(Vr).max()


def test_cluster_many_waves_parity():
    """Eight waters on a 30 x 86 grid, split over several waves, PBE."""
    w = cfg_water_cluster(8, n_rad=30, n_ang=86)
    Pa, Pb = _open_shell(w, n_beta_drop=3)
    say("case uks cluster8 pbe, 1 MiB waves")
    g = _gpu_uks(w, Pa, Pb, "pbe", wave_bytes=1 << 20)
    say(f"  waves {g[4]['n_waves']} batches {g[4]['n_batches']}")
    assert g[4]["n_waves"] > 1
    _compare("pbe", g, _oracle_uks(w, Pa, Pb, "pbe"))


def test_fully_polarised_and_empty_beta():
    """P^b = 0: zeta = 1 everywhere (clamped) and V^b still defined by the
    functional's beta derivative; compared with the oracle."""
    w = cfg_water(n_rad=40, n_ang=110)
    Pa, _ = _open_shell(w)
    Pb = np.zeros_like(Pa)
    for f in ("lda", "pbe"):
        say(f"case uks fully polarised {f}")
        _compare(f, _gpu_uks(w, Pa, Pb, f), _oracle_uks(w, Pa, Pb, f))


def test_mixed_precision_rejected():
    import torch
    from paper_2007_03143_amd import XcContext, XcError
    w = cfg_water(n_rad=20, n_ang=50)
    ctx = XcContext(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w))
    try:
        P = torch.from_numpy(w.P / 2).cuda()
        with pytest.raises(XcError):
            ctx.integrate_uks(P, P, "pbe", precision="fp32")
    finally:
        ctx.close()


def _golden_ext():
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "cluster64_ext_atoms.json")))


def _check_v(tag, V, rec, r, c):
    dv = np.abs(V[r, c] - np.array(rec["sample_values"])).max()
    drs = np.abs(V.sum(axis=1) - np.array(rec["row_sums"])).max()
    say(f"  {tag}: sampled max dV {dv:.3e} ({len(r)} entries), max d(row sum) {drs:.3e}")
    assert dv <= TOL and drs <= TOL
    assert np.array_equal(V, V.T)


def test_cluster_atoms_match_golden():
    """The 64-water cluster (192 atoms, 1600 functions, 100 x 590) with an
    open-shell density pair (P^a over 256 orbitals, P^b over the first 250),
    one parent atom at a time (an O and an H), against stored oracle values
    (tests/golden/cluster64_ext_atoms.json, written by
    make_cluster64_ext_golden.py from the oracle alone): E_xc, N_e, V^a and
    V^b on a seeded sample of entries and every row sum, to 1e-10."""
    from workloads.density import open_shell_densities
    gold = _golden_ext()
    w = cfg_water_cluster()
    assert (w.n_rad, w.n_ang, w.nbf) == (gold["n_rad"], gold["n_ang"], gold["nbf"])
    o = gold["open_shell"]
    Pa, Pb = open_shell_densities(w.S, o["n_alpha"], o["n_beta"], seed=o["seed"])
    for g in gold["atoms"]:
        mask = np.zeros(w.natoms, np.uint8)
        mask[g["atom"]] = 1
        say(f"case uks cluster64 atom {g['atom']} (Z {g['Z']})")
        E, N, Va, Vb, st = _gpu_uks(w, Pa, Pb, "pbe", atom_mask=mask)
        u = g["uks_pbe"]
        say(f"  dE {E - u['E_xc']:.3e} dN {N - u['N_e']:.3e} max n_b {st['max_nb']}")
        assert abs(E - u["E_xc"]) <= TOL and abs(N - u["N_e"]) <= TOL
        r, c = np.array(g["sample_rows"]), np.array(g["sample_cols"])
        _check_v("Va", Va, u["Va"], r, c)
        _check_v("Vb", Vb, u["Vb"], r, c)


def test_becke_partition_parity():
    """Open-shell water, PBE, Becke's size-adjusted partition (40 x 110)."""
    w = cfg_water(n_rad=40, n_ang=110)
    Pa, Pb = _open_shell(w)
    say("case uks water becke")
    g = _gpu_uks(w, Pa, Pb, "pbe", partition="becke", becke_radius=w.becke_radius)
    o = integrate_uks(w.coords, w.mk_alpha, w.basis, Pa, Pb, "pbe", w.n_rad, w.ang,
                      ssf_a=w.ssf_a, screen_eta=w.screen_eta, rho_thresh=w.rho_thresh,
                      partition="becke", becke_radius=w.becke_radius)
    _compare("pbe becke", g, o)
