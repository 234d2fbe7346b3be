"""Meta-GGA (TPSS) integration on the HIP path against the oracle's
meta-GGA quadrature (oracle/meta.py), through the C ABI: the kinetic energy
density from the contraction of P with the gradient slabs, the TPSS
functional and the v_tau term of V. Same bar as the other FP64 parity
tests: |dE_xc|, |dN_e| and max|dV| at most 1e-10."""
import numpy as np
import pytest

from gpu_util import gpu_integrate, say
from oracle.meta import integrate_mgga
from workloads import cfg_water, cfg_water_cluster, grid_spec_dict

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _oracle(w, P=None, **over):
    return integrate_mgga(w.coords, w.mk_alpha, w.basis, w.P if P is None else P, w.n_rad,
                          w.ang, ssf_a=w.ssf_a, screen_eta=w.screen_eta,
                          rho_thresh=w.rho_thresh, **over)


def _compare(tag, g, o):
    E, N, V = g[:3]
    Eo, No, Vo = o[:3]
    say(f"  {tag}: E gpu {E!r} oracle {Eo!r} dE {E - Eo:.3e} dN {N - No:.3e} "
        f"max dV {np.abs(V - Vo).max():.3e}")
    assert abs(E - Eo) <= TOL and abs(N - No) <= TOL
    assert np.abs(V - Vo).max() <= TOL
    assert np.array_equal(V, V.T)


def test_water_parity():
    w = cfg_water(n_rad=50, n_ang=194)
    say("case tpss water 50 x 194")
    _compare("tpss", gpu_integrate(w, "tpss"), _oracle(w))


def test_spherical_water_parity():
    w = cfg_water(polarisation=True, pure=True, n_rad=40, n_ang=146)
    say("case tpss spherical water (f on O, d on H)")
    _compare("tpss", gpu_integrate(w, "tpss"), _oracle(w))


def test_cluster_many_waves_parity():
    w = cfg_water_cluster(8, n_rad=30, n_ang=86)
    say("case tpss cluster8, 1 MiB waves")
    g = gpu_integrate(w, "tpss", wave_bytes=1 << 20)
    say(f"  waves {g[3]['n_waves']} batches {g[3]['n_batches']}")
    assert g[3]["n_waves"] > 1
    _compare("tpss", g, _oracle(w))


def test_indefinite_density_parity():
    """P_0 - 0.2 I: points with rho < 0 (skipped), with tau < tau_W (z held
    at 1) and with large reduced gradients, against the oracle."""
    from workloads import cfg_chain
    w = cfg_chain(n_atoms=9, n_rad=30, n_ang=86)
    P = w.P - 0.2 * np.eye(w.nbf)
    o = _oracle(w, P=P, details=True)
    rho, sig, tau = o[3]
    pos = rho >= 1e-15
    n_clamp = int((tau[pos] <= sig[pos] / (8 * rho[pos])).sum())
    say(f"case tpss indefinite density: {int((rho < 0).sum())} points with rho < 0, "
        f"{n_clamp} with tau <= tau_W, of {rho.size}")
    assert n_clamp > 100
    _compare("tpss", gpu_integrate(w, "tpss", P=P), o)


def test_chain_atom_wide_tiles_parity():
    """One H parent atom of the 600-atom chain on a small grid (12 x 26
    points; partition over all 600 atoms, 6280 functions): its batches
    screen in more than 512 functions, so the density passes (rho and the
    three gradient slabs of tau) run on 64 x 128 tiles."""
    from gpu_util import chain600
    w = chain600(n_rad=12, n_ang=26)
    mask = np.zeros(w.natoms, np.uint8)
    mask[int(np.nonzero(w.mol.Z == 1)[0][7])] = 1
    say("case tpss chain600 one H atom 12 x 26")
    g = gpu_integrate(w, "tpss", atom_mask=mask)
    say(f"  waves {g[3]['n_waves']} wide {g[3]['n_wide_waves']} max n_b {g[3]['max_nb']}")
    assert g[3]["n_wide_waves"] == g[3]["n_waves"] > 0
    _compare("tpss", g, _oracle(w, atom_mask=mask))


def test_context_switches_between_plans():
    """On one context: PBE, TPSS (re-plans with the meta-GGA room), PBE
    again: the restricted results are unchanged bit for bit in E_xc and N_e."""
    import torch
    from paper_2007_03143_amd import XcContext
    w = cfg_water()
    ctx = XcContext(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w))
    try:
        P = torch.from_numpy(w.P).cuda()
        out = []
        for f in ("pbe", "tpss", "pbe"):
            V, EN = ctx.integrate(P, f)
            torch.cuda.synchronize()
            out.append((float(EN[0]), float(EN[1]), V.cpu().numpy()))
        say(f"case plan switch: E pbe {out[0][0]!r} tpss {out[1][0]!r} pbe {out[2][0]!r}")
        assert out[0][0] == out[2][0] and out[0][1] == out[2][1]
        assert np.abs(out[0][2] - out[2][2]).max() <= 1e-14 * np.abs(out[0][2]).max()
        Eo, No, Vo = _oracle(w)
        assert abs(out[1][0] - Eo) <= TOL and np.abs(out[1][2] - Vo).max() <= TOL
    finally:
        ctx.close()


def test_one_shot_host_entry():
    import paper_2007_03143_amd as pkg
    w = cfg_water(n_rad=40, n_ang=110)
    say("case tpss one-shot host entry")
    E, N, V = pkg.xc_integrate(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w), "tpss", w.P)
    _compare("tpss", (E, N, V), _oracle(w))


def test_unsupported_combinations_rejected():
    import torch
    from paper_2007_03143_amd import XcContext, XcError
    w = cfg_water(n_rad=20, n_ang=50)
    ctx = XcContext(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w))
    try:
        P = torch.from_numpy(w.P).cuda()
        with pytest.raises(XcError):
            ctx.integrate(P, "tpss", "fp32")
        with pytest.raises(XcError):
            ctx.integrate_uks(P / 2, P / 2, "tpss")
    finally:
        ctx.close()


def test_cluster_atoms_match_golden():
    """TPSS on the 64-water cluster (192 atoms, 1600 functions, 100 x 590),
    one parent atom at a time (an O and an H), against stored oracle values
    (tests/golden/cluster64_ext_atoms.json, written by
    make_cluster64_ext_golden.py from the oracle alone): E_xc, N_e, V on a
    seeded sample of entries and every row sum, to 1e-10."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "cluster64_ext_atoms.json")))
    w = cfg_water_cluster()
    assert (w.n_rad, w.n_ang, w.nbf) == (gold["n_rad"], gold["n_ang"], gold["nbf"])
    for g in gold["atoms"]:
        mask = np.zeros(w.natoms, np.uint8)
        mask[g["atom"]] = 1
        say(f"case tpss cluster64 atom {g['atom']} (Z {g['Z']})")
        E, N, V, st = gpu_integrate(w, "tpss", atom_mask=mask)
        t = g["tpss"]
        r, c = np.array(g["sample_rows"]), np.array(g["sample_cols"])
        dv = np.abs(V[r, c] - np.array(t["V"]["sample_values"])).max()
        drs = np.abs(V.sum(axis=1) - np.array(t["V"]["row_sums"])).max()
        say(f"  dE {E - t['E_xc']:.3e} dN {N - t['N_e']:.3e} sampled max dV {dv:.3e} "
            f"max d(row sum) {drs:.3e} max n_b {st['max_nb']}")
        assert abs(E - t["E_xc"]) <= TOL and abs(N - t["N_e"]) <= TOL
        assert dv <= TOL and drs <= TOL
        assert np.array_equal(V, V.T)


@pytest.mark.parametrize("functional", ["tpss"])
def test_becke_partition_parity(functional):
    """TPSS with Becke's size-adjusted partition (water, 40 x 110)."""
    w = cfg_water(n_rad=40, n_ang=110)
    say("case tpss water becke")
    g = gpu_integrate(w, "tpss", partition="becke", becke_radius=w.becke_radius)
    _compare("tpss becke", g, _oracle(w, partition="becke", becke_radius=w.becke_radius))
