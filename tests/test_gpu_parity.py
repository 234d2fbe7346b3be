"""HIP path against the oracle, through the C ABI (Sec. 2.1-2.3).

Tolerances: |dE_xc| <= 1e-10 Eh and max|dV_xc| <= 1e-10 for FP64; grid
points and weights to 1e-13 relative; batching and screening lists exact.
"""
import numpy as np
import pytest

import oracle
from gpu_util import gpu_integrate, oracle_integrate, say
from workloads import cfg_water, cfg_water_cluster, grid_spec_dict, make_basis
from workloads.molecules import Molecule
from workloads.configs import Workload
from workloads.basis import overlap_matrix
from workloads.density import random_density

pytestmark = pytest.mark.gpu

TOL_E = 1e-10
TOL_V = 1e-10


def _check(w, functional, **kw):
    say(f"case {w.name} {functional} " + str({k: (np.nonzero(v)[0].tolist() if k == 'atom_mask' else v) for k, v in kw.items() if k != "becke_radius"}))
    E, N, V, st = gpu_integrate(w, functional, **kw)
    okw = {k: v for k, v in kw.items()
           if k in ("atom_mask", "screen_eta", "n_rad", "partition", "becke_radius")}
    Eo, No, Vo = oracle_integrate(w, functional, **okw)
    say(f"  E gpu {E!r} oracle {Eo!r} dE {E - Eo:.3e} dN {N - No:.3e} "
        f"max dV {np.abs(V - Vo).max():.3e} batches {st['n_batches']} "
        f"max n_b {st['max_nb']} (row tiles {(st['max_nb'] + 63) // 64})")
    assert 0 < st["max_nb"] <= w.nbf
    assert abs(E - Eo) <= TOL_E
    assert abs(N - No) <= TOL_E
    assert np.abs(V - Vo).max() <= TOL_V
    assert np.array_equal(V, V.T)
    return E, N, V, st


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_water_parity(functional):
    E, N, V, st = _check(cfg_water(), functional)
    assert st["n_wide_waves"] == 0    # small batches: 64 x 64 density tiles


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_f_shell_parity(functional):
    """Angular momentum 3: an f shell on O and a d shell on each H (47
    Cartesian functions); the f shell's ten rows straddle the 16-row groups
    of the density epilogue."""
    w = cfg_water(polarisation=True)
    assert 3 in set(w.basis.shell_L.tolist())
    _check(w, functional)


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_spherical_shell_parity(functional):
    """Spherical shells (2L+1 real solid harmonics for the f shell on O and
    the d shells; 41 functions): the collocation, the density epilogue and
    the Z kernel form them from the Cartesian components; FP64 parity, and
    split BF16 within the mixed-precision bound."""
    from gpu_util import gpu_integrate_prec
    w = cfg_water(polarisation=True, pure=True)
    assert w.nbf == 41 and w.basis.any_pure
    _check(w, functional)
    Eo, No, Vo = oracle_integrate(w, functional)
    E, N, V, _ = gpu_integrate_prec(w, functional, "bf16")
    say(f"  bf16: dE {E - Eo:.3e} dN {N - No:.3e} max dV {np.abs(V - Vo).max():.3e}")
    assert abs(E - Eo) <= 1e-6 and abs(N - No) <= 1e-6


def test_water_no_truncation_parity():
    _check(cfg_water(n_rad=40, n_ang=146), "pbe", screen_eta=0.0)


def test_single_atom_parity():
    Z = np.array([1])
    X = np.array([[0.3, -0.2, 0.1]])
    b = make_basis(Z)
    S = overlap_matrix(b, X)
    P = random_density(S, 1, seed=3) + 0.01 * np.eye(b.nbf)
    w = Workload("h_atom", Molecule(Z.astype(np.int32), X), b, P, 1, 50, 194, "pbe")
    for f in ("lda", "pbe"):
        _check(w, f)


def test_empty_mask_gives_zero():
    w = cfg_water()
    E, N, V, st = gpu_integrate(w, "pbe", atom_mask=np.zeros(3, np.uint8))
    assert E == 0.0 and N == 0.0 and not V.any() and st["n_points"] == 0


def test_mask_parity_and_additivity():
    w = cfg_water()
    m = np.array([1, 0, 1], np.uint8)
    Ea, Na, Va, _ = _check(w, "pbe", atom_mask=m)
    Eb, Nb, Vb, _ = gpu_integrate(w, "pbe", atom_mask=1 - m)
    E, N, V, _ = gpu_integrate(w, "pbe")
    assert abs(Ea + Eb - E) <= 1e-12 * abs(E)
    assert np.abs(Va + Vb - V).max() <= 1e-12 * np.abs(V).max()


@pytest.mark.parametrize("batch_max,wave_bytes,merge", [(64, 0, 1), (1024, 0, 1),
                                                        (512, 1 << 20, 1), (512, 0, 0)])
def test_batching_and_wave_invariance(batch_max, wave_bytes, merge):
    w = cfg_water()
    E0, N0, V0, st0 = gpu_integrate(w, "pbe")
    E, N, V, st = gpu_integrate(w, "pbe", batch_max=batch_max, wave_bytes=wave_bytes,
                                batch_merge=merge)
    say(f"  batch_max {batch_max} merge {merge} waves {st['n_waves']} "
        f"batches {st['n_batches']} (default {st0['n_batches']})")
    assert st["max_ng"] <= batch_max
    assert abs(E - E0) <= 1e-12 * abs(E0)
    assert np.abs(V - V0).max() <= 1e-12 * np.abs(V0).max()


def test_repeat_runs_deterministic():
    w = cfg_water()
    E1, N1, V1, _ = gpu_integrate(w, "pbe")
    E2, N2, V2, _ = gpu_integrate(w, "pbe")
    assert E1 == E2 and N1 == N2
    assert np.abs(V1 - V2).max() <= 1e-14 * np.abs(V1).max()


def _grid_ctx(w, **over):
    from paper_2007_03143_amd import XcContext
    ctx = XcContext(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w, **over))
    ctx.build_grid()
    return ctx


def test_grid_points_and_weights_match_oracle():
    w = cfg_water()
    say("case grid export water")
    ctx = _grid_ctx(w)
    try:
        xyzw, idx = ctx.export_grid()
    finally:
        ctx.close()
    pts, wq, par = oracle.molecular_grid(w.coords, w.mk_alpha, w.n_rad, w.ang)
    wo = oracle.ssf_weights(pts, wq, par, w.coords)
    assert len(np.unique(idx)) == len(idx)
    assert np.abs(xyzw[:, :3] - pts[idx]).max() <= 1e-13 * np.abs(pts).max()
    full = np.zeros_like(wo)
    full[idx] = xyzw[:, 3]
    assert np.all(np.abs(full - wo) <= 1e-13 * wq)
    # every dropped point had zero weight up to the partition's rounding
    dropped = np.setdiff1d(np.arange(len(wo)), idx)
    assert np.all(wo[dropped] <= 1e-13 * wq[dropped])


@pytest.mark.parametrize("n_waters,n_rad,n_ang", [(400, 6, 14), (1400, 4, 6)])
def test_large_molecule_weights_match_oracle(n_waters, n_rad, n_ang):
    """Partition weights of molecules past the one-wave-per-point limit:
    1200 atoms (distance-ordered neighbour lists) and 4200 atoms (all-pairs
    products). The grids of two parent atoms (an O and an H) are built; the
    partition runs over every atom on both sides."""
    from paper_2007_03143_amd import XcContext
    from workloads.molecules import water_cluster
    from workloads.angular import lebedev_table
    from workloads.configs import MK_ALPHA
    mol = water_cluster(n_waters, box=25.0 * (n_waters / 64.0) ** (1.0 / 3.0), seed=11)
    basis = make_basis(mol.Z)
    mk = np.array([MK_ALPHA[int(z)] for z in mol.Z])
    ang = lebedev_table(n_ang)
    mask = np.zeros(mol.natoms, np.uint8)
    mask[[0, 3 * (n_waters // 2) + 1]] = 1
    say(f"case weights {mol.natoms} atoms, {n_rad} x {n_ang}")
    grid = dict(n_rad=n_rad, n_ang=n_ang, ang=ang, ssf_a=0.64, screen_eta=1e-10,
                batch_max=512, rho_thresh=1e-15, atom_mask=mask)
    ctx = XcContext(mol.coords, mk, basis, grid)
    try:
        ctx.build_grid()
        xyzw, idx = ctx.export_grid()
    finally:
        ctx.close()
    pts, wq, par = oracle.molecular_grid(mol.coords, mk, n_rad, ang, atom_mask=mask)
    wo = oracle.ssf_weights(pts, wq, par, mol.coords)
    assert len(np.unique(idx)) == len(idx)
    assert np.abs(xyzw[:, :3] - pts[idx]).max() <= 1e-13 * np.abs(pts).max()
    full = np.zeros_like(wo)
    full[idx] = xyzw[:, 3]
    say(f"  kept {len(idx)} of {len(wo)} points, max |dw|/w_q "
        f"{np.max(np.abs(full - wo) / wq):.2e}")
    assert np.all(np.abs(full - wo) <= 1e-13 * wq)
    dropped = np.setdiff1d(np.arange(len(wo)), idx)
    assert np.all(wo[dropped] <= 1e-13 * wq[dropped])


@pytest.mark.parametrize("name", ["water", "cluster8"])
def test_batches_and_screening_lists(name):
    w = cfg_water() if name == "water" else cfg_water_cluster(8, functional="pbe",
                                                               n_rad=40, n_ang=110)
    say(f"case batches {name}")
    ctx = _grid_ctx(w)
    try:
        xyzw, idx = ctx.export_grid()
        pp, bb, sp, sh = ctx.export_batches()
        st = ctx.stats()
    finally:
        ctx.close()
    n = xyzw.shape[0]
    assert pp[0] == 0 and pp[-1] == n and np.all(np.diff(pp) >= 1)
    assert np.all(np.diff(pp) <= w.batch_max)
    rng = np.random.default_rng(0)
    nb = len(pp) - 1
    check = np.arange(nb) if nb <= 400 else rng.choice(nb, 400, replace=False)
    rc2 = np.array([oracle.shell_rcut(w.basis.shell(s)[2], w.screen_eta) ** 2
                    for s in range(w.basis.nshells)])
    cen = w.coords[w.basis.shell_atom]
    for j in check:
        p = xyzw[pp[j]:pp[j + 1], :3]
        assert np.array_equal(bb[j, :3], p.min(0)) and np.array_equal(bb[j, 3:], p.max(0))
        ref = oracle.screen_batch(p, w.coords, w.basis, w.screen_eta)
        got = sh[sp[j]:sp[j + 1]]
        assert list(got) == ref, j
        # conservative: every shell that reaches a point of the batch is listed
        d2 = ((p[:, None, :] - cen[None]) ** 2).sum(-1)
        reach = np.nonzero((d2 <= rc2[None]).any(0))[0]
        assert set(reach) <= set(got)
    # batches never straddle parent atoms
    parent = idx // (w.n_rad * w.n_ang)
    for j in check:
        assert len(np.unique(parent[pp[j]:pp[j + 1]])) == 1


@pytest.mark.parametrize("atom", [0, 100])
def test_cluster_sampled_atoms_parity(atom):
    """The 64-water cluster at full size (192 atoms, 1600 functions, 100 x 590
    grid); the oracle checks the integrals over one parent atom's grid
    (an O and an H): FP64 to 1e-10, split BF16 to 1e-6 in E_xc and N_e
    (the mixed-precision bound), FP32 reported."""
    from gpu_util import gpu_integrate_prec
    w = cfg_water_cluster()
    mask = np.zeros(w.natoms, np.uint8)
    mask[atom] = 1
    say(f"case {w.name} pbe atom {atom}")
    E, N, V, st = gpu_integrate(w, "pbe", atom_mask=mask)
    Eo, No, Vo = oracle_integrate(w, "pbe", atom_mask=mask)
    say(f"  fp64: dE {E - Eo:.3e} dN {N - No:.3e} max dV {np.abs(V - Vo).max():.3e} "
        f"max n_b {st['max_nb']}")
    assert abs(E - Eo) <= TOL_E and abs(N - No) <= TOL_E
    assert np.abs(V - Vo).max() <= TOL_V and np.array_equal(V, V.T)
    for prec in ("bf16", "fp32"):
        Em, Nm, Vm, _ = gpu_integrate_prec(w, "pbe", prec, atom_mask=mask)
        say(f"  {prec}: dE {Em - Eo:.3e} dN {Nm - No:.3e} max dV {np.abs(Vm - Vo).max():.3e}")
        assert np.array_equal(Vm, Vm.T)
        if prec == "bf16":
            assert abs(Em - Eo) <= 1e-6 and abs(Nm - No) <= 1e-6
            assert np.abs(Vm - Vo).max() <= 1e-3
        else:
            assert abs(Em - Eo) <= 1e-4 and np.abs(Vm - Vo).max() <= 1e-3


def test_chain600_sampled_atoms_parity():
    """The 600-atom polypeptide-like chain (6280 functions with the diffuse
    shell): ten atoms per lane in the partition kernel and a large P. The
    radial x angular grid is reduced (30 x 50) so that the oracle's all-pairs
    partition over the two sampled parent atoms (a C and an H) stays short;
    the GPU still builds, partitions and batches every atom's grid."""
    from gpu_util import chain600
    say("case chain600 build workload")
    w = chain600(n_rad=30, n_ang=50)
    mask = np.zeros(w.natoms, np.uint8)
    heavy = int(np.nonzero(w.mol.Z == 6)[0][3])
    light = int(np.nonzero(w.mol.Z == 1)[0][7])
    mask[[heavy, light]] = 1
    _check(w, "pbe", atom_mask=mask)


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_mixed_fp32_error_vs_oracle(functional):
    """FP32 collocation and contractions, FP64 functional and sums: errors
    against the FP64 oracle are reported and bounded."""
    w = cfg_water()
    say(f"case water {functional} fp32")
    from gpu_util import gpu_integrate_prec
    E, N, V, st = gpu_integrate_prec(w, functional, "fp32")
    Eo, No, Vo = oracle_integrate(w, functional)
    say(f"  fp32: dE {E - Eo:.3e} dN {N - No:.3e} max dV {np.abs(V - Vo).max():.3e}")
    assert abs(E - Eo) <= 1e-5 and abs(N - No) <= 1e-5
    assert np.abs(V - Vo).max() <= 1e-4
    assert np.array_equal(V, V.T)


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_mixed_bf16_error_vs_oracle(functional):
    """Split BF16 (exact digit products in the density contraction, hi/lo
    products in the potential contraction), FP64 functional and sums: E_xc
    and N_e within 1e-6 of the FP64 oracle, V within 1e-3."""
    w = cfg_water()
    say(f"case water {functional} bf16")
    from gpu_util import gpu_integrate_prec
    E, N, V, st = gpu_integrate_prec(w, functional, "bf16")
    Eo, No, Vo = oracle_integrate(w, functional)
    say(f"  bf16: dE {E - Eo:.3e} dN {N - No:.3e} max dV {np.abs(V - Vo).max():.3e}")
    assert abs(E - Eo) <= 1e-6 and abs(N - No) <= 1e-6
    assert np.abs(V - Vo).max() <= 1e-3
    assert np.array_equal(V, V.T)


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_mixed_fp32_potential_error_vs_oracle(functional):
    """FP64 collocation and density contraction, FP32 Z and potential
    contraction: E_xc and N_e equal the FP64 path's bit for bit (and so meet
    the FP64 tolerance against the oracle); the V error is reported and
    bounded."""
    w = cfg_water()
    say(f"case water {functional} fp32v")
    from gpu_util import gpu_integrate_prec
    E, N, V, st = gpu_integrate_prec(w, functional, "fp32v")
    E64, N64, V64, _ = gpu_integrate_prec(w, functional, "fp64")
    Eo, No, Vo = oracle_integrate(w, functional)
    say(f"  fp32v: dE {E - Eo:.3e} dN {N - No:.3e} max dV {np.abs(V - Vo).max():.3e}")
    assert E == E64 and N == N64
    assert abs(E - Eo) <= TOL_E and abs(N - No) <= TOL_E
    assert np.abs(V - Vo).max() <= 1e-4
    assert np.array_equal(V, V.T)


def test_phi_cache_bitwise_and_invalidation():
    """Keeping Phi between integrations (one wave) gives the same E, N and V
    as recomputing it, across density matrices, functionals and the Phi
    storage types, and collocation runs only when the cached Phi cannot
    serve (first call, a change of storage type, a grid rebuild, several
    waves)."""
    import torch
    from paper_2007_03143_amd import XcContext
    w = cfg_water_cluster(n_waters=4, n_rad=30, n_ang=110)
    rng = np.random.default_rng(11)
    d = rng.normal(size=w.P.shape)
    P1 = w.P + 1e-3 * (d + d.T) / np.linalg.norm(d + d.T)
    Ps = [torch.from_numpy(np.ascontiguousarray(P)).cuda() for P in (w.P, P1)]
    calls = [(0, "pbe", "fp64"), (1, "pbe", "fp64"), (0, "lda", "fp64"),
             (1, "pbe", "fp32"), (0, "pbe", "bf16"), (1, "pbe", "fp32v"),
             (0, "lda", "fp64")]
    g = grid_spec_dict(w)
    ref = XcContext(w.coords, w.mk_alpha, w.basis, g)
    cached = XcContext(w.coords, w.mk_alpha, w.basis, g)
    multi = XcContext(w.coords, w.mk_alpha, w.basis, g, wave_bytes=4 << 20)
    try:
        for c in (ref, cached, multi):
            c.build_grid()
            c.set_timing(True)
        cached.set_phi_cache(True)
        multi.set_phi_cache(True)
        nw = multi.stats()["n_waves"]
        assert cached.stats()["n_waves"] == 1 and nw > 1

        def run(c, k, f, p):
            V, EN = c.integrate(Ps[k], f, p)
            torch.cuda.synchronize()
            return EN.cpu().numpy().copy(), V.cpu().numpy().copy()

        for k, f, p in calls:
            say(f"case phi cache: P{k} {f} {p}")
            en0, V0 = run(ref, k, f, p)
            en1, V1 = run(cached, k, f, p)
            en2, V2 = run(multi, k, f, p)
            tol = 1e-14 * np.abs(V0).max()
            assert np.array_equal(en0, en1), (en0, en1)
            assert np.abs(V1 - V0).max() <= tol
            assert np.abs(en2 - en0).max() <= 1e-12 * np.abs(en0).max()
            assert np.abs(V2 - V0).max() <= 1e-12 * np.abs(V0).max()
        # what collocation stores, by call: FP64, FP64, FP64, FP32, FP64 with
        # digit scales, FP64, FP64 -> collocation at calls 1, 4, 5 and 6
        assert ref.timing()["colloc"]["launches"] == len(calls)
        assert cached.timing()["colloc"]["launches"] == 4
        assert multi.timing()["colloc"]["launches"] == len(calls) * nw
        # a rebuild drops the cache; switching it off drops it too
        cached.build_grid()
        cached.set_timing(True)
        en1, V1 = run(cached, 0, "pbe", "fp64")
        en1b, _ = run(cached, 0, "pbe", "fp64")
        cached.set_phi_cache(False)
        en1c, _ = run(cached, 0, "pbe", "fp64")
        assert cached.timing()["colloc"]["launches"] == 2
        en0, V0 = run(ref, 0, "pbe", "fp64")
        assert np.array_equal(en0, en1) and np.array_equal(en0, en1b)
        assert np.array_equal(en0, en1c)
    finally:
        for c in (ref, cached, multi):
            c.close()


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_one_shot_host_entry_matches_oracle(functional):
    """xc_integrate with host P and host V (the one-shot entry point: it
    creates a context on the null stream, copies P in and V out) against the
    oracle, and equal to the context path's result."""
    import paper_2007_03143_amd as pkg
    w = cfg_water(functional)
    say(f"case one-shot host entry water {functional}")
    E, N, V = pkg.xc_integrate(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w), functional, w.P)
    Eo, No, Vo = oracle_integrate(w, functional)
    say(f"  dE {E - Eo:.3e} dN {N - No:.3e} max dV {np.abs(V - Vo).max():.3e}")
    assert abs(E - Eo) <= TOL_E and abs(N - No) <= TOL_E
    assert np.abs(V - Vo).max() <= TOL_V
    assert np.array_equal(V, V.T)
    Ec, Nc, Vc, _ = gpu_integrate(w, functional)
    assert Ec == E and Nc == N
    assert np.abs(Vc - V).max() <= 1e-14 * np.abs(V).max()
    # a mixed mode through the same entry
    E32, N32, V32 = pkg.xc_integrate(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w),
                                     functional, w.P, "fp32v")
    assert E32 == E and N32 == N
    assert np.abs(V32 - Vo).max() <= 1e-4


def test_footprint_matches_the_built_plan():
    """xc_context_footprint: before the build an estimate of min_bytes only;
    after it, cached_bytes is exactly what a one-wave context holds and
    min_bytes what a context with one batch per wave holds."""
    from paper_2007_03143_amd import XcContext
    w = cfg_water_cluster(n_waters=4, n_rad=30, n_ang=110)
    g = grid_spec_dict(w)
    one = XcContext(w.coords, w.mk_alpha, w.basis, g)
    each = XcContext(w.coords, w.mk_alpha, w.basis, g, wave_bytes=1)
    try:
        mn0, al0 = one.footprint()
        assert mn0 > 0 and al0 == 0
        one.build_grid()
        each.build_grid()
        mn, al = one.footprint()
        st1, st2 = one.stats(), each.stats()
        say(f"case footprint: estimate {mn0}, min {mn}, cached {al}, batches {st1['n_batches']}")
        assert st1["n_waves"] == 1 and st2["n_waves"] == st2["n_batches"] > 1
        assert al == st1["persistent_bytes"] + st1["wave_bytes"]
        assert each.footprint() == (mn, al)
        assert mn == st2["persistent_bytes"] + st2["wave_bytes"]
        assert 0 < mn < al
    finally:
        one.close()
        each.close()


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_becke_partition_sfg_parity(functional):
    """Becke's size-adjusted partition on the SFG grid of Table 2 (175 x 974
    per atom, 511,350 points for the water)."""
    w = cfg_water(n_rad=175, n_ang=974)
    E, N, V, st = _check(w, functional, partition="becke", becke_radius=w.becke_radius)
    assert st["n_points_nominal"] == 3 * 175 * 974


def test_becke_weights_match_oracle():
    """Grid weights of an 8-water cluster with Becke's partition against the
    oracle's, point by point, with and without the size adjustment."""
    w = cfg_water_cluster(8, functional="pbe", n_rad=30, n_ang=110)
    for radius in (w.becke_radius, None):
        say(f"case becke weights cluster8 adjusted={radius is not None}")
        ctx = _grid_ctx(w, partition="becke", becke_radius=radius)
        try:
            xyzw, idx = ctx.export_grid()
        finally:
            ctx.close()
        pts, wq, par = oracle.molecular_grid(w.coords, w.mk_alpha, w.n_rad, w.ang)
        wo = oracle.becke_weights(pts, wq, par, w.coords, radius)
        full = np.zeros_like(wo)
        full[idx] = xyzw[:, 3]
        say(f"  kept {len(idx)} of {len(wo)}, max |dw|/w_q {np.max(np.abs(full - wo) / wq):.2e}")
        assert np.all(np.abs(full - wo) <= 1e-13 * wq)


@pytest.mark.parametrize("n_waters", [40, 120, 300])
def test_becke_weights_many_atoms(n_waters):
    """Becke weights with the size adjustment for 120, 360 and 900 atoms (4,
    2 and 1 points per wave pass, up to 16 atoms per lane); the grids of two
    parent atoms (an O and an H) on a 4 x 6 grid, the partition over every
    atom on both sides."""
    from paper_2007_03143_amd import XcContext
    from workloads.molecules import water_cluster
    from workloads.angular import lebedev_table
    from workloads.configs import MK_ALPHA, BECKE_RADIUS
    mol = water_cluster(n_waters, box=25.0 * (n_waters / 64.0) ** (1.0 / 3.0), seed=13)
    basis = make_basis(mol.Z)
    mk = np.array([MK_ALPHA[int(z)] for z in mol.Z])
    rad = np.array([BECKE_RADIUS[int(z)] for z in mol.Z])
    ang = lebedev_table(6)
    mask = np.zeros(mol.natoms, np.uint8)
    mask[[0, 3 * (n_waters // 2) + 1]] = 1
    say(f"case becke weights {mol.natoms} atoms")
    grid = dict(n_rad=4, n_ang=6, ang=ang, ssf_a=0.64, screen_eta=1e-10, batch_max=512,
                rho_thresh=1e-15, atom_mask=mask, partition="becke", becke_radius=rad)
    ctx = XcContext(mol.coords, mk, basis, grid)
    try:
        ctx.build_grid()
        xyzw, idx = ctx.export_grid()
    finally:
        ctx.close()
    pts, wq, par = oracle.molecular_grid(mol.coords, mk, 4, ang, atom_mask=mask)
    wo = oracle.becke_weights(pts, wq, par, mol.coords, rad)
    full = np.zeros_like(wo)
    full[idx] = xyzw[:, 3]
    say(f"  kept {len(idx)} of {len(wo)}, max |dw|/w_q {np.max(np.abs(full - wo) / wq):.2e}")
    assert np.all(np.abs(full - wo) <= 1e-13 * wq)


def test_becke_cluster_parity():
    w = cfg_water_cluster(8, functional="pbe", n_rad=30, n_ang=110)
    _check(w, "pbe", partition="becke", becke_radius=w.becke_radius)


def test_functional_edge_cases_parity():
    """The functional kernel's threshold, large reduced gradient and small
    sigma branches against the oracle: an indefinite density (P_0 - 0.2 I,
    so rho < 0 wherever the basis functions' squares outweigh rho_0) on a
    fragment of the chain with its diffuse shells (long tails, large s)."""
    from workloads import cfg_chain
    w = cfg_chain(n_atoms=9, n_rad=40, n_ang=110)
    P = w.P - 0.2 * np.eye(w.nbf)
    Ep, Np, Vp, det = oracle.integrate(w.coords, w.mk_alpha, w.basis, P, "pbe", w.n_rad,
                                       w.ang, details=True)
    rho, sig = det["rho"], det["sigma"]
    pos = rho > 1e-15
    kf = (3 * np.pi ** 2 * np.abs(rho[pos])) ** (1 / 3)
    s_red = np.sqrt(sig[pos]) / (2 * kf * rho[pos])
    n_neg, n_big_s = int((rho < 0).sum()), int((s_red > 10).sum())
    n_small_sig = int((sig[pos] < 1e-20).sum())
    say(f"case functional edges: {n_neg} points with rho < 0, {n_big_s} with s > 10, "
        f"{n_small_sig} with sigma < 1e-20, of {rho.size}")
    assert n_neg > 500 and n_big_s > 100 and n_small_sig > 100
    for functional in ("lda", "pbe"):
        E, N, V, st = gpu_integrate(w, functional, P=P)
        if functional == "lda":
            Eo, No, Vo = oracle.integrate(w.coords, w.mk_alpha, w.basis, P, "lda", w.n_rad,
                                          w.ang)
        else:
            Eo, No, Vo = Ep, Np, Vp
        say(f"  {functional}: dE {E - Eo:.3e} dN {N - No:.3e} max dV {np.abs(V - Vo).max():.3e}")
        assert abs(E - Eo) <= TOL_E and abs(N - No) <= TOL_E
        assert np.abs(V - Vo).max() <= TOL_V


def test_chain600_full_grid_atoms_match_golden():
    """The 600-atom chain at its full grid (99 x 590 per atom, the partition
    over all 600 atoms, 6280 functions) against stored oracle values for a C
    and an H parent atom (tests/golden/chain600_atoms.json, written by
    make_chain600_golden.py from the oracle alone): E_xc and N_e, V on a
    seeded sample of entries and every row sum of V, all to 1e-10. Both atoms
    reach screened function counts above 2048 (more than 32 row tiles)."""
    import json
    import os
    from gpu_util import chain600
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "chain600_atoms.json")))
    w = chain600()
    assert (w.n_rad, w.n_ang, w.nbf) == (gold["n_rad"], gold["n_ang"], gold["nbf"])
    for g in gold["atoms"]:
        mask = np.zeros(w.natoms, np.uint8)
        mask[g["atom"]] = 1
        say(f"case chain600 full grid atom {g['atom']} (Z {g['Z']})")
        E, N, V, st = gpu_integrate(w, "pbe", atom_mask=mask)
        r, c = np.array(g["sample_rows"]), np.array(g["sample_cols"])
        dv = np.abs(V[r, c] - np.array(g["sample_values"])).max()
        drs = np.abs(V.sum(axis=1) - np.array(g["row_sums"])).max()
        say(f"  dE {E - g['E_xc']:.3e} dN {N - g['N_e']:.3e} sampled max dV {dv:.3e} "
            f"({len(r)} entries) max d(row sum) {drs:.3e}; batches {st['n_batches']} "
            f"max n_b {st['max_nb']} (row tiles {(st['max_nb'] + 63) // 64})")
        assert st["max_nb"] > 2048
        # these batches are large enough for the 64 x 128 FP64 density tiles
        say(f"  waves {st['n_waves']}, with 64 x 128 density tiles {st['n_wide_waves']}")
        assert st["n_wide_waves"] == st["n_waves"]
        assert abs(E - g["E_xc"]) <= TOL_E and abs(N - g["N_e"]) <= TOL_E
        assert dv <= TOL_V and drs <= TOL_V
        assert np.array_equal(V, V.T)


@pytest.mark.parametrize("prec", ["bf16", pytest.param("fp32", marks=pytest.mark.xfail(
    strict=True, reason="FP32 collocation and contractions: the rounding errors of P and "
                        "Phi are coherent over a radial shell's equal s-function values, "
                        "-8.4e-6 Eh on this cluster (1.1e-7 on one water)"))])
def test_mixed_whole_cluster_within_1e6_of_fp64(prec):
    """The mixed-precision bound on the whole 64-water cluster (192 atoms,
    100 x 590), against the FP64 path: split BF16 meets |dE_xc| <= 1e-6 Eh;
    all-FP32 does not (expected failure, kept to record it)."""
    from gpu_util import gpu_integrate_prec
    w = cfg_water_cluster()
    E, N, V, st = gpu_integrate(w, "pbe")
    Em, Nm, Vm, _ = gpu_integrate_prec(w, "pbe", prec)
    say(f"case water64 whole cluster {prec}: dE {Em - E:.3e} dN {Nm - N:.3e} "
        f"max dV {np.abs(Vm - V).max():.3e}")
    assert abs(Em - E) <= 1e-6 and abs(Nm - N) <= 1e-6
