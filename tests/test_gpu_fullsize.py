"""The 600-atom chain at its full size: 99 x 590 grid per atom (35,046,000
points), 6280 functions with the diffuse shell, PBE, in the launch
configuration bench.py uses (one context, waves planned from free memory).

A dense oracle evaluation of even one parent atom's grid of this molecule
takes minutes, so its oracle comparison runs on the reduced grid in
test_gpu_parity.py; here the full-size run is checked through properties
that hold at any size: exact symmetry of V, run-to-run determinism,
additivity over disjoint sets of parent atoms, independence of the batch
size, the electron count tr(PS) recovered by the grid, and the FP32
potential mode reproducing the FP64 density results bit for bit.
"""

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _chain():
    from gpu_util import chain600
    say("case chain600 full size")
    return chain600()


def _run(w, precision="fp64", atom_mask=None, **over):
    import torch
    from paper_2007_03143_amd import XcContext
    from workloads import grid_spec_dict
    ctx = XcContext(w.coords, w.mk_alpha, w.basis,
                    grid_spec_dict(w, atom_mask=atom_mask, **over))
    try:
        ctx.build_grid()
        P = torch.from_numpy(w.P).cuda()
        V, EN = ctx.integrate(P, "pbe", precision)
        torch.cuda.synchronize()
        en = EN.cpu().numpy()
        return float(en[0]), float(en[1]), V.cpu().numpy(), ctx.stats()
    finally:
        ctx.close()
        torch.cuda.empty_cache()


def test_chain600_full_size_properties():
    w = _chain()
    say(f"case chain600 full size: {w.natoms} atoms, {w.nbf} functions, "
        f"{w.n_rad} x {w.n_ang}")
    E, N, V, st = _run(w)
    say(f"  E {E!r} N {N!r} kept points {st['n_points']} batches {st['n_batches']} "
        f"waves {st['n_waves']} max n_b {st['max_nb']}")
    assert st["n_points"] > 0 and np.isfinite(E)
    assert np.array_equal(V, V.T) and np.isfinite(V).all()
    # the grid integrates the density to the electron count tr(PS) = 2 n_occ
    say(f"  N - tr(PS) = {N - 2 * w.n_occ:.3e}")
    assert abs(N - 2 * w.n_occ) <= 1e-5 * 2 * w.n_occ
    vmax = np.abs(V).max()

    # determinism: E and N come from fixed-order sums
    E2, N2, V2, _ = _run(w)
    assert E2 == E and N2 == N
    assert np.abs(V2 - V).max() <= 1e-12 * vmax

    # additivity over parent atoms (batches never straddle atoms)
    even = (np.arange(w.natoms) % 2 == 0).astype(np.uint8)
    Ea, Na, Va, _ = _run(w, atom_mask=even)
    Eb, Nb, Vb, _ = _run(w, atom_mask=1 - even)
    say(f"  even + odd - all: dE {Ea + Eb - E:.3e} dN {Na + Nb - N:.3e} "
        f"max dV {np.abs(Va + Vb - V).max():.3e}")
    assert abs(Ea + Eb - E) <= 1e-12 * abs(E)
    assert abs(Na + Nb - N) <= 1e-12 * abs(N)
    assert np.abs(Va + Vb - V).max() <= 1e-12 * vmax

    # a different batch size changes only the rounding
    E3, N3, V3, st3 = _run(w, batch_max=256)
    say(f"  batch_max 256: {st3['n_batches']} batches, dE {E3 - E:.3e} "
        f"max dV {np.abs(V3 - V).max():.3e}")
    assert abs(E3 - E) <= 1e-11 * abs(E) and abs(N3 - N) <= 1e-11 * abs(N)
    assert np.abs(V3 - V).max() <= 1e-11 * vmax

    # FP32 potential: the density side is FP64, so E and N are unchanged
    E4, N4, V4, _ = _run(w, precision="fp32v")
    say(f"  fp32v: dE {E4 - E:.3e} max dV {np.abs(V4 - V).max():.3e}")
    assert E4 == E and N4 == N
    assert np.abs(V4 - V).max() <= 1e-4
