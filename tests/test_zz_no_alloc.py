"""xc_context_integrate_noalloc (scratch in the library's static device array,
no allocation) against xc_context_integrate on the same built contexts,
through the C ABI: two calls in a row, the second on a smaller molecule, so
that scratch contents left by the first call would show in the second."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _both(w, functional, precision, wave_bytes):
    import torch
    import paper_2007_03143_amd as pkg
    from workloads import grid_spec_dict
    stream = torch.cuda.current_stream()
    h, nbf = pkg.xc_context_create(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w),
                                   stream.cuda_stream, wave_bytes)
    try:
        pkg.xc_context_build_grid(h)
        st = pkg.xc_context_stats(h)
        P = torch.from_numpy(np.ascontiguousarray(w.P)).cuda()
        V1 = torch.empty((nbf, nbf), dtype=torch.float64, device="cuda")
        EN1 = torch.empty(2, dtype=torch.float64, device="cuda")
        pkg.xc_context_integrate(h, functional, precision, P.data_ptr(), V1.data_ptr(),
                                 EN1.data_ptr())
        V2 = torch.full((nbf, nbf), float("nan"), dtype=torch.float64, device="cuda")
        EN2 = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        pkg.xc_context_integrate_noalloc(h, functional, precision, P.data_ptr(),
                                         V2.data_ptr(), EN2.data_ptr())
        torch.cuda.synchronize()
        return (EN1.cpu().numpy(), V1.cpu().numpy(), EN2.cpu().numpy(), V2.cpu().numpy(),
                st)
    finally:
        pkg.xc_context_destroy(h)


@pytest.mark.parametrize("functional,precision", [("pbe", "fp64"), ("lda", "fp64"),
                                                  ("pbe", "fp32"), ("pbe", "bf16")])
def test_noalloc_matches_context_entry(functional, precision):
    from workloads import cfg_water, cfg_water_cluster
    big = cfg_water_cluster(4, functional=functional, n_rad=40, n_ang=110, seed=11)
    small = cfg_water(functional=functional, n_rad=30, n_ang=50)
    # the larger molecule in several waves (2 MiB each), the smaller one in one
    for w, wave_bytes in ((big, 2 << 20), (small, 0)):
        say(f"noalloc {w.name} {functional} {precision} wave_bytes={wave_bytes}")
        en1, v1, en2, v2, st = _both(w, functional, precision, wave_bytes)
        say(f"  waves {st['n_waves']} batches {st['n_batches']} wave scratch "
            f"{st['wave_bytes']} E {en1[0]:.14f} / {en2[0]:.14f}")
        if wave_bytes:
            assert st["n_waves"] > 1
        assert np.all(np.isfinite(en2)) and np.all(np.isfinite(v2))
        assert abs(en1[0] - en2[0]) <= 1e-10 and abs(en1[1] - en2[1]) <= 1e-10
        assert float(np.abs(v1 - v2).max()) <= 1e-10
        assert np.array_equal(v2, v2.T)


def test_noalloc_rejects_waves_above_the_static_maximum():
    import torch
    import paper_2007_03143_amd as pkg
    from workloads import cfg_water_cluster, grid_spec_dict
    w = cfg_water_cluster(8, functional="pbe", n_rad=40, n_ang=110, seed=12)
    stream = torch.cuda.current_stream()
    h, nbf = pkg.xc_context_create(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w),
                                   stream.cuda_stream, 0)
    try:
        pkg.xc_context_build_grid(h)
        st = pkg.xc_context_stats(h)
        say(f"one-wave scratch {st['wave_bytes']} bytes, static {pkg.STATIC_SCRATCH_BYTES}")
        assert st["n_waves"] == 1 and st["wave_bytes"] > pkg.STATIC_SCRATCH_BYTES
        P = torch.from_numpy(np.ascontiguousarray(w.P)).cuda()
        V = torch.zeros((nbf, nbf), dtype=torch.float64, device="cuda")
        EN = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
        with pytest.raises(pkg.XcError) as e:
            pkg.xc_context_integrate_noalloc(h, "pbe", "fp64", P.data_ptr(), V.data_ptr(),
                                             EN.data_ptr())
        assert e.value.code == pkg.XC_ERR_NOMEM and "static maximum" in str(e.value)
        torch.cuda.synchronize()
        assert EN.cpu().numpy().tolist() == [7.0, 7.0]
    finally:
        pkg.xc_context_destroy(h)


def test_noalloc_needs_a_built_context():
    import torch
    import paper_2007_03143_amd as pkg
    from workloads import cfg_water, grid_spec_dict
    w = cfg_water(n_rad=20, n_ang=50)
    h, nbf = pkg.xc_context_create(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w),
                                   torch.cuda.current_stream().cuda_stream, 0)
    try:
        P = torch.from_numpy(np.ascontiguousarray(w.P)).cuda()
        V = torch.zeros((nbf, nbf), dtype=torch.float64, device="cuda")
        EN = torch.zeros(2, dtype=torch.float64, device="cuda")
        with pytest.raises(pkg.XcError) as e:
            pkg.xc_context_integrate_noalloc(h, "lda", "fp64", P.data_ptr(), V.data_ptr(),
                                             EN.data_ptr())
        assert e.value.code == pkg.XC_ERR_STATE
    finally:
        pkg.xc_context_destroy(h)
