"""Device memory from a caller-supplied allocator (xc_device_opts alloc/free):
torch's caching allocator and a counting allocator give the same E_xc, N_e
and V as the library's own hipMalloc, every buffer is given back on close,
and an allocation failure injected through the callback surfaces as
XC_ERR_NOMEM with the context still releasable and no memory leaked."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run(w, functional, allocator, wave_bytes=0):
    import torch
    from paper_2007_03143_amd import XcContext
    from workloads import grid_spec_dict
    ctx = XcContext(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w), wave_bytes=wave_bytes,
                    allocator=allocator)
    try:
        ctx.build_grid()
        P = torch.from_numpy(np.ascontiguousarray(w.P)).cuda()
        V, EN = ctx.integrate(P, functional)
        torch.cuda.synchronize()
        return EN.cpu().numpy().copy(), V.cpu().numpy().copy()
    finally:
        ctx.close()


class Counting:
    """Allocator over torch's caching allocator that counts live blocks and
    fails every request after the first `fail_after` ones."""

    def __init__(self, fail_after=None):
        self.live = {}
        self.calls = 0
        self.fail_after = fail_after

    def alloc(self, n):
        import torch
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return 0
        p = torch.cuda.caching_allocator_alloc(n)
        self.live[p] = n
        return p

    def free(self, p):
        import torch
        assert p in self.live, "free of a pointer the allocator did not give"
        del self.live[p]
        torch.cuda.caching_allocator_delete(p)


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_torch_allocator_matches_hipmalloc(functional):
    from workloads import cfg_water
    w = cfg_water(n_rad=40, n_ang=110)
    en0, v0 = _run(w, functional, None)
    en1, v1 = _run(w, functional, "torch")
    assert np.array_equal(en0, en1)
    assert np.abs(v1 - v0).max() <= 1e-13 * np.abs(v0).max()


def test_counting_allocator_gives_everything_back():
    from workloads import cfg_water_cluster
    w = cfg_water_cluster(4, n_rad=30, n_ang=50)
    ref, vref = _run(w, "pbe", None)
    c = Counting()
    # several waves, so buffers are also grown and re-obtained
    en, v = _run(w, "pbe", (c.alloc, c.free), wave_bytes=8 << 20)
    assert c.calls > 10
    assert not c.live, f"{len(c.live)} device buffers not given back"
    assert np.array_equal(en, ref)
    assert np.abs(v - vref).max() <= 1e-13 * np.abs(vref).max()


# the 0th and 5th allocations fall in the context's creation (atoms, pair
# tables, shells, primitives, angular table), the 30th in the grid build
@pytest.mark.parametrize("fail_after", [0, 5, 30])
def test_injected_allocation_failure(fail_after):
    import torch
    import paper_2007_03143_amd as pkg
    from paper_2007_03143_amd import XcContext
    from workloads import cfg_water, grid_spec_dict
    w = cfg_water(n_rad=30, n_ang=50)
    c = Counting(fail_after=fail_after)
    ctx = None
    try:
        with pytest.raises(pkg.XcError) as e:
            ctx = XcContext(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w),
                            allocator=(c.alloc, c.free))
            ctx.build_grid()
            P = torch.from_numpy(np.ascontiguousarray(w.P)).cuda()
            ctx.integrate(P, "lda")
            torch.cuda.synchronize()
        assert e.value.code == pkg.XC_ERR_NOMEM
        assert "allocator returned NULL" in str(e.value)
        assert c.calls == fail_after + 1
    finally:
        if ctx is not None:
            ctx.close()
    assert not c.live
    # the library is still usable afterwards
    en, _ = _run(w, "lda", None)
    assert np.isfinite(en).all()
