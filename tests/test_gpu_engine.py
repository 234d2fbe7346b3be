"""Continuous-batching engine through the C ABI: every integration gives the
same result alone and co-batched with other requests (FP64: 1e-12 relative;
the only difference is the order of the FP64 atomic adds into V), admission
under a small device budget, and one request against the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import say
from workloads import cfg_water_cluster, grid_spec_dict
from workloads.density import perturbed_density

pytestmark = pytest.mark.gpu


def _requests(n=5, n_iter=3, precision="fp64"):
    from paper_2007_03143_amd.serving import ServeRequest
    out = []
    for i in range(n):
        nw = 1 + (i % 3)
        f = "lda" if i % 2 == 0 else "pbe"
        w = cfg_water_cluster(nw, functional=f, n_rad=40, n_ang=110, seed=100 + i,
                              n_occ=5 * nw)
        dens = [perturbed_density(w.P, 1e-3, seed=1000 * i + k) for k in range(n_iter)]
        out.append(ServeRequest(w.coords, w.mk_alpha, w.basis, grid_spec_dict(w), f, dens,
                                arrival=0.004 * i, precision=precision, name=w.name,
                                n_points_nominal=w.n_points_nominal))
    return out


def _alone(r):
    import torch
    from paper_2007_03143_amd import XcContext
    ctx = XcContext(r.coords, r.mk_alpha, r.basis, r.grid)
    res = []
    try:
        for P in r.densities:
            V, EN = ctx.integrate(torch.from_numpy(P).cuda(), r.functional, r.precision)
            torch.cuda.synchronize()
            en = EN.cpu().numpy()
            res.append((float(en[0]), float(en[1]), V.cpu().numpy()))
    finally:
        ctx.close()
    return res


@pytest.mark.parametrize("wave_bytes,budget", [(4 << 20, 0), (64 << 20, 0),
                                               (4 << 20, 96 << 20)])
def test_engine_alone_equals_mixed(wave_bytes, budget):
    from paper_2007_03143_amd.serving import serve
    reqs = _requests()
    say(f"case engine wave_bytes {wave_bytes} budget {budget}")
    ref = [_alone(r) for r in reqs]
    summary = serve(reqs, hbm_budget=budget, wave_bytes=wave_bytes, keep_v=lambda i: True)
    say(f"  {summary['integrations']} integrations, steps {summary['engine']['steps']}, "
        f"p50 {summary['latency_p50_ms']:.2f} ms p99 {summary['latency_p99_ms']:.2f} ms")
    assert summary["integrations"] == sum(len(r.densities) for r in reqs)
    for r, rr in zip(reqs, ref):
        assert len(r.results) == len(rr)
        for (E, N, V), (E0, N0, V0) in zip(r.results, rr):
            assert abs(E - E0) <= 1e-12 * abs(E0)
            assert abs(N - N0) <= 1e-12 * abs(N0)
            assert np.abs(V - V0).max() <= 1e-12 * np.abs(V0).max()
            assert np.array_equal(V, V.T)


def test_engine_mixed_precisions_and_oracle():
    from paper_2007_03143_amd.serving import serve
    reqs = _requests(n=4, n_iter=2)
    reqs[1].precision = "fp32"
    reqs[2].precision = "fp32v"
    reqs[3].precision = "bf16"
    ref = [_alone(r) for r in reqs]
    serve(reqs, wave_bytes=8 << 20, keep_v=lambda i: True)
    for r, rr in zip(reqs, ref):
        for (E, N, V), (E0, N0, V0) in zip(r.results, rr):
            assert abs(E - E0) <= 1e-12 * abs(E0)
            assert np.abs(V - V0).max() <= 1e-12 * np.abs(V0).max()
    r = reqs[0]
    Eo, No, Vo = oracle.integrate(r.coords, r.mk_alpha, r.basis, r.densities[1],
                                  r.functional, r.grid["n_rad"], r.grid["ang"])
    E, N, V = r.results[1]
    say(f"  engine vs oracle: dE {E - Eo:.2e} dN {N - No:.2e} dV {np.abs(V - Vo).max():.2e}")
    assert abs(E - Eo) <= 1e-10 and abs(N - No) <= 1e-10
    assert np.abs(V - Vo).max() <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_engine_phi_cache_same_results_fewer_collocations(precision):
    """Keeping each request's Phi across its integrations gives E_xc and N_e
    bit for bit (V to the atomic-add order) and runs collocation only for a
    request's first integration; without the cache every integration
    collocates."""
    from paper_2007_03143_amd.serving import serve
    runs = {}
    for cache in (False, True):
        reqs = _requests(n=4, n_iter=3, precision=precision)
        summary = serve(reqs, wave_bytes=8 << 20, keep_v=lambda i: True, cache_phi=cache)
        runs[cache] = (reqs, summary["engine"])
        say(f"case engine {precision} cache={cache}: colloc batches "
            f"{summary['engine']['colloc_batches']}, launched "
            f"{summary['engine']['batches_launched']}")
    (r0, e0), (r1, e1) = runs[False], runs[True]
    assert e0["colloc_batches"] == e0["batches_launched"]
    # first integration of each request only: a third of the batches
    assert e1["colloc_batches"] * 3 == e1["batches_launched"]
    for a, b in zip(r0, r1):
        for (E0, N0, V0), (E1, N1, V1) in zip(a.results, b.results):
            assert E0 == E1 and N0 == N1
            assert np.abs(V0 - V1).max() <= 1e-13 * np.abs(V0).max()


def test_release_with_work_in_flight_is_busy():
    """xc_engine_release of a request with a queued integration returns
    XC_ERR_BUSY and leaves it intact; once its ticket polls done the same
    release succeeds."""
    import torch
    import paper_2007_03143_amd as pkg
    from paper_2007_03143_amd.serving import XcEngine
    r = _requests(n=1, n_iter=1)[0]
    eng = XcEngine()
    try:
        rid, nbf = eng.add(r)
        P = torch.from_numpy(r.densities[0]).cuda()
        V = torch.empty((nbf, nbf), dtype=torch.float64, device="cuda")
        EN = torch.empty(2, dtype=torch.float64, device="cuda")
        t = eng.submit(rid, P, V, EN)
        with pytest.raises(pkg.XcError) as e:
            eng.release(rid)
        assert e.value.code == pkg.XC_ERR_BUSY
        import time
        done, t0 = False, time.monotonic()
        while not done and time.monotonic() - t0 < 60.0:
            eng.step()
            done = eng.poll(t)
            if not done:
                time.sleep(0.001)   # the grid is built on the engine's builder thread
        assert done
        torch.cuda.synchronize()
        eng.release(rid)
        E0 = _alone(r)[0][0]
        assert abs(float(EN[0]) - E0) <= 1e-12 * abs(E0)
    finally:
        eng.close()
