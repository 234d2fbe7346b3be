"""Request loop over the continuous-batching engine of the C ABI.

Requests (molecules with a sequence of SCF densities) arrive over time; each
is added to the engine, which admits it when its device footprint fits and
then keeps its grid on the device while its integrations run one after the
other. Every loop turn calls one engine step, which co-batches the pending
grid batches of all in-flight integrations, and polls the tickets. Latency of
an integration is submit -> done as seen by this loop; throughput counts
nominal grid points of finished integrations per second of wall time.

The loop is argument marshalling and bookkeeping only: grid builds and all
integration work run in the library's HIP kernels.
"""
import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as B


@dataclass
class ServeRequest:
    coords: np.ndarray
    mk_alpha: np.ndarray
    basis: object
    grid: dict
    functional: str
    densities: object          # list of host (nbf, nbf) arrays, or a DeviceDensities
    arrival: float = 0.0       # seconds after the start of the stream
    precision: str = "fp64"
    name: str = ""
    n_points_nominal: int = 0
    # filled in by the loop
    req_id: int = -1
    k: int = 0
    results: list = field(default_factory=list)    # (E, N, V or None)
    int_latency: list = field(default_factory=list)
    t_done: float = 0.0


class DeviceDensities:
    """Seeded SCF-like densities made on the device from an S-orthonormal
    orbital set: C_raw ~ N(0, 1) (nbf x n_occ), C = C_raw (C_raw^T S C_raw)^-1/2,
    P_0 = 2 C C^T (so tr(P_0 S) = 2 n_occ), P_k = P_0 + delta_k with delta_k
    symmetric, standard normal, scaled to Frobenius norm `norm`. S is the
    host overlap matrix of the request's basis. Input generation only (torch
    on the device); the integrations themselves run in the library."""

    def __init__(self, S, n_occ, n_iter, seed, norm=1e-3):
        self.S, self.n_occ, self.n_iter, self.seed, self.norm = S, n_occ, n_iter, seed, norm
        self.nbf = S.shape[0]
        self._p0 = None

    def __len__(self):
        return self.n_iter

    def _gen(self, salt):
        import torch
        g = torch.Generator(device="cuda")
        g.manual_seed(int(self.seed) * 1000003 + salt)
        return g

    def device(self, k):
        import torch
        if self._p0 is None:
            C = torch.randn(self.nbf, self.n_occ, generator=self._gen(0), device="cuda",
                            dtype=torch.float64)
            S = torch.from_numpy(np.ascontiguousarray(self.S)).cuda()
            M = C.T @ (S @ C)
            ev, U = torch.linalg.eigh(0.5 * (M + M.T))
            C = C @ ((U / torch.sqrt(ev)) @ U.T)
            P0 = 2.0 * (C @ C.T)
            self._p0 = (0.5 * (P0 + P0.T)).contiguous()
        d = torch.randn(self.nbf, self.nbf, generator=self._gen(k + 1), device="cuda",
                        dtype=torch.float64)
        d = 0.5 * (d + d.T)
        d *= self.norm / torch.linalg.norm(d)
        return (self._p0 + d).contiguous()

    def host(self, k):
        return self.device(k).cpu().numpy()

    def release(self):
        self._p0 = None


class XcEngine:
    """Thin owner of an engine handle and its torch buffers."""

    def __init__(self, hbm_budget=0, wave_bytes=0, stream=None, cache_phi=True):
        import torch
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = B.xc_engine_create(self.stream.cuda_stream, hbm_budget, wave_bytes,
                                         cache_phi)

    def add(self, r):
        rid, nbf = B.xc_engine_add_request(self.handle, r.coords, r.mk_alpha, r.basis,
                                           r.grid, r.functional, r.precision)
        return rid, nbf

    def submit(self, rid, P, V, EN):
        return B.xc_engine_submit(self.handle, rid, P.data_ptr(), V.data_ptr(),
                                  EN.data_ptr())

    def step(self):
        return B.xc_engine_step(self.handle)

    def poll(self, ticket):
        return B.xc_engine_poll(self.handle, ticket)

    def release(self, rid):
        B.xc_engine_release(self.handle, rid)

    def stats(self):
        return B.xc_engine_stats(self.handle)

    def close(self):
        if self.handle is not None:
            B.xc_engine_destroy(self.handle)
            self.handle = None


def serve(requests, hbm_budget=0, wave_bytes=0, keep_v=None, log=None, exclude=(),
          cache_phi=True, log_every=1):
    """Run the request stream; returns a summary dict. keep_v(i) -> bool selects
    requests whose V matrices are copied back (for accuracy checks); requests
    whose index is in `exclude` are served like the others but left out of
    the throughput and latency figures. log(msg), if given, hears of every
    log_every-th finished request."""
    import torch
    eng = XcEngine(hbm_budget, wave_bytes, cache_phi=cache_phi)
    order = sorted(range(len(requests)), key=lambda i: requests[i].arrival)
    nxt = 0
    inflight = {}      # ticket -> (request index, submit time, P, V, EN)
    n_done_int = 0
    n_done_req = 0
    points_done = 0
    t0 = time.perf_counter()

    def submit(i):
        r = requests[i]
        if isinstance(r.densities, DeviceDensities):
            P = r.densities.device(r.k)
        else:
            P = torch.from_numpy(np.ascontiguousarray(r.densities[r.k])).cuda()
        nbf = P.shape[0]
        V = torch.empty((nbf, nbf), dtype=torch.float64, device="cuda")
        EN = torch.empty(2, dtype=torch.float64, device="cuda")
        t = eng.submit(r.req_id, P, V, EN)
        inflight[t] = (i, time.perf_counter(), P, V, EN)

    try:
        while nxt < len(order) or inflight:
            now = time.perf_counter() - t0
            while nxt < len(order) and requests[order[nxt]].arrival <= now:
                i = order[nxt]
                r = requests[i]
                r.req_id, _ = eng.add(r)
                submit(i)
                nxt += 1
            if not inflight:
                wait = requests[order[nxt]].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
                continue
            eng.step()
            for t in list(inflight):
                if not eng.poll(t):
                    continue
                i, ts, P, V, EN = inflight.pop(t)
                r = requests[i]
                te = time.perf_counter()
                en = EN.cpu().numpy()
                vv = V.cpu().numpy() if (keep_v is not None and keep_v(i)) else None
                r.results.append((float(en[0]), float(en[1]), vv))
                r.int_latency.append(te - ts)
                if i not in exclude:
                    n_done_int += 1
                    points_done += r.n_points_nominal
                r.k += 1
                if r.k < len(r.densities):
                    submit(i)
                else:
                    r.t_done = te - t0
                    eng.release(r.req_id)
                    if isinstance(r.densities, DeviceDensities):
                        r.densities.release()
                    n_done_req += 1
                    if log and n_done_req % log_every == 0:
                        log(f"request {i} {r.name} done ({n_done_req} of {len(requests)}): "
                            f"{len(r.results)} iterations, t = {r.t_done:.3f} s")
        wall = time.perf_counter() - t0
        st = eng.stats()
    finally:
        eng.close()
    kept = [r for i, r in enumerate(requests) if i not in exclude]
    lat = np.array([x for r in kept for x in r.int_latency])
    req_lat = np.array([r.t_done - r.arrival for r in kept])
    return {
        "wall_s": wall,
        "integrations": n_done_int,
        "points_per_s": points_done / wall if wall > 0 else 0.0,
        "integrations_per_s": n_done_int / wall if wall > 0 else 0.0,
        "latency_p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
        "latency_p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
        "request_latency_p50_s": float(np.percentile(req_lat, 50)) if req_lat.size else None,
        "request_latency_p99_s": float(np.percentile(req_lat, 99)) if req_lat.size else None,
        "engine": st,
    }
