"""Helpers shared by the GPU tests: run the HIP path through the C ABI with
torch-owned device buffers, and the oracle on the same inputs."""
import sys

import numpy as np

import oracle


def gpu_integrate_prec(w, functional, precision, atom_mask=None, **grid_over):
    import torch
    from paper_2007_03143_amd import XcContext
    from workloads import grid_spec_dict
    ctx = XcContext(w.coords, w.mk_alpha, w.basis,
                    grid_spec_dict(w, atom_mask=atom_mask, **grid_over))
    try:
        Pd = torch.from_numpy(np.ascontiguousarray(w.P)).cuda()
        V, EN = ctx.integrate(Pd, functional, precision)
        torch.cuda.synchronize()
        en = EN.cpu().numpy()
        return float(en[0]), float(en[1]), V.cpu().numpy(), ctx.stats()
    finally:
        ctx.close()


def gpu_integrate(w, functional, atom_mask=None, wave_bytes=0, P=None, **grid_over):
    import torch
    from paper_2007_03143_amd import XcContext
    from workloads import grid_spec_dict
    g = grid_spec_dict(w, atom_mask=atom_mask, **grid_over)
    ctx = XcContext(w.coords, w.mk_alpha, w.basis, g, wave_bytes=wave_bytes)
    try:
        ctx.build_grid()
        Pd = torch.from_numpy(np.ascontiguousarray(w.P if P is None else P)).cuda()
        V, EN = ctx.integrate(Pd, functional)
        torch.cuda.synchronize()
        en = EN.cpu().numpy()
        return float(en[0]), float(en[1]), V.cpu().numpy(), ctx.stats()
    finally:
        ctx.close()


def _progress(stage, done, total):
    print(f"    oracle {stage} {done}/{total}", flush=True)


def oracle_integrate(w, functional, atom_mask=None, P=None, **grid_over):
    g = dict(ssf_a=w.ssf_a, screen_eta=w.screen_eta, rho_thresh=w.rho_thresh,
             partition="ssf", becke_radius=None)
    g.update({k: v for k, v in grid_over.items() if k in g})
    n_rad = grid_over.get("n_rad", w.n_rad)
    ang = grid_over.get("ang", w.ang)
    return oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P if P is None else P,
                            functional, n_rad, ang, atom_mask=atom_mask,
                            progress=_progress if w.natoms > 8 else None, **g)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


_CHAIN = {}


def chain600(n_rad=99, n_ang=590):
    """The 600-atom chain workload on an n_rad x n_ang grid. Its basis, S and
    P do not depend on the grid, so they are built once per process and
    shared (building them takes tens of seconds)."""
    import dataclasses
    from workloads import cfg_chain
    if "base" not in _CHAIN:
        say("  building the 600-atom chain workload (basis, S, P)")
        _CHAIN["base"] = cfg_chain()
    base = _CHAIN["base"]
    if (n_rad, n_ang) == (base.n_rad, base.n_ang):
        return base
    return dataclasses.replace(base, n_rad=n_rad, n_ang=n_ang, ang=None)
