"""Plain, slow FP64 CPU oracle for the XC integration of arXiv 2007.03143.

TEST INFRASTRUCTURE ONLY. Nothing in the library's product path may import,
call or link this package: it exists so that tests, the smoke check and the
CPU-baseline leg of the benchmark can check the HIP path against an
independent reading of the paper. It shares no code, constants or helpers
with the HIP implementation.

What it computes (Sec. 2.1-2.2 of the paper, summed over all batches):

    rho_i   = sum_{mu nu} P_{mu nu} phi~_mu(r_i) phi~_nu(r_i)
    grad_i  = 2 sum_{mu nu} P_{mu nu} grad phi~_mu(r_i) phi~_nu(r_i)
    sigma_i = grad_i . grad_i
    E_xc    = sum_i w_i e(rho_i, sigma_i)             (points with rho_i >= thresh)
    N_e     = sum_i w_i rho_i                          (all points)
    V_{mu nu} = sum_i w_i [ v_rho phi~_mu phi~_nu
                            + 2 v_sigma grad_i . (phi~_mu grad phi~_nu
                                                  + grad phi~_mu phi~_nu) ]

where phi~ is a basis function truncated at its shell's cutoff radius
(eq. rcut), w_i are the Stratmann-Scuseria-Frisch scaled weights of the
Mura-Knowles x Lebedev product grid (eq. num_int), and e = rho * eps is the
energy per unit volume with v_rho = de/drho and v_sigma = de/dsigma.
The batches, screening lists, compressed matrices and batched BLAS of
Sec. 2.2-2.3 reach exactly this result faster, so the oracle has no batches.

Parity unpinned: the absolute values of the VWN5 and PBE formulas against an
external functional library (none is available); they are pinned only by
the internal properties listed in the tests (limits, special cases,
symbolic derivatives, V = dE/dP by finite differences).
"""
from .quadrature import mura_knowles, atomic_grid, molecular_grid
from .partition import (ssf_cell, ssf_partition, ssf_weights, becke_cell,
                        becke_size_adjustment, becke_partition, becke_weights)
from .basis import cart_exponents, shell_rcut, collocation
from .screening import cuboid_sphere_intersect, screen_batch
from .functionals import slater, vwn5, pbe_x, pbe_c, evaluate
from .integrate import integrate, density_on_points, grid_and_weights

__all__ = [
    "mura_knowles", "atomic_grid", "molecular_grid", "ssf_cell",
    "ssf_partition", "ssf_weights", "becke_cell", "becke_size_adjustment",
    "becke_partition", "becke_weights", "cart_exponents", "shell_rcut",
    "collocation", "cuboid_sphere_intersect", "screen_batch", "slater",
    "vwn5", "pbe_x", "pbe_c", "evaluate", "integrate", "density_on_points",
    "grid_and_weights",
]
