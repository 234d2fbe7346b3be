"""Seeded synthetic workloads for the XC integration path.

This module produces *inputs only*: molecular geometries, a contracted
Cartesian Gaussian basis, a density matrix, and the Lebedev angular table.
It holds none of the integration arithmetic (no grid, no partition weights,
no collocation, no functional). Both the oracle and the HIP path receive
the arrays it returns.

The paper's molecules (Taxol ... Ubiquitin) and its basis-set data are not
available; these seeded generators stand in for them with the same kinds of
structure (atom-centred contracted shells with core and diffuse exponents,
water clusters, a polypeptide-like chain).
"""
from .basis import BasisSet, make_basis, overlap_matrix, n_cart
from .molecules import (water, water_cluster, peptide_chain, Molecule)
from .density import random_density
from .angular import lebedev_table
from .configs import (Workload, cfg_water, cfg_water_cluster, cfg_chain,
                      cfg_serving_request, grid_spec_dict)

__all__ = [
    "BasisSet", "make_basis", "overlap_matrix", "n_cart", "water",
    "water_cluster", "peptide_chain", "Molecule", "random_density",
    "lebedev_table", "Workload", "cfg_water", "cfg_water_cluster",
    "cfg_chain", "cfg_serving_request", "grid_spec_dict",
]
