"""Seeded contracted Cartesian Gaussian basis sets and their analytic overlap.

A basis shell follows the paper's definition (Sec. 2.1, eq. gau_cart): one
centre, one angular momentum L, one list of exponents and contraction
coefficients shared by its (L+1)(L+2)/2 Cartesian functions. The coefficient
array stored here is used verbatim as d_xi by every consumer; the
normalisation below is only a property of how the inputs are generated.

The overlap matrix S (Gaussian product rule with a binomial expansion of the
one-dimensional moments) is used to scale the density matrix so that
tr(P S) equals the electron count, and by the tests that check the grid
recovers tr(P S).
"""
from dataclasses import dataclass
from math import comb

import numpy as np


def n_cart(L):
    return (L + 1) * (L + 2) // 2


def cart_exponents(L):
    """Cartesian (l, m, n) triples of one shell, lexicographic: for L=2
    xx, xy, xz, yy, yz, zz."""
    out = []
    for l in range(L, -1, -1):
        for m in range(L - l, -1, -1):
            out.append((l, m, L - l - m))
    return out


def _dfact(n):
    """(n)!! with (-1)!! = 0!! = 1."""
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


@dataclass
class BasisSet:
    shell_atom: np.ndarray    # int32 [nshells]
    shell_L: np.ndarray       # int32 [nshells]
    shell_nprim: np.ndarray   # int32 [nshells]
    prim_alpha: np.ndarray    # float64 [sum nprim], packed in shell order
    prim_coef: np.ndarray     # float64 [sum nprim]
    # int32 [nshells] or None: 1 marks a shell of L >= 2 whose functions are
    # the 2L+1 real solid harmonics instead of the Cartesian components
    # (L <= 1 shells stay Cartesian whatever the flag says)
    shell_pure: np.ndarray = None

    @property
    def nshells(self):
        return int(self.shell_L.shape[0])

    def is_pure(self, s):
        return (self.shell_pure is not None and bool(self.shell_pure[s])
                and int(self.shell_L[s]) >= 2)

    @property
    def any_pure(self):
        return any(self.is_pure(s) for s in range(self.nshells))

    def cartesian(self):
        """The same shells with every function Cartesian."""
        return BasisSet(self.shell_atom, self.shell_L, self.shell_nprim, self.prim_alpha,
                        self.prim_coef)

    @property
    def prim_offset(self):
        off = np.zeros(self.nshells + 1, dtype=np.int64)
        np.cumsum(self.shell_nprim, out=off[1:])
        return off

    @property
    def shell_nfunc(self):
        return np.array([2 * int(L) + 1 if self.is_pure(s) else n_cart(int(L))
                         for s, L in enumerate(self.shell_L)], dtype=np.int64)

    @property
    def first_func(self):
        f = np.zeros(self.nshells + 1, dtype=np.int64)
        np.cumsum(self.shell_nfunc, out=f[1:])
        return f

    @property
    def nbf(self):
        return int(self.shell_nfunc.sum())

    def shell(self, s):
        o = self.prim_offset
        return (int(self.shell_atom[s]), int(self.shell_L[s]),
                self.prim_alpha[o[s]:o[s + 1]], self.prim_coef[o[s]:o[s + 1]])


# --- element recipes -----------------------------------------------------
# A geometric ladder of 12 exponents spanning [0.1, 5e3]. Each contracted
# shell takes a contiguous window of rungs (3-6 of them, seeded). Windows are
# (L, anchor, where) with where = "top" (window ends at the anchor rung) or
# "bottom" (window starts at the anchor rung).
LADDER = np.geomspace(0.1, 5.0e3, 12)

_HEAVY = [(0, 11, "top"), (0, 5, "top"), (0, 0, "bottom"),
          (1, 6, "top"), (1, 0, "bottom"), (2, 1, "bottom")]
_HYDROGEN = [(0, 5, "top"), (0, 0, "bottom"), (1, 1, "bottom")]
RECIPES = {1: _HYDROGEN, 6: _HEAVY, 7: _HEAVY, 8: _HEAVY}


def _prim_norm(alpha, L):
    """Normalisation of x^L exp(-alpha r^2)."""
    return np.sqrt((4.0 * alpha) ** L / _dfact(2 * L - 1)
                   * (2.0 * alpha / np.pi) ** 1.5)


def _self_overlap_xL(alpha, d, L):
    a = alpha[:, None] + alpha[None, :]
    m = _dfact(2 * L - 1) / (2.0 * a) ** L * (np.pi / a) ** 1.5
    return float(d @ m @ d)


def _contract(alpha, rng, L):
    c = rng.uniform(0.1, 1.0, size=alpha.shape[0])
    d = c * _prim_norm(alpha, L)
    return d / np.sqrt(_self_overlap_xL(alpha, d, L))


def element_shells(Z, seed, diffuse=None, polarisation=False):
    """The shells (L, alpha, d) of one element; identical for every atom of
    that element for a given seed. polarisation=True appends one more shell
    of higher angular momentum (f on C, N, O; d on H), two rungs wide, after
    the others (the earlier shells are unchanged)."""
    rng = np.random.default_rng([seed, int(Z)])
    out = []
    for L, anchor, where in RECIPES[int(Z)]:
        if L == 2:
            n = int(rng.integers(3, 5))
        else:
            n = int(rng.integers(3, 7))
        if where == "top":
            lo = max(0, anchor - n + 1)
            idx = np.arange(lo, anchor + 1)
        else:
            idx = np.arange(anchor, min(len(LADDER), anchor + n))
        alpha = LADDER[idx][::-1].copy()          # tight -> diffuse
        out.append((L, alpha, _contract(alpha, rng, L)))
    if diffuse is not None:
        alpha = np.array([float(diffuse)])
        out.append((0, alpha, _contract(alpha, rng, 0)))
    if polarisation:
        L = 2 if int(Z) == 1 else 3
        alpha = LADDER[[3, 2]].copy()
        out.append((L, alpha, _contract(alpha, rng, L)))
    return out


def make_basis(Z, seed=2007, diffuse=None, polarisation=False, pure=False):
    """Basis for a molecule with atomic numbers Z (shells in atom order).
    pure=True marks every shell spherical (2L+1 real solid harmonics for
    L >= 2), as in the correlation-consistent basis sets."""
    atom, Ls, npr, al, co = [], [], [], [], []
    cache = {}
    for a, z in enumerate(Z):
        z = int(z)
        if z not in cache:
            cache[z] = element_shells(z, seed, diffuse, polarisation)
        for L, alpha, d in cache[z]:
            atom.append(a)
            Ls.append(L)
            npr.append(alpha.shape[0])
            al.append(alpha)
            co.append(d)
    return BasisSet(np.array(atom, dtype=np.int32), np.array(Ls, dtype=np.int32),
                    np.array(npr, dtype=np.int32),
                    np.ascontiguousarray(np.concatenate(al)),
                    np.ascontiguousarray(np.concatenate(co)),
                    np.ones(len(Ls), dtype=np.int32) if pure else None)


# --- analytic overlap ------------------------------------------------------
def _moment(t, p):
    """integral x^t exp(-p x^2) dx over the real line (array p)."""
    if t % 2:
        return np.zeros_like(p)
    return _dfact(t - 1) / (2.0 * p) ** (t // 2) * np.sqrt(np.pi / p)


def overlap_matrix(basis, coords, chunk=200000):
    """Analytic overlap S of the Cartesian basis at atom coordinates coords.
    A basis with spherical shells is refused (use basis.cartesian() for the
    overlap of the Cartesian functions the shells are built from)."""
    if basis.any_pure:
        raise ValueError("overlap_matrix covers Cartesian shells only")
    nb = basis.nbf
    S = np.zeros((nb, nb))
    ff = basis.first_func
    po = basis.prim_offset
    cen = coords[basis.shell_atom]
    maxp = int(basis.shell_nprim.max())
    # padded primitive tables (zero coefficient for padding)
    A = np.ones((basis.nshells, maxp))
    D = np.zeros((basis.nshells, maxp))
    for s in range(basis.nshells):
        n = po[s + 1] - po[s]
        A[s, :n] = basis.prim_alpha[po[s]:po[s + 1]]
        D[s, :n] = basis.prim_coef[po[s]:po[s + 1]]
    Ls = basis.shell_L
    for La in np.unique(Ls):
        for Lb in np.unique(Ls):
            sa = np.nonzero(Ls == La)[0]
            sb = np.nonzero(Ls == Lb)[0]
            ia, ib = np.meshgrid(sa, sb, indexing="ij")
            ia = ia.ravel()
            ib = ib.ravel()
            ca, cb = cart_exponents(int(La)), cart_exponents(int(Lb))
            for c0 in range(0, ia.shape[0], chunk):
                pa, pb = ia[c0:c0 + chunk], ib[c0:c0 + chunk]
                RA, RB = cen[pa], cen[pb]
                AB2 = ((RA - RB) ** 2).sum(axis=1)
                blk = np.zeros((pa.shape[0], len(ca), len(cb)))
                for xi in range(maxp):
                    for eta in range(maxp):
                        a_all, b_all = A[pa, xi], A[pb, eta]
                        w_all = D[pa, xi] * D[pb, eta]
                        # pairs whose Gaussian prefactor underflows to exactly 0
                        # (exponent beyond 746) add exactly nothing: skip them
                        keep = np.nonzero((w_all != 0.0) & (
                            a_all * b_all / (a_all + b_all) * AB2 < 746.0))[0]
                        if keep.size == 0:
                            continue
                        a, b, w = a_all[keep], b_all[keep], w_all[keep]
                        RAk, RBk = RA[keep], RB[keep]
                        p = a + b
                        pref = w * np.exp(-a * b / p * AB2[keep])
                        Pc = (a[:, None] * RAk + b[:, None] * RBk) / p[:, None]
                        PA, PB = Pc - RAk, Pc - RBk
                        # one-dimensional overlaps I[axis][l1][l2]
                        I = np.zeros((3, La + 1, Lb + 1, keep.size))
                        for ax in range(3):
                            for l1 in range(La + 1):
                                for l2 in range(Lb + 1):
                                    acc = np.zeros(keep.size)
                                    for i in range(l1 + 1):
                                        for j in range(l2 + 1):
                                            t = i + j
                                            if t % 2:
                                                continue
                                            acc += (comb(l1, i) * comb(l2, j)
                                                    * PA[:, ax] ** (l1 - i)
                                                    * PB[:, ax] ** (l2 - j)
                                                    * _moment(t, p))
                                    I[ax, l1, l2] = acc
                        for u, (l1, m1, n1) in enumerate(ca):
                            for v, (l2, m2, n2) in enumerate(cb):
                                blk[keep, u, v] += (pref * I[0, l1, l2]
                                                    * I[1, m1, m2] * I[2, n1, n2])
                rows = ff[pa][:, None, None] + np.arange(len(ca))[None, :, None]
                cols = ff[pb][:, None, None] + np.arange(len(cb))[None, None, :]
                S[rows, cols] = blk
    return S
