"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmarks.

This module only draws random numbers and shapes them into lattice fields.  It
holds none of the domain-wall operator's arithmetic, so the CPU oracle and the
GPU library can both read its arrays without sharing any method code.

Canonical host layouts (complex128, C order):

* gauge field      ``[V][mu=x,y,z,t][row 3][col 3]``; ``U_mu(x)`` links x -> x+mu
* 5D fermion       ``[V][s][spin 4][colour 3]``
* 4D site index    ``n = x + Lx*(y + Ly*(z + Lz*t))``

The random SU(3) links follow the usual "hot-ish start" recipe: draw eight
standard normal coefficients h_a, form H = sum_a h_a lambda_a / 2 from the
Gell-Mann matrices, exponentiate U = exp(i eps H) through the eigen
decomposition of the Hermitian H, and re-unitarise (Gram-Schmidt of rows 0 and
1, row 2 = conj(row0 x row1)) so that det U = 1 to rounding.  The paper's own
runs use a thermalised 16^3x48 Iwasaki ensemble which is not available; these
fields stand in for it in lattice shape and size only.
"""

from __future__ import annotations

import dataclasses
import numpy as np

__all__ = [
    "gell_mann",
    "random_su3",
    "gauge_field",
    "gauge_transform",
    "gaussian_fermion",
    "rational_shifts",
    "Workload",
    "WORKLOADS",
]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3) complex128."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _reunitarise(u: np.ndarray) -> np.ndarray:
    r0 = u[:, 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=1, keepdims=True)
    r1 = u[:, 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=1, keepdims=True)
    r2 = np.cross(r0, r1).conj()
    return np.stack([r0, r1, r2], axis=1)


def random_su3(n: int, eps: float, rng: np.random.Generator, chunk: int = 1 << 18) -> np.ndarray:
    """``n`` matrices exp(i eps H), H = sum_a h_a lambda_a/2, h_a ~ N(0,1); shape (n,3,3)."""
    lam = gell_mann() / 2
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        h = rng.standard_normal((hi - lo, 8))
        H = np.einsum("na,aij->nij", h, lam)
        w, v = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        u = np.einsum("nij,nj,nkj->nik", v, ph, v.conj())
        out[lo:hi] = _reunitarise(u)
    return out


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """Seeded SU(3) gauge field in canonical layout ``[V][4][3][3]`` complex128."""
    V = int(np.prod(dims))
    rng = np.random.Generator(np.random.PCG64(seed))
    return random_su3(4 * V, eps, rng).reshape(V, 4, 3, 3)


def gauge_transform(dims, seed: int, eps: float = 1.0) -> np.ndarray:
    """Seeded local SU(3) rotation g(x), shape ``[V][3][3]``."""
    V = int(np.prod(dims))
    rng = np.random.Generator(np.random.PCG64(seed))
    return random_su3(V, eps, rng)


def gaussian_fermion(dims, Ls: int, seed: int, nsites: int | None = None) -> np.ndarray:
    """Seeded 5D fermion, Re and Im i.i.d. N(0,1); shape ``[V][Ls][4][3]``.

    ``nsites`` overrides the 4D site count (used for single-parity fields,
    whose first axis is the checkerboard index of length V/2).
    """
    V = int(np.prod(dims)) if nsites is None else int(nsites)
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((V, Ls, 4, 3, 2))
    return z[..., 0] + 1j * z[..., 1]


def rational_shifts(n: int = 12, lo: float = 1e-4, hi: float = 10.0) -> np.ndarray:
    """n shifts log-spaced in [lo, hi] with both endpoints included."""
    return np.logspace(np.log10(lo), np.log10(hi), n)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One benchmark / parity workload: lattice, Moebius parameters and seeds."""

    name: str
    dims: tuple
    Ls: int
    b: float
    c: float
    M5: float
    mf: float
    dirichlet: tuple
    eps: float
    gauge_seed: int
    source_seeds: tuple
    tol: float

    @property
    def V(self) -> int:
        return int(np.prod(self.dims))


# Sizes and parameters of the five workloads the hot path is measured on.
# Gauge seed 1000+i for workload i; source seeds as listed.
WORKLOADS = {
    "4^4x8_periodic": Workload("4^4x8_periodic", (4, 4, 4, 4), 8, 1.5, 0.5, 1.8, 0.01,
                               (0, 0, 0, 0), 0.4, 1001, (2001,), 1e-10),
    "16^4x12_dirichlet": Workload("16^4x12_dirichlet", (16, 16, 16, 16), 12, 1.5, 0.5, 1.8, 0.01,
                                  (1, 1, 1, 1), 0.7, 1002, (2002,), 1e-8),
    "32^4x12_dirichlet": Workload("32^4x12_dirichlet", (32, 32, 32, 32), 12, 1.5, 0.5, 1.8, 0.005,
                                  (1, 1, 1, 1), 0.9, 1003, (2003, 2004, 2005, 2006), 1e-8),
    "16^4x12_multishift": Workload("16^4x12_multishift", (16, 16, 16, 16), 12, 1.5, 0.5, 1.8, 0.01,
                                   (1, 1, 1, 1), 0.7, 1004, tuple(range(2010, 2018)), 1e-8),
    "24^4x12_fgcr": Workload("24^4x12_fgcr", (24, 24, 24, 24), 12, 1.5, 0.5, 1.8, 0.01,
                             (0, 0, 0, 0), 0.7, 1005, (2020, 2021, 2022, 2023), 1e-8),
    "8^4x8_train": Workload("8^4x8_train", (8, 8, 8, 8), 8, 1.5, 0.5, 1.8, 0.01,
                            (0, 0, 0, 0), 0.7, 1100, (), 1e-8),
}
