"""Synthetic workloads: grid sizes, coefficient fields and right-hand sides.

Conventions shared by every consumer:

* ``n`` is the number of unknowns per side; there are ``N = n**dim`` unknowns,
  ordered lexicographically with coordinate ``x0`` fastest.  The grid spacing
  is ``h = 1/(n+1)`` with homogeneous Dirichlet data on the boundary of the
  unit square/cube (the model problem of Sections 3.1-3.2 of the paper).
* ``a[k]`` holds the coefficient on the staggered links along axis ``k``.  As
  a C-ordered numpy array its shape lists the axes from ``x_{dim-1}`` down to
  ``x0`` and has ``n+1`` entries along axis ``k`` and ``n`` along the others.
  Link ``j`` along axis ``k`` joins the unknowns with ``x_k = j-1`` and
  ``x_k = j``; links ``0`` and ``n`` touch the boundary.
* Right-hand sides are ``N x nrhs`` Fortran-ordered arrays (column ``r`` is
  one right-hand side).

Every random draw uses numpy's PCG64 generator with the seed stated on the
workload, so both sides of a comparison see identical bits.
"""
from __future__ import annotations

from dataclasses import dataclass, field as dc_field
from typing import Dict, List, Optional

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    dim: int
    n: int
    leaf: int
    eps: float
    field: str
    nrhs: int
    seed_a: Optional[int]
    seed_f: int
    precision: str
    note: str = ""
    extra_nrhs: tuple = dc_field(default_factory=tuple)
    wavelengths: float = 0.0   # kappa > 0: b = -(2 pi kappa)^2 (Helmholtz), else b = 0
    sketch: bool = False       # randomized ID (Gaussian sketch of each tall group block)

    @property
    def N(self) -> int:
        return self.n ** self.dim


# The paper's benchmark families (Examples 1, 2, 4, 5) at the sizes this
# project measures.  Field recipes:
#   const               a = 1 on every link (Examples 1 and 4)
#   bernoulli_contrast  a = 10**(4*Bernoulli(1/2) - 2) i.i.d. per link, i.e.
#                       {1e-2, 1e2} (a quantized high-contrast field with
#                       contrast 1e4 as in Example 2, without the smoothing
#                       step)
#   lognormal_grf       log a a stationary Gaussian field, covariance
#                       exp(-r^2 / (2 (8h)^2)), standardized to mean 0, std 1
#   loguniform          a = 10**(2*U(-1,1)) i.i.d. per link
WORKLOADS: Dict[str, Workload] = {
    "laplace2d_n64": Workload(
        "laplace2d_n64", 2, 64, 8, 1e-6, "const", 1, None, 0, "fp64",
        "2D five-point Laplacian, N=4096, leaf 8x8"),
    "contrast2d_n1024": Workload(
        "contrast2d_n1024", 2, 1024, 16, 1e-6, "bernoulli_contrast", 16, 2, 20,
        "mixed_elim64", "2D high-contrast (1e4) field, N=1048576, leaf 16x16"),
    "laplace3d_n64": Workload(
        "laplace3d_n64", 3, 64, 4, 1e-6, "const", 64, None, 30, "mixed",
        "3D seven-point Laplacian, N=262144, leaf 4^3", sketch=True),
    "grf3d_n128": Workload(
        "grf3d_n128", 3, 128, 4, 1e-3, "lognormal_grf", 256, 4, 40, "mixed",
        "3D log-normal coefficient, N=2097152, leaf 4^3, eps=1e-3",
        extra_nrhs=(1,), sketch=True),
    # Example 3: a = 1, b = -k^2 with k = 2 pi kappa, 32 unknowns per
    # wavelength (kappa = 32 on the 1024^2 grid); indefinite, solved by GMRES
    "helmholtz2d_n1024": Workload(
        "helmholtz2d_n1024", 2, 1024, 16, 1e-6, "const", 16, None, 50, "mixed_elim64",
        "2D Helmholtz, 32 wavelengths across the square, N=1048576, leaf 16x16",
        wavelengths=32.0),
    # Example 6: the 3D analogue at 8 unknowns per wavelength (kappa = 8 on
    # the 64^3 grid)
    "helmholtz3d_n64": Workload(
        "helmholtz3d_n64", 3, 64, 4, 1e-6, "const", 16, None, 60, "mixed_elim64",
        "3D Helmholtz, 8 wavelengths across the cube, N=262144, leaf 4^3",
        wavelengths=8.0, sketch=True),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def coeff_shape(dim: int, n: int, k: int) -> tuple:
    """C-order shape of the link array along axis ``k``."""
    return tuple(n + 1 if (dim - 1 - pos) == k else n for pos in range(dim))


def _gaussian_field_half_lattice(dim: int, n: int, corr_len_cells: float,
                                 rng: np.random.Generator) -> np.ndarray:
    """White noise on the half-spacing lattice, smoothed by FFT filtering.

    The lattice has ``2n+3`` points per axis (positions ``i*h/2``), so DOF
    ``x`` sits at index ``2x+2`` and link ``j`` at index ``2j+1``.  Filtering
    white noise with a Gaussian kernel of standard deviation ``ell/sqrt(2)``
    gives the covariance ``exp(-r^2/(2 ell^2))`` with ``ell`` in lattice
    units (two per cell).
    """
    m = 2 * n + 3
    noise = rng.standard_normal((m,) * dim)
    ell = 2.0 * corr_len_cells
    sig = ell / np.sqrt(2.0)
    freqs = [np.fft.fftfreq(m)] * dim
    grids = np.meshgrid(*freqs, indexing="ij")
    k2 = sum(g * g for g in grids)
    filt = np.exp(-2.0 * (np.pi ** 2) * (sig ** 2) * k2)
    return np.real(np.fft.ifftn(np.fft.fftn(noise) * filt))


def make_field(dim: int, n: int, field: str, seed: Optional[int]) -> List[np.ndarray]:
    """Coefficient arrays ``a[0..dim-1]`` for one field recipe."""
    shapes = [coeff_shape(dim, n, k) for k in range(dim)]
    if field == "const":
        return [np.ones(s) for s in shapes]
    rng = np.random.Generator(np.random.PCG64(seed))
    if field == "bernoulli_contrast":
        out = []
        for s in shapes:
            bits = rng.integers(0, 2, size=s)
            out.append(10.0 ** (4.0 * bits - 2.0))
        return out
    if field == "loguniform":
        return [10.0 ** (2.0 * rng.uniform(-1.0, 1.0, size=s)) for s in shapes]
    if field == "lognormal_grf":
        g = _gaussian_field_half_lattice(dim, n, 8.0, rng)
        # g is indexed [i0, i1, ...] along x0, x1, ...; our arrays list axes
        # from x_{dim-1} down to x0, so transpose at the end.
        vals = []
        dof_idx = 2 * np.arange(n) + 2
        link_idx = 2 * np.arange(n + 1) + 1
        for k in range(dim):
            idx = [dof_idx] * dim
            idx[k] = link_idx
            sub = g[np.ix_(*idx)]            # axes x0, x1, ...
            vals.append(np.transpose(sub, tuple(range(dim - 1, -1, -1))))
        allv = np.concatenate([v.ravel() for v in vals])
        mu, sd = allv.mean(), allv.std()
        return [np.exp((v - mu) / sd) for v in vals]
    raise ValueError(f"unknown field {field!r}")


def make_coefficients(w: Workload) -> List[np.ndarray]:
    return make_field(w.dim, w.n, w.field, w.seed_a)


def helmholtz_b(N: int, wavelengths: float) -> np.ndarray:
    """The constant ``b = -(2 pi kappa)^2`` of a Helmholtz problem with
    ``kappa`` wavelengths across the unit square/cube."""
    return np.full(N, -(2.0 * np.pi * wavelengths) ** 2)


def make_b(w: Workload) -> Optional[np.ndarray]:
    """``b`` of a workload, or None (b = 0)."""
    return helmholtz_b(w.N, w.wavelengths) if w.wavelengths > 0 else None


def make_rhs(N: int, nrhs: int, seed: int) -> np.ndarray:
    """``N x nrhs`` standard normal right-hand sides, Fortran order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asfortranarray(rng.standard_normal((nrhs, N)).T)


def rank_model_problems():
    """The 48 problems of the rank-predictor study: 16 each at n=256, 512, 1024.

    Each entry is ``(problem_id, n, seed)``; the coefficient recipe is
    ``loguniform`` on a 2D grid with leaf 16 and eps 1e-6.  Problems 0-10 of
    each size are the training split, 11-15 the held-out split.
    """
    out = []
    pid = 0
    for n in (256, 512, 1024):
        for j in range(16):
            out.append((pid, n, 500 + pid, "train" if j < 11 else "test"))
            pid += 1
    return out
