"""Configuration records and seeded random draws (no model or method arithmetic).

Every random quantity of a workload is drawn here from
``numpy.random.default_rng([config_id, stream])`` with a fixed stream per kind of
draw, so that the oracle and the GPU path see bit-identical inputs:

  stream 0  lattice jitter          stream 3  sketch matrix Omega
  stream 1  nuclear charges Z       stream 4  sizes of a ragged batch
  stream 2  vacancies               stream 5  network initialisation
                                    stream 6  training-pair sampling

The physical setting follows the one-dimensional reduced Hartree-Fock model of
Sec. 4.1 (Eqs. (4.1)-(4.4)): Gaussian pseudocharges of width sigma and charge Z
on a periodic lattice, Yukawa interaction with screening kappa and prefactor
4*pi/eps0.  The two-dimensional lattices of Sec. 4.2 use the same model on a
square grid.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Config:
    """One workload.

    dim        spatial dimension d (1 or 2)
    sites      lattice sites per axis (n_1[, n_2]); N_A = prod(sites) before vacancies
    a          lattice spacing (bohr)
    jitter     half-width of the uniform per-axis offset of every site
    z          ("const", Z) or ("uniform", lo, hi); uniform draws are rescaled so
               that sum(Z) = f * N_e exactly (charge neutrality)
    sigma      Gaussian pseudocharge width
    n          grid points per axis; h = a * sites / n
    n_cheb     number of Chebyshev shifts N_c
    n_mu       ISDF rank N_mu
    r          sketch width r (columns of Omega)
    kappa, eps0  Yukawa screening and dielectric prefactor
    f          electrons per orbital (2 = spin degenerate)
    vacancy_frac  fraction of sites removed at random (0 = none)
    """
    cid: int
    dim: int
    sites: Tuple[int, ...]
    a: float
    jitter: float
    z: tuple
    sigma: float
    n: Tuple[int, ...]
    n_cheb: int
    n_mu: int
    r: int
    kappa: float = 0.01
    eps0: float = 1.0
    f: float = 2.0
    vacancy_frac: float = 0.0
    name: str = ""

    @property
    def box(self) -> Tuple[float, ...]:
        return tuple(self.a * s for s in self.sites)

    @property
    def h(self) -> float:
        hs = [self.a * s / n for s, n in zip(self.sites, self.n)]
        assert max(hs) - min(hs) < 1e-12, "grid spacing must be equal on all axes"
        return hs[0]

    @property
    def n_grid(self) -> int:
        return int(np.prod(self.n))


# The five workloads.  Readings of unstated parameters: eps0 = 1, f = 2,
# r = 8 (1D) / 16 (2D), jitter only where the workload names one, N_mu = 4 N_e
# where unstated.
CONFIGS = {
    1: Config(1, 1, (8,), 10.0, 0.1, ("const", 2.0), 1.0, (320,), 4, 32, 8,
              name="1D, 8 atoms, 320 grid points, N_c=4, N_mu=32"),
    2: Config(2, 1, (128,), 10.0, 0.0, ("uniform", 1.8, 2.2), 1.0, (5120,), 8, 512, 8,
              name="1D semiconductor-like, 128 atoms, 5120 grid points, N_c=8, N_mu=512"),
    3: Config(3, 2, (16, 16), 6.0, 0.05, ("const", 2.0), 0.8, (192, 192), 8, 1024, 16,
              name="2D insulator, 16x16 atoms, 192x192 grid, N_c=8, N_mu=1024"),
    5: Config(5, 2, (32, 32), 6.0, 0.0, ("uniform", 1.8, 2.2), 0.8, (384, 384), 8, 4096, 16,
              name="2D, 32x32 atoms, 384x384 grid, N_c=8, N_mu=4096"),
    # The paper's own 1D model (Sec. 4.1): spacing 2.4, kappa = 0.1, Z = 1,
    # sigma = 0.3, one electron per orbital, eps0 = 1 (insulator) or 10
    # (semiconductor); small jittered chains whose phonons are well conditioned.
    11: Config(11, 1, (8,), 2.4, 0.05, ("const", 1.0), 0.3, (192,), 8, 32, 8,
               kappa=0.1, eps0=1.0, f=1.0, name="paper 1D insulator, 8 atoms, h=0.1"),
    12: Config(12, 1, (8,), 2.4, 0.05, ("const", 1.0), 0.3, (192,), 8, 32, 8,
               kappa=0.1, eps0=10.0, f=1.0, name="paper 1D semiconductor, 8 atoms, h=0.1"),
    13: Config(13, 1, (60,), 2.4, 0.0, ("const", 1.0), 0.3, (1440,), 20, 240, 8,
               kappa=0.1, eps0=1.0, f=1.0, name="paper 1D insulator, 60 atoms, h=0.1"),
}


def get_config(cid: int) -> Config:
    return CONFIGS[cid]


def small_config(cid: int, dim: int, n_sites: int, pts_per_site: int, *, a: float = 10.0,
                 jitter: float = 0.1, z=("const", 2.0), sigma: float = 1.0,
                 n_cheb: int = 4, mu_per_e: int = 4, r: Optional[int] = None,
                 vacancy_frac: float = 0.0, kappa: float = 0.01, eps0: float = 1.0,
                 f: float = 2.0) -> Config:
    """A small workload of the same family (used for tests and the ragged batch)."""
    sites = (n_sites,) * dim
    n = (n_sites * pts_per_site,) * dim
    n_a = n_sites ** dim
    if r is None:
        r = 8 if dim == 1 else 16
    return Config(cid, dim, sites, a, jitter, z, sigma, n, n_cheb,
                  mu_per_e * n_a, r, kappa=kappa, eps0=eps0, f=f,
                  vacancy_frac=vacancy_frac, name=f"small-{cid}")


def _rng(cid: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([cid, stream])


def draw_sites(cfg: Config):
    """Site positions R (N_A x d), charges Z (N_A) after vacancies and rescaling.

    Site I of the ideal lattice sits at (I + 1/2) * a along each axis; the
    jitter is an independent uniform offset per site and axis.
    """
    d = cfg.dim
    grids = np.meshgrid(*[np.arange(s) for s in cfg.sites], indexing="ij")
    # first axis fastest (x fastest), matching the grid ordering alpha = ix + nx*iy
    idx = np.stack([g.ravel(order="F") for g in grids], axis=1)
    R = (idx + 0.5) * cfg.a
    n_all = R.shape[0]
    if cfg.jitter > 0:
        R = R + _rng(cfg.cid, 0).uniform(-cfg.jitter, cfg.jitter, size=R.shape)
    keep = np.ones(n_all, dtype=bool)
    if cfg.vacancy_frac > 0:
        n_vac = max(1, int(round(cfg.vacancy_frac * n_all)))
        vac = _rng(cfg.cid, 2).choice(n_all, size=n_vac, replace=False)
        keep[vac] = False
    kind = cfg.z[0]
    if kind == "const":
        Z = np.full(n_all, float(cfg.z[1]))
    elif kind == "uniform":
        Z = _rng(cfg.cid, 1).uniform(cfg.z[1], cfg.z[2], size=n_all)
    else:
        raise ValueError(kind)
    R = R[keep]
    Z = Z[keep]
    n_a = R.shape[0]
    n_e = n_a  # one doubly occupied orbital per site for Z ~ 2, f = 2
    if kind == "uniform":
        Z = Z * (cfg.f * n_e / Z.sum())
    # box lengths
    return R.reshape(n_a, d), Z, n_e


def n_electrons_orbitals(cfg: Config) -> int:
    return draw_sites(cfg)[2]


def draw_sketch(cfg: Config, n_p: int, seed_stream: int = 3) -> np.ndarray:
    """Gaussian sketch Omega (n_p x r), i.i.d. N(0, 1), column-major friendly."""
    return np.asfortranarray(_rng(cfg.cid, seed_stream).standard_normal((n_p, cfg.r)))


def draw_ragged_sizes(cid: int, count: int, lo: int, hi: int) -> np.ndarray:
    """Integer sizes drawn uniformly from [lo, hi] (inclusive)."""
    return _rng(cid, 4).integers(lo, hi + 1, size=count)


def ragged_batch_configs_2d(count: int = 16, lo: int = 4, hi: int = 12, *, pts_per_site: int = 12,
                            n_cheb: int = 8, vacancy_frac: float = 0.05, cid_base: int = 500,
                            size_seed: int = 5):
    """The 2D half of the uneven batch: `count` square lattices of k x k sites
    with k drawn uniformly from [lo, hi], spacing 6, Z = 2, sigma = 0.8, jitter
    0.05, 12 x 12 grid points per site, 5% vacancies (at least one), N_c = 8,
    N_mu = 4 N_e, r = 16.  Each system has its own seed streams (cid_base +
    index)."""
    sizes = draw_ragged_sizes(size_seed, count, lo, hi)
    out = []
    for i, k in enumerate(sizes):
        cfg = small_config(cid_base + i, 2, int(k), pts_per_site, a=6.0, sigma=0.8, jitter=0.05,
                           n_cheb=n_cheb, vacancy_frac=vacancy_frac, r=16)
        n_e = draw_sites(cfg)[2]
        out.append(dataclasses.replace(cfg, n_mu=4 * n_e,
                                       name=f"ragged 2D lattice {i}: {k}x{k} sites, {n_e} occupied"))
    return out


def ragged_batch_configs(count: int = 16, lo: int = 16, hi: int = 128, *, pts_per_site: int = 40,
                         n_cheb: int = 8, vacancy_frac: float = 0.05, cid_base: int = 400,
                         size_seed: int = 4):
    """The 1D half of the uneven batch: `count` chains with N_A drawn uniformly
    from [lo, hi], spacing 10, Z = 2, sigma = 1, 40 grid points per site, 5%
    vacancies (at least one), N_c = 8, N_mu = 4 N_e (N_e after the vacancies),
    r = 8.  Each system has its own seed streams (cid_base + index)."""
    sizes = draw_ragged_sizes(size_seed, count, lo, hi)
    out = []
    for i, n_a in enumerate(sizes):
        cfg = small_config(cid_base + i, 1, int(n_a), pts_per_site, jitter=0.0, n_cheb=n_cheb,
                           vacancy_frac=vacancy_frac)
        n_e = draw_sites(cfg)[2]
        out.append(dataclasses.replace(cfg, n_mu=4 * n_e,
                                       name=f"ragged 1D chain {i}: {n_a} sites, {n_e} occupied"))
    return out
