"""Seeded synthetic inputs for the ParO plane-wave eigenproblem.

The paper's crystals (MgO, Al, Si inside Quantum ESPRESSO with norm-conserving
pseudopotential files) are not available, so cells of Gaussian
pseudo-atoms stand in for them: a local potential made of Gaussian wells
sampled on the FFT grid, Kleinman-Bylander projector descriptors (centre,
angular channel, width, energy) and random trial orbitals.

This module holds none of the eigensolver's arithmetic: no G-sphere, no
Fourier transform, no Hamiltonian.  It only draws random numbers in a fixed
order and evaluates the synthetic potential on grid points.  Both the CPU
oracle and the GPU path take their inputs from here.

Draw order for a cell with seed ``s`` (``numpy.random.default_rng(s)``):
atom positions ``U[0, a)^3``, well depths ``U(lo, hi)``, then one KB energy
``U(-1, 1)`` per (atom, l) with l = 0 (s) and l = 1 (p, shared by
p_x, p_y, p_z).  Trial orbitals come from an independent stream
``default_rng([s, 1])``: each coefficient is ``(x + i y)/sqrt(2)`` with
``x, y ~ N(0, 1)``, drawn as a (bands, n_g) array, band-major.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["CellSpec", "WORKLOADS", "make_cell", "vloc_on_grid", "trial_block",
           "small_cell", "batch_specs", "FFT_LENGTHS"]

# FFT grid lengths 2^a * {1, 3, 5} the GPU transforms support
FFT_LENGTHS = (8, 16, 24, 32, 40, 48, 64, 80, 96, 160)


@dataclass(frozen=True)
class CellSpec:
    """Shape of one synthetic workload (a cubic cell of Gaussian pseudo-atoms)."""
    name: str
    a: float                 # cubic lattice constant (bohr)
    ecut: float              # plane-wave cutoff (Ha)
    grid: int                # FFT grid points per axis
    n_atoms: int
    depth: tuple = (1.0, 3.0)   # well depth range (Ha), uniform
    width: float = 1.0          # well standard deviation (bohr)
    projectors: bool = False    # s + 3 p KB projectors per atom
    proj_width: float = 0.8     # projector Gaussian width (bohr)
    n_bands: int = 8            # N: orbitals whose eigenvalues are reported
    n_buffer: int = 0           # extra orbitals carried ("compute more orbitals")
    n_outer: int = 10           # ParO outer iterations (fixed-work runs)
    n_cg: int = 20              # PCG steps per source problem
    extra: dict = field(default_factory=dict)

    @property
    def cell(self) -> np.ndarray:
        return np.eye(3) * self.a

    @property
    def n_carried(self) -> int:
        return self.n_bands + self.n_buffer


# The workloads: a 1.5k-plane-wave cell without nonlocal part, a
# 34k-plane-wave cell with 32 atoms carrying s + p KB projectors (128 in all),
# and a 161k-plane-wave cell with 128 such atoms (512 projectors).
WORKLOADS = {
    "c0": CellSpec(name="c0_a10_ecut10_g32_n8", a=10.0, ecut=10.0, grid=32,
                   n_atoms=4, width=1.0, projectors=False,
                   n_bands=8, n_buffer=0, n_outer=10, n_cg=20),
    "c1": CellSpec(name="c1_a20_ecut20_g96_n128_p128", a=20.0, ecut=20.0,
                   grid=96, n_atoms=32, width=0.8, projectors=True,
                   proj_width=0.8, n_bands=128, n_buffer=32, n_outer=10,
                   n_cg=20),
    # mixed precision at scale: 161k plane waves, 128 atoms (512 projectors),
    # 512 orbitals plus 128 buffer orbitals
    "c3": CellSpec(name="c3_a30_ecut25_g160_n512_p512", a=30.0, ecut=25.0,
                   grid=160, n_atoms=128, width=0.8, projectors=True,
                   proj_width=0.8, n_bands=512, n_buffer=128, n_outer=10,
                   n_cg=20),
}


def small_cell(a=6.0, ecut=4.0, grid=16, n_atoms=2, projectors=True,
               n_bands=4, width=0.9, proj_width=0.7) -> CellSpec:
    """A tiny cell (a few hundred plane waves) for brute-force checks."""
    return CellSpec(name=f"tiny_a{a:g}_ecut{ecut:g}_g{grid}", a=a, ecut=ecut,
                    grid=grid, n_atoms=n_atoms, width=width,
                    projectors=projectors, proj_width=proj_width,
                    n_bands=n_bands, n_buffer=0, n_outer=4, n_cg=10)


def make_cell(spec: CellSpec, seed: int) -> dict:
    """Draw one cell: atom positions, well depths and KB projector descriptors.

    Returns a dict with ``cell`` (3x3, rows a1 a2 a3), ``ecut``, ``grid``
    (3 ints), ``positions`` (n_atoms x 3, Cartesian bohr), ``depths``,
    ``widths`` and ``projectors``: a list of dicts with keys ``center``,
    ``l``, ``m`` (m = 0, 1, 2 for p_x, p_y, p_z), ``width`` and ``d``.
    """
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, spec.a, size=(spec.n_atoms, 3))
    depths = rng.uniform(spec.depth[0], spec.depth[1], size=spec.n_atoms)
    projs = []
    if spec.projectors:
        dkb = rng.uniform(-1.0, 1.0, size=(spec.n_atoms, 2))
        for ia in range(spec.n_atoms):
            projs.append(dict(center=pos[ia].copy(), l=0, m=0,
                              width=spec.proj_width, d=float(dkb[ia, 0])))
            for m in range(3):
                projs.append(dict(center=pos[ia].copy(), l=1, m=m,
                                  width=spec.proj_width, d=float(dkb[ia, 1])))
    return dict(cell=spec.cell.copy(), ecut=float(spec.ecut),
                grid=(spec.grid,) * 3, positions=pos, depths=depths,
                widths=np.full(spec.n_atoms, spec.width), projectors=projs)


def vloc_on_grid(cell, grid, positions, depths, widths, images=2) -> np.ndarray:
    """Sum of Gaussian wells sampled on the FFT grid.

    V(r) = -sum_a d_a sum_L exp(-|r - R_a - L|^2 / (2 w_a^2)), with lattice
    images L = (l1 a1, l2 a2, l3 a3), |l_d| <= ``images``, and grid points
    r = (j1/N1) a1 + (j2/N2) a2 + (j3/N3) a3.  Returned in C order
    [j1][j2][j3].  The cell must be orthorhombic (all workloads are cubic),
    which makes each well a product of three one-dimensional factors.
    """
    cell = np.asarray(cell, dtype=np.float64)
    if np.any(np.abs(cell - np.diag(np.diag(cell))) > 0):
        raise ValueError("vloc_on_grid: orthorhombic cells only")
    lens = np.diag(cell)
    grid = tuple(int(g) for g in grid)
    v = np.zeros(grid, dtype=np.float64)
    ls = np.arange(-images, images + 1, dtype=np.float64)
    for R, d, w in zip(np.asarray(positions), np.asarray(depths), np.asarray(widths)):
        f = []
        for ax in range(3):
            x = np.arange(grid[ax], dtype=np.float64) * (lens[ax] / grid[ax])
            dx = x[:, None] - R[ax] - ls[None, :] * lens[ax]
            f.append(np.exp(-dx * dx / (2.0 * w * w)).sum(axis=1))
        v -= d * f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]
    return v


def trial_block(n_g: int, n_bands: int, seed: int) -> np.ndarray:
    """Random trial orbitals, (n_bands, n_g) complex128, band-major."""
    rng = np.random.default_rng([seed, 1])
    x = rng.standard_normal((n_bands, n_g))
    y = rng.standard_normal((n_bands, n_g))
    return (x + 1j * y) / np.sqrt(2.0)


def batch_specs(seed: int, n_cells: int = 24, a_range=(8.0, 18.0), ecut_range=(8.0, 20.0),
                bands_range=(8, 96), atoms_range=(4, 24)) -> list:
    """Independent cubic cells of uneven size for the batched runs.

    Draw order (``default_rng([seed, 2])``), per cell: lattice constant
    ``a ~ U(a_range)`` bohr, cutoff ``E_cut ~ U(ecut_range)`` Ha, orbital
    count ``N ~ U{bands_range}``, atom count ``~ U{atoms_range}``; every atom
    carries s + p projectors.  The FFT grid of each cell is an input of its
    problem statement: the smallest length of ``FFT_LENGTHS`` that is at least
    4 m + 1, with m = floor(sqrt(2 E_cut) a / (2 pi)) the largest Miller index
    a cubic cell's cutoff admits along an axis.  Cell ``i`` then draws its
    atoms with ``make_cell(spec, seed * 1000 + i)``.
    """
    rng = np.random.default_rng([seed, 2])
    out = []
    for i in range(n_cells):
        a = float(rng.uniform(*a_range))
        ecut = float(rng.uniform(*ecut_range))
        nb = int(rng.integers(bands_range[0], bands_range[1] + 1))
        na = int(rng.integers(atoms_range[0], atoms_range[1] + 1))
        m = int(np.floor(np.sqrt(2.0 * ecut) * a / (2.0 * np.pi)))
        grid = next(n for n in FFT_LENGTHS if n >= 4 * m + 1)
        out.append(CellSpec(name=f"batch{seed}_{i}_a{a:.2f}_ecut{ecut:.2f}_g{grid}_n{nb}", a=a, ecut=ecut,
                            grid=grid, n_atoms=na, width=0.9, projectors=True, proj_width=0.7,
                            n_bands=nb, n_buffer=0, n_outer=10, n_cg=10))
    return out
