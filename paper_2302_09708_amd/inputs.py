"""Seeded synthetic inputs for one CheFSI problem (grid, Veff, projectors, X0).

This module only *synthesises* problem data.  It holds none of the
eigensolver's arithmetic (no finite-difference weights, no Hamiltonian
application, no filter, no spectral bounds): both the GPU library and the
FP64 CPU oracle consume what it produces and each derives everything else on
its own.

Workload shapes follow the paper's test systems (Section 3): bulk metals on a
cubic periodic grid at Gamma (real arithmetic), slabs periodic in x/y and
finite in z, grid spacings 0.22-0.372 bohr, and Ns of about 1.2x the number of
occupied states.  The pseudopotentials and atomic configurations of the paper
are not available, so the potential is a sum of Gaussian wells and the
Kleinman-Bylander projectors are Gaussian s/p functions (see ``make_problem``).

Layout conventions shared with the library's C-ABI:
  * grid point (x, y, z) has linear index i = x + Nx*(y + Ny*z);
  * an orbital block is an Nd x Ns column-major array, i.e. a row-major
    (Ns, Nd) array whose row j is orbital j;
  * projectors are given per atom J as a sorted list of support indices
    S_J, a column-major n_J x np_J matrix chi_J, and per-projector energies
    gamma (Ha).  Projector values are normalised so that sum_i chi(i)^2 dV = 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

PERIODIC = 0
DIRICHLET = 1


@dataclasses.dataclass
class Problem:
    """Plain arrays describing H = -1/2 Lap_FD + Veff + sum_J chi_J gamma_J chi_J^T dV."""

    n: tuple            # (Nx, Ny, Nz)
    h: tuple            # (hx, hy, hz) bohr
    bc: tuple           # per direction: 0 periodic, 1 Dirichlet
    fd_order: int       # even, 2..12
    veff: np.ndarray    # (Nd,) float64, Ha
    atoms: np.ndarray   # (n_atoms, 3) bohr
    supp_ptr: np.ndarray  # (n_atoms+1,) int64
    supp_idx: np.ndarray  # (sum n_J,) int32, sorted ascending within an atom
    nproj: np.ndarray     # (n_atoms,) int32
    chi: np.ndarray       # (sum n_J*np_J,) float64, per atom column-major n_J x np_J
    gamma: np.ndarray     # (sum np_J,) float64, Ha
    name: str = ""

    @property
    def nd(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    @property
    def dv(self) -> float:
        return float(self.h[0]) * float(self.h[1]) * float(self.h[2])

    @property
    def n_atoms(self) -> int:
        return int(len(self.nproj))


@dataclasses.dataclass
class Config:
    """One workload: grid, atoms, projector count, Ns and Chebyshev degree."""

    name: str
    n: tuple
    h: tuple
    bc: tuple
    lattice: str          # "uniform", "bcc", "slab", "fcc_subset"
    n_atoms: int
    nproj_per_atom: int   # 1 (s) or 4 (s + 3 p)
    ns: int
    degree: int
    n_iter: int
    atom_seed: int
    x_seed: int
    fd_order: int = 12
    lattice_cells: tuple = (1, 1, 1)


# The five workloads.  Seeds: atoms 1000+k, X0 2000+k for workload k.
CONFIGS: Dict[str, Config] = {
    # Plain FP64, 24^3 periodic, h = 0.3, 8 atoms with one s projector each.
    "cfg1": Config("cfg1", (24, 24, 24), (0.3, 0.3, 0.3), (0, 0, 0), "uniform", 8, 1,
                   40, 20, 10, 1001, 2001),
    # Plain FP64, 72^3 periodic, h = 0.25, 128 atoms (bcc 4^3) with s + 3 p projectors.
    "cfg2": Config("cfg2", (72, 72, 72), (0.25, 0.25, 0.25), (0, 0, 0), "bcc", 128, 4,
                   600, 20, 10, 1002, 2002, lattice_cells=(4, 4, 4)),
    # Mixed-precision slab, 60 x 60 x 180, Dirichlet in z, 200 atoms in the central third.
    "cfg3": Config("cfg3", (60, 60, 180), (0.3, 0.3, 0.3), (0, 0, 1), "slab", 200, 4,
                   1200, 24, 6, 1003, 2003, lattice_cells=(5, 5, 8)),
    # Large metallic cell, 120^3 periodic, h = 0.22, 1000 atoms from a jittered FCC 7^3 lattice.
    "cfg4": Config("cfg4", (120, 120, 120), (0.22, 0.22, 0.22), (0, 0, 0), "fcc_subset", 1000, 4,
                   7200, 16, 4, 1004, 2004, lattice_cells=(7, 7, 7)),
    # Reduced twin of cfg3 (half the grid per direction, an eighth of the atoms, Ns 300):
    # small enough for the FP64 oracle to run whole iterations on the host.
    "cfg3_twin": Config("cfg3_twin", (30, 30, 90), (0.3, 0.3, 0.3), (0, 0, 1), "slab", 25, 4,
                        300, 24, 6, 1013, 2013, lattice_cells=(3, 3, 3)),
    # Reduced twin of cfg4 (half the cell per direction at the same spacing and atom density:
    # 125 atoms from a jittered FCC 4^3 lattice, Ns 900, degree 16): whole oracle iterations
    # fit on the host.
    "cfg4_twin": Config("cfg4_twin", (60, 60, 60), (0.22, 0.22, 0.22), (0, 0, 0), "fcc_subset", 125, 4,
                        900, 16, 6, 1014, 2014, lattice_cells=(4, 4, 4)),
    # Test-sized slab (same recipe), for mixed/FP64 parity of whole iterations.
    "slab_small": Config("slab_small", (16, 16, 48), (0.3, 0.3, 0.3), (0, 0, 1), "slab", 6, 4,
                         48, 24, 6, 1023, 2023, lattice_cells=(2, 2, 2)),
}

WELL_DEPTH = 2.0     # Ha
WELL_SIGMA = 1.0     # bohr
PROJ_RC = 1.5        # bohr, support radius of each projector
PROJ_SIGMA = 0.5     # bohr (rc / 3)
PROJ_GAMMA = 0.5     # Ha, KB energy of every projector
JITTER = 0.25        # bohr, uniform jitter per coordinate


def _box(cfg_n, cfg_h):
    return tuple(float(cfg_n[d]) * float(cfg_h[d]) for d in range(3))


def atom_positions(cfg: Config) -> np.ndarray:
    """Seeded atom positions (bohr) for a workload."""
    rng = np.random.Generator(np.random.PCG64(cfg.atom_seed))
    L = _box(cfg.n, cfg.h)
    if cfg.lattice == "uniform":
        return rng.uniform(0.0, 1.0, size=(cfg.n_atoms, 3)) * np.array(L)
    if cfg.lattice == "bcc":
        c = cfg.lattice_cells
        a = np.array(L) / np.array(c)
        basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
        sites = []
        for k in range(c[2]):
            for j in range(c[1]):
                for i in range(c[0]):
                    for b in basis:
                        sites.append((np.array([i, j, k]) + b + 0.25) * a)
        sites = np.array(sites)[: cfg.n_atoms]
        return sites + rng.uniform(-JITTER, JITTER, size=sites.shape)
    if cfg.lattice == "slab":
        # atoms on a jittered lattice filling the central third of z
        c = cfg.lattice_cells
        z0, z1 = L[2] / 3.0, 2.0 * L[2] / 3.0
        sx, sy, sz = L[0] / c[0], L[1] / c[1], (z1 - z0) / c[2]
        sites = []
        for k in range(c[2]):
            for j in range(c[1]):
                for i in range(c[0]):
                    sites.append(((i + 0.5) * sx, (j + 0.5) * sy, z0 + (k + 0.5) * sz))
        sites = np.array(sites)[: cfg.n_atoms]
        return sites + rng.uniform(-JITTER, JITTER, size=sites.shape)
    if cfg.lattice == "fcc_subset":
        c = cfg.lattice_cells
        a = np.array(L) / np.array(c)
        basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
        sites = []
        for k in range(c[2]):
            for j in range(c[1]):
                for i in range(c[0]):
                    for b in basis:
                        sites.append((np.array([i, j, k]) + b + 0.25) * a)
        sites = np.array(sites)
        pick = np.sort(rng.choice(len(sites), size=cfg.n_atoms, replace=False))
        sites = sites[pick]
        return sites + rng.uniform(-JITTER, JITTER, size=sites.shape)
    raise ValueError(f"unknown lattice {cfg.lattice}")


def _axis_offsets(coord_grid: np.ndarray, pos: float, length: float, periodic: bool) -> np.ndarray:
    """Signed distance from pos to every grid coordinate along one axis (minimum image if periodic)."""
    d = coord_grid - pos
    if periodic:
        d = d - length * np.round(d / length)
    return d


def gaussian_wells(n, h, bc, atoms, depth=WELL_DEPTH, sigma=WELL_SIGMA) -> np.ndarray:
    """Veff(r) = -depth * sum_J exp(-|r - R_J|^2 / (2 sigma^2)), minimum image in periodic directions."""
    nx, ny, nz = n
    L = _box(n, h)
    v = np.zeros((nz, ny, nx))
    axes = [np.arange(n[d]) * h[d] for d in range(3)]
    for R in atoms:
        g = []
        for d in range(3):
            off = _axis_offsets(axes[d], R[d], L[d], bc[d] == PERIODIC)
            gd = np.exp(-off * off / (2.0 * sigma * sigma))
            g.append(gd)
        keep = [np.nonzero(g[d] > 1e-30)[0] for d in range(3)]
        block = np.multiply.outer(np.multiply.outer(g[2][keep[2]], g[1][keep[1]]), g[0][keep[0]])
        v[np.ix_(keep[2], keep[1], keep[0])] -= depth * block
    return v.reshape(-1)


def kb_projectors(n, h, bc, atoms, nproj_per_atom, rc=PROJ_RC, sigma=PROJ_SIGMA, gamma=PROJ_GAMMA):
    """Gaussian s (and p_x, p_y, p_z) projectors truncated at rc, normalised with sum chi^2 dV = 1."""
    nx, ny, nz = n
    L = _box(n, h)
    dv = float(h[0] * h[1] * h[2])
    axes = [np.arange(n[d]) * h[d] for d in range(3)]
    supp_ptr = [0]
    supp_idx: List[np.ndarray] = []
    chis: List[np.ndarray] = []
    for R in atoms:
        offs, idxs = [], []
        for d in range(3):
            off = _axis_offsets(axes[d], R[d], L[d], bc[d] == PERIODIC)
            sel = np.nonzero(np.abs(off) <= rc)[0]
            offs.append(off[sel])
            idxs.append(sel)
        dz, dy, dx = np.meshgrid(offs[2], offs[1], offs[0], indexing="ij")
        iz, iy, ix = np.meshgrid(idxs[2], idxs[1], idxs[0], indexing="ij")
        r2 = dx * dx + dy * dy + dz * dz
        inside = r2 <= rc * rc
        lin = (ix + nx * (iy + ny * iz))[inside].astype(np.int64)
        order = np.argsort(lin, kind="stable")
        lin = lin[order]
        dxi, dyi, dzi = dx[inside][order], dy[inside][order], dz[inside][order]
        env = np.exp(-(dxi * dxi + dyi * dyi + dzi * dzi) / (2.0 * sigma * sigma))
        cols = [env]
        if nproj_per_atom == 4:
            cols += [dxi / sigma * env, dyi / sigma * env, dzi / sigma * env]
        elif nproj_per_atom != 1:
            raise ValueError("nproj_per_atom must be 1 or 4")
        c = np.stack(cols, axis=1)
        c = c / np.sqrt((c * c).sum(axis=0) * dv)[None, :]
        supp_idx.append(lin.astype(np.int32))
        chis.append(c.T.reshape(-1))  # column-major n_J x np_J
        supp_ptr.append(supp_ptr[-1] + len(lin))
    n_atoms = len(atoms)
    return (np.array(supp_ptr, dtype=np.int64),
            np.concatenate(supp_idx) if supp_idx else np.zeros(0, np.int32),
            np.full(n_atoms, nproj_per_atom, dtype=np.int32),
            np.concatenate(chis) if chis else np.zeros(0),
            np.full(n_atoms * nproj_per_atom, gamma, dtype=np.float64))


def support_images(prob: Problem) -> np.ndarray:
    """(sum n_J, 3) int32: for every support point of atom J, the lattice image m (per
    periodic direction; 0 in Dirichlet ones) with point = R_J + m L + offset, offset the
    minimum-image displacement used to build chi_J."""
    nx, ny, nz = prob.n
    L = _box(prob.n, prob.h)
    out = np.zeros((len(prob.supp_idx), 3), dtype=np.int32)
    for J in range(prob.n_atoms):
        lo, hi = int(prob.supp_ptr[J]), int(prob.supp_ptr[J + 1])
        lin = np.asarray(prob.supp_idx[lo:hi], dtype=np.int64)
        coords = (lin % nx, (lin // nx) % ny, lin // (nx * ny))
        for d in range(3):
            if prob.bc[d] == PERIODIC:
                out[lo:hi, d] = np.round((coords[d] * prob.h[d] - prob.atoms[J][d]) / L[d]).astype(np.int32)
    return out


def support_displacements(prob: Problem) -> np.ndarray:
    """(sum n_J, 3) float64: for every support point of atom J, its displacement from the
    atom, r_i - R_J - m L (bohr), the minimum-image offset chi_J was evaluated at (m from
    ``support_images``; plain r_i - R_J in Dirichlet directions)."""
    nx, ny = prob.n[0], prob.n[1]
    L = _box(prob.n, prob.h)
    img = support_images(prob)
    out = np.zeros((len(prob.supp_idx), 3), dtype=np.float64)
    for J in range(prob.n_atoms):
        lo, hi = int(prob.supp_ptr[J]), int(prob.supp_ptr[J + 1])
        lin = np.asarray(prob.supp_idx[lo:hi], dtype=np.int64)
        coords = (lin % nx, (lin // nx) % ny, lin // (nx * ny))
        for d in range(3):
            out[lo:hi, d] = coords[d] * prob.h[d] - prob.atoms[J][d] - img[lo:hi, d] * L[d]
    return out


def make_problem(cfg: Config) -> Problem:
    atoms = atom_positions(cfg)
    veff = gaussian_wells(cfg.n, cfg.h, cfg.bc, atoms)
    sp, si, npj, chi, gam = kb_projectors(cfg.n, cfg.h, cfg.bc, atoms, cfg.nproj_per_atom)
    return Problem(tuple(cfg.n), tuple(cfg.h), tuple(cfg.bc), cfg.fd_order, veff, atoms,
                   sp, si, npj, chi, gam, name=cfg.name)


def initial_block(nd: int, ns: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) starting block, shape (Ns, Nd): row j is orbital j."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((ns, nd))


def small_problem(n=(12, 10, 14), h=(0.35, 0.3, 0.4), bc=(0, 0, 0), fd_order=12, n_atoms=3,
                  nproj_per_atom=4, seed=7, with_veff=True, gamma=PROJ_GAMMA) -> Problem:
    """A small seeded problem with ragged grid sizes, for parity and edge-case tests."""
    L = _box(n, h)
    rng = np.random.Generator(np.random.PCG64(seed))
    atoms = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * np.array(L)
    for d in range(3):
        if bc[d] == DIRICHLET:  # keep atoms away from the finite boundary
            atoms[:, d] = L[d] * (0.3 + 0.4 * rng.uniform(size=n_atoms))
    veff = gaussian_wells(n, h, bc, atoms) if with_veff else np.zeros(int(np.prod(n)))
    if n_atoms > 0 and nproj_per_atom > 0:
        sp, si, npj, chi, gam = kb_projectors(n, h, bc, atoms, nproj_per_atom, gamma=gamma)
    else:
        sp, si, npj, chi, gam = (np.zeros(1, np.int64), np.zeros(0, np.int32),
                                 np.zeros(0, np.int32), np.zeros(0), np.zeros(0))
        atoms = np.zeros((0, 3))
    return Problem(tuple(n), tuple(h), tuple(bc), fd_order, veff, atoms, sp, si, npj, chi, gam,
                   name="small")


def serving_request(k: int, stream_seed: int = 5000):
    """Request k of the serving stream: cubic N ~ U{24..64}, h = 0.3, atoms ~ U{8..96} x 4
    projectors, Ns ~ U{40..400} capped at Nd/8, periodic or slab (Dirichlet z) 50/50, degree 20."""
    rng = np.random.Generator(np.random.PCG64([stream_seed, k]))
    N = int(rng.integers(24, 65))
    n_atoms = int(rng.integers(8, 97))
    ns = int(rng.integers(40, 401))
    ns = min(ns, (N ** 3) // 8)
    slab = bool(rng.integers(0, 2))
    bc = (0, 0, 1) if slab else (0, 0, 0)
    h = (0.3, 0.3, 0.3)
    L = N * 0.3
    pos = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * L
    if slab:
        pos[:, 2] = L / 3.0 + rng.uniform(0.0, 1.0, size=n_atoms) * (L / 3.0)
    veff = gaussian_wells((N, N, N), h, bc, pos)
    sp, si, npj, chi, gam = kb_projectors((N, N, N), h, bc, pos, 4)
    prob = Problem((N, N, N), h, bc, 12, veff, pos, sp, si, npj, chi, gam, name=f"req{k}")
    return prob, ns, 20, 2000 + 100000 + k
