"""Seeded synthetic inputs for the Z4c hot path (shared by the oracle tests,
the GPU tests and the benchmark).

This module holds no part of the method's arithmetic: it lays out MeshBlocks,
evaluates closed-form initial data (gauge wave, conformally flat star-like
metric, Gaussian matter blobs) converted from ADM to Z4c variables, and adds
seeded uniform noise.  Nothing here computes a right-hand side, a derivative
stencil, a dissipation operator or a Runge-Kutta combination.

Field order (structure of arrays, one contiguous array per field):
  state  : chi, gt_xx, gt_xy, gt_xz, gt_yy, gt_yz, gt_zz, Khat,
           At_xx, At_xy, At_xz, At_yy, At_yz, At_zz, Theta,
           Gt^x, Gt^y, Gt^z, alpha, beta^x, beta^y, beta^z          (22)
  matter : rho, S_x, S_y, S_z, S_xx, S_xy, S_xz, S_yy, S_yz, S_zz  (10)
  constraints (output): H, M_x, M_y, M_z, Theta, Z^x, Z^y, Z^z     (8)

Storage of one block: (nz+2ng, ny+2ng, nx+2ng) points, x fastest; point
(i, j, k) with i in [-ng, nx+ng) sits at x = x0 + i*dx.  Blocks are stored
one after another ("block-major"): block b, field f starts at element
offset_b + f*field_stride_b.

Units G = c = 1 (the paper's geometric units for the spacetime solver).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

NF = 22
NM = 10
NC = 8

FIELDS = ["chi", "gxx", "gxy", "gxz", "gyy", "gyz", "gzz", "Khat",
          "Axx", "Axy", "Axz", "Ayy", "Ayz", "Azz", "Theta",
          "Gx", "Gy", "Gz", "alpha", "bx", "by", "bz"]
MATTER = ["rho", "Sx", "Sy", "Sz", "Sxx", "Sxy", "Sxz", "Syy", "Syz", "Szz"]
CONSTRAINTS = ["H", "Mx", "My", "Mz", "Theta", "Zx", "Zy", "Zz"]
F = {n: i for i, n in enumerate(FIELDS)}
SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]

SEED_BASE = 231104989

# Gauge / parameter enums (mirrors the C-ABI values; plain integers)
LAPSE_1PLUSLOG, LAPSE_HARMONIC, LAPSE_FROZEN = 0, 1, 2
SHIFT_GAMMADRIVER, SHIFT_FROZEN = 0, 1
GHOST_NONE, GHOST_PERIODIC, GHOST_NEIGHBOUR, GHOST_FROZEN = 0, 1, 2, 3


@dataclasses.dataclass
class Block:
    nx: int
    ny: int
    nz: int
    ng: int
    dx: float
    dy: float
    dz: float
    x0: float = 0.0
    y0: float = 0.0
    z0: float = 0.0

    @property
    def shape(self):
        return (self.nz + 2 * self.ng, self.ny + 2 * self.ng, self.nx + 2 * self.ng)

    @property
    def npts(self) -> int:
        s = self.shape
        return s[0] * s[1] * s[2]

    @property
    def ninterior(self) -> int:
        return self.nx * self.ny * self.nz

    def coords(self):
        """Coordinates of every stored point, each of shape `self.shape`."""
        ng = self.ng
        x = self.x0 + (np.arange(self.nx + 2 * ng) - ng) * self.dx
        y = self.y0 + (np.arange(self.ny + 2 * ng) - ng) * self.dy
        z = self.z0 + (np.arange(self.nz + 2 * ng) - ng) * self.dz
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return X, Y, Z


@dataclasses.dataclass
class Params:
    """Scheme parameters (paper: 6th-order FD, kappa1 = 0.02, kappa2 = 0,
    sigma_KO = 0.5; gauge choices as in the moving-puncture family)."""
    fd_order: int = 6
    ko_sigma: float = 0.5
    kappa1: float = 0.02
    kappa2: float = 0.0
    eta: float = 2.0
    lapse: int = LAPSE_1PLUSLOG
    shift: int = SHIFT_GAMMADRIVER
    advect_gauge: int = 1
    chi_floor: float = 1e-6
    alpha_floor: float = 1e-8
    advection: int = 0        # 0 centred, 1 lopsided (shifted towards the sign of beta^k)


def _pad_even(n: int) -> int:
    return n + (n & 1)


class Batch:
    """A set of MeshBlocks with their state (and optional matter) arrays."""

    def __init__(self, blocks: List[Block], with_matter: bool = False):
        self.blocks = list(blocks)
        nb = len(self.blocks)
        self.field_stride = np.array([_pad_even(b.npts) for b in self.blocks], dtype=np.int64)
        starts = np.zeros(nb + 1, dtype=np.int64)
        np.cumsum(self.field_stride, out=starts[1:])
        self.starts = starts              # per-block start in units of "one field"
        self.offsets = NF * starts[:-1]
        self.moffsets = NM * starts[:-1]
        self.coffsets = NC * starts[:-1]
        self.total_u = int(NF * starts[-1])
        self.total_m = int(NM * starts[-1])
        self.total_c = int(NC * starts[-1])
        self.u = np.zeros(self.total_u, dtype=np.float64)
        self.matter = np.zeros(self.total_m, dtype=np.float64) if with_matter else None
        self.params = Params()
        self.ghost = GHOST_NONE
        self.neighbours: Optional[np.ndarray] = None   # (nb, 27) int32, -1 = outer
        self.frozen: Optional[np.ndarray] = None       # copy of u used for frozen ghosts
        # outer ghost points (neighbour entry -1) advanced by the radiative
        # (Sommerfeld) law in every stage instead of being frozen
        self.sommerfeld = False
        self.dt = 0.25 * min(min(b.dx, b.dy, b.dz) for b in self.blocks)
        self.name = ""

    # --- views -------------------------------------------------------------
    def view(self, arr: np.ndarray, b: int, f: int, nfields: int = NF) -> np.ndarray:
        blk = self.blocks[b]
        if nfields == NF:
            off = self.offsets[b]
        elif nfields == NM:
            off = self.moffsets[b]
        else:
            off = self.coffsets[b]
        s = off + f * self.field_stride[b]
        return arr[s:s + blk.npts].reshape(blk.shape)

    def interior(self, arr: np.ndarray, b: int, f: int, nfields: int = NF) -> np.ndarray:
        blk = self.blocks[b]
        g = blk.ng
        v = self.view(arr, b, f, nfields)
        return v[g:g + blk.nz, g:g + blk.ny, g:g + blk.nx]

    @property
    def ninterior(self) -> int:
        return sum(b.ninterior for b in self.blocks)

    @property
    def nstored(self) -> int:
        return sum(b.npts for b in self.blocks)

    def origins(self) -> np.ndarray:
        """Coordinates of interior point (0, 0, 0) of every block, (nb, 3)."""
        return np.array([(b.x0, b.y0, b.z0) for b in self.blocks], dtype=np.float64)

    def block_table(self) -> np.ndarray:
        """Structured array matching the C `z4c_block` descriptor."""
        tab = np.zeros(len(self.blocks), dtype=BLOCK_DTYPE)
        for i, b in enumerate(self.blocks):
            tab[i] = (self.offsets[i], self.moffsets[i], self.coffsets[i],
                      self.field_stride[i], b.nx, b.ny, b.nz, b.ng, b.dx, b.dy, b.dz)
        return tab

    def subset(self, idx) -> "Batch":
        """A new batch holding copies of the selected blocks (for sampled checks)."""
        idx = [int(i) for i in idx]
        sub = Batch([self.blocks[i] for i in idx], with_matter=self.matter is not None)
        sub.params = dataclasses.replace(self.params)
        sub.ghost = self.ghost
        sub.dt = self.dt
        for j, i in enumerate(idx):
            for f in range(NF):
                sub.view(sub.u, j, f)[...] = self.view(self.u, i, f)
            if self.matter is not None:
                for f in range(NM):
                    sub.view(sub.matter, j, f, NM)[...] = self.view(self.matter, i, f, NM)
        if self.frozen is not None:
            sub.frozen = np.zeros_like(sub.u)
            for j, i in enumerate(idx):
                for f in range(NF):
                    sub.view(sub.frozen, j, f)[...] = self.view(self.frozen, i, f)
        return sub


BLOCK_DTYPE = np.dtype([("offset", np.int64), ("moffset", np.int64), ("coffset", np.int64),
                        ("field_stride", np.int64), ("nx", np.int32), ("ny", np.int32),
                        ("nz", np.int32), ("ng", np.int32), ("dx", np.float64),
                        ("dy", np.float64), ("dz", np.float64)])


# --- closed-form initial data (ADM -> Z4c) ------------------------------------

def gauge_wave(X, Y, Z, amp=0.01, wavelength=1.0, t=0.0):
    """1-D gauge wave along x: ds^2 = -H dt^2 + H dx^2 + dy^2 + dz^2 with
    H = 1 - A sin(2 pi (x - t)/d).  Returns the 22 Z4c fields.

    ADM: gamma_xx = H, alpha = sqrt(H), K_xx = -d_t H / (2 alpha), beta = 0.
    Z4c: chi = det(gamma)^(-1/3), gt = chi gamma, Khat = K, Theta = 0,
    At = chi (K_ij - gamma_ij K / 3), Gt^i = -d_j gt^{ij} (det gt = 1).
    """
    k = 2.0 * math.pi / wavelength
    ph = k * (X - t)
    H = 1.0 - amp * np.sin(ph)
    dHdx = -amp * k * np.cos(ph)
    dHdt = amp * k * np.cos(ph)
    sq = np.sqrt(H)
    Kxx = -dHdt / (2.0 * sq)
    K = Kxx / H
    chi = H ** (-1.0 / 3.0)
    out = {n: np.zeros_like(X) for n in FIELDS}
    out["chi"] = chi
    out["gxx"] = H ** (2.0 / 3.0)
    out["gyy"] = chi.copy()
    out["gzz"] = chi.copy()
    out["Khat"] = K
    out["Axx"] = chi * (Kxx - H * K / 3.0)
    out["Ayy"] = chi * (-K / 3.0)
    out["Azz"] = chi * (-K / 3.0)
    # gt^{xx} = H^(-2/3): Gt^x = -d_x H^(-2/3) = (2/3) H^(-5/3) H'
    out["Gx"] = (2.0 / 3.0) * H ** (-5.0 / 3.0) * dHdx
    out["alpha"] = sq
    return out


def star_metric(X, Y, Z, M=1.4, s=2.0):
    """Conformally flat star-like metric: psi = 1 + M / (2 sqrt(r^2 + s^2)),
    gamma_ij = psi^4 delta_ij, alpha = psi^-2, zero shift and curvature."""
    r2 = X * X + Y * Y + Z * Z
    psi = 1.0 + M / (2.0 * np.sqrt(r2 + s * s))
    out = {n: np.zeros_like(X) for n in FIELDS}
    out["chi"] = psi ** -4.0
    out["gxx"] = np.ones_like(X)
    out["gyy"] = np.ones_like(X)
    out["gzz"] = np.ones_like(X)
    out["alpha"] = psi ** -2.0
    return out


def flat(X, Y=None, Z=None):
    out = {n: np.zeros_like(X) for n in FIELDS}
    for n in ("chi", "gxx", "gyy", "gzz", "alpha"):
        out[n] = np.ones_like(X)
    return out


def matter_blobs(rng, nblobs=NM, amp=1e-3, width=2.0, box=4.0):
    """Seeded Gaussian blob parameters, one blob per matter field.
    rho and the diagonal S_ii are positive with peak `amp`; S_i and the
    off-diagonal S_ij get a seeded amplitude in [-amp, amp]."""
    centres = rng.uniform(-box, box, size=(nblobs, 3))
    amps = np.full(nblobs, amp)
    for f, n in enumerate(MATTER):
        if n in ("Sx", "Sy", "Sz", "Sxy", "Sxz", "Syz"):
            amps[f] = amp * rng.uniform(-1.0, 1.0)
    return centres, amps, width


def eval_blobs(X, Y, Z, blobs):
    centres, amps, w = blobs
    out = []
    for f in range(NM):
        c = centres[f]
        d2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
        out.append(amps[f] * np.exp(-d2 / (2.0 * w * w)))
    return out


def fill_fields(batch: Batch, fn, **kw):
    for b, blk in enumerate(batch.blocks):
        X, Y, Z = blk.coords()
        vals = fn(X, Y, Z, **kw)
        for f, n in enumerate(FIELDS):
            batch.view(batch.u, b, f)[...] = vals[n]


def fill_matter(batch: Batch, blobs):
    for b, blk in enumerate(batch.blocks):
        X, Y, Z = blk.coords()
        vals = eval_blobs(X, Y, Z, blobs)
        for f in range(NM):
            batch.view(batch.matter, b, f, NM)[...] = vals[f]


def add_noise(batch: Batch, rng, a: float):
    """Uniform U(-a, a) noise, drawn block by block, field by field in field
    order, over the whole stored array (ghosts included)."""
    for b, blk in enumerate(batch.blocks):
        for f in range(NF):
            v = batch.view(batch.u, b, f)
            v += rng.uniform(-a, a, size=v.shape)


def self_neighbours(nb: int) -> np.ndarray:
    """Neighbour table in which every block is its own neighbour in all 26
    directions (periodic wrap of each block on itself)."""
    t = np.empty((nb, 27), dtype=np.int32)
    t[:] = np.arange(nb, dtype=np.int32)[:, None]
    return t


def dir_index(ox: int, oy: int, oz: int) -> int:
    """Index of direction (ox, oy, oz) in {-1,0,1}^3 within a 27-entry row."""
    return (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)


# --- the five workload configurations ------------------------------------------

def config1(seed_offset: int = 1) -> Batch:
    """One 16^3 block + 3 ghosts, periodic unit box, 4th-order FD, KO 0.02,
    x-aligned gauge wave (A = 0.01, wavelength 1) + U(-1e-10, 1e-10) noise,
    1+log lapse, Gamma-driver eta = 2, no matter; one RK4 step, dt = 1/64."""
    n = 16
    blk = Block(n, n, n, 3, 1.0 / n, 1.0 / n, 1.0 / n, 0.0, 0.0, 0.0)
    bt = Batch([blk])
    fill_fields(bt, gauge_wave, amp=0.01, wavelength=1.0)
    add_noise(bt, np.random.default_rng(SEED_BASE + seed_offset), 1e-10)
    bt.params = Params(fd_order=4, ko_sigma=0.02)
    bt.ghost = GHOST_PERIODIC
    bt.neighbours = self_neighbours(1)
    bt.dt = 1.0 / 64.0
    bt.name = "gauge-wave 16^3+3g p4"
    return bt


def config2(seed_offset: int = 2, n: int = 64) -> Batch:
    """One 64^3 block + 4 ghosts on [-16, 16]^3 (dx = 0.5, points offset by
    dx/2), 6th-order FD, KO 0.5; star-like conformally flat metric
    (M = 1.4, s = 2) with Gaussian matter blobs of peak 1e-3; frozen ghosts."""
    dx = 32.0 / n
    blk = Block(n, n, n, 4, dx, dx, dx, -16.0 + 0.5 * dx, -16.0 + 0.5 * dx, -16.0 + 0.5 * dx)
    bt = Batch([blk], with_matter=True)
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    fill_fields(bt, star_metric)
    fill_matter(bt, matter_blobs(rng))
    bt.params = Params(fd_order=6, ko_sigma=0.5)
    bt.ghost = GHOST_FROZEN
    bt.frozen = bt.u.copy()
    bt.dt = 0.25 * dx
    bt.name = f"star {n}^3+4g p6 matter"
    return bt


def config3(seed_offset: int = 3, nblocks: int = 512, n: int = 16) -> Batch:
    """512 blocks of 16^3 + 4 ghosts, 6th order, dx_b = 0.5 / 2^L_b with
    L_b ~ U{0..6}, origins U[0,1)^3; the gauge wave + 1e-10 noise sampled at
    each block's points.  Workload: one fused RHS+RK stage."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    levels = rng.integers(0, 7, size=nblocks)
    origins = rng.uniform(0.0, 1.0, size=(nblocks, 3))
    blocks = []
    for b in range(nblocks):
        d = 0.5 / 2.0 ** int(levels[b])
        blocks.append(Block(n, n, n, 4, d, d, d, *origins[b]))
    bt = Batch(blocks)
    fill_fields(bt, gauge_wave, amp=0.01, wavelength=1.0)
    add_noise(bt, rng, 1e-10)
    bt.params = Params(fd_order=6, ko_sigma=0.5)
    bt.ghost = GHOST_NONE
    bt.name = f"level set {nblocks}x{n}^3+4g p6"
    return bt


def config4_counts(nblocks: int = 1024):
    """Largest-remainder split of `nblocks` in ratio 4:3:2:1."""
    w = np.array([4, 3, 2, 1], dtype=np.float64)
    exact = nblocks * w / w.sum()
    c = np.floor(exact).astype(int)
    rem = nblocks - c.sum()
    order = np.argsort(-(exact - c), kind="stable")
    c[order[:rem]] += 1
    return c


def config4(seed_offset: int = 4, nblocks: int = 1024, sizes=(8, 16, 24, 32)) -> Batch:
    """1,024 blocks of sizes 8/16/24/32 cubed (counts 410/307/205/102) + 4
    ghosts, shuffled, dx_b = 0.5 / 2^L_b, flat space + U(-1e-8, 1e-8) noise,
    6th order, each block periodic on itself; 4 RK4 stages per step."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    counts = config4_counts(nblocks)
    ns = np.concatenate([np.full(c, s) for c, s in zip(counts, sizes)])
    rng.shuffle(ns)
    levels = rng.integers(0, 7, size=nblocks)
    origins = rng.uniform(0.0, 1.0, size=(nblocks, 3))
    blocks = []
    for b in range(nblocks):
        d = 0.5 / 2.0 ** int(levels[b])
        blocks.append(Block(int(ns[b]), int(ns[b]), int(ns[b]), 4, d, d, d, *origins[b]))
    bt = Batch(blocks)
    for b, blk in enumerate(bt.blocks):
        for n in ("chi", "gxx", "gyy", "gzz", "alpha"):
            bt.view(bt.u, b, F[n])[...] = 1.0
    add_noise(bt, rng, 1e-8)
    bt.params = Params(fd_order=6, ko_sigma=0.5)
    bt.ghost = GHOST_PERIODIC
    bt.neighbours = self_neighbours(nblocks)
    bt.name = f"uneven level set {nblocks} blocks {'/'.join(str(s) for s in sizes)}^3+4g p6"
    return bt


def config5(seed_offset: int = 5, n: int = 128, noise: float = 1e-6) -> Batch:
    """8 blocks of 128^3 + 4 ghosts tiling [-16, 16]^3 (dx = 0.125), star
    metric + matter blobs (as config 2) + U(-1e-6, 1e-6) noise; same-level
    neighbour ghost copies, frozen outer ghosts; 6th order, KO 0.5."""
    dx = 16.0 / n
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    blocks = []
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                blocks.append(Block(n, n, n, 4, dx, dx, dx,
                                    -16.0 + 16.0 * bx + 0.5 * dx,
                                    -16.0 + 16.0 * by + 0.5 * dx,
                                    -16.0 + 16.0 * bz + 0.5 * dx))
    bt = Batch(blocks, with_matter=True)
    fill_fields(bt, star_metric)
    fill_matter(bt, matter_blobs(rng))
    add_noise(bt, rng, noise)
    nbr = np.full((8, 27), -1, dtype=np.int32)
    for b in range(8):
        bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
        for oz in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for ox in (-1, 0, 1):
                    cx, cy, cz = bx + ox, by + oy, bz + oz
                    if 0 <= cx < 2 and 0 <= cy < 2 and 0 <= cz < 2:
                        nbr[b, dir_index(ox, oy, oz)] = cx + 2 * cy + 4 * cz
    bt.params = Params(fd_order=6, ko_sigma=0.5)
    bt.ghost = GHOST_NEIGHBOUR
    bt.neighbours = nbr
    bt.frozen = bt.u.copy()
    bt.dt = 0.25 * dx
    bt.name = f"precision study 8x{n}^3+4g p6 matter"
    return bt


def random_batch(seed: int, nblocks: int = 3, nmax: int = 40, ng=None, fd_order=None,
                 amp: float = 1e-3, with_matter: bool = True) -> Batch:
    """Random small shapes (sizes in [1, nmax], ng in {3, 4} compatible with the
    order, random spacings) holding a smooth perturbation of flat space plus
    noise; used for shape-robustness parity checks."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    p = fd_order if fd_order is not None else int(rng.choice([4, 6]))
    blocks = []
    for _ in range(nblocks):
        nx, ny, nz = (int(v) for v in rng.integers(1, nmax + 1, size=3))
        g = ng if ng is not None else (4 if p == 6 else int(rng.choice([3, 4])))
        dx, dy, dz = (float(v) for v in rng.uniform(0.05, 0.5, size=3))
        blocks.append(Block(nx, ny, nz, g, dx, dy, dz, *rng.uniform(-1, 1, size=3)))
    bt = Batch(blocks, with_matter=with_matter)
    for b, blk in enumerate(bt.blocks):
        X, Y, Z = blk.coords()
        for f in range(NF):
            kx, ky, kz = rng.uniform(0.5, 2.0, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            base = 1.0 if FIELDS[f] in ("chi", "gxx", "gyy", "gzz", "alpha") else 0.0
            bt.view(bt.u, b, f)[...] = base + amp * np.sin(kx * X + ky * Y + kz * Z + ph)
        if with_matter:
            for f in range(NM):
                v = bt.view(bt.matter, b, f, NM)
                v[...] = amp * (1.0 + np.cos(X + 2 * Y - Z + f))
    add_noise(bt, rng, amp * 1e-3)
    bt.params = Params(fd_order=p, ko_sigma=float(rng.uniform(0.0, 0.5)),
                       kappa1=0.02, kappa2=float(rng.uniform(0.0, 0.5)))
    bt.ghost = GHOST_NONE
    bt.name = f"random shapes seed {seed}"
    return bt


def level_neighbours(bt: Batch, locs) -> np.ndarray:
    """Same-level neighbour table of a level set (nblocks x 27, -1 where the
    adjacent position holds no block of the same level): the block of level
    L whose vertex 0 sits n steps further in that direction."""
    lmax = max(L for L, _ in locs)
    where = {(L, tuple(o)): b for b, (L, o) in enumerate(locs)}
    nbr = np.full((len(bt.blocks), 27), -1, dtype=np.int32)
    for b, (blk, (L, o)) in enumerate(zip(bt.blocks, locs)):
        s = 1 << (lmax - L)
        for oz in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for ox in (-1, 0, 1):
                    key = (L, (o[0] + ox * blk.nx * s, o[1] + oy * blk.ny * s,
                               o[2] + oz * blk.nz * s))
                    nbr[b, dir_index(ox, oy, oz)] = where.get(key, -1)
    return nbr


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}



# --- matter coupling: vertex-centred Z4c grid, cell-centred fluid grid ------

NGEOM = 7    # CC geometry: chi, gt_xx, gt_xy, gt_xz, gt_yy, gt_yz, gt_zz
NPRIM = 8    # CC primitives: rho, ut^x, ut^y, ut^z, p, B^x, B^y, B^z
PRIMS = ["rho", "utx", "uty", "utz", "p", "Bx", "By", "Bz"]

MBLOCK_DTYPE = np.dtype([("vs_offset", np.int64), ("vm_offset", np.int64),
                         ("vc_stride", np.int64), ("cg_offset", np.int64),
                         ("cp_offset", np.int64), ("ca_offset", np.int64),
                         ("cq_offset", np.int64), ("cf_offset", np.int64),
                         ("cc_stride", np.int64), ("ncx", np.int32), ("ncy", np.int32),
                         ("ncz", np.int32), ("ngv", np.int32), ("ngc", np.int32),
                         ("pad", np.int32)])


@dataclasses.dataclass
class MBlock:
    """One MeshBlock of nc cells (nc + 1 vertices) per direction; vertex i at
    x0 + i*dx, the centre of cell i at x0 + (i + 1/2)*dx."""
    ncx: int
    ncy: int
    ncz: int
    ngv: int
    ngc: int
    dx: float
    x0: tuple = (0.0, 0.0, 0.0)

    @property
    def vshape(self):
        g = 2 * self.ngv
        return (self.ncz + 1 + g, self.ncy + 1 + g, self.ncx + 1 + g)

    @property
    def cshape(self):
        g = 2 * self.ngc
        return (self.ncz + g, self.ncy + g, self.ncx + g)

    def vcoords(self):
        """Coordinates of every stored vertex (ghosts included), (z, y, x) order."""
        r = [self.x0[d] + (np.arange(n) - self.ngv) * self.dx
             for d, n in enumerate(self.vshape[::-1])]
        Z, Y, X = np.meshgrid(r[2], r[1], r[0], indexing="ij")
        return X, Y, Z

    def ccoords(self):
        r = [self.x0[d] + (np.arange(n) - self.ngc + 0.5) * self.dx
             for d, n in enumerate(self.cshape[::-1])]
        Z, Y, X = np.meshgrid(r[2], r[1], r[0], indexing="ij")
        return X, Y, Z


class MatterBatch:
    """Blocks with their arrays: VC state (22 fields), VC matter (10), CC
    geometry (7), CC primitives (8), CC ADM sources (10), CC conservatives
    (8), CC status (one int32 per cell); block-major, fields strided by the
    per-block vertex / cell counts (padded to even)."""

    def __init__(self, blocks: List[MBlock]):
        self.blocks = list(blocks)
        vs = np.array([_pad_even(int(np.prod(b.vshape))) for b in self.blocks], dtype=np.int64)
        cs = np.array([_pad_even(int(np.prod(b.cshape))) for b in self.blocks], dtype=np.int64)
        vstart = np.concatenate([[0], np.cumsum(vs)])
        cstart = np.concatenate([[0], np.cumsum(cs)])
        self.vc_stride, self.cc_stride = vs, cs
        self.vs_offset, self.vm_offset = NF * vstart[:-1], NM * vstart[:-1]
        self.cg_offset, self.cp_offset = NGEOM * cstart[:-1], NPRIM * cstart[:-1]
        self.ca_offset = NM * cstart[:-1]
        self.cq_offset = NPRIM * cstart[:-1]
        self.cf_offset = cstart[:-1].copy()
        nv, nc = int(vstart[-1]), int(cstart[-1])
        self.cons = np.zeros(NPRIM * nc)
        self.status = np.zeros(nc, dtype=np.int32)
        self.u = np.zeros(NF * nv)
        self.matter = np.zeros(NM * nv)
        self.geom = np.zeros(NGEOM * nc)
        self.prim = np.zeros(NPRIM * nc)
        self.adm = np.zeros(NM * nc)
        self.name = ""

    _KIND = {"u": ("vs_offset", "vc_stride", "vshape"), "matter": ("vm_offset", "vc_stride", "vshape"),
             "geom": ("cg_offset", "cc_stride", "cshape"), "prim": ("cp_offset", "cc_stride", "cshape"),
             "adm": ("ca_offset", "cc_stride", "cshape"), "cons": ("cq_offset", "cc_stride", "cshape"),
             "status": ("cf_offset", "cc_stride", "cshape")}

    def view(self, kind: str, arr: np.ndarray, b: int, f: int) -> np.ndarray:
        """Stored (ghosts included) field f of block b of an array of `kind`
        ("u", "matter", "geom", "prim" or "adm"), indexed [k, j, i]."""
        off, st, shp = self._KIND[kind]
        blk = self.blocks[b]
        shape = getattr(blk, shp)
        s = int(getattr(self, off)[b] + f * getattr(self, st)[b])
        return arr[s:s + int(np.prod(shape))].reshape(shape)

    def table(self) -> np.ndarray:
        t = np.zeros(len(self.blocks), dtype=MBLOCK_DTYPE)
        for i, b in enumerate(self.blocks):
            t[i] = (self.vs_offset[i], self.vm_offset[i], self.vc_stride[i], self.cg_offset[i],
                    self.cp_offset[i], self.ca_offset[i], self.cq_offset[i], self.cf_offset[i],
                    self.cc_stride[i], b.ncx, b.ncy, b.ncz, b.ngv, b.ngc, 0)
        return t

    @property
    def ncells(self) -> int:
        return sum(b.ncx * b.ncy * b.ncz for b in self.blocks)

    @property
    def nvertices(self) -> int:
        return sum((b.ncx + 1) * (b.ncy + 1) * (b.ncz + 1) for b in self.blocks)


def fill_fluid(mb: MatterBatch, rng, K=100.0, gamma_ad=2.0, rho_peak=1e-3, omega=0.02,
               B0=1e-3, noise=1e-6):
    """Conformally flat star-like metric (config-2 parameters) with a smooth
    anisotropic perturbation of gt_ij at the vertices (ghosts included);
    at the cells: Gaussian density blobs of peak `rho_peak`, polytropic
    pressure p = K rho^Gamma (the TOV polytrope K = 100, Gamma = 2), a rigid
    rotation ut = omega (-y, x, 0) plus a seeded vertical velocity, and a
    smooth tilted magnetic field of strength ~B0 scaled by the density;
    U(-noise, noise) on every field."""
    centres = rng.uniform(-4.0, 4.0, size=(4, 3))
    tilt = rng.normal(size=3)
    tilt /= np.linalg.norm(tilt)
    vz = rng.uniform(-0.05, 0.05)
    for b, blk in enumerate(mb.blocks):
        X, Y, Z = blk.vcoords()
        st = star_metric(X, Y, Z)
        for f in range(NF):
            mb.view("u", mb.u, b, f)[...] = st[FIELDS[f]]
        h = 0.02 * np.sin(0.3 * X + 0.2 * Y) * np.cos(0.25 * Z)
        for q, (i, j) in enumerate(SYM):
            v = mb.view("u", mb.u, b, 1 + q)
            v += h * (1.0 if i == j else 0.5) * (1 + q) / 6.0
        for f in range(NF):
            v = mb.view("u", mb.u, b, f)
            v += rng.uniform(-noise, noise, size=v.shape)
        X, Y, Z = blk.ccoords()
        rho = np.zeros_like(X)
        for c in centres:
            rho += rho_peak * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / 8.0)
        shape = 1.0 + rho / rho_peak
        vals = [rho, -omega * Y, omega * X, vz * np.ones_like(X), K * rho ** gamma_ad,
                B0 * tilt[0] * shape, B0 * tilt[1] * shape, B0 * tilt[2] * shape + 0.2 * B0 * np.sin(0.3 * X)]
        for f in range(NPRIM):
            v = mb.view("prim", mb.prim, b, f)
            v[...] = vals[f] + rng.uniform(-noise, noise, size=v.shape) * (rho_peak if f in (0, 4) else 1.0)
        np.maximum(mb.view("prim", mb.prim, b, 0), 0.0, out=mb.view("prim", mb.prim, b, 0))
        np.maximum(mb.view("prim", mb.prim, b, 4), 0.0, out=mb.view("prim", mb.prim, b, 4))


def matter_level_set(seed_offset: int = 6, nc: int = 128, ngv: int = 4, ngc: int = 3) -> MatterBatch:
    """Matter coupling on the precision-study level set: 2x2x2 blocks of nc^3
    cells ((nc+1)^3 vertices) tiling [-16, 16]^3, 4 ghost vertices, 3 ghost
    cells."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    dx = 16.0 / nc
    blocks = [MBlock(nc, nc, nc, ngv, ngc, dx, (-16.0 + 16.0 * bx, -16.0 + 16.0 * by, -16.0 + 16.0 * bz))
              for bz in range(2) for by in range(2) for bx in range(2)]
    mb = MatterBatch(blocks)
    fill_fluid(mb, rng)
    mb.name = f"matter coupling 8x{nc}^3 cells, {ngv} ghost vertices, {ngc} ghost cells"
    return mb


def random_matter_batch(seed: int, nblocks: int = 3, nmax: int = 24, ngv: int = 4,
                        ngc: int = 3) -> MatterBatch:
    """Small blocks of seeded uneven cell counts (1 .. nmax per direction)."""
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    blocks = []
    for _ in range(nblocks):
        n = rng.integers(1, nmax + 1, size=3)
        blocks.append(MBlock(int(n[0]), int(n[1]), int(n[2]), ngv, ngc,
                             float(rng.uniform(0.2, 1.0)), tuple(rng.uniform(-6.0, 2.0, size=3))))
    mb = MatterBatch(blocks)
    fill_fluid(mb, rng, B0=3e-3, omega=0.04)
    mb.name = f"random matter blocks seed {seed}"
    return mb


def c2p_states(mb: MatterBatch, rng, wmax=10.0, mag=10.0, n_atm=0, n_fast=0, ut_fast=30.0):
    """Overwrite the CC geometry and primitives of every stored cell with
    seeded independent states: a random symmetric positive conformal metric
    (eigenvalues > 0.3) and chi in [0.3, 1]; rho log-uniform in [1e-8, 1e-2],
    p / rho log-uniform in [1e-3, 10], W log-uniform in [1, wmax] along a
    random direction, B with b^2 / rho log-uniform in [1e-4, mag].  Then
    `n_atm` random cells per block get rho = 1e-16 (below any atmosphere
    threshold used in the tests) and `n_fast` cells |ut| = ut_fast."""
    for b, blk in enumerate(mb.blocks):
        shape = blk.cshape
        n = int(np.prod(shape))
        a = rng.normal(size=(n, 3, 3))
        g = np.eye(3)[None] + 0.15 * (a + np.transpose(a, (0, 2, 1)))
        bad = np.linalg.eigvalsh(g).min(axis=1) <= 0.3
        g[bad] = np.eye(3)
        chi = rng.uniform(0.3, 1.0, size=n)
        for q, (i, j) in enumerate(SYM):
            mb.view("geom", mb.geom, b, 1 + q)[...] = g[:, i, j].reshape(shape)
        mb.view("geom", mb.geom, b, 0)[...] = chi.reshape(shape)
        gam = g / chi[:, None, None]
        rho = 10.0 ** rng.uniform(-8.0, -2.0, size=n)
        p = rho * 10.0 ** rng.uniform(-3.0, 1.0, size=n)
        d = rng.normal(size=(n, 3))
        d /= np.sqrt(np.einsum("ni,nij,nj->n", d, gam, d))[:, None]
        W = 10.0 ** rng.uniform(0.0, math.log10(wmax), size=n)
        ut = d * np.sqrt(W * W - 1.0)[:, None]
        Bv = rng.normal(size=(n, 3))
        Bv *= np.sqrt(rho * 10.0 ** rng.uniform(-4.0, math.log10(mag), size=n)
                      / np.einsum("ni,nij,nj->n", Bv, gam, Bv))[:, None]
        if n_atm:
            idx = rng.choice(n, size=n_atm, replace=False)
            rho[idx] = 1e-16
            p[idx] = 1e-20
        if n_fast:
            idx = rng.choice(n, size=n_fast, replace=False)
            ut[idx] = d[idx] * ut_fast
        vals = [rho, ut[:, 0], ut[:, 1], ut[:, 2], p, Bv[:, 0], Bv[:, 1], Bv[:, 2]]
        for f in range(NPRIM):
            mb.view("prim", mb.prim, b, f)[...] = vals[f].reshape(shape)


def refined_pair(seed: int = 0, n_c: int = 24, n_f: int = 16, ng: int = 4, dx_c: float = 1.0,
                 c0=(4, 4, 4), nfine: int = 2, fill=None):
    """A coarse block and `nfine` fine blocks (spacing dx_c / 2) side by side
    along x inside it: fine block m has its vertex 0 on coarse vertex
    (c0[0] + m (n_f / 2), c0[1], c0[2]).  Fields: `fill(X, Y, Z, f)` at
    every stored point (default: smooth seeded trigonometric data).
    Returns the batch and the c0 of every fine block."""
    rng = np.random.default_rng(SEED_BASE + 2000 + seed)
    blocks = [Block(n_c, n_c, n_c, ng, dx_c, dx_c, dx_c)]
    origins = []
    for m in range(nfine):
        o = (c0[0] + m * (n_f // 2), c0[1], c0[2])
        origins.append(o)
        blocks.append(Block(n_f, n_f, n_f, ng, dx_c / 2, dx_c / 2, dx_c / 2,
                            x0=o[0] * dx_c, y0=o[1] * dx_c, z0=o[2] * dx_c))
    bt = Batch(blocks)
    a = rng.uniform(0.1, 0.4, size=(NF, 3))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=NF)
    for b, blk in enumerate(bt.blocks):
        X, Y, Z = blk.coords()
        for f in range(NF):
            if fill is None:
                v = np.sin(a[f, 0] * X + ph[f]) * np.cos(a[f, 1] * Y) + np.cos(a[f, 2] * Z + ph[f])
            else:
                v = fill(X, Y, Z, f)
            bt.view(bt.u, b, f)[...] = v
    bt.name = f"coarse {n_c}^3 + {nfine} fine {n_f}^3 blocks"
    return bt, origins


def level_jump(seed_offset: int = 7, ncoarse: int = 64, n: int = 16, ng: int = 4):
    """Transfers of a level jump at scale: `ncoarse` coarse blocks of n^3 + ng
    ghosts (spacing 1) and 8 fine blocks (spacing 1/2) per coarse block, fine
    block k being octant k % 8 of coarse block k // 8.
    * prolongation: every fine block receives its six face slabs (ng deep,
      n x n across; the edges and corners left out so that no two boxes
      meet), each from a coarse block drawn at random, whose vertex (4, 4, 4)
      lies under fine vertex 0 (so an order-6 stencil stays inside the
      coarse block's stored points);
    * restriction: every fine block injects its even interior vertices into
      its octant of its coarse block (coarse box 8 m .. 8 m + 8 per direction,
      m the octant bit, when n = 16).
    State: seeded uniform values in [-1, 1).  Returns (batch, prolongation
    transfers, restriction transfers) as dicts with coarse, fine, c0, lo, hi."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    h = n // 2
    blocks = [Block(n, n, n, ng, 1.0, 1.0, 1.0, x0=n * c, y0=0.0, z0=0.0)
              for c in range(ncoarse)]
    for k in range(8 * ncoarse):
        p, o = divmod(k, 8)
        m = (o & 1, (o >> 1) & 1, (o >> 2) & 1)
        blocks.append(Block(n, n, n, ng, 0.5, 0.5, 0.5, x0=n * p + h * m[0], y0=h * m[1],
                            z0=h * m[2]))
    bt = Batch(blocks)
    bt.u[:] = rng.uniform(-1.0, 1.0, size=bt.u.size)
    pro, res = [], []
    src = rng.integers(0, ncoarse, size=(8 * ncoarse, 6))
    for k in range(8 * ncoarse):
        fine = ncoarse + k
        s = 0
        for d in range(3):
            for lo, hi in ((-ng, 0), (n, n + ng)):
                b_lo, b_hi = [0] * 3, [n] * 3
                b_lo[d], b_hi[d] = lo, hi
                pro.append(dict(coarse=int(src[k, s]), fine=fine, c0=[4, 4, 4], lo=b_lo, hi=b_hi))
                s += 1
        p, o = divmod(k, 8)
        c0 = [h * ((o >> d) & 1) for d in range(3)]
        res.append(dict(coarse=p, fine=fine, c0=c0, lo=list(c0), hi=[c + h for c in c0]))
    bt.name = (f"level jump: {ncoarse} coarse + {8 * ncoarse} fine blocks of {n}^3+{ng}g; "
               f"{len(pro)} face slabs prolongated, {len(res)} octants restricted")
    return bt, pro, res


def refined_level_set(n: int = 8, ng: int = 4, grid=(3, 2, 2), refine=(1, 0, 0),
                      h0: float = 1.0 / 16.0, refine2=None):
    """An AMR level set with one level jump: level-0 blocks of n^3 points
    (spacing h0) on a grid of grid[0] x grid[1] x grid[2] blocks, the one at
    `refine` replaced by its 8 children (level 1, spacing h0 / 2, n^3
    points each); with `refine2` (0..7) that child replaced in turn by its 8
    children (level 2).  Positions on the integer lattice of the finest
    level (step 2^(Lmax - L) for level L): block vertex i sits at lattice
    o + i * step.  Returns (batch, locs) with locs[b] = (level, o); the state
    is zero."""
    lmax = 1 if refine2 is None else 2
    st = [1 << (lmax - L) for L in range(lmax + 1)]
    hl = h0 / st[0]                       # spacing of the lattice
    blocks, locs = [], []

    def add(level, o):
        h = h0 / (1 << level)
        blocks.append(Block(n, n, n, ng, h, h, h, o[0] * hl, o[1] * hl, o[2] * hl))
        locs.append((level, o))

    for gz in range(grid[2]):
        for gy in range(grid[1]):
            for gx in range(grid[0]):
                if (gx, gy, gz) != tuple(refine):
                    add(0, (n * st[0] * gx, n * st[0] * gy, n * st[0] * gz))
    r = tuple(refine)
    for m in range(8):
        mx, my, mz = m & 1, (m >> 1) & 1, (m >> 2) & 1
        o = (n * st[0] * r[0] + n * st[1] * mx, n * st[0] * r[1] + n * st[1] * my,
             n * st[0] * r[2] + n * st[1] * mz)
        if m != refine2:
            add(1, o)
            continue
        for m2 in range(8):
            ax, ay, az = m2 & 1, (m2 >> 1) & 1, (m2 >> 2) & 1
            add(2, (o[0] + n * st[2] * ax, o[1] + n * st[2] * ay, o[2] + n * st[2] * az))
    bt = Batch(blocks)
    bt.params = Params(fd_order=6)
    bt.name = (f"level set {grid[0]}x{grid[1]}x{grid[2]} blocks of {n}^3+{ng}g, block {refine} "
               f"refined into 8" + ("" if refine2 is None else f", child {refine2} again"))
    return bt, locs
