"""Seeded synthetic geomodels for the TPFA flux path.

This module holds random draws and physical constants only: none of the flux
method's arithmetic (density law, transmissibility, potential difference,
upwinding, flux or derivatives) lives here. Both the CPU oracle and the GPU
library are fed from it, so the two sides always see identical bytes.

The paper (Sec. 6) loads an Nx x Ny x Nz mesh with X innermost and Z
outermost but never describes its contents, so every field is synthetic:

* ln(kx) ~ Normal(ln 1e-13, sigma^2), i.i.d. per cell (log-normal permeability
  with median 1e-13 m^2); ky = ry * kx and kz = rz * kx;
* porosity ~ Uniform(0.1, 0.3) (drawn on request; the flux path never reads it);
* seal bits: bit a of a cell closes the face towards its +a neighbour
  (a = 0, 1, 2 for x, y, z); each interior face is closed with probability
  ``seal_prob`` independently;
* pressure noise ~ Uniform(-1e5, 1e5) Pa per cell: the pressure field is the
  hydrostatic reference profile of the column plus this noise. Computing the
  reference profile uses the density law, so it is left to the consumer.

Arrays are C-ordered with shape (nz, ny, nx), i.e. x fastest, which is the
layout idx = i + nx * (j + ny * k) used everywhere else.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

LN_K_MEDIAN = math.log(1e-13)
NOISE_AMP = 1e5


@dataclass(frozen=True)
class Grid:
    """Cartesian grid: cell counts, cell sizes (m) and gravity along +k (m/s^2)."""
    nx: int
    ny: int
    nz: int
    dx: float = 10.0
    dy: float = 10.0
    dz: float = 2.0
    gk: float = 9.81  # k points down (depth); a k-up grid passes -9.81

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass(frozen=True)
class Fluid:
    """Slightly compressible fluid: reference density, compressibility,
    reference pressure and constant viscosity (SI)."""
    rho0: float = 1000.0
    cf: float = 1e-9
    p0: float = 1e7
    mu: float = 1e-3


@dataclass
class Geomodel:
    name: str
    grid: Grid
    fluid: Fluid
    sigma: float
    seed: int
    logk: np.ndarray            # ln kx, float64, (nz, ny, nx)
    kx: np.ndarray              # exp(logk), float64
    ry: float
    rz: float
    seal: np.ndarray            # uint8 bits, (nz, ny, nx)
    noise: List[np.ndarray]     # pressure offsets from the reference profile, float64
    p_top: float = 1e7          # reference pressure of the top layer (k = 0)
    porosity: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def ncell(self) -> int:
        return self.grid.ncell

    def kx32(self) -> np.ndarray:
        return self.kx.astype(np.float32)

    def dp32(self, r: int = 0) -> np.ndarray:
        """Pressure offset field r stored in FP32 (the precision form's state)."""
        return self.noise[r].astype(np.float32)


def _seal_bits(rng: np.random.Generator, grid: Grid, prob: float) -> np.ndarray:
    seal = np.zeros(grid.shape, dtype=np.uint8)
    if prob <= 0.0:
        return seal
    for axis in range(3):
        closed = rng.random(grid.shape, dtype=np.float32) < np.float32(prob)
        # only interior faces exist: the last layer along the axis has no +face
        if axis == 0:
            closed[:, :, -1] = False
        elif axis == 1:
            closed[:, -1, :] = False
        else:
            closed[-1, :, :] = False
        seal |= closed.astype(np.uint8) << np.uint8(axis)
    return seal


def draw(name: str, grid: Grid, *, sigma: float, seed: int, ry: float = 1.0,
         rz: float = 1.0, seal_prob: float = 0.0, noise_seeds=(None,),
         fluid: Fluid = Fluid(), with_porosity: bool = False) -> Geomodel:
    """Draw one geomodel. Each field comes from its own child stream of
    ``SeedSequence(seed)`` so that skipping one draw leaves the others
    unchanged; pressure-noise field r comes from ``default_rng(noise_seeds[r])``
    (``None`` means a fourth child stream of the geomodel seed)."""
    ss = np.random.SeedSequence(seed)
    s_logk, s_phi, s_seal, s_noise = ss.spawn(4)
    logk = np.random.default_rng(s_logk).standard_normal(grid.shape)
    logk *= sigma
    logk += LN_K_MEDIAN
    kx = np.exp(logk)
    phi = None
    if with_porosity:
        phi = np.random.default_rng(s_phi).uniform(0.1, 0.3, grid.shape)
    seal = _seal_bits(np.random.default_rng(s_seal), grid, seal_prob)
    noise = []
    for ns in noise_seeds:
        rng = np.random.default_rng(s_noise if ns is None else ns)
        noise.append(rng.uniform(-NOISE_AMP, NOISE_AMP, grid.shape))
    return Geomodel(name=name, grid=grid, fluid=fluid, sigma=sigma, seed=seed,
                    logk=logk, kx=kx, ry=ry, rz=rz, seal=seal, noise=noise,
                    p_top=fluid.p0, porosity=phi)


# ---------------------------------------------------------------------------
# The workloads. Shared physics: dx = dy = 10 m, dz = 2 m, rho0 = 1000 kg/m^3,
# cf = 1e-9 1/Pa, p0 = 1e7 Pa, mu = 1e-3 Pa s, gk = +9.81 m/s^2.
# ---------------------------------------------------------------------------

def tiny16(seed: int = 1) -> Geomodel:
    """16x16x16, sigma = 1, isotropic, no seals, one pressure field."""
    return draw("tiny16", Grid(16, 16, 16), sigma=1.0, seed=seed,
                noise_seeds=(None,), with_porosity=True)


BIG_NOISE_SEEDS = (2, 21, 22, 23)


def big512(seed: int = 2, nx: int = 512, ny: int = 512, nz: int = 256,
           noise_seeds=BIG_NOISE_SEEDS) -> Geomodel:
    """512x512x256 (67,108,864 cells): sigma = 1.5, ky = kx, kz = 0.1 kx,
    1% of interior faces sealed per direction, four pressure fields.
    Smaller nx/ny/nz give the same recipe at other sizes."""
    return draw(f"big{nx}x{ny}x{nz}", Grid(nx, ny, nz), sigma=1.5, seed=seed,
                ry=1.0, rz=0.1, seal_prob=0.01, noise_seeds=noise_seeds)


def ensemble_dims(n_models: int = 64, base_seed: int = 4000):
    """Per-model (nx, ny, nz, sigma) of the uneven ensemble: nx, ny ~ U{32..256},
    nz ~ U{32..128}, sigma ~ U(0.5, 2.0), model m seeded with base_seed + m."""
    out = []
    for m in range(n_models):
        rng = np.random.default_rng(base_seed + m)
        nx = int(rng.integers(32, 257))
        ny = int(rng.integers(32, 257))
        nz = int(rng.integers(32, 129))
        sigma = float(rng.uniform(0.5, 2.0))
        out.append((nx, ny, nz, sigma))
    return out


def ensemble(n_models: int = 64, base_seed: int = 4000, scale: float = 1.0) -> List[Geomodel]:
    """The uneven ensemble, one pressure field per model. ``scale`` < 1 shrinks
    every dimension (at least 2 cells) for quick tests of the same structure."""
    models = []
    for m, (nx, ny, nz, sigma) in enumerate(ensemble_dims(n_models, base_seed)):
        if scale != 1.0:
            nx, ny, nz = (max(2, int(round(v * scale))) for v in (nx, ny, nz))
        models.append(draw(f"ens{m}", Grid(nx, ny, nz), sigma=sigma,
                           seed=base_seed + m, ry=1.0, rz=0.1, seal_prob=0.01,
                           noise_seeds=(None,)))
    return models


def adjoint256(seed: int = 5, nx: int = 256, ny: int = 256, nz: int = 128,
               n_sets: int = 4) -> Geomodel:
    """256x256x128 with the big512 recipe; n_sets pressure fields and as many
    cotangents w ~ N(0, 1) in ``extra['w']`` (w set r seeded with 11*seed + r,
    so the 256x256x128 case uses seeds 55..58)."""
    noise_seeds = (None,) + tuple(100 * seed + r for r in range(1, n_sets))
    g = draw(f"adj{nx}x{ny}x{nz}", Grid(nx, ny, nz), sigma=1.5, seed=seed,
             ry=1.0, rz=0.1, seal_prob=0.01, noise_seeds=noise_seeds)
    g.extra["w"] = [np.random.default_rng(11 * seed + r).standard_normal(g.grid.shape)
                    for r in range(n_sets)]
    return g


def fd32(seed: int = 6) -> Geomodel:
    """32^3 grid of the adjoint recipe for finite-difference checks."""
    return adjoint256(seed=seed, nx=32, ny=32, nz=32, n_sets=1)


def random_small(seed: int, nx: int, ny: int, nz: int, *, sigma: float = 1.0,
                 ry: float = 1.0, rz: float = 0.1, seal_prob: float = 0.05,
                 gk: float = 9.81) -> Geomodel:
    """Small odd-shaped grids for parity and property tests."""
    return draw(f"small{nx}x{ny}x{nz}s{seed}", Grid(nx, ny, nz, gk=gk), sigma=sigma,
                seed=seed, ry=ry, rz=rz, seal_prob=seal_prob, noise_seeds=(None,))


# The paper's own workloads (Sec. 7, weak-scaling table): Nx x Ny x 246 meshes
# from 200 x 200 up to the full 750 x 994 fabric, residual only, 10 fluxes per
# cell, FP32.
PAPER10_SHAPES = ((200, 200, 246), (400, 400, 246), (600, 600, 246), (750, 600, 246),
                  (750, 800, 246), (750, 994, 246))
LN_T_DIAG_MEDIAN = math.log(1e-13)


def paper10(nx: int = 750, ny: int = 994, nz: int = 246, seed: int = 8) -> Geomodel:
    """A 10-flux workload, drawn directly in FP32 (the paper's precision) to keep
    the 183M-cell case small: ln kx ~ N(ln 1e-13, 1), ky = kx, kz = 0.1 kx, no
    seals, pressure noise ~ U(-1e5, 1e5) Pa, and the two diagonal
    transmissibility fields (m^3) ``extra['tne']``, ``extra['tse']`` with
    ln t ~ N(ln 1e-13, 1) i.i.d. per cell. All arrays are float32."""
    grid = Grid(nx, ny, nz)
    s_logk, s_noise, s_tne, s_tse = np.random.SeedSequence(seed).spawn(4)
    logk = np.random.default_rng(s_logk).standard_normal(grid.shape, dtype=np.float32)
    logk += np.float32(LN_K_MEDIAN)
    kx = np.exp(logk)
    noise = np.random.default_rng(s_noise).random(grid.shape, dtype=np.float32)
    noise *= np.float32(2 * NOISE_AMP)
    noise -= np.float32(NOISE_AMP)
    geo = Geomodel(name=f"paper10_{nx}x{ny}x{nz}", grid=grid, fluid=Fluid(), sigma=1.0,
                   seed=seed, logk=logk, kx=kx, ry=1.0, rz=0.1,
                   seal=np.zeros(grid.shape, np.uint8), noise=[noise])
    for key, s in (("tne", s_tne), ("tse", s_tse)):
        t = np.random.default_rng(s).standard_normal(grid.shape, dtype=np.float32)
        t += np.float32(LN_T_DIAG_MEDIAN)
        geo.extra[key] = np.exp(t)
    return geo


def paper10_trans(nx: int = 750, ny: int = 994, nz: int = 246, seed: int = 18) -> dict:
    """All ten transmissibilities of the paper's data model (Sec. 5), one per
    face: tx, ty, tz with ln t ~ N(ln(a_d r_d 1e-13), 1) (a_x = a_y = 2 m,
    a_z = 50 m, r_z = 0.1) and the diagonal tne, tse as in paper10; float32."""
    grid = Grid(nx, ny, nz)
    out = {}
    medians = {"tx": grid.dy * grid.dz / grid.dx * 1e-13, "ty": grid.dx * grid.dz / grid.dy * 1e-13,
               "tz": 0.1 * grid.dx * grid.dy / grid.dz * 1e-13, "tne": 1e-13, "tse": 1e-13}
    for key, s in zip(("tx", "ty", "tz", "tne", "tse"), np.random.SeedSequence(seed).spawn(5)):
        t = np.random.default_rng(s).standard_normal(grid.shape, dtype=np.float32)
        t += np.float32(math.log(medians[key]))
        out[key] = np.exp(t)
    return out


def diagonal_t(grid: Grid, seed: int, zero_prob: float = 0.1) -> tuple:
    """Diagonal transmissibility fields (tne, tse), float64, for small grids:
    ln t ~ N(ln 1e-13, 1), with a fraction ``zero_prob`` of faces closed (t = 0)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(2):
        t = np.exp(LN_T_DIAG_MEDIAN + rng.standard_normal(grid.shape))
        t[rng.random(grid.shape) < zero_prob] = 0.0
        out.append(t)
    return tuple(out)


# Per-direction permeability arrays: the geomodel's kx with independent
# log-normal anisotropy factors for ky and kz (kz around the recipe's 0.1 kx).
def k3_fields(kx: np.ndarray, seed: int, sigma_y: float = 0.3, sigma_z: float = 0.5,
              rz: float = 0.1) -> tuple:
    """(kx, ky, kz), float64: ky = kx exp(sigma_y N(0, 1)), kz = rz kx
    exp(sigma_z N(0, 1)), the two normal fields drawn in that order from
    default_rng(seed)."""
    rng = np.random.default_rng(seed)
    kx = np.asarray(kx, dtype=np.float64)
    ky = kx * np.exp(sigma_y * rng.standard_normal(kx.shape))
    kz = rz * kx * np.exp(sigma_z * rng.standard_normal(kx.shape))
    return kx, ky, kz


# Backward-Euler inputs (accumulation term of Eq. (2)): reference porosity,
# previous-level pressure noise and a Krylov direction.
BE_DT = 86400.0   # one day (s)
BE_CR = 5e-10     # rock compressibility (1/Pa)


def be_fields(grid: Grid, seed: int, step_amp: float = 5e4) -> dict:
    """phi_ref ~ U(0.1, 0.3); the previous level's pressure differs from the
    current one by U(-step_amp, step_amp) Pa per cell (``dp_step``, to be
    subtracted from the current pressure); v ~ N(0, 1). Float64, (nz, ny, nx)."""
    s_phi, s_step, s_v = np.random.SeedSequence(seed).spawn(3)
    return {"phi": np.random.default_rng(s_phi).uniform(0.1, 0.3, grid.shape),
            "dp_step": np.random.default_rng(s_step).uniform(-step_amp, step_amp, grid.shape),
            "v": np.random.default_rng(s_v).standard_normal(grid.shape),
            "dt": BE_DT, "cr": BE_CR}


# Spatially correlated permeability and planar fault barriers (structured
# geomodels beyond i.i.d. fields).

def correlated_logk(grid: Grid, seed: int, sigma: float = 1.5,
                    corr_len=(8.0, 8.0, 2.0)) -> np.ndarray:
    """ln kx with a Gaussian covariance: white noise filtered by a Gaussian
    kernel of standard deviation ``corr_len`` cells along (x, y, z) through
    the FFT (periodic), rescaled to unit variance, times sigma, plus
    ln 1e-13."""
    w = np.random.default_rng(seed).standard_normal(grid.shape)
    f = np.fft.rfftn(w)
    kz = np.fft.fftfreq(grid.nz)[:, None, None]
    ky = np.fft.fftfreq(grid.ny)[None, :, None]
    kx = np.fft.rfftfreq(grid.nx)[None, None, :]
    lx, ly, lz = corr_len
    f *= np.exp(-2.0 * np.pi ** 2 * ((kx * lx) ** 2 + (ky * ly) ** 2 + (kz * lz) ** 2))
    x = np.fft.irfftn(f, s=grid.shape, axes=(0, 1, 2))
    x /= x.std() if x.std() > 0 else 1.0
    return LN_K_MEDIAN + sigma * x


def fault_seals(grid: Grid, *, x_fault: Optional[int] = None, y_fault: Optional[int] = None,
                z_barrier: Optional[int] = None, gaps: float = 0.0, seed: int = 0) -> np.ndarray:
    """Seal bits of planar barriers: every +x face of the cells at i = x_fault
    (a vertical fault normal to x), every +y face at j = y_fault, every +z face
    at k = z_barrier (a shale layer); a fraction ``gaps`` of each barrier's
    faces is left open at random."""
    seal = np.zeros(grid.shape, np.uint8)
    rng = np.random.default_rng(seed)
    for bit, idx, axis_len in ((0, x_fault, grid.nx), (1, y_fault, grid.ny), (2, z_barrier, grid.nz)):
        if idx is None or not (0 <= idx < axis_len - 1):
            continue
        sl = [slice(None)] * 3
        sl[2 - bit] = idx
        face = np.ones(seal[tuple(sl)].shape, bool)
        if gaps > 0:
            face &= rng.random(face.shape) >= gaps
        seal[tuple(sl)] |= (face.astype(np.uint8) << np.uint8(bit))
    return seal


def faulted(seed: int = 12, nx: int = 96, ny: int = 80, nz: int = 40) -> Geomodel:
    """Correlated ln k (sigma 1.5, correlation 8 x 8 x 2 cells), kz = 0.1 kx, a
    vertical fault at i = nx/3 and a shale barrier at k = nz/2 with 10% gaps,
    plus 0.5% random seals; one pressure field."""
    grid = Grid(nx, ny, nz)
    geo = draw(f"faulted{nx}x{ny}x{nz}", grid, sigma=1.5, seed=seed, ry=1.0, rz=0.1,
               seal_prob=0.005)
    geo.logk = correlated_logk(grid, seed + 1)
    geo.kx = np.exp(geo.logk)
    geo.seal |= fault_seals(grid, x_fault=nx // 3, z_barrier=nz // 2, gaps=0.1, seed=seed + 2)
    return geo
