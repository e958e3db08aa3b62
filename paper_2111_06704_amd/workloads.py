"""Seeded synthetic workloads: electrode geometries and electrolyte frames.

This module is the only code shared by the CPU oracle and the GPU path. It
holds no arithmetic of the constant-potential method itself: it places
electrode atoms on graphene / AB-graphite lattices, draws random +-1 e point
charges between the electrodes, and assigns each electrode atom its potential
in volts. Units: lengths in Angstrom, charges in e, potentials in V.

Lattice (graphene, C-C bond R = 1.42 A): rectangular 4-atom cell of edges
3R (armchair) x sqrt(3)R (zigzag), basis (0,0), (R,0), (1.5R, sqrt(3)/2 R),
(2.5R, sqrt(3)/2 R) along (armchair, zigzag). AB stacking shifts every other
layer by R along the armchair direction; graphite interlayer spacing 3.35 A.

Workload sizes follow the constant-potential electrode study of the paper
(graphene electrodes, 1 V, slit filled with electrolyte; Sec. IV) at the
sizes listed in ``WORKLOAD_SIZES``; the paper's equilibrated water/NaCl frames are
replaced by uniform random +-1 e point charges.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BOND = 1.42                      # graphene C-C bond length, Angstrom
INTERLAYER = 3.35                # graphite interlayer spacing, Angstrom
ARMCHAIR = 3.0 * BOND            # rectangular cell edge along armchair
ZIGZAG = math.sqrt(3.0) * BOND   # rectangular cell edge along zigzag

# Default electrostatic parameters of the workloads: Gaussian inverse width
# of electrode charges (1/A), Ewald splitting (1/A), real-space cutoff (A),
# reciprocal-space accuracy (dimensionless), applied voltage (V).
GAUSS_INV_WIDTH = 1.979
EWALD_SPLIT = 0.3
RCUT = 12.0
KSPACE_EPS = 1e-6
DELTA_V = 1.0


@dataclasses.dataclass(frozen=True)
class Geometry:
    name: str
    pos: np.ndarray          # (N, 3) float64 electrode atom positions
    box: np.ndarray          # (3,) float64 orthorhombic box edges
    layer: np.ndarray        # (N,) int32 global layer index (0 .. n_layers-1)
    electrode: np.ndarray    # (N,) int8: 0 = electrode A (chi = +dV/2), 1 = B
    n_layers: int
    ion_zlo: float           # electrolyte slab [ion_zlo, ion_zhi]
    ion_zhi: float
    sheet_density: float     # atoms per A^2 per layer

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def _sheet(ncell_arm: int, ncell_zig: int, armchair_along_x: bool,
           shift: bool) -> np.ndarray:
    """In-plane positions of one graphene sheet, (4*ncell_arm*ncell_zig, 2)."""
    basis = np.array([[0.0, 0.0], [BOND, 0.0],
                      [1.5 * BOND, 0.5 * ZIGZAG], [2.5 * BOND, 0.5 * ZIGZAG]])
    ia, iz = np.meshgrid(np.arange(ncell_arm), np.arange(ncell_zig), indexing="ij")
    origin = np.stack([ia.ravel() * ARMCHAIR, iz.ravel() * ZIGZAG], axis=1)
    pts = (origin[:, None, :] + basis[None, :, :]).reshape(-1, 2)
    if shift:
        pts[:, 0] = pts[:, 0] + BOND
    pts[:, 0] = np.mod(pts[:, 0], ncell_arm * ARMCHAIR)
    if armchair_along_x:
        return pts
    return pts[:, ::-1].copy()


def electrode_geometry(name: str, ncell_arm: int, ncell_zig: int,
                       armchair_along_x: bool, layers_a: list[float],
                       layers_b: list[float], lz: float,
                       ion_margin: float = 2.0) -> Geometry:
    if armchair_along_x:
        lx, ly = ncell_arm * ARMCHAIR, ncell_zig * ZIGZAG
    else:
        lx, ly = ncell_zig * ZIGZAG, ncell_arm * ARMCHAIR
    pos, layer, elec = [], [], []
    zs = list(layers_a) + list(layers_b)
    for li, z in enumerate(zs):
        xy = _sheet(ncell_arm, ncell_zig, armchair_along_x, shift=(li % 2 == 1))
        pos.append(np.column_stack([xy, np.full(len(xy), z)]))
        layer.append(np.full(len(xy), li, dtype=np.int32))
        elec.append(np.full(len(xy), 0 if li < len(layers_a) else 1, dtype=np.int8))
    density = 4.0 / (ARMCHAIR * ZIGZAG)
    return Geometry(name=name, pos=np.concatenate(pos), box=np.array([lx, ly, lz]),
                    layer=np.concatenate(layer), electrode=np.concatenate(elec),
                    n_layers=len(zs), ion_zlo=max(layers_a) + ion_margin,
                    ion_zhi=min(layers_b) - ion_margin, sheet_density=density)


def _stack(face: float, nlay: int, outward: float) -> list[float]:
    """Layer heights of an electrode whose face is at ``face``; layers stack
    away from the gap in direction ``outward`` (-1 or +1)."""
    zs = [face + outward * INTERLAYER * k for k in range(nlay)]
    return sorted(zs)


def geometry(cfg: int) -> Geometry:
    """Electrode geometry of workload ``cfg`` (1, 2, 3, 4 or 5).

    1: two graphene sheets, 6x6 cells each (N = 288), 25.56 x 14.757 x 60 A,
       sheets at z = 10 and 50.
    2/4: two 3-layer AB graphite electrodes, 16x12 cells/layer (N = 4608),
       39.352 x 51.12 x 100 A, 50 A gap centred in z.
    3: two 4-layer electrodes, 32x32 cells/layer (N = 32768),
       78.704 x 136.32 x 120 A, 50 A gap.
    5: two 4-layer electrodes, 64x64 cells/layer (N = 131072),
       157.41 x 272.64 x 120 A, 50 A gap.
    """
    if cfg == 1:
        return electrode_geometry("graphene_2x144", 6, 6, True, [10.0], [50.0], 60.0)
    if cfg in (2, 4):
        lz = 100.0
        return electrode_geometry("graphite_2x3x768", 12, 16, False,
                                  _stack(lz / 2 - 25.0, 3, -1), _stack(lz / 2 + 25.0, 3, +1), lz)
    if cfg == 3:
        lz = 120.0
        return electrode_geometry("graphite_2x4x4096", 32, 32, False,
                                  _stack(lz / 2 - 25.0, 4, -1), _stack(lz / 2 + 25.0, 4, +1), lz)
    if cfg == 5:
        lz = 120.0
        return electrode_geometry("graphite_2x4x16384", 64, 64, False,
                                  _stack(lz / 2 - 25.0, 4, -1), _stack(lz / 2 + 25.0, 4, +1), lz)
    raise ValueError(f"unknown workload {cfg}")


# ions per frame and frames per workload
WORKLOAD_SIZES = {
    1: dict(m=200, frames=16),
    2: dict(m=2000, frames=16),
    3: dict(m=20000, frames=64),
    4: dict(m=2000, frames=16, train_frames=10000),
    5: dict(m=200000, frames=32),
}


def frame_seed(cfg: int, f: int) -> int:
    return 1_000_000 * cfg + f


def train_seed(t: int) -> int:
    return 4_000_000 + t


def ion_frame(geo: Geometry, m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """One electrolyte frame: m point charges, the first m//2 at +1 e and the
    rest at -1 e, uniform in x, y and in z within [ion_zlo, ion_zhi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((m, 3))
    lx, ly, _ = geo.box
    pos = np.empty((m, 3))
    pos[:, 0] = u[:, 0] * lx
    pos[:, 1] = u[:, 1] * ly
    pos[:, 2] = geo.ion_zlo + u[:, 2] * (geo.ion_zhi - geo.ion_zlo)
    q = np.empty(m)
    q[: m // 2] = 1.0
    q[m // 2:] = -1.0
    return pos, q


def ion_frames(geo: Geometry, m: int, seeds) -> tuple[np.ndarray, np.ndarray]:
    """Stack of frames: positions (F, m, 3) and charges (F, m)."""
    ps, qs = zip(*(ion_frame(geo, m, s) for s in seeds))
    return np.stack(ps), np.stack(qs)


def electrode_potential(geo: Geometry, delta_v: float = DELTA_V) -> np.ndarray:
    """Applied potential per electrode atom in volts: +dV/2 on A, -dV/2 on B."""
    return np.where(geo.electrode == 0, 0.5 * delta_v, -0.5 * delta_v).astype(np.float64)


def jitter(geo: Geometry, amp: float, seed: int) -> Geometry:
    """Copy of ``geo`` with positions displaced by U(-amp, amp) per component."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = geo.pos + rng.uniform(-amp, amp, size=geo.pos.shape)
    return dataclasses.replace(geo, pos=pos, name=geo.name + "_jit")


def workload(cfg: int, frames: int | None = None, first_frame: int = 0):
    """Geometry, ion positions (F, M, 3), ion charges (F, M) and electrode
    potentials (N,) in volts for workload ``cfg``."""
    geo = geometry(cfg)
    c = WORKLOAD_SIZES[cfg]
    nf = c["frames"] if frames is None else frames
    seed_cfg = 2 if cfg == 4 else cfg
    ipos, iq = ion_frames(geo, c["m"], [frame_seed(seed_cfg, first_frame + f) for f in range(nf)])
    return geo, ipos, iq, electrode_potential(geo)
