"""Seeded synthetic workloads (inputs only: geometry, media, field points, seeds).

This module is shared by the tests, the benchmark and the smoke check.  It holds no
step of the method: sample points, transmission coefficients and fields are computed
by the library (and, in tests, independently by the reference).  It only fixes the
configurations, as plain numbers and numpy arrays:

  piston_axis  (Sec. 3 piston in water, 1 MHz, on-axis line)
  one_interface (water -> 5900 m/s solid at 50 mm, 10 deg tilt, 5 MHz, 512 x 512 image)
  layered_stack (three interfaces 2 mm apart, 64 frequencies 1-10 MHz, 128^3 volume)
  focused_normal (Sec. 3.3: spherical-cap transducer over a water/steel interface)
  ray_crossover (Sec. 3.5: RSI vs ray tracing against the number of field points)
  scan_batch   (256 uneven scan positions of the piston in water)
  surrogate    (parameter box of the learned surrogate)

Material constants of Sec. 3: water rho 1000 kg/m^3, c 1480 m/s; the solids use the
speeds named by each workload with the densities listed below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

WATER = (1480.0, 1000.0)          # (c m/s, rho kg/m^3), Sec. 3
STEEL_5900 = (5900.0, 7800.0)     # second medium of the interface workloads
STEEL_PAPER = (5840.0, 7800.0)    # steel of Sec. 3 (the paper-geometry variants)
ALU_PAPER = (6409.0, 2700.0)      # aluminium of Sec. 3
MID_2700 = (2700.0, 2700.0)       # middle layer of the stack (speed 2700 m/s)
PISTON_RADIUS = 6.35e-3           # Sec. 3


def deg(a: float) -> float:
    return a * math.pi / 180.0


@dataclass
class PistonAxis:
    """Plain piston in water at 1 MHz, 4096 samples (seed 0), 1024 on-axis points."""
    radius: float = PISTON_RADIUS
    freq: float = 1.0e6
    medium: Tuple[float, float] = WATER
    n_src: int = 4096
    seed: int = 0
    n_tgt: int = 1024
    z0: float = 1.0e-3
    z1: float = 0.1

    def targets(self):
        z = np.linspace(self.z0, self.z1, self.n_tgt)
        return np.zeros_like(z), np.zeros_like(z), z


@dataclass
class OneInterface:
    """Water -> solid interface at z = 50 mm under a 10 deg tilted piston at 5 MHz."""
    radius: float = PISTON_RADIUS
    freq: float = 5.0e6
    tilt: float = deg(10.0)
    n_xd: int = 1 << 16
    xd_seed: int = 0
    z_if: float = 0.05
    n_if: int = 1 << 18
    if_seed: int = 1
    half_width: float = 0.03
    media: Tuple[Tuple[float, float], ...] = (WATER, STEEL_5900)
    nx: int = 512
    nz: int = 512
    depth0: float = 1.0e-3
    depth1: float = 40.0e-3

    @property
    def patch_centre(self) -> Tuple[float, float]:
        # where the piston axis meets the interface plane
        return (self.z_if * math.tan(self.tilt), 0.0)

    @property
    def axis(self):
        return (math.sin(self.tilt), 0.0, math.cos(self.tilt))

    def targets(self, nx=None, nz=None):
        """Image in the x-z plane (y = 0), row-major [z][x]."""
        nx = nx or self.nx
        nz = nz or self.nz
        xc = self.patch_centre[0]
        x = np.linspace(xc - 0.020, xc + 0.040, nx)
        z = self.z_if + np.linspace(self.depth0, self.depth1, nz)
        X, Z = np.meshgrid(x, z)
        return X.ravel().copy(), np.zeros(X.size), Z.ravel().copy()

    @property
    def pairs(self) -> int:
        return self.n_xd * self.n_if + self.n_if * self.nx * self.nz


@dataclass
class InterfaceContinuity:
    """Points on the beam axis within 1 mm on each side of a water -> solid interface at
    oblique incidence (the configuration of the paper's near-interface comparison,
    Sec. 3.2): along the incident axis above the plane and the refracted axis (eq. 15)
    below it.  The interface is sampled densely (2^22 points over 60 mm, spacing 0.03 mm)
    so that the integrals stay resolved 0.1 mm from the plane."""
    radius: float = PISTON_RADIUS
    freq: float = 2.5e6
    tilt: float = deg(10.0)
    n_xd: int = 1 << 16
    xd_seed: int = 0
    z_if: float = 0.05
    n_if: int = 1 << 22
    if_seed: int = 1
    half_width: float = 0.03
    media: Tuple[Tuple[float, float], ...] = (WATER, STEEL_5900)
    n_d: int = 10
    d_min: float = 1.0e-4
    d_max: float = 1.0e-3

    @property
    def patch_centre(self) -> Tuple[float, float]:
        return (self.z_if * math.tan(self.tilt), 0.0)

    @property
    def axis(self):
        return (math.sin(self.tilt), 0.0, math.cos(self.tilt))

    @property
    def distances(self) -> np.ndarray:
        return np.geomspace(self.d_min, self.d_max, self.n_d)

    def points(self, side: str):
        """side 'above': back along the incident axis; 'below': along the refracted axis."""
        x0, d = self.patch_centre[0], self.distances
        if side == "above":
            ux, uz = -math.sin(self.tilt), -math.cos(self.tilt)
        else:
            s2 = self.media[1][0] / self.media[0][0] * math.sin(self.tilt)
            ux, uz = s2, math.sqrt(1.0 - s2 * s2)
        return x0 + d * ux, np.zeros_like(d), self.z_if + d * uz


@dataclass
class FocusedNormal:
    """Focused transducer at normal incidence (Sec. 3.3): a spherical cap of aperture
    radius 6.35 mm and radius of curvature 33 mm, apex at the origin, 10 mm of water
    above a steel half-space, 2.5 MHz, 10^5 Halton samples on every surface (Sec. 2.3),
    interface sampled over +-3a (Sec. 2.3) about the axis.  Field: a 401 x 401 slice of
    the y-z plane (x = 0) in the steel, 1-25 mm below the interface, an on-axis line
    and the off-axis line at z = 14 mm (the paper's stated focal depth)."""
    radius: float = PISTON_RADIUS
    curvature: float = 0.033
    freq: float = 2.5e6
    water_path: float = 0.010
    media: Tuple[Tuple[float, float], ...] = (WATER, STEEL_PAPER)
    n_xd: int = 100000
    n_if: int = 100000
    xd_seed: int = 0
    if_seed: int = 1 << 20       # Halton: the interface starts 2^20 indices further on
    n_grid: int = 401
    half_y: float = 0.010
    depth0: float = 1.0e-3
    depth1: float = 25.0e-3
    n_axis: int = 1001
    z_focus_paper: float = 0.014
    apod_width: float = PISTON_RADIUS

    @property
    def half_width(self) -> float:
        return 3.0 * self.radius

    @property
    def axis_z(self) -> np.ndarray:
        return self.water_path + np.linspace(self.depth0, self.depth1, self.n_axis)

    def grid(self, n=None):
        """y-z slice at x = 0, row-major [z][y]."""
        n = n or self.n_grid
        y = np.linspace(-self.half_y, self.half_y, n)
        z = self.water_path + np.linspace(self.depth0, self.depth1, n)
        Z, Y = np.meshgrid(z, y, indexing="ij")
        return np.zeros(Z.size), Y.ravel().copy(), Z.ravel().copy()

    def axis_line(self):
        z = self.axis_z
        return np.zeros_like(z), np.zeros_like(z), z

    def focal_line(self, n=None):
        n = n or self.n_grid
        y = np.linspace(-self.half_y, self.half_y, n)
        return np.zeros_like(y), y, np.full_like(y, self.z_focus_paper)


@dataclass
class RayCrossover:
    """Cost of the two models against the number of field points (Sec. 3.5): the
    oblique piston (10 deg, 2.5 MHz, 0.1 m water path) above no plane (water), one
    (water/steel) or four (water/steel/aluminium/steel/water, 2 mm layers, the
    materials of Sec. 3), 10^5 Halton samples on every sampled surface (Sec. 3),
    interface patches of half-width 3a (Sec. 2.3) centred on the Snell-chained beam
    intercepts.  Field points: seeded uniform in a box about the refracted beam axis
    2-20 mm below the last plane (the paper spreads them over all layers; here they all
    lie in the last medium, which every method evaluates the same way)."""
    radius: float = PISTON_RADIUS
    freq: float = 2.5e6
    tilt: float = deg(10.0)
    water_path: float = 0.1
    layer: float = 0.002
    n_samples: int = 100000
    xd_seed: int = 0
    n_field: Tuple[int, ...] = (1, 10, 100, 1000, 10000, 100000, 1000000)
    stacks: Tuple[Tuple[Tuple[float, float], ...], ...] = (
        (WATER,),
        (WATER, STEEL_PAPER),
        (WATER, STEEL_PAPER, ALU_PAPER, STEEL_PAPER, WATER),
    )

    @property
    def half_width(self) -> float:
        return 3.0 * self.radius

    @property
    def axis(self):
        return (math.sin(self.tilt), 0.0, math.cos(self.tilt))

    def planes(self, media) -> List[float]:
        return [self.water_path + m * self.layer for m in range(len(media) - 1)]

    def patch_centres(self, media) -> List[float]:
        zs = self.planes(media)
        return snell_intercepts(0.0, self.tilt, zs, [m[0] for m in media]) if zs else []

    def field(self, media, n: int, seed: int = 0):
        zs = self.planes(media)
        z_top = zs[-1] if zs else self.water_path
        speeds = [m[0] for m in media]
        if zs:
            x_top = self.patch_centres(media)[-1]
            s = min(math.sin(self.tilt) / speeds[0] * speeds[-1], 0.999999)
        else:
            x_top, s = z_top * math.tan(self.tilt), math.sin(self.tilt)
        t = s / math.sqrt(1 - s * s)
        rng = np.random.default_rng([seed, len(media), n])
        d = rng.uniform(0.002, 0.020, n)
        x = x_top + d * t + rng.uniform(-0.010, 0.010, n)
        y = rng.uniform(-0.005, 0.005, n)
        return x, y, z_top + d


def snell_intercepts(x0: float, tilt: float, z_if, speeds) -> List[float]:
    """Horizontal positions where the beam axis crosses each plane (input recipe only)."""
    C = math.sin(tilt) / speeds[0]
    xs = [x0 + (z_if[0]) * math.tan(tilt)]
    for l in range(1, len(z_if)):
        s = min(C * speeds[l], 0.999999)
        xs.append(xs[-1] + (z_if[l] - z_if[l - 1]) * s / math.sqrt(1 - s * s))
    return xs


@dataclass
class MultilayerNoise:
    """QMC noise of the RSI chain through thin layers (Sec. 3.4): the piston tilted 10 deg
    at 2.5 MHz under 10 mm of water, six 2 mm layers alternating steel and aluminium and a
    steel half-space below (seven planes), Halton samples on the piston (index 1..) and on
    every interface patch (index (m+1) 2^24 + 1.., half-width 3a about the Snell-chained
    intercepts); field points on the refracted beam axis 1-20 mm below the last plane and
    across it 10 mm below.  The field at N samples per surface against N_ref; the same for
    one plane (water over the steel half-space) for contrast."""
    radius: float = PISTON_RADIUS
    freq: float = 2.5e6
    tilt: float = deg(10.0)
    water_path: float = 0.010
    layer: float = 0.002
    counts: Tuple[int, ...] = (10000, 30000, 100000, 300000, 1000000)
    n_ref: int = 2000000
    n_line: int = 41
    media: Tuple[Tuple[float, float], ...] = (WATER, STEEL_PAPER, ALU_PAPER, STEEL_PAPER, ALU_PAPER,
                                              STEEL_PAPER, ALU_PAPER, STEEL_PAPER)
    one_plane: Tuple[Tuple[float, float], ...] = (WATER, STEEL_PAPER)

    @property
    def half_width(self) -> float:
        return 3.0 * self.radius

    @property
    def axis(self):
        return (math.sin(self.tilt), 0.0, math.cos(self.tilt))

    def planes(self, media) -> List[float]:
        return [self.water_path + m * self.layer for m in range(len(media) - 1)]

    def patch_centres(self, media) -> List[float]:
        return snell_intercepts(0.0, self.tilt, self.planes(media), [m[0] for m in media])

    def field(self, media):
        zs = self.planes(media)
        s = min(math.sin(self.tilt) / media[0][0] * media[-1][0], 0.999999)
        t = s / math.sqrt(1 - s * s)
        x_top = self.patch_centres(media)[-1]
        d = np.linspace(0.001, 0.020, self.n_line)
        xa, za = x_top + d * t, zs[-1] + d
        xc = x_top + 0.010 * t + np.linspace(-0.008, 0.008, self.n_line)
        zc = np.full(self.n_line, zs[-1] + 0.010)
        x = np.concatenate([xa, xc])
        return x, np.zeros_like(x), np.concatenate([za, zc])


@dataclass
class LayeredStack:
    """Three interfaces 2 mm apart; 64 frequencies 1-10 MHz; 128^3 volume below."""
    radius: float = PISTON_RADIUS
    tilt: float = deg(10.0)
    n_xd: int = 1 << 16
    xd_seed: int = 0
    z_if: Tuple[float, ...] = (0.050, 0.052, 0.054)
    n_if: int = 1 << 18
    if_seeds: Tuple[int, ...] = (1, 2, 3)
    half_width: float = 0.03
    media: Tuple[Tuple[float, float], ...] = (WATER, STEEL_5900, MID_2700, STEEL_5900)
    n_freq: int = 64
    f0: float = 1.0e6
    f1: float = 10.0e6
    nvol: int = 128
    depth0: float = 1.0e-3
    depth1: float = 31.0e-3
    half_xy: float = 0.015

    @property
    def freqs(self) -> np.ndarray:
        return self.f0 + (self.f1 - self.f0) * np.arange(self.n_freq) / (self.n_freq - 1)

    @property
    def patch_centres(self) -> List[Tuple[float, float]]:
        xs = snell_intercepts(0.0, self.tilt, self.z_if, [m[0] for m in self.media])
        return [(x, 0.0) for x in xs]

    @property
    def axis(self):
        return (math.sin(self.tilt), 0.0, math.cos(self.tilt))

    def volume_centre_x(self) -> float:
        # beam axis at mid-depth of the volume, in the last medium
        x3 = self.patch_centres[-1][0]
        C = math.sin(self.tilt) / self.media[0][0]
        s = min(C * self.media[-1][0], 0.999999)
        mid = 0.5 * (self.depth0 + self.depth1)
        return x3 + mid * s / math.sqrt(1 - s * s)

    def targets(self, n=None):
        n = n or self.nvol
        xc = self.volume_centre_x()
        x = np.linspace(xc - self.half_xy, xc + self.half_xy, n)
        y = np.linspace(-self.half_xy, self.half_xy, n)
        z = self.z_if[-1] + np.linspace(self.depth0, self.depth1, n)
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()


@dataclass
class ScanInstance:
    index: int
    x_offset: float
    tilt: float
    n_src: int
    n_fld: int
    seed: int


@dataclass
class ScanBatch:
    """256 scan positions of the piston in water at 1 MHz, uneven sizes (seeded)."""
    n_inst: int = 256
    radius: float = PISTON_RADIUS
    freq: float = 1.0e6
    medium: Tuple[float, float] = WATER
    seed: int = 0

    def instances(self) -> List[ScanInstance]:
        rng = np.random.default_rng(self.seed)
        off = rng.uniform(-0.020, 0.020, self.n_inst)
        tilt = rng.uniform(0.0, deg(20.0), self.n_inst)
        nsrc = np.rint(2.0 ** rng.uniform(12.0, 18.0, self.n_inst)).astype(np.int64)
        nfld = np.rint(10.0 ** rng.uniform(3.0, 5.0, self.n_inst)).astype(np.int64)
        return [ScanInstance(i, float(off[i]), float(tilt[i]), int(nsrc[i]), int(nfld[i]), i)
                for i in range(self.n_inst)]

    def field_points(self, inst: ScanInstance):
        rng = np.random.default_rng([self.seed, inst.index])
        x = inst.x_offset + rng.uniform(-0.020, 0.020, inst.n_fld)
        y = rng.uniform(-0.010, 0.010, inst.n_fld)
        z = rng.uniform(0.001, 0.100, inst.n_fld)
        return x, y, z

    def pairs(self) -> int:
        return int(sum(i.n_src * i.n_fld for i in self.instances()))


@dataclass
class SurrogateBox:
    """Parameter box of the learned surrogate (piston + one interface)."""
    radius: float = PISTON_RADIUS
    media: Tuple[Tuple[float, float], ...] = (WATER, STEEL_5900)
    f_range: Tuple[float, float] = (1.0e6, 10.0e6)
    depth_range: Tuple[float, float] = (0.030, 0.070)
    tilt_range: Tuple[float, float] = (0.0, deg(20.0))
    x_range: Tuple[float, float] = (-0.010, 0.030)
    z_below: Tuple[float, float] = (0.002, 0.030)


# --------------------------------------------------------------------------- generic
def random_cloud(seed: int, n: int, centre=(0.0, 0.0, 0.0), half=(0.01, 0.01, 0.01)):
    """Uniform random points in a box (for parity cases that need no geometry)."""
    rng = np.random.default_rng(seed)
    return tuple(centre[k] + rng.uniform(-half[k], half[k], n) for k in range(3))


def random_complex(seed: int, n: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(n) + 1j * rng.standard_normal(n))


def random_weights(seed: int, n: int, total: float = 1e-4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, n)
    return w * (total / w.sum())
