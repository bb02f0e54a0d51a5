"""Seeded synthetic inputs: source models, phantoms, beams, measurement maps.

This module only *generates inputs*.  It holds none of the method's arithmetic
(no PSR->PSL conversion, no sampling, no transport, no tally), so that both the
GPU engine and the CPU oracle can be fed the very same arrays.  All randomness
comes from numpy's PCG64 seeded by ``(seed, tag)``; the method's own random
numbers are drawn by each side from its own Philox4x32-10 generator.

Geometry convention (cm, MeV, g/cm^3):
  * beam frame: the focal spot (target) is at z = -100, the PSR/PSL plane at
    z = 0, which is also the isocentre plane (SAD = 100 cm); particles travel
    towards +z.  The extra-focal scatter source sits at z = -90.  The upper
    surfaces of the Y and X jaws are at z = -72 and z = -63.
  * patient frame: at gantry 0 / couch 0 it coincides with the beam frame
    translated to the isocentre; the gantry turns about +y, the couch about +z.
  * phantoms are dense float32 arrays indexed [iz][iy][ix] (x fastest).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Sub-stream tags for numpy seeding of the input generators.
TAG_MODEL = 11
TAG_PHANTOM = 12
TAG_BEAMS = 13
TAG_TARGET = 14

MODEL_GEOMETRY = dict(z_target=-100.0, z_plane=0.0, z_scatter=-90.0,
                      z_jaw_y=-72.0, z_jaw_x=-63.0)


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(tag)]))


@dataclass
class PsrModel:
    """A phase-space-ring source model: 3 sub-sources x n_ebin x n_ring PSRs.

    Sub-source order is (primary photon, scatter photon, electron).
    """
    n_ebin: int
    n_ring: int
    n_comp: int
    n_psl: int
    e_lo: float
    e_width: float
    ring_dr: float
    psl_x0: float
    psl_dx: float
    z_target: float
    z_plane: float
    z_scatter: float
    z_jaw_y: float
    z_jaw_x: float
    sigma_spot: float
    sig_ea: float
    sig_eb: float
    w_psr: np.ndarray          # [3][n_ebin][n_ring] float64
    sc_c: np.ndarray           # [n_ebin][n_ring][K] float64 mixture weights
    sc_mu: np.ndarray          # [n_ebin][n_ring][K] alpha means (rad)
    sc_sa: np.ndarray          # [n_ebin][n_ring][K] alpha sigmas (rad)
    sc_sb: np.ndarray          # [n_ebin][n_ring][K] beta sigmas (rad)

    @property
    def e_max(self) -> float:
        return self.e_lo + self.n_ebin * self.e_width


def triangle_spectrum(e: np.ndarray, e_max: float = 6.0, mode: float = 1.0) -> np.ndarray:
    """Triangular 6 MV-like spectral shape on [0, e_max] peaking at ``mode``."""
    e = np.asarray(e, dtype=np.float64)
    up = e / mode
    down = (e_max - e) / (e_max - mode)
    return np.clip(np.where(e <= mode, up, down), 0.0, None)


def psr_model(seed: int = 1, *, noise: bool = True, simple_scatter: bool = False,
              n_ebin: int = 24, n_ring: int = 30, e_lo: float = 0.25, e_hi: float = 6.0,
              ring_dr: float = 0.5, n_psl: int = 60, psl_dx: float = 0.5,
              sigma_spot: float = 0.1, scatter_sigma_cm: float = 1.5,
              sub_fraction=(0.90, 0.09, 0.01), sig_e: float = 0.05) -> PsrModel:
    """Synthetic 6 MV-like PSR model.

    PSR weight: W[s,b,j] = f_s * T(E_b) * (ring area 2 pi r_j dr) * U[0.5,1.5]
    (``noise=False`` sets U = 1).  The ring-area factor makes the fluence per
    unit area independent of r before the random factor.

    Scatter direction mixture (K = 3 Gaussians in alpha/beta): mean alpha
    points back to the scatter source on the axis, widths are multiples of the
    angle a 1.5 cm Gaussian source subtends from the plane.  Unless
    ``simple_scatter`` is set, every (bin, ring, component) parameter carries an
    independent seeded perturbation so that indexing mistakes are visible.
    """
    rng = _rng(seed, TAG_MODEL)
    e_width = (e_hi - e_lo) / n_ebin
    e_mid = e_lo + (np.arange(n_ebin) + 0.5) * e_width
    r_mid = (np.arange(n_ring) + 0.5) * ring_dr
    ring_area = 2.0 * math.pi * r_mid * ring_dr
    spec = triangle_spectrum(e_mid)
    f = np.asarray(sub_fraction, dtype=np.float64)
    w = f[:, None, None] * spec[None, :, None] * ring_area[None, None, :]
    if noise:
        w = w * rng.uniform(0.5, 1.5, size=w.shape)
    K = 3
    dz = MODEL_GEOMETRY["z_plane"] - MODEL_GEOMETRY["z_scatter"]
    base_c = np.array([0.6, 0.3, 0.1])
    mult = np.array([1.0, 1.5, 2.0])
    s0 = math.atan(scatter_sigma_cm / dz)
    mu = np.broadcast_to(np.arctan(r_mid / dz)[None, :, None], (n_ebin, n_ring, K)).copy()
    sa = np.broadcast_to((mult * s0)[None, None, :], (n_ebin, n_ring, K)).copy()
    sb = sa.copy()
    c = np.broadcast_to(base_c[None, None, :], (n_ebin, n_ring, K)).copy()
    if not simple_scatter:
        c = c * rng.uniform(0.8, 1.2, size=c.shape)
        mu = mu * rng.uniform(0.9, 1.1, size=mu.shape)
        sa = sa * rng.uniform(0.9, 1.1, size=sa.shape)
        sb = sb * rng.uniform(0.9, 1.1, size=sb.shape)
    half = n_psl * psl_dx / 2.0
    return PsrModel(n_ebin=n_ebin, n_ring=n_ring, n_comp=K, n_psl=n_psl, e_lo=e_lo,
                    e_width=e_width, ring_dr=ring_dr, psl_x0=-half, psl_dx=psl_dx,
                    sigma_spot=sigma_spot, sig_ea=sig_e, sig_eb=sig_e,
                    w_psr=np.ascontiguousarray(w, dtype=np.float64),
                    sc_c=np.ascontiguousarray(c), sc_mu=np.ascontiguousarray(mu),
                    sc_sa=np.ascontiguousarray(sa), sc_sb=np.ascontiguousarray(sb),
                    **MODEL_GEOMETRY)


@dataclass
class Beam:
    x1: float
    x2: float
    y1: float
    y2: float
    gantry_deg: float = 0.0
    couch_deg: float = 0.0
    iso: tuple = (0.0, 0.0, 0.0)


def square_beam(size_cm: float, gantry_deg: float = 0.0, iso=(0.0, 0.0, 0.0)) -> Beam:
    h = size_cm / 2.0
    return Beam(-h, h, -h, h, gantry_deg, 0.0, tuple(float(v) for v in iso))


@dataclass
class Phantom:
    density: np.ndarray        # [nz][ny][nx] float32
    vox: tuple                 # (dx, dy, dz) cm
    origin: tuple              # corner of voxel (0,0,0), cm

    @property
    def shape_xyz(self):
        nz, ny, nx = self.density.shape
        return nx, ny, nz


def water_phantom(n: int, vox: float, rho: float = 1.0) -> Phantom:
    """Water cube whose top face (z = 0) holds the isocentre at its centre (SSD 100)."""
    half = n * vox / 2.0
    dens = np.full((n, n, n), rho, dtype=np.float32)
    return Phantom(dens, (vox, vox, vox), (-half, -half, 0.0))


def water_box(nx: int, ny: int, nz: int, vox, rho: float = 1.0) -> Phantom:
    """Water box of nx x ny x nz voxels of size vox = (dx, dy, dz) cm, top face
    at z = 0 with the isocentre at its centre (SSD 100)."""
    vox = tuple(float(v) for v in vox)
    dens = np.full((nz, ny, nx), rho, dtype=np.float32)
    return Phantom(dens, vox, (-nx * vox[0] / 2.0, -ny * vox[1] / 2.0, 0.0))


def slab_phantom(n_xy: int, vox_xy: float, slabs, vox_z: float) -> Phantom:
    """Laterally uniform slabs stacked along z: ``slabs`` = [(n_vox_z, rho), ...]."""
    nz = sum(n for n, _ in slabs)
    dens = np.empty((nz, n_xy, n_xy), dtype=np.float32)
    k = 0
    for n, rho in slabs:
        dens[k:k + n] = rho
        k += n
    half = n_xy * vox_xy / 2.0
    return Phantom(dens, (vox_xy, vox_xy, vox_z), (-half, -half, 0.0))


def hetero_phantom(seed: int, nx: int = 256, ny: int = 128, nz: int = 256,
                   vox: float = 0.2) -> Phantom:
    """Water box centred on the isocentre with lung (0.26) and bone (1.85) ellipsoids.

    x and z are the transverse axes, y is the longitudinal (gantry) axis.
    Counts: 2-4 lung and 1-3 bone ellipsoids; centres uniform in the central
    80% of the box; semi-axes U[2,8] cm (lung) and U[0.5,2] cm (bone); bone is
    painted last; membership is tested at voxel centres.
    """
    rng = _rng(seed, TAG_PHANTOM)
    ext = np.array([nx, ny, nz], dtype=np.float64) * vox
    origin = -ext / 2.0
    dens = np.ones((nz, ny, nx), dtype=np.float32)
    xc = origin[0] + (np.arange(nx) + 0.5) * vox
    yc = origin[1] + (np.arange(ny) + 0.5) * vox
    zc = origin[2] + (np.arange(nz) + 0.5) * vox
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    n_lung = int(rng.integers(2, 5))
    n_bone = int(rng.integers(1, 4))
    for rho, n, (a_lo, a_hi) in ((0.26, n_lung, (2.0, 8.0)), (1.85, n_bone, (0.5, 2.0))):
        for _ in range(n):
            c = rng.uniform(-0.4 * ext, 0.4 * ext)
            a = rng.uniform(a_lo, a_hi, size=3)
            inside = (((X - c[0]) / a[0]) ** 2 + ((Y - c[1]) / a[1]) ** 2
                      + ((Z - c[2]) / a[2]) ** 2) <= 1.0
            dens[inside] = rho
    return Phantom(dens, (vox, vox, vox), tuple(float(v) for v in origin))


def hetero_beams(seed: int, n_beams: int = 5) -> list:
    """Coplanar fields at 360/n spacing with jaw sizes Fx, Fy ~ U[3, 15] cm."""
    rng = _rng(seed, TAG_BEAMS)
    beams = []
    for i in range(n_beams):
        fx, fy = rng.uniform(3.0, 15.0, size=2)
        beams.append(Beam(-fx / 2, fx / 2, -fy / 2, fy / 2, 360.0 * i / n_beams, 0.0,
                          (0.0, 0.0, 0.0)))
    return beams


def _grid(nx, ny, nz, vox):
    ext = np.array([nx, ny, nz], dtype=np.float64) * np.asarray(vox, dtype=np.float64)
    origin = -ext / 2.0
    xc = origin[0] + (np.arange(nx) + 0.5) * vox[0]
    yc = origin[1] + (np.arange(ny) + 0.5) * vox[1]
    zc = origin[2] + (np.arange(nz) + 0.5) * vox[2]
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    return X, Y, Z, origin


def head_phantom(seed: int, nx: int = 160, ny: int = 176, nz: int = 160,
                 vox=(0.137, 0.125, 0.137)) -> Phantom:
    """Head-and-neck-like phantom on the paper's H&N voxel size (0.137 cm
    transverse, 0.125 cm along the patient axis y), centred on the isocentre:
    an ellipsoidal head of soft tissue (1.04) in air (0.0012) with a 0.6 cm
    skull shell (1.85), two air sinuses and a cervical spine column (1.6);
    sizes jittered from the seed."""
    rng = _rng(seed, TAG_PHANTOM + 100)
    X, Y, Z, origin = _grid(nx, ny, nz, vox)
    a = np.array([8.0, 10.0, 9.5]) * rng.uniform(0.95, 1.05, 3)       # semi-axes x, y, z
    r = (X / a[0]) ** 2 + (Y / a[1]) ** 2 + (Z / a[2]) ** 2
    dens = np.full(X.shape, 0.0012, dtype=np.float32)
    dens[r <= 1.0] = 1.04
    ai = a - 0.6
    ri = (X / ai[0]) ** 2 + (Y / ai[1]) ** 2 + (Z / ai[2]) ** 2
    dens[(r <= 1.0) & (ri > 1.0) & (Y > -3.0)] = 1.85                 # skull above the neck
    for sx in (-1.0, 1.0):
        c = np.array([sx * 2.0, 3.0, -4.5]) + rng.uniform(-0.5, 0.5, 3)
        dens[((X - c[0]) / 1.5) ** 2 + ((Y - c[1]) / 1.8) ** 2 + ((Z - c[2]) / 1.5) ** 2 <= 1.0] = 0.0012
    dens[(X ** 2 + (Z - 4.0) ** 2 <= 1.2 ** 2) & (Y < 2.0)] = 1.6       # spine column
    return Phantom(dens, tuple(float(v) for v in vox), tuple(float(v) for v in origin))


def hn_beams(seed: int) -> list:
    """Five coplanar fields at 72 degree spacing and one non-coplanar field
    at couch 90 (the paper's H&N plan shape), jaws U[4, 8] cm."""
    rng = _rng(seed, TAG_BEAMS + 100)
    beams = []
    for i in range(5):
        fx, fy = rng.uniform(4.0, 8.0, size=2)
        beams.append(Beam(-fx / 2, fx / 2, -fy / 2, fy / 2, 72.0 * i, 0.0, (0.0, 0.0, 0.0)))
    fx, fy = rng.uniform(4.0, 8.0, size=2)
    beams.append(Beam(-fx / 2, fx / 2, -fy / 2, fy / 2, 40.0, 90.0, (0.0, 0.0, 0.0)))
    return beams


def pelvis_phantom(seed: int, nx: int = 200, ny: int = 96, nz: int = 128,
                   vox=(0.195, 0.25, 0.195)) -> Phantom:
    """Pelvis-like phantom on the paper's prostate voxel size (0.195 cm
    transverse, 0.25 cm along y): an elliptic body cylinder of soft tissue
    (1.02) in air, two femoral heads and a sacrum of bone (1.85), a rectal gas
    pocket (0.0012); sizes jittered from the seed."""
    rng = _rng(seed, TAG_PHANTOM + 200)
    X, Y, Z, origin = _grid(nx, ny, nz, vox)
    ax, az = 18.0 * rng.uniform(0.95, 1.05), 11.5 * rng.uniform(0.95, 1.05)
    dens = np.full(X.shape, 0.0012, dtype=np.float32)
    dens[(X / ax) ** 2 + (Z / az) ** 2 <= 1.0] = 1.02
    for sx in (-1.0, 1.0):
        c = np.array([sx * 8.5, 0.0, 0.5]) + rng.uniform(-0.5, 0.5, 3)
        dens[((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) <= 2.4 ** 2] = 1.85
    dens[((X / 4.0) ** 2 + ((Z - 7.5) / 1.6) ** 2 <= 1.0)] = 1.85      # sacrum
    c = np.array([0.0, 0.0, 4.2]) + rng.uniform(-0.3, 0.3, 3)
    dens[((X - c[0]) ** 2 + (Y - c[1]) ** 2 / 4.0 + (Z - c[2]) ** 2) <= 0.8 ** 2] = 0.0012
    return Phantom(dens, tuple(float(v) for v in vox), tuple(float(v) for v in origin))


def prostate_beams(seed: int) -> list:
    """Seven coplanar fields at 360/7 spacing (the paper's prostate plan
    shape), jaws U[7, 10] cm."""
    rng = _rng(seed, TAG_BEAMS + 200)
    beams = []
    for i in range(7):
        fx, fy = rng.uniform(7.0, 10.0, size=2)
        beams.append(Beam(-fx / 2, fx / 2, -fy / 2, fy / 2, 360.0 * i / 7, 0.0, (0.0, 0.0, 0.0)))
    return beams


def commissioning_basis_map(model: PsrModel, rings_per_group: int = 3) -> np.ndarray:
    """Basis id per PSR: s * (n_ebin * groups) + b * groups + ring // rings_per_group."""
    groups = (model.n_ring + rings_per_group - 1) // rings_per_group
    s = np.arange(3)[:, None, None]
    b = np.arange(model.n_ebin)[None, :, None]
    j = np.arange(model.n_ring)[None, None, :]
    m = s * (model.n_ebin * groups) + b * groups + j // rings_per_group
    return np.ascontiguousarray(m, dtype=np.uint16)


def commissioning_index_map(n: int, vox: float, depths_cm=(1.5, 10.0, 20.0)):
    """Voxel -> row+1 map (0 = not measured) for a CAX depth dose plus inline and
    crossline profiles at the given depths, on an n^3 water cube.

    The central column is (n/2, n/2); rows are numbered in [iz][iy][ix] raster
    order of the selected voxels.
    """
    c = n // 2
    sel = np.zeros((n, n, n), dtype=bool)
    sel[:, c, c] = True
    for d in depths_cm:
        k = int(math.floor(d / vox))
        sel[k, :, c] = True       # inline profile (along y)
        sel[k, c, :] = True       # crossline profile (along x)
    imap = np.zeros((n, n, n), dtype=np.int32)
    idx = np.flatnonzero(sel.ravel())
    imap.ravel()[idx] = np.arange(1, idx.size + 1, dtype=np.int32)
    return imap, int(idx.size)


def commissioning_target(a: np.ndarray, seed: int, noise_rel: float = 0.005):
    """Seeded true weights x ~ U[0.8,1.2] and b = (A x)(1 + noise_rel * N(0,1))."""
    rng = _rng(seed, TAG_TARGET)
    x_true = rng.uniform(0.8, 1.2, size=a.shape[1])
    b = (a @ x_true) * (1.0 + noise_rel * rng.standard_normal(a.shape[0]))
    return x_true, b


@dataclass
class Workload:
    name: str
    model: PsrModel
    phantom: Phantom
    beams: list
    n_hist: int
    n_replica: int
    seed: int
    e_cut_electron: float = 0.2
    e_cut_photon: float = 0.01
    extra: dict = field(default_factory=dict)


def workload(name: str, seed: int = 20150306) -> Workload:
    """Named synthetic workloads.

    * ``water60_10x10``: 60^3 water at 0.5 cm, one 10x10 field, 1e5 histories.
    * ``water128_{5,10,20}``: 128^3 water at 0.25 cm, one square field, 1e8 histories.
    * ``hetero256_5beam``: 256x128x256 heterogeneous phantom at 0.2 cm, 5 coplanar
      fields of random jaw sizes, 2e8 histories over all beams.
    * ``hn_6beam``: head-and-neck-like phantom at 0.137 x 0.125 x 0.137 cm,
      five coplanar fields and one at couch 90, 2e8 histories over all beams.
    * ``prostate_7beam``: pelvis-like phantom at 0.195 x 0.25 x 0.195 cm,
      seven coplanar fields, 2e8 histories over all beams.
    * ``water240_table1``: the water phantom shape of the paper's efficiency
      test (Table 1): 240 x 240 x 300 voxels of 0.25 x 0.25 x 0.2 cm (60 cm
      cube), one 10x10 field, 1e8 histories.
    * ``commission60``: 60^3 water, fields 3/6/10/20 cm, 720 basis doses, 1e6
      histories per basis and field.
    """
    model = psr_model(seed)
    if name == "water60_10x10":
        return Workload(name, model, water_phantom(60, 0.5), [square_beam(10.0)],
                        10 ** 5, 10, seed)
    if name.startswith("water128_"):
        size = float(name.split("_")[1])
        return Workload(name, model, water_phantom(128, 0.25), [square_beam(size)],
                        10 ** 8, 10, seed)
    if name == "water240_table1":
        return Workload(name, model, water_box(240, 240, 300, (0.25, 0.25, 0.2)),
                        [square_beam(10.0)], 10 ** 8, 10, seed)
    if name == "hetero256_5beam":
        return Workload(name, model, hetero_phantom(seed), hetero_beams(seed),
                        2 * 10 ** 8, 10, seed)
    if name == "hn_6beam":
        return Workload(name, model, head_phantom(seed), hn_beams(seed), 2 * 10 ** 8, 10, seed)
    if name == "prostate_7beam":
        return Workload(name, model, pelvis_phantom(seed), prostate_beams(seed), 2 * 10 ** 8, 10,
                        seed)
    if name == "commission60":
        imap, n_rows = commissioning_index_map(60, 0.5)
        beams = [square_beam(s) for s in (3.0, 6.0, 10.0, 20.0)]
        return Workload(name, model, water_phantom(60, 0.5), beams, 0, 1, seed,
                        extra=dict(index_map=imap, n_rows=n_rows,
                                   basis_map=commissioning_basis_map(model),
                                   n_basis=720, hist_per_basis=10 ** 6))
    raise KeyError(name)
