"""Seeded synthetic workloads for polarised A x W gridding.

This module is shared by the FP64 oracle (tests) and the HIP path (bench).
It only builds inputs: array layouts, Earth-rotation uvw tracks, source
lists, the beam/leakage (Jones) model, w-plane placement and the per-plane
support table.  None of the gridding, kernel-generation or imaging
arithmetic lives here.

The paper measured on ASKAP and ALMA measurement sets (Sec. 2.1, Sec. 2.3);
none ships with it, so every workload here is synthetic, with the sizes of
the five configurations the library is built for:

  c1  Stokes-I, 256^2 grid, 8 w-planes, support 7, os 4, 20k visibilities
  c2  full-pol A+W, 2048^2 x 4, 32 w-planes, support 16-48, os 8, 2.3M rows
  c3  batched, 16 fields on their own 4096^2 x 4 grids, FP16 tables
  c4  learned kernel surrogate (training draws)
  c5  major cycle, 8192^2 x 4, 128 w-planes, 20M rows
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2206151170
C_LIGHT = 299792458.0
DEG = math.pi / 180.0
ARCSEC = DEG / 3600.0
SIDEREAL_RATE = 2.0 * math.pi / 86164.0905  # rad/s


@dataclass
class Geometry:
    """Grid, oversampling and w-plane layout shared by every stage.

    n          grid side (even; image and uv grids are n x n)
    cell       image pixel size in radians (the uv cell is 1/(n*cell) wavelengths)
    os         oversampling factor of the kernel table (even)
    w_planes   float64 [P], ascending w-plane centres in wavelengths
    support    int32 [P], kernel support (taps per axis) of each plane
    tile       int32 [P], uv tile side used to bin visibilities of each plane
    aa_support support of the prolate-spheroidal anti-aliasing function
    mk         samples per side of the image-domain lattice kernels are built on
    """

    n: int
    cell: float
    os: int
    w_planes: np.ndarray
    support: np.ndarray
    tile: np.ndarray = None
    aa_support: int = 7
    mk: int = 0

    def __post_init__(self):
        self.w_planes = np.ascontiguousarray(self.w_planes, dtype=np.float64)
        self.support = np.ascontiguousarray(self.support, dtype=np.int32)
        if self.tile is None:
            self.tile = default_tiles(self.support, 4)
        self.tile = np.ascontiguousarray(self.tile, dtype=np.int32)
        if self.mk == 0:
            self.mk = self.n

    @property
    def fov(self) -> float:
        return self.n * self.cell

    @property
    def nplanes(self) -> int:
        return int(self.w_planes.shape[0])


def lds_pitch(width: int, support: int) -> int:
    """Row pitch of a sub-grid in LDS: >= width and congruent to the support modulo 32."""
    return width + (support - width) % 32


def default_tiles(support, q, lds_bytes=163840 - 1280):
    """Largest tile T per plane whose (T+S-1) x pitch x q complex64 sub-grid fits lds_bytes."""
    out = []
    for s in np.asarray(support):
        s = int(s)
        t = 1
        while t < 256:
            w = t + 1 + s - 1
            if w * lds_pitch(w, s) * q * 8 > lds_bytes:
                break
            t += 1
        out.append(t)
    return np.asarray(out, dtype=np.int32)


def linear_w_planes(nplanes: int, w_max: float) -> np.ndarray:
    """Signed, symmetric, evenly spaced w-plane centres in [-w_max, w_max]."""
    if nplanes == 1:
        return np.zeros(1)
    return np.array([-w_max + p * 2.0 * w_max / (nplanes - 1) for p in range(nplanes)])


def support_rule(w_planes, fov, s_min=16, s_max=48):
    """Per-plane support: 7 anti-aliasing taps plus the w-chirp spread, rounded up to even."""
    s = [2 * math.ceil((7 + 0.8 * abs(w) * fov * fov) / 2.0) for w in w_planes]
    return np.clip(np.asarray(s, dtype=np.int32), s_min, s_max).astype(np.int32)


# --------------------------------------------------------------------------- arrays and tracks

def antennas_in_disk(n_ant: int, radius_m: float, rng) -> np.ndarray:
    """ENU positions (metres, flat, up = 0) uniform in a disk."""
    r = radius_m * np.sqrt(rng.uniform(0.0, 1.0, n_ant))
    t = rng.uniform(0.0, 2.0 * math.pi, n_ant)
    return np.stack([r * np.cos(t), r * np.sin(t), np.zeros(n_ant)], axis=1)


def baseline_pairs(n_ant: int) -> np.ndarray:
    return np.array([(i, j) for i in range(n_ant) for j in range(i + 1, n_ant)], dtype=np.int32)


def uvw_tracks(enu, lat, dec, hour_angles, freq_hz) -> np.ndarray:
    """Textbook (H, dec) rotation of ENU baselines into uvw, in wavelengths.

    Rows are time-major (all baselines of dump 0, then dump 1, ...), the order of
    a measurement set.  Returns float64 [n_dumps * n_baselines, 3].
    """
    pairs = baseline_pairs(enu.shape[0])
    b = enu[pairs[:, 1]] - enu[pairs[:, 0]]
    e, nn, up = b[:, 0], b[:, 1], b[:, 2]
    x = -math.sin(lat) * nn + math.cos(lat) * up
    y = e
    z = math.cos(lat) * nn + math.sin(lat) * up
    h = np.asarray(hour_angles)[:, None]
    sd, cd = math.sin(dec), math.cos(dec)
    u = np.sin(h) * x + np.cos(h) * y
    v = -sd * np.cos(h) * x + sd * np.sin(h) * y + cd * z
    w = cd * np.cos(h) * x - cd * np.sin(h) * y + sd * z
    lam = C_LIGHT / freq_hz
    return np.stack([u, v, w], axis=-1).reshape(-1, 3) / lam


# --------------------------------------------------------------------------- beam / leakage model

@dataclass
class GaussianLeakageBeam:
    """Identical-antenna Jones model J = E(r) [[1, d_xy], [d_yx, 1]].

    E is the voltage pattern exp(-2 ln2 (r/theta)^2), so the power beam E^2 has
    FWHM theta.  d = level * (a + b l/theta + c m/theta) with seeded complex a, b, c.
    """

    theta: float
    dxy: np.ndarray = field(default_factory=lambda: np.zeros(3, complex))
    dyx: np.ndarray = field(default_factory=lambda: np.zeros(3, complex))
    level: float = 0.01

    def jones(self, l, m) -> np.ndarray:
        l = np.asarray(l, dtype=np.float64)
        m = np.asarray(m, dtype=np.float64)
        r2 = l * l + m * m
        e = np.exp(-2.0 * math.log(2.0) * r2 / (self.theta * self.theta))
        dxy = self.level * (self.dxy[0] + self.dxy[1] * l / self.theta + self.dxy[2] * m / self.theta)
        dyx = self.level * (self.dyx[0] + self.dyx[1] * l / self.theta + self.dyx[2] * m / self.theta)
        j = np.empty(l.shape + (2, 2), dtype=np.complex128)
        j[..., 0, 0] = e
        j[..., 0, 1] = e * dxy
        j[..., 1, 0] = e * dyx
        j[..., 1, 1] = e
        return j


@dataclass
class OffsetBeam:
    """A beam model centred on a mosaic pointing at (l0, m0) of the common frame: the Jones matrix
    and the power beam E^2 at (l, m) are those of `base` at (l - l0, m - m0)."""

    base: GaussianLeakageBeam
    l0: float
    m0: float

    def jones(self, l, m) -> np.ndarray:
        return self.base.jones(np.asarray(l) - self.l0, np.asarray(m) - self.m0)

    def power(self, l, m) -> np.ndarray:
        return np.abs(self.jones(l, m)[..., 0, 0]) ** 2


def antenna_types(theta: float, k: int, rng, pointing_sigma: float, level: float = 0.01) -> list:
    """k antenna types: the Gaussian beam of power FWHM theta, each type with its own seeded leakage
    pattern and a pointing error drawn N(0, pointing_sigma) per axis (radians)."""
    out = []
    for _ in range(k):
        b = seeded_leakage_beam(theta, rng, level=level)
        out.append(OffsetBeam(b, float(rng.normal(0.0, pointing_sigma)), float(rng.normal(0.0, pointing_sigma))))
    return out


def baseline_type_pairs(n_rows: int, n_ant: int, k: int) -> np.ndarray:
    """Ordered antenna-type pair index (type_a k + type_b) of every row of time-major tracks
    (row r is baseline r mod n_baselines), antenna i being of type i mod k."""
    pairs = baseline_pairs(n_ant)
    bl = pairs[np.arange(n_rows) % pairs.shape[0]]
    return (bl[:, 0] % k) * k + (bl[:, 1] % k)


def power_on_pixels(beam, n: int, cell: float) -> np.ndarray:
    """float64 [n (m, rows)][n (l, columns)] power beam at the image pixel centres."""
    x = (np.arange(n) - n // 2) * cell
    mm, ll = np.meshgrid(x, x, indexing="ij")
    return beam.power(ll, mm)


def seeded_leakage_beam(theta, rng, level=0.01) -> GaussianLeakageBeam:
    def cn(k):
        return (rng.standard_normal(k) + 1j * rng.standard_normal(k)) / math.sqrt(2.0)

    return GaussianLeakageBeam(theta=theta, dxy=cn(3), dyx=cn(3), level=level)


def lattice_coords(mk: int, fov: float) -> np.ndarray:
    """Image-domain lattice the kernels are sampled on: (a - mk/2) * fov / mk."""
    return (np.arange(mk) - mk // 2) * (fov / mk)


def jones_on_lattice(beam, mk: int, fov: float) -> np.ndarray:
    """complex128 [2][2][mk (m, rows)][mk (l, columns)], the layout make_kernels takes."""
    x = lattice_coords(mk, fov)
    mm, ll = np.meshgrid(x, x, indexing="ij")
    j = beam.jones(ll, mm)  # [mk][mk][2][2]
    return np.ascontiguousarray(np.moveaxis(j, (2, 3), (0, 1)))


# --------------------------------------------------------------------------- sources and values

def random_vis(nvis: int, npol: int, rng) -> np.ndarray:
    """complex64 [nvis][npol], unit-variance complex normal."""
    v = (rng.standard_normal((nvis, npol)) + 1j * rng.standard_normal((nvis, npol))) / math.sqrt(2)
    return v.astype(np.complex64)


@dataclass
class Workload:
    name: str
    geom: Geometry
    uvw: np.ndarray                  # float64 [nvis][3], wavelengths
    npol: int                        # 1 (Stokes I) or 4 (XX, XY, YX, YY in, I, Q, U, V out)
    src_l: np.ndarray = None
    src_m: np.ndarray = None
    src_iquv: np.ndarray = None      # [nsrc][npol]
    beam: GaussianLeakageBeam = None
    eps_null: float = 0.2
    extra: dict = field(default_factory=dict)

    @property
    def nvis(self):
        return int(self.uvw.shape[0])


def config1(seed: int = SEED_BASE + 1, nvis: int = 20000) -> Workload:
    """Stokes-I, 256^2 grid, 8 planes |w| <= 200, PSWF support 7, os 4, no A-term."""
    rng = np.random.default_rng(seed)
    n = 256
    cell = 0.1 / n
    planes = linear_w_planes(8, 200.0)
    geom = Geometry(n=n, cell=cell, os=4, w_planes=planes, support=np.full(8, 7, np.int32),
                    tile=np.full(8, 16, np.int32), aa_support=7, mk=n)
    r = 100.0 * np.sqrt(rng.uniform(0, 1, nvis))
    t = rng.uniform(0, 2 * math.pi, nvis)
    w = rng.uniform(-200.0, 200.0, nvis)
    uvw = np.stack([r * np.cos(t), r * np.sin(t), w], axis=1)
    half = 0.25 * geom.fov
    sl = rng.uniform(-half, half, 5)
    sm = rng.uniform(-half, half, 5)
    flux = rng.uniform(0.1, 1.0, 5)
    return Workload("c1-stokesI-256", geom, uvw, 1, sl, sm, flux[:, None])


ASKAP_LAT = -26.7 * DEG


def polarised_sources(nsrc, r_max, rng):
    r = r_max * np.sqrt(rng.uniform(0, 1, nsrc))
    t = rng.uniform(0, 2 * math.pi, nsrc)
    i = rng.uniform(0.1, 1.0, nsrc)
    p = rng.uniform(0.0, 0.1, nsrc)
    chi = rng.uniform(0.0, math.pi, nsrc)
    vfrac = rng.uniform(-0.01, 0.01, nsrc)
    iquv = np.stack([i, p * i * np.cos(2 * chi), p * i * np.sin(2 * chi), vfrac * i], axis=1)
    return r * np.cos(t), r * np.sin(t), iquv


def config2(seed: int = SEED_BASE + 2, nvis: int = 2_300_000, n: int = 2048,
            nplanes: int = 32, cell: float = 7.0 * ARCSEC, freq: float = 1.4e9,
            mk: int = 256) -> Workload:
    """Full-pol A+W: 36 antennas (630 baselines), 8 h tracks, 50 polarised sources."""
    rng = np.random.default_rng(seed)
    enu = antennas_in_disk(36, 1500.0, rng)
    nbl = 36 * 35 // 2
    ndump = -(-nvis // nbl)
    ha = np.linspace(-4.0, 4.0, ndump) * (15.0 * DEG)
    uvw = uvw_tracks(enu, ASKAP_LAT, -45.0 * DEG, ha, freq)[:nvis]
    fov = n * cell
    w_max = math.ceil(np.abs(uvw[:, 2]).max() / 100.0) * 100.0
    planes = linear_w_planes(nplanes, w_max)
    support = support_rule(planes, fov)
    geom = Geometry(n=n, cell=cell, os=8, w_planes=planes, support=support,
                    tile=default_tiles(support, 4), aa_support=7, mk=mk)
    beam = seeded_leakage_beam(1.0 * DEG, rng)
    sl, sm, iquv = polarised_sources(50, 1.0 * DEG, rng)
    return Workload("c2-fullpol-AW-2048", geom, uvw, 4, sl, sm, iquv, beam, 0.2,
                    extra={"freq_hz": freq, "n_ant": 36, "n_dumps": ndump})


def scaled_config2(nvis: int, n: int = 256, nplanes: int = 8, seed: int = SEED_BASE + 2,
                   mk: int = 64, support=None, tile=None) -> Workload:
    """Config-2 physics on a smaller grid for oracle-sized parity cases.

    Same array, tracks, beam and leakage; the 7 arcsec cell is kept so the uv tracks still
    fill the grid (the field of view shrinks with n).  `support` overrides the per-plane
    support table (default: the support rule with a floor of 8 taps).
    """
    w = config2(seed=seed, nvis=nvis, n=n, nplanes=nplanes, mk=mk)
    g = w.geom
    if support is None:
        support = support_rule(g.w_planes, g.fov, s_min=8, s_max=48)
    support = np.asarray(support, dtype=np.int32)
    if tile is None:
        tile = default_tiles(support, 4)
    w.geom = Geometry(n=g.n, cell=g.cell, os=g.os, w_planes=g.w_planes, support=support,
                      tile=np.asarray(tile, dtype=np.int32), aa_support=g.aa_support, mk=mk)
    w.name = f"c2-fullpol-AW-{n}"
    return w


def config3(seed: int = SEED_BASE + 3, nfields: int = 16, n: int = 4096, cell: float = 3.5 * ARCSEC,
            nplanes: int = 32, vis_lo: int = 100_000, vis_hi: int = 4_000_000, mk: int = 256,
            count_scale: float = 1.0) -> list:
    """Batched: nfields channels 700-1800 MHz, each with its own grid, beam and visibility count.

    Counts are log-uniform in [vis_lo, vis_hi] (times count_scale); each field is the 36-antenna
    array tracked over 8 h with count/630 dumps at its own frequency; the power-beam FWHM is
    1 deg x 1.4 GHz / nu; the cell keeps the field of view (and so the supports) of config 2.
    """
    rng = np.random.default_rng(seed)
    enu = antennas_in_disk(36, 1500.0, rng)
    counts = np.exp(rng.uniform(math.log(vis_lo), math.log(vis_hi), nfields))
    counts = np.maximum(1, (counts * count_scale).astype(np.int64))
    nbl = 36 * 35 // 2
    out = []
    for i in range(nfields):
        nu = 700e6 + i * 1100e6 / max(1, nfields - 1)
        ndump = max(1, -(-int(counts[i]) // nbl))
        ha = np.linspace(-4.0, 4.0, ndump) * (15.0 * DEG)
        uvw = uvw_tracks(enu, ASKAP_LAT, -45.0 * DEG, ha, nu)[:int(counts[i])]
        fov = n * cell
        w_max = max(100.0, math.ceil(np.abs(uvw[:, 2]).max() / 100.0) * 100.0)
        planes = linear_w_planes(nplanes, w_max)
        support = support_rule(planes, fov)
        geom = Geometry(n=n, cell=cell, os=8, w_planes=planes, support=support,
                        tile=default_tiles(support, 4), aa_support=7, mk=mk)
        beam = seeded_leakage_beam(1.0 * DEG * 1.4e9 / nu, rng)
        out.append(Workload(f"c3-field{i:02d}-{nu / 1e6:.0f}MHz", geom, uvw, 4, beam=beam,
                            extra={"freq_hz": nu}))
    return out


# --------------------------------------------------------------------------- c4: kernel surrogate

@dataclass
class RotatedLeakageBeam:
    """The leakage beam of an alt-az antenna seen at parallactic angle pa.

    The pattern turns with pa on the sky and the X/Y feed basis turns with it:
    J(l, m) = J0(l cos pa + m sin pa, -l sin pa + m cos pa) R(pa), R(pa) = [[cos, -sin], [sin, cos]].
    """

    base: GaussianLeakageBeam
    pa: float

    def jones(self, l, m) -> np.ndarray:
        l = np.asarray(l, dtype=np.float64)
        m = np.asarray(m, dtype=np.float64)
        c, s = math.cos(self.pa), math.sin(self.pa)
        j = self.base.jones(c * l + s * m, -s * l + c * m)
        rot = np.array([[c, -s], [s, c]], dtype=np.complex128)
        return j @ rot


@dataclass
class SurrogateSetup:
    """Kernel-surrogate workload (c4).

    Kernels: 48 x 48 taps x 8 x 8 phases on the config-1 grid (256^2, field of view 0.1 rad),
    lattice mk = 256, for w in [-w_max, w_max], frequency in [nu_lo, nu_hi] (power-beam FWHM
    1 deg x 1.4 GHz / nu) and parallactic angle in [-pi, pi]; one leakage pattern (seeded) for all.
    Evaluation: the config-1 uv coverage and point sources, full polarisation, at (nu_eval, pa_eval).
    """

    geom: Geometry                 # 8 linear planes on [-w_max, w_max]: the nearest-plane baseline
    leakage: GaussianLeakageBeam   # theta is replaced per frequency
    w_max: float
    nu_lo: float
    nu_hi: float
    nu_eval: float
    pa_eval: float
    uvw: np.ndarray
    src_l: np.ndarray
    src_m: np.ndarray
    src_iquv: np.ndarray

    def beam(self, nu: float, pa: float) -> RotatedLeakageBeam:
        b = GaussianLeakageBeam(theta=1.0 * DEG * 1.4e9 / nu, dxy=self.leakage.dxy, dyx=self.leakage.dyx,
                                level=self.leakage.level)
        return RotatedLeakageBeam(b, pa)

    def plane_geometry(self, w_planes) -> Geometry:
        """The same grid and kernels with another (ascending) w-plane set."""
        p = len(w_planes)
        return Geometry(n=self.geom.n, cell=self.geom.cell, os=self.geom.os, w_planes=np.asarray(w_planes),
                        support=np.full(p, int(self.geom.support[0]), np.int32),
                        tile=np.full(p, int(self.geom.tile[0]), np.int32), aa_support=self.geom.aa_support,
                        mk=self.geom.mk)

    def draw(self, count: int, rng):
        """count seeded (w, nu, pa) draws: w ~ U(-w_max, w_max), nu ~ U(nu_lo, nu_hi), pa ~ U(-pi, pi)."""
        return (rng.uniform(-self.w_max, self.w_max, count), rng.uniform(self.nu_lo, self.nu_hi, count),
                rng.uniform(-math.pi, math.pi, count))


def config4(seed: int = SEED_BASE + 4, nvis: int = 20000) -> SurrogateSetup:
    rng = np.random.default_rng(seed)
    c1 = config1(nvis=nvis)
    n, cell, support = 256, 0.1 / 256, 48
    planes = linear_w_planes(8, 200.0)
    geom = Geometry(n=n, cell=cell, os=8, w_planes=planes, support=np.full(8, support, np.int32),
                    tile=default_tiles(np.full(8, support, np.int32), 4), aa_support=7, mk=256)
    leak = seeded_leakage_beam(1.0 * DEG, rng)
    iquv = np.zeros((len(c1.src_l), 4))
    iquv[:, 0] = c1.src_iquv[:, 0]
    return SurrogateSetup(geom=geom, leakage=leak, w_max=200.0, nu_lo=700e6, nu_hi=1800e6, nu_eval=700e6,
                          pa_eval=0.4, uvw=c1.uvw, src_l=c1.src_l, src_m=c1.src_m, src_iquv=iquv)


# --------------------------------------------------------------------------- c5: major cycle at scale

def config5(seed: int = SEED_BASE + 5, nvis: int = 20_000_000, n: int = 8192, cell: float = 1.76 * ARCSEC,
            nplanes: int = 128, nchan: int = 288, f0: float = 1.2955e9, df: float = 1e6, ndump: int = 110,
            nsrc: int = 1000, mk: int = 256) -> Workload:
    """Major cycle at scale: 8192^2 x 4, 128 w-planes, the 36-antenna array over 8 h with `ndump`
    dumps in each of `nchan` 1 MHz channels from f0 (one kernel set for all channels, the beams
    averaged over the band), padded with further dumps to `nvis` rows; a 1000-component polarised
    point model within 1 degree.  Rows are channel-major, then time-major."""
    rng = np.random.default_rng(seed)
    enu = antennas_in_disk(36, 1500.0, rng)
    nbl = 36 * 35 // 2
    per_chan = max(ndump, -(-nvis // (nbl * nchan)))
    ha = np.linspace(-4.0, 4.0, per_chan) * (15.0 * DEG)
    uvw = np.empty((nchan * per_chan * nbl, 3))
    for c in range(nchan):
        uvw[c * per_chan * nbl:(c + 1) * per_chan * nbl] = uvw_tracks(enu, ASKAP_LAT, -45.0 * DEG, ha, f0 + c * df)
    uvw = np.ascontiguousarray(uvw[:nvis])
    fov = n * cell
    w_max = math.ceil(np.abs(uvw[:, 2]).max() / 100.0) * 100.0
    planes = linear_w_planes(nplanes, w_max)
    support = support_rule(planes, fov)
    geom = Geometry(n=n, cell=cell, os=8, w_planes=planes, support=support,
                    tile=default_tiles(support, 4), aa_support=7, mk=mk)
    beam = seeded_leakage_beam(1.0 * DEG, rng)
    sl, sm, iquv = polarised_sources(nsrc, 1.0 * DEG, rng)
    return Workload(f"c5-majorcycle-{n}", geom, uvw, 4, sl, sm, iquv, beam, 0.2,
                    extra={"freq_hz": f0 + 0.5 * (nchan - 1) * df, "n_chan": nchan, "dumps_per_chan": per_chan})


def mosaic7_pointings(ra0: float, dec0: float, spacing: float):
    """Seven pointing centres (radians): ra0, dec0 and a hexagon of six at `spacing` radians."""
    out = [(ra0, dec0)]
    for k in range(6):
        a = k * math.pi / 3.0
        out.append((ra0 + spacing * math.cos(a) / math.cos(dec0), dec0 + spacing * math.sin(a)))
    return out


def config5_mosaic(nfields: int = 7, spacing: float = 0.5 * DEG, ra0: float = 1.0, dec0: float = -45.0 * DEG,
                   pad: float = 1.25, **kw):
    """The major-cycle workload as a 7-field image-domain mosaic: config 5's 20M rows split into
    seven consecutive blocks (channel ranges), one per pointing (the centre and a hexagon at
    half the 1-degree beam width), each field imaged on its own 8192^2 x 4 frame about its
    pointing; the mosaic frame has the same cell, centred on the middle pointing, `pad` times
    the field size.  Returns (workload, list of (ra, dec) field centres, mosaic frame (n, cell,
    ra, dec))."""
    w = config5(**kw)
    centres = mosaic7_pointings(ra0, dec0, spacing)[:nfields]
    nm = int(round(w.geom.n * pad / 16.0)) * 16
    return w, centres, (nm, w.geom.cell, ra0, dec0)

