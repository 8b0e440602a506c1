"""Seeded synthetic inputs: phantoms, arrays and frequency lists.

This module holds input generation only (rasterised speed-of-sound and
attenuation maps, element positions, frequency lists, seeded data noise). It
contains none of the method's arithmetic, so both the HIP path and the FP64
oracle can be fed from it without sharing any numerical code.

Recipes follow the paper's problem statement (Sec. II: constant density, a
speed-of-sound map c(x) and attenuation alpha(x) in Np/m/Hz, elements on the
edge of the domain) and its experiments (Sec. V: thyroid-like cysts and
nodules, a linear array on the top face, ellipsoidal inclusions in 3D). The
paper's own phantoms are not published; these stand in for them.

Conventions
-----------
* Grids are stored depth-major: 2D arrays have shape (nz, nx), 3D arrays
  (nz, ny, nx); x (lateral) is the fastest index.
* Cell centres sit at ((ix+1/2)dx, (iy+1/2)dx, (iz+1/2)dx); the top face of the
  domain is z = 0 and every element lies on it.
* Random numbers come from numpy.random.default_rng(seed) in the draw order
  written in each function.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
import numpy as np

C0 = 1540.0                     # background speed of sound [m/s]
DB_PER_NEPER = 20.0 / math.log(10.0)   # 8.6859 dB per neper


def db_cm_mhz_to_np_m_hz(a_db_cm_mhz):
    """Attenuation unit change: dB/cm/MHz -> Np/m/Hz (1 Np = 8.686 dB)."""
    return np.asarray(a_db_cm_mhz, dtype=np.float64) * (100.0 * 1e-6) / DB_PER_NEPER


@dataclass
class Problem:
    """One imaging problem: grid, array, frequencies and a medium.

    c, alpha: speed of sound [m/s] and attenuation [Np/m/Hz], grid-shaped.
    elems: [ne, 3] element positions (x, y, z) in metres, z = 0.
    """
    name: str
    dim: int
    nx: int
    ny: int
    nz: int
    dx: float
    c0: float
    freqs: np.ndarray
    elems: np.ndarray
    c: np.ndarray
    alpha: np.ndarray
    extra: dict = field(default_factory=dict)
    # element aperture on the top face [m] (0: point elements) and the
    # Gauss-Legendre points per aperture direction
    elem_width: float = 0.0
    elem_height: float = 0.0
    elem_quad: int = 1
    # background attenuation [Np/m/Hz] (0: lossless background)
    alpha0: float = 0.0

    @property
    def shape(self):
        return (self.nz, self.nx) if self.dim == 2 else (self.nz, self.ny, self.nx)

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    @property
    def ne(self):
        return self.elems.shape[0]

    @property
    def nf(self):
        return len(self.freqs)


def linear_array(nx, ny, dx, ne, pitch, dim, max_frac=0.9):
    """Element positions of a linear array centred on the top face (z = 0).

    x_e = W_x/2 + (e - (ne-1)/2) * pitch, y_e = W_y/2 (3D) or 0 (2D).
    If the aperture would exceed max_frac of the lateral width, the pitch is
    compressed to max_frac * W_x / ne.
    """
    wx = nx * dx
    if ne * pitch > max_frac * wx:
        pitch = max_frac * wx / ne
    e = np.arange(ne, dtype=np.float64)
    xs = wx / 2.0 + (e - (ne - 1) / 2.0) * pitch
    ys = np.full(ne, (ny * dx) / 2.0 if dim == 3 else 0.0)
    zs = np.zeros(ne)
    return np.stack([xs, ys, zs], axis=1)


def cell_coords(dim, nx, ny, nz, dx):
    """Cell-centre coordinate arrays (broadcastable, grid-shaped)."""
    x = (np.arange(nx) + 0.5) * dx
    z = (np.arange(nz) + 0.5) * dx
    if dim == 2:
        zz, xx = np.meshgrid(z, x, indexing="ij")
        return xx, None, zz
    y = (np.arange(ny) + 0.5) * dx
    zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    return xx, yy, zz


def _raster_ellipses(rng, dim, nx, ny, nz, dx, c, alpha, count_range=(1, 5)):
    """Draw 1-5 ellipses (ellipsoids in 3D) and paint them in order.

    Draw order per config: count ~ U{lo..hi}; then per shape: semi-axes
    U[1,6] mm (2 or 3 of them), rotation angle U[0,pi) (3D: the angle rotates
    in the x-z plane), centre x ~ U[10%,90%] W_x, (3D: y ~ U[10%,90%] W_y),
    z ~ U[15%,90%] W_z, c ~ U[1480,1600] m/s, alpha ~ U[0,0.5] dB/cm/MHz.
    Later shapes overwrite earlier ones (pixel-centre-inside test).
    """
    xx, yy, zz = cell_coords(dim, nx, ny, nz, dx)
    wx, wy, wz = nx * dx, ny * dx, nz * dx
    count = int(rng.integers(count_range[0], count_range[1] + 1))
    shapes = []
    for _ in range(count):
        semi = rng.uniform(1e-3, 6e-3, size=dim)
        ang = rng.uniform(0.0, math.pi)
        cx = rng.uniform(0.1 * wx, 0.9 * wx)
        cy = rng.uniform(0.1 * wy, 0.9 * wy) if dim == 3 else 0.0
        cz = rng.uniform(0.15 * wz, 0.9 * wz)
        cval = rng.uniform(1480.0, 1600.0)
        aval = rng.uniform(0.0, 0.5)
        ca, sa = math.cos(ang), math.sin(ang)
        u = (xx - cx) * ca + (zz - cz) * sa
        v = -(xx - cx) * sa + (zz - cz) * ca
        if dim == 2:
            inside = (u / semi[0]) ** 2 + (v / semi[1]) ** 2 <= 1.0
        else:
            w = yy - cy
            inside = (u / semi[0]) ** 2 + (v / semi[2]) ** 2 + (w / semi[1]) ** 2 <= 1.0
        c[inside] = cval
        alpha[inside] = db_cm_mhz_to_np_m_hz(aval)
        shapes.append(dict(semi=semi.tolist(), angle=ang, centre=(cx, cy, cz),
                           c=cval, alpha_db=aval))
    return shapes


def perturb_sos(c, seed, rel=0.01):
    """Observed-model SoS: c_obs = c * (1 + rel * xi), xi ~ U[0,1) per cell."""
    rng = np.random.default_rng(seed)
    return c * (1.0 + rel * rng.random(c.shape))


def config0():
    """2D plain FP64: 64x64, dx = 0.154 mm, 1 MHz, 2 mm disk at 1500 m/s, 16 elements."""
    nx = nz = 64
    dx = 0.154e-3
    xx, _, zz = cell_coords(2, nx, 1, nz, dx)
    c = np.full((nz, nx), C0)
    r2 = (xx - nx * dx / 2) ** 2 + (zz - nz * dx / 2) ** 2
    c[r2 <= (2e-3) ** 2] = 1500.0
    alpha = np.zeros_like(c)
    elems = linear_array(nx, 1, dx, 16, 0.3e-3, 2)
    p = Problem("cfg0_2d_64", 2, nx, 1, nz, dx, C0, np.array([1.0e6]), elems, c, alpha)
    p.extra["c_obs"] = perturb_sos(c, seed=0)
    return p


def config1(seed=1, n=256, nf=8, ne=64):
    """2D 256^2, dx = 0.154 mm, 8 frequencies 0.3-1.0 MHz, 64 elements at 0.3 mm,
    1-5 seeded ellipses; observed model = phantom with +1% seeded SoS noise."""
    dx = 0.154e-3
    rng = np.random.default_rng(seed)
    c = np.full((n, n), C0)
    alpha = np.zeros_like(c)
    shapes = _raster_ellipses(rng, 2, n, 1, n, dx, c, alpha)
    elems = linear_array(n, 1, dx, ne, 0.3e-3, 2)
    freqs = np.linspace(0.3e6, 1.0e6, nf)
    p = Problem(f"cfg1_2d_{n}", 2, n, 1, n, dx, C0, freqs, elems, c, alpha)
    p.extra["shapes"] = shapes
    p.extra["c_obs"] = perturb_sos(c, seed=seed + 100)
    return p


def config2(seed=2, count=32):
    """32 uneven 2D instances: N ~ U{128,192,256,384,512}, ne ~ U{32..128},
    nf ~ U{1..4} sorted frequencies ~ U[0.3,1.5] MHz, dx = c0/(10*1.5 MHz).

    Draw order per instance: N, ne, nf, the nf frequencies, then the phantom
    (as config1)."""
    rng = np.random.default_rng(seed)
    dx = C0 / (10 * 1.5e6)
    out = []
    for k in range(count):
        n = int(rng.choice([128, 192, 256, 384, 512]))
        ne = int(rng.integers(32, 129))
        nf = int(rng.integers(1, 5))
        freqs = np.sort(rng.uniform(0.3e6, 1.5e6, size=nf))
        c = np.full((n, n), C0)
        alpha = np.zeros_like(c)
        shapes = _raster_ellipses(rng, 2, n, 1, n, dx, c, alpha)
        elems = linear_array(n, 1, dx, ne, 0.3e-3, 2)
        p = Problem(f"cfg2_inst{k}_{n}", 2, n, 1, n, dx, C0, freqs, elems, c, alpha)
        p.extra["shapes"] = shapes
        out.append(p)
    return out


def config3(seed=3, n=384, nf=12, ne=128):
    """2D 384^2, dx = 0.1283 mm, 12 frequencies 0.3-1.2 MHz, 128 elements at 0.3 mm.
    Thyroid-like phantom: cyst (1500 m/s, r = 4 mm), nodule (1580 m/s, r = 3 mm),
    depths U[10,25] mm, lateral offsets U[-8,8] mm from centre, non-overlapping
    (redrawn until the gap is > 0.5 mm). Draw order: cyst (z, x), nodule (z, x)."""
    dx = C0 / (10 * 1.2e6)
    rng = np.random.default_rng(seed)
    xx, _, zz = cell_coords(2, n, 1, n, dx)
    wx = n * dx
    while True:
        cz, cx = rng.uniform(10e-3, 25e-3), wx / 2 + rng.uniform(-8e-3, 8e-3)
        nz_, nx_ = rng.uniform(10e-3, 25e-3), wx / 2 + rng.uniform(-8e-3, 8e-3)
        if math.hypot(cz - nz_, cx - nx_) > 4e-3 + 3e-3 + 0.5e-3:
            break
    c = np.full((n, n), C0)
    c[(xx - cx) ** 2 + (zz - cz) ** 2 <= (4e-3) ** 2] = 1500.0
    c[(xx - nx_) ** 2 + (zz - nz_) ** 2 <= (3e-3) ** 2] = 1580.0
    alpha = np.zeros_like(c)
    elems = linear_array(n, 1, dx, ne, 0.3e-3, 2)
    freqs = np.linspace(0.3e6, 1.2e6, nf)
    p = Problem(f"cfg3_2d_{n}", 2, n, 1, n, dx, C0, freqs, elems, c, alpha)
    p.extra.update(cyst=(cx, cz), nodule=(nx_, nz_), lam=1e-3, rho=1e-2,
                   gamma=1e-5, n_cg=10, admm_steps=5)
    return p


def config4(seed=4, nx=128, ny=128, nz=96, nf=4, ne=64):
    """3D 128x128x96, dx = 0.2 mm, 4 frequencies 0.4-0.8 MHz, 64 point elements
    along x at y = centre, z = 0, pitch 0.3 mm; 1-5 seeded ellipsoids."""
    dx = 0.2e-3
    rng = np.random.default_rng(seed)
    c = np.full((nz, ny, nx), C0)
    alpha = np.zeros_like(c)
    shapes = _raster_ellipses(rng, 3, nx, ny, nz, dx, c, alpha)
    elems = linear_array(nx, ny, dx, ne, 0.3e-3, 3)
    freqs = np.linspace(0.4e6, 0.8e6, nf)
    p = Problem(f"cfg4_3d_{nx}x{ny}x{nz}", 3, nx, ny, nz, dx, C0, freqs, elems, c, alpha)
    p.extra["shapes"] = shapes
    p.extra["c_obs"] = perturb_sos(c, seed=seed + 100)
    return p


def small2d(seed=10, nx=24, nz=20, ne=6, nf=2, dx=0.154e-3, f_lo=0.6e6, f_hi=1.0e6,
            with_alpha=True):
    """Small 2D problem for parity: a few random ellipses on a ragged grid."""
    rng = np.random.default_rng(seed)
    c = np.full((nz, nx), C0)
    alpha = np.zeros_like(c)
    # scaled-down ellipses: semi-axes in cells
    count = int(rng.integers(1, 4))
    xx, _, zz = cell_coords(2, nx, 1, nz, dx)
    for _ in range(count):
        a, b = rng.uniform(1.5, 5.0, size=2) * dx
        cx, cz = rng.uniform(0.2, 0.8) * nx * dx, rng.uniform(0.25, 0.85) * nz * dx
        ang = rng.uniform(0, math.pi)
        cval = rng.uniform(1480.0, 1600.0)
        aval = rng.uniform(0.0, 0.5) if with_alpha else 0.0
        u = (xx - cx) * math.cos(ang) + (zz - cz) * math.sin(ang)
        v = -(xx - cx) * math.sin(ang) + (zz - cz) * math.cos(ang)
        ins = (u / a) ** 2 + (v / b) ** 2 <= 1
        c[ins] = cval
        alpha[ins] = db_cm_mhz_to_np_m_hz(aval)
    elems = linear_array(nx, 1, dx, ne, 0.3e-3, 2)
    freqs = np.linspace(f_lo, f_hi, nf)
    p = Problem(f"small2d_{nx}x{nz}", 2, nx, 1, nz, dx, C0, freqs, elems, c, alpha)
    p.extra["c_obs"] = perturb_sos(c, seed=seed + 100)
    return p


def small3d(seed=11, nx=12, ny=10, nz=9, ne=4, nf=1, dx=0.2e-3, f_lo=0.8e6, f_hi=0.8e6):
    """Small 3D problem for parity: one random ellipsoid on a ragged grid."""
    rng = np.random.default_rng(seed)
    c = np.full((nz, ny, nx), C0)
    alpha = np.zeros_like(c)
    xx, yy, zz = cell_coords(3, nx, ny, nz, dx)
    a, b, h = rng.uniform(1.5, 3.5, size=3) * dx
    cx, cy, cz = (rng.uniform(0.3, 0.7) * nx * dx, rng.uniform(0.3, 0.7) * ny * dx,
                  rng.uniform(0.3, 0.7) * nz * dx)
    ins = ((xx - cx) / a) ** 2 + ((yy - cy) / b) ** 2 + ((zz - cz) / h) ** 2 <= 1
    c[ins] = rng.uniform(1480.0, 1600.0)
    alpha[ins] = db_cm_mhz_to_np_m_hz(rng.uniform(0.0, 0.5))
    elems = linear_array(nx, ny, dx, ne, 0.3e-3, 3)
    freqs = np.linspace(f_lo, f_hi, nf)
    p = Problem(f"small3d_{nx}x{ny}x{nz}", 3, nx, ny, nz, dx, C0, freqs, elems, c, alpha)
    p.extra["c_obs"] = perturb_sos(c, seed=seed + 100)
    return p


def plane_wave_weights(freqs, elems, angles_deg, c0=C0):
    """Transmit weights [nf, nt, ne] of plane waves steered to the given angles
    (from the depth axis) by the element array (Sec. V synthesises its
    transmissions this way; the paper gives no formula). Reading: element e
    fires with delay (x_e - x_mid) sin(theta) / c0, which under the
    exp(-i omega t) convention is the complex weight exp(i k (x_e - x_mid) sin(theta)),
    k = 2 pi f / c0; unit amplitudes."""
    x = np.asarray(elems, dtype=np.float64)[:, 0]
    x = x - 0.5 * (x.min() + x.max())
    th = np.deg2rad(np.asarray(angles_deg, dtype=np.float64))
    k = 2.0 * math.pi * np.asarray(freqs, dtype=np.float64) / c0
    return np.exp(1j * k[:, None, None] * np.sin(th)[None, :, None] * x[None, None, :])


def add_noise(d, rel, seed):
    """d plus circular complex Gaussian noise of total norm about rel ||d||
    (per-entry standard deviation rel ||d|| / sqrt(N)): the reading of the
    paper's "2% Gaussian noise" on simulated data (Sec. V). Draw order: real
    parts, then imaginary parts."""
    d = np.asarray(d)
    rng = np.random.default_rng(seed)
    sigma = rel * np.linalg.norm(d) / math.sqrt(d.size)
    re = rng.standard_normal(d.shape)
    im = rng.standard_normal(d.shape)
    return d + sigma * (re + 1j * im) / math.sqrt(2.0)


def random_data(seed, nf, ne, scale=1.0):
    """Seeded complex data array [nf][ne][ne] (stand-in for measured data)."""
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal((nf, ne, ne)) + 1j * rng.standard_normal((nf, ne, ne)))


def random_complex(seed, shape, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
