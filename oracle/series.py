"""Series (Mie-type) solution for a penetrable disk lit by a line source.

TEST INFRASTRUCTURE (see oracle/fwi_oracle.py). Used to pin the physics of
the discrete model in 2D: the continuous problem behind Eq. 4-5 for a
homogeneous disk of contrast m (interior wavenumber k1 = k0 sqrt(1+m)),
constant density, and an exterior unit line source G(x, x_s).

Fields are expanded in cylindrical harmonics about the disk centre:
  incident  (r < r_s): (i/4) sum_n H_n(k0 r_s) J_n(k0 r) e^{i n (phi - phi_s)}
  scattered (r > a)  : sum_n a_n H_n(k0 r) e^{i n (phi - phi_s)}
  interior  (r < a)  : sum_n b_n J_n(k1 r) e^{i n (phi - phi_s)}
with continuity of p and dp/dr at r = a (constant density).
"""
from __future__ import annotations

import math
import numpy as np
import scipy.special as sp


def _coeffs(k0, k1, a, rs, nmax):
    n = np.arange(-nmax, nmax + 1)
    c_n = 0.25j * sp.hankel1(n, k0 * rs)
    j0a, dj0a = sp.jv(n, k0 * a), sp.jvp(n, k0 * a)
    j1a, dj1a = sp.jv(n, k1 * a), sp.jvp(n, k1 * a)
    h0a, dh0a = sp.hankel1(n, k0 * a), sp.h1vp(n, k0 * a)
    a_n = c_n * (k1 * j0a * dj1a - k0 * dj0a * j1a) / (k0 * j1a * dh0a - k1 * dj1a * h0a)
    b_n = (c_n * j0a + a_n * h0a) / j1a
    return n, a_n, b_n


def disk_scattered(k0, m_disk, a, centre, src, pts):
    """Scattered field at points outside the disk (|pts - centre| > a).

    centre, src: (x, z); pts: [np, 2] (x, z)."""
    k1 = k0 * np.sqrt(1.0 + m_disk + 0j)
    rs = math.hypot(src[0] - centre[0], src[1] - centre[1])
    phs = math.atan2(src[1] - centre[1], src[0] - centre[0])
    nmax = int(abs(k1) * a + 20)
    n, a_n, _ = _coeffs(k0, k1, a, rs, nmax)
    pts = np.asarray(pts, dtype=np.float64)
    r = np.hypot(pts[:, 0] - centre[0], pts[:, 1] - centre[1])
    ph = np.arctan2(pts[:, 1] - centre[1], pts[:, 0] - centre[0])
    H = sp.hankel1(n[None, :], k0 * r[:, None])
    E = np.exp(1j * n[None, :] * (ph[:, None] - phs))
    return np.sum(a_n[None, :] * H * E, axis=1)


def disk_total_inside(k0, m_disk, a, centre, src, pts):
    """Total field at points inside the disk."""
    k1 = k0 * np.sqrt(1.0 + m_disk + 0j)
    rs = math.hypot(src[0] - centre[0], src[1] - centre[1])
    phs = math.atan2(src[1] - centre[1], src[0] - centre[0])
    nmax = int(abs(k1) * a + 20)
    n, _, b_n = _coeffs(k0, k1, a, rs, nmax)
    pts = np.asarray(pts, dtype=np.float64)
    r = np.hypot(pts[:, 0] - centre[0], pts[:, 1] - centre[1])
    ph = np.arctan2(pts[:, 1] - centre[1], pts[:, 0] - centre[0])
    J = sp.jv(n[None, :], k1 * r[:, None])
    E = np.exp(1j * n[None, :] * (ph[:, None] - phs))
    return np.sum(b_n[None, :] * J * E, axis=1)
