"""Plain FP64 CPU oracle for the TV-regularized frequency-domain FWI hot path.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or run this module. The product path (the HIP
library and its Python binding) never calls it, and it imports nothing from
the product path: it is written from the paper, in the paper's order, as
plainly as possible (numpy / scipy, complex128 throughout).

Time convention: e^{-i omega t}. The paper writes kappa = kappa' - j kappa''
(an e^{+j omega t} convention); every complex quantity here is the complex
conjugate of the paper's, while misfits, magnitudes, speeds of sound and the
real gradients are unchanged.

Discrete problem (the paper says only "after discretization", Sec. IV-A):
pulse basis on square/cubic cells, collocation at cell centres, and the cell
integral of the Green's function done over the equal-area disk (2D) or
equal-volume ball (3D) of the cell (Richmond's method). Point elements on the
top face z = 0; point receivers with the midpoint rule for the data integral.

Every function cites the passage of the paper it follows.
"""
from __future__ import annotations

import math
import numpy as np
import scipy.fft
import scipy.linalg
import scipy.sparse.linalg
import scipy.special as sp

DENSE_MAX = 1600          # dense LU up to this many unknowns, GMRES above
GMRES_RTOL = 1e-12
FFT_WORKERS = -1          # scipy.fft worker count (-1: all host cores)


# --------------------------------------------------------------------------
# Medium (Sec. II, Eq. 1-3)
# --------------------------------------------------------------------------

class Background:
    """A lossy background (Sec. II: background compressibility kappa_0 from the
    background SoS c0 and attenuation alpha0 [Np/m/Hz]); wherever the oracle
    takes c0 it also takes a Background. A plain number is the lossless
    background alpha0 = 0."""

    def __init__(self, c0, alpha0=0.0):
        self.c0, self.alpha0 = float(c0), float(alpha0)


def kappa0_rho(c0):
    """kappa_0 rho_0 of the background (Eq. 2 at the background values)."""
    if isinstance(c0, Background):
        a0 = c0.alpha0
        return 1.0 / c0.c0**2 - a0**2 / (2.0 * math.pi) ** 2 + 1j * a0 / (math.pi * c0.c0)
    return 1.0 / c0**2


def contrast(c, alpha, c0):
    """Contrast m = kappa/kappa0 - 1 (Eq. 3) from speed of sound and attenuation.

    Eq. 1-2 with constant density rho0: kappa*rho0 = 1/c^2 - alpha^2/(2 pi)^2
    + i alpha/(pi c) (e^{-i omega t}; the alpha^2 term of Eq. 2 is kept);
    kappa0*rho0 of the background as in kappa0_rho (1/c0^2 when lossless).
    alpha in Np/m/Hz.
    """
    c = np.asarray(c, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)
    kappa_rho = 1.0 / c**2 - alpha**2 / (2.0 * math.pi) ** 2 + 1j * alpha / (math.pi * c)
    return kappa_rho / kappa0_rho(c0) - 1.0


def contrast_derivs(c, alpha, c0):
    """dm/dc and dm/dalpha of the contrast above (for the chain rule)."""
    k0r = kappa0_rho(c0)
    dm_dc = (-2.0 / c**3 - 1j * alpha / (math.pi * c**2)) / k0r
    dm_da = (-2.0 * alpha / (2.0 * math.pi) ** 2 + 1j / (math.pi * c)) / k0r
    return dm_dc, dm_da


def wavenumber(freq, c0):
    """Background wavenumber k_{l,0} = omega_l sqrt(kappa0 rho0) (Sec. II):
    2 pi f / c0 for a lossless background, the root with Im k > 0 (outgoing,
    decaying under exp(-i omega t)) for a lossy one."""
    if isinstance(c0, Background):
        return 2.0 * math.pi * float(freq) * np.sqrt(complex(kappa0_rho(c0)))
    return 2.0 * math.pi * float(freq) / c0


# --------------------------------------------------------------------------
# Grid geometry
# --------------------------------------------------------------------------

def grid_shape(dim, nx, ny, nz):
    return (nz, nx) if dim == 2 else (nz, ny, nx)


def cell_centres(dim, nx, ny, nz, dx):
    """[n, 3] cell-centre coordinates, flattened in (z, y, x) order, x fastest."""
    x = (np.arange(nx) + 0.5) * dx
    z = (np.arange(nz) + 0.5) * dx
    if dim == 2:
        zz, xx = np.meshgrid(z, x, indexing="ij")
        yy = np.zeros_like(xx)
    else:
        y = (np.arange(ny) + 0.5) * dx
        zz, yy, xx = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)


def cell_volume(dim, dx):
    return dx**dim


# --------------------------------------------------------------------------
# Green's function and cell weights (Sec. II "analytically known"; Sec. IV-A)
# --------------------------------------------------------------------------

def green(k, r, dim):
    """Outgoing free-space Green's function of (nabla^2 + k^2) G = -delta.

    2D: (i/4) H0^(1)(k r); 3D: exp(i k r) / (4 pi r).
    """
    r = np.asarray(r, dtype=np.float64)
    if dim == 2:
        return 0.25j * sp.hankel1(0, k * r)
    return np.exp(1j * k * r) / (4.0 * math.pi * r)


def richmond_radius(dx, dim):
    """Radius of the disk (2D) / ball (3D) with the cell's area / volume."""
    if dim == 2:
        return dx / math.sqrt(math.pi)
    return dx * (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0)


def cell_weight(k, r, dx, dim):
    """W(r): integral of G over the equal-area disk / equal-volume ball of a
    cell whose centre is at distance r from the observation point.

    2D, r > 0: (i/4)(2 pi a / k) J1(k a) H0(k r)      (Graf addition theorem)
    2D, r = 0: (i pi a/(2k)) H1(k a) - 1/k^2          (integral of r H0 dr)
    3D, r > 0: (4 pi/k^3)(sin ka - ka cos ka) e^{ikr}/(4 pi r)
    3D, r = 0: ((1 - i k a) e^{i k a} - 1) / k^2
    """
    r = np.asarray(r, dtype=np.float64)
    a = richmond_radius(dx, dim)
    ka = k * a
    out = np.empty(r.shape, dtype=np.complex128)
    off = r > 0
    if dim == 2:
        out[off] = 0.25j * (2.0 * math.pi * a / k) * sp.jv(1, ka) * sp.hankel1(0, k * r[off])
        out[~off] = 1j * math.pi * a / (2.0 * k) * sp.hankel1(1, ka) - 1.0 / k**2
    else:
        fac = 4.0 * math.pi / k**3 * (np.sin(ka) - ka * np.cos(ka))
        out[off] = fac * np.exp(1j * k * r[off]) / (4.0 * math.pi * r[off])
        out[~off] = ((1.0 - 1j * ka) * np.exp(1j * ka) - 1.0) / k**2
    return out


class FiniteElements:
    """Elements with an aperture on the top face (Sec. V models a finite-length
    array; Eq. 4 integrates over the receiver region): a width x height
    rectangle centred at each position (height only in 3D). Reading: each
    element transmits and receives as the average of the point-source field
    over its aperture, so a vanishing aperture is the point element; the
    average is taken with a quad-point Gauss-Legendre rule per direction."""

    def __init__(self, xyz, width=0.0, height=0.0, quad=1):
        self.xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
        self.width, self.height, self.quad = float(width), float(height), int(quad)

    def __len__(self):
        return len(self.xyz)


def incident_fields(k, centres, elems, dim):
    """P0[e, n] = G(|x_n - x_e|): field of a unit point source at element e in the
    homogeneous background (Sec. II, the incident field p_{i,0}); for
    FiniteElements the aperture average of that field."""
    if isinstance(elems, FiniteElements):
        def rule(extent):
            if extent <= 0.0:
                return np.zeros(1), np.ones(1)
            x, w = np.polynomial.legendre.leggauss(elems.quad)
            return 0.5 * extent * x, 0.5 * w
        xa, wa = rule(elems.width)
        xb, wb = rule(elems.height)
        out = 0.0
        for a in range(len(xa)):
            for b in range(len(xb)):
                sub = elems.xyz + np.array([xa[a], xb[b], 0.0])
                out = out + wa[a] * wb[b] * incident_fields(k, centres, sub, dim)
        return out
    d = np.linalg.norm(centres[None, :, :] - elems[:, None, :], axis=2)
    return green(k, d, dim)


# --------------------------------------------------------------------------
# The discrete volume integral operator (Eq. 5; Sec. IV-A)
# --------------------------------------------------------------------------

def _axis_offsets(N):
    """Offsets of a length-2N circulant axis: i for i < N, i - 2N for i > N;
    index N is the unused wrap entry."""
    i = np.arange(2 * N)
    off = np.where(i < N, i, i - 2 * N).astype(np.float64)
    return off, i != N


def green_table(k, dim, nx, ny, nz, dx):
    """k^2 W(|Delta| dx) on the 2N-per-axis circulant grid (zero at wrap entries)."""
    if dim == 2:
        oz, mz = _axis_offsets(nz)
        ox, mx = _axis_offsets(nx)
        Z, X = np.meshgrid(oz, ox, indexing="ij")
        r = dx * np.sqrt(Z**2 + X**2)
        mask = mz[:, None] & mx[None, :]
    else:
        oz, mz = _axis_offsets(nz)
        oy, my = _axis_offsets(ny)
        ox, mx = _axis_offsets(nx)
        Z, Y, X = np.meshgrid(oz, oy, ox, indexing="ij")
        r = dx * np.sqrt(Z**2 + Y**2 + X**2)
        mask = mz[:, None, None] & my[None, :, None] & mx[None, None, :]
    T = k**2 * cell_weight(k, r, dx, dim)
    T[~mask] = 0.0
    return T


def green_spectrum(k, dim, nx, ny, nz, dx):
    """FFT of the circulant Green table (the convolution kernel of Sec. IV-A)."""
    return scipy.fft.fftn(green_table(k, dim, nx, ny, nz, dx), workers=FFT_WORKERS)


def convolve(Ghat, u):
    """Linear convolution of the grid-shaped u with the Green table via FFT:
    zero-pad to the 2N grid, multiply spectra, inverse FFT, crop."""
    shape = u.shape
    pad = np.zeros(Ghat.shape, dtype=np.complex128)
    pad[tuple(slice(0, s) for s in shape)] = u
    y = scipy.fft.ifftn(Ghat * scipy.fft.fftn(pad, workers=FFT_WORKERS), workers=FFT_WORKERS)
    return y[tuple(slice(0, s) for s in shape)]


def vie_apply(Ghat, m, x):
    """(A x) = x - k^2 sum_n' W(|x_n - x_n'|) m_n' x_n'  (Eq. 5 discretised)."""
    return x - convolve(Ghat, m * x)


def dense_operator(k, m_flat, centres, dx, dim):
    """Dense A[n, n'] = delta_nn' - k^2 W(|x_n - x_n'|) m_n' for tiny grids."""
    d = np.linalg.norm(centres[:, None, :] - centres[None, :, :], axis=2)
    W = cell_weight(k, d, dx, dim)
    return np.eye(len(m_flat), dtype=np.complex128) - k**2 * W * m_flat[None, :]


def solve(k, m, rhs, dim, nx, ny, nz, dx, Ghat=None, rtol=GMRES_RTOL):
    """Solve A p = rhs for every row of rhs ([nb, n]).

    Dense LU when n <= DENSE_MAX; otherwise GMRES (Sec. IV-A names GMRES;
    the converged solution does not depend on the Krylov method)."""
    shape = grid_shape(dim, nx, ny, nz)
    n = int(np.prod(shape))
    rhs = np.atleast_2d(rhs)
    mf = m.reshape(-1)
    if n <= DENSE_MAX:
        cen = cell_centres(dim, nx, ny, nz, dx)
        A = dense_operator(k, mf, cen, dx, dim)
        lu = scipy.linalg.lu_factor(A)
        return scipy.linalg.lu_solve(lu, rhs.T).T
    if Ghat is None:
        Ghat = green_spectrum(k, dim, nx, ny, nz, dx)
    mg = m.reshape(shape)
    op = scipy.sparse.linalg.LinearOperator(
        (n, n), dtype=np.complex128,
        matvec=lambda v: vie_apply(Ghat, mg, v.reshape(shape)).reshape(-1))
    out = np.empty_like(rhs, dtype=np.complex128)
    for b in range(rhs.shape[0]):
        x, info = scipy.sparse.linalg.gmres(op, rhs[b], x0=rhs[b], rtol=rtol, atol=0.0,
                                            restart=60, maxiter=400)
        if info != 0:
            raise RuntimeError(f"oracle GMRES did not converge (info={info})")
        out[b] = x
    return out


# --------------------------------------------------------------------------
# Forward model F(m) (Eq. 4-6)
# --------------------------------------------------------------------------

def scattered_data(k, m_flat, P0, fields, dx, dim):
    """P^s[i, j] = k^2 dV sum_n G(x_j, x_n) m_n p_i(x_n)  (Eq. 4, point receiver,
    midpoint rule); G(x_j, x_n) = P0[j, n]."""
    dV = cell_volume(dim, dx)
    return k**2 * dV * (fields * m_flat[None, :]) @ P0.T


def forward_m(m, dim, nx, ny, nz, dx, c0, freqs, elems, tx=None):
    """F(m): fields p_{l,i} = A_l^{-1} P0_l[i] and data [nf, ne, ne] (layout [l][i][j]).

    tx: optional subset of transmit indices (data rows restricted to it)."""
    cen = cell_centres(dim, nx, ny, nz, dx)
    mf = m.reshape(-1)
    tx = np.arange(len(elems)) if tx is None else np.asarray(tx)
    data, fields, P0s = [], [], []
    for f in freqs:
        k = wavenumber(f, c0)
        P0 = incident_fields(k, cen, elems, dim)
        p = solve(k, m, P0[tx], dim, nx, ny, nz, dx)
        data.append(scattered_data(k, mf, P0, p, dx, dim))
        fields.append(p)
        P0s.append(P0)
    return np.array(data), np.array(fields), np.array(P0s)


def forward(c, alpha, dim, nx, ny, nz, dx, c0, freqs, elems, tx=None):
    """F(m(c, alpha)) for a speed-of-sound / attenuation model (Eq. 3-6)."""
    return forward_m(contrast(c, alpha, c0), dim, nx, ny, nz, dx, c0, freqs, elems, tx)


def misfit(data, d_obs):
    """phi = 1/2 ||F(m) - d_obs||^2 (data term of Eq. 7)."""
    return 0.5 * float(np.sum(np.abs(data - d_obs) ** 2))


# --------------------------------------------------------------------------
# Jacobian products (Eq. 15-17, Sec. IV-B/C)
# --------------------------------------------------------------------------

def jacobian_apply(fields, a_flat, freqs, c0, dx, dim):
    """(J a)_{l,i,j} = k_l^2 dV sum_n p_{l,i}(x_n) p_{l,j}(x_n) a_n  (Eq. 16).

    With transmit set = receive set the adjoint field of receiver j equals
    the forward field p_j exactly for this discretisation (Eq. 15 holds with
    equality)."""
    dV = cell_volume(dim, dx)
    out = []
    for l, f in enumerate(freqs):
        k = wavenumber(f, c0)
        p = fields[l]
        out.append(k**2 * dV * (p * a_flat[None, :]) @ p.T)
    return np.array(out)


def jacobian_adjoint_apply(fields, b, freqs, c0, dx, dim):
    """(J^H b)_n = sum_{l,i,j} conj(k_l^2 dV p_{l,i}(x_n) p_{l,j}(x_n)) b_{l,i,j}  (Eq. 17).

    The frequency-dependent k_l^2 is taken inside the sum over l and
    conjugated (the exact adjoint of Eq. 16)."""
    dV = cell_volume(dim, dx)
    n = fields.shape[-1]
    out = np.zeros(n, dtype=np.complex128)
    for l, f in enumerate(freqs):
        k = wavenumber(f, c0)
        p = fields[l]
        out += np.conj(k**2 * dV) * np.einsum("in,jn,ij->n", np.conj(p), np.conj(p), b[l])
    return out


def adjoint_gradient_m(m, d_obs, dim, nx, ny, nz, dx, c0, freqs, elems, upstream=None):
    """Misfit and its gradient g = J^H r (r = F(m) - d_obs) by adjoint solves.

    For each frequency: adjoint sources s_{l,i} = sum_j conj(r_{l,i,j}) P0_l[j],
    adjoint fields lam_{l,i} = A_l^{-1} s_{l,i} (the same operator: the
    discrete M A^{-1} is symmetric), and
    g_n = dV sum_l conj(k_l^2) sum_i conj(p_{l,i}(x_n) lam_{l,i}(x_n)).
    g packs d phi/d Re m + i d phi/d Im m. With `upstream` given, r is replaced
    by that data-space vector (a vector-Jacobian product J^H b)."""
    cen = cell_centres(dim, nx, ny, nz, dx)
    mf = m.reshape(-1)
    dV = cell_volume(dim, dx)
    data, fields, P0s = forward_m(m, dim, nx, ny, nz, dx, c0, freqs, elems)
    r = data - d_obs if upstream is None else upstream
    phi = misfit(data, d_obs) if d_obs is not None else None
    g = np.zeros(mf.shape, dtype=np.complex128)
    for l, f in enumerate(freqs):
        k = wavenumber(f, c0)
        S = np.conj(r[l]) @ P0s[l]
        lam = solve(k, m, S, dim, nx, ny, nz, dx)
        g += dV * np.conj(k**2) * np.sum(np.conj(fields[l] * lam), axis=0)
    return phi, g, data, fields


def adjoint_gradient(c, alpha, d_obs, dim, nx, ny, nz, dx, c0, freqs, elems):
    """Misfit, gradient w.r.t. m, and the chain rule to c and alpha:
    d phi/d c = Re(conj(g) dm/dc), d phi/d alpha = Re(conj(g) dm/dalpha)."""
    m = contrast(c, alpha, c0)
    phi, g, data, fields = adjoint_gradient_m(m, d_obs, dim, nx, ny, nz, dx, c0, freqs, elems)
    dm_dc, dm_da = contrast_derivs(np.asarray(c).reshape(-1), np.asarray(alpha).reshape(-1), c0)
    gc = np.real(np.conj(g) * dm_dc)
    ga = np.real(np.conj(g) * dm_da)
    return phi, g, gc, ga, data


# --------------------------------------------------------------------------
# Transmits other than the single elements (Sec. IV-B, Sec. V)
# --------------------------------------------------------------------------

def forward_tx_m(m, dim, nx, ny, nz, dx, c0, freqs, elems, weights):
    """Fields and data of transmits synthesised from the elements (Sec. V fires
    steered plane waves from the array; every element receives). Transmit t
    at frequency l drives element e with the complex weight weights[l, t, e],
    so its incident field is sum_e weights[l, t, e] P0_l[e] and its total field
    p_{l,t} solves A_l p = that incident field (Eq. 5). Data [nf, nt, ne] by the
    point-receiver rule of Eq. 4 (receivers are the elements)."""
    cen = cell_centres(dim, nx, ny, nz, dx)
    mf = m.reshape(-1)
    data, fields, P0s = [], [], []
    for l, f in enumerate(freqs):
        k = wavenumber(f, c0)
        P0 = incident_fields(k, cen, elems, dim)
        p = solve(k, m, weights[l] @ P0, dim, nx, ny, nz, dx)
        data.append(scattered_data(k, mf, P0, p, dx, dim))
        fields.append(p)
        P0s.append(P0)
    return np.array(data), np.array(fields), np.array(P0s)


def receiver_fields(m, dim, nx, ny, nz, dx, c0, freqs, elems):
    """Fields p~_{l,j} of sources placed at the receivers (Sec. IV-B, the
    adjoint fields of the Jacobian): with receivers = elements these are the
    element fields, A_l^{-1} P0_l[j]."""
    return forward_m(m, dim, nx, ny, nz, dx, c0, freqs, elems)[1]


def jacobian_apply_tx(tx_fields, rx_fields, a_flat, freqs, c0, dx, dim):
    """(J a)_{l,t,j} = k_l^2 dV sum_n p_{l,t}(x_n) p~_{l,j}(x_n) a_n: the
    sensitivity of Sec. IV-B with transmit fields p and receiver fields p~
    (midpoint rule over each cell)."""
    dV = cell_volume(dim, dx)
    out = []
    for l, f in enumerate(freqs):
        k = wavenumber(f, c0)
        out.append(k**2 * dV * (tx_fields[l] * a_flat[None, :]) @ rx_fields[l].T)
    return np.array(out)


def jacobian_adjoint_apply_tx(tx_fields, rx_fields, b, freqs, c0, dx, dim):
    """(J^H b)_n = sum_{l,t,j} conj(k_l^2 dV p_{l,t}(x_n) p~_{l,j}(x_n)) b_{l,t,j}."""
    dV = cell_volume(dim, dx)
    out = np.zeros(tx_fields.shape[-1], dtype=np.complex128)
    for l, f in enumerate(freqs):
        k = wavenumber(f, c0)
        out += np.conj(k**2 * dV) * np.einsum("tn,jn,tj->n", np.conj(tx_fields[l]), np.conj(rx_fields[l]), b[l])
    return out


def adjoint_gradient_tx_m(m, d_obs, dim, nx, ny, nz, dx, c0, freqs, elems, weights, upstream=None):
    """Misfit and gradient J^H r for synthesised transmits by adjoint solves:
    adjoint sources s_{l,t} = sum_j conj(r_{l,t,j}) P0_l[j], adjoint fields
    lam = A_l^{-1} s, g_n = dV sum_l conj(k_l^2) sum_t conj(p_{l,t}(x_n) lam_{l,t}(x_n))
    (as for element transmits; only the transmit fields change)."""
    mf = m.reshape(-1)
    dV = cell_volume(dim, dx)
    data, fields, P0s = forward_tx_m(m, dim, nx, ny, nz, dx, c0, freqs, elems, weights)
    r = data - d_obs if upstream is None else upstream
    phi = misfit(data, d_obs) if d_obs is not None else None
    g = np.zeros(mf.shape, dtype=np.complex128)
    for l, f in enumerate(freqs):
        k = wavenumber(f, c0)
        lam = solve(k, m, np.conj(r[l]) @ P0s[l], dim, nx, ny, nz, dx)
        g += dV * np.conj(k**2) * np.sum(np.conj(fields[l] * lam), axis=0)
    return phi, g, data, fields


def adjoint_gradient_tx(c, alpha, d_obs, dim, nx, ny, nz, dx, c0, freqs, elems, weights):
    """adjoint_gradient_tx_m at m(c, alpha) with the chain rule to c and alpha."""
    m = contrast(c, alpha, c0)
    phi, g, data, fields = adjoint_gradient_tx_m(m, d_obs, dim, nx, ny, nz, dx, c0, freqs, elems, weights)
    dm_dc, dm_da = contrast_derivs(np.asarray(c).reshape(-1), np.asarray(alpha).reshape(-1), c0)
    return phi, g, np.real(np.conj(g) * dm_dc), np.real(np.conj(g) * dm_da), data


# --------------------------------------------------------------------------
# TV operators and the ADMM step (Eq. 7-14, Algorithm 1)
# --------------------------------------------------------------------------

def _axis_of(q, dim):
    """Component q (0 = x, 1 = y or z, 2 = z) -> array axis of the depth-major grid."""
    return dim - 1 - q


def tv_grad(m):
    """Discrete gradient [d_x m; (d_y m;) d_z m] (Eq. 7): forward differences with
    unit spacing, zero at the last index of each axis."""
    dim = m.ndim
    out = np.zeros((dim,) + m.shape, dtype=np.complex128)
    for q in range(dim):
        ax = _axis_of(q, dim)
        d = np.diff(m, axis=ax)
        sl = [slice(None)] * dim
        sl[ax] = slice(0, m.shape[ax] - 1)
        out[q][tuple(sl)] = d
    return out


def tv_grad_T(a):
    """nabla^T a = sum_q d_q^T a_q (Sec. III, after Eq. 12), the exact transpose of
    tv_grad: (d^T v)[i] = v[i-1] [i >= 1] - v[i] [i <= N-2]."""
    dim = a.ndim - 1
    out = np.zeros(a.shape[1:], dtype=np.complex128)
    for q in range(dim):
        ax = _axis_of(q, dim)
        N = a.shape[1 + ax]
        v = a[q]
        lo = [slice(None)] * dim
        hi = [slice(None)] * dim
        lo[ax] = slice(0, N - 1)
        hi[ax] = slice(1, N)
        out[tuple(hi)] += v[tuple(lo)]
        out[tuple(lo)] -= v[tuple(lo)]
    return out


def shrink(a, tau):
    """Isotropic shrinkage (Eq. 14): max(1 - tau/||a_n||, 0) a_n, with
    ||a_n|| = sqrt(sum_q |a_{n,q}|^2) and shrink(0) = 0."""
    norm = np.sqrt(np.sum(np.abs(a) ** 2, axis=0))
    fac = np.where(norm > 0, np.maximum(1.0 - tau / np.where(norm > 0, norm, 1.0), 0.0), 0.0)
    return fac[None] * a


def tv_norm(g):
    """||g||_{1,2} = sum_n sqrt(sum_q |g_{n,q}|^2) (Sec. III)."""
    return float(np.sum(np.sqrt(np.sum(np.abs(g) ** 2, axis=0))))


def conjugate_gradient(apply_A, b, n_iter):
    """n_iter iterations of CG for Hermitian positive definite A from x = 0."""
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rs = float(np.real(np.vdot(r, r)))
    for _ in range(n_iter):
        if rs == 0.0:
            break
        Ap = apply_A(p)
        alpha = rs / float(np.real(np.vdot(p, Ap)))
        x = x + alpha * p
        r = r - alpha * Ap
        rs_new = float(np.real(np.vdot(r, r)))
        p = r + (rs_new / rs) * p
        rs = rs_new
    return x


def coarse_shape(dim, nx, ny, nz, r):
    """Inversion-mesh shape for an integer coarsening r of the forward mesh
    (ceil per axis; the last cell of an axis may cover fewer forward cells)."""
    cz, cx = -(-nz // r), -(-nx // r)
    return (cz, cx) if dim == 2 else (cz, -(-ny // r), cx)


def prolong(mc, dim, nx, ny, nz, r):
    """Forward-mesh values of an inversion-mesh field (Sec. IV: the contrast is
    represented on a coarser grid than the forward mesh). Reading: piecewise
    constant, forward cell (i, j, k) takes inversion cell (i // r, j // r, k // r)."""
    mc = np.asarray(mc).reshape(coarse_shape(dim, nx, ny, nz, r))
    out = mc
    for ax, nfine in enumerate(grid_shape(dim, nx, ny, nz)):
        out = np.repeat(out, r, axis=ax).take(np.arange(nfine), axis=ax)
    return out


def restrict(gf, dim, nx, ny, nz, r):
    """Adjoint of prolong: each inversion cell sums its forward cells."""
    out = np.asarray(gf).reshape(grid_shape(dim, nx, ny, nz))
    for ax, nfine in enumerate(grid_shape(dim, nx, ny, nz)):
        out = np.add.reduceat(out, np.arange(0, nfine, r), axis=ax)
    return out


def admm_step(m, g, u, m_ref, d_obs, dim, nx, ny, nz, dx, c0, freqs, elems,
              lam, rho, gamma, n_cg, data_scale=1.0, dual_step=None, inv_factor=1):
    """One iteration of Algorithm 1 (forward, model update, g update, u update).

    Model update: Gauss-Newton normal equations (Eq. 11-12) with the data term
    scaled by data_scale,
      A_k = s J^H J + rho nabla^T nabla + gamma I,
      b_k = s J^H (d_obs - F(m_k)) + rho nabla^T (g_k + u_k - nabla m_k)
            + gamma (m_ref - m_k),
    solved by exactly n_cg CG iterations from zero (the gamma terms are dropped
    when m_ref is None). Then g = shrink_{lam/rho}(nabla m_{k+1} - u_k) (Eq. 13-14)
    and u += dual_step (g - nabla m_{k+1}) with dual_step = rho as printed.
    inv_factor r > 1: m, g, u, m_ref live on the inversion mesh (coarse_shape),
    the forward model is prolong(m), the Jacobian is J P (its adjoint
    P^T J^H) and nabla acts on the inversion mesh.
    Returns (m, g, u, report)."""
    if dual_step is None:
        dual_step = rho
    r_ = int(inv_factor)
    shape = grid_shape(dim, nx, ny, nz) if r_ <= 1 else coarse_shape(dim, nx, ny, nz, r_)
    P = (lambda a: a) if r_ <= 1 else (lambda a: prolong(a, dim, nx, ny, nz, r_))
    PT = (lambda a: a) if r_ <= 1 else (lambda a: restrict(a, dim, nx, ny, nz, r_))
    m = m.reshape(shape)
    data, fields, _ = forward_m(P(m), dim, nx, ny, nz, dx, c0, freqs, elems)
    r = d_obs - data
    gm = tv_grad(m)
    b = data_scale * PT(jacobian_adjoint_apply(fields, r, freqs, c0, dx, dim)).reshape(shape)
    b = b + rho * tv_grad_T(g + u - gm)
    use_ref = m_ref is not None and gamma != 0.0
    if use_ref:
        b = b + gamma * (m_ref.reshape(shape) - m)

    def apply_A(a):
        a = a.reshape(shape)
        Ja = jacobian_apply(fields, P(a).reshape(-1), freqs, c0, dx, dim)
        out = data_scale * PT(jacobian_adjoint_apply(fields, Ja, freqs, c0, dx, dim)).reshape(shape)
        out = out + rho * tv_grad_T(tv_grad(a))
        if use_ref:
            out = out + gamma * a
        return out

    dm = conjugate_gradient(apply_A, b, n_cg)
    m_new = m + dm
    gm_new = tv_grad(m_new)
    g_new = shrink(gm_new - u, lam / rho)
    u_new = u + dual_step * (g_new - gm_new)
    report = dict(misfit=misfit(data, d_obs), tv=tv_norm(gm_new),
                  dm_norm=float(np.linalg.norm(dm)))
    return m_new, g_new, u_new, report


def admm_step_tx(m, g, u, m_ref, d_obs, dim, nx, ny, nz, dx, c0, freqs, elems, weights,
                 lam, rho, gamma, n_cg, rx_fields=None, data_scale=1.0, dual_step=None):
    """admm_step for synthesised transmits (weights [nf, nt, ne], d_obs
    [nf, nt, ne]): the Jacobian of Sec. IV-B from the transmit fields at m_k
    and the receiver fields p~. rx_fields None: p~ recomputed at m_k (the
    distorted-Born Jacobian); given: used as they are (the paper's Born reuse
    of receiver fields from an earlier iterate). Returns (m, g, u, report,
    receiver fields used)."""
    if dual_step is None:
        dual_step = rho
    shape = grid_shape(dim, nx, ny, nz)
    m = m.reshape(shape)
    data, fields, _ = forward_tx_m(m, dim, nx, ny, nz, dx, c0, freqs, elems, weights)
    rx = receiver_fields(m, dim, nx, ny, nz, dx, c0, freqs, elems) if rx_fields is None else rx_fields
    r = d_obs - data
    gm = tv_grad(m)
    b = data_scale * jacobian_adjoint_apply_tx(fields, rx, r, freqs, c0, dx, dim).reshape(shape)
    b = b + rho * tv_grad_T(g + u - gm)
    use_ref = m_ref is not None and gamma != 0.0
    if use_ref:
        b = b + gamma * (m_ref.reshape(shape) - m)

    def apply_A(a):
        a = a.reshape(shape)
        Ja = jacobian_apply_tx(fields, rx, a.reshape(-1), freqs, c0, dx, dim)
        out = data_scale * jacobian_adjoint_apply_tx(fields, rx, Ja, freqs, c0, dx, dim).reshape(shape)
        out = out + rho * tv_grad_T(tv_grad(a))
        if use_ref:
            out = out + gamma * a
        return out

    dm = conjugate_gradient(apply_A, b, n_cg)
    m_new = m + dm
    gm_new = tv_grad(m_new)
    g_new = shrink(gm_new - u, lam / rho)
    u_new = u + dual_step * (g_new - gm_new)
    report = dict(misfit=misfit(data, d_obs), tv=tv_norm(gm_new), dm_norm=float(np.linalg.norm(dm)))
    return m_new, g_new, u_new, report, rx


def sos_from_contrast(m, c0):
    if isinstance(c0, Background):
        # kappa rho = (m + 1) kappa_0 rho_0 = A + i B; 1/c^2 - alpha^2/(4 pi^2) = A,
        # alpha/(pi c) = B: x = c^2 solves (B^2/4) x^2 + A x - 1 = 0
        kr = (np.asarray(m, dtype=np.complex128) + 1.0) * kappa0_rho(c0)
        A, B = kr.real, kr.imag
        c = np.sqrt(2.0 / (A + np.sqrt(A**2 + B**2)))
        return c, math.pi * c * B
    return _sos_from_contrast_lossless(m, c0)


def _sos_from_contrast_lossless(m, c0):
    """Speed of sound and attenuation of a contrast (inverse of Eq. 1-3): with
    R = Re m + 1 and I = Im m, Eq. 3 gives R = c0^2/c^2 - c0^2 alpha^2/(4 pi^2)
    and I = c0^2 alpha/(pi c); eliminating alpha = pi c I / c0^2 leaves the
    quadratic (I^2/(4 c0^2)) x^2 + R x - c0^2 = 0 in x = c^2, of which c^2 is
    the positive root, (-R + sqrt(R^2 + I^2)) 2 c0^2 / I^2, taken in the
    equivalent form 2 c0^2 / (R + sqrt(R^2 + I^2)) (no cancellation for small
    I; c0^2 / R at I = 0)."""
    m = np.asarray(m, dtype=np.complex128)
    R, I = m.real + 1.0, m.imag
    c = np.sqrt(2.0 * c0**2 / (R + np.sqrt(R**2 + I**2)))
    return c, math.pi * c * I / c0**2


def invert(m0, d_obs, dim, nx, ny, nz, dx, c0, freqs, elems, lam, rho, gamma, n_cg, max_iter, tol=0.0,
           m_ref=None, data_scale=1.0, dual_step=None, weights=None, born_every=0, inv_factor=1):
    """Algorithm 1: g_0 = nabla m_0, u_0 = 0, then ADMM iterations (admm_step,
    or admm_step_tx with receiver fields recomputed at the first iteration and
    every born_every-th one, reused in between) until the misfit at an iterate
    is <= tol * 1/2 ||d_obs||^2 (that iteration's update kept) or max_iter
    iterations have run. Returns (m, g, u, misfits per iteration)."""
    shape = grid_shape(dim, nx, ny, nz) if inv_factor <= 1 else coarse_shape(dim, nx, ny, nz, inv_factor)
    m = np.asarray(m0, dtype=np.complex128).reshape(shape)
    g = tv_grad(m)
    u = np.zeros_like(g)
    half = 0.5 * float(np.sum(np.abs(d_obs) ** 2))
    args = (dim, nx, ny, nz, dx, c0, freqs, elems)
    hist, rx = [], None
    for k in range(max_iter):
        if weights is None:
            m, g, u, rep = admm_step(m, g, u, m_ref, d_obs, *args, lam, rho, gamma, n_cg, data_scale, dual_step,
                                     inv_factor=inv_factor)
        else:
            refresh = k == 0 or (born_every > 0 and k % born_every == 0)
            m, g, u, rep, rx = admm_step_tx(m, g, u, m_ref, d_obs, *args, weights, lam, rho, gamma, n_cg,
                                            rx_fields=None if refresh else rx, data_scale=data_scale,
                                            dual_step=dual_step)
        hist.append(rep["misfit"])
        if rep["misfit"] <= tol * half:
            break
    return m, g, u, hist
