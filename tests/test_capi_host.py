"""Host-side checks of the C ABI (no GPU): exports, validation, workspace
arithmetic and the FP64 Bessel routine the kernels evaluate."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest
import scipy.special as sp

from paper_2604_15796_amd import fwi, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    L = fwi.lib()
    hdr = open(os.path.join(ROOT, "include", "fwi.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*|size_t)\s+(fwi_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(fwi.EXPORTED)


def test_host_bessel_matches_scipy():
    xs = np.concatenate([np.geomspace(1e-3, 24.99, 300), np.geomspace(25.0, 3000.0, 300)])
    for x in xs:
        j0, j1, y0, y1 = fwi.host_bessel01(x)
        h0, h1 = j0 + 1j * y0, j1 + 1j * y1
        assert abs(h0 - sp.hankel1(0, x)) <= 5e-15 * abs(sp.hankel1(0, x))
        assert abs(h1 - sp.hankel1(1, x)) <= 5e-15 * abs(sp.hankel1(1, x))


def test_padded_lengths():
    L = fwi.lib()
    assert [L.fwi_padded_length(n) for n in (1, 16, 20, 64, 96, 100, 256, 384, 512, 513)] == \
        [32, 32, 48, 128, 192, 256, 512, 768, 1024, 0]


def _prob(**kw):
    p = W.small2d(nx=24, nz=20, ne=4, nf=2)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_validation_codes():
    assert fwi.validate_problem(_prob()) == fwi.FWI_OK
    assert fwi.validate_problem(_prob(dim=4)) == fwi.FWI_E_UNSUPPORTED
    assert fwi.validate_problem(_prob(nx=600)) == fwi.FWI_E_UNSUPPORTED
    # largest grid extent the FFT lengths cover (2 x 512 = 1024), and one past it
    assert fwi.validate_problem(_prob(nx=512, c=np.full((20, 512), 1540.0), alpha=np.zeros((20, 512)))) == fwi.FWI_OK
    assert fwi.validate_problem(_prob(nz=513)) == fwi.FWI_E_UNSUPPORTED
    # empty inputs: no frequency, no element, no cell
    assert fwi.validate_problem(_prob(freqs=np.array([]))) == fwi.FWI_E_INVAL
    assert fwi.validate_problem(_prob(elems=np.zeros((0, 3)))) == fwi.FWI_E_INVAL
    assert fwi.validate_problem(_prob(nx=0)) == fwi.FWI_E_INVAL
    assert fwi.validate_problem(_prob(dx=-1.0)) == fwi.FWI_E_INVAL
    assert fwi.validate_problem(_prob(c0=float("nan"))) == fwi.FWI_E_INVAL
    assert fwi.validate_problem(_prob(freqs=np.array([1e6, -1.0]))) == fwi.FWI_E_INVAL
    e = W.small2d(nx=24, nz=20, ne=4).elems.copy()
    e[1, 2] = 1e-4
    assert fwi.validate_problem(_prob(elems=e)) == fwi.FWI_E_UNSUPPORTED    # off the top face
    e = W.small2d(nx=24, nz=20, ne=4).elems.copy()
    e[1] = e[0]
    assert fwi.validate_problem(_prob(elems=e)) == fwi.FWI_E_INVAL          # duplicate
    e = W.small2d(nx=24, nz=20, ne=4).elems.copy()
    e[0, 0] = -1e-3
    assert fwi.validate_problem(_prob(elems=e)) == fwi.FWI_E_INVAL          # outside
    p3 = W.small3d()
    assert fwi.validate_problem(p3) == fwi.FWI_OK
    p2 = _prob(ny=3)
    assert fwi.validate_problem(p2) == fwi.FWI_E_INVAL


def test_workspace_size_arithmetic():
    p = W.small2d(nx=24, nz=20, ne=4, nf=2)
    o64 = fwi.SolveOptions(precision=fwi.FWI_FP64, restart=16)
    o32 = fwi.SolveOptions(precision=fwi.FWI_FP32_REFINE, restart=16)
    f64 = fwi.workspace_size(p, o64, fwi.ENTRY_FORWARD)
    g64 = fwi.workspace_size(p, o64, fwi.ENTRY_GRADIENT)
    a64 = fwi.workspace_size(p, o64, fwi.ENTRY_ADMM)
    assert 0 < f64 < g64 and f64 < a64
    n, B, JM = p.n, p.nf * p.ne, 16
    # the Krylov basis dominates: (JM+1) B n complex entries
    assert f64 >= (JM + 1) * B * n * 16
    assert fwi.workspace_size(p, o32, fwi.ENTRY_FORWARD) >= (JM + 1) * B * n * 8
    # frequency grouping caps the batch
    og = fwi.SolveOptions(precision=fwi.FWI_FP64, restart=16, max_rhs=p.ne)
    assert fwi.workspace_size(p, og, fwi.ENTRY_FORWARD) < f64
    with pytest.raises(fwi.FWIError):
        fwi.workspace_size(p, fwi.SolveOptions(restart=12))
    with pytest.raises(fwi.FWIError):
        fwi.workspace_size(p, fwi.SolveOptions(rtol=2.0))


def test_aperture_rule_and_validation():
    """The library's Gauss-Legendre rule (host) against numpy's, and the
    aperture fields of the problem checked like the others."""
    for q in (1, 3, 8, 16):
        x, w = fwi.host_gauss_legendre(q)
        X, Wt = np.polynomial.legendre.leggauss(q)
        o = np.argsort(x)
        np.testing.assert_allclose(x[o], X, rtol=0, atol=1e-15)
        np.testing.assert_allclose(w[o], Wt, rtol=0, atol=1e-14)
    with pytest.raises(ValueError):
        fwi.host_gauss_legendre(17)
    assert fwi.validate_problem(_prob(elem_width=0.2e-3, elem_quad=4)) == fwi.FWI_OK
    assert fwi.validate_problem(_prob(elem_width=0.2e-3, elem_quad=0)) == fwi.FWI_E_INVAL
    assert fwi.validate_problem(_prob(elem_width=-1e-3, elem_quad=4)) == fwi.FWI_E_INVAL
    assert fwi.validate_problem(_prob(elem_height=1e-3, elem_quad=4)) == fwi.FWI_E_INVAL  # 2D: no height
    # lossy background
    assert fwi.validate_problem(_prob(alpha0=-1e-6)) == fwi.FWI_E_INVAL
    assert fwi.validate_problem(_prob(alpha0=1e-6)) == fwi.FWI_OK
    p3 = W.small3d()
    p3.alpha0 = 1e-6
    assert fwi.validate_problem(p3) == fwi.FWI_OK


def test_host_complex_bessel_and_hankel_match_scipy():
    """The complex-argument J0, J1, Y0, Y1 and H0^(1) of the lossy 2D
    background (the same code the kernels run) against scipy, from small
    arguments to the largest k r of the workloads, just above the real axis and
    further out."""
    L = fwi.lib()
    fb = L.fwi_host_cbessel01
    fb.restype, fb.argtypes = None, [C.c_double, C.c_double, C.POINTER(C.c_double)]
    fh = L.fwi_host_chankel0
    fh.restype, fh.argtypes = None, [C.c_double, C.c_double, C.POINTER(C.c_double)]
    o8, o2 = (C.c_double * 8)(), (C.c_double * 2)()
    for mag in np.geomspace(1e-3, 600, 120):
        for arg in (0.0, 1e-3, 0.01, 0.05) + ((0.3,) if mag < 40 else ()):
            z = mag * np.exp(1j * arg)
            fh(z.real, z.imag, o2)
            ref = sp.hankel1(0, z)
            tol = 1e-12 if arg <= 0.05 else 1e-9
            assert abs(o2[0] + 1j * o2[1] - ref) <= tol * abs(ref), z
            if mag < 25:
                fb(z.real, z.imag, o8)
                got = np.array(o8[:]).reshape(4, 2) @ np.array([1, 1j])
                want = np.array([sp.jv(0, z), sp.jv(1, z), sp.yv(0, z), sp.yv(1, z)])
                scale = np.maximum(np.abs(want), abs(sp.hankel1(0, z)))
                assert np.all(np.abs(got - want) <= 1e-11 * scale), z
