"""Python binding of libfwi.so (include/fwi.h).

Argument marshalling only: every step of the hot path runs in the HIP library.
PyTorch provides device memory (tensors, the workspace) and the HIP stream.
The library is loaded from this package directory; if it is missing, every
call raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfwi.so")

FWI_OK = 0
FWI_E_INVAL = -1
FWI_E_NOMEM = -2
FWI_E_NOCONV = -3
FWI_E_NONFINITE = -4
FWI_E_DEVICE = -5
FWI_E_UNSUPPORTED = -6
FWI_FP64 = 0
FWI_FP32_REFINE = 1
ENTRY_FORWARD, ENTRY_GRADIENT, ENTRY_ADMM = 0, 1, 2

ERROR_NAMES = {FWI_E_INVAL: "FWI_E_INVAL", FWI_E_NOMEM: "FWI_E_NOMEM", FWI_E_NOCONV: "FWI_E_NOCONV",
               FWI_E_NONFINITE: "FWI_E_NONFINITE", FWI_E_DEVICE: "FWI_E_DEVICE",
               FWI_E_UNSUPPORTED: "FWI_E_UNSUPPORTED"}


class FWIError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class CProblem(C.Structure):
    _fields_ = [("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx", C.c_double),
                ("c0", C.c_double), ("nf", C.c_int), ("freq_hz", C.POINTER(C.c_double)), ("ne", C.c_int),
                ("elem_xyz", C.POINTER(C.c_double)), ("elem_width", C.c_double), ("elem_height", C.c_double),
                ("elem_quad", C.c_int), ("alpha0", C.c_double)]


class CSolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("rtol", C.c_double), ("max_iter", C.c_int), ("restart", C.c_int),
                ("max_refine", C.c_int), ("inner_rtol", C.c_double), ("max_rhs", C.c_int),
                ("check_every", C.c_int), ("reciprocity_adjoint", C.c_int), ("fields_c64", C.c_int),
                ("tx_chunk", C.c_int)]


class CStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("cycles", C.c_int), ("unconverged", C.c_int),
                ("max_rel_residual", C.c_double), ("solves", C.c_longlong), ("matvecs", C.c_longlong),
                ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double), ("t_total_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CAdmmParams(C.Structure):
    _fields_ = [("lam", C.c_double), ("rho", C.c_double), ("gamma", C.c_double), ("n_cg", C.c_int),
                ("data_scale", C.c_double), ("dual_step", C.c_double), ("inv_factor", C.c_int)]


class CAdmmReport(C.Structure):
    _fields_ = [("misfit", C.c_double), ("tv", C.c_double), ("dm_norm", C.c_double)]


_lib = None


def lib():
    """Load libfwi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, ip, dp = C.c_void_p, C.c_int, C.POINTER(C.c_double)
    pp = C.POINTER(CProblem)
    op = C.POINTER(CSolveOpts)
    sp = C.POINTER(CStats)
    sig = {
        "fwi_create": (ip, [C.POINTER(vp), ip, vp]),
        "fwi_destroy": (None, [vp]),
        "fwi_last_error": (C.c_char_p, [vp]),
        "fwi_set_stream": (ip, [vp, vp]),
        "fwi_set_addressing": (ip, [vp, ip]),
        "fwi_set_plane_fusion": (ip, [vp, ip]),
        "fwi_default_opts": (None, [op]),
        "fwi_validate_problem": (ip, [pp]),
        "fwi_padded_length": (ip, [ip]),
        "fwi_workspace_size": (ip, [pp, op, ip, C.POINTER(C.c_size_t)]),
        "fwi_set_workspace": (ip, [vp, vp, C.c_size_t]),
        "fwi_forward": (ip, [vp, pp, vp, vp, op, vp, vp, sp]),
        "fwi_forward_m": (ip, [vp, pp, vp, op, vp, vp, sp]),
        "fwi_adjoint_gradient": (ip, [vp, pp, vp, vp, vp, op, dp, vp, vp, vp, sp]),
        "fwi_vjp": (ip, [vp, pp, vp, vp, op, vp, sp]),
        "fwi_vjp_fields": (ip, [vp, pp, vp, vp, vp, op, vp, sp]),
        "fwi_tv_admm_step": (ip, [vp, pp, C.POINTER(CAdmmParams), vp, vp, vp, vp, vp, op,
                                  C.POINTER(CAdmmReport), sp]),
        "fwi_apply_operator": (ip, [vp, pp, ip, vp, ip, C.POINTER(C.c_int), vp, vp]),
        "fwi_apply_operator_noalloc": (ip, [vp, pp, ip, vp, ip, C.POINTER(C.c_int), vp, vp]),
        "fwi_solve": (ip, [vp, pp, vp, ip, C.POINTER(C.c_int), vp, op, vp, sp]),
        "fwi_incident": (ip, [vp, pp, ip, vp]),
        "fwi_green_spectrum": (ip, [vp, pp, ip, vp]),
        "fwi_fft_padded": (ip, [vp, pp, ip, vp, vp]),
        "fwi_jacobian_apply": (ip, [vp, pp, vp, vp, vp]),
        "fwi_jacobian_adjoint_apply": (ip, [vp, pp, vp, vp, vp]),
        "fwi_forward_tx": (ip, [vp, pp, vp, vp, ip, vp, op, vp, vp, sp]),
        "fwi_adjoint_gradient_tx": (ip, [vp, pp, vp, vp, ip, vp, vp, op, dp, vp, vp, vp, sp]),
        "fwi_jacobian_apply_tx": (ip, [vp, pp, ip, vp, vp, vp, vp]),
        "fwi_invert": (ip, [vp, pp, C.POINTER(CAdmmParams), ip, C.c_double, ip, vp, vp, ip, vp, vp, vp, vp, vp, op,
                            dp, C.POINTER(C.c_int), sp]),
        "fwi_sos_from_contrast": (ip, [vp, pp, vp, vp, vp]),
        "fwi_tv_admm_step_tx": (ip, [vp, pp, C.POINTER(CAdmmParams), ip, vp, vp, ip, vp, vp, vp, vp, vp, op,
                                     C.POINTER(CAdmmReport), sp]),
        "fwi_jacobian_adjoint_apply_tx": (ip, [vp, pp, ip, vp, vp, vp, vp]),
        "fwi_host_bessel01": (None, [C.c_double, dp]),
        "fwi_host_gauss_legendre": (ip, [ip, dp, dp]),
        "fwi_profile": (ip, [vp, C.c_uint]),
        "fwi_profile_read": (ip, [vp, ip, dp, C.POINTER(C.c_longlong), dp]),
        "fwi_autotune": (ip, [vp, pp, ip, ip, ip, C.POINTER(CTuneReport)]),
        "fwi_adjoint_gradient_batch": (ip, [vp, ip, pp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), op, dp,
                                            C.POINTER(vp), C.POINTER(CBatchStats)]),
        "fwi_forward_batch": (ip, [vp, ip, pp, C.POINTER(vp), C.POINTER(vp), op, C.POINTER(vp),
                                   C.POINTER(CBatchStats)]),
        "fwi_autotune_solver": (ip, [vp, pp, vp, vp, vp, op, C.POINTER(C.c_int), ip, C.POINTER(C.c_int), ip,
                                     C.POINTER(C.c_double), ip, ip, C.POINTER(CSolverTuneReport)]),
        "fwi_get_tuning": (ip, [vp, C.POINTER(C.c_byte), ip]),
        "fwi_set_tuning": (ip, [vp, C.POINTER(C.c_byte), ip]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = ["fwi_create", "fwi_destroy", "fwi_last_error", "fwi_set_stream", "fwi_default_opts",
            "fwi_validate_problem", "fwi_padded_length", "fwi_workspace_size", "fwi_set_workspace",
            "fwi_forward", "fwi_forward_m", "fwi_adjoint_gradient", "fwi_vjp", "fwi_vjp_fields", "fwi_tv_admm_step",
            "fwi_apply_operator", "fwi_apply_operator_noalloc", "fwi_solve", "fwi_incident", "fwi_green_spectrum", "fwi_fft_padded",
            "fwi_jacobian_apply", "fwi_jacobian_adjoint_apply", "fwi_host_bessel01", "fwi_profile",
            "fwi_profile_read", "fwi_autotune", "fwi_get_tuning", "fwi_set_tuning", "fwi_adjoint_gradient_batch",
            "fwi_forward_batch", "fwi_set_addressing", "fwi_forward_tx", "fwi_adjoint_gradient_tx",
            "fwi_jacobian_apply_tx", "fwi_jacobian_adjoint_apply_tx", "fwi_tv_admm_step_tx", "fwi_invert",
            "fwi_sos_from_contrast", "fwi_host_gauss_legendre", "fwi_autotune_solver", "fwi_set_plane_fusion"]
TUNING_BYTES = 4 * 2 * 11
PASS_NAMES = ["row_fwd", "conv", "row_inv", "y_fwd", "y_inv"]

_BASE_CLASSES = ["row_fwd", "conv", "row_inv", "y_fwd", "y_inv", "dots", "orth", "orth_fwd"]
# class k: complex64 launches; class k + 7: complex128 launches
KERNEL_CLASSES = [f"{c}_c64" for c in _BASE_CLASSES] + [f"{c}_c128" for c in _BASE_CLASSES]


class CBatchStats(C.Structure):
    _fields_ = [("waves", C.c_int), ("graph_launches", C.c_int), ("iterations", C.c_int), ("unconverged", C.c_int),
                ("max_rel_residual", C.c_double), ("solves", C.c_longlong), ("t_setup_ms", C.c_double),
                ("t_solve_ms", C.c_double), ("t_total_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CTuneReport(C.Structure):
    _fields_ = [("variant_ms", (C.c_double * 3) * 5), ("variant", C.c_int * 5), ("default_variant", C.c_int * 5)]


class CSolverTuneReport(C.Structure):
    _fields_ = [("max_rhs", C.c_int), ("restart", C.c_int), ("inner_rtol", C.c_double),
                ("ms", ((C.c_double * 3) * 8) * 3)]


# ---------------------------------------------------------------- structs ---
class ProblemArgs:
    """Host-side fwi_problem built from any object with dim, nx, ny, nz, dx, c0,
    freqs, elems (e.g. workloads.Problem); keeps its arrays alive."""

    def __init__(self, p):
        self.dim, self.nx, self.ny, self.nz = int(p.dim), int(p.nx), int(p.ny), int(p.nz)
        self.dx, self.c0 = float(p.dx), float(p.c0)
        self.freqs = np.ascontiguousarray(np.asarray(p.freqs, dtype=np.float64))
        self.elems = np.ascontiguousarray(np.asarray(p.elems, dtype=np.float64).reshape(-1, 3))
        self.nf, self.ne = len(self.freqs), self.elems.shape[0]
        self.n = self.nx * self.ny * self.nz
        # element aperture (point elements when absent)
        self.elem_width = float(getattr(p, "elem_width", 0.0))
        self.elem_height = float(getattr(p, "elem_height", 0.0))
        self.elem_quad = int(getattr(p, "elem_quad", 1))
        self.alpha0 = float(getattr(p, "alpha0", 0.0))  # background attenuation [Np/m/Hz]
        self.c = CProblem(self.dim, self.nx, self.ny, self.nz, self.dx, self.c0, self.nf,
                          self.freqs.ctypes.data_as(C.POINTER(C.c_double)), self.ne,
                          self.elems.ctypes.data_as(C.POINTER(C.c_double)), self.elem_width, self.elem_height,
                          self.elem_quad, self.alpha0)

    @property
    def shape(self):
        return (self.nz, self.nx) if self.dim == 2 else (self.nz, self.ny, self.nx)

    def ref(self):
        return C.byref(self.c)


@dataclass
class SolveOptions:
    precision: int = FWI_FP64
    rtol: float = 1e-10
    max_iter: int = 2000
    restart: int = 32
    max_refine: int = 12
    inner_rtol: float = 1e-3
    max_rhs: int = 0
    check_every: int = 1
    reciprocity_adjoint: int = 0
    fields_c64: int = 0
    tx_chunk: int = 0

    def c(self):
        return CSolveOpts(self.precision, self.rtol, self.max_iter, self.restart, self.max_refine,
                          self.inner_rtol, self.max_rhs, self.check_every, self.reciprocity_adjoint,
                          self.fields_c64, self.tx_chunk)


def _field_dtype(o):
    """dtype of the fields_out array of the forward entries under options o."""
    return torch.complex64 if o.fields_c64 else torch.complex128


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def inversion_shape(prob, r):
    """Shape of the inversion mesh r times coarser than the forward mesh."""
    if r <= 1:
        return prob.shape
    cz, cx = -(-prob.nz // r), -(-prob.nx // r)
    return (cz, cx) if prob.dim == 2 else (cz, -(-prob.ny // r), cx)


def _check_dtype(t, dtype, shape, what):
    if t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape) and t.numel() != int(np.prod(shape)):
        raise ValueError(f"{what}: expected shape {shape}, got {tuple(t.shape)}")


class Context:
    """One fwi_ctx bound to a HIP device; calls run on torch's current stream."""

    def __init__(self, device=0, use_torch_workspace=True):
        self.L = lib()
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        rc = self.L.fwi_create(C.byref(h), device, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
        if rc != FWI_OK:
            raise FWIError(rc, "fwi_create failed")
        self.h = h
        self.use_torch_workspace = use_torch_workspace
        self._ws = None

    def close(self):
        if getattr(self, "h", None):
            self.L.fwi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_noconv=False):
        if rc == FWI_OK or (allow_noconv and rc == FWI_E_NOCONV):
            return rc
        raise FWIError(rc, self.L.fwi_last_error(self.h).decode())

    def _stream(self):
        self.L.fwi_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _workspace(self, prob, opts, entry):
        if not self.use_torch_workspace:
            self.L.fwi_set_workspace(self.h, None, 0)
            return
        nbytes = C.c_size_t()
        self._check(self.L.fwi_workspace_size(prob.ref(), C.byref(opts), entry, C.byref(nbytes)))
        if self._ws is None or self._ws.numel() < nbytes.value:
            self._ws = None
            self._ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=self.device)
        self.L.fwi_set_workspace(self.h, C.c_void_p(self._ws.data_ptr()), self._ws.numel())

    def _internal_workspace(self):
        self.L.fwi_set_workspace(self.h, None, 0)

    def release_workspace(self):
        self._internal_workspace()
        self._ws = None

    # ------------------------------------------------------------ entries ---
    def forward(self, prob, c, alpha=None, opts=None, fields=False, allow_noconv=False):
        """Scattered data [nf, ne, ne] (and fields [nf, ne, n]) for c, alpha grids."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        _check_dtype(c, torch.float64, prob.shape, "c")
        if alpha is not None:
            _check_dtype(alpha, torch.float64, prob.shape, "alpha")
        data = torch.empty((prob.nf, prob.ne, prob.ne), dtype=torch.complex128, device=self.device)
        F = torch.empty((prob.nf, prob.ne, prob.n), dtype=_field_dtype(o), device=self.device) if fields else None
        st = CStats()
        self._stream()
        self._workspace(prob, o, ENTRY_FORWARD)
        rc = self.L.fwi_forward(self.h, prob.ref(), _ptr(c), _ptr(alpha), C.byref(o), _ptr(data), _ptr(F),
                                C.byref(st))
        self._check(rc, allow_noconv)
        return (data, F, st.as_dict()) if fields else (data, st.as_dict())

    def forward_m(self, prob, m, opts=None, fields=False, allow_noconv=False):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        _check_dtype(m, torch.complex128, prob.shape, "m")
        data = torch.empty((prob.nf, prob.ne, prob.ne), dtype=torch.complex128, device=self.device)
        F = torch.empty((prob.nf, prob.ne, prob.n), dtype=_field_dtype(o), device=self.device) if fields else None
        st = CStats()
        self._stream()
        self._workspace(prob, o, ENTRY_FORWARD)
        rc = self.L.fwi_forward_m(self.h, prob.ref(), _ptr(m), C.byref(o), _ptr(data), _ptr(F), C.byref(st))
        self._check(rc, allow_noconv)
        return (data, F, st.as_dict()) if fields else (data, st.as_dict())

    def adjoint_gradient(self, prob, c, alpha, d_obs, opts=None, chain=True, allow_noconv=False):
        """(misfit, grad_m [n] complex, grad_c [n], grad_alpha [n], stats)."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        _check_dtype(c, torch.float64, prob.shape, "c")
        _check_dtype(d_obs, torch.complex128, (prob.nf, prob.ne, prob.ne), "d_obs")
        gm = torch.empty(prob.n, dtype=torch.complex128, device=self.device)
        gc = torch.empty(prob.n, dtype=torch.float64, device=self.device) if chain else None
        ga = torch.empty(prob.n, dtype=torch.float64, device=self.device) if chain else None
        phi = C.c_double()
        st = CStats()
        self._stream()
        self._workspace(prob, o, ENTRY_GRADIENT)
        rc = self.L.fwi_adjoint_gradient(self.h, prob.ref(), _ptr(c), _ptr(alpha), _ptr(d_obs), C.byref(o),
                                         C.byref(phi), _ptr(gm), _ptr(gc), _ptr(ga), C.byref(st))
        self._check(rc, allow_noconv)
        return phi.value, gm, gc, ga, st.as_dict()

    # ------------------------------------------- synthesised transmits ---
    def _tx_weights(self, prob, w):
        if w.dtype != torch.complex128 or w.dim() != 3 or w.shape[0] != prob.nf or w.shape[2] != prob.ne:
            raise ValueError(f"tx_weights: expected complex128 [nf={prob.nf}, nt, ne={prob.ne}], "
                             f"got {w.dtype} {tuple(w.shape)}")
        if not w.is_contiguous():
            raise ValueError("tx_weights must be contiguous")
        return int(w.shape[1])

    def forward_tx(self, prob, c, alpha, w, opts=None, fields=False, allow_noconv=False):
        """Data [nf, nt, ne] (and fields [nf, nt, n]) of transmits with element
        weights w [nf, nt, ne] (complex128, device)."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        _check_dtype(c, torch.float64, prob.shape, "c")
        nt = self._tx_weights(prob, w)
        data = torch.empty((prob.nf, nt, prob.ne), dtype=torch.complex128, device=self.device)
        F = torch.empty((prob.nf, nt, prob.n), dtype=_field_dtype(o), device=self.device) if fields else None
        st = CStats()
        self._stream()
        self._workspace(prob, o, ENTRY_GRADIENT)
        rc = self.L.fwi_forward_tx(self.h, prob.ref(), _ptr(c), _ptr(alpha), nt, _ptr(w), C.byref(o), _ptr(data),
                                   _ptr(F), C.byref(st))
        self._check(rc, allow_noconv)
        return (data, F, st.as_dict()) if fields else (data, st.as_dict())

    def adjoint_gradient_tx(self, prob, c, alpha, w, d_obs, opts=None, allow_noconv=False):
        """(misfit, grad_m [n] complex, grad_c [n], grad_alpha [n], stats) for
        transmits with element weights w [nf, nt, ne]; d_obs [nf, nt, ne]."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        _check_dtype(c, torch.float64, prob.shape, "c")
        nt = self._tx_weights(prob, w)
        _check_dtype(d_obs, torch.complex128, (prob.nf, nt, prob.ne), "d_obs")
        gm = torch.empty(prob.n, dtype=torch.complex128, device=self.device)
        gc = torch.empty(prob.n, dtype=torch.float64, device=self.device)
        ga = torch.empty(prob.n, dtype=torch.float64, device=self.device)
        phi = C.c_double()
        st = CStats()
        self._stream()
        self._workspace(prob, o, ENTRY_GRADIENT)
        rc = self.L.fwi_adjoint_gradient_tx(self.h, prob.ref(), _ptr(c), _ptr(alpha), nt, _ptr(w), _ptr(d_obs),
                                            C.byref(o), C.byref(phi), _ptr(gm), _ptr(gc), _ptr(ga), C.byref(st))
        self._check(rc, allow_noconv)
        return phi.value, gm, gc, ga, st.as_dict()

    def jacobian_apply_tx(self, prob, tx_fields, rx_fields, a):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        nt = int(tx_fields.shape[1])
        _check_dtype(tx_fields, torch.complex128, (prob.nf, nt, prob.n), "tx_fields")
        _check_dtype(rx_fields, torch.complex128, (prob.nf, prob.ne, prob.n), "rx_fields")
        out = torch.empty((prob.nf, nt, prob.ne), dtype=torch.complex128, device=self.device)
        self._stream()
        self._internal_workspace()
        self._check(self.L.fwi_jacobian_apply_tx(self.h, prob.ref(), nt, _ptr(tx_fields), _ptr(rx_fields), _ptr(a),
                                                 _ptr(out)))
        return out

    def jacobian_adjoint_apply_tx(self, prob, tx_fields, rx_fields, b):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        nt = int(tx_fields.shape[1])
        _check_dtype(tx_fields, torch.complex128, (prob.nf, nt, prob.n), "tx_fields")
        _check_dtype(rx_fields, torch.complex128, (prob.nf, prob.ne, prob.n), "rx_fields")
        _check_dtype(b, torch.complex128, (prob.nf, nt, prob.ne), "b")
        out = torch.empty(prob.n, dtype=torch.complex128, device=self.device)
        self._stream()
        self._internal_workspace()
        self._check(self.L.fwi_jacobian_adjoint_apply_tx(self.h, prob.ref(), nt, _ptr(tx_fields), _ptr(rx_fields),
                                                         _ptr(b), _ptr(out)))
        return out

    def vjp(self, prob, m, grad_data, opts=None, allow_noconv=False):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        _check_dtype(m, torch.complex128, prob.shape, "m")
        _check_dtype(grad_data, torch.complex128, (prob.nf, prob.ne, prob.ne), "grad_data")
        gm = torch.empty(prob.n, dtype=torch.complex128, device=self.device)
        st = CStats()
        self._stream()
        self._workspace(prob, o, ENTRY_GRADIENT)
        rc = self.L.fwi_vjp(self.h, prob.ref(), _ptr(m), _ptr(grad_data), C.byref(o), _ptr(gm), C.byref(st))
        self._check(rc, allow_noconv)
        return gm, st.as_dict()

    def vjp_fields(self, prob, m, fields, grad_data, opts=None, allow_noconv=False):
        """J^H grad_data with the forward fields [nf, ne, n] given (complex128,
        from forward_m at the same m): adjoint solves only."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        _check_dtype(m, torch.complex128, prob.shape, "m")
        _check_dtype(fields, torch.complex128, (prob.nf, prob.ne, prob.n), "fields")
        _check_dtype(grad_data, torch.complex128, (prob.nf, prob.ne, prob.ne), "grad_data")
        gm = torch.empty(prob.n, dtype=torch.complex128, device=self.device)
        st = CStats()
        self._stream()
        self._workspace(prob, o, ENTRY_GRADIENT)
        rc = self.L.fwi_vjp_fields(self.h, prob.ref(), _ptr(m), _ptr(fields), _ptr(grad_data), C.byref(o), _ptr(gm),
                                   C.byref(st))
        self._check(rc, allow_noconv)
        return gm, st.as_dict()

    def tv_admm_step(self, prob, m, g, u, d_obs, lam, rho, gamma=0.0, n_cg=10, m_ref=None, data_scale=0.0,
                     dual_step=None, opts=None, allow_noconv=False, inv_factor=1):
        """One ADMM iteration; m, g, u (complex128 device tensors, on the
        inversion mesh when inv_factor > 1) are updated in place."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        shp = inversion_shape(prob, inv_factor)
        _check_dtype(m, torch.complex128, shp, "m")
        _check_dtype(g, torch.complex128, (prob.dim,) + shp, "g")
        _check_dtype(u, torch.complex128, (prob.dim,) + shp, "u")
        prm = CAdmmParams(lam, rho, gamma, n_cg, data_scale, rho if dual_step is None else dual_step, inv_factor)
        rep = CAdmmReport()
        st = CStats()
        self._stream()
        self._workspace(prob, o, ENTRY_ADMM)
        rc = self.L.fwi_tv_admm_step(self.h, prob.ref(), C.byref(prm), _ptr(m), _ptr(g), _ptr(u), _ptr(m_ref),
                                     _ptr(d_obs), C.byref(o), C.byref(rep), C.byref(st))
        self._check(rc, allow_noconv)
        return {"misfit": rep.misfit, "tv": rep.tv, "dm_norm": rep.dm_norm}, st.as_dict()

    def tv_admm_step_tx(self, prob, w, rx_fields, m, g, u, d_obs, lam, rho, gamma=0.0, n_cg=10, m_ref=None,
                        data_scale=0.0, dual_step=None, refresh_rx=True, opts=None, allow_noconv=False):
        """One ADMM iteration with synthesised transmits (weights w [nf, nt, ne]);
        rx_fields [nf, ne, n] complex128 are recomputed at m (refresh_rx) or used
        as given (Born reuse). m, g, u, rx_fields are updated in place."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        nt = self._tx_weights(prob, w)
        _check_dtype(m, torch.complex128, prob.shape, "m")
        _check_dtype(g, torch.complex128, (prob.dim,) + prob.shape, "g")
        _check_dtype(u, torch.complex128, (prob.dim,) + prob.shape, "u")
        _check_dtype(rx_fields, torch.complex128, (prob.nf, prob.ne, prob.n), "rx_fields")
        _check_dtype(d_obs, torch.complex128, (prob.nf, nt, prob.ne), "d_obs")
        prm = CAdmmParams(lam, rho, gamma, n_cg, data_scale, rho if dual_step is None else dual_step, 1)
        rep = CAdmmReport()
        st = CStats()
        self._stream()
        self._workspace(prob, o, ENTRY_ADMM)
        rc = self.L.fwi_tv_admm_step_tx(self.h, prob.ref(), C.byref(prm), nt, _ptr(w), _ptr(rx_fields),
                                        1 if refresh_rx else 0, _ptr(m), _ptr(g), _ptr(u), _ptr(m_ref), _ptr(d_obs),
                                        C.byref(o), C.byref(rep), C.byref(st))
        self._check(rc, allow_noconv)
        return {"misfit": rep.misfit, "tv": rep.tv, "dm_norm": rep.dm_norm}, st.as_dict()

    def invert(self, prob, m, d_obs, lam, rho, gamma=0.0, n_cg=10, max_iter=20, tol=0.0, m_ref=None,
               data_scale=0.0, dual_step=None, w=None, born_every=0, opts=None, allow_noconv=False, inv_factor=1):
        """Algorithm 1 from m (complex128 device tensor, updated in place): up to
        max_iter ADMM iterations, stopping once the misfit at an iterate is
        <= tol * 1/2 ||d_obs||^2. w [nf, nt, ne]: synthesised transmits with
        receiver fields refreshed every born_every iterations. Returns
        (misfit per iteration, g, u, stats)."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        shp = inversion_shape(prob, inv_factor)
        _check_dtype(m, torch.complex128, shp, "m")
        nt = self._tx_weights(prob, w) if w is not None else 0
        _check_dtype(d_obs, torch.complex128, (prob.nf, nt or prob.ne, prob.ne), "d_obs")
        g = torch.empty((prob.dim,) + shp, dtype=torch.complex128, device=self.device)
        u = torch.empty_like(g)
        rx = torch.empty((prob.nf, prob.ne, prob.n), dtype=torch.complex128, device=self.device) if nt else None
        prm = CAdmmParams(lam, rho, gamma, n_cg, data_scale, rho if dual_step is None else dual_step, inv_factor)
        hist = (C.c_double * max(max_iter, 1))()
        done = C.c_int()
        st = CStats()
        self._stream()
        self._workspace(prob, o, ENTRY_ADMM)
        rc = self.L.fwi_invert(self.h, prob.ref(), C.byref(prm), max_iter, tol, nt, _ptr(w), _ptr(rx), born_every,
                               _ptr(m), _ptr(g), _ptr(u), _ptr(m_ref), _ptr(d_obs), C.byref(o), hist, C.byref(done),
                               C.byref(st))
        self._check(rc, allow_noconv)
        return list(hist)[:done.value], g, u, st.as_dict()

    def sos_from_contrast(self, prob, m):
        """(c [n], alpha [n]) float64 device tensors: the inverse of Eq. 1-3."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        _check_dtype(m, torch.complex128, prob.shape, "m")
        c = torch.empty(prob.shape, dtype=torch.float64, device=self.device)
        a = torch.empty_like(c)
        self._stream()
        self._check(self.L.fwi_sos_from_contrast(self.h, prob.ref(), _ptr(m), _ptr(c), _ptr(a)))
        return c, a

    def profile(self, classes):
        """Start HIP-event timing of the named kernel classes (empty: stop)."""
        mask = 0
        for name in classes:
            mask |= 1 << KERNEL_CLASSES.index(name)
        self._check(self.L.fwi_profile(self.h, mask))

    def profile_read(self):
        out = {}
        for k, name in enumerate(KERNEL_CLASSES):
            t, n, b = C.c_double(), C.c_longlong(), C.c_double()
            self._check(self.L.fwi_profile_read(self.h, k, C.byref(t), C.byref(n), C.byref(b)))
            if n.value:
                out[name] = {"ms": t.value, "launches": n.value, "bytes": b.value}
        return out

    def autotune(self, prob, precision=FWI_FP32_REFINE, B=64, reps=3):
        """Time every tile variant of every FFT pass for this grid on the device and
        keep the fastest in the context. Returns {pass: {"ms": [..3], "chosen", "default"}}."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        rep = CTuneReport()
        self._stream()
        self._internal_workspace()
        self._check(self.L.fwi_autotune(self.h, prob.ref(), precision, B, reps, C.byref(rep)))
        out = {}
        for k, name in enumerate(PASS_NAMES):
            ms = [rep.variant_ms[k][v] for v in range(3)]
            if any(ms):
                out[name] = {"ms": ms, "chosen": rep.variant[k], "default": rep.default_variant[k]}
        return out

    def autotune_solver(self, prob, c, alpha, d_obs, opts=None, max_rhs=(0,), restart=(8,), inner_rtol=None,
                        reps=1):
        """Time the gradient step for every (max_rhs, restart, inner_rtol)
        combination (inner_rtol=None: the options' own) and return
        {"max_rhs", "restart", "inner_rtol" (the fastest),
        "ms": {(max_rhs, restart, inner_rtol): ms}}.
        Uses the library's own workspace; the context's tuning is unchanged."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        _check_dtype(c, torch.float64, prob.shape, "c")
        _check_dtype(d_obs, torch.complex128, (prob.nf, prob.ne, prob.ne), "d_obs")
        mr = (C.c_int * len(max_rhs))(*[int(v) for v in max_rhs])
        rs = (C.c_int * len(restart))(*[int(v) for v in restart])
        inner = [float(o.inner_rtol)] if inner_rtol is None else [float(v) for v in inner_rtol]
        ir = None if inner_rtol is None else (C.c_double * len(inner))(*inner)
        rep = CSolverTuneReport()
        self._stream()
        self._internal_workspace()
        self._check(self.L.fwi_autotune_solver(self.h, prob.ref(), _ptr(c), _ptr(alpha), _ptr(d_obs), C.byref(o),
                                               mr, len(max_rhs), rs, len(restart), ir, len(inner), reps,
                                               C.byref(rep)))
        ms = {(int(a), int(b), t): rep.ms[h][i][j] for h, t in enumerate(inner)
              for i, a in enumerate(max_rhs) for j, b in enumerate(restart)}
        return {"max_rhs": rep.max_rhs, "restart": rep.restart, "inner_rtol": rep.inner_rtol, "ms": ms}

    def set_addressing(self, wide):
        """wide=True forces the 64-bit addressing path of the strided FFT passes
        (otherwise used only for planes of 2 GiB or more)."""
        self._check(self.L.fwi_set_addressing(self.h, 1 if wide else 0))

    def set_plane_fusion(self, on):
        """on=True: the 3D complex64 operator uses the fused per-plane
        lateral-elevation pass where the grid allows it (off by default)."""
        self._check(self.L.fwi_set_plane_fusion(self.h, 1 if on else 0))

    def get_tuning(self):
        buf = (C.c_byte * TUNING_BYTES)()
        self._check(self.L.fwi_get_tuning(self.h, buf, TUNING_BYTES))
        return bytes(bytearray(buf))

    def set_tuning(self, table=None):
        if table is None:
            self._check(self.L.fwi_set_tuning(self.h, None, 0))
            return
        buf = (C.c_byte * TUNING_BYTES).from_buffer_copy(bytes(table))
        self._check(self.L.fwi_set_tuning(self.h, buf, TUNING_BYTES))

    # ----------------------------------------------------------- batches ---
    def _batch_args(self, probs, cs, alphas):
        pas = [p if isinstance(p, ProblemArgs) else ProblemArgs(p) for p in probs]
        arr = (CProblem * len(pas))(*[pa.c for pa in pas])
        for pa, c_ in zip(pas, cs):
            _check_dtype(c_, torch.float64, pa.shape, "c")
        cp = (C.c_void_p * len(pas))(*[t.data_ptr() for t in cs])
        ap = None
        if alphas is not None:
            ap = (C.c_void_p * len(pas))(*[t.data_ptr() for t in alphas])
        return pas, arr, cp, ap

    def forward_batch(self, probs, cs, alphas=None, opts=None, allow_noconv=False):
        """Data of many problems of different shapes, solved together (list of [nf, ne, ne])."""
        pas, arr, cp, ap = self._batch_args(probs, cs, alphas)
        o = (opts or SolveOptions()).c()
        outs = [torch.empty((pa.nf, pa.ne, pa.ne), dtype=torch.complex128, device=self.device) for pa in pas]
        op_ = (C.c_void_p * len(pas))(*[t.data_ptr() for t in outs])
        st = CBatchStats()
        self._stream()
        self._internal_workspace()
        rc = self.L.fwi_forward_batch(self.h, len(pas), arr, cp, ap, C.byref(o), op_, C.byref(st))
        self._check(rc, allow_noconv)
        return outs, st.as_dict()

    def adjoint_gradient_batch(self, probs, cs, alphas, d_obs, opts=None, allow_noconv=False):
        """(misfits [ninst], gradients list of [n] complex, stats) for many problems."""
        pas, arr, cp, ap = self._batch_args(probs, cs, alphas)
        o = (opts or SolveOptions()).c()
        dp_ = (C.c_void_p * len(pas))(*[t.data_ptr() for t in d_obs])
        grads = [torch.empty(pa.n, dtype=torch.complex128, device=self.device) for pa in pas]
        gp = (C.c_void_p * len(pas))(*[t.data_ptr() for t in grads])
        mis = (C.c_double * len(pas))()
        st = CBatchStats()
        self._stream()
        self._internal_workspace()
        rc = self.L.fwi_adjoint_gradient_batch(self.h, len(pas), arr, cp, ap, dp_, C.byref(o), mis, gp,
                                               C.byref(st))
        self._check(rc, allow_noconv)
        return list(mis), grads, st.as_dict()

    # ---------------------------------------------------- building blocks ---
    def apply_operator(self, prob, m, freq_index, x, precision=FWI_FP64):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        fi = np.ascontiguousarray(np.asarray(freq_index, dtype=np.int32))
        dt = torch.complex64 if precision == FWI_FP32_REFINE else torch.complex128
        _check_dtype(x, dt, (len(fi), prob.n), "x")
        y = torch.empty_like(x)
        self._stream()
        self._internal_workspace()
        rc = self.L.fwi_apply_operator(self.h, prob.ref(), precision, _ptr(m), len(fi),
                                       fi.ctypes.data_as(C.POINTER(C.c_int)), _ptr(x), _ptr(y))
        self._check(rc)
        return y

    def apply_operator_noalloc(self, prob, m, freq_index, x, precision=FWI_FP64):
        """apply_operator with the library's static scratch (allocates nothing on
        the device; the problem's spectra must already be cached)."""
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        fi = np.ascontiguousarray(np.asarray(freq_index, dtype=np.int32))
        dt = torch.complex64 if precision == FWI_FP32_REFINE else torch.complex128
        _check_dtype(x, dt, (len(fi), prob.n), "x")
        y = torch.empty_like(x)
        self._stream()
        rc = self.L.fwi_apply_operator_noalloc(self.h, prob.ref(), precision, _ptr(m), len(fi),
                                               fi.ctypes.data_as(C.POINTER(C.c_int)), _ptr(x), _ptr(y))
        self._check(rc)
        return y

    def solve(self, prob, m, freq_index, rhs, opts=None, allow_noconv=False):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        o = (opts or SolveOptions()).c()
        fi = np.ascontiguousarray(np.asarray(freq_index, dtype=np.int32))
        x = torch.empty_like(rhs)
        st = CStats()
        self._stream()
        self._internal_workspace()
        rc = self.L.fwi_solve(self.h, prob.ref(), _ptr(m), len(fi), fi.ctypes.data_as(C.POINTER(C.c_int)),
                              _ptr(rhs), C.byref(o), _ptr(x), C.byref(st))
        self._check(rc, allow_noconv)
        return x, st.as_dict()

    def incident(self, prob, l):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        out = torch.empty((prob.ne, prob.n), dtype=torch.complex128, device=self.device)
        self._stream()
        self._check(self.L.fwi_incident(self.h, prob.ref(), l, _ptr(out)))
        return out

    def padded_shape(self, prob):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        Lx, Lz = self.L.fwi_padded_length(prob.nx), self.L.fwi_padded_length(prob.nz)
        if prob.dim == 2:
            return (Lz, Lx)
        return (Lz, self.L.fwi_padded_length(prob.ny), Lx)

    def green_spectrum(self, prob, l):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        out = torch.empty(self.padded_shape(prob), dtype=torch.complex128, device=self.device)
        self._stream()
        self._check(self.L.fwi_green_spectrum(self.h, prob.ref(), l, _ptr(out)))
        return out

    def fft_padded(self, prob, x, precision=FWI_FP64):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        dt = torch.complex64 if precision == FWI_FP32_REFINE else torch.complex128
        out = torch.empty(self.padded_shape(prob), dtype=dt, device=self.device)
        self._stream()
        self._internal_workspace()
        self._check(self.L.fwi_fft_padded(self.h, prob.ref(), precision, _ptr(x), _ptr(out)))
        return out

    def jacobian_apply(self, prob, fields, a):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        out = torch.empty((prob.nf, prob.ne, prob.ne), dtype=torch.complex128, device=self.device)
        self._stream()
        self._internal_workspace()
        self._check(self.L.fwi_jacobian_apply(self.h, prob.ref(), _ptr(fields), _ptr(a), _ptr(out)))
        return out

    def jacobian_adjoint_apply(self, prob, fields, b):
        prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
        out = torch.empty(prob.n, dtype=torch.complex128, device=self.device)
        self._stream()
        self._internal_workspace()
        self._check(self.L.fwi_jacobian_adjoint_apply(self.h, prob.ref(), _ptr(fields), _ptr(b), _ptr(out)))
        return out


def host_gauss_legendre(q):
    """(nodes, weights) of the library's q-point element-aperture rule."""
    x, w = (C.c_double * q)(), (C.c_double * q)()
    if lib().fwi_host_gauss_legendre(q, x, w) != 0:
        raise ValueError("q must be in 1..16")
    return np.array(x[:]), np.array(w[:])


def host_bessel01(x):
    """{J0, J1, Y0, Y1}(x) from the library's own FP64 routine (host evaluation)."""
    out = (C.c_double * 4)()
    lib().fwi_host_bessel01(float(x), out)
    return np.array(out[:])


def validate_problem(p):
    pa = p if isinstance(p, ProblemArgs) else ProblemArgs(p)
    return lib().fwi_validate_problem(pa.ref())


def workspace_size(p, opts=None, entry=ENTRY_FORWARD):
    pa = p if isinstance(p, ProblemArgs) else ProblemArgs(p)
    o = (opts or SolveOptions()).c()
    nb = C.c_size_t()
    rc = lib().fwi_workspace_size(pa.ref(), C.byref(o), entry, C.byref(nb))
    if rc != FWI_OK:
        raise FWIError(rc, "fwi_workspace_size failed")
    return nb.value


# ------------------------------------------------------------- autograd ---
class FWIData(torch.autograd.Function):
    """d = F(m) with the adjoint-state backward J^H grad_d (Eq. 17): adjoint
    solves in the library with the forward fields either kept from the
    forward pass (when they fit `store_bytes`) or recomputed in the backward
    (in the frequency groups and transmit chunks of the options, so that
    never all fields are held). Both give the same gradient bit for bit."""

    @staticmethod
    def forward(ctx, m, context, prob, opts, store_bytes):
        need = prob.nf * prob.ne * prob.n * 16
        if store_bytes is None:
            store_bytes = torch.cuda.mem_get_info(context.device)[0] // 4
        store = need <= store_bytes
        o = opts if not opts.fields_c64 else SolveOptions(**{**opts.__dict__, "fields_c64": 0})
        if store:
            data, fields, _ = context.forward_m(prob, m.contiguous(), o, fields=True)
            ctx.save_for_backward(m, fields)
        else:
            data, _ = context.forward_m(prob, m.contiguous(), o)
            ctx.save_for_backward(m)
        ctx.fwi = (context, prob, o, store)
        return data

    @staticmethod
    def backward(ctx, grad_data):
        context, prob, opts, store = ctx.fwi
        b = grad_data.contiguous().to(torch.complex128)
        if store:
            m, fields = ctx.saved_tensors
            gm, _ = context.vjp_fields(prob, m.contiguous(), fields, b, opts)
        else:
            (m,) = ctx.saved_tensors
            gm, _ = context.vjp(prob, m.contiguous(), b, opts)
        return gm.reshape(m.shape), None, None, None, None


def fwi_data(m, context, prob, opts=None, store_bytes=None):
    """Differentiable forward model d = F(m) (complex128). store_bytes: device
    bytes the forward fields may occupy between the forward and the backward
    pass (None: a quarter of the free device memory; 0: always recompute)."""
    prob = prob if isinstance(prob, ProblemArgs) else ProblemArgs(prob)
    return FWIData.apply(m, context, prob, opts or SolveOptions(), store_bytes)
