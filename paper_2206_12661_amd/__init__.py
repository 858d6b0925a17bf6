"""Python binding of the gfx950 GSW-MTP library (``libgswmtp.so``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides the HIP runtime, device memory for the
``*_device`` calls and the stream every call is ordered on.  There is no CPU
fallback: importing this package without the built library raises.

The method is the weighted Gerchberg-Saxton iteration of Liu et al., "Fast
generation of arbitrary optical focus array" (arXiv:2206.12661, Algorithm 1)
with the matrix-triple-product diffraction operator of its Eq. 2.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch  # loads the HIP runtime the library binds to; must precede the CDLL

HERE = os.path.dirname(os.path.abspath(__file__))
# GSWMTP_LIBRARY names another build of the same library (the sanitized
# host-only build the CPU tests use); it must exist like the default one.
LIB_PATH = os.environ.get("GSWMTP_LIBRARY") or os.path.join(HERE, "libgswmtp.so")

FP32, BF16X3, FP16X3, BF16X6 = 0, 1, 2, 3
PRECISIONS = {"fp32": FP32, "bf16x3": BF16X3, "fp16x3": FP16X3, "bf16x6": BF16X6}
WEIGHT_GSW, WEIGHT_GS = 0, 1
N_STAGES = 5
STAGES = ("forward_product", "focus_update", "scatter", "adjoint_product_project",
          "adjoint_split_k_tail")

STATUS = {0: "OK", -1: "E_INVAL", -2: "E_DUPFOCUS", -3: "E_EMPTYAPERTURE", -4: "E_NOMEM",
          -5: "E_HIP", -6: "E_NONFINITE", -7: "E_NODEV", -8: "E_UNSUPPORTED"}


class GswmtpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class gswmtp_desc(ctypes.Structure):
    _fields_ = [
        ("ny", ctypes.c_int), ("nx", ctypes.c_int),
        ("amplitude", ctypes.c_void_p), ("mask", ctypes.c_void_p),
        ("u", ctypes.c_void_p), ("v", ctypes.c_void_p),
        ("s_x", ctypes.c_double), ("s_y", ctypes.c_double),
        ("n_foci", ctypes.c_int),
        ("fx", ctypes.c_void_p), ("fy", ctypes.c_void_p), ("target", ctypes.c_void_p),
        ("phi0", ctypes.c_void_p),
        ("precision", ctypes.c_int), ("axis", ctypes.c_int), ("weighting", ctypes.c_int),
        ("fz", ctypes.c_void_p),
    ]


class gswmtp_index_info(ctypes.Structure):
    _fields_ = [
        ("n_foci", ctypes.c_int), ("ux", ctypes.c_int), ("uy", ctypes.c_int),
        ("ny_kept", ctypes.c_int), ("nx_kept", ctypes.c_int), ("axis", ctypes.c_int),
        ("n_aperture", ctypes.c_int), ("sum_a2", ctypes.c_double),
    ]


_MAX_CAND = 8


class gswmtp_batch_class(ctypes.Structure):
    _fields_ = [
        ("product", ctypes.c_int), ("m", ctypes.c_int), ("n", ctypes.c_int), ("k", ctypes.c_int),
        ("n_plans", ctypes.c_int), ("config", ctypes.c_int * 6), ("ms", ctypes.c_double),
        ("source", ctypes.c_int), ("n_tried", ctypes.c_int),
        ("tried_config", (ctypes.c_int * 6) * _MAX_CAND),
        ("tried_ms", ctypes.c_double * _MAX_CAND),
    ]


_P = ctypes.c_void_p
_SIGNATURES = {
    "gswmtp_version": ([], ctypes.c_int),
    "gswmtp_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "gswmtp_last_error": ([_P], ctypes.c_char_p),
    "gswmtp_desc_init": ([ctypes.POINTER(gswmtp_desc)], ctypes.c_int),
    "gswmtp_plan_create": ([ctypes.POINTER(_P), ctypes.POINTER(gswmtp_desc), _P], ctypes.c_int),
    "gswmtp_plan_workspace_size": ([ctypes.POINTER(gswmtp_desc), ctypes.POINTER(ctypes.c_size_t)],
                                   ctypes.c_int),
    "gswmtp_plan_create_with_workspace": ([ctypes.POINTER(_P), ctypes.POINTER(gswmtp_desc), _P,
                                           ctypes.c_size_t, _P], ctypes.c_int),
    "gswmtp_plan_destroy": ([_P], ctypes.c_int),
    "gswmtp_set_stream": ([_P, _P], ctypes.c_int),
    "gswmtp_sync": ([_P], ctypes.c_int),
    "gswmtp_iterate": ([_P, ctypes.c_int, ctypes.c_double], ctypes.c_int),
    "gswmtp_iterate_measured": ([_P, _P], ctypes.c_int),
    "gswmtp_iterations_done": ([_P, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "gswmtp_get_phase": ([_P, _P], ctypes.c_int),
    "gswmtp_get_phase_device": ([_P, _P], ctypes.c_int),
    "gswmtp_set_phase": ([_P, _P], ctypes.c_int),
    "gswmtp_set_phase_device": ([_P, _P], ctypes.c_int),
    "gswmtp_get_foci_field": ([_P, _P], ctypes.c_int),
    "gswmtp_get_foci_field_device": ([_P, _P, _P], ctypes.c_int),
    "gswmtp_get_stats": ([_P, _P, _P, _P], ctypes.c_int),
    "gswmtp_get_weights": ([_P, _P], ctypes.c_int),
    "gswmtp_set_weights": ([_P, _P], ctypes.c_int),
    "gswmtp_get_history": ([_P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "gswmtp_get_state": ([_P, _P, _P, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "gswmtp_set_state": ([_P, _P, _P, ctypes.c_int], ctypes.c_int),
    "gswmtp_set_phase_fixing": ([_P, ctypes.c_int], ctypes.c_int),
    "gswmtp_get_index": ([_P, ctypes.POINTER(gswmtp_index_info), _P, _P, _P, _P, _P, _P],
                         ctypes.c_int),
    "gswmtp_forward_field": ([_P, _P, _P], ctypes.c_int),
    "gswmtp_forward_field_noalloc": ([_P, _P, _P], ctypes.c_int),
    "gswmtp_adjoint_field": ([_P, _P, _P], ctypes.c_int),
    "gswmtp_phase_gradient_device": ([_P, _P, _P], ctypes.c_int),
    "gswmtp_phase_gradient_adam_device": ([_P, _P, _P, _P, _P, _P, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double],
                                          ctypes.c_int),
    "gswmtp_design_loss_device": ([_P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, _P, _P, _P], ctypes.c_int),
    "gswmtp_design_loss_record_device": ([_P, _P, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, _P, _P, _P,
                                          ctypes.c_int, _P, _P], ctypes.c_int),
    "gswmtp_adam_step_device": ([_P, _P, _P, _P, _P, ctypes.c_size_t, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, _P],
                                ctypes.c_int),
    "gswmtp_time_stages": ([_P, ctypes.c_int, _P], ctypes.c_int),
    "gswmtp_stage_kernel": ([_P, ctypes.c_int], ctypes.c_char_p),
    "gswmtp_batch_create": ([ctypes.POINTER(_P), _P, ctypes.c_int, _P], ctypes.c_int),
    "gswmtp_batch_iterate": ([_P, ctypes.c_int, ctypes.c_double], ctypes.c_int),
    "gswmtp_batch_set_stream": ([_P, _P], ctypes.c_int),
    "gswmtp_batch_sync": ([_P], ctypes.c_int),
    "gswmtp_batch_tiles": ([_P, _P, _P], ctypes.c_int),
    "gswmtp_batch_n_classes": ([_P, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "gswmtp_batch_class_info": ([_P, ctypes.c_int, ctypes.POINTER(gswmtp_batch_class)],
                                ctypes.c_int),
    "gswmtp_batch_tune_ms": ([_P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "gswmtp_batch_last_error": ([_P], ctypes.c_char_p),
    "gswmtp_batch_destroy": ([_P], ctypes.c_int),
}

_lib = None


def load_library():
    """Load ``libgswmtp.so`` (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.data_ptr()
    return a.ctypes.data


def _stream_handle() -> Optional[int]:
    if not torch.cuda.is_available():
        return None
    return torch.cuda.current_stream().cuda_stream


def status_string(status: int) -> str:
    return load_library().gswmtp_status_string(status).decode()


def _make_desc(holo=None, *, ny=None, nx=None, amplitude=None, mask=None, u=None, v=None,
               s_x=None, s_y=None, fx=None, fy=None, target=None, phi0=None, fz=None,
               precision="fp32", axis=-1, weighting="gsw"):
    """A filled ``gswmtp_desc`` and the host arrays it points into (keep them
    alive until the call that reads the descriptor returns)."""
    lib = load_library()
    g = (lambda k, val: val if val is not None else getattr(holo, k, None)) if holo is not None \
        else (lambda k, val: val)
    keep = []

    def arr(x, dt):
        if x is None:
            return None
        a = np.ascontiguousarray(np.asarray(x, dtype=dt))
        keep.append(a)
        return a.ctypes.data

    d = gswmtp_desc()
    lib.gswmtp_desc_init(ctypes.byref(d))
    d.ny, d.nx = int(g("ny", ny)), int(g("nx", nx))
    d.amplitude = arr(g("amplitude", amplitude), np.float32)
    d.mask = arr(mask, np.uint8)
    d.u = arr(g("u", u), np.float64)
    d.v = arr(g("v", v), np.float64)
    d.s_x = float(g("s_x", s_x))
    d.s_y = float(g("s_y", s_y))
    fxa = np.ascontiguousarray(np.asarray(g("fx", fx), dtype=np.float64))
    d.n_foci = int(fxa.shape[0])
    d.fx = arr(fxa, np.float64)
    d.fy = arr(g("fy", fy), np.float64)
    d.target = arr(g("target", target), np.float64)
    d.phi0 = arr(g("phi0", phi0), np.float32)
    d.fz = arr(g("fz", fz), np.float64)
    d.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    d.axis = int(axis)
    d.weighting = {"gsw": WEIGHT_GSW, "gs": WEIGHT_GS}[weighting] \
        if isinstance(weighting, str) else int(weighting)
    return d, keep


class Plan:
    """A GSW-MTP plan: pupil, sampling and foci of one hologram, and its state.

    Parameters mirror ``gswmtp_desc`` (see ``include/gswmtp.h``).  All host
    arrays are copied at creation; ``workspace`` (optional) is a contiguous
    device tensor of at least ``Plan.workspace_size(...)`` bytes that holds the
    plan's device memory.  ``holo`` may be any object with the fields
    ny, nx, amplitude, u, v, s_x, s_y, fx, fy, target, phi0 and optionally fz
    (axial focus positions; for example a ``synth_ofa.Hologram``); keyword
    arguments override its fields.
    """

    def __init__(self, holo=None, *, ny=None, nx=None, amplitude=None, mask=None, u=None,
                 v=None, s_x=None, s_y=None, fx=None, fy=None, target=None, phi0=None,
                 fz=None, precision="fp32", axis=-1, weighting="gsw", workspace=None):
        lib = load_library()
        d, keep = _make_desc(holo, ny=ny, nx=nx, amplitude=amplitude, mask=mask, u=u, v=v,
                             s_x=s_x, s_y=s_y, fx=fx, fy=fy, target=target, phi0=phi0, fz=fz,
                             precision=precision, axis=axis, weighting=weighting)
        self.ny, self.nx, self.n_foci = d.ny, d.nx, d.n_foci
        self.precision = d.precision
        h = _P()
        if workspace is None:
            rc = lib.gswmtp_plan_create(ctypes.byref(h), ctypes.byref(d), _stream_handle())
        else:
            # a device tensor owned by the caller; kept alive with the plan
            if not workspace.is_cuda or not workspace.is_contiguous():
                raise ValueError("workspace must be a contiguous device tensor")
            nbytes = workspace.numel() * workspace.element_size()
            rc = lib.gswmtp_plan_create_with_workspace(ctypes.byref(h), ctypes.byref(d),
                                                       workspace.data_ptr(), nbytes,
                                                       _stream_handle())
            self._workspace = workspace
        if rc != 0:
            raise GswmtpError(rc, lib.gswmtp_last_error(None).decode())
        self._h = h
        self._lib = lib

    @staticmethod
    def workspace_size(holo=None, **kw) -> int:
        """Bytes of device workspace a plan with these arguments needs
        (``gswmtp_plan_workspace_size``; host-only, no GPU work)."""
        lib = load_library()
        d, _keep = _make_desc(holo, **kw)
        n = ctypes.c_size_t(0)
        rc = lib.gswmtp_plan_workspace_size(ctypes.byref(d), ctypes.byref(n))
        if rc != 0:
            raise GswmtpError(rc, "gswmtp_plan_workspace_size")
        return n.value

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.gswmtp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def _check(self, rc: int):
        if rc != 0:
            raise GswmtpError(rc, self._lib.gswmtp_last_error(self._h).decode())

    def _sync_stream(self):
        self._check(self._lib.gswmtp_set_stream(self._h, _stream_handle()))

    # -- iteration ---------------------------------------------------------
    def iterate(self, n_iter: int, stop_accuracy: float = 0.0):
        self._sync_stream()
        self._check(self._lib.gswmtp_iterate(self._h, int(n_iter), float(stop_accuracy)))

    def iterate_measured(self, measured):
        """One pass whose weight update uses measured focus intensities of the
        current phase (caller order) in place of the computed ones."""
        m = np.ascontiguousarray(np.asarray(measured, dtype=np.float64))
        if m.shape != (self.n_foci,):
            raise ValueError(f"measured must have shape ({self.n_foci},)")
        self._sync_stream()
        self._check(self._lib.gswmtp_iterate_measured(self._h, m.ctypes.data))

    def camera_loop(self, n_iter: int, capture, xi_switch: float = 0.95):
        """n_iter passes with a camera in the loop: ordinary passes until the
        accuracy of the current phase's computed field reaches xi_switch,
        then measured passes with intensities from ``capture(plan)`` (a
        callable that captures the current phase's foci intensities).
        Returns the pass index at which the loop switched, or None."""
        switched = None
        for k in range(int(n_iter)):
            if switched is None and self.stats()["xi"] >= xi_switch:
                switched = k
            if switched is None:
                self.iterate(1)
            else:
                self.iterate_measured(capture(self))
        return switched

    def set_phase_fixing(self, from_pass: int):
        """Freeze the focal phases from updating pass `from_pass` on (0: off)."""
        self._sync_stream()
        self._check(self._lib.gswmtp_set_phase_fixing(self._h, int(from_pass)))

    def iterations_done(self) -> int:
        n = ctypes.c_int(0)
        self._check(self._lib.gswmtp_iterations_done(self._h, ctypes.byref(n)))
        return n.value

    def sync(self):
        self._check(self._lib.gswmtp_sync(self._h))

    # -- state -------------------------------------------------------------
    def phase(self) -> np.ndarray:
        out = np.empty((self.ny, self.nx), np.float32)
        self._sync_stream()
        self._check(self._lib.gswmtp_get_phase(self._h, out.ctypes.data))
        return out

    def phase_device(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float32, device="cuda")
        assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
        assert out.numel() == self.ny * self.nx
        self._sync_stream()
        self._check(self._lib.gswmtp_get_phase_device(self._h, out.data_ptr()))
        return out

    def set_phase(self, phi):
        self._sync_stream()
        if isinstance(phi, torch.Tensor) and phi.is_cuda:
            phi = phi.detach().to(torch.float32).contiguous()
            assert phi.numel() == self.ny * self.nx
            self._check(self._lib.gswmtp_set_phase_device(self._h, phi.data_ptr()))
        else:
            a = np.ascontiguousarray(np.asarray(phi, dtype=np.float32))
            assert a.size == self.ny * self.nx
            self._check(self._lib.gswmtp_set_phase(self._h, a.ctypes.data))

    def foci_field(self) -> np.ndarray:
        out = np.empty(2 * self.n_foci, np.float32)
        self._sync_stream()
        self._check(self._lib.gswmtp_get_foci_field(self._h, out.ctypes.data))
        return out[0::2] + 1j * out[1::2]

    def foci_field_device(self, intensity: bool = True, field: bool = True):
        """(Theta as interleaved float32 [2N] or None, I = |Theta|^2 [N] or None)
        as device tensors on the current stream."""
        if not (intensity or field):
            raise ValueError("ask for the field, the intensities or both")
        field = torch.empty(2 * self.n_foci, dtype=torch.float32, device="cuda") if field else None
        inten = torch.empty(self.n_foci, dtype=torch.float32, device="cuda") if intensity else None
        self._sync_stream()
        self._check(self._lib.gswmtp_get_foci_field_device(self._h, _ptr(field), _ptr(inten)))
        return field, inten

    def stats(self) -> dict:
        xi, eta, u = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._sync_stream()
        self._check(self._lib.gswmtp_get_stats(self._h, ctypes.addressof(xi),
                                               ctypes.addressof(eta), ctypes.addressof(u)))
        return {"xi": xi.value, "eta": eta.value, "uniformity": u.value}

    def weights(self) -> np.ndarray:
        out = np.empty(self.n_foci, np.float64)
        self._check(self._lib.gswmtp_get_weights(self._h, out.ctypes.data))
        return out

    def set_weights(self, w):
        a = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        assert a.size == self.n_foci
        self._check(self._lib.gswmtp_set_weights(self._h, a.ctypes.data))

    def history(self, cap: int = 4096) -> np.ndarray:
        buf = np.empty((cap, 3), np.float64)
        n = ctypes.c_int(0)
        self._check(self._lib.gswmtp_get_history(self._h, buf.ctypes.data, cap, ctypes.byref(n)))
        return buf[: n.value].copy()

    def state(self):
        phi = np.empty((self.ny, self.nx), np.float32)
        w = np.empty(self.n_foci, np.float64)
        it = ctypes.c_int(0)
        self._check(self._lib.gswmtp_get_state(self._h, phi.ctypes.data, w.ctypes.data,
                                               ctypes.byref(it)))
        return phi, w, it.value

    def set_state(self, phi, w, iters: int):
        pa = np.ascontiguousarray(np.asarray(phi, dtype=np.float32))
        wa = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
        self._check(self._lib.gswmtp_set_state(self._h, pa.ctypes.data, wa.ctypes.data,
                                               int(iters)))

    def index(self) -> dict:
        info = gswmtp_index_info()
        self._check(self._lib.gswmtp_get_index(self._h, ctypes.byref(info), None, None, None,
                                               None, None, None))
        ix = np.empty(self.n_foci, np.int32)
        iy = np.empty(self.n_foci, np.int32)
        xu = np.empty(info.ux, np.float64)
        yu = np.empty(info.uy, np.float64)
        rows = np.empty(info.ny_kept, np.int32)
        cols = np.empty(info.nx_kept, np.int32)
        self._check(self._lib.gswmtp_get_index(self._h, ctypes.byref(info), ix.ctypes.data,
                                               iy.ctypes.data, xu.ctypes.data, yu.ctypes.data,
                                               rows.ctypes.data, cols.ctypes.data))
        return {"ix": ix, "iy": iy, "xu": xu, "yu": yu, "rows": rows, "cols": cols,
                "axis": info.axis, "ux": info.ux, "uy": info.uy, "ny_kept": info.ny_kept,
                "nx_kept": info.nx_kept, "n_aperture": info.n_aperture, "sum_a2": info.sum_a2}

    # -- operators ---------------------------------------------------------
    def forward_field(self, E, noalloc: bool = False) -> np.ndarray:
        """Theta = P(E) at the foci for a complex pupil field E [ny, nx].
        noalloc: through gswmtp_forward_field_noalloc (scratch in the
        library's static device array, same result)."""
        e = np.asarray(E, dtype=np.complex64)
        assert e.shape == (self.ny, self.nx)
        inter = np.ascontiguousarray(np.stack([e.real, e.imag], axis=-1).astype(np.float32))
        out = np.empty(2 * self.n_foci, np.float32)
        self._sync_stream()
        fn = self._lib.gswmtp_forward_field_noalloc if noalloc else self._lib.gswmtp_forward_field
        self._check(fn(self._h, inter.ctypes.data, out.ctypes.data))
        return out[0::2] + 1j * out[1::2]

    def adjoint_field(self, theta) -> np.ndarray:
        """E' = P^H(theta) (no projection) as complex [ny, nx]."""
        t = np.asarray(theta, dtype=np.complex64)
        inter = np.ascontiguousarray(np.stack([t.real, t.imag], axis=-1).astype(np.float32))
        out = np.empty(2 * self.ny * self.nx, np.float32)
        self._sync_stream()
        self._check(self._lib.gswmtp_adjoint_field(self._h, inter.ctypes.data, out.ctypes.data))
        return (out[0::2] + 1j * out[1::2]).reshape(self.ny, self.nx)

    def phase_gradient_device(self, g: torch.Tensor,
                              out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """dL/dphi for L = sum g_n |Theta_n|^2 at the current phase."""
        g = g.detach().to(torch.float32).contiguous()
        assert g.is_cuda and g.numel() == self.n_foci
        if out is None:
            out = torch.empty((self.ny, self.nx), dtype=torch.float32, device="cuda")
        self._sync_stream()
        self._check(self._lib.gswmtp_phase_gradient_device(self._h, g.data_ptr(),
                                                            out.data_ptr()))
        return out

    def phase_gradient_adam_device(self, g: torch.Tensor, phi: torch.Tensor, m: torch.Tensor,
                                   v: torch.Tensor, step: torch.Tensor, lr: float,
                                   betas=(0.9, 0.999), eps: float = 1e-8):
        """The phase gradient of L = sum g_n |Theta_n|^2 at the current phase
        applied at once by one Adam step to phi, m, v (contiguous float32 CUDA
        tensors of ny * nx values, in place); ``step`` holds the step number
        (one float32 CUDA value)."""
        g = g.detach().to(torch.float32).contiguous()
        assert g.is_cuda and g.numel() == self.n_foci
        for t in (phi, m, v):
            if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and
                    t.numel() == self.ny * self.nx):
                raise TypeError("phi, m, v must be contiguous float32 CUDA tensors of ny*nx")
        if not (step.is_cuda and step.dtype == torch.float32 and step.numel() == 1):
            raise TypeError("step must be one float32 CUDA value")
        self._sync_stream()
        self._check(self._lib.gswmtp_phase_gradient_adam_device(
            self._h, g.data_ptr(), phi.data_ptr(), m.data_ptr(), v.data_ptr(), step.data_ptr(),
            float(lr), float(betas[0]), float(betas[1]), float(eps)))

    # -- profiling ---------------------------------------------------------
    def time_stages(self, n_iter: int) -> dict:
        out = np.zeros(N_STAGES, np.float64)
        self._sync_stream()
        self._check(self._lib.gswmtp_time_stages(self._h, int(n_iter), out.ctypes.data))
        return dict(zip(STAGES, out.tolist()))

    def stage_kernel(self, stage: int) -> str:
        return self._lib.gswmtp_stage_kernel(self._h, stage).decode()


_LOOPS = {0: "plain", 1: "pipe", 2: "direct", 3: "b16"}
_SOURCES = {0: "plan", 1: "tuned", 2: "cache", 3: "env"}


def adam_step_device(phi: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
                     step: torch.Tensor, lr: float, betas=(0.9, 0.999), eps: float = 1e-8):
    """One Adam step in the library (gswmtp_adam_step_device) on contiguous
    float32 CUDA tensors, in place on phi, m and v; ``step`` is a one-element
    float32 CUDA tensor holding this step's number (advanced by the caller)."""
    for t in (phi, grad, m, v, step):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError("Adam operands must be contiguous float32 CUDA tensors")
    n = phi.numel()
    if not (grad.numel() == m.numel() == v.numel() == n and step.numel() == 1):
        raise ValueError("Adam operands differ in size")
    rc = load_library().gswmtp_adam_step_device(
        phi.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), step.data_ptr(), n,
        float(lr), float(betas[0]), float(betas[1]), float(eps), _stream_handle())
    if rc != 0:
        raise GswmtpError(rc, "gswmtp_adam_step_device")


def _config_text(c) -> str:
    bm, bn, bk, kg, loop, split = list(c)
    return f"{bm}x{bn}/{'kg2' if kg == 2 else _LOOPS.get(loop, loop)}/k{split}"


class Batch:
    """Several plans iterated together: the tiles of every plan's products
    on per-configuration device work lists (persistent launches, one per
    kernel configuration and stage), focus update and scatter grouped, a pass
    replayed from a captured HIP graph.  Each shape class of a product gets
    its own tuned configuration (``classes()``).  The plans stay usable:
    their state is read and set through each ``Plan``; keep them open while
    the batch lives."""

    def __init__(self, plans):
        lib = load_library()
        self.plans = list(plans)
        arr = (_P * len(self.plans))(*[p.handle for p in self.plans])
        h = _P()
        rc = lib.gswmtp_batch_create(ctypes.byref(h), arr, len(self.plans), _stream_handle())
        if rc != 0:
            raise GswmtpError(rc, lib.gswmtp_batch_last_error(None).decode())
        self._h = h
        self._lib = lib

    def _check(self, rc: int):
        if rc != 0:
            raise GswmtpError(rc, self._lib.gswmtp_batch_last_error(self._h).decode())

    def iterate(self, n_iter: int, stop_accuracy: float = 0.0):
        self._check(self._lib.gswmtp_batch_set_stream(self._h, _stream_handle()))
        self._check(self._lib.gswmtp_batch_iterate(self._h, int(n_iter), float(stop_accuracy)))

    def sync(self):
        self._check(self._lib.gswmtp_batch_sync(self._h))

    def tiles(self) -> dict:
        t = np.zeros(4, np.int32)
        ms = np.zeros(8, np.float64)
        self._check(self._lib.gswmtp_batch_tiles(self._h, t.ctypes.data, ms.ctypes.data))
        cands = ("64x64", "64x128", "128x64", "128x128")
        return {"forward": f"{t[0]}x{t[1]}", "adjoint": f"{t[2]}x{t[3]}",
                "tune_ms": {"forward": {c: ms[i] for i, c in enumerate(cands) if ms[i] > 0},
                            "adjoint": {c: ms[4 + i] for i, c in enumerate(cands)
                                        if ms[4 + i] > 0}}}

    def classes(self) -> list:
        """Shape classes (product, padded M x N x K) with their configuration,
        where it came from and the tuning table (candidate -> ms per copy of
        the class's tiles)."""
        n = ctypes.c_int(0)
        self._check(self._lib.gswmtp_batch_n_classes(self._h, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            c = gswmtp_batch_class()
            self._check(self._lib.gswmtp_batch_class_info(self._h, i, ctypes.byref(c)))
            out.append({
                "product": "forward" if c.product == 0 else "adjoint",
                "mnk": [c.m, c.n, c.k], "plans": c.n_plans,
                "config": _config_text(c.config), "ms": c.ms,
                "source": _SOURCES.get(c.source, c.source),
                "tried": {_config_text(c.tried_config[k]): c.tried_ms[k]
                          for k in range(c.n_tried)},
            })
        return out

    def tune_ms(self) -> float:
        v = ctypes.c_double(0.0)
        self._check(self._lib.gswmtp_batch_tune_ms(self._h, ctypes.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.gswmtp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


from .autograd import (MTPIntensity, adam_design, design_loss, design_loss_fused,  # noqa: E402
                       foci_intensity)

__all__ = ["Plan", "Batch", "GswmtpError", "load_library", "status_string", "MTPIntensity",
           "foci_intensity", "design_loss", "adam_design", "design_loss_fused", "FP32", "BF16X3", "FP16X3", "BF16X6", "STAGES", "adam_step_device"]
