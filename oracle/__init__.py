"""FP64 CPU oracle of the GSW-MTP iteration (Liu et al., arXiv:2206.12661).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
(``paper_2206_12661_amd``) never imports it and shares no code with it.

Two parts:
  * the propagation operators and Algorithm 1, in plain C (``gsw_oracle.c``),
    double precision, called through ctypes;
  * the index work (unique focal coordinates, gather indices, aperture
    compaction, axis choice, per-row focus lists) written out with numpy's
    sort-based ``unique`` and ``searchsorted``: integer results that the GPU
    must reproduce bit for bit.

Pins that tie this oracle to something other than itself live in
``tests/test_oracle_pins.py``.  One function has no external pin: the full
multi-step GSW trajectory (the paper prints no worked example), reported as
"parity unpinned" there and in the design notes; its single steps are pinned.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_forward.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, _D, _D, _D, _D]
    lib.oracle_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, _D, _D, _D, _D, _D]
    lib.oracle_stats.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double, ctypes.c_double, _D]
    lib.oracle_stats.restype = None
    lib.oracle_weight_update.argtypes = [ctypes.c_int, _D, _D, _D, _D]
    lib.oracle_weight_update.restype = None
    lib.oracle_weight_update_ex.argtypes = [ctypes.c_int, _D, _D, _D, _D, ctypes.c_int, _D, _D]
    lib.oracle_weight_update_ex.restype = None
    lib.oracle_project.argtypes = [ctypes.c_int, _D, _D, _D, _D]
    lib.oracle_project.restype = None
    lib.oracle_gsw.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, _D, _D, _D, _D, _D, ctypes.c_int,
                               ctypes.c_double, _D, _I, _D]
    lib.oracle_gsw_ex.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, _D, _D, _D, _D, _D, _D,
                                  ctypes.c_int,
                                  ctypes.c_double, _D, _I, _D, ctypes.c_int, ctypes.c_int]
    lib.oracle_gsw_measured_pass.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                             _D, _D, _D, _D, _D, _D, _D, _D]
    lib.oracle_phase_gradient.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, _D,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int, _D,
                                          _D, _D, _D, _D, _D, _D]
    _lib = lib
    return lib


def _d(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _fz(holo):
    """Axial positions of a hologram's foci (None: all on the focal plane)."""
    fz = getattr(holo, "fz", None)
    return None if fz is None else _f64(fz)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (results do not depend on it)."""
    _load().oracle_set_threads(int(n))


# ----------------------------------------------------------------------------
# Propagation operators (Eq. 1 / Eq. 2 and its adjoint)
# ----------------------------------------------------------------------------

def forward(E, u, v, s_x, s_y, fx, fy, fz=None) -> np.ndarray:
    """Focal field Theta_n of the complex pupil field E[ny, nx] (complex128);
    fz (optional): axial positions (defocus phase of the pupil)."""
    E = np.ascontiguousarray(np.asarray(E, dtype=np.complex128))
    ny, nx = E.shape
    u, v, fx, fy = _f64(u), _f64(v), _f64(fx), _f64(fy)
    fz = None if fz is None else _f64(fz)
    out = np.zeros(fx.shape[0], dtype=np.complex128)
    rc = _load().oracle_forward(ny, nx, E.view(np.float64).ctypes.data_as(_D), _d(u), _d(v),
                                float(s_x), float(s_y), fx.shape[0], _d(fx), _d(fy), _d(fz),
                                out.view(np.float64).ctypes.data_as(_D))
    if rc:
        raise MemoryError("oracle_forward")
    return out


def adjoint(theta, ny, nx, u, v, s_x, s_y, fx, fy, fz=None) -> np.ndarray:
    """Adjoint field E'[ny, nx] of focal values theta[N] (zero off the foci)."""
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.complex128))
    u, v, fx, fy = _f64(u), _f64(v), _f64(fx), _f64(fy)
    fz = None if fz is None else _f64(fz)
    out = np.zeros((ny, nx), dtype=np.complex128)
    rc = _load().oracle_adjoint(ny, nx, _d(u), _d(v), float(s_x), float(s_y), fx.shape[0],
                                _d(fx), _d(fy), _d(fz), theta.view(np.float64).ctypes.data_as(_D),
                                out.view(np.float64).ctypes.data_as(_D))
    if rc:
        raise MemoryError("oracle_adjoint")
    return out


def stats(theta, target, amplitude) -> dict:
    """xi (accuracy), eta (efficiency), U (uniformity) and sum I of one field."""
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.complex128))
    target = _f64(target)
    amp = np.asarray(amplitude, dtype=np.float64)
    n_ap = float(np.count_nonzero(amp > 0))
    sum_a2 = float(np.sum(amp * amp))
    out = np.zeros(4)
    _load().oracle_stats(theta.shape[0], theta.view(np.float64).ctypes.data_as(_D),
                         _d(target), n_ap, sum_a2, _d(out))
    return {"xi": out[0], "eta": out[1], "uniformity": out[2], "sum_I": out[3]}


def weight_update(theta, target, w, weighting: str = "gsw", fixed=None, measured=None):
    """One weight update + focal-field update (Algorithm 1); returns
    (w_new, theta_new).  This calls the same C function that every pass of
    ``gsw`` and ``gsw_measured_pass`` runs.  weighting "gs" keeps the weights
    (plain GS, Sec. 2); fixed (complex [N], optional): frozen focal phasors
    (phase fixing); measured (optional): camera intensities that replace
    |theta|^2 in the weight update (Sec. 2 experiments)."""
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.complex128))
    target = _f64(target)
    w = _f64(w).copy()
    out = np.zeros_like(theta)
    fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, dtype=np.complex128))
    ms = None if measured is None else _f64(measured)
    _load().oracle_weight_update_ex(theta.shape[0], theta.view(np.float64).ctypes.data_as(_D),
                                    _d(target), _d(w), out.view(np.float64).ctypes.data_as(_D),
                                    {"gsw": 0, "gs": 1}[weighting],
                                    None if fx is None else fx.view(np.float64).ctypes.data_as(_D),
                                    _d(ms))
    return w, out


def project(amplitude, Ep):
    """Phase-only projection of Algorithm 1 (the C function every pass runs):
    phi = arg E' where A > 0 and E' != 0 (0 elsewhere), range (-pi, pi];
    returns (phi, E = A exp(i phi))."""
    amp = np.ascontiguousarray(np.asarray(amplitude, dtype=np.float64))
    Ep = np.ascontiguousarray(np.asarray(Ep, dtype=np.complex128))
    assert amp.shape == Ep.shape
    phi = np.zeros(amp.shape)
    E = np.zeros(amp.shape, dtype=np.complex128)
    _load().oracle_project(amp.size, _d(amp), Ep.view(np.float64).ctypes.data_as(_D), _d(phi),
                           E.view(np.float64).ctypes.data_as(_D))
    return phi, E


def gsw(holo, n_iter: Optional[int] = None, stop: float = 0.0, phi=None, w=None,
        weighting: str = "gsw", phase_fix: int = 0) -> dict:
    """Run Algorithm 1 on a ``synth_ofa.Hologram`` (or any object with the same
    fields).  Returns phi (float64 [ny, nx]), w, history [passes, 3],
    iters_done and the field of the returned phase.  weighting "gs" keeps
    unit weights (plain GS); phase_fix = k > 0 freezes the focal phases from
    the k-th updating pass on (Sec. 2)."""
    n_iter = holo.n_iter if n_iter is None else n_iter
    ny, nx = holo.ny, holo.nx
    amp = _f64(holo.amplitude)
    ph = _f64(holo.phi0 if phi is None else phi).copy()
    ww = np.ones(holo.n_foci) if w is None else _f64(w).copy()
    hist = np.zeros((max(n_iter, 1), 3))
    done = ctypes.c_int(0)
    th = np.zeros(holo.n_foci, dtype=np.complex128)
    rc = _load().oracle_gsw_ex(ny, nx, _d(amp), _d(_f64(holo.u)), _d(_f64(holo.v)),
                               float(holo.s_x), float(holo.s_y), holo.n_foci, _d(_f64(holo.fx)),
                               _d(_f64(holo.fy)), _d(_fz(holo)), _d(_f64(holo.target)), _d(ph),
                               _d(ww),
                               int(n_iter), float(stop), _d(hist), ctypes.byref(done),
                               th.view(np.float64).ctypes.data_as(_D),
                               {"gsw": 0, "gs": 1}[weighting], int(phase_fix))
    if rc:
        raise MemoryError("oracle_gsw")
    passes = done.value + (1 if (stop > 0 and done.value < n_iter) else 0)
    return {"phi": ph, "w": ww, "history": hist[:passes], "iters_done": done.value,
            "theta": th}


def gsw_measured_pass(holo, phi, w, measured) -> dict:
    """One pass of Algorithm 1 whose weight update takes the focus
    intensities from ``measured`` (a camera capture of the field of phi,
    normalised to unit sum) instead of |Theta|^2: the camera-in-the-loop
    strategy of the experiments in Sec. 2.  Returns phi, w and the
    statistics (xi, eta, U) of the computed field the pass started from."""
    ph = _f64(phi).copy()
    ww = _f64(w).copy()
    hist = np.zeros(3)
    rc = _load().oracle_gsw_measured_pass(
        holo.ny, holo.nx, _d(_f64(holo.amplitude)), _d(_f64(holo.u)), _d(_f64(holo.v)),
        float(holo.s_x), float(holo.s_y), holo.n_foci, _d(_f64(holo.fx)), _d(_f64(holo.fy)),
        _d(_fz(holo)), _d(_f64(holo.target)), _d(ph), _d(ww), _d(_f64(measured)), _d(hist))
    if rc:
        raise MemoryError("oracle_gsw_measured_pass")
    return {"phi": ph, "w": ww, "history": hist}


def camera_loop(holo, n_iter: int, capture, xi_switch: float = 0.95, phi=None, w=None) -> dict:
    """Algorithm 1 with a camera in the loop (Sec. 2 experiments): plain
    passes until the accuracy xi of the current phase's computed field
    reaches xi_switch, then every pass takes its weight-update intensities
    from ``capture(theta)`` - a camera model mapping the computed focal field
    of the current phase to measured intensities.  Returns phi, w, the
    per-pass history, the pass at which the loop switched (None if never)
    and the field of the returned phase."""
    ph = _f64(holo.phi0 if phi is None else phi).copy()
    ww = np.ones(holo.n_foci) if w is None else _f64(w).copy()
    hist, switched = [], None
    fz = _fz(holo)
    for k in range(n_iter):
        th = forward(pupil_field(holo, ph), holo.u, holo.v, holo.s_x, holo.s_y, holo.fx,
                     holo.fy, fz)
        if switched is None and stats(th, holo.target, holo.amplitude)["xi"] >= xi_switch:
            switched = k
        if switched is not None:
            r = gsw_measured_pass(holo, ph, ww, capture(th))
        else:
            r = gsw(holo, n_iter=1, phi=ph, w=ww)
            r["history"] = r["history"][0]
        ph, ww = r["phi"], r["w"]
        hist.append(r["history"])
    th = forward(pupil_field(holo, ph), holo.u, holo.v, holo.s_x, holo.s_y, holo.fx, holo.fy, fz)
    return {"phi": ph, "w": ww, "history": np.array(hist).reshape(-1, 3), "switched": switched,
            "theta": th}


def phase_gradient(holo, phi, g):
    """dL/dphi for L = sum_n g_n |Theta_n(phi)|^2; returns (grad [ny, nx], theta)."""
    ny, nx = holo.ny, holo.nx
    grad = np.zeros((ny, nx))
    th = np.zeros(holo.n_foci, dtype=np.complex128)
    rc = _load().oracle_phase_gradient(
        ny, nx, _d(_f64(holo.amplitude)), _d(_f64(holo.u)), _d(_f64(holo.v)),
        float(holo.s_x), float(holo.s_y), holo.n_foci, _d(_f64(holo.fx)), _d(_f64(holo.fy)),
        _d(_fz(holo)), _d(_f64(phi)), _d(_f64(g)), _d(grad),
        th.view(np.float64).ctypes.data_as(_D))
    if rc:
        raise MemoryError("oracle_phase_gradient")
    return grad, th


def design_loss(I, target, n_ap: int, sum_a2: float, eta_weight: float = 0.1):
    """Loss of the differentiable phase design and its gradient in I:

        L = sum_n (i_n - t_n)^2 - eta_weight * eta,
        i_n = I_n / sum_m I_m,   eta = sum_m I_m / (n_ap * sum A^2)

    (normalised intensities against normalised targets t = T / sum T, as in
    the weight update of Algorithm 1; eta is the diffraction efficiency of
    Sec. 2, energy at the foci over the energy through the aperture, with the
    incident energy of the discrete sums taken as n_ap * sum A^2).
    Returns (L, dL/dI)."""
    I = np.asarray(I, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    t = t / t.sum()
    S = I.sum()
    i = I / S
    r = i - t
    c = 1.0 / (float(n_ap) * float(sum_a2))
    L = float(np.sum(r * r) - eta_weight * S * c)
    # d i_m / d I_n = (delta_mn - i_m) / S
    dI = 2.0 * r / S - 2.0 * np.sum(r * i) / S - eta_weight * c
    return L, dI


def adam_design(holo, steps: int, lr: float = 0.05, betas=(0.9, 0.999), eps: float = 1e-8,
                eta_weight: float = 0.1, phi=None):
    """Gradient-descent phase design: Adam (Kingma and Ba, bias-corrected
    moments) on ``design_loss`` of the foci intensities, with the gradient
    dL/dphi = 2 Im(conj(E) P^H(dL/dI * Theta)) from ``phase_gradient``.
    Returns (phi after the last step, loss before each step [steps])."""
    ph = _f64(holo.phi0 if phi is None else phi).copy()
    amp = _f64(holo.amplitude)
    n_ap = int(np.count_nonzero(amp > 0))
    sum_a2 = float(np.sum(amp * amp))
    b1, b2 = betas
    m = np.zeros_like(ph)
    v = np.zeros_like(ph)
    hist = np.zeros(steps)
    for k in range(1, steps + 1):
        th = forward(pupil_field(holo, ph), holo.u, holo.v, holo.s_x, holo.s_y, holo.fx, holo.fy,
                     _fz(holo))
        L, gI = design_loss(np.abs(th) ** 2, holo.target, n_ap, sum_a2, eta_weight)
        hist[k - 1] = L
        grad, _ = phase_gradient(holo, ph, gI)
        m = b1 * m + (1.0 - b1) * grad
        v = b2 * v + (1.0 - b2) * grad * grad
        mh = m / (1.0 - b1 ** k)
        vh = v / (1.0 - b2 ** k)
        ph = ph - lr * mh / (np.sqrt(vh) + eps)
    return ph, hist


def pupil_field(holo, phi=None) -> np.ndarray:
    """E = A exp(i phi) in complex128 (phi defaults to the initial phase)."""
    ph = np.asarray(holo.phi0 if phi is None else phi, dtype=np.float64)
    return np.asarray(holo.amplitude, dtype=np.float64) * np.exp(1j * ph)


# ----------------------------------------------------------------------------
# Index work: reduced focal grid, gather indices, aperture compaction
# ----------------------------------------------------------------------------

def canonical(c) -> np.ndarray:
    """Focal coordinates with -0.0 replaced by +0.0 (equal values, one key)."""
    c = np.asarray(c, dtype=np.float64)
    return np.where(c == 0.0, 0.0, c)


def unique_coords(c, z=None):
    """Sorted unique focal coordinates and the gather index of every focus
    into them.  The reduced focal grid of the paper keeps one sample row
    (column) per distinct focus y (x) coordinate: k x l grid foci give l
    unique x and k unique y values.  With axial positions z, a reduced row is
    a distinct (coordinate, z) pair (its kernel row carries that plane's
    defocus phase), ordered by coordinate, then z."""
    key = canonical(c)
    if z is None:
        uniq = np.unique(key)
        idx = np.searchsorted(uniq, key).astype(np.int32)
        return uniq, idx
    zk = canonical(z)
    pairs = sorted(set(zip(key.tolist(), zk.tolist())))
    pos = {pz: i for i, pz in enumerate(pairs)}
    idx = np.array([pos[(a, b)] for a, b in zip(key.tolist(), zk.tolist())], dtype=np.int32)
    return np.array([a for a, _ in pairs]), idx


def compaction(amplitude):
    """Pupil rows and columns holding any non-zero amplitude, ascending
    (the zero padding the MTP does not need is never sampled)."""
    nz = np.asarray(amplitude) != 0
    rows = np.nonzero(nz.any(axis=1))[0].astype(np.int32)
    cols = np.nonzero(nz.any(axis=0))[0].astype(np.int32)
    return rows, cols


def axis_choice(ux: int, uy: int) -> int:
    """Which focal axis the dense product reduces: 0 (y) unless x has fewer
    unique coordinates.  The dense cost is U_axis * Ny' * Nx' either way."""
    return 1 if ux < uy else 0


def has_duplicate_foci(fx, fy, fz=None) -> bool:
    cols = [canonical(fx), canonical(fy)] + ([] if fz is None else [canonical(fz)])
    pts = np.stack(cols, axis=1)
    return np.unique(pts, axis=0).shape[0] != pts.shape[0]


def index_plan(fx, fy, amplitude, fz=None) -> dict:
    """Every integer the GPU plan derives from the foci and the aperture."""
    xu, ix = unique_coords(fx, fz)
    yu, iy = unique_coords(fy, fz)
    rows, cols = compaction(amplitude)
    axis = axis_choice(xu.shape[0], yu.shape[0])
    ir, ic = (iy, ix) if axis == 0 else (ix, iy)
    order = np.lexsort((ic, ir)).astype(np.int32)        # sort by (ir, ic)
    ur = (yu if axis == 0 else xu).shape[0]
    row_ptr = np.searchsorted(ir[order], np.arange(ur + 1)).astype(np.int32)
    return {"xu": xu, "yu": yu, "ix": ix, "iy": iy, "rows": rows, "cols": cols,
            "axis": axis, "order": order, "row_ptr": row_ptr,
            "duplicate": has_duplicate_foci(fx, fy, fz)}
