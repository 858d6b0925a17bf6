"""Pins of the FP64 oracle against facts it does not compute itself.

Every test here runs on the CPU.  Each one fixes the oracle to the
mathematics the paper rests on (the DFT, its adjoint, Parseval), to closed
forms (the single-focus grating), to invariances of Algorithm 1, to a
hand-worked example, or to brute force, so that a dropped term, a wrong
sign, a swapped index or a transposed operand in the oracle fails at least
one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth_ofa

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_field(rng, ny, nx):
    return rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))


def _full_grid(ny, nx):
    """Every integer focal point (x = k, y = l), focus n = l * nx + k."""
    yy, xx = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    return xx.reshape(-1), yy.reshape(-1)


# --------------------------------------------------------------------------
# Forward operator (Eq. 1 sampled, Eq. 2 separable)
# --------------------------------------------------------------------------

def test_forward_equals_fft2_on_integer_grid():
    """With pupil samples u = 0..nx-1, v = 0..ny-1, s = 1/n and foci on every
    integer point, the MTP is the 2-D DFT: Theta = numpy.fft.fft2(E)."""
    rng = np.random.default_rng(1)
    ny, nx = 7, 12
    E = _rand_field(rng, ny, nx)
    fx, fy = _full_grid(ny, nx)
    th = oracle.forward(E, np.arange(nx, dtype=float), np.arange(ny, dtype=float),
                        1.0 / nx, 1.0 / ny, fx, fy)
    ref = np.fft.fft2(E).reshape(-1)
    assert np.max(np.abs(th - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_forward_fractional_points_equal_zero_padded_fft():
    """Foci on a grid P times finer than the DFT grid equal the FFT of the
    pupil zero-padded P times: the conventional IFTA's padding (Eq. 3) that
    the MTP avoids.  Negative coordinates wrap modulo the padded length."""
    rng = np.random.default_rng(2)
    ny, nx, P = 6, 10, 4
    E = _rand_field(rng, ny, nx)
    kx = rng.integers(-nx * P // 2, nx * P // 2, size=25)
    ky = rng.integers(-ny * P // 2, ny * P // 2, size=25)
    th = oracle.forward(E, np.arange(nx, dtype=float), np.arange(ny, dtype=float),
                        1.0 / nx, 1.0 / ny, kx / P, ky / P)
    F = np.fft.fft2(E, s=(ny * P, nx * P))
    ref = F[ky % (ny * P), kx % (nx * P)]
    assert np.max(np.abs(th - ref)) <= 1e-11 * np.max(np.abs(F))


def test_forward_centred_coordinates_shift_theorem():
    """Centred pupil coordinates u - c multiply each focal value by the
    closed-form phase exp(+2 pi i s c x) relative to the uncentred DFT."""
    rng = np.random.default_rng(3)
    ny, nx = 8, 6
    E = _rand_field(rng, ny, nx)
    fx, fy = _full_grid(ny, nx)
    cx, cy = (nx - 1) / 2, (ny - 1) / 2
    th = oracle.forward(E, synth_ofa.centred(nx), synth_ofa.centred(ny), 1.0 / nx, 1.0 / ny,
                        fx, fy)
    ref = np.fft.fft2(E).reshape(-1) * np.exp(2j * np.pi * (cx * fx / nx + cy * fy / ny))
    assert np.max(np.abs(th - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_forward_nonuniform_sampling_brute_force():
    """Arbitrary, non-uniform pupil and focal samples (the decoupled sampling
    the MTP allows): compare with a direct 2-D sum of exp terms over every
    (pupil sample, focus) pair.  A consistency check of the separable
    evaluation; the independent pins are the FFT ones above."""
    rng = np.random.default_rng(4)
    ny, nx = 5, 7
    E = _rand_field(rng, ny, nx)
    u = np.sort(rng.uniform(-3, 3, nx))
    v = np.sort(rng.uniform(-2, 2, ny))
    fx, fy = rng.uniform(-4, 4, 6), rng.uniform(-4, 4, 6)
    sx, sy = 0.37, 0.21
    th = oracle.forward(E, u, v, sx, sy, fx, fy)
    ref = np.array([sum(E[j, i] * np.exp(-2j * np.pi * (sx * u[i] * fx[n] + sy * v[j] * fy[n]))
                        for j in range(ny) for i in range(nx)) for n in range(6)])
    assert np.max(np.abs(th - ref)) <= 1e-12 * np.max(np.abs(ref))


# --------------------------------------------------------------------------
# Inverse operator (adjoint)
# --------------------------------------------------------------------------

def test_adjoint_dot_product_identity():
    """<P E, T> = <E, P^H T> for random fields at arbitrary coordinates."""
    rng = np.random.default_rng(5)
    ny, nx, n = 9, 11, 13
    E = _rand_field(rng, ny, nx)
    T = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    u, v = synth_ofa.centred(nx), rng.uniform(-5, 5, ny)
    fx, fy = rng.uniform(-4, 4, n), rng.uniform(-4, 4, n)
    lhs = np.vdot(oracle.forward(E, u, v, 1 / nx, 1 / ny, fx, fy), T)
    rhs = np.vdot(E, oracle.adjoint(T, ny, nx, u, v, 1 / nx, 1 / ny, fx, fy))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_adjoint_equals_scaled_ifft2_on_full_grid():
    """On the full integer grid the adjoint is ny nx ifft2."""
    rng = np.random.default_rng(6)
    ny, nx = 6, 9
    T = _rand_field(rng, ny, nx)
    fx, fy = _full_grid(ny, nx)
    E = oracle.adjoint(T.reshape(-1), ny, nx, np.arange(nx, dtype=float),
                       np.arange(ny, dtype=float), 1 / nx, 1 / ny, fx, fy)
    ref = ny * nx * np.fft.ifft2(T)
    assert np.max(np.abs(E - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_parseval_on_full_grid():
    """sum |Theta|^2 = ny nx sum |E|^2 over the full integer grid."""
    rng = np.random.default_rng(7)
    ny, nx = 8, 8
    E = _rand_field(rng, ny, nx)
    fx, fy = _full_grid(ny, nx)
    th = oracle.forward(E, synth_ofa.centred(nx), synth_ofa.centred(ny), 1 / nx, 1 / ny, fx, fy)
    assert np.sum(np.abs(th) ** 2) == pytest.approx(ny * nx * np.sum(np.abs(E) ** 2), rel=1e-12)


# --------------------------------------------------------------------------
# Algorithm 1 steps
# --------------------------------------------------------------------------

def test_weight_update_hand_example():
    """Hand-worked three-focus example (exact rationals) of the intensity,
    accuracy, uniformity, weight update and focal-field update."""
    g = json.load(open(os.path.join(GOLDEN, "weight_update_3foci.json")))
    theta = np.array([complex(a, b) for a, b in g["theta"]])
    target = np.array(g["target"], dtype=float)
    ex = g["expected"]
    st = oracle.stats(theta, target, np.ones((2, 2)))
    assert st["xi"] == pytest.approx(1 - math.sqrt(float(Fraction(ex["xi_sqrt_arg"]))), abs=1e-15)
    assert st["uniformity"] == pytest.approx(float(Fraction(ex["uniformity"])), abs=1e-15)
    w, tn = oracle.weight_update(theta, target, np.array(g["w0"], dtype=float))
    w_ref = np.sqrt([float(Fraction(s)) for s in ex["w_squared"]])
    assert np.allclose(w, w_ref, rtol=1e-15, atol=0)
    re = [math.sqrt(float(Fraction(a))) * float(Fraction(b)) for a, b in ex["theta_new_re_over_sqrt"]]
    im = [math.sqrt(float(Fraction(a))) * float(Fraction(b)) for a, b in ex["theta_new_im_over_sqrt"]]
    assert np.allclose(tn.real, re, rtol=1e-14, atol=1e-15)
    assert np.allclose(tn.imag, im, rtol=1e-14, atol=1e-15)


def test_weight_update_dark_focus_stays_finite():
    theta = np.array([0j, 1 + 0j, 2j])
    w, tn = oracle.weight_update(theta, np.array([1.0, 1.0, 1.0]), np.ones(3))
    assert np.all(np.isfinite(w)) and np.all(np.isfinite(tn))
    assert tn[0].imag == 0.0 and tn[0].real > 0.0          # phasor 1 for a zero field


def _q(x):
    return float(Fraction(str(x)))


@pytest.mark.parametrize("case", ["gsw", "gs", "fixed", "measured"])
def test_weight_update_branches_hand_worked(case):
    """Hand-worked cases (exact rationals) of every branch of the one update
    function that each pass of the iteration runs: GSW with non-unit start
    weights, plain GS, frozen focal phasors and camera intensities.  Target 2
    at the second focus separates w sqrt(target) from w target; non-unit
    start weights separate w0 sqrt(t/i) from sqrt(t/i)."""
    g = json.load(open(os.path.join(GOLDEN, "weight_update_branches.json")))
    c = g["cases"][case]
    theta = np.array([complex(a, b) for a, b in g["theta"]])
    target = np.array(g["target"], dtype=float)
    fixed = None if "fixed" not in c else np.array([complex(_q(a), _q(b)) for a, b in c["fixed"]])
    measured = None if "measured" not in c else np.array(c["measured"], dtype=float)
    w, tn = oracle.weight_update(theta, target, np.array(g["w0"], dtype=float),
                                 weighting=c["weighting"], fixed=fixed, measured=measured)
    assert np.allclose(w, np.sqrt([_q(s) for s in c["w_squared"]]), rtol=1e-15, atol=0)
    re = [math.sqrt(_q(a)) * _q(b) for a, b in c["theta_new_re"]]
    im = [math.sqrt(_q(a)) * _q(b) for a, b in c["theta_new_im"]]
    assert np.allclose(tn.real, re, rtol=1e-14, atol=1e-15)
    assert np.allclose(tn.imag, im, rtol=1e-14, atol=1e-15)


def test_projection_closed_form():
    """Phase-only projection: the phase of E' at known angles, 0 where the
    amplitude or E' is zero, -pi reported as +pi, and E = A exp(i phi)."""
    ang = np.array([[0.3, -2.9, np.pi / 2], [-np.pi, 1.0, 2.0]])
    mag = np.array([[2.0, 0.5, 7.0], [3.0, 0.0, 1.0]])
    Ep = mag * np.exp(1j * ang)
    Ep[1, 0] = complex(-3.0, -0.0)                 # angle -pi
    amp = np.array([[1.0, 2.0, 0.0], [0.5, 1.0, 4.0]])
    phi, E = oracle.project(amp, Ep)
    expect = np.array([[0.3, -2.9, 0.0], [np.pi, 0.0, 2.0]])
    assert np.allclose(phi, expect, rtol=0, atol=1e-15)
    assert phi[1, 0] == np.pi
    assert np.allclose(E, amp * np.exp(1j * expect), rtol=0, atol=1e-15)


def _one_pass_composed(h, phi, w, weighting="gsw", fixed=None, measured=None):
    """One pass of Algorithm 1 composed from the separately pinned pieces:
    forward operator, weight/field update, adjoint operator, projection."""
    th = oracle.forward(oracle.pupil_field(h, phi), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    w2, thn = oracle.weight_update(th, h.target, w, weighting=weighting, fixed=fixed,
                                   measured=measured)
    Ep = oracle.adjoint(thn, h.ny, h.nx, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    phi2, _ = oracle.project(h.amplitude, Ep)
    return phi2, w2, th


@pytest.mark.parametrize("weighting", ["gsw", "gs"])
def test_gsw_pass_is_the_composition_of_pinned_pieces(weighting):
    """Two passes of the iteration equal forward -> update -> adjoint ->
    projection, twice, built from the functions pinned above (FFT, adjoint
    identity, hand-worked update, projection)."""
    h = _small(11, radius=7.0)
    w0 = np.linspace(0.5, 2.0, h.n_foci)
    r = oracle.gsw(h, n_iter=2, w=w0, weighting=weighting)
    phi, w = np.asarray(h.phi0, np.float64), w0
    for _ in range(2):
        phi, w, _th = _one_pass_composed(h, phi, w, weighting)
    on = h.amplitude > 0
    assert np.max(np.abs(np.angle(np.exp(1j * (r["phi"] - phi)))[on])) < 1e-12
    assert np.allclose(r["w"], w, rtol=1e-13, atol=0)


def test_phase_fixed_and_measured_passes_are_compositions():
    """Phase fixing from the second pass uses the second pass's own phasors
    from then on; a measured pass takes its weights from the capture; both
    are the composed pinned pieces."""
    h = _small(12, radius=7.0)
    r = oracle.gsw(h, n_iter=3, phase_fix=2)
    phi, w = np.asarray(h.phi0, np.float64), np.ones(h.n_foci)
    phi, w, _ = _one_pass_composed(h, phi, w)
    th = oracle.forward(oracle.pupil_field(h, phi), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    frozen = th / np.abs(th)
    for _ in range(2):
        phi, w, _ = _one_pass_composed(h, phi, w, fixed=frozen)
    on = h.amplitude > 0
    assert np.max(np.abs(np.angle(np.exp(1j * (r["phi"] - phi)))[on])) < 1e-12
    assert np.allclose(r["w"], w, rtol=1e-13, atol=0)
    meas = np.random.default_rng(3).uniform(0.2, 1.0, h.n_foci)
    w0 = np.linspace(1.0, 1.5, h.n_foci)
    m = oracle.gsw_measured_pass(h, h.phi0, w0, meas)
    phi_c, w_c, _ = _one_pass_composed(h, np.asarray(h.phi0, np.float64), w0, measured=meas)
    assert np.max(np.abs(np.angle(np.exp(1j * (m["phi"] - phi_c)))[on])) < 1e-12
    assert np.allclose(m["w"], w_c, rtol=1e-13, atol=0)


@pytest.mark.parametrize("aperture", ["rect", "disc"])
def test_single_focus_grating_closed_form(aperture):
    """One focus at a non-grid point, uniform amplitude: after one pass the
    phase is the linear grating arg(c) + 2 pi (s_x u x0 + s_y v y0) and the
    next forward field puts all the light on the focus: |Theta|^2 = (sum A)^2,
    accuracy 1 and efficiency 1."""
    ny, nx = 24, 20
    amp = synth_ofa.disc(ny, nx, 10.0).astype(np.float32) if aperture == "disc" \
        else np.ones((ny, nx), np.float32)
    rng = np.random.default_rng(8)
    h = synth_ofa.Hologram("grating", ny, nx, amp, synth_ofa.centred(nx), synth_ofa.centred(ny),
                           1 / nx, 1 / ny, np.array([3.37]), np.array([-2.81]), np.array([0.7]),
                           synth_ofa.initial_phase(rng, ny, nx), n_iter=2)
    r = oracle.gsw(h, n_iter=1)
    th0 = oracle.forward(oracle.pupil_field(h), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)[0]
    ramp = 2 * np.pi * (h.s_x * h.u[None, :] * h.fx[0] + h.s_y * h.v[:, None] * h.fy[0])
    expect = np.angle(th0) + ramp
    on = amp > 0
    d = np.angle(np.exp(1j * (r["phi"] - expect)))
    assert np.max(np.abs(d[on])) < 1e-12
    assert np.all(r["phi"][~on] == 0.0)
    assert abs(r["theta"][0]) ** 2 == pytest.approx(float(amp.sum()) ** 2, rel=1e-12)
    st = oracle.stats(r["theta"], h.target, amp)
    assert st["xi"] == pytest.approx(1.0, abs=1e-12)
    assert st["eta"] == pytest.approx(1.0, rel=1e-12)


def _small(seed=0, ny=16, nx=20, n=7, radius=None):
    return synth_ofa.random_case(seed, ny, nx, n, radius=radius, amplitude="random", n_iter=4)


def test_gsw_scale_invariance():
    """A -> 4 A and targets -> 2 targets leave the phase trajectory unchanged
    (the weighting uses unit-sum intensities; the projection drops scale)."""
    h = _small(1)
    r1 = oracle.gsw(h)
    h.amplitude = (4 * h.amplitude).astype(np.float32)
    h.target = 2 * h.target
    r2 = oracle.gsw(h)
    on = h.amplitude > 0
    assert np.max(np.abs(np.angle(np.exp(1j * (r1["phi"] - r2["phi"])))[on])) < 1e-10
    assert np.allclose(r1["history"][:, 0], r2["history"][:, 0], rtol=0, atol=1e-12)


def test_gsw_translation_adds_linear_ramp():
    """Shifting every focus by (dx, dy) while adding the matching linear phase
    to the start phase leaves all intensities unchanged and adds the same
    ramp to the final phase (Fourier shift theorem through every step)."""
    h = _small(2, radius=8.0)
    r1 = oracle.gsw(h)
    dx, dy = 1.75, -2.5
    ramp = 2 * np.pi * (h.s_x * h.u[None, :] * dx + h.s_y * h.v[:, None] * dy)
    h2 = _small(2, radius=8.0)
    h2.fx = h.fx + dx
    h2.fy = h.fy + dy
    r2 = oracle.gsw(h2, phi=np.asarray(h.phi0, np.float64) + ramp)
    on = h.amplitude > 0
    d = np.angle(np.exp(1j * (r2["phi"] - r1["phi"] - ramp)))
    assert np.max(np.abs(d[on])) < 1e-9
    assert np.allclose(np.abs(r1["theta"]), np.abs(r2["theta"]), rtol=1e-10)


def test_gsw_mirror_conjugates_phase():
    """Foci (x, y) -> (-x, -y) with phi0 -> -phi0 conjugates every field of the
    iteration, so the final phase is negated."""
    h = _small(3)
    r1 = oracle.gsw(h)
    h2 = _small(3)
    h2.fx, h2.fy = -h.fx, -h.fy
    r2 = oracle.gsw(h2, phi=-np.asarray(h.phi0, np.float64))
    on = h.amplitude > 0
    assert np.max(np.abs(np.angle(np.exp(1j * (r1["phi"] + r2["phi"])))[on])) < 1e-10


def test_gsw_termination_before_update():
    """The accuracy test runs before the update: the pass whose forward field
    first exceeds the threshold leaves the phase as it was and is not counted;
    the returned phase equals that of an unstopped run after as many passes."""
    h = _small(4)
    full = oracle.gsw(h, n_iter=8)
    xi = full["history"][:, 0]
    k = next(k for k in range(1, 8) if xi[k] > np.max(xi[:k]))
    stop = 0.5 * (np.max(xi[:k]) + xi[k])
    r = oracle.gsw(h, n_iter=8, stop=stop)
    assert r["iters_done"] == k
    assert r["history"].shape[0] == k + 1
    ref = oracle.gsw(h, n_iter=k)
    assert np.array_equal(r["phi"], ref["phi"])
    # a threshold met by the start phase leaves it untouched
    one = synth_ofa.random_case(5, 12, 12, 1, n_iter=3)
    r1 = oracle.gsw(one, stop=0.5)
    assert r1["iters_done"] == 0
    assert np.array_equal(r1["phi"], one.phi0.astype(np.float64))


def test_gsw_convergence_soft_check():
    """Plausibility, not parity: the paper reports 99% intensity accuracy after
    16 iterations for a 9x9 array with various intensities and efficiency
    above 90% (Sec. 2, Fig. 2(g)-(h)); a 9x9 array on a smaller pupil reaches
    the same regime."""
    rng = np.random.default_rng(9)
    ny = nx = 128
    amp = synth_ofa.disc(ny, nx, 64.0).astype(np.float32)
    fx, fy = synth_ofa.grid_foci(9, 9, 4.39)
    h = synth_ofa.Hologram("9x9", ny, nx, amp, synth_ofa.centred(nx), synth_ofa.centred(ny),
                           1 / nx, 1 / ny, fx, fy, rng.uniform(0.5, 1.0, 81),
                           synth_ofa.initial_phase(rng, ny, nx), n_iter=30)
    r = oracle.gsw(h)
    xi = r["history"][:, 0]
    assert np.max(xi[:25]) > 0.99
    assert oracle.stats(r["theta"], h.target, amp)["eta"] > 0.85


def _grid9x9(n_iter=40):
    rng = np.random.default_rng(9)
    ny = nx = 128
    amp = synth_ofa.disc(ny, nx, 64.0).astype(np.float32)
    fx, fy = synth_ofa.grid_foci(9, 9, 4.39)
    return synth_ofa.Hologram("9x9", ny, nx, amp, synth_ofa.centred(nx), synth_ofa.centred(ny),
                              1 / nx, 1 / ny, fx, fy, rng.uniform(0.5, 1.0, 81),
                              synth_ofa.initial_phase(rng, ny, nx), n_iter=n_iter)


def test_gs_variant_against_the_papers_comparison():
    """Plain GS (unit weights) is the comparison method of Sec. 2: on a 9x9
    array of uneven targets its accuracy stays below 90% while the weighted
    iteration passes 99% (Fig. 2(h)), and its efficiency is at least the
    weighted one's (Fig. 2(g)); its weights never move; with a single focus
    the two iterations coincide."""
    h = _grid9x9()
    r_w = oracle.gsw(h)
    r_g = oracle.gsw(h, weighting="gs")
    assert np.max(r_g["history"][:, 0]) < 0.90
    assert np.max(r_w["history"][:, 0]) > 0.99
    amp = h.amplitude
    assert oracle.stats(r_g["theta"], h.target, amp)["eta"] >= \
        oracle.stats(r_w["theta"], h.target, amp)["eta"]
    assert np.all(r_g["w"] == 1.0)
    h1 = synth_ofa.random_case(60, 48, 40, 1)
    a, b = oracle.gsw(h1, n_iter=4), oracle.gsw(h1, n_iter=4, weighting="gs")
    assert np.array_equal(a["phi"], b["phi"])


@pytest.mark.parametrize("k", [2, 5])
def test_phase_fixing_freezes_from_pass_k(k):
    """Phase fixing from the k-th updating pass: that pass records the
    phasors it would use anyway, so the forward fields of passes 1 .. k+1
    equal the unfixed run's; the next one differs."""
    h = _grid9x9(n_iter=k + 4)
    a = oracle.gsw(h)
    b = oracle.gsw(h, phase_fix=k)
    assert np.array_equal(a["history"][:k + 1], b["history"][:k + 1])
    assert not np.array_equal(a["history"][k + 1], b["history"][k + 1])


def test_phase_fixing_trades_efficiency_for_convergence():
    """Sec. 2 (after Kim et al.): phase fixing speeds up convergence at the
    cost of diffraction efficiency.  Fixed once the weighted iteration has
    settled (pass 8 of the 9x9 array), the accuracy passes 99% sooner and
    the efficiency ends lower."""
    h = _grid9x9()
    a = oracle.gsw(h)
    b = oracle.gsw(h, phase_fix=8)
    first = lambda r: next(i for i, x in enumerate(r["history"][:, 0]) if x > 0.99)  # noqa: E731
    assert first(b) < first(a)
    amp = h.amplitude
    assert oracle.stats(b["theta"], h.target, amp)["eta"] < \
        oracle.stats(a["theta"], h.target, amp)["eta"]


# --------------------------------------------------------------------------
# Gradient (differentiable form)
# --------------------------------------------------------------------------

def test_phase_gradient_matches_central_differences():
    h = synth_ofa.config5_gradcheck()
    rng = np.random.default_rng(10)
    g = rng.standard_normal(h.n_foci)
    phi = np.asarray(h.phi0, np.float64)
    grad, _ = oracle.phase_gradient(h, phi, g)

    def loss(p):
        th = oracle.forward(oracle.pupil_field(h, p), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
        return float(np.dot(g, np.abs(th) ** 2))

    on = np.argwhere(h.amplitude > 0)
    pick = on[rng.choice(on.shape[0], 12, replace=False)]
    eps = 1e-5
    for (j, i) in pick:
        pp, pm = phi.copy(), phi.copy()
        pp[j, i] += eps
        pm[j, i] -= eps
        fd = (loss(pp) - loss(pm)) / (2 * eps)
        assert fd == pytest.approx(grad[j, i], rel=1e-6, abs=1e-6 * np.max(np.abs(grad)))
    off = h.amplitude == 0
    assert np.all(grad[off] == 0.0)


def test_design_loss_gradient_matches_central_differences():
    """dL/dI of the design loss against central differences of L itself."""
    rng = np.random.default_rng(12)
    I = rng.uniform(0.1, 2.0, 25)
    t = rng.uniform(0.5, 1.0, 25)
    t /= t.sum()
    n_ap, sum_a2 = 3000, 2500.0
    L0, dI = oracle.design_loss(I, t, n_ap, sum_a2)
    eps = 1e-6
    for n in range(25):
        ip, im = I.copy(), I.copy()
        ip[n] += eps
        im[n] -= eps
        fd = (oracle.design_loss(ip, t, n_ap, sum_a2)[0] -
              oracle.design_loss(im, t, n_ap, sum_a2)[0]) / (2 * eps)
        assert fd == pytest.approx(dI[n], rel=1e-6, abs=1e-9)
    # special cases: intensities proportional to the target leave only the
    # efficiency term, L = -0.1 eta, and the loss is invariant to the
    # scale of I apart from that term
    L1, _ = oracle.design_loss(7.0 * t, t, n_ap, sum_a2)
    assert L1 == pytest.approx(-0.1 * 7.0 / (n_ap * sum_a2), rel=1e-12)
    La, _ = oracle.design_loss(I, t, n_ap, sum_a2, eta_weight=0.0)
    Lb, _ = oracle.design_loss(3.0 * I, t, n_ap, sum_a2, eta_weight=0.0)
    assert La == pytest.approx(Lb, rel=1e-12)


def test_adam_design_first_step_and_descent():
    """Adam's bias-corrected first step has m^ = g and v^ = g^2, so every
    coordinate moves by lr |g| / (|g| + eps) against the sign of its gradient
    (lr to within lr eps / |g|); coordinates with no gradient (outside the
    aperture) do not move; the loss goes down."""
    h = synth_ofa.config5_gradcheck()
    lr = 0.05
    phi1, hist1 = oracle.adam_design(h, 1, lr=lr)
    phi0 = np.asarray(h.phi0, np.float64)
    amp = np.asarray(h.amplitude, np.float64)
    th = oracle.forward(oracle.pupil_field(h), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    _, gI = oracle.design_loss(np.abs(th) ** 2, h.target, int(np.count_nonzero(amp > 0)),
                               float(np.sum(amp * amp)))
    grad, _ = oracle.phase_gradient(h, phi0, gI)
    step = phi1 - phi0
    on = amp > 0
    assert np.allclose(step[on], -lr * grad[on] / (np.abs(grad[on]) + 1e-8), rtol=0, atol=1e-12)
    big = np.abs(grad) > 1e-4 * np.max(np.abs(grad))
    assert np.all(np.abs(np.abs(step[big]) - lr) <= lr * 1e-8 / np.abs(grad[big]) * 1.0001)
    assert np.all(phi1[amp == 0] == phi0[amp == 0])
    _, hist = oracle.adam_design(h, 25, lr=lr)
    assert hist[0] == pytest.approx(hist1[0], rel=1e-14)
    assert hist[-1] < 0.5 * hist[0]


# --------------------------------------------------------------------------
# Index work
# --------------------------------------------------------------------------

def _brute_unique(c):
    vals = []
    for x in c:
        x = 0.0 if x == 0.0 else float(x)
        if not any(x == y for y in vals):
            vals.append(x)
    vals.sort()
    idx = [sum(1 for y in vals if y < (0.0 if x == 0.0 else x)) for x in c]
    return np.array(vals), np.array(idx)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_index_oracle_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 40
    base = rng.uniform(-5, 5, 12)
    c = base[rng.integers(0, 12, n)]
    c[rng.integers(0, n, 3)] = -0.0
    c[rng.integers(0, n, 3)] = 0.0
    u, idx = oracle.unique_coords(c)
    bu, bidx = _brute_unique(c)
    assert np.array_equal(u, bu) and np.array_equal(idx, bidx)
    assert not np.any(np.signbit(u[u == 0.0]))


def test_index_grid_semantics_reduced_grid():
    """A k x l grid of foci reduces to l unique x and k unique y coordinates
    (the 9x9 reduced sampling grid of Sec. 2 / Fig. 2(c))."""
    fx, fy = synth_ofa.grid_foci(9, 9, 4.39)
    assert oracle.unique_coords(fx)[0].shape[0] == 9
    assert oracle.unique_coords(fy)[0].shape[0] == 9
    fx, fy = synth_ofa.grid_foci(3, 5, 2.0)
    plan = oracle.index_plan(fx, fy, np.ones((4, 4)))
    assert plan["xu"].shape[0] == 5 and plan["yu"].shape[0] == 3
    assert plan["axis"] == 0          # fewer unique y than x: reduce along y
    fx, fy = synth_ofa.grid_foci(5, 3, 2.0)
    assert oracle.index_plan(fx, fy, np.ones((4, 4)))["axis"] == 1


def test_index_compaction_and_csr():
    amp = np.zeros((6, 7))
    amp[1, 2] = 1
    amp[4, 5] = 0.5
    rows, cols = oracle.compaction(amp)
    assert rows.tolist() == [1, 4] and cols.tolist() == [2, 5]
    fx = np.array([1.0, 2.0, 1.0, 3.0])
    fy = np.array([0.5, 0.5, -1.0, 0.5])
    p = oracle.index_plan(fx, fy, amp)
    assert p["yu"].tolist() == [-1.0, 0.5]
    assert p["row_ptr"].tolist() == [0, 1, 4]
    assert p["order"].tolist() == [2, 0, 1, 3]
    assert not p["duplicate"]
    assert oracle.has_duplicate_foci(np.array([0.0, -0.0]), np.array([1.0, 1.0]))


# --------------------------------------------------------------------------
# Units of the paper's system (Table 1, Eq. 3)
# --------------------------------------------------------------------------

def test_table1_zero_padding_and_focal_unit():
    """Table 1: 785 nm, 1000 SLM pixels of 12.5 um, camera pitch 3.45 um,
    f = 250 mm.  Eq. 3 gives the IFTA padding M = M0 lambda / (2 NA dd) = 4550.7
    (the paper quotes 4551); the focal unit lambda f / (M0 p) is 15.7 um, i.e.
    4.55 camera pixels, and 4551 / 20 leaves 227 foci per axis at a 20-pixel gap."""
    lam, m0, p, dd, f = 785e-9, 1000, 12.5e-6, 3.45e-6, 0.25
    na = (m0 * p / 2) / f
    M = m0 * lam / (2 * na * dd)
    assert M == pytest.approx(4550.7, abs=0.05)
    assert math.ceil(M) == 4551
    unit = lam * f / (m0 * p)
    assert unit == pytest.approx(15.7e-6, rel=1e-9)
    assert unit / dd == pytest.approx(M / m0, rel=1e-12)
    assert math.ceil(M) // 20 == 227


def test_config1_aperture_pixel_count():
    h = synth_ofa.config1()
    assert int(np.count_nonzero(h.amplitude)) == 3228
    rows, cols = oracle.compaction(h.amplitude)
    assert rows.shape[0] == 64 and cols.shape[0] == 64


# --------------------------------------------------------------------------
# 3-D foci: the axial position as a defocus phase of the pupil
# --------------------------------------------------------------------------

def test_volume_focal_plane_equals_2d():
    """All foci at z = 0: the 3-D operators are the 2-D ones, exactly."""
    h = synth_ofa.random_case(90, 40, 36, 12)
    E = oracle.pupil_field(h)
    a = oracle.forward(E, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    b = oracle.forward(E, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy, np.zeros(h.n_foci))
    assert np.array_equal(a, b)


def test_volume_defocus_compensated_pupil_focuses_perfectly():
    """A pupil carrying the conjugate of a plane's defocus phase (a lens of
    the opposite power) focuses on that plane as a flat pupil does on the
    focal plane: the on-axis field of plane z is sum A, and off-axis foci on
    that plane see the plain Fourier kernel."""
    ny, nx = 48, 56
    u, v = synth_ofa.centred(nx), synth_ofa.centred(ny)
    sx, sy = 1.0 / nx, 1.0 / ny
    amp = synth_ofa.disc(ny, nx, 22.0).astype(np.float64)
    for z in (-25.0, 12.5, 40.0):
        lens = np.exp(-1j * np.pi * z * ((sy * v[:, None]) ** 2 + (sx * u[None, :]) ** 2))
        th = oracle.forward(amp * lens, u, v, sx, sy, np.array([0.0, 3.0]), np.array([0.0, -2.0]),
                            np.array([z, z]))
        flat = oracle.forward(amp.astype(np.complex128), u, v, sx, sy, np.array([0.0, 3.0]),
                              np.array([0.0, -2.0]))
        assert th[0] == pytest.approx(amp.sum(), rel=1e-12)
        assert abs(th[1] - flat[1]) <= 1e-10 * amp.sum()


def test_volume_adjoint_identity():
    """<P(E), T> = <E, P^H(T)> with foci on several planes."""
    h = synth_ofa.volume_case(91, 30, 34, 5)
    rng = np.random.default_rng(4)
    E = rng.standard_normal((h.ny, h.nx)) + 1j * rng.standard_normal((h.ny, h.nx))
    T = rng.standard_normal(h.n_foci) + 1j * rng.standard_normal(h.n_foci)
    pe = oracle.forward(E, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy, h.fz)
    pt = oracle.adjoint(T, h.ny, h.nx, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy, h.fz)
    lhs = np.vdot(T, pe)
    rhs = np.vdot(pt, E)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_volume_index_pairs_brute_force():
    """Reduced rows and columns are distinct (coordinate, z) pairs, ordered by
    coordinate then z; foci sharing (x, y) on different planes are distinct."""
    fx = np.array([1.0, 1.0, -0.0, 0.0, 2.5, 1.0])
    fy = np.array([0.5, 0.5, 0.5, 0.5, -1.0, 0.5])
    fz = np.array([0.0, 10.0, 10.0, -0.0, 10.0, -5.0])
    xu, ix = oracle.unique_coords(fx, fz)
    # pairs (x, z): (0, 0) (0, 10) (1, -5) (1, 0) (1, 10) (2.5, 10)
    assert list(xu) == [0.0, 0.0, 1.0, 1.0, 1.0, 2.5]
    assert list(ix) == [3, 4, 1, 0, 5, 2]
    assert not oracle.has_duplicate_foci(fx, fy, fz)
    assert oracle.has_duplicate_foci(fx[:2], fy[:2], np.array([10.0, 10.0]))


# --------------------------------------------------------------------------
# Camera in the loop: measured intensities in the weight update
# --------------------------------------------------------------------------

def test_camera_never_switching_is_plain_gsw():
    """A threshold no field reaches leaves Algorithm 1 untouched, bit for bit."""
    h = synth_ofa.config1()
    r = oracle.gsw(h, n_iter=6)
    c = oracle.camera_loop(h, 6, lambda th: np.abs(th) ** 2, xi_switch=2.0)
    assert c["switched"] is None
    assert np.array_equal(c["phi"], r["phi"]) and np.array_equal(c["w"], r["w"])
    assert np.array_equal(c["history"], r["history"])


def test_camera_ideal_and_scaled_match_plain_gsw():
    """A camera that reports |Theta|^2, or any constant multiple of it (its
    gain is unknown), gives Algorithm 1's result: intensities enter the
    weight update only through their unit-sum normalisation."""
    h = synth_ofa.random_case(92, 40, 48, 9, radius=18.0)
    r = oracle.gsw(h, n_iter=5)
    amp = np.asarray(h.amplitude, np.float64)
    for gain in (1.0, 37.5):
        c = oracle.camera_loop(h, 5, lambda th: gain * np.abs(th) ** 2, xi_switch=-np.inf)
        assert c["switched"] == 0
        err = np.linalg.norm(amp * np.exp(1j * c["phi"]) - amp * np.exp(1j * r["phi"]))
        assert err <= 1e-9 * np.linalg.norm(amp)
        assert np.allclose(c["w"], r["w"], rtol=1e-9, atol=0)


def test_camera_compensates_a_per_focus_system_gain():
    """The point of the strategy: with a system that delivers g_n I_n to the
    camera (uneven transmission), feedback from the camera drives the
    MEASURED intensities to the targets, so the computed ones settle near
    t_n / g_n; plain GSW drives the computed ones to the targets instead."""
    h = synth_ofa.config1()
    g = np.random.default_rng(93).uniform(0.6, 1.4, h.n_foci)

    def acc(i, t):
        i, t = i / i.sum(), t / t.sum()
        return 1.0 - np.linalg.norm(t - i) / np.linalg.norm(i)

    r = oracle.gsw(h, n_iter=40)
    c = oracle.camera_loop(h, 40, lambda th: g * np.abs(th) ** 2, xi_switch=0.9)
    assert c["switched"] is not None and c["switched"] > 0
    I_c, I_r = np.abs(c["theta"]) ** 2, np.abs(r["theta"]) ** 2
    assert acc(g * I_c, h.target) > 0.99          # the camera sees the targets
    assert acc(I_c, h.target / g) > 0.99          # the field pre-compensates g
    assert acc(g * I_r, h.target) < 0.95          # plain GSW does not
