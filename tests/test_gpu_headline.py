"""Parity at the benchmark size (1152 x 1920 pupil, 1000 dart-thrown foci)
and on the 64-hologram workload, at each mode's plain bar.

Every pass here starts from an identical, well-conditioned state on both
sides: the phase and weights the GPU reached after a few float32 passes,
handed to a fresh plan and to the oracle.  From such a state the weight
update's gain kappa is 1 (asserted), so no condition factor enters a bar:
float32 fields 1e-5 relative L2, the split modes their term-arithmetic bars
(FP16X3 and BF16X6 1e-5, BF16X3 5e-5).
"""
import numpy as np
import pytest

import oracle
import synth_ofa
from gpu_util import announce, cuda_ok, rel_l2

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a gfx950 GPU")]

TOL = {"fp32": 1e-5, "fp16x3": 1e-5, "bf16x6": 1e-5, "bf16x3": 5e-5}


@pytest.fixture(scope="module")
def g():
    import paper_2206_12661_amd as g
    return g


@pytest.fixture(scope="module")
def c3_state(g):
    """Config 3 after 5 float32 GPU passes, and the oracle's pass from it."""
    h = synth_ofa.config3()
    announce("config3: 5 float32 passes for the identical start state")
    with g.Plan(h) as p:
        p.iterate(5)
        phi_k, w_k, _ = p.state()
    hk = synth_ofa.Hologram(h.name, h.ny, h.nx, h.amplitude, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy,
                            h.target, phi_k, 1)
    r = oracle.gsw(hk, n_iter=1, w=w_k)
    thk = oracle.forward(oracle.pupil_field(hk), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    return h, phi_k, w_k, r, thk


def _kappa(theta, target, w):
    x = np.abs(theta) ** 2 / np.mean(np.abs(theta) ** 2)
    _, tn = oracle.weight_update(theta, target, w)
    a2 = np.abs(tn) ** 2
    return max(1.0, float(np.sqrt(np.sum(a2 / np.maximum(x, 1e-300)) / np.sum(a2))))


def _field(h, phi):
    return np.asarray(h.amplitude, np.float64) * np.exp(1j * np.asarray(phi, np.float64))


def _one_pass(g, h, phi_k, w_k, mode, env=None, monkeypatch=None, expect_kernel=None):
    if env:
        for k, v in env.items():
            monkeypatch.setenv(k, v)
    with g.Plan(h, precision=mode) as q:
        if expect_kernel:
            assert q.stage_kernel(2) == expect_kernel
        q.set_state(phi_k, w_k, 0)
        q.iterate(1)
        out = (q.phase(), q.weights(), q.foci_field())
    if env:
        for k in env:
            monkeypatch.delenv(k, raising=False)
    return out


def test_fp32_identical_state_pass_config3(g, c3_state):
    """One float32 pass at 1152 x 1920 / 1000 foci from the state after 5
    passes: weights, the new foci field and the pupil field at the plain
    float32 bar."""
    h, phi_k, w_k, r, thk = c3_state
    kap = _kappa(thk, h.target, w_k)
    announce("config3 float32 identical-state pass")
    phi1, w1, th1 = _one_pass(g, h, phi_k, w_k, "fp32")
    ew, et = rel_l2(w1, r["w"]), rel_l2(th1, r["theta"])
    ee = rel_l2(_field(h, phi1), _field(h, r["phi"]))
    print(f"  kappa {kap:.3f}: w {ew:.2e} theta {et:.2e} E {ee:.2e}")
    assert kap < 1.01
    assert ew <= TOL["fp32"] and et <= TOL["fp32"] and ee <= TOL["fp32"]


def test_fp32_adjoint_operator_config3(g):
    """The float32 adjoint operator at 1152 x 1920 with K = 1000 foci, every
    pupil sample against the oracle's double sum."""
    h = synth_ofa.config3()
    rng = np.random.default_rng(31)
    T = (rng.standard_normal(h.n_foci) + 1j * rng.standard_normal(h.n_foci)).astype(np.complex64)
    announce("config3 float32 adjoint operator")
    with g.Plan(h) as p:
        got = p.adjoint_field(T)
    ref = oracle.adjoint(T.astype(np.complex128), h.ny, h.nx, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    err = rel_l2(got, ref)
    rows = rng.choice(h.ny, 16, replace=False)
    row_err = max(rel_l2(got[j], ref[j]) for j in rows)
    print(f"  rel err {err:.2e}, worst of 16 sampled rows {row_err:.2e}")
    assert err <= TOL["fp32"] and row_err <= TOL["fp32"]


def test_fp32_forward_operator_config3(g):
    """The float32 forward operator of a random (not phase-only) field at the
    benchmark size, every focus."""
    h = synth_ofa.config3()
    rng = np.random.default_rng(32)
    E = (rng.standard_normal((h.ny, h.nx)) + 1j * rng.standard_normal((h.ny, h.nx)))
    E = E.astype(np.complex64)
    announce("config3 float32 forward operator")
    with g.Plan(h) as p:
        got = p.forward_field(E)
    ref = oracle.forward(E.astype(np.complex128), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    err = rel_l2(got, ref)
    print(f"  rel err {err:.2e}")
    assert err <= TOL["fp32"]


@pytest.mark.parametrize("mode", ["bf16x3", "fp16x3", "bf16x6"])
def test_split_adjoint_forms_config3(g, c3_state, mode, monkeypatch):
    """The re-associated split adjoint ((Omega_r^H diag Theta') times the
    conjugated Omega_c rows of the foci), which the benchmark size runs in
    every split mode, and the scatter form: one pass each from the identical
    state, both against the oracle and against each other at the mode's
    plain bar."""
    h, phi_k, w_k, r, thk = c3_state
    assert _kappa(thk, h.target, w_k) < 1.01
    announce(f"config3 {mode} adjoint forms")
    outs = {
        "scaled": _one_pass(g, h, phi_k, w_k, mode, expect_kernel="k_scale_adjoint_split"),
        "scatter": _one_pass(g, h, phi_k, w_k, mode, env={"GSWMTP_ADJOINT": "scatter"},
                             monkeypatch=monkeypatch, expect_kernel="focus_scatter_split"),
    }
    for form, (phi1, w1, th1) in outs.items():
        ew, et = rel_l2(w1, r["w"]), rel_l2(th1, r["theta"])
        ee = rel_l2(_field(h, phi1), _field(h, r["phi"]))
        print(f"  {form}: w {ew:.2e} theta {et:.2e} E {ee:.2e}")
        assert ew <= TOL[mode] and et <= TOL[mode] and ee <= TOL[mode]
    (pa, wa, ta), (pb, wb, tb) = outs["scaled"], outs["scatter"]
    assert rel_l2(_field(h, pa), _field(h, pb)) <= TOL[mode]
    assert rel_l2(wa, wb) <= TOL[mode] and rel_l2(ta, tb) <= TOL[mode]


def _config4_subset():
    hs = synth_ofa.config4()
    order = sorted(range(len(hs)), key=lambda k: hs[k].ny * hs[k].nx * hs[k].fx.shape[0])
    return [hs[k] for k in order[:8] + order[-1:]]


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_batch_config4_subset_against_oracle(g, mode):
    """The 64-hologram workload's 8 smallest holograms and its largest,
    batched: 4 batched float32 passes give each plan a well-conditioned
    state; a second batch in the mode under test then runs one pass from
    exactly that state, and every plan's weights, foci field and pupil field
    are held to the oracle's pass from the same state at the plain bar."""
    sel = _config4_subset()
    announce(f"config4 subset of {len(sel)} vs oracle, {mode}")
    plans = [g.Plan(h) for h in sel]
    with g.Batch(plans) as b:
        b.iterate(4)
    states = [p.state() for p in plans]
    for p in plans:
        p.close()
    plans = [g.Plan(h, precision=mode) for h in sel]
    for p, (phi_k, w_k, _) in zip(plans, states):
        p.set_state(phi_k, w_k, 0)
    with g.Batch(plans) as b:
        b.iterate(1)
    for h, p, (phi_k, w_k, _) in zip(sel, plans, states):
        hk = synth_ofa.Hologram(h.name, h.ny, h.nx, h.amplitude, h.u, h.v, h.s_x, h.s_y,
                                h.fx, h.fy, h.target, phi_k, 1)
        r = oracle.gsw(hk, n_iter=1, w=w_k)
        thk = oracle.forward(oracle.pupil_field(hk), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
        kap = _kappa(thk, h.target, w_k)
        ew, et = rel_l2(p.weights(), r["w"]), rel_l2(p.foci_field(), r["theta"])
        ee = rel_l2(_field(h, p.phase()), _field(h, r["phi"]))
        print(f"  {h.name}: kappa {kap:.3f} w {ew:.2e} theta {et:.2e} E {ee:.2e}")
        assert kap < 1.01
        assert ew <= TOL[mode] and et <= TOL[mode] and ee <= TOL[mode]
        p.close()


@pytest.mark.parametrize("mode", ["bf16x3", "fp16x3"])
def test_d16_forward_loop_config3(g, c3_state, mode, monkeypatch):
    """The forward product with the fused focus gather on the 16x16-block loop
    (64 x 128 tiles, the default at this size; GSWMTP_FWD_LOOP=d16 asserts it)
    at the benchmark size: the field of phi0 at every focus, and one pass
    from the identical state, against the oracle at the mode's bar."""
    h, phi_k, w_k, r, thk = c3_state
    monkeypatch.setenv("GSWMTP_FWD_LOOP", "d16")
    announce(f"config3 {mode} forward on the 16x16-block loop")
    with g.Plan(h, precision=mode) as p:
        assert p.stage_kernel(0) == "cgemm_split_d16"
        th0 = p.foci_field()
    ref0 = oracle.forward(oracle.pupil_field(h), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    phi1, w1, th1 = _one_pass(g, h, phi_k, w_k, mode)
    e0, ew, et = rel_l2(th0, ref0), rel_l2(w1, r["w"]), rel_l2(th1, r["theta"])
    ee = rel_l2(_field(h, phi1), _field(h, r["phi"]))
    print(f"  phi0 field {e0:.2e}; pass: w {ew:.2e} theta {et:.2e} E {ee:.2e}")
    assert e0 <= TOL[mode] and ew <= TOL[mode] and et <= TOL[mode] and ee <= TOL[mode]
