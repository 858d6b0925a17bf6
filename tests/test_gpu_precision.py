"""Split-precision modes (bfloat16 / float16 term splits on the 16-bit matrix
cores, float32 accumulation) against the FP64 oracle.

Tolerances, derived from the term arithmetic (relative L2 of a product
result, per operand representation error r and dropped term products):
  FP16X3  two float16 terms (11 + 11 significant bits): r <= 2^-24, dropped
          a1 b1 <= 2^-24 -> the float32 bar, 1e-5.
  BF16X6  three bfloat16 terms (3 x 8 bits): r <= 2^-27 -> 1e-5.
  BF16X3  two bfloat16 terms (8 + 8 bits): r <= 2^-18 per operand, dropped
          a1 b1 <= 2^-18 -> at most 3 * 2^-18 = 1.1e-5 per real product;
          stated bar 5e-5 (a 4x margin over that bound for the two products
          and the gather).
"""
import numpy as np
import pytest

import oracle
import synth_ofa
from gpu_util import announce, cuda_ok, rel_l2

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a gfx950 GPU")]

TOL = {"fp16x3": 1e-5, "bf16x6": 1e-5, "bf16x3": 5e-5}
MODES = list(TOL)


@pytest.fixture(scope="module")
def g():
    import paper_2206_12661_amd as g
    return g


def _cases():
    return {
        "ragged-100x150-N70": synth_ofa.random_case(10, 100, 150, 70, amplitude="random"),
        "ragged-130x200-N130-disc": synth_ofa.random_case(11, 130, 200, 130, radius=60.0,
                                                          amplitude="random"),
        "grid-96x96-7x5": synth_ofa.random_case(12, 96, 96, 0, grid=(7, 5)),
        "config1": synth_ofa.config1(),
        "config2": synth_ofa.config2(),
        # split-K tail tiles: the forward's (gather, axis 0) and the adjoint's
        # 64 x 128 direct-loop tiles (store epilogue of the operator call)
        "512x2048-1060": synth_ofa.random_case(47, 512, 2048, 1060),
    }


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("name", list(_cases().keys()))
@pytest.mark.parametrize("mode", MODES)
def test_forward_operator_split(g, mode, name, axis):
    h = _cases()[name]
    rng = np.random.default_rng(7)
    E = rng.standard_normal((h.ny, h.nx)) + 1j * rng.standard_normal((h.ny, h.nx))
    E = np.where(h.amplitude > 0, E, 0).astype(np.complex64)
    announce(f"forward {mode} {name} axis={axis}")
    with g.Plan(h, axis=axis, precision=mode) as p:
        got = p.forward_field(E)
        th = p.foci_field()              # field of the plan's own phi0
    ref = oracle.forward(E.astype(np.complex128), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    ref0 = oracle.forward(oracle.pupil_field(h), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    e1, e2 = rel_l2(got, ref), rel_l2(th, ref0)
    print(f"  rel err {e1:.3e} / phi0 field {e2:.3e}")
    assert e1 <= TOL[mode] and e2 <= TOL[mode]


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("name", list(_cases().keys()))
@pytest.mark.parametrize("mode", MODES)
def test_adjoint_operator_split(g, mode, name, axis):
    h = _cases()[name]
    rng = np.random.default_rng(8)
    T = (rng.standard_normal(h.n_foci) + 1j * rng.standard_normal(h.n_foci)).astype(np.complex64)
    announce(f"adjoint {mode} {name} axis={axis}")
    with g.Plan(h, axis=axis, precision=mode) as p:
        got = p.adjoint_field(T)
        idx = p.index()
    ref = oracle.adjoint(T.astype(np.complex128), h.ny, h.nx, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    kept = np.zeros((h.ny, h.nx), bool)
    kept[np.ix_(idx["rows"], idx["cols"])] = True
    assert np.all(got[~kept] == 0)
    err = rel_l2(got[kept], ref[kept])
    print(f"  rel err {err:.3e}")
    assert err <= TOL[mode]


@pytest.mark.parametrize("scale", [1e-6, 1.0, 3e4])
def test_fp16_amplitude_scaling(g, scale):
    """float16 terms carry the pupil at unit scale whatever the amplitude."""
    h = synth_ofa.random_case(30, 80, 90, 40, amplitude="random")
    h.amplitude = (h.amplitude * scale).astype(np.float32)
    announce(f"fp16 amplitude scale {scale}")
    with g.Plan(h, precision="fp16x3") as p:
        th = p.foci_field()
        p.iterate(2)
        phi = p.phase()
    ref = oracle.forward(oracle.pupil_field(h), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    assert rel_l2(th, ref) <= TOL["fp16x3"]
    assert np.all(np.isfinite(phi))


def _large_case(name):
    if name == "config3":
        return synth_ofa.config3()
    return synth_ofa.random_case(47, 512, 2048, 1060)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", ["config3", "512x2048-1060"])
def test_full_size_forward_split(g, mode, case):
    h = _large_case(case)
    announce(f"large forward {case} {mode}")
    with g.Plan(h, precision=mode) as p:
        th = p.foci_field()
    ref = oracle.forward(oracle.pupil_field(h), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    err = rel_l2(th, ref)
    print(f"  {mode}: rel err {err:.3e}")
    assert err <= TOL[mode]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", ["config3", "512x2048-1060"])
def test_full_size_pass_split(g, mode, case):
    """One split-precision pass at a large size from an identical state after
    5 float32 passes, where the weight update's gain kappa is 1 (asserted):
    weights and the new foci field at the mode's plain bar.  The benchmark
    size (1152 x 1920, 1000 foci) runs the two-term modes on the 16x16-block
    loop (64 x 128 forward tiles, the re-associated adjoint on 48 x 192
    tiles, one round and no split-K tail) and BF16x6 on 64 x 64 tiles with
    the split-K tail; 512 x 2048 with 1060 foci has tile counts that leave a
    short last round, so its products take the split-K tail launches (the
    kernels each stage ran are printed)."""
    h = _large_case(case)
    announce(f"large pass {case} {mode}")
    with g.Plan(h) as p:
        p.iterate(5)
        phi_k, w_k, _ = p.state()
    with g.Plan(h, precision=mode) as q:
        q.set_state(phi_k, w_k, 0)
        q.iterate(1)
        w1 = q.weights()
        th1 = q.foci_field()
        print("  stages:", [q.stage_kernel(i) for i in range(5)])
    hk = synth_ofa.Hologram(h.name, h.ny, h.nx, h.amplitude, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy,
                            h.target, phi_k, 1)
    r = oracle.gsw(hk, n_iter=1, w=w_k)
    thk = oracle.forward(oracle.pupil_field(hk), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    x = np.abs(thk) ** 2 / np.mean(np.abs(thk) ** 2)
    _, tn = oracle.weight_update(thk, h.target, w_k)
    a2 = np.abs(tn) ** 2
    kap = max(1.0, float(np.sqrt(np.sum(a2 / np.maximum(x, 1e-300)) / np.sum(a2))))
    ew, et = rel_l2(w1, r["w"]), rel_l2(th1, r["theta"])
    print(f"  {mode}: kappa {kap:.3f} w {ew:.2e} theta {et:.2e}")
    assert kap < 1.01
    assert ew <= TOL[mode]
    assert et <= TOL[mode]


@pytest.mark.parametrize("mode", MODES)
def test_local_pass_split(g, mode):
    """One pass from an identical, well-conditioned state (after 10 float32
    passes) on both sides."""
    h = synth_ofa.config2()
    announce(f"local pass {mode}")
    with g.Plan(h) as p:
        p.iterate(10)
        phi_k, w_k, _ = p.state()
    with g.Plan(h, precision=mode) as q:
        q.set_state(phi_k, w_k, 0)
        q.iterate(1)
        phi1, w1, th1 = q.phase(), q.weights(), q.foci_field()
    hk = synth_ofa.Hologram(h.name, h.ny, h.nx, h.amplitude, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy,
                            h.target, phi_k, 1)
    r = oracle.gsw(hk, n_iter=1, w=w_k)
    amp = np.asarray(h.amplitude, np.float64)
    e = rel_l2(amp * np.exp(1j * phi1.astype(np.float64)), amp * np.exp(1j * r["phi"]))
    print(f"  {mode}: w {rel_l2(w1, r['w']):.2e} E {e:.2e} theta {rel_l2(th1, r['theta']):.2e}")
    assert rel_l2(w1, r["w"]) <= TOL[mode]
    assert rel_l2(th1, r["theta"]) <= TOL[mode]
    assert e <= 2 * TOL[mode]


@pytest.mark.parametrize("mode", MODES)
def test_split_graph_equals_eager_and_deterministic(g, mode, monkeypatch):
    h = synth_ofa.random_case(31, 130, 100, 50, radius=55.0)
    announce(f"graph/eager/determinism {mode}")
    outs = []
    for env in ("0", "0", "1"):
        monkeypatch.setenv("GSWMTP_NO_GRAPH", env)
        with g.Plan(h, precision=mode) as p:
            p.iterate(9)
            outs.append((p.phase(), p.weights()))
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0]) and np.array_equal(outs[0][1], o[1])


@pytest.mark.parametrize("mode", MODES)
def test_split_phase_roundtrip(g, mode):
    h = synth_ofa.random_case(32, 40, 52, 9, radius=18.0)
    announce(f"set/get phase {mode}")
    with g.Plan(h, precision=mode) as p:
        p.set_phase(h.phi0)
        phi = p.phase()
    on = h.amplitude > 0
    d = np.angle(np.exp(1j * (phi[on].astype(np.float64) - h.phi0[on])))
    bound = 1e-5 if mode == "bf16x3" else 1e-6
    assert np.max(np.abs(d)) < bound
    assert np.all(phi[~on] == 0)


def test_split_gradient_is_unsupported(g):
    import torch
    h = synth_ofa.config5_gradcheck()
    with g.Plan(h, precision="fp16x3") as p:
        with pytest.raises(g.GswmtpError) as e:
            p.phase_gradient_device(torch.zeros(h.n_foci, device="cuda"))
    assert e.value.status == -8
