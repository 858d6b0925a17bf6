"""The largest focus count a plan accepts (262144 foci: a 512 x 512 grid on a
1024 x 1024 pupil), float32 (grid form of the second product) and BF16x3
(gather form, many-foci update), checked against the FP64 oracle on sampled
outputs the oracle can compute one by one: the forward field at 64 sampled
foci, the adjoint field at an 8 x 8 sample of pupil points (the oracle's
adjoint evaluated on that sub-grid), and a few passes that stay finite.
Bars as elsewhere: 1e-5 (float32), 5e-5 (BF16x3) relative L2 over the
sample.
"""
import numpy as np
import pytest

import oracle
import synth_ofa
from gpu_util import announce, cuda_ok, rel_l2

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a gfx950 GPU")]

TOL = {"fp32": 1e-5, "bf16x3": 5e-5}


@pytest.fixture(scope="module")
def g():
    import paper_2206_12661_amd as g
    return g


def _max_foci():
    h = synth_ofa.random_case(50, 1024, 1024, 0, grid=(512, 512))
    h.fx, h.fy = synth_ofa.grid_foci(512, 512, 0.45)
    h.target = np.random.default_rng(51).uniform(0.5, 1.0, h.fx.shape[0])
    return h


@pytest.mark.parametrize("mode", list(TOL))
def test_max_foci_count(g, mode):
    h = _max_foci()
    assert h.n_foci == 262144
    rng = np.random.default_rng(52)
    E = (rng.standard_normal((h.ny, h.nx)) + 1j * rng.standard_normal((h.ny, h.nx)))
    T = rng.standard_normal(h.n_foci) + 1j * rng.standard_normal(h.n_foci)
    fs = np.sort(rng.choice(h.n_foci, 64, replace=False))
    rs = np.sort(rng.choice(h.ny, 8, replace=False))
    cs = np.sort(rng.choice(h.nx, 8, replace=False))
    announce(f"max foci 262144 on 1024x1024, {mode}")
    with g.Plan(h, precision=mode) as p:
        fwd = p.forward_field(E.astype(np.complex64))
        adj = p.adjoint_field(T.astype(np.complex64))
        p.iterate(3)
        phi = p.phase()
        st = p.stats()
        hist = p.history()
    ref_f = oracle.forward(E, h.u, h.v, h.s_x, h.s_y, h.fx[fs], h.fy[fs])
    ref_a = oracle.adjoint(T, 8, 8, h.u[cs], h.v[rs], h.s_x, h.s_y, h.fx, h.fy)
    ef, ea = rel_l2(fwd[fs], ref_f), rel_l2(adj[np.ix_(rs, cs)], ref_a)
    print(f"  forward {ef:.2e} adjoint {ea:.2e}; xi after 3 passes {st['xi']:.4f}")
    assert ef <= TOL[mode]
    assert ea <= TOL[mode]
    assert np.all(np.isfinite(phi)) and np.all(np.isfinite(hist))
    assert hist.shape == (3, 3)


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_nonfinite_intensities_status(g, mode):
    """A valid descriptor whose amplitude (3e38 inside the aperture, finite in
    float32) overflows the float32 accumulation of the forward product, so the
    focal field and its intensity sum (kept in float64, which would hold any
    finite float32 field's) become non-finite: the pass runs to its end (no
    fault), and the next call that reads the control block reports
    GSWMTP_E_NONFINITE as an ordinary status, with its message."""
    h = synth_ofa.config1()
    h.amplitude = (np.asarray(h.amplitude, np.float64) * 3e38).astype(np.float32)
    assert np.all(np.isfinite(h.amplitude)) and h.amplitude.max() == np.float32(3e38)
    announce(f"non-finite intensities, amplitude 3e38, {mode}")
    with g.Plan(h, precision=mode) as p:
        p.iterate(2)
        with pytest.raises(g.GswmtpError) as ei:
            p.iterations_done()
        assert ei.value.status == -6
        assert "non-finite" in str(ei.value)


def _free_bytes():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("setting", ["alloc", "alloc:1", "alloc:2"])
def test_fault_inject_alloc_releases_everything(g, monkeypatch, setting):
    """Injected device-allocation failures (the plan's index pool, then its
    product pool) return GSWMTP_E_NOMEM naming the injection, leave no device
    memory behind, and a plan created afterwards works."""
    h = synth_ofa.config3()
    announce(f"fault injection {setting}, 1152x1920 / 1000 foci")
    free0 = _free_bytes()
    monkeypatch.setenv("GSWMTP_FAULT_INJECT", setting)
    with pytest.raises(g.GswmtpError) as ei:
        g.Plan(h)
    assert ei.value.status == -4 and "injected" in str(ei.value)
    monkeypatch.delenv("GSWMTP_FAULT_INJECT")
    assert abs(_free_bytes() - free0) <= (4 << 20)
    with g.Plan(h) as p:
        p.iterate(1)
        assert p.iterations_done() == 1


@pytest.mark.parametrize("setting", ["alloc", "alloc:1"])
def test_fault_inject_alloc_batch(g, monkeypatch, setting):
    """The batch's allocations (tuner scratch, pool) under injection: the
    create fails with GSWMTP_E_NOMEM and releases what it made; the plans stay
    usable and a batch created afterwards runs."""
    hs = [synth_ofa.random_case(60 + i, 96 + 32 * i, 128, 40 + 10 * i) for i in range(3)]
    announce(f"batch fault injection {setting}")
    plans = [g.Plan(h) for h in hs]
    try:
        free0 = _free_bytes()
        monkeypatch.setenv("GSWMTP_FAULT_INJECT", setting)
        with pytest.raises(g.GswmtpError) as ei:
            g.Batch(plans)
        assert ei.value.status == -4 and "injected" in str(ei.value)
        monkeypatch.delenv("GSWMTP_FAULT_INJECT")
        assert abs(_free_bytes() - free0) <= (4 << 20)
        with g.Batch(plans) as b:
            b.iterate(2)
            b.sync()
        assert all(p.iterations_done() == 2 for p in plans)
    finally:
        for p in plans:
            p.close()
