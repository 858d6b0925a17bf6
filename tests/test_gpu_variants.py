"""The iteration variants of Sec. 2 on the GPU: plain GS weighting and phase
fixing, against the FP64 oracle and against the GPU's own unfixed runs.

Bars: bit-exact where the variant leaves the arithmetic unchanged (passes up
to the fixing pass, chunked vs one-call runs, batched vs single plans); the
trajectory bar of the parity tests elsewhere (max(1e-5, the oracle's own
divergence under a 1e-6 rad perturbation of the start phase)).
"""
import numpy as np
import pytest

import oracle
import synth_ofa
from gpu_util import announce, cuda_ok, rel_l2

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a gfx950 GPU")]


@pytest.fixture(scope="module")
def g():
    import paper_2206_12661_amd as g
    return g


def _traj_bound(h, n, **kw):
    r = oracle.gsw(h, n_iter=n, **kw)
    rng = np.random.default_rng(99)
    rp = oracle.gsw(h, n_iter=n, phi=np.asarray(h.phi0, np.float64) +
                    1e-6 * rng.standard_normal(h.phi0.shape), **kw)
    return r, max(1e-5, rel_l2(rp["theta"], r["theta"]))


@pytest.mark.parametrize("mode", ["fp32", "fp16x3"])
@pytest.mark.parametrize("k", [3, 7])
def test_phase_fixing_leaves_passes_up_to_k_unchanged(g, mode, k):
    h = synth_ofa.config1()
    announce(f"phase fixing {mode} k={k}")
    with g.Plan(h, precision=mode) as p:
        p.iterate(k + 4)
        ha = p.history()
    with g.Plan(h, precision=mode) as p:
        p.set_phase_fixing(k)
        p.iterate(k + 4)
        hb = p.history()
    assert np.array_equal(ha[:k + 1], hb[:k + 1])
    assert not np.array_equal(ha[k + 1:], hb[k + 1:])


@pytest.mark.parametrize("k", [4, 8])
def test_phase_fixing_against_oracle(g, k):
    h = synth_ofa.config1()
    n = 20
    announce(f"phase fixing vs oracle k={k}")
    with g.Plan(h) as p:
        p.set_phase_fixing(k)
        p.iterate(n)
        th = p.foci_field()
        hist = p.history()
    r, bound = _traj_bound(h, n, phase_fix=k)
    err = rel_l2(th, r["theta"])
    dxi = np.max(np.abs(hist[:, 0] - r["history"][:, 0]))
    print(f"  field {err:.2e} (bound {bound:.2e}) max|dxi| {dxi:.2e}")
    assert err <= bound
    assert dxi <= max(1e-5, bound)


def test_gs_weighting_against_oracle(g):
    h = synth_ofa.config1()
    n = 12
    announce("GS weighting vs oracle")
    with g.Plan(h, weighting="gs") as p:
        p.iterate(n)
        th = p.foci_field()
        w = p.weights()
    r, bound = _traj_bound(h, n, weighting="gs")
    err = rel_l2(th, r["theta"])
    print(f"  field {err:.2e} (bound {bound:.2e})")
    assert err <= bound
    assert np.all(w == 1.0)


def test_phase_fixing_persists_across_calls(g):
    h = synth_ofa.random_case(61, 90, 110, 40, radius=45.0)
    announce("phase fixing chunked")
    with g.Plan(h) as p:
        p.set_phase_fixing(5)
        p.iterate(13)
        a = (p.phase(), p.weights())
    with g.Plan(h) as p:
        p.set_phase_fixing(5)
        p.iterate(3)
        p.iterate(2)
        p.iterate(8)
        b = (p.phase(), p.weights())
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_phase_fixing_batched_equals_single(g, monkeypatch):
    monkeypatch.setenv("GSWMTP_NO_SPLITK", "1")
    monkeypatch.setenv("GSWMTP_BATCH_TILE", "64x64")
    monkeypatch.setenv("GSWMTP_SECOND", "gather")
    hs = [synth_ofa.config1(), synth_ofa.random_case(62, 100, 80, 30)]
    announce("phase fixing batched")
    single = []
    for h in hs:
        with g.Plan(h) as p:
            p.set_phase_fixing(4)
            p.iterate(10)
            single.append((p.phase(), p.weights()))
    plans = [g.Plan(h) for h in hs]
    for p in plans:
        p.set_phase_fixing(4)
    with g.Batch(plans) as b:
        b.iterate(10)
    for p, s in zip(plans, single):
        assert np.array_equal(p.phase(), s[0]) and np.array_equal(p.weights(), s[1])
        p.close()


def test_phase_fixing_rejects_negative(g):
    h = synth_ofa.random_case(63, 40, 40, 6)
    with g.Plan(h) as p:
        with pytest.raises(g.GswmtpError) as e:
            p.set_phase_fixing(-1)
        assert e.value.status == -1
