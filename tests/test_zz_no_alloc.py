"""The allocation-free forward operator (gswmtp_forward_field_noalloc): the
scratch of the call lives in the library's static device array instead of the
plan's buffers.  Its result must equal gswmtp_forward_field's bit for bit
(same kernels, same data, same order), call after call, when a larger call
is followed by a smaller one (the array keeps the last call's contents), and
the plan's own state must be untouched."""
import numpy as np
import pytest

import synth_ofa
from gpu_util import announce, cuda_ok

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a gfx950 GPU")]


@pytest.fixture(scope="module")
def g():
    import paper_2206_12661_amd as g
    return g


def _field(h, seed):
    rng = np.random.default_rng(seed)
    E = rng.standard_normal((h.ny, h.nx)) + 1j * rng.standard_normal((h.ny, h.nx))
    return np.where(h.amplitude > 0, E, 0).astype(np.complex64)


@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "fp16x3", "bf16x6"])
def test_noalloc_forward_equals_forward_large_then_small(g, mode):
    cases = [synth_ofa.config3(),                                   # 1152 x 1920, 1000 foci
             synth_ofa.random_case(10, 100, 150, 70, amplitude="random")]
    for k, h in enumerate(cases):
        announce(f"noalloc forward {mode} call {k + 1}: {h.ny}x{h.nx} N={h.n_foci}")
        E = _field(h, 50 + k)
        with g.Plan(h, precision=mode) as p:
            ref = p.forward_field(E)
            got = p.forward_field(E, noalloc=True)
            again = p.forward_field(E)            # the plan's own path is unchanged
            th = p.foci_field()                   # the plan's state is untouched
        assert np.array_equal(got, ref), f"call {k + 1}"
        assert np.array_equal(again, ref)
        with g.Plan(h, precision=mode) as q:
            assert np.array_equal(q.foci_field(), th)


def test_noalloc_forward_grid_form(g, monkeypatch):
    """A float32 plan on the dense second product (grid form) uses the
    array for its intermediate products too."""
    monkeypatch.setenv("GSWMTP_SECOND", "grid")
    h = synth_ofa.random_case(12, 96, 96, 0, grid=(7, 5))
    announce("noalloc forward grid form")
    E = _field(h, 60)
    with g.Plan(h) as p:
        ref = p.forward_field(E)
        got = p.forward_field(E, noalloc=True)
    assert np.array_equal(got, ref)


def test_noalloc_forward_rejects_plans_beyond_the_array(g):
    """A 3000 x 3000 pupil needs more than the 64 MiB array: a clear error,
    and the plan keeps working."""
    h = synth_ofa.random_case(13, 3000, 3000, 8)
    announce("noalloc forward beyond the static scratch")
    E = _field(h, 61)
    with g.Plan(h) as p:
        with pytest.raises(g.GswmtpError) as e:
            p.forward_field(E, noalloc=True)
        assert e.value.status == -4
        assert "static" in str(e.value)
        assert p.forward_field(E).shape == (h.n_foci,)
