"""Plans whose device memory is a caller's workspace (a torch tensor): the
size the library reports is enough, the plan then behaves bit for bit like a
plan that allocates for itself, a short workspace is refused cleanly, and the
workspace outlives the plan untouched by its destruction.
"""
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


def _cases():
    return {
        "config1-fp32": (synth_ofa.config1(), "fp32"),
        "grid-96x96-7x5-fp32": (synth_ofa.random_case(12, 96, 96, 0, grid=(7, 5)), "fp32"),
        "ragged-130x200-bf16x3": (synth_ofa.random_case(11, 130, 200, 130, radius=60.0,
                                                        amplitude="random"), "bf16x3"),
        "volume-96x128-fp16x3": (synth_ofa.volume_case(1, 96, 128, 30), "fp16x3"),
        "config3-bf16x3": (synth_ofa.config3(), "bf16x3"),
    }


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_workspace_plan_is_bit_identical(g, name):
    import torch
    h, prec = _cases()[name]
    n = g.Plan.workspace_size(h, precision=prec)
    announce(f"workspace {name}: {n} bytes")
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    with g.Plan(h, precision=prec) as p:
        p.iterate(4)
        ref_phi, ref_th, ref_w = p.phase(), p.foci_field(), p.weights()
    with g.Plan(h, precision=prec, workspace=ws) as q:
        q.iterate(4)
        phi, th, w = q.phase(), q.foci_field(), q.weights()
    assert np.array_equal(phi, ref_phi)
    assert np.array_equal(th, ref_th)
    assert np.array_equal(w, ref_w)


def test_short_workspace_is_refused_and_outlives_the_plan(g):
    import torch
    h = synth_ofa.random_case(40, 72, 96, 50, amplitude="random")
    n = g.Plan.workspace_size(h)
    announce(f"short workspace ({n} bytes needed)")
    short = torch.zeros(n - 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(g.GswmtpError) as e:
        g.Plan(h, workspace=short)
    assert e.value.status == -4
    assert "needed" in str(e.value) or "smaller" in str(e.value)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    with g.Plan(h, workspace=ws) as p:
        p.iterate(2)
    ws.fill_(7)                      # still the caller's, still usable
    torch.cuda.synchronize()
    assert int(ws[-1]) == 7 and int(ws[0]) == 7
