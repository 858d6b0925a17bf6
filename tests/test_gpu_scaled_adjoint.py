"""The re-associated adjoint of the split modes: when every reduced row holds
one focus (N = U_r), Omega_r^H S is formed as (Omega_r^H diag Theta') times
the conjugated Omega_c rows of the foci, with no scatter into S.  It must
agree with the scatter form (GSWMTP_ADJOINT=scatter) and with the FP64 oracle
to each mode's bar, with ragged row counts (U_r below the 32-row k-block and
the 64-row padding), at the benchmark size (1152 x 1920, 1000 foci: the
48 x 192 adjoint tiles of the 16x16-block loop) and under graph replay."""
import numpy as np
import pytest

import oracle
import synth_ofa
from gpu_util import announce, cuda_ok, rel_l2

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a gfx950 GPU")]

# the split modes' bars (same derivation as the split-precision tests)
TOL = {"fp16x3": 1e-5, "bf16x6": 1e-5, "bf16x3": 5e-5}
MODES = list(TOL)


@pytest.fixture(scope="module")
def g():
    import paper_2206_12661_amd as g
    return g


def _cases():
    return {
        "config2": synth_ofa.config2(),
        "config3-1152x1920-1000": synth_ofa.config3(),
        "ragged-100x150-N70": synth_ofa.random_case(10, 100, 150, 70, amplitude="random"),
        "ragged-130x200-N45-disc": synth_ofa.random_case(11, 130, 200, 45, radius=60.0),
    }


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_scaled_form_is_selected_for_one_focus_per_row(g, name):
    h = _cases()[name]
    announce(f"scaled adjoint selection {name}")
    for axis in (0, 1):
        with g.Plan(h, axis=axis, precision="bf16x3") as p:
            idx = p.index()
            ur = idx["uy"] if idx["axis"] == 0 else idx["ux"]
            want = "k_scale_adjoint_split" if ur == h.fx.size else "focus_scatter_split"
            assert p.stage_kernel(2) == want


def test_scatter_form_kept_when_rows_share_foci(g):
    h = synth_ofa.config1()          # 4 x 4 grid: four foci per reduced row
    announce("scaled adjoint not selected on a grid")
    with g.Plan(h, precision="bf16x3") as p:
        assert p.stage_kernel(2) == "focus_scatter_split"
    with g.Plan(h) as p:             # float32 keeps its own scatter
        assert p.stage_kernel(2) == "focus_scatter"


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("name", list(_cases().keys()))
@pytest.mark.parametrize("mode", MODES)
def test_scaled_pass_matches_scatter_and_oracle(g, mode, name, axis, monkeypatch):
    """One pass from an identical, well-conditioned state (10 float32
    passes) in both adjoint forms and in the oracle."""
    h = _cases()[name]
    announce(f"scaled adjoint pass {mode} {name} axis={axis}")
    with g.Plan(h, axis=axis) as p:
        p.iterate(10)
        phi_k, w_k, _ = p.state()
    out = {}
    for form in ("scaled", "scatter"):
        if form == "scatter":
            monkeypatch.setenv("GSWMTP_ADJOINT", "scatter")
        with g.Plan(h, axis=axis, precision=mode) as q:
            if form == "scatter":
                assert q.stage_kernel(2) == "focus_scatter_split"
            q.set_state(phi_k, w_k, 0)
            q.iterate(1)
            out[form] = (q.phase(), q.weights(), q.foci_field())
        monkeypatch.delenv("GSWMTP_ADJOINT", raising=False)
    hk = synth_ofa.Hologram(h.name, h.ny, h.nx, h.amplitude, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy,
                            h.target, phi_k, 1)
    r = oracle.gsw(hk, n_iter=1, w=w_k)
    amp = np.asarray(h.amplitude, np.float64)
    field = lambda phi: amp * np.exp(1j * phi.astype(np.float64))
    for form, (phi1, w1, th1) in out.items():
        e = rel_l2(field(phi1), field(r["phi"]))
        print(f"  {form}: w {rel_l2(w1, r['w']):.2e} E {e:.2e} "
              f"theta {rel_l2(th1, r['theta']):.2e}")
        assert rel_l2(w1, r["w"]) <= TOL[mode]
        assert rel_l2(th1, r["theta"]) <= TOL[mode]
        assert e <= 2 * TOL[mode]
    (pa, wa, _), (pb, wb, _) = out["scaled"], out["scatter"]
    assert rel_l2(field(pa), field(pb)) <= 2 * TOL[mode]
    assert rel_l2(wa, wb) <= 2 * TOL[mode]


@pytest.mark.parametrize("mode", MODES)
def test_scaled_form_many_passes_graph_and_early_stop(g, mode, monkeypatch):
    """Nine graph-replayed passes equal nine eager ones bit for bit, and a
    stop accuracy ends the run at the same pass in both adjoint forms."""
    h = synth_ofa.random_case(31, 130, 100, 50, radius=55.0)
    announce(f"scaled adjoint graph/eager/stop {mode}")
    outs = []
    for env in ("0", "1"):
        monkeypatch.setenv("GSWMTP_NO_GRAPH", env)
        with g.Plan(h, precision=mode) as p:
            assert p.stage_kernel(2) == "k_scale_adjoint_split"
            p.iterate(9)
            outs.append((p.phase(), p.weights()))
    monkeypatch.delenv("GSWMTP_NO_GRAPH", raising=False)
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    with g.Plan(h, precision=mode) as p:
        p.iterate(20)
        xi = p.history()[:, 0]
    # a threshold halfway into the first clear rise of xi after pass 3
    k = next(k for k in range(3, 20) if xi[k] > np.max(xi[:k]) + 1e-3)
    stop = 0.5 * (np.max(xi[:k]) + xi[k])
    for form in ("scaled", "scatter"):
        if form == "scatter":
            monkeypatch.setenv("GSWMTP_ADJOINT", "scatter")
        with g.Plan(h, precision=mode) as p:
            p.iterate(20, stop)
            assert p.iterations_done() == k, form
        monkeypatch.delenv("GSWMTP_ADJOINT", raising=False)


@pytest.mark.parametrize("form", ["scaled", "scatter"])
@pytest.mark.parametrize("mode", ["bf16x3", "fp16x3"])
def test_d16_adjoint_loop_forced(g, mode, form, monkeypatch):
    """The 16x16-block adjoint loop (48 x 192 tiles, B straight into
    registers) forced on a 384 x 576 pupil (8 x 3 tiles), both adjoint forms:
    the adjoint operator and one pass from a well-conditioned state against
    the oracle at the mode's bar, and against the 64 x 64 loop."""
    h = synth_ofa.random_case(48, 384, 576, 150, amplitude="random")
    announce(f"d16 adjoint forced {mode} {form}")
    if form == "scatter":
        monkeypatch.setenv("GSWMTP_ADJOINT", "scatter")
    with g.Plan(h) as p:
        p.iterate(6)
        phi_k, w_k, _ = p.state()
    rng = np.random.default_rng(9)
    T = (rng.standard_normal(h.n_foci) + 1j * rng.standard_normal(h.n_foci)).astype(np.complex64)
    out = {}
    for loop in ("d16", "default"):
        monkeypatch.setenv("GSWMTP_ADJ_LOOP", loop)
        with g.Plan(h, precision=mode) as q:
            assert (q.stage_kernel(3) == "cgemm_split_d16") == (loop == "d16")
            adj = q.adjoint_field(T)
            q.set_state(phi_k, w_k, 0)
            q.iterate(1)
            out[loop] = (adj, q.phase(), q.weights(), q.foci_field())
    ref = oracle.adjoint(T.astype(np.complex128), h.ny, h.nx, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    hk = synth_ofa.Hologram(h.name, h.ny, h.nx, h.amplitude, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy,
                            h.target, phi_k, 1)
    r = oracle.gsw(hk, n_iter=1, w=w_k)
    amp = np.asarray(h.amplitude, np.float64)
    field = lambda phi: amp * np.exp(1j * phi.astype(np.float64))
    for loop, (adj, phi1, w1, th1) in out.items():
        ea, ew, et = rel_l2(adj, ref), rel_l2(w1, r["w"]), rel_l2(th1, r["theta"])
        ee = rel_l2(field(phi1), field(r["phi"]))
        print(f"  {loop}: adjoint {ea:.2e} w {ew:.2e} theta {et:.2e} E {ee:.2e}")
        assert ea <= TOL[mode] and ew <= TOL[mode] and et <= TOL[mode] and ee <= 2 * TOL[mode]
    a, b = out["d16"], out["default"]
    assert rel_l2(a[0], b[0]) <= TOL[mode]
    assert rel_l2(field(a[1]), field(b[1])) <= 2 * TOL[mode]
