"""3-D foci (axial positions z through the pupil's defocus phase): the HIP
path through the C ABI against the FP64 oracle.

Bars as for foci on the focal plane: index work bit-exact (reduced rows and
columns are (coordinate, z) pairs); float32 operators within 1e-5 relative
L2; split precisions at their term-arithmetic bars (1e-5 for FP16X3, 5e-5 for
BF16X3); post-update quantities at 1e-5 times the oracle's own condition
numbers kappa and c_E (first-order propagation through the weight update and
the phase projection); whole runs within the oracle's self-sensitivity to a
1e-6 rad perturbation of the start phase.  With every z = 0 (or -0.0) the
plan is the focal-plane plan, bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth_ofa
from gpu_util import announce, cuda_ok, rel_l2

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not cuda_ok(), reason="needs a gfx950 GPU")]

FIELD_TOL = 1e-5
SPLIT_TOL = {"fp16x3": 1e-5, "bf16x3": 5e-5}


@pytest.fixture(scope="module")
def g():
    import paper_2206_12661_amd as g
    return g


def _shared_planes():
    """The same 24 lateral positions on two planes (z = 0 written both as +0.0
    and -0.0, and z = 12.5), coordinates rounded so many are shared."""
    h = synth_ofa.random_case(21, 72, 96, 24, amplitude="random")
    fx, fy = np.round(h.fx), np.round(h.fy * 2) / 2
    key = np.stack([oracle.canonical(fx), oracle.canonical(fy)], 1)
    _, first = np.unique(key, axis=0, return_index=True)
    first = np.sort(first)
    fx, fy = fx[first], fy[first]
    z0 = np.zeros(fx.shape[0])
    z0[::3] = -0.0
    h.fx = np.concatenate([fx, fx])
    h.fy = np.concatenate([fy, fy])
    h.fz = np.concatenate([z0, np.full(fx.shape[0], 12.5)])
    h.target = np.random.default_rng(5).uniform(0.3, 1.0, h.fx.shape[0])
    return h


def _lattice_planes(n, seed):
    """n distinct (x, y, z) foci from a coarse lateral lattice on 7 planes
    (z both signs, -0.0 among them), random order: many foci share a lateral
    coordinate on several planes, so the (coordinate, z) keys span several
    sort chunks."""
    rng = np.random.default_rng(seed)
    h = synth_ofa.volume_case(4, 96, 128, 4)
    xs = np.arange(-40, 41) * 0.9
    ys = np.arange(-30, 31) * 1.1
    zs = np.array([-30.0, -12.5, -0.0, 0.0, 12.5, 30.0, 47.0])
    pick = rng.choice(xs.size * ys.size * zs.size, n, replace=False)
    fx = xs[pick % xs.size]
    fy = ys[(pick // xs.size) % ys.size]
    fz = zs[pick // (xs.size * ys.size)]
    key = np.stack([oracle.canonical(fx), oracle.canonical(fy), oracle.canonical(fz)], 1)
    _, first = np.unique(key, axis=0, return_index=True)   # -0.0 and 0.0 planes merge
    first = np.sort(first)
    h.fx, h.fy, h.fz = fx[first].copy(), fy[first].copy(), fz[first].copy()
    h.target = rng.uniform(0.3, 1.0, h.fx.shape[0])
    return h


def _cases():
    return {
        "lattice-7planes-9000": _lattice_planes(9000, 31),
        "random-3planes-96x128": synth_ofa.volume_case(1, 96, 128, 30),
        "grid-3planes-64x64-disc": synth_ofa.volume_case(2, 64, 64, 0, grid=(5, 4),
                                                         radius=28.0, planes=(-20.0, 0.0, 20.0)),
        "random-5planes-130x200-disc": synth_ofa.volume_case(
            3, 130, 200, 26, planes=(-40.0, -15.0, 0.0, 15.0, 40.0), radius=60.0),
        "shared-lateral-2planes": _shared_planes(),
    }


def _fwd(h, E, sample=None):
    fx, fy, fz = (h.fx, h.fy, h.fz) if sample is None else \
        (h.fx[sample], h.fy[sample], h.fz[sample])
    return oracle.forward(E, h.u, h.v, h.s_x, h.s_y, fx, fy, fz)


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_index_bit_exact(g, name):
    h = _cases()[name]
    announce(f"volume index {name} N={h.n_foci}")
    with g.Plan(h) as p:
        got = p.index()
    ref = oracle.index_plan(h.fx, h.fy, h.amplitude, h.fz)
    for k in ["xu", "yu"]:
        assert got[k].shape == ref[k].shape, k
        assert np.array_equal(got[k].view(np.uint64), ref[k].view(np.uint64)), k
    for k in ["ix", "iy", "rows", "cols"]:
        assert np.array_equal(got[k], ref[k]), k
    assert got["axis"] == ref["axis"]
    assert not ref["duplicate"]


def test_duplicate_triplet_rejected_and_lateral_repeat_accepted(g):
    h = synth_ofa.random_case(22, 32, 32, 6)
    h.fz = np.zeros(6)
    h.fx[3], h.fy[3] = h.fx[1], h.fy[1]
    h.fz[3], h.fz[1] = 7.0, -7.0
    announce("volume duplicate rules")
    with g.Plan(h) as p:                    # same (x, y), different z: allowed
        assert p.n_foci == 6 and p.index()["ux"] == len(set(zip(oracle.canonical(h.fx), h.fz)))
    h.fz[3], h.fz[1] = -0.0, 0.0            # same (x, y, z)
    with pytest.raises(g.GswmtpError) as e:
        g.Plan(h)
    assert e.value.status == -2
    h.fz[3] = np.nan
    with pytest.raises(g.GswmtpError) as e:
        g.Plan(h)
    assert e.value.status == -1


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("name", list(_cases().keys()))
def test_forward_operator(g, name, axis):
    h = _cases()[name]
    rng = np.random.default_rng(17)
    E = rng.standard_normal((h.ny, h.nx)) + 1j * rng.standard_normal((h.ny, h.nx))
    E = np.where(h.amplitude > 0, E, 0).astype(np.complex64)
    announce(f"volume forward {name} axis={axis}")
    with g.Plan(h, axis=axis) as p:
        got = p.forward_field(E)
    err = rel_l2(got, _fwd(h, E.astype(np.complex128)))
    print(f"  rel err {err:.3e}")
    assert err <= FIELD_TOL


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("name", list(_cases().keys()))
def test_adjoint_operator(g, name, axis):
    h = _cases()[name]
    rng = np.random.default_rng(18)
    T = (rng.standard_normal(h.n_foci) + 1j * rng.standard_normal(h.n_foci)).astype(np.complex64)
    announce(f"volume adjoint {name} axis={axis}")
    with g.Plan(h, axis=axis) as p:
        got = p.adjoint_field(T)
        idx = p.index()
    ref = oracle.adjoint(T.astype(np.complex128), h.ny, h.nx, h.u, h.v, h.s_x, h.s_y,
                         h.fx, h.fy, h.fz)
    kept = np.zeros((h.ny, h.nx), bool)
    kept[np.ix_(idx["rows"], idx["cols"])] = True
    assert np.all(got[~kept] == 0)
    err = rel_l2(got[kept], ref[kept])
    print(f"  rel err {err:.3e}")
    assert err <= FIELD_TOL


@pytest.mark.parametrize("mode", list(SPLIT_TOL))
@pytest.mark.parametrize("name", ["random-3planes-96x128", "random-5planes-130x200-disc"])
def test_forward_operator_split(g, mode, name):
    h = _cases()[name]
    rng = np.random.default_rng(19)
    E = rng.standard_normal((h.ny, h.nx)) + 1j * rng.standard_normal((h.ny, h.nx))
    E = np.where(h.amplitude > 0, E, 0).astype(np.complex64)
    announce(f"volume forward {mode} {name}")
    with g.Plan(h, precision=mode) as p:
        got = p.forward_field(E)
    err = rel_l2(got, _fwd(h, E.astype(np.complex128)))
    print(f"  rel err {err:.3e}")
    assert err <= SPLIT_TOL[mode]


def _kappa(theta, target, w):
    x = np.abs(theta) ** 2 / np.mean(np.abs(theta) ** 2)
    _, tn = oracle.weight_update(theta, target, w)
    a2 = np.abs(tn) ** 2
    return max(1.0, float(np.sqrt(np.sum(a2 / np.maximum(x, 1e-300)) / np.sum(a2))))


def _c_E(h, theta_new):
    Ep = oracle.adjoint(theta_new, h.ny, h.nx, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy, h.fz)
    on = h.amplitude > 0
    a2 = np.asarray(h.amplitude, np.float64)[on] ** 2
    m2 = np.abs(Ep[on]) ** 2
    rms2 = np.sum(a2 * m2) / np.sum(a2)
    return max(1.0, float(np.sqrt(np.sum(a2 * rms2 / np.maximum(m2, 1e-300)) / np.sum(a2))))


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_one_pass(g, name):
    h = _cases()[name]
    announce(f"volume one pass {name}")
    with g.Plan(h) as p:
        th0 = p.foci_field()
        p.iterate(1)
        phi, w, th1 = p.phase(), p.weights(), p.foci_field()
    r0 = _fwd(h, oracle.pupil_field(h))
    r = oracle.gsw(h, n_iter=1)
    kap = _kappa(r0, h.target, np.ones(h.n_foci))
    cE = _c_E(h, oracle.weight_update(r0, h.target, np.ones(h.n_foci))[1])
    amp = np.asarray(h.amplitude, np.float64)
    e_field = rel_l2(amp * np.exp(1j * phi.astype(np.float64)), amp * np.exp(1j * r["phi"]))
    print(f"  kappa {kap:.2f} c_E {cE:.2f}: theta0 {rel_l2(th0, r0):.2e} "
          f"w {rel_l2(w, r['w']):.2e} E {e_field:.2e} theta1 {rel_l2(th1, r['theta']):.2e}")
    assert rel_l2(th0, r0) <= FIELD_TOL
    assert rel_l2(w, r["w"]) <= FIELD_TOL * kap
    assert e_field <= FIELD_TOL * kap * cE
    assert rel_l2(th1, r["theta"]) <= FIELD_TOL * kap


@pytest.mark.parametrize("mode", list(SPLIT_TOL))
@pytest.mark.parametrize("name", ["random-3planes-96x128", "random-5planes-130x200-disc"])
def test_one_pass_split_scaled_adjoint(g, mode, name):
    """Split modes on random multi-plane foci: every reduced (row, z) pair
    holds one focus, so the pass runs the re-associated adjoint (Omega_r^H
    with its defocus factor, scaled by Theta', times the fixed conjugated
    Omega_c rows).  One pass from the state after 5 float32 passes against
    the oracle: weights and foci field at the mode's plain bar, the pupil
    field at twice it (as for the focal-plane split passes)."""
    h = _cases()[name]
    announce(f"volume split one pass {mode} {name}")
    with g.Plan(h) as p:
        p.iterate(5)
        phi_k, w_k, _ = p.state()
    with g.Plan(h, precision=mode) as q:
        assert q.stage_kernel(2) == "k_scale_adjoint_split"
        q.set_state(phi_k, w_k, 0)
        q.iterate(1)
        phi1, w1, th1 = q.phase(), q.weights(), q.foci_field()
    hk = synth_ofa.Hologram(h.name, h.ny, h.nx, h.amplitude, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy,
                            h.target, phi_k, 1)
    hk.fz = h.fz
    r = oracle.gsw(hk, n_iter=1, w=w_k)
    amp = np.asarray(h.amplitude, np.float64)
    e = rel_l2(amp * np.exp(1j * phi1.astype(np.float64)), amp * np.exp(1j * r["phi"]))
    ew, et = rel_l2(w1, r["w"]), rel_l2(th1, r["theta"])
    print(f"  {mode}: w {ew:.2e} theta {et:.2e} E {e:.2e}")
    assert ew <= SPLIT_TOL[mode] and et <= SPLIT_TOL[mode]
    assert e <= 2 * SPLIT_TOL[mode]


def test_trajectory_three_planes(g):
    """20 passes on three planes from the seeded start, bounded by the
    oracle's self-sensitivity (floored at 1e-5)."""
    h = synth_ofa.volume_case(4, 96, 96, 12, planes=(-25.0, 0.0, 25.0), radius=44.0)
    announce(f"volume trajectory {h.n_iter} passes N={h.n_foci}")
    with g.Plan(h) as p:
        p.iterate(h.n_iter)
        th = p.foci_field()
        st = p.stats()
    r = oracle.gsw(h)
    rng = np.random.default_rng(98)
    rp = oracle.gsw(h, phi=np.asarray(h.phi0, np.float64) +
                    1e-6 * rng.standard_normal(h.phi0.shape))
    sens = rel_l2(rp["theta"], r["theta"])
    err = rel_l2(th, r["theta"])
    ro = oracle.stats(r["theta"], h.target, h.amplitude)
    print(f"  field {err:.2e} (self-sensitivity {sens:.2e}); xi {st['xi']:.5f} vs "
          f"{ro['xi']:.5f}; uniformity {st['uniformity']:.4f}")
    bound = max(FIELD_TOL, sens)
    assert err <= bound
    assert abs(st["xi"] - ro["xi"]) <= max(1e-5, bound)


def test_zero_z_is_the_focal_plane_plan(g):
    """fz all zero (either sign) reproduces the plan without fz bit for bit."""
    h = synth_ofa.random_case(23, 100, 150, 70, amplitude="random")
    announce("volume z = 0 identity")
    with g.Plan(h) as p:
        p.iterate(3)
        ref_phi, ref_th = p.phase(), p.foci_field()
    for z in (np.zeros(h.n_foci), np.full(h.n_foci, -0.0)):
        with g.Plan(h, fz=z) as p:
            p.iterate(3)
            assert np.array_equal(p.phase(), ref_phi)
            assert np.array_equal(p.foci_field(), ref_th)


def test_full_size_1152x1920_three_planes(g):
    """1152 x 1920 pupil, 999 foci on three planes (z = -30, 0, 30): the forward
    field of phi0 on sampled foci and one pass at the kappa-scaled bar."""
    h = synth_ofa.volume_case(5, 1152, 1920, 333, radius=None, roi=300.0)
    announce(f"volume full size 1152x1920 N={h.n_foci}")
    rng = np.random.default_rng(4)
    sample = np.sort(rng.choice(h.n_foci, 48, replace=False))
    with g.Plan(h) as p:
        th0 = p.foci_field()
        p.iterate(1)
        th1 = p.foci_field()
        w1 = p.weights()
    r0 = _fwd(h, oracle.pupil_field(h))
    r = oracle.gsw(h, n_iter=1)
    r1 = _fwd(h, oracle.pupil_field(h, r["phi"]), sample)
    kap = _kappa(r0, h.target, np.ones(h.n_foci))
    print(f"  kappa {kap:.2f}: theta0 {rel_l2(th0, r0):.2e} w {rel_l2(w1, r['w']):.2e} "
          f"theta1 {rel_l2(th1[sample], r1):.2e}")
    assert rel_l2(th0, r0) <= FIELD_TOL
    assert rel_l2(w1, r["w"]) <= FIELD_TOL * kap
    assert rel_l2(th1[sample], r1) <= FIELD_TOL * kap
