"""Differentiable form: phase design by gradient descent through the library's
forward product and adjoint-gradient epilogue, against the FP64 oracle.

Bars: gradients of the design loss within 1e-4 relative L2 of the oracle's
chain rule (dL/dI has a cancellation between its two terms that float32
intensities feed with ~1e-6 relative error, amplified by up to ~10x at these
cases; 1e-4 keeps a further 10x margin).  Adam trajectories: the oracle's own
sensitivity to a float32-sized (1e-6 rad) perturbation of the start phase,
times ten, floored at 1e-5 - Adam normalises every coordinate's step, so
float32 rounding of tiny gradient components moves phases by up to lr per
step and nothing tighter holds over many steps.
"""
import time

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


def _medium():
    h = synth_ofa.random_case(50, 200, 300, 0, radius=90.0, grid=(8, 8))
    return h


def _oracle_grad(h, phi):
    amp = np.asarray(h.amplitude, np.float64)
    th = oracle.forward(oracle.pupil_field(h, phi), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    I = np.abs(th) ** 2
    L, gI = oracle.design_loss(I, h.target, int(np.count_nonzero(amp > 0)),
                               float(np.sum(amp * amp)))
    grad, _ = oracle.phase_gradient(h, phi, gI)
    return L, grad, I


@pytest.mark.parametrize("case", ["gradcheck-64x64-4x4", "disc-200x300-8x8"])
def test_design_loss_gradient(g, case):
    import torch
    h = synth_ofa.config5_gradcheck() if case.startswith("gradcheck") else _medium()
    announce(f"design-loss gradient {case}")
    with g.Plan(h) as p:
        idx = p.index()
        phi = torch.tensor(h.phi0, device="cuda", requires_grad=True)
        t = torch.tensor(h.target, device="cuda", dtype=torch.float32)
        loss = g.design_loss(g.foci_intensity(phi, p), t, idx["n_aperture"], idx["sum_a2"])
        loss.backward()
        gphi = phi.grad.cpu().numpy()
        L_gpu = float(loss)
    L, ref, _ = _oracle_grad(h, np.asarray(h.phi0, np.float64))
    err = rel_l2(gphi, ref)
    print(f"  loss {L_gpu:.6e} vs {L:.6e}; gradient rel err {err:.2e}")
    assert L_gpu == pytest.approx(L, rel=1e-5, abs=1e-7)
    assert err <= 1e-4
    assert np.all(gphi[h.amplitude == 0] == 0)


def test_adam_trajectory(g):
    import torch
    h = synth_ofa.config5_gradcheck()
    steps = 30
    announce(f"Adam {steps} steps, 64x64 / 16 foci")
    with g.Plan(h) as p:
        phi, hist = g.adam_design(p, steps, phi0=h.phi0, target=h.target)
        phi = phi.cpu().numpy().astype(np.float64)
        hist = hist.cpu().numpy().astype(np.float64)
    phi_o, hist_o = oracle.adam_design(h, steps)
    # the oracle against itself from a start phase perturbed by 1e-6 rad
    rng = np.random.default_rng(3)
    phi_p, hist_p = oracle.adam_design(h, steps, phi=np.asarray(h.phi0, np.float64) +
                                       1e-6 * rng.standard_normal(h.phi0.shape))
    amp = np.asarray(h.amplitude, np.float64)
    field = lambda ph: amp * np.exp(1j * ph)  # noqa: E731
    sens_f = rel_l2(field(phi_p), field(phi_o))
    sens_l = np.max(np.abs(hist_p - hist_o))
    e_f = rel_l2(field(phi), field(phi_o))
    e_l = np.max(np.abs(hist - hist_o))
    print(f"  field {e_f:.2e} (oracle self-sensitivity {sens_f:.2e}); "
          f"loss {e_l:.2e} (self {sens_l:.2e}); loss {hist_o[0]:.4e} -> {hist_o[-1]:.4e}")
    assert e_f <= max(10 * sens_f, 1e-5)
    assert e_l <= max(10 * sens_l, 1e-5 * np.max(np.abs(hist_o)))


def test_c5_step0_gradient_full_size(g):
    """The design-loss gradient of the full 1152 x 1920 / 50 x 50 design at
    its start phase, every pixel, against the oracle's chain rule (dL/dI from
    the loss, then dL/dphi = 2 Im(conj(E) P^H(dL/dI * Theta)), Sec. 2 forward
    model and its adjoint)."""
    import torch
    h = synth_ofa.config5()
    announce("C-5 step-0 gradient, 1152x1920 / 50x50 grid")
    with g.Plan(h) as p:
        idx = p.index()
        phi = torch.tensor(h.phi0, device="cuda", requires_grad=True)
        t = torch.tensor(h.target, device="cuda", dtype=torch.float32)
        loss = g.design_loss(g.foci_intensity(phi, p), t, idx["n_aperture"], idx["sum_a2"])
        loss.backward()
        gphi = phi.grad.cpu().numpy().astype(np.float64)
        L_gpu = float(loss)
    L, ref, _ = _oracle_grad(h, np.asarray(h.phi0, np.float64))
    err = rel_l2(gphi, ref)
    worst = float(np.max(np.abs(gphi - ref)) / np.max(np.abs(ref)))
    print(f"  loss {L_gpu:.6e} vs {L:.6e}; gradient rel L2 {err:.2e}, max {worst:.2e}")
    assert L_gpu == pytest.approx(L, rel=1e-5, abs=1e-7)
    assert err <= 1e-4
    assert worst <= 1e-3


@pytest.mark.parametrize("case", ["gradcheck-64x64-4x4", "disc-200x300-8x8"])
def test_adam_graph_replay_equals_eager(g, case):
    """The captured-and-replayed design step is the eager one: same phases and
    losses, bit for bit, over 20 steps (both run Adam's device-side step
    count; the library's kernels are deterministic)."""
    h = synth_ofa.config5_gradcheck() if case.startswith("gradcheck") else _medium()
    announce(f"Adam graph vs eager, {case}")
    with g.Plan(h) as p:
        phi_g, hist_g = g.adam_design(p, 20, phi0=h.phi0, target=h.target, graph=True)
        phi_e, hist_e = g.adam_design(p, 20, phi0=h.phi0, target=h.target, graph=False)
        phi_g, phi_e = phi_g.cpu().numpy(), phi_e.cpu().numpy()
        hist_g, hist_e = hist_g.cpu().numpy(), hist_e.cpu().numpy()
    print(f"  max |dphi| {np.max(np.abs(phi_g - phi_e)):.3e}, "
          f"max |dloss| {np.max(np.abs(hist_g - hist_e)):.3e}")
    assert hist_g.shape == (20,) and np.all(np.isfinite(hist_g))
    assert np.array_equal(phi_g, phi_e)
    assert np.array_equal(hist_g, hist_e)


@pytest.mark.parametrize("n", [2500, 70001])
def test_design_loss_fused_against_oracle(g, n):
    """The library's design loss and dL/dI (one workgroup, float64 sums)
    against the oracle's (float64) on seeded intensities and targets, and
    against the torch form of the same loss."""
    import torch
    announce(f"fused design loss, {n} foci")
    rng = np.random.default_rng(n)
    I = rng.uniform(0.0, 2.0, n).astype(np.float32)
    T = rng.uniform(0.5, 1.0, n).astype(np.float32)
    n_ap, sum_a2 = 2211840, 2211840.0
    It = torch.tensor(I, device="cuda", requires_grad=True)
    Tt = torch.tensor(T, device="cuda")
    L = g.design_loss_fused(It, Tt, n_ap, sum_a2)
    L.backward()
    L_o, dI_o = oracle.design_loss(I.astype(np.float64), T.astype(np.float64), n_ap, sum_a2)
    dI = It.grad.cpu().numpy().astype(np.float64)
    It2 = torch.tensor(I, device="cuda", requires_grad=True)
    L2 = g.design_loss(It2, Tt, n_ap, sum_a2)
    L2.backward()
    print(f"  L {float(L):.9e} oracle {L_o:.9e} torch {float(L2):.9e}; "
          f"dL/dI rel {rel_l2(dI, dI_o):.2e}")
    assert float(L) == pytest.approx(L_o, rel=1e-6, abs=1e-9)
    assert rel_l2(dI, dI_o) <= 1e-6
    assert rel_l2(It2.grad.cpu().numpy(), dI_o) <= 1e-3   # the float32 torch form


@pytest.mark.parametrize("shape", [(130, 200), (131, 199)])
def test_phase_gradient_adam_equals_the_two_calls(g, shape):
    """gswmtp_phase_gradient_adam_device against gswmtp_phase_gradient_device
    followed by gswmtp_adam_step_device (its 16-byte kernel for 130 x 200, the
    one-value kernel for 131 x 199): phases and moments bit for bit over
    three steps, on a disc whose compacted-away border rows and columns take
    a zero gradient."""
    import torch
    ny, nx = shape
    h = synth_ofa.random_case(11, ny, nx, 45, radius=60.0)
    announce(f"phase gradient + Adam in one call {ny}x{nx}")
    rng = np.random.default_rng(5)
    bits = lambda t: t.view(torch.int32).cpu().numpy()  # noqa: E731
    with g.Plan(h) as p:
        assert len(p.index()["rows"]) < ny and len(p.index()["cols"]) < nx
        phi_a = torch.tensor(np.asarray(h.phi0, np.float32).reshape(-1), device="cuda")
        phi_b = phi_a.clone()
        m_a, v_a = torch.zeros_like(phi_a), torch.zeros_like(phi_a)
        m_b, v_b = m_a.clone(), v_a.clone()
        step = torch.zeros(1, dtype=torch.float32, device="cuda")
        for _ in range(3):
            step += 1.0
            gv = torch.tensor(rng.standard_normal(h.n_foci).astype(np.float32), device="cuda")
            p.set_phase(phi_a.view(ny, nx))
            grad = p.phase_gradient_device(gv)
            g.adam_step_device(phi_a, grad.reshape(-1), m_a, v_a, step, 0.05)
            p.set_phase(phi_b.view(ny, nx))
            p.phase_gradient_adam_device(gv, phi_b, m_b, v_b, step, 0.05)
            for a, b in ((phi_a, phi_b), (m_a, m_b), (v_a, v_b)):
                assert np.array_equal(bits(a), bits(b))
        assert float((phi_a - torch.tensor(np.asarray(h.phi0, np.float32).reshape(-1),
                                           device="cuda")).abs().max()) > 0


def test_design_loss_record_keeps_the_books(g):
    """gswmtp_design_loss_record_device: the same loss and dL/dI as the plain
    entry point, the loss written to hist[step] while step < capacity, and
    the step counter advanced by one on every call (capacity 2, three calls:
    the third loss is not recorded)."""
    import torch
    from paper_2206_12661_amd.autograd import _loss_and_gradient
    announce("design loss with the loop's books")
    rng = np.random.default_rng(7)
    n_ap, sum_a2 = 4096, 4096.0
    hist = torch.full((2,), -7.0, dtype=torch.float32, device="cuda")
    step = torch.zeros(1, dtype=torch.float32, device="cuda")
    Tt = torch.tensor(rng.uniform(0.5, 1.0, 300).astype(np.float32), device="cuda")
    losses = []
    for k in range(3):
        It = torch.tensor(rng.uniform(0.0, 2.0, 300).astype(np.float32), device="cuda")
        L0, d0 = _loss_and_gradient(It, Tt, n_ap, sum_a2, 0.1)
        L1, d1 = _loss_and_gradient(It, Tt, n_ap, sum_a2, 0.1, hist, step)
        assert torch.equal(L0, L1) and torch.equal(d0, d1)
        assert float(step) == k + 1
        losses.append(float(L1))
    h = hist.cpu().numpy()
    assert h[0] == np.float32(losses[0]) and h[1] == np.float32(losses[1])
    assert losses[2] not in h.tolist()


@pytest.mark.parametrize("n", [300001, 300000])
def test_adam_kernel_matches_torch_adam(g, n):
    """The library's Adam step against torch.optim.Adam (float32, the same
    published update) on random data over five steps, both from zero moments:
    phases within a few float32 roundings of each other.  n = 300001 runs the
    one-value-per-thread kernel (a ragged tail past the 256-wide blocks),
    n = 300000 the 16-byte one."""
    import torch
    announce(f"Adam kernel vs torch.optim.Adam, n = {n}")
    gen = torch.Generator(device="cpu").manual_seed(5)
    phi0 = torch.randn(n, generator=gen)
    grads = [torch.randn(n, generator=gen) * 10.0 ** -k for k in range(5)]
    p_ref = torch.nn.Parameter(phi0.clone().cuda())
    opt = torch.optim.Adam([p_ref], lr=0.05, betas=(0.9, 0.999), eps=1e-8, foreach=False)
    phi = phi0.clone().cuda()
    m = torch.zeros_like(phi)
    v = torch.zeros_like(phi)
    step = torch.zeros(1, device="cuda")
    for gr in grads:
        gr = gr.cuda()
        p_ref.grad = gr.clone()
        opt.step()
        step += 1.0
        g.adam_step_device(phi, gr, m, v, step, 0.05)
    torch.cuda.synchronize()
    d = (phi - p_ref.detach()).abs().max().item()
    print(f"  max |phi - torch| {d:.3e}")
    assert d <= 1e-5
    assert torch.equal(step.cpu(), torch.tensor([5.0]))


def test_c5_adam_200_steps(g):
    """The full 1152 x 1920 / 50 x 50 design: 200 Adam steps (lr 0.05).  The
    loss before the first step and the foci intensities of the final phase
    are checked against the oracle's forward at the same phases."""
    import torch
    h = synth_ofa.config5()
    announce("C-5 Adam 200 steps")
    with g.Plan(h) as p:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi, hist = g.adam_design(p, 200, phi0=h.phi0, target=h.target)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        phi_np = phi.cpu().numpy()
        p.set_phase(phi_np)
        I_gpu = np.abs(p.foci_field().astype(np.complex128)) ** 2
        st = p.stats()
    hist = hist.cpu().numpy().astype(np.float64)
    print(f"  {200 / dt:.1f} steps/s; loss {hist[0]:.5e} -> {hist[-1]:.5e}; "
          f"uniformity {st['uniformity']:.4f} efficiency {st['eta']:.4f}")
    assert np.all(np.isfinite(hist)) and np.all(np.isfinite(phi_np))
    amp = np.asarray(h.amplitude, np.float64)
    n_ap, sum_a2 = int(np.count_nonzero(amp > 0)), float(np.sum(amp * amp))
    th0 = oracle.forward(oracle.pupil_field(h), h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    L0, _ = oracle.design_loss(np.abs(th0) ** 2, h.target, n_ap, sum_a2)
    assert hist[0] == pytest.approx(L0, rel=1e-5)
    th1 = oracle.forward(oracle.pupil_field(h, phi_np.astype(np.float64)), h.u, h.v, h.s_x,
                         h.s_y, h.fx, h.fy)
    assert rel_l2(I_gpu, np.abs(th1) ** 2) <= 1e-5
    assert hist[-1] < hist[0]
