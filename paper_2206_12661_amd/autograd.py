"""Differentiable focus intensities: phase (real tensor) -> I_n = |Theta_n|^2.

Forward runs E = A exp(i phi) and the forward matrix triple product (Eq. 2)
at the foci in the library's kernels.  Backward receives g = dL/dI and runs
the adjoint product with a gradient epilogue in the library:

    dL/dphi = 2 Im( conj(E) * P^H(g * Theta) ).

Intensities are real, so no complex-gradient convention crosses the boundary.
"""
from __future__ import annotations

import itertools

import torch

_tokens = itertools.count(1)


class MTPIntensity(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi: torch.Tensor, plan) -> torch.Tensor:
        if not (phi.is_cuda and phi.dtype == torch.float32):
            raise TypeError("phi must be a float32 CUDA tensor")
        if phi.numel() != plan.ny * plan.nx:
            raise ValueError("phi has the wrong number of elements")
        plan.set_phase(phi)
        token = next(_tokens)
        plan._phase_token = token
        _, inten = plan.foci_field_device(intensity=True, field=False)
        ctx.plan = plan
        ctx.token = token
        ctx.save_for_backward(phi)
        return inten

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (phi,) = ctx.saved_tensors
        plan = ctx.plan
        if getattr(plan, "_phase_token", None) != ctx.token:
            plan.set_phase(phi)
            plan._phase_token = ctx.token
        grad = plan.phase_gradient_device(g.contiguous())
        return grad.view_as(phi), None


def foci_intensity(phi: torch.Tensor, plan) -> torch.Tensor:
    """I_n(phi) for the plan's pupil and foci, differentiable in phi."""
    return MTPIntensity.apply(phi, plan)


def design_loss(I: torch.Tensor, target: torch.Tensor, n_ap: int, sum_a2: float,
                eta_weight: float = 0.1) -> torch.Tensor:
    """L = sum_n (i_n - t_n)^2 - eta_weight * eta, with normalised
    intensities i = I / sum I against normalised targets t = T / sum T and
    the diffraction efficiency eta = sum I / (n_ap * sum A^2) (Sec. 2; the
    incident energy of the discrete sums is n_ap * sum A^2)."""
    S = I.sum()
    r = I / S - target / target.sum()
    return (r * r).sum() - eta_weight * S / (float(n_ap) * float(sum_a2))


def _loss_and_gradient(I: torch.Tensor, target: torch.Tensor, n_ap: int, sum_a2: float,
                       eta_weight: float, hist: torch.Tensor = None, step: torch.Tensor = None):
    """(loss [1], dL/dI [N]) of ``design_loss`` from the library kernel, on the
    current stream; with ``step`` (float32 CUDA [1]) the kernel also records
    the loss in ``hist[step]`` and advances ``step`` by one
    (gswmtp_design_loss_record_device)."""
    from . import GswmtpError, _stream_handle, load_library
    if not (I.is_cuda and I.dtype == torch.float32 and target.is_cuda and
            target.dtype == torch.float32 and I.numel() == target.numel()):
        raise TypeError("I and target must be float32 CUDA tensors of one size")
    I = I.detach().contiguous()
    target = target.contiguous()
    loss = torch.empty(1, dtype=torch.float32, device=I.device)
    dI = torch.empty_like(I)
    args = (I.data_ptr(), target.data_ptr(), I.numel(), float(n_ap), float(sum_a2),
            float(eta_weight), loss.data_ptr(), dI.data_ptr())
    if step is None:
        name = "gswmtp_design_loss_device"
        rc = load_library().gswmtp_design_loss_device(*args, _stream_handle())
    else:
        if not (step.is_cuda and step.dtype == torch.float32 and step.numel() == 1 and
                hist.is_cuda and hist.dtype == torch.float32 and hist.is_contiguous()):
            raise TypeError("hist and step must be float32 CUDA tensors (step of one value)")
        name = "gswmtp_design_loss_record_device"
        rc = load_library().gswmtp_design_loss_record_device(
            *args, hist.data_ptr(), hist.numel(), step.data_ptr(), _stream_handle())
    if rc != 0:
        raise GswmtpError(rc, name)
    return loss, dI


class DesignLoss(torch.autograd.Function):
    """``design_loss`` as one library kernel (gswmtp_design_loss_device), which
    forms the loss and dL/dI together (float64 sums in a fixed order); the
    backward scales the saved dL/dI by the incoming gradient."""

    @staticmethod
    def forward(ctx, I: torch.Tensor, target: torch.Tensor, n_ap: int, sum_a2: float,
                eta_weight: float):
        loss, dI = _loss_and_gradient(I, target, n_ap, sum_a2, eta_weight)
        ctx.save_for_backward(dI)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (dI,) = ctx.saved_tensors
        return g * dI, None, None, None, None


def design_loss_fused(I: torch.Tensor, target: torch.Tensor, n_ap: int, sum_a2: float,
                      eta_weight: float = 0.1) -> torch.Tensor:
    """``design_loss`` in the library: the same value and gradient, with sums in
    float64, in one kernel instead of a dozen small tensor operations."""
    return DesignLoss.apply(I, target, n_ap, sum_a2, eta_weight)


def adam_design(plan, steps: int, lr: float = 0.05, betas=(0.9, 0.999), eps: float = 1e-8,
                eta_weight: float = 0.1, phi0=None, target=None, graph: bool = True):
    """Phase design by gradient descent: Adam on ``design_loss`` of the plan's
    foci intensities, the update in the library's Adam kernel (the update
    of ``adam_step_device``).  Returns (phi [ny, nx] float32 CUDA tensor, loss
    before each step [steps] tensor).

    A step is the chain rule that ``foci_intensity`` and ``design_loss_fused``
    run under autograd, called directly: the forward to I, the loss kernel
    with dL/dI, the phase gradient of that dL/dI (``MTPIntensity``'s
    backward) applied by Adam in the same library call
    (``Plan.phase_gradient_adam_device``: the update reads the gradient where
    the adjoint product leaves it), so no seed gradient or scaling by it
    (autograd's seed is 1.0: the same gradient bit for bit) and no gradient
    array.

    graph=True captures one whole step - the phase encode, the forward product
    with the focus gather, the loss and its gradient, the adjoint product with
    the gradient epilogue, and the Adam update with its step count on the
    device - in one graph and replays it ``steps`` times, so no step waits on
    the host; every kernel of the step is the library's.  The library's
    calls only record and wait on events against the
    caller's stream, so its internal stream joins the capture.  The captured
    step is the eager one: a warm-up step (which sets up the plan's lazy
    buffers) is undone before capture, and both forms give the same
    trajectory.
    graph=False runs the same step eagerly."""
    idx = plan.index()
    n_ap, sum_a2 = idx["n_aperture"], idx["sum_a2"]
    if target is None:
        raise ValueError("target intensities are required")
    if steps < 0:
        raise ValueError("steps must be >= 0")
    t = torch.as_tensor(target, dtype=torch.float32, device="cuda")
    if phi0 is None:
        phi0 = torch.zeros(plan.ny, plan.nx)
    start = torch.as_tensor(phi0, dtype=torch.float32, device="cuda").clone()
    phi = start.clone()
    m = torch.zeros_like(start)
    v = torch.zeros_like(start)
    count = torch.zeros(1, dtype=torch.float32, device="cuda")   # steps recorded so far
    hist = torch.zeros(max(steps, 1), dtype=torch.float32, device="cuda")

    def step():
        plan.set_phase(phi)
        plan._phase_token = next(_tokens)   # a pending MTPIntensity backward re-sets its phase
        _, inten = plan.foci_field_device(intensity=True, field=False)
        # the loss kernel records L in hist[count] and advances count, which is
        # then this step's number t for Adam
        _, dI = _loss_and_gradient(inten, t, n_ap, sum_a2, eta_weight, hist, count)
        plan.phase_gradient_adam_device(dI, phi, m, v, count, lr, betas, eps)

    if not graph or steps == 0:
        for _ in range(steps):
            step()
        return phi.detach(), hist[:steps]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    # undo the warm-up: start phase, zero moments and step counts
    phi.copy_(start)
    m.zero_()
    v.zero_()
    count.zero_()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for _ in range(steps):
        g.replay()
    out = phi.detach().clone(), hist[:steps].clone()
    del g
    return out
