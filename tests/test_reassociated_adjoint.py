"""The identity behind the split modes' re-associated adjoint, checked on the
host against the FP64 oracle: with S the focal field scattered onto the
unique rows (one focus per row),

    Omega_r^H S = (Omega_r^H diag Theta') conj(Omega_c rows of the foci),

and the adjoint of Eq. 2 (the transposed kernels of the two products,
conjugated) is that product times the conjugated column kernel.  The
identity needs no row to be free of other foci (then K = N rather than the
row count), so a grid case checks it too."""
import numpy as np
import pytest

import oracle
import synth_ofa


def _kernels(h):
    """Adjoint kernel factors, written out from the kernel definition:
    Ar[j, n] = conj exp(-2 pi i s_y v_j fy_n), Bc[n, i] = conj exp(-2 pi i s_x u_i fx_n)."""
    v = np.asarray(h.v, np.float64)
    u = np.asarray(h.u, np.float64)
    fy = np.asarray(h.fy, np.float64)
    fx = np.asarray(h.fx, np.float64)
    Ar = np.exp(2j * np.pi * h.s_y * np.outer(v, fy))
    Bc = np.exp(2j * np.pi * h.s_x * np.outer(fx, u))
    return Ar, Bc


@pytest.mark.parametrize("case", ["random-70", "random-disc-45", "grid-7x5"])
def test_reassociated_adjoint_equals_oracle_adjoint(case):
    h = {"random-70": synth_ofa.random_case(10, 100, 150, 70),
         "random-disc-45": synth_ofa.random_case(11, 130, 200, 45, radius=60.0),
         "grid-7x5": synth_ofa.random_case(12, 96, 96, 0, grid=(7, 5))}[case]
    rng = np.random.default_rng(3)
    n = h.fx.size
    th = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = oracle.adjoint(th, h.ny, h.nx, h.u, h.v, h.s_x, h.s_y, h.fx, h.fy)
    Ar, Bc = _kernels(h)
    # (Omega_r^H diag Theta') conj(Omega_c rows): K = N, one column per focus
    got = (Ar * th[None, :]) @ Bc
    # the scatter form: S on the unique rows, then Omega_r^H S
    yu, iy = np.unique(np.asarray(h.fy, np.float64), return_inverse=True)
    S = np.zeros((yu.size, h.nx), np.complex128)
    np.add.at(S, iy, th[:, None] * Bc)
    Aru = np.exp(2j * np.pi * h.s_y * np.outer(np.asarray(h.v, np.float64), yu))
    via_s = Aru @ S
    scale = np.linalg.norm(ref)
    assert np.linalg.norm(got - ref) <= 1e-11 * scale
    assert np.linalg.norm(via_s - ref) <= 1e-11 * scale
    if case.startswith("random"):
        assert yu.size == n          # one focus per row: K stays the row count
    else:
        assert yu.size < n           # rows shared: the plan keeps the scatter
