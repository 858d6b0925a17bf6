"""The C-ABI library loads and exports every symbol its header declares, and
host-side validation rejects bad descriptors before any GPU work (no compute
calls here: these run without a GPU)."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gswmtp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gswmtp_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2206_12661_amd as g
    return g.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["gswmtp_plan_create", "gswmtp_iterate", "gswmtp_get_phase",
                 "gswmtp_get_foci_field", "gswmtp_plan_destroy"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    so = os.path.join(ROOT, "paper_2206_12661_amd", "libgswmtp.so")
    out = subprocess.run(["nm", "-D", "--defined-only", so], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (gswmtp_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        getattr(lib, n)


def test_exports_no_cpp_or_oracle_symbols():
    so = os.path.join(ROOT, "paper_2206_12661_amd", "libgswmtp.so")
    out = subprocess.run(["nm", "-D", "--defined-only", so], capture_output=True, text=True,
                         check=True).stdout
    assert "oracle_" not in out


def test_status_strings_and_version(lib):
    import paper_2206_12661_amd as g
    assert lib.gswmtp_version() == 100
    for code in range(-8, 1):
        s = g.status_string(code)
        assert s.startswith("GSWMTP_")
    assert "unknown" in g.status_string(-99)


def _desc(g, **over):
    d = g.gswmtp_desc()
    g.load_library().gswmtp_desc_init(ctypes.byref(d))
    keep = []

    def put(name, arr):
        a = np.ascontiguousarray(arr)
        keep.append(a)
        setattr(d, name, a.ctypes.data)

    d.ny, d.nx, d.n_foci = 8, 8, 3
    d.s_x = d.s_y = 1 / 8
    put("fx", np.array([0.0, 1.0, 2.0]))
    put("fy", np.array([0.5, 0.5, 0.5]))
    put("target", np.array([1.0, 1.0, 1.0]))
    for k, v in over.items():
        if isinstance(v, np.ndarray):
            put(k, v)
        else:
            setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("case", [
    "ny0", "nf0", "nfhuge", "sx0", "sxnan", "fxnan", "targetneg", "targetzero", "ampneg",
    "ampnan", "phinan", "unan", "precision", "axis", "weighting", "fznan", "fzinf", "side_over",
    "nf_over"])
def test_validation_rejects_bad_descriptors(case):
    import paper_2206_12661_amd as g
    lib = g.load_library()
    over = {
        "ny0": {"ny": 0}, "nf0": {"n_foci": 0}, "nfhuge": {"n_foci": 1 << 20},
        "sx0": {"s_x": 0.0}, "sxnan": {"s_x": math.nan},
        "fxnan": {"fx": np.array([0.0, math.nan, 2.0])},
        "targetneg": {"target": np.array([1.0, -1.0, 1.0])},
        "targetzero": {"target": np.zeros(3)},
        "ampneg": {"amplitude": -np.ones(64, np.float32)},
        "ampnan": {"amplitude": np.full(64, np.nan, np.float32)},
        "phinan": {"phi0": np.full(64, np.inf, np.float32)},
        "unan": {"u": np.full(8, np.nan)},
        "precision": {"precision": 9}, "axis": {"axis": 2}, "weighting": {"weighting": 5},
        "fznan": {"fz": np.array([0.0, math.nan, 0.0])},
        "fzinf": {"fz": np.array([math.inf, 0.0, 0.0])},
        "side_over": {"nx": 16385}, "nf_over": {"n_foci": 262145},
    }[case]
    d, keep = _desc(g, **over)
    h = ctypes.c_void_p()
    rc = lib.gswmtp_plan_create(ctypes.byref(h), ctypes.byref(d), None)
    assert rc == -1
    assert not h.value
    assert lib.gswmtp_last_error(None).decode() != ""


def test_null_arguments(lib):
    assert lib.gswmtp_plan_create(None, None, None) == -1
    h = ctypes.c_void_p()
    assert lib.gswmtp_plan_create(ctypes.byref(h), None, None) == -1
    assert lib.gswmtp_plan_destroy(None) == 0
    assert lib.gswmtp_desc_init(None) == -1
    assert lib.gswmtp_iterate(None, 1, 0.0) == -1
    assert lib.gswmtp_set_phase_fixing(None, 1) == -1
    assert lib.gswmtp_iterate_measured(None, None) == -1
    assert lib.gswmtp_batch_destroy(None) == 0
    b = ctypes.c_void_p()
    assert lib.gswmtp_batch_create(None, None, 1, None) == -1
    assert lib.gswmtp_batch_create(ctypes.byref(b), None, 1, None) == -1
    arr = (ctypes.c_void_p * 2)(None, None)
    assert lib.gswmtp_batch_create(ctypes.byref(b), arr, 0, None) == -1
    assert lib.gswmtp_batch_create(ctypes.byref(b), arr, 2, None) == -1
    assert not b.value
    assert lib.gswmtp_batch_last_error(None).decode() != ""
    assert lib.gswmtp_batch_iterate(None, 1, 0.0) == -1
    assert lib.gswmtp_batch_sync(None) == -1
    assert lib.gswmtp_batch_set_stream(None, None) == -1
    assert lib.gswmtp_batch_tiles(None, None, None) == -1


def test_product_path_does_not_import_oracle():
    src = os.path.join(ROOT, "paper_2206_12661_amd")
    for dirpath, _, files in os.walk(src):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "gsw_oracle" not in text and "liboracle" not in text, f


def test_workspace_size_host_only():
    """Sizing needs no GPU: validation codes as at creation, and the size
    grows with what the plan holds."""
    import paper_2206_12661_amd as g
    import synth_ofa
    lib = g.load_library()
    n = ctypes.c_size_t(123)
    assert lib.gswmtp_plan_workspace_size(None, ctypes.byref(n)) == -1
    d, keep = _desc(g)
    assert lib.gswmtp_plan_workspace_size(ctypes.byref(d), None) == -1
    assert lib.gswmtp_plan_workspace_size(ctypes.byref(d), ctypes.byref(n)) == 0
    assert n.value > 0
    d, keep = _desc(g, s_x=0.0)
    assert lib.gswmtp_plan_workspace_size(ctypes.byref(d), ctypes.byref(n)) == -1
    d, keep = _desc(g, amplitude=np.zeros(64, np.float32))
    assert lib.gswmtp_plan_workspace_size(ctypes.byref(d), ctypes.byref(n)) == -3
    small = g.Plan.workspace_size(synth_ofa.config1())
    big = g.Plan.workspace_size(synth_ofa.config3())
    assert 0 < small < big
    # three-term split planes hold more than two-term ones
    h = synth_ofa.config2()
    assert g.Plan.workspace_size(h, precision="bf16x6") > g.Plan.workspace_size(
        h, precision="bf16x3")


def test_create_with_workspace_rejects_bad_buffers():
    import paper_2206_12661_amd as g
    lib = g.load_library()
    d, keep = _desc(g)
    h = ctypes.c_void_p()
    assert lib.gswmtp_plan_create_with_workspace(None, ctypes.byref(d), None, 0, None) == -1
    assert lib.gswmtp_plan_create_with_workspace(ctypes.byref(h), ctypes.byref(d), None, 4096,
                                                 None) == -1
    assert lib.gswmtp_plan_create_with_workspace(ctypes.byref(h), ctypes.byref(d), 256, 0,
                                                 None) == -1
    assert lib.gswmtp_plan_create_with_workspace(ctypes.byref(h), ctypes.byref(d), 4096 + 8,
                                                 4096, None) == -1
    assert not h.value
    assert "aligned" in lib.gswmtp_last_error(None).decode()


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asking for more exits with a message
    before anything touches a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("setting", ["alloc", "alloc:1", "alloc:2", "alloc:0", "allocate", ""])
def test_fault_inject_alloc(monkeypatch, setting):
    """GSWMTP_FAULT_INJECT=alloc fails plan creation with GSWMTP_E_NOMEM on the
    host, after validation and before any device work (so also here, without a
    GPU); alloc:K fails only the K-th device allocation (reached on a GPU only:
    here creation stops at the device check, GSWMTP_E_NODEV); malformed
    settings are off.  A bad descriptor still reports GSWMTP_E_INVAL first."""
    import paper_2206_12661_amd as g
    from gpu_util import cuda_ok
    lib = g.load_library()
    monkeypatch.setenv("GSWMTP_FAULT_INJECT", setting)
    d, keep = _desc(g)
    h = ctypes.c_void_p()
    rc = lib.gswmtp_plan_create(ctypes.byref(h), ctypes.byref(d), None)
    msg = lib.gswmtp_last_error(None).decode()
    created = bool(h.value)
    if created:
        lib.gswmtp_plan_destroy(h)
    if setting == "alloc":
        assert rc == -4 and "injected" in msg and not created
        bad, keep2 = _desc(g, s_x=0.0)
        h2 = ctypes.c_void_p()
        assert lib.gswmtp_plan_create(ctypes.byref(h2), ctypes.byref(bad), None) == -1
    elif not cuda_ok():
        assert rc == -7 and "injected" not in msg and not created
    elif setting in ("alloc:1", "alloc:2"):
        assert rc == -4 and "injected" in msg and not created
    else:
        assert rc == 0 and created


def test_adam_step_validation(lib):
    """The Adam entry point checks its arguments on the host (no GPU needed):
    n = 0 is a no-op, null pointers and out-of-range betas are rejected."""
    P = ctypes.c_void_p
    buf = (ctypes.c_float * 4)()
    p = ctypes.cast(buf, P)
    call = lambda *a: lib.gswmtp_adam_step_device(*a)  # noqa: E731
    assert call(None, None, None, None, None, 0, 0.05, 0.9, 0.999, 1e-8, None) == 0
    assert call(None, p, p, p, p, 4, 0.05, 0.9, 0.999, 1e-8, None) == -1
    assert call(p, p, p, p, None, 4, 0.05, 0.9, 0.999, 1e-8, None) == -1
    assert call(p, p, p, p, p, 4, 0.05, 1.0, 0.999, 1e-8, None) == -1
    assert call(p, p, p, p, p, 4, 0.05, 0.9, -0.1, 1e-8, None) == -1
    assert call(p, p, p, p, p, 4, math.nan, 0.9, 0.999, 1e-8, None) == -1
    assert call(p, p, p, p, p, 4, 0.05, 0.9, 0.999, -1.0, None) == -1


def test_phase_gradient_adam_validation(lib):
    """The fused gradient + Adam entry point rejects a null plan or pointer
    and bad hyper-parameters on the host (no GPU needed)."""
    P = ctypes.c_void_p
    buf = (ctypes.c_float * 4)()
    p = ctypes.cast(buf, P)
    call = lambda *a: lib.gswmtp_phase_gradient_adam_device(*a)  # noqa: E731
    assert call(None, p, p, p, p, p, 0.05, 0.9, 0.999, 1e-8) == -1
    fake = p   # never dereferenced: every case below fails before the plan is used
    assert call(fake, None, p, p, p, p, 0.05, 0.9, 0.999, 1e-8) == -1
    assert call(fake, p, p, p, p, None, 0.05, 0.9, 0.999, 1e-8) == -1
    assert call(fake, p, p, p, p, p, math.nan, 0.9, 0.999, 1e-8) == -1
    assert call(fake, p, p, p, p, p, 0.05, 1.0, 0.999, 1e-8) == -1
    assert call(fake, p, p, p, p, p, 0.05, 0.9, 0.999, -1.0) == -1


def test_design_loss_validation(lib):
    """The fused design-loss entry point rejects bad sizes and pointers on the
    host (no GPU needed)."""
    P = ctypes.c_void_p
    buf = (ctypes.c_float * 4)()
    p = ctypes.cast(buf, P)
    call = lambda *a: lib.gswmtp_design_loss_device(*a)  # noqa: E731
    assert call(p, p, 0, 10.0, 10.0, 0.1, p, p, None) == -1
    assert call(None, p, 4, 10.0, 10.0, 0.1, p, p, None) == -1
    assert call(p, p, 4, 10.0, 10.0, 0.1, p, None, None) == -1
    assert call(p, p, 4, 0.0, 10.0, 0.1, p, p, None) == -1
    assert call(p, p, 4, 10.0, -1.0, 0.1, p, p, None) == -1
    assert call(p, p, 4, 10.0, 10.0, math.inf, p, p, None) == -1
    rec = lambda *a: lib.gswmtp_design_loss_record_device(*a)  # noqa: E731
    assert rec(p, p, 4, 10.0, 10.0, 0.1, p, p, p, 4, None, None) == -1   # no step counter
    assert rec(p, p, 4, 10.0, 10.0, 0.1, p, p, p, -1, p, None) == -1    # negative capacity
    assert rec(p, p, 4, 10.0, 10.0, 0.1, p, p, None, 4, p, None) == -1  # no history buffer
    assert rec(p, p, 0, 10.0, 10.0, 0.1, p, p, p, 4, p, None) == -1     # the loss's own checks
