"""dlr_q1_sweep_noalloc (the Q1 sweep for callers that cannot allocate device memory)
against the operator-handle entry point dlr_q1_sweep on the same inputs: two calls in a
row, the second on a smaller problem, in FP64 and FP32.  Both run the same sweep kernel with
the same hand-off order, so the results must be bitwise equal; the smaller problem is also
checked against the oracle's cell-by-cell solve.  Oversized problems are rejected on the host
before any work is queued."""
import ctypes

import numpy as np
import pytest

from oracle import q1_oracle as Q
from synth import problems

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1


def _tensors(inp, precision):
    import torch
    dt = torch.float64 if precision == FP64 else torch.float32
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(inp[k])).to(dev, dt)
         for k in ("sigma_t", "src", "inflow_x", "inflow_y")}
    t["mu"] = torch.from_numpy(np.ascontiguousarray(inp["mu"], np.float64)).to(dev)
    t["eta"] = torch.from_numpy(np.ascontiguousarray(inp["eta"], np.float64)).to(dev)
    return t


def handle_sweep(inp, precision):
    import torch
    from paper_2601_18705_amd import dlrtrt
    t = _tensors(inp, precision)
    psi = torch.full(inp["src"].shape, float("nan"), dtype=t["src"].dtype, device=t["src"].device)
    with dlrtrt.Q1Sweep(inp["nx"], inp["ny"], inp["hx"], inp["hy"], inp["mu"], inp["eta"], precision) as op:
        op.sweep(t["sigma_t"], t["src"], t["inflow_x"], t["inflow_y"], psi)
        op.sync()
    return psi.double().cpu().numpy()


def noalloc_sweep(inp, precision):
    import torch
    from paper_2601_18705_amd import dlrtrt
    t = _tensors(inp, precision)
    psi = torch.full(inp["src"].shape, float("nan"), dtype=t["src"].dtype, device=t["src"].device)
    status = torch.zeros(1, dtype=torch.int32, device=t["src"].device)
    dlrtrt.q1_sweep_noalloc(inp["nx"], inp["ny"], inp["hx"], inp["hy"], t["mu"], t["eta"], precision,
                            t["sigma_t"], t["src"], t["inflow_x"], t["inflow_y"], psi, status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0, "a hand-off wait exceeded its spin limit"
    return psi.double().cpu().numpy()


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_noalloc_equals_handle_two_calls(precision):
    big = problems.q1_sweep_inputs(300, 37, 8, seed=21, sigma_shift=50.0)
    small = problems.q1_sweep_inputs(65, 9, 4, seed=22, sigma_shift=50.0)
    for name, inp in (("300x37, 8 directions", big), ("65x9, 4 directions", small)):
        print(f"[no-alloc] {name} precision {precision}", flush=True)
        want = handle_sweep(inp, precision)
        got = noalloc_sweep(inp, precision)
        assert np.all(np.isfinite(got)), name
        assert np.array_equal(got, want), f"{name}: max diff {np.max(np.abs(got - want)):.3e}"
    ref = Q.sweep(small["nx"], small["ny"], small["hx"], small["hy"], small["mu"], small["eta"], small["sigma_t"],
                  small["src"], small["inflow_x"], small["inflow_y"])
    bound = 1e-12 if precision == FP64 else (small["nx"] + small["ny"] + 16) * 2.0 ** -21
    assert np.max(np.abs(got - ref)) <= bound * np.max(np.abs(ref))


def test_noalloc_rejects_oversized_problem():
    import torch
    from paper_2601_18705_amd import dlrtrt
    lib = dlrtrt.library()
    nd = 256
    mu = torch.full((nd,), 0.5, dtype=torch.float64, device="cuda:0")
    buf = torch.zeros(64, dtype=torch.float64, device="cuda:0")
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    p = ctypes.c_void_p(buf.data_ptr())
    st = lib.dlr_q1_sweep_noalloc(1024, 1024, 1e-3, 1e-3, nd, ctypes.c_void_p(mu.data_ptr()),
                                  ctypes.c_void_p(mu.data_ptr()), FP64, None, p, p, p, p, p,
                                  ctypes.c_void_p(status.data_ptr()))
    assert st == -1
    assert b"scratch" in lib.dlr_last_error()
