"""hfmm_apply_noalloc (the apply with the library's fixed workspace) against
hfmm_apply, through the C interface.

Two calls in a row, the second with a smaller input (a smaller plan, one
right-hand side); the first needs several passes through the fixed
workspace. Bar: relative L2 difference below 1e-12 (the two entry points run
the same kernels; only the order of the atomic additions of the near field
differs). A plan too large for the fixed workspace is refused with
HFMM_ERR_NO_MEMORY before any launch.
"""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _call(lib, plan, q, u, fn):
    import torch
    st = getattr(lib, fn)(plan._h, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(u.data_ptr()), q.shape[0],
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st


def test_noalloc_matches_apply(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    lib = gpu_lib.load()
    cases = [workloads.two_layer_uniform(n=20000, seed=61, nrhs=40),   # several passes
             workloads.two_layer_uniform(n=3000, seed=62, nrhs=1)]     # then a smaller input
    for w in cases:
        pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
        q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
        plan = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-8, leaf_size=32)
        u_ref = torch.empty_like(q)
        u_na = torch.full_like(q, complex("nan+nanj"))
        print("case n=%d nrhs=%d" % (w.n, q.shape[0]), flush=True)
        assert _call(lib, plan, q, u_ref, "hfmm_apply") == 0
        st = _call(lib, plan, q, u_na, "hfmm_apply_noalloc")
        assert st == 0, lib.hfmm_last_error_message().decode()
        e = rel(u_na.cpu().numpy(), u_ref.cpu().numpy())
        print("  noalloc vs apply: %.2e" % e, flush=True)
        assert e < 1e-12
        plan.close()


def test_noalloc_refuses_a_plan_beyond_its_workspace(gpu_lib):
    import torch
    dev = torch.device("cuda:0")
    lib = gpu_lib.load()
    w = workloads.two_layer_hf(n=1 << 19, seed=63)
    pts = torch.tensor(w.xy, dtype=torch.float64, device=dev)
    q = torch.tensor(w.q, dtype=torch.complex128, device=dev)
    plan = gpu_lib.Plan(w.k, w.interfaces, pts, tol=1e-8, leaf_size=64)
    u = torch.zeros_like(q)
    st = _call(lib, plan, q, u, "hfmm_apply_noalloc")
    msg = lib.hfmm_last_error_message().decode()
    print("large plan:", st, msg)
    assert st == 4 and "workspace" in msg
    assert float(u.abs().max()) == 0.0
    plan.close()
