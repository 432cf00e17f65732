"""The entry point that allocates nothing, dm_solve_pcg_noalloc, through the C ABI.

For callers that cannot allocate device memory: its results are checked
against the allocating entry point it stands in for, dm_solve in the PCG64
mode, at the FP64 bar (1e-12 of the solution's largest entry; the two run
the same arithmetic, so the iteration counts must be equal), on two calls in
a row, the second on a smaller grid (24^3 sphere, then 16^3), so the second
call meets the scratch array as the first left it.  Also: a grid whose work
vectors exceed the scratch array is refused with DM_EINVAL, and the device's
free memory is unchanged across a call (no allocation).
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def c_noalloc(dm):
    L = dm.lib()
    f = L.dm_solve_pcg_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                  ctypes.POINTER(dm.SolveInfo), ctypes.c_void_p]
    f.restype = ctypes.c_int
    return f


def call_noalloc(dm, op, f, x, rtol, maxit):
    info = dm.SolveInfo()
    rc = c_noalloc(dm)(op._op, f.data_ptr(), x.data_ptr(), rtol, maxit, ctypes.byref(info), None)
    return rc, info


def free_device_bytes():
    free, total = torch.cuda.mem_get_info()
    return free


def sphere_case(dm, n, seed):
    op = dm.Operator(dm.sphere((0.5, 0.5, 0.5), 0.45), (n, n, n), 1.0 / n, 5.0, levels=3)
    P = op.layout(0)["P"]
    mask = torch.tensor(op.fractions(0)[:3].reshape(-1) > 0)
    g = torch.Generator().manual_seed(seed)
    f = (torch.randn(3 * P, dtype=torch.float64, generator=g) * mask).cuda()
    return op, f


@pytest.mark.parametrize("maxit", [300, 3])
def test_noalloc_matches_allocating_solve(maxit):
    from paper_1301_3794_amd import dm
    print(f"[case] no-alloc PCG, 24^3 then 16^3, maxit {maxit}", flush=True)
    for n, seed in ((24, 1), (16, 2)):          # second call: smaller input
        op, f = sphere_case(dm, n, seed)
        ref = op.face_tensor()
        want = op.solve(f, ref, mode=dm.SOLVE_PCG64, rtol=1e-11, maxit=maxit)
        x = torch.full_like(ref, 7.0)          # the call must overwrite every entry
        rc, info = call_noalloc(dm, op, f, x, 1e-11, maxit)
        assert rc == want["status"], (rc, dm.lib().dm_last_error_message())
        assert info.iterations == want["iterations"]
        err = float((x - ref).abs().max() / ref.abs().max())
        assert err <= 1e-12, err
        assert abs(info.rel_residual - want["rel_residual"]) <= 1e-12 + 1e-9 * want["rel_residual"]
        op.close()


def test_noalloc_allocates_nothing():
    from paper_1301_3794_amd import dm
    op, f = sphere_case(dm, 16, 3)
    x = op.face_tensor()
    rc, _ = call_noalloc(dm, op, f, x, 1e-10, 200)      # warm: kernels loaded
    assert rc == 0
    torch.cuda.synchronize()
    before = free_device_bytes()
    rc, _ = call_noalloc(dm, op, f, x, 1e-10, 200)
    torch.cuda.synchronize()
    assert rc == 0
    assert free_device_bytes() >= before
    op.close()


def test_noalloc_rejects_large_grid():
    from paper_1301_3794_amd import dm
    # 80^3 box: 3P = 3 * 82^3 = 1,654,104 doubles per vector, over the limit
    op = dm.Operator(dm.box(), (80, 80, 80), 1.0 / 80, 5.0, levels=5)
    f = op.face_tensor()
    rc, _ = call_noalloc(dm, op, f, op.face_tensor(), 1e-10, 10)
    assert rc == dm.DM_EINVAL
    op.close()
