"""Documented error paths of the C ABI that need a plan on the GPU (include/pat.h).

Non-finite inputs must come back as PAT_ERR_NONFINITE from the calls that reduce
to a reported scalar (the FISTA energy, the power-iteration norm); invalid
arguments as PAT_ERR_INVALID before any work is enqueued. Every kernel still
runs to its normal end: NaN and Inf are ordinary floating-point values to it.
"""

import ctypes as C

import numpy as np
import pytest

from gpu_cases import empty, gpu_plan, oracle_sampling, to_dev

pytestmark = pytest.mark.gpu

N, NT = 16, 24


def _plan():
    return gpu_plan(N, NT, oracle_sampling("points", N), pml=2)


def _status(fn, *args):
    from paper_1605_00133_amd import pat as P
    with pytest.raises(P.PatError) as e:
        fn(*args)
    return e.value.status, str(e.value)


@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_reconstruct_nonfinite_data(bad):
    from paper_1605_00133_amd import pat as P
    plan = _plan()
    f = np.zeros(plan.data_shape)
    f[3, 5] = bad
    p = empty(plan.vol_shape)
    st, msg = _status(P.pat_reconstruct, plan, to_dev(f), p, 1e-3, 1.0, 1, 2, 5, "dirichlet")
    print(msg)
    assert st == 5 and "energy" in msg


def test_power_iteration_nonfinite_or_zero_start():
    from paper_1605_00133_amd import pat as P
    plan = _plan()
    x0 = np.zeros((N, N, N))
    st, _ = _status(P.pat_power_iteration, plan, to_dev(x0), 2)
    assert st == 5
    x0[4, 4, 4] = np.nan
    st, _ = _status(P.pat_power_iteration, plan, to_dev(x0), 2)
    assert st == 5


def test_invalid_arguments_are_rejected_before_launch():
    from paper_1605_00133_amd import pat as P
    import torch
    plan = _plan()
    lib = P.lib()
    h = plan.handle
    buf = torch.zeros(max(N ** 3, NT * plan.mc) + 16, device="cuda:0")
    a = C.c_void_p(buf.data_ptr())
    b = C.c_void_p(buf.data_ptr() + 64)                       # overlaps a
    assert lib.pat_forward(h, a, b) == 1 and b"overlap" in lib.pat_last_error()
    assert lib.pat_adjoint(h, a, b) == 1 and b"overlap" in lib.pat_last_error()
    assert lib.pat_forward(h, None, a) == 1
    assert lib.pat_tv_prox(h, a, a, 0.1, 3, 2, a) == 1                  # bc must be 0 or 1
    assert lib.pat_tv_prox(h, a, a, -0.1, 3, 1, a) == 1                 # alpha >= 0
    assert lib.pat_tv_prox(h, a, a, 0.1, -1, 1, a) == 1                 # n_iter >= 0
    assert lib.pat_plan_set_scheme(h, 7) == 1
    assert lib.pat_plan_set_fft_precision(h, 16) == 1
    assert lib.pat_power_iteration(h, a, 0, C.byref(C.c_double())) == 1
    assert lib.pat_profile_end(h, None, None) == 1                      # not begun
    p = empty(plan.vol_shape)
    f = empty(plan.data_shape)
    for kwargs, what in [({"L": 0.0}, "L must be > 0"), ({"lam": -1.0}, "lambda"), ({"n_inner": -1}, "iteration"),
                         ({"n_outer": 0}, "iteration")]:
        args = {"lam": 1e-3, "L": 1.0, "n_outer": 1, "n_inner": 1}
        args.update(kwargs)
        st, msg = _status(P.pat_reconstruct, plan, f, p, args["lam"], args["L"], args["n_outer"], args["n_inner"], 2,
                          "dirichlet")
        assert st == 1 and what in msg, msg
    torch.cuda.synchronize()


def test_plan_workspace_too_small_or_misaligned():
    from paper_1605_00133_amd import pat as P
    import torch
    g = P.make_grid(N, N, N, 100e-6, 1500.0, 20e-9, NT, 2)
    smp, keep = P.make_sampling("full", N * N)
    need = P.pat_plan_workspace_bytes(g, smp)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda:0")
    base = (ws.data_ptr() + 255) // 256 * 256
    h = C.c_void_p()
    lib = P.lib()
    assert lib.pat_plan_create(C.byref(g), C.byref(smp), None, C.c_void_p(base), need - 256, C.byref(h)) == 3
    assert lib.pat_plan_create(C.byref(g), C.byref(smp), None, C.c_void_p(base + 4), need, C.byref(h)) == 1
    assert not h.value
    assert lib.pat_plan_create(C.byref(g), C.byref(smp), None, C.c_void_p(base), need, C.byref(h)) == 0
    assert lib.pat_plan_destroy(h) == 0


def test_copy_probe_copies_and_rejects_bad_arguments():
    """The bench's copy kernel: exact copies of sizes that are and are not a multiple of a block's
    4 x 256 16-byte words (the guarded tail), nothing written past nbytes, and the documented
    argument errors."""
    import torch
    from paper_1605_00133_amd import pat as P
    for n in (4, 4 * 1023, 4 * 4096 * 7 + 12, 1 << 22):
        src = torch.arange(n, dtype=torch.float32, device="cuda")
        dst = torch.full((n + 4,), -1.0, device="cuda")
        P.pat_copy_probe(src, dst[:n])
        torch.cuda.synchronize()
        assert torch.equal(dst[:n], src) and bool((dst[n:] == -1.0).all())
    lib = P.lib()
    a = torch.zeros(64, device="cuda")
    b = torch.zeros(64, device="cuda")
    for args in ((a.data_ptr(), b.data_ptr(), 20), (a.data_ptr() + 4, b.data_ptr(), 16),
                 (a.data_ptr(), a.data_ptr() + 16, 64), (0, b.data_ptr(), 16), (a.data_ptr(), b.data_ptr(), -16)):
        st = lib.pat_copy_probe(C.c_void_p(args[0]), C.c_void_p(args[1]), args[2], None)
        assert st == 1, args                                             # PAT_ERR_INVALID
    assert lib.pat_copy_probe(None, None, 0, None) == 0                  # nothing to copy: PAT_OK
