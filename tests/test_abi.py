"""C-ABI checks that need no GPU: exports, host index generators, validation."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.sampling import rsp_mask, shd_pattern
from paper_1605_00133_amd import pat as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pat.h")
NN_HEADER = os.path.join(ROOT, "include", "pat_nn.h")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pat_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = P.lib()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/pat.h but not exported"
    assert set(names) == set(P.SIGNATURES), "binding and header disagree"


def test_library_exports_every_nn_function():
    from paper_1605_00133_amd import nn
    lib = nn.lib()
    names = declared_functions(NN_HEADER)
    assert len(names) == 16
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/pat_nn.h but not exported"
    assert set(names) == set(nn.SIGNATURES), "nn binding and header disagree"


def test_nn_validation_without_gpu():
    from paper_1605_00133_amd import nn
    lib = nn.lib()
    # K = 27 * 3 + 1 bias column; the LDS weight gradient sums one partial per chunk of row groups:
    # here every row group (2 batches x 5 planes x 2 groups of 4 rows) is a chunk
    assert lib.pat_conv3d_backward_weight_workspace_bytes(2, 3, 20, 5, 6, 37) == 20 * 20 * 82 * 4
    # a narrow layer (one group of <= 32 output tiles: 1 x 28) takes 1024 chunks, a wider one 256
    assert lib.pat_conv3d_backward_weight_workspace_bytes(4, 16, 16, 128, 128, 128) == 1024 * 16 * 433 * 4
    assert lib.pat_conv3d_backward_weight_workspace_bytes(4, 24, 24, 32, 32, 32) == 256 * 24 * 649 * 4
    assert lib.pat_conv3d_backward_weight_workspace_bytes(1, 0, 16, 8, 8, 8) == 0
    # packed weights: ceil(co / 16) tiles x ceil(27 cpad / 32) chunks x 512 bfloat16, cpad = ci rounded up to 8
    assert lib.pat_conv3d_workspace_bytes(3, 20) == max(2 * 7 * 1024, 1 * 21 * 1024)
    assert lib.pat_conv3d_workspace_bytes(24, 24) == 2 * 21 * 1024
    assert lib.pat_conv3d_workspace_bytes(70, 70) == 256          # both directions use the unpacked kernel
    assert lib.pat_conv3d_workspace_bytes(0, 4) == 0
    assert lib.pat_conv3d_forward(None, None, None, None, 1, 0, 4, 8, 8, 8, 0, None, 0, None) == 1
    assert b"sizes must be positive" in P.lib().pat_last_error()
    assert lib.pat_conv3d_forward(None, None, None, None, 1, 2, 4, 8, 8, 8, 0, None, 0, None) == 1
    assert b"null pointer" in P.lib().pat_last_error()
    assert lib.pat_conv3d_forward(None, None, None, None, 0, 2, 4, 8, 8, 8, 0, None, 0, None) == 0   # empty batch
    assert lib.pat_adam_step(None, None, None, None, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == 1
    assert lib.pat_relu_backward(None, None, -1, None) == 1


def test_version_string():
    assert b"gfx950" in P.lib().pat_version()


@pytest.mark.parametrize("n_pix,mc", [(1024, 256), (16384, 2048)])
def test_rsp_mask_bit_exact_with_oracle(n_pix, mc):
    for seed in range(20):
        assert np.array_equal(P.pat_make_rsp_mask(n_pix, mc, seed), rsp_mask(n_pix, mc, seed))


@pytest.mark.parametrize("n_pix,mc", [(1024, 128), (16384, 2048)])
def test_shd_pattern_bit_exact_with_oracle(n_pix, mc):
    for seed in range(20):
        perm, rows = P.pat_make_shd_pattern(n_pix, mc, seed)
        operm, orows = shd_pattern(n_pix, mc, seed)
        assert np.array_equal(perm, operm) and np.array_equal(rows, orows)


def test_generators_reject_bad_arguments():
    with pytest.raises(P.PatError) as e:
        P.pat_make_rsp_mask(100, 101, 1)
    assert e.value.status == 1
    with pytest.raises(P.PatError) as e:
        P.pat_make_shd_pattern(96 * 96, 10, 1)
    assert e.value.status == 2


def _grid(n=32, nt=190, pml=8):
    return P.make_grid(n, n, n, 100e-6, 1500.0, 20e-9, nt, pml)


def test_workspace_bytes_and_validation():
    g = _grid()
    full, _ = P.make_sampling("full", 32 * 32)
    assert P.pat_plan_workspace_bytes(g, full) > 6 * 4 * 32 ** 3
    bad_full, _ = P.make_sampling("full", 100)
    assert P.pat_plan_workspace_bytes(g, bad_full) == 0
    idx = np.array([3, 2, 9], dtype=np.int32)            # not increasing
    bad_pts, keep = P.make_sampling("points", 3, idx)
    assert P.pat_plan_workspace_bytes(g, bad_pts) == 0
    assert P.pat_plan_workspace_bytes(_grid(n=48), full) == 0        # size not built
    assert P.pat_plan_workspace_bytes(_grid(pml=16), full) == 0      # PML too thick
    assert P.pat_plan_workspace_bytes(_grid(nt=0), full) == 0


def test_plan_create_reports_validation_errors_without_gpu():
    g = _grid()
    perm = np.arange(32 * 32, dtype=np.int32)
    perm[0] = 1                                         # not a permutation
    smp, keep = P.make_sampling("hadamard", 4, np.array([0, 1, 2, 3], dtype=np.int32), perm)
    h = C.c_void_p()
    st = P.lib().pat_plan_create(C.byref(g), C.byref(smp), None, None, 0, C.byref(h))
    assert st == 1 and b"permutation" in P.lib().pat_last_error()
    assert not h.value


def test_tv_dual_floats():
    g = _grid()
    assert P.pat_tv_dual_floats(g, "neumann") == 3 * 32 ** 3
    assert P.pat_tv_dual_floats(g, "dirichlet") == 3 * 33 ** 3


def test_plan_create_workspace_checks_without_gpu():
    """Workspace errors are found before the library touches the GPU (no device needed)."""
    g = _grid()
    smp, keep = P.make_sampling("full", 32 * 32)
    need = P.pat_plan_workspace_bytes(g, smp)
    h = C.c_void_p()
    lib = P.lib()
    assert lib.pat_plan_create(C.byref(g), C.byref(smp), None, None, need, C.byref(h)) == 1
    assert b"workspace is NULL" in lib.pat_last_error()
    assert lib.pat_plan_create(C.byref(g), C.byref(smp), None, C.c_void_p(0x10000 + 8), need, C.byref(h)) == 1
    assert b"aligned" in lib.pat_last_error()
    assert lib.pat_plan_create(C.byref(g), C.byref(smp), None, C.c_void_p(0x10000), need - 1, C.byref(h)) == 3
    assert b"workspace has" in lib.pat_last_error()
    assert not h.value
    assert lib.pat_plan_create(C.byref(g), C.byref(smp), None, None, 0, None) == 1


def test_concurrent_first_load_binds_once():
    """Threads that load the library at the same moment all get one fully bound handle."""
    import threading
    from paper_1605_00133_amd import nn
    P.lib()
    saved = P._lib
    try:
        for _ in range(5):
            P._lib = None
            nn._bound = False
            start = threading.Barrier(8)
            got = []

            def load():
                start.wait()
                L = nn.lib()
                got.append((L, L.pat_conv3d_forward.restype, L.pat_forward.argtypes))

            ts = [threading.Thread(target=load) for _ in range(8)]
            for t in ts:
                t.start()
            for t in ts:
                t.join()
            assert len(got) == 8
            assert len({id(L) for L, _, _ in got}) == 1
            assert all(r is C.c_int and a is not None for _, r, a in got)
    finally:
        P._lib = saved
        nn._bound = False
        nn.lib()
