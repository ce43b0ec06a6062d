"""ctypes binding of libpat.so (the C ABI declared in include/pat.h).

Argument marshalling only: every step of the computation runs in the HIP
library. Torch tensors supply device memory (data_ptr) and the HIP stream
(torch.cuda.current_stream().cuda_stream); shapes, dtypes and devices are
checked here so a mistaken call raises instead of reaching a kernel.
The module raises at import of the library if libpat.so has not been built.
"""

import ctypes as C
import os
import threading

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; PAT_LIB names another build of the same library
LIB_PATH = os.environ.get("PAT_LIB") or os.path.join(_PKG, "libpat.so")

PAT_SAMPLE_FULL, PAT_SAMPLE_POINTS, PAT_SAMPLE_HADAMARD = 0, 1, 2
KIND = {"full": PAT_SAMPLE_FULL, "points": PAT_SAMPLE_POINTS, "hadamard": PAT_SAMPLE_HADAMARD}
BC = {"neumann": 0, "dirichlet": 1, 0: 0, 1: 1}
STATUS = {0: "PAT_OK", 1: "PAT_ERR_INVALID", 2: "PAT_ERR_UNSUPPORTED", 3: "PAT_ERR_NOMEM",
          4: "PAT_ERR_HIP", 5: "PAT_ERR_NONFINITE"}


class PatError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class pat_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dx", C.c_double),
                ("c0", C.c_double), ("rho0", C.c_double), ("dt", C.c_double), ("nt", C.c_int32),
                ("pml_size", C.c_int32), ("pml_alpha", C.c_double)]


class pat_sampling(C.Structure):
    _fields_ = [("kind", C.c_int32), ("mc", C.c_int32), ("idx", C.POINTER(C.c_int32)),
                ("perm", C.POINTER(C.c_int32))]


class pat_recon_params(C.Structure):
    _fields_ = [("lam", C.c_double), ("L", C.c_double), ("n_outer", C.c_int32), ("n_inner", C.c_int32),
                ("n_prox", C.c_int32), ("bc", C.c_int32), ("restart", C.c_int32),
                ("max_backtrack", C.c_int32), ("p_ref", C.c_void_p)]


class pat_recon_report(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("n_log", C.c_int32), ("energy", C.POINTER(C.c_double)),
                ("residual", C.POINTER(C.c_double)), ("tv", C.POINTER(C.c_double)),
                ("flags", C.POINTER(C.c_int32)), ("psnr", C.POINTER(C.c_double)),
                ("t_ms", C.POINTER(C.c_double)), ("bregman_residual", C.POINTER(C.c_double))]


_P = C.c_void_p
# name -> (restype, argtypes)
SIGNATURES = {
    "pat_plan_workspace_bytes": (C.c_size_t, [C.POINTER(pat_grid), C.POINTER(pat_sampling)]),
    "pat_plan_create": (C.c_int, [C.POINTER(pat_grid), C.POINTER(pat_sampling), _P, _P, C.c_size_t,
                                  C.POINTER(_P)]),
    "pat_plan_destroy": (C.c_int, [_P]),
    "pat_plan_set_stream": (C.c_int, [_P, _P]),
    "pat_plan_set_fft_precision": (C.c_int, [_P, C.c_int32]),
    "pat_plan_set_sensitivity": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "pat_plan_set_sound_speed": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "pat_plan_set_scheme": (C.c_int, [_P, C.c_int32]),
    "pat_forward": (C.c_int, [_P, _P, _P]),
    "pat_adjoint": (C.c_int, [_P, _P, _P]),
    "pat_time_reversal": (C.c_int, [_P, _P, _P]),
    "pat_sample": (C.c_int, [_P, _P, _P]),
    "pat_sample_adjoint": (C.c_int, [_P, _P, _P]),
    "pat_tv_dual_floats": (C.c_size_t, [C.POINTER(pat_grid), C.c_int32]),
    "pat_tv_prox": (C.c_int, [_P, _P, _P, C.c_float, C.c_int32, C.c_int32, _P]),
    "pat_tv_norm": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_double)]),
    "pat_power_iteration": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_double)]),
    "pat_reconstruct": (C.c_int, [_P, _P, _P, C.POINTER(pat_recon_params), C.POINTER(pat_recon_report)]),
    "pat_psnr": (C.c_int, [_P, _P, _P, C.POINTER(C.c_double)]),
    "pat_fista_enqueue": (C.c_int, [_P, _P, _P, C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_int32, _P]),
    "pat_fista_enqueue_from": (C.c_int, [_P, _P, _P, C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_int32,
                                         C.c_int32, _P]),
    "pat_make_rsp_mask": (C.c_int, [C.c_int32, C.c_int32, C.c_uint64, C.POINTER(C.c_int32)]),
    "pat_make_shd_pattern": (C.c_int, [C.c_int32, C.c_int32, C.c_uint64, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]),
    "pat_profile_begin": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "pat_profile_end": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "pat_kernel_info": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_char_p), C.POINTER(C.c_double)]),
    "pat_copy_probe": (C.c_int, [_P, _P, C.c_int64, _P]),
    "pat_last_error": (C.c_char_p, []),
    "pat_version": (C.c_char_p, []),
}

_lib = None
_lib_lock = threading.Lock()


def lib():
    """Load libpat.so (raises if it has not been built).

    torch is imported first so that its bundled HIP runtime is the only one in
    the process: libpat.so then binds to it by soname instead of mapping a
    second runtime from /opt/rocm, which would fail to initialise next to
    torch's. Thread-safe: the first caller loads and binds under a lock, and
    the handle is published only once every signature is set.
    """
    global _lib
    if _lib is not None:
        return _lib
    with _lib_lock:
        if _lib is None:
            import torch  # noqa: F401  (load order matters, see docstring)
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1605_00133_amd.build`")
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise PatError(status, lib().pat_last_error().decode())


def _i32ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32)) if a is not None else None


# ---- host-only generators -------------------------------------------------------------
def pat_make_rsp_mask(n_pix, mc, seed):
    out = np.zeros(mc, dtype=np.int32)
    _check(lib().pat_make_rsp_mask(n_pix, mc, seed, _i32ptr(out)))
    return out


def pat_make_shd_pattern(n_pix, mc, seed):
    perm = np.zeros(n_pix, dtype=np.int32)
    rows = np.zeros(mc, dtype=np.int32)
    _check(lib().pat_make_shd_pattern(n_pix, mc, seed, _i32ptr(perm), _i32ptr(rows)))
    return perm, rows


def make_grid(nx, ny, nz, dx, c0, dt, nt, pml_size=8, pml_alpha=2.0, rho0=1.0):
    return pat_grid(nx, ny, nz, dx, c0, rho0, dt, nt, pml_size, pml_alpha)


def make_sampling(kind, mc, idx=None, perm=None):
    """Returns (struct, keepalive) for a sampling description with host int32 arrays."""
    idx = None if idx is None else np.ascontiguousarray(idx, dtype=np.int32)
    perm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    s = pat_sampling(KIND[kind] if isinstance(kind, str) else int(kind), mc, _i32ptr(idx), _i32ptr(perm))
    return s, (idx, perm)


def pat_plan_workspace_bytes(grid, smp):
    return lib().pat_plan_workspace_bytes(C.byref(grid), C.byref(smp))


def pat_tv_dual_floats(grid, bc):
    return lib().pat_tv_dual_floats(C.byref(grid), BC[bc])


# ---- plan ----------------------------------------------------------------------------
class Plan:
    """Owns a pat_plan and its device workspace (a torch uint8 tensor)."""

    def __init__(self, grid, kind="full", mc=None, idx=None, perm=None, device="cuda:0"):
        import torch
        self.torch = torch
        self.grid = grid
        self.device = torch.device(device)
        npix = grid.nx * grid.ny
        mc = npix if mc is None else int(mc)
        self.mc = mc
        self.kind = kind
        self.smp, self._keep = make_sampling(kind, mc, idx, perm)
        nbytes = pat_plan_workspace_bytes(grid, self.smp)
        if nbytes == 0:
            # re-run creation to obtain the validation message
            handle = C.c_void_p()
            _check(lib().pat_plan_create(C.byref(grid), C.byref(self.smp), None, None, 0, C.byref(handle)))
            raise PatError(1, "invalid plan arguments")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.handle = C.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _check(lib().pat_plan_create(C.byref(grid), C.byref(self.smp), C.c_void_p(stream),
                                         C.c_void_p(aligned), nbytes, C.byref(self.handle)))

    @property
    def vol_shape(self):
        g = self.grid
        return (g.nz, g.ny, g.nx)

    @property
    def data_shape(self):
        return (self.grid.nt, self.mc)

    @property
    def plane_shape(self):
        g = self.grid
        return (g.nt, g.ny, g.nx)

    def set_fft_precision(self, bits):
        _check(lib().pat_plan_set_fft_precision(self.handle, int(bits)))

    def set_sensitivity(self, w):
        """Per-pixel sensor sensitivity W_s (host array [ny][nx] or None for the ideal sensor)."""
        if w is None:
            _check(lib().pat_plan_set_sensitivity(self.handle, None))
            return
        w = np.ascontiguousarray(w, dtype=np.float32).ravel()
        if w.size != self.grid.nx * self.grid.ny:
            raise ValueError(f"w must have {self.grid.nx * self.grid.ny} entries")
        _check(lib().pat_plan_set_sensitivity(self.handle, w.ctypes.data_as(C.POINTER(C.c_float))))

    def set_sound_speed(self, c):
        """Heterogeneous sound speed [nz][ny][nx] (host array, each <= c0) for data generation, or None."""
        if c is None:
            _check(lib().pat_plan_set_sound_speed(self.handle, None))
            return
        c = np.ascontiguousarray(c, dtype=np.float32).ravel()
        g = self.grid
        if c.size != g.nx * g.ny * g.nz:
            raise ValueError(f"c must have {g.nx * g.ny * g.nz} entries")
        _check(lib().pat_plan_set_sound_speed(self.handle, c.ctypes.data_as(C.POINTER(C.c_float))))

    def set_scheme(self, scheme):
        """PAT_SCHEME_LINE (default on cubic grids) or PAT_SCHEME_SLAB; the names "line"/"slab" work too."""
        if isinstance(scheme, str):
            scheme = {"slab": PAT_SCHEME_SLAB, "line": PAT_SCHEME_LINE}[scheme]
        _check(lib().pat_plan_set_scheme(self.handle, int(scheme)))

    def sync_stream(self):
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().pat_plan_set_stream(self.handle, C.c_void_p(stream)))

    def check(self, t, shape, name):
        torch = self.torch
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != torch.float32 or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 tensor on {self.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        return C.c_void_p(t.data_ptr())

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            _check(lib().pat_plan_destroy(self.handle))
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pat_forward(plan, p0, f):
    plan.sync_stream()
    _check(lib().pat_forward(plan.handle, plan.check(p0, plan.vol_shape, "p0"), plan.check(f, plan.data_shape, "f")))


def pat_adjoint(plan, f, p):
    plan.sync_stream()
    _check(lib().pat_adjoint(plan.handle, plan.check(f, plan.data_shape, "f"), plan.check(p, plan.vol_shape, "p")))


def pat_time_reversal(plan, f, p):
    plan.sync_stream()
    _check(lib().pat_time_reversal(plan.handle, plan.check(f, plan.data_shape, "f"),
                                   plan.check(p, plan.vol_shape, "p")))


def pat_sample(plan, s, f):
    plan.sync_stream()
    _check(lib().pat_sample(plan.handle, plan.check(s, plan.plane_shape, "s"), plan.check(f, plan.data_shape, "f")))


def pat_sample_adjoint(plan, f, s):
    plan.sync_stream()
    _check(lib().pat_sample_adjoint(plan.handle, plan.check(f, plan.data_shape, "f"),
                                    plan.check(s, plan.plane_shape, "s")))


def pat_tv_prox(plan, v, q, alpha, n_iter, bc, dual):
    plan.sync_stream()
    nd = pat_tv_dual_floats(plan.grid, bc)
    _check(lib().pat_tv_prox(plan.handle, plan.check(v, plan.vol_shape, "v"), plan.check(q, plan.vol_shape, "q"),
                             float(alpha), int(n_iter), BC[bc], plan.check(dual, (nd,), "dual")))


def pat_tv_norm(plan, p, bc):
    plan.sync_stream()
    out = C.c_double()
    _check(lib().pat_tv_norm(plan.handle, plan.check(p, plan.vol_shape, "p"), BC[bc], C.byref(out)))
    return out.value


def pat_psnr(plan, p, p_ref):
    plan.sync_stream()
    out = C.c_double()
    _check(lib().pat_psnr(plan.handle, plan.check(p, plan.vol_shape, "p"), plan.check(p_ref, plan.vol_shape, "p_ref"),
                          C.byref(out)))
    return out.value


def pat_power_iteration(plan, x0, n_iter):
    plan.sync_stream()
    out = C.c_double()
    _check(lib().pat_power_iteration(plan.handle, plan.check(x0, plan.vol_shape, "x0"), int(n_iter), C.byref(out)))
    return out.value


def pat_copy_probe(src, dst):
    """dst = src (contiguous CUDA tensors of the same byte size, a multiple of 16) with the library's
    copy kernel, on the current stream: the HBM copy-rate probe of the bench."""
    import torch
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous CUDA tensors")
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("src and dst must have the same size in bytes")
    stream = torch.cuda.current_stream(dst.device).cuda_stream
    _check(lib().pat_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), int(nb), C.c_void_p(stream)))


PAT_K_COUNT = 10
PAT_K_LINE_FWD = 8
PAT_K_LINE_ADJ = 9
PAT_SCHEME_SLAB = 0
PAT_SCHEME_LINE = 1


def pat_profile_begin(plan, kernel_id=-2, max_launches=8192):
    _check(lib().pat_profile_begin(plan.handle, int(kernel_id), int(max_launches)))


def pat_profile_end(plan):
    """Returns (total_ms[PAT_K_COUNT], launches[PAT_K_COUNT]) as numpy arrays."""
    tot = (C.c_double * PAT_K_COUNT)()
    cnt = (C.c_int32 * PAT_K_COUNT)()
    _check(lib().pat_profile_end(plan.handle, tot, cnt))
    return np.array(tot[:]), np.array(cnt[:])


def pat_kernel_info(plan, kernel_id):
    name = C.c_char_p()
    nbytes = C.c_double()
    _check(lib().pat_kernel_info(plan.handle, int(kernel_id), C.byref(name), C.byref(nbytes)))
    return name.value.decode(), nbytes.value


def pat_reconstruct(plan, f, p, lam, L, n_outer=1, n_inner=10, n_prox=50, bc="dirichlet", restart=True,
                    max_backtrack=5, p_ref=None, log_capacity=None):
    """Runs TV+ / TV+Br; returns the per-iteration log as a dict of numpy arrays."""
    plan.sync_stream()
    cap = n_outer * n_inner if log_capacity is None else int(log_capacity)
    arrs = {k: np.full(max(cap, 1), np.nan) for k in ("energy", "residual", "tv", "psnr", "t_ms")}
    flags = np.zeros(max(cap, 1), dtype=np.int32)
    breg = np.full(max(n_outer, 1), np.nan)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    rep = pat_recon_report(cap, 0, dp(arrs["energy"]), dp(arrs["residual"]), dp(arrs["tv"]),
                           flags.ctypes.data_as(C.POINTER(C.c_int32)), dp(arrs["psnr"]), dp(arrs["t_ms"]), dp(breg))
    pref = None if p_ref is None else plan.check(p_ref, plan.vol_shape, "p_ref")
    prm = pat_recon_params(float(lam), float(L), int(n_outer), int(n_inner), int(n_prox), BC[bc],
                           1 if restart else 0, int(max_backtrack), pref)
    _check(lib().pat_reconstruct(plan.handle, plan.check(f, plan.data_shape, "f"), plan.check(p, plan.vol_shape, "p"),
                                 C.byref(prm), C.byref(rep)))
    n = rep.n_log
    out = {k: v[:n].copy() for k, v in arrs.items()}
    out["flags"] = flags[:n].copy()
    out["bregman_residual"] = breg[:n_outer].copy()
    return out


def _enqueue_log(plan, log, n_iter):
    if log is None:
        return None
    t = plan.torch
    if log.dtype != t.float64 or log.device != plan.device or not log.is_contiguous() or \
            tuple(log.shape) != (int(n_iter), 2):
        raise ValueError(f"log must be a contiguous float64 tensor [{n_iter}, 2] on {plan.device}")
    return C.c_void_p(log.data_ptr())


def pat_fista_enqueue(plan, f, p, lam, L, n_iter=30, n_prox=50, bc="dirichlet", log=None):
    """Enqueues n_iter TV+ FISTA iterations (no restart, no host synchronisation: capturable in a
    HIP graph). log: None or a float64 device tensor [n_iter, 2] (sum r^2, TV per iteration)."""
    plan.sync_stream()
    lp = _enqueue_log(plan, log, n_iter)
    _check(lib().pat_fista_enqueue(plan.handle, plan.check(f, plan.data_shape, "f"), plan.check(p, plan.vol_shape, "p"),
                                   float(lam), float(L), int(n_iter), int(n_prox), BC[bc], lp))


def pat_fista_enqueue_from(plan, f, p, lam, L, it0, n_iter, n_prox=50, bc="dirichlet", log=None):
    """Iterations it0 .. it0 + n_iter - 1 of the loop of pat_fista_enqueue, continuing from the state
    the call for iterations 0 .. it0 - 1 left in the plan (same f, lam, L, n_prox, bc): the parts give
    the one-call result bit for bit. log: None or float64 [n_iter, 2] for these iterations."""
    plan.sync_stream()
    lp = _enqueue_log(plan, log, n_iter)
    _check(lib().pat_fista_enqueue_from(plan.handle, plan.check(f, plan.data_shape, "f"),
                                        plan.check(p, plan.vol_shape, "p"), float(lam), float(L), int(it0),
                                        int(n_iter), int(n_prox), BC[bc], lp))
