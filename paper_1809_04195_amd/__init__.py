"""Python binding of ``libt2s.so`` (the gfx950 T2-Shuffling slice solver).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels behind the C ABI declared in ``include/t2s.h``.  The functions below have
the same names as the C entry points.  PyTorch is used for device memory (the
workspace, device-resident inputs and outputs) and for streams.

If the shared library has not been built, importing works but every call raises
``RuntimeError`` -- there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# T2S_LIB points at another build of the same library (the sanitizer build of the CPU tests)
LIB_PATH = os.environ.get("T2S_LIB") or os.path.join(HERE, "libt2s.so")

T2S_OK = 0
T2S_WNOTCONVERGED = 1
T2S_EINVAL = -1
T2S_ESHAPE = -2
T2S_ENOMEM = -3
T2S_EHIP = -4
T2S_ESTATE = -5
T2S_ENONFINITE = -6
T2S_EUNSUPPORTED = -7
T2S_HOST = 0
T2S_DEVICE = 1
T2S_BATCHED = 0
T2S_PER_SLICE = 1
T2S_BATCHED_GRAPH = 2
T2S_ALPHA = 0
T2S_Z = 1
T2S_U = 2
T2S_ADJOINT = 3
T2S_RESIDUAL = 4
T2S_KERNEL_PASS_A = 0
T2S_KERNEL_PASS_B = 1
T2S_KERNEL_PASS_C = 2
T2S_ORDER_XCD_PASS_A = 1
T2S_ORDER_XCD_PASS_C = 2
T2S_ORDER_XCD_PASS_B = 4
T2S_ORDER_PASS_C_LDS2 = 8
T2S_KERNEL_LLR = 3
T2S_KERNEL_LOAD = 4
KERNEL_NAMES = ("pass_a", "pass_b", "pass_c", "llr_admm", "load_adjoint")


class t2s_params(ctypes.Structure):
    _fields_ = [
        ("T", ctypes.c_int),
        ("K", ctypes.c_int),
        ("phi", ctypes.POINTER(ctypes.c_float)),
        ("lambda_", ctypes.c_float),
        ("rho", ctypes.c_float),
        ("block", ctypes.c_int),
        ("n_outer", ctypes.c_int),
        ("n_cg", ctypes.c_int),
        ("tol", ctypes.c_float),
        ("seed", ctypes.c_uint64),
        ("freeze_window", ctypes.c_int),
        ("freeze_stall", ctypes.c_float),
        ("check_every", ctypes.c_int),
    ]


class t2s_class(ctypes.Structure):
    _fields_ = [
        ("ny", ctypes.c_int),
        ("nz", ctypes.c_int),
        ("ncoils", ctypes.c_int),
        ("nslices", ctypes.c_int),
        ("masks", ctypes.POINTER(ctypes.c_uint8)),
        ("nmaps", ctypes.c_int),
    ]


class t2s_slice_report(ctypes.Structure):
    _fields_ = [
        ("outer_iterations", ctypes.c_int),
        ("k_freeze", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("r_primal", ctypes.c_double),
        ("r_dual", ctypes.c_double),
    ]


class t2s_stream_status(ctypes.Structure):
    _fields_ = [
        ("done", ctypes.c_int),
        ("in_flight", ctypes.c_int),
        ("loaded", ctypes.c_int64),
        ("slice_outer", ctypes.c_int64),
    ]


class T2SError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"t2s error {code}: {msg}")
        self.code = code


_lib = None

_SIGS = {
    "t2s_version": ([], ctypes.c_int),
    "t2s_last_error": ([], ctypes.c_char_p),
    "t2s_plan_create": ([ctypes.POINTER(t2s_params), ctypes.POINTER(t2s_class), ctypes.c_int,
                         ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "t2s_plan_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "t2s_plan_workspace_bytes": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "t2s_plan_bind_workspace": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "t2s_load_slices": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "t2s_set_initial": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                         ctypes.c_void_p], ctypes.c_int),
    "t2s_reconstruct": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "t2s_read_coeffs": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                         ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "t2s_get_slice_report": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(t2s_slice_report)],
                             ctypes.c_int),
    "t2s_apply_normal": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_float, ctypes.c_void_p], ctypes.c_int),
    "t2s_apply_llr": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_float, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p], ctypes.c_int),
    "t2s_get_psi": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "t2s_lipschitz": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p],
                      ctypes.c_int),
    "t2s_fista": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_void_p], ctypes.c_int),
    "t2s_wavelet_denoise": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                             ctypes.c_void_p], ctypes.c_int),
    "t2s_backproject": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                         ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "t2s_readout_ifft": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                         ctypes.c_int),
    "t2s_profile_enable": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "t2s_profile_read": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)],
                         ctypes.c_int),
    "t2s_set_schedule": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "t2s_get_schedule": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
                         ctypes.c_int),
    "t2s_autotune": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "t2s_set_order": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "t2s_set_slice_offset": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "t2s_get_order": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "t2s_unet_create": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                         ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "t2s_unet_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "t2s_unet_param_count": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "t2s_unet_workspace_bytes": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "t2s_unet_bind_workspace": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "t2s_unet_set_params": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_void_p], ctypes.c_int),
    "t2s_unet_get_params": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_void_p], ctypes.c_int),
    "t2s_unet_forward": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p],
                         ctypes.c_int),
    "t2s_unet_get_shape": ([ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int)] * 4, ctypes.c_int),
    "t2s_stream_open": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "t2s_stream_submit": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_void_p, ctypes.POINTER(t2s_slice_report)], ctypes.c_int),
    "t2s_stream_run": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(t2s_stream_status), ctypes.c_void_p],
                       ctypes.c_int),
    "t2s_stream_close": ([ctypes.c_void_p], ctypes.c_int),
    "t2s_unet_train_step": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                             ctypes.POINTER(ctypes.c_double), ctypes.c_void_p], ctypes.c_int),
    "t2s_unet_loss_grad": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                            ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float),
                            ctypes.c_void_p], ctypes.c_int),
    "t2s_unet_init_params": ([ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "t2s_unet_adam_apply": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_float, ctypes.c_void_p],
                            ctypes.c_int),
    "t2s_unet_get_adam_state": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                ctypes.POINTER(ctypes.c_int), ctypes.c_void_p], ctypes.c_int),
    "t2s_unet_mfma_probe": ([ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "t2s_unet_mfma_probe32": ([ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                               ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "t2s_unet_mfma_probe_static": ([ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                    ctypes.POINTER(ctypes.c_float), ctypes.c_int], ctypes.c_int),
    "t2s_block_shift": ([ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                         ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
}

EXPORTED = tuple(_SIGS)


def lib():
    """Load libt2s.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no non-HIP implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(code, allow_warn=False):
    if code < 0 or (code > 0 and not allow_warn):
        raise T2SError(code, lib().t2s_last_error().decode())
    return code


def _ptr(x):
    """Raw address of a numpy array (host) or torch tensor (device or host)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    raise TypeError(f"unsupported buffer type {type(x)}")


def _mem(x):
    if hasattr(x, "is_cuda") and x.is_cuda:
        return T2S_DEVICE
    return T2S_HOST


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return int(stream)


# ---- thin wrappers with the C names ----------------------------------------------


def t2s_version():
    return lib().t2s_version()


def t2s_last_error():
    return lib().t2s_last_error().decode()


def t2s_block_shift(seed, g, k, b):
    sy, sz = ctypes.c_int(), ctypes.c_int()
    _check(lib().t2s_block_shift(ctypes.c_uint64(seed), g, k, b, ctypes.byref(sy), ctypes.byref(sz)))
    return sy.value, sz.value


def make_params(phi, lam, rho, block=8, n_outer=20, n_cg=5, tol=0.0, seed=0, freeze_window=5,
                freeze_stall=0.05, check_every=5):
    phi = np.ascontiguousarray(phi, dtype=np.float32)
    p = t2s_params(T=phi.shape[0], K=phi.shape[1], phi=phi.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                   lambda_=lam, rho=rho, block=block, n_outer=n_outer, n_cg=n_cg, tol=tol, seed=seed,
                   freeze_window=freeze_window, freeze_stall=freeze_stall, check_every=check_every)
    p._keep = phi
    return p


def make_classes(classes):
    """classes: list of (ny, nz, ncoils, nslices, masks uint8 [T, ny, nz][, nmaps])."""
    arr = (t2s_class * len(classes))()
    keep = []
    for i, cl in enumerate(classes):
        ny, nz, nc, ns, masks = cl[:5]
        nmaps = cl[5] if len(cl) > 5 else 1
        m = np.ascontiguousarray(masks, dtype=np.uint8)
        keep.append(m)
        arr[i] = t2s_class(ny=ny, nz=nz, ncoils=nc, nslices=ns,
                           masks=m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), nmaps=nmaps)
    return arr, keep


def t2s_plan_create(params, classes_arr, n_classes):
    h = ctypes.c_void_p()
    _check(lib().t2s_plan_create(ctypes.byref(params), classes_arr, n_classes, ctypes.byref(h)))
    return h


def t2s_plan_destroy(plan):
    return _check(lib().t2s_plan_destroy(plan))


def t2s_plan_workspace_bytes(plan):
    n = ctypes.c_size_t()
    _check(lib().t2s_plan_workspace_bytes(plan, ctypes.byref(n)))
    return n.value


def t2s_plan_bind_workspace(plan, ptr, nbytes, stream=None):
    return _check(lib().t2s_plan_bind_workspace(plan, ptr, nbytes, _stream(stream)))


def t2s_load_slices(plan, cls, first, count, sens, ksp, stream=None):
    return _check(lib().t2s_load_slices(plan, cls, first, count, _ptr(sens), _ptr(ksp), _mem(sens), _stream(stream)))


def t2s_set_initial(plan, cls, first, count, alpha0, stream=None):
    return _check(lib().t2s_set_initial(plan, cls, first, count, _ptr(alpha0), _mem(alpha0), _stream(stream)))


def t2s_reconstruct(plan, mode=T2S_BATCHED, stream=None):
    return _check(lib().t2s_reconstruct(plan, mode, _stream(stream)), allow_warn=True)


def t2s_read_coeffs(plan, cls, first, count, out, which=T2S_ALPHA, stream=None):
    return _check(lib().t2s_read_coeffs(plan, cls, first, count, _ptr(out), which, _mem(out), _stream(stream)))


def t2s_get_slice_report(plan, cls, slice_):
    r = t2s_slice_report()
    _check(lib().t2s_get_slice_report(plan, cls, slice_, ctypes.byref(r)))
    return _report_dict(r)


def _report_dict(r):
    return dict(outer_iterations=r.outer_iterations, k_freeze=r.k_freeze, converged=r.converged,
                r_primal=r.r_primal, r_dual=r.r_dual)


def t2s_stream_open(plan, cls=0, net=None, mode=T2S_BATCHED_GRAPH):
    """net: a UNet (or its handle) for the warm start, None for a cold start."""
    h = None if net is None else getattr(net, "handle", net)
    return _check(lib().t2s_stream_open(plan, cls, h, mode))


def t2s_stream_submit(plan, count, first_global, sens, ksp, alpha_out, reports=None):
    """reports: a ctypes array of `count` t2s_slice_report (kept alive by the caller) or None."""
    return _check(lib().t2s_stream_submit(plan, count, first_global, _ptr(sens), _ptr(ksp), _ptr(alpha_out),
                                          reports))


def t2s_stream_run(plan, min_done=0, stream=None):
    """(code, {done, in_flight, loaded, slice_outer}: counts since open)."""
    st = t2s_stream_status()
    code = _check(lib().t2s_stream_run(plan, min_done, ctypes.byref(st), _stream(stream)), allow_warn=True)
    return code, dict(done=st.done, in_flight=st.in_flight, loaded=st.loaded, slice_outer=st.slice_outer)


def t2s_stream_close(plan):
    return _check(lib().t2s_stream_close(plan))


def t2s_apply_normal(plan, cls, first, count, inp, out, rho_add=0.0, stream=None):
    return _check(lib().t2s_apply_normal(plan, cls, first, count, _ptr(inp), _ptr(out), rho_add, _stream(stream)))


def t2s_apply_llr(plan, cls, first, count, inp, out, tau, shifts, stream=None):
    sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.int32).reshape(-1))
    return _check(lib().t2s_apply_llr(plan, cls, first, count, _ptr(inp), _ptr(out), tau,
                                      sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _stream(stream)))


def t2s_profile_enable(plan, enable=True):
    return _check(lib().t2s_profile_enable(plan, 1 if enable else 0))


def t2s_profile_read(plan, kernel):
    n, ms = ctypes.c_int(), ctypes.c_double()
    _check(lib().t2s_profile_read(plan, kernel, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def t2s_set_schedule(plan, cls, chunk, nstreams):
    return _check(lib().t2s_set_schedule(plan, cls, chunk, nstreams))


def t2s_get_schedule(plan, cls):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(lib().t2s_get_schedule(plan, cls, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def t2s_set_order(plan, cls, order):
    return _check(lib().t2s_set_order(plan, cls, order))


def t2s_set_slice_offset(plan, cls, first_global):
    return _check(lib().t2s_set_slice_offset(plan, cls, first_global))


def t2s_get_order(plan, cls):
    o = ctypes.c_int()
    _check(lib().t2s_get_order(plan, cls, ctypes.byref(o)))
    return o.value


def t2s_autotune(plan, reps=3, stream=None):
    return _check(lib().t2s_autotune(plan, reps, _stream(stream)))


def t2s_lipschitz(plan, cls, nslices, iters=30, stream=None):
    out = np.zeros(nslices, dtype=np.float64)
    _check(lib().t2s_lipschitz(plan, cls, iters, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               _stream(stream)))
    return out


def t2s_fista(plan, mode, n_iter, step, stream=None):
    return _check(lib().t2s_fista(plan, mode, n_iter, step, _stream(stream)))


def t2s_wavelet_denoise(plan, cls, first, count, levels, thresh, stream=None):
    return _check(lib().t2s_wavelet_denoise(plan, cls, first, count, levels, thresh, _stream(stream)))


def t2s_backproject(plan, cls, first, count, phi_te, out, stream=None):
    """phi_te: host [n_te][K] basis rows; out: device complex64 [count][n_te][ny][nz]."""
    ph = np.ascontiguousarray(np.asarray(phi_te, dtype=np.float32))
    return _check(lib().t2s_backproject(plan, cls, first, count, ph.shape[0],
                                        ph.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _ptr(out), _stream(stream)))


def t2s_readout_ifft(inp, out, stream=None):
    """inp: device complex64 [C][P][nx]; out: device complex64 [nx][C][P]."""
    C, P, nx = inp.shape
    if tuple(out.shape) != (nx, C, P):
        raise ValueError(f"out must have shape {(nx, C, P)}")
    return _check(lib().t2s_readout_ifft(nx, C, P, _ptr(inp), _ptr(out), _stream(stream)))


def t2s_get_psi(plan, cls, K, ny, nz):
    out = np.empty((K * (K + 1) // 2, nz, ny), dtype=np.float32)
    _check(lib().t2s_get_psi(plan, cls, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


# ---- convenience object -------------------------------------------------------------


class Plan:
    """A plan plus its torch-allocated workspace.

    classes: list of dicts with keys ny, nz, ncoils, nslices, masks.
    """

    def __init__(self, phi, classes, lam, rho, block=8, n_outer=20, n_cg=5, tol=0.0, seed=0,
                 freeze_window=5, freeze_stall=0.05, check_every=5, device="cuda"):
        import torch
        self.phi = np.ascontiguousarray(phi, dtype=np.float32)
        self.K = self.phi.shape[1]
        self.classes = classes
        self._params = make_params(self.phi, lam, rho, block, n_outer, n_cg, tol, seed, freeze_window,
                                   freeze_stall, check_every)
        arr, self._keep = make_classes([(c["ny"], c["nz"], c["ncoils"], c["nslices"], c["masks"], c.get("nmaps", 1))
                                        for c in classes])
        self.handle = t2s_plan_create(self._params, arr, len(classes))
        self.nbytes = t2s_plan_workspace_bytes(self.handle)
        self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        t2s_plan_bind_workspace(self.handle, aligned, self.nbytes)

    def load(self, cls, first, sens, ksp, stream=None):
        return t2s_load_slices(self.handle, cls, first, sens.shape[0], sens, ksp, stream)

    def set_initial(self, cls, first, alpha0, stream=None):
        return t2s_set_initial(self.handle, cls, first, alpha0.shape[0], alpha0, stream)

    def reconstruct(self, mode=T2S_BATCHED, stream=None):
        return t2s_reconstruct(self.handle, mode, stream)

    def lipschitz(self, cls, iters=30, stream=None):
        return t2s_lipschitz(self.handle, cls, self.classes[cls]["nslices"], iters, stream)

    def fista(self, n_iter, step, mode=T2S_BATCHED, stream=None):
        return t2s_fista(self.handle, mode, n_iter, step, stream)

    def wavelet_denoise(self, cls, first, count, levels, thresh, stream=None):
        return t2s_wavelet_denoise(self.handle, cls, first, count, levels, thresh, stream)

    def backproject(self, cls, first, count, phi_te, stream=None):
        """Device complex64 [count][n_te][ny][nz] images at the echo times of the rows of phi_te."""
        import torch
        ph = np.asarray(phi_te, dtype=np.float32).reshape(-1, self.K)
        c = self.classes[cls]
        M = c.get("nmaps", 1)
        shape = (count, ph.shape[0], c["ny"], c["nz"]) if M <= 1 else (count, M, ph.shape[0], c["ny"], c["nz"])
        out = torch.empty(shape, dtype=torch.complex64, device="cuda")
        t2s_backproject(self.handle, cls, first, count, ph, out, stream)
        return out

    def read(self, cls, first, count, which=T2S_ALPHA, device=False, stream=None):
        c = self.classes[cls]
        M = c.get("nmaps", 1)
        shape = (count, self.K, c["ny"], c["nz"]) if M <= 1 else (count, M, self.K, c["ny"], c["nz"])
        if device:
            import torch
            out = torch.empty(shape, dtype=torch.complex64, device="cuda")
        else:
            out = np.empty(shape, dtype=np.complex64)
        t2s_read_coeffs(self.handle, cls, first, count, out, which, stream)
        return out

    def report(self, cls, s):
        return t2s_get_slice_report(self.handle, cls, s)

    # continuous batching: the slices of a one-class plan become slots fed from a queue
    def stream_open(self, net=None, mode=T2S_BATCHED_GRAPH):
        self._stream_reports = []
        return t2s_stream_open(self.handle, 0, net, mode)

    def stream_submit(self, sens, ksp, alpha_out, first_global):
        """Queue the slices of device tensors sens [n][C](M)[ny][nz] and ksp [n][C][P];
        results go to alpha_out [n](M)[K][ny][nz]; returns the report array (filled as
        slices complete; `stream_reports` turns it into dicts)."""
        n = sens.shape[0]
        if ksp.shape[0] != n or alpha_out.shape[0] != n:
            raise ValueError("sens, ksp and alpha_out must hold the same number of slices")
        rep = (t2s_slice_report * n)()
        self._stream_reports.append(rep)     # the library writes into it until the slices complete
        t2s_stream_submit(self.handle, n, first_global, sens, ksp, alpha_out, rep)
        return rep

    def stream_run(self, min_done=0, stream=None):
        return t2s_stream_run(self.handle, min_done, stream)

    def stream_close(self):
        return t2s_stream_close(self.handle)

    @staticmethod
    def stream_reports(rep):
        return [_report_dict(r) for r in rep]

    def close(self):
        if self.handle is not None:
            t2s_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- warm-start network ---------------------------------------------------------------

_FP = ctypes.POINTER(ctypes.c_float)


def _fptr(a):
    return a.ctypes.data_as(_FP)


def t2s_unet_mfma_probe(A, B):
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    D = np.empty((16, 16), dtype=np.float32)
    _check(lib().t2s_unet_mfma_probe(_fptr(A), _fptr(B), _fptr(D)))
    return D


def t2s_unet_mfma_probe32(A, B):
    """D = A B for A [16, 32], B [32, 16] through the 32-deep bf16 matrix-core product."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    if A.shape != (16, 32) or B.shape != (32, 16):
        raise ValueError("A must be [16, 32] and B [32, 16]")
    D = np.empty((16, 16), dtype=np.float32)
    _check(lib().t2s_unet_mfma_probe32(_fptr(A), _fptr(B), _fptr(D)))
    return D


def t2s_unet_mfma_probe_static(A, B):
    """A, B: [count, 16, 16]; D[i] = A[i] B[i] through the allocation-free entry point."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    if A.shape != B.shape or A.ndim != 3 or A.shape[1:] != (16, 16):
        raise ValueError("A and B must both be [count, 16, 16]")
    D = np.empty(A.shape, dtype=np.float32)
    _check(lib().t2s_unet_mfma_probe_static(_fptr(A), _fptr(B), _fptr(D), A.shape[0]))
    return D


class UNet:
    """The warm-start network (kernels in libt2s.so) with a torch-allocated workspace."""

    def __init__(self, K, base=32, levels=4, max_batch=16, H=256, W=256, device="cuda"):
        import torch
        self.K, self.base, self.levels, self.max_batch, self.H, self.W = K, base, levels, max_batch, H, W
        h = ctypes.c_void_p()
        _check(lib().t2s_unet_create(K, base, levels, max_batch, H, W, ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_size_t()
        _check(lib().t2s_unet_param_count(h, ctypes.byref(n)))
        self.nparams = n.value
        _check(lib().t2s_unet_workspace_bytes(h, ctypes.byref(n)))
        self.nbytes = n.value
        self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        base_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        _check(lib().t2s_unet_bind_workspace(h, base_ptr, self.nbytes, _stream(None)))

    def set_params(self, params, stream=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {p.size}")
        _check(lib().t2s_unet_set_params(self.handle, _fptr(p), _stream(stream)))

    def init_params(self, seed=0):
        """Library-generated initial parameters (host float32, packed)."""
        p = np.empty(self.nparams, dtype=np.float32)
        _check(lib().t2s_unet_init_params(self.handle, ctypes.c_uint64(seed), _fptr(p)))
        return p

    def get_params(self, stream=None):
        p = np.empty(self.nparams, dtype=np.float32)
        _check(lib().t2s_unet_get_params(self.handle, _fptr(p), _stream(stream)))
        return p

    def forward(self, b0, out, stream=None):
        """b0, out: device complex64 tensors [B, K, H, W]."""
        _check(lib().t2s_unet_forward(self.handle, _ptr(b0), _ptr(out), b0.shape[0], _stream(stream)))
        return out

    def train_step(self, b0, target, lr, want_loss=False, stream=None):
        loss = ctypes.c_double()
        _check(lib().t2s_unet_train_step(self.handle, _ptr(b0), _ptr(target), b0.shape[0], lr,
                                         ctypes.byref(loss) if want_loss else None, _stream(stream)))
        return loss.value if want_loss else None

    def loss_grad(self, x, t, stream=None):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        g = np.empty(self.nparams, dtype=np.float32)
        loss = ctypes.c_double()
        _check(lib().t2s_unet_loss_grad(self.handle, _fptr(x), _fptr(t), x.shape[0], ctypes.byref(loss), _fptr(g),
                                        _stream(stream)))
        return loss.value, g

    def adam_apply(self, grad, lr, stream=None):
        """One Adam step of the training path with the given host gradient."""
        g = np.ascontiguousarray(grad, dtype=np.float32)
        if g.size != self.nparams:
            raise ValueError(f"expected {self.nparams} gradient values, got {g.size}")
        _check(lib().t2s_unet_adam_apply(self.handle, _fptr(g), lr, _stream(stream)))

    def adam_state(self, stream=None):
        """(m, v, step) of the optimiser."""
        m = np.empty(self.nparams, dtype=np.float32)
        v = np.empty(self.nparams, dtype=np.float32)
        step = ctypes.c_int()
        _check(lib().t2s_unet_get_adam_state(self.handle, _fptr(m), _fptr(v), ctypes.byref(step), _stream(stream)))
        return m, v, step.value

    def close(self):
        if self.handle is not None:
            lib().t2s_unet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
