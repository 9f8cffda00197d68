"""Python binding of the C ABI declared in include/heget.h (argument marshalling only).

Every computation happens in the HIP library libheget.so; this module only
passes device pointers, sizes and the current HIP stream through ctypes.  It
raises if the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HEGET_LIB", os.path.join(HERE, "libheget.so"))

HEGET_OK = 0
HEGET_FP64 = 0
HEGET_MIXED = 1
PRECISIONS = {"fp64": HEGET_FP64, "mixed": HEGET_MIXED}

_lib = None


class BatchItem(ctypes.Structure):
    """heget_batch_item of include/heget.h."""
    _fields_ = [("process", ctypes.c_void_p), ("momenta", ctypes.c_void_p),
                ("n_events", ctypes.c_int64), ("me2", ctypes.c_void_p)]


class Cuts(ctypes.Structure):
    """heget_cuts of include/heget.h: pT_min (GeV), eta_max, Delta R_min (<= 0: no pair cut)."""
    _fields_ = [("pt_min", ctypes.c_double), ("eta_max", ctypes.c_double), ("delta_r_min", ctypes.c_double)]


class HegetError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {lib().heget_status_string(status).decode()} (status {status})")
        self.status = status


def lib():
    """Load libheget.so (once) and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_0909_5257_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    pi32, pi64, pdbl = ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(dbl)
    L.heget_create_process.argtypes = [ctypes.c_char_p, i32, ctypes.POINTER(vp)]
    L.heget_create_process.restype = i32
    L.heget_process_info.argtypes = [vp, pi32, pi32, pi32, pi32]
    L.heget_process_info.restype = i32
    L.heget_matrix_elements.argtypes = [vp, vp, i64, dbl, vp, vp]
    L.heget_matrix_elements.restype = i32
    L.heget_matrix_elements_helicity.argtypes = [vp, vp, vp, i64, dbl, vp, vp]
    L.heget_matrix_elements_helicity.restype = i32
    L.heget_color_matrix.argtypes = [vp, pi32, pi64, pi64, pdbl]
    L.heget_color_matrix.restype = i32
    L.heget_process_flops.argtypes = [vp, pi64]
    L.heget_process_flops.restype = i32
    L.heget_destroy_process.argtypes = [vp]
    L.heget_destroy_process.restype = None
    L.heget_status_string.argtypes = [i32]
    L.heget_status_string.restype = ctypes.c_char_p
    L.heget_matrix_elements_batch.argtypes = [ctypes.POINTER(BatchItem), i32, dbl, i32, vp]
    L.heget_matrix_elements_batch.restype = i32
    L.heget_colour_quadratic_form.argtypes = [i32, vp, vp, i64, i32, vp, vp]
    L.heget_colour_quadratic_form.restype = i32
    L.heget_rambo.argtypes = [i32, i64, vp, vp, vp, vp, vp]
    L.heget_rambo.restype = i32
    L.heget_apply_cuts.argtypes = [i32, i64, vp, ctypes.POINTER(Cuts), vp, vp]
    L.heget_apply_cuts.restype = i32
    L.heget_integrate_step.argtypes = [vp, i64, vp, vp, vp, dbl, ctypes.POINTER(Cuts), vp, vp, vp, vp, vp]
    L.heget_integrate_step.restype = i32
    L.heget_integrate_step_noalloc.argtypes = [vp, i64, vp, vp, vp, dbl, ctypes.POINTER(Cuts), vp, vp, vp, vp, vp]
    L.heget_integrate_step_noalloc.restype = i32
    L.heget_colour_reduction.argtypes = [vp, pi32, pi32, pi64, pi64, pi64, pi64, pi32]
    L.heget_colour_reduction.restype = i32
    L.heget_matrix_elements_hook.argtypes = [vp, vp, i64, dbl, i32, vp, vp, vp]
    L.heget_matrix_elements_hook.restype = i32
    L.heget_num_processes.argtypes = []
    L.heget_num_processes.restype = i32
    L.heget_process_spec.argtypes = [i32]
    L.heget_process_spec.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status, what):
    if status != HEGET_OK:
        raise HegetError(status, what)


def supported_processes() -> list:
    L = lib()
    return [L.heget_process_spec(i).decode() for i in range(L.heget_num_processes())]


def _launch_stream(device, stream):
    """The stream to launch on.  A caller-given stream other than the current one first waits for
    the current stream, so that buffers prepared there (copies, allocations) are ready."""
    import torch
    cur = torch.cuda.current_stream(device)
    if stream is None:
        return cur, False
    if stream != cur:
        stream.wait_stream(cur)
        return stream, True
    return stream, False


def _keep_alive(side_stream: bool, stream, *tensors):
    """Tell the caching allocator that temporaries are used on a side stream (no reuse before the
    work queued there has run)."""
    if side_stream:
        for t in tensors:
            t.record_stream(stream)


def _check_out(out, n, device):
    import torch
    if out.dtype != torch.float64 or out.device != device or not out.is_contiguous() or tuple(out.shape) != (n,):
        raise TypeError(f"out must be a contiguous float64 tensor of shape ({n},) on {device}")


def _check_momenta(momenta, n_ext):
    import torch
    if momenta.dtype != torch.float64 or not momenta.is_cuda:
        raise TypeError("momenta must be a float64 tensor on the GPU")
    if momenta.dim() != 3 or momenta.shape[1:] != (n_ext, 4):
        raise ValueError(f"momenta must have shape [N, {n_ext}, 4]")


class Process:
    """A process handle bound to the current HIP device."""

    def __init__(self, spec: str, precision: str = "fp64"):
        self.spec = spec
        self.precision = precision
        h = ctypes.c_void_p()
        _check(lib().heget_create_process(spec.encode(), PRECISIONS[precision], ctypes.byref(h)),
               f"heget_create_process({spec!r})")
        self._h = h
        n = [ctypes.c_int() for _ in range(4)]
        _check(lib().heget_process_info(h, *[ctypes.byref(x) for x in n]), "heget_process_info")
        self.n_ext, self.n_diagrams, self.n_colours, self.n_helicities = (x.value for x in n)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.heget_destroy_process(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def flops_per_event(self) -> int:
        f = ctypes.c_int64()
        _check(lib().heget_process_flops(self._h, ctypes.byref(f)), "heget_process_flops")
        return f.value

    def color_matrix(self):
        """(num, den, values) numpy arrays [K, K] of the exact colour matrix."""
        k = ctypes.c_int()
        _check(lib().heget_color_matrix(self._h, ctypes.byref(k), None, None, None), "heget_color_matrix")
        kk = k.value
        num = np.zeros(kk * kk, dtype=np.int64)
        den = np.zeros(kk * kk, dtype=np.int64)
        val = np.zeros(kk * kk, dtype=np.float64)
        _check(lib().heget_color_matrix(
            self._h, ctypes.byref(k),
            num.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            den.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            val.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "heget_color_matrix")
        return num.reshape(kk, kk), den.reshape(kk, kk), val.reshape(kk, kk)

    def matrix_elements_ptr(self, momenta_ptr: int, n_events: int, alpha_s: float, me2_ptr: int, stream: int = 0):
        """Raw call: device pointers as integers, stream as a hipStream_t integer."""
        _check(lib().heget_matrix_elements(self._h, ctypes.c_void_p(momenta_ptr), n_events, alpha_s,
                                           ctypes.c_void_p(me2_ptr), ctypes.c_void_p(stream)),
               "heget_matrix_elements")

    def matrix_elements(self, momenta, alpha_s: float, out=None, stream=None):
        """|M|^2 for a device tensor of momenta [N, n_ext, 4] float64 (torch, on the GPU)."""
        import torch
        _check_momenta(momenta, self.n_ext)
        momenta = momenta.contiguous()
        n = momenta.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        _check_out(out, n, momenta.device)
        stream, side = _launch_stream(momenta.device, stream)
        self.matrix_elements_ptr(momenta.data_ptr(), n, alpha_s, out.data_ptr(), stream.cuda_stream)
        _keep_alive(side, stream, momenta, out)
        return out

    def matrix_elements_helicity(self, momenta, helicity, alpha_s: float, out=None, stream=None):
        """One helicity term per event: helicity is an int32 device tensor [N] of bit patterns."""
        import torch
        _check_momenta(momenta, self.n_ext)
        if helicity.dtype != torch.int32 or not helicity.is_cuda or helicity.shape != momenta.shape[:1]:
            raise TypeError("helicity must be an int32 GPU tensor [N]")
        momenta, helicity = momenta.contiguous(), helicity.contiguous()
        n = momenta.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        _check_out(out, n, momenta.device)
        stream, side = _launch_stream(momenta.device, stream)
        _check(lib().heget_matrix_elements_helicity(self._h, ctypes.c_void_p(momenta.data_ptr()),
                                                    ctypes.c_void_p(helicity.data_ptr()), n, alpha_s,
                                                    ctypes.c_void_p(out.data_ptr()),
                                                    ctypes.c_void_p(stream.cuda_stream)),
               "heget_matrix_elements_helicity")
        _keep_alive(side, stream, momenta, helicity, out)
        return out

    def colour_reduction(self):
        """(M, W, slot_helicity): exact y = M J (Fractions, [K', K]), Q = y^H W y ([K', K']) and the
        helicity bit pattern of every evaluated configuration (the jamp slots of matrix_elements_hook)."""
        from fractions import Fraction
        kr, ns = ctypes.c_int(), ctypes.c_int()
        L = lib()
        _check(L.heget_colour_reduction(self._h, ctypes.byref(kr), ctypes.byref(ns), None, None, None, None, None),
               "heget_colour_reduction")
        k, kr, ns = self.n_colours, kr.value, ns.value
        mn, md = np.zeros(kr * k, np.int64), np.zeros(kr * k, np.int64)
        wn, wd = np.zeros(kr * kr, np.int64), np.zeros(kr * kr, np.int64)
        sh = np.zeros(ns, np.int32)
        p64 = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        _check(L.heget_colour_reduction(self._h, ctypes.byref(ctypes.c_int()), ctypes.byref(ctypes.c_int()),
                                        p64(mn), p64(md), p64(wn), p64(wd),
                                        sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
               "heget_colour_reduction")
        m = [[Fraction(int(mn[a * k + b]), int(md[a * k + b])) for b in range(k)] for a in range(kr)]
        w = [[Fraction(int(wn[a * kr + b]), int(wd[a * kr + b])) for b in range(kr)] for a in range(kr)]
        return m, w, sh

    def matrix_elements_hook(self, momenta, alpha_s: float, gauge_leg: int = -1, with_jamp: bool = False,
                             stream=None):
        """Test hook: (me2 [N], jamp [N, n_slots, K', 2] or None) through the test-hook kernels."""
        import torch
        _check_momenta(momenta, self.n_ext)
        momenta = momenta.contiguous()
        n = momenta.shape[0]
        out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        jamp = None
        if with_jamp:
            kr, ns = ctypes.c_int(), ctypes.c_int()
            _check(lib().heget_colour_reduction(self._h, ctypes.byref(kr), ctypes.byref(ns), None, None, None, None,
                                                None), "heget_colour_reduction")
            jamp = torch.empty((n, ns.value, kr.value, 2), dtype=torch.float64, device=momenta.device)
        stream, side = _launch_stream(momenta.device, stream)
        _check(lib().heget_matrix_elements_hook(self._h, ctypes.c_void_p(momenta.data_ptr()), n, alpha_s,
                                                gauge_leg, ctypes.c_void_p(out.data_ptr()),
                                                ctypes.c_void_p(None if jamp is None else jamp.data_ptr()),
                                                ctypes.c_void_p(stream.cuda_stream)),
               "heget_matrix_elements_hook")
        _keep_alive(side, stream, momenta, out, *([] if jamp is None else [jamp]))
        return out, jamp


def matrix_elements_batch(items, alpha_s: float, use_graph: bool = False, stream=None):
    """Fused uneven batch: items = [(Process, momenta tensor, out tensor), ...] on the GPU."""
    import torch
    arr = (BatchItem * len(items))()
    for i, (proc, mom, out) in enumerate(items):
        if mom.dtype != torch.float64 or not mom.is_cuda or not mom.is_contiguous():
            raise TypeError("momenta must be contiguous float64 GPU tensors")
        if mom.dim() != 3 or mom.shape[1:] != (proc.n_ext, 4):
            raise ValueError("bad momenta shape")
        _check_out(out, mom.shape[0], mom.device)
        arr[i] = BatchItem(proc.handle.value, mom.data_ptr(), mom.shape[0], out.data_ptr())
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().heget_matrix_elements_batch(arr, len(items), alpha_s, int(use_graph),
                                             ctypes.c_void_p(stream.cuda_stream)),
           "heget_matrix_elements_batch")


COLOUR_MODES = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp64_valu": 3}


def colour_quadratic_form(nmat, jamp, mode: str = "fp64", out=None, stream=None):
    """q_r = J_r N J_r^* for device tensors nmat [K, K] and jamp [R, 2, K] (float64)."""
    import torch
    if nmat.dtype != torch.float64 or jamp.dtype != torch.float64 or not (nmat.is_cuda and jamp.is_cuda):
        raise TypeError("float64 GPU tensors required")
    k = nmat.shape[0]
    if nmat.shape != (k, k) or jamp.dim() != 3 or jamp.shape[1:] != (2, k):
        raise ValueError("nmat must be [K, K] and jamp [R, 2, K]")
    nmat, jamp = nmat.contiguous(), jamp.contiguous()
    rows = jamp.shape[0]
    if out is None:
        out = torch.empty(rows, dtype=torch.float64, device=jamp.device)
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().heget_colour_quadratic_form(k, nmat.data_ptr(), jamp.data_ptr(), rows, COLOUR_MODES[mode],
                                             out.data_ptr(), ctypes.c_void_p(stream.cuda_stream)),
           "heget_colour_quadratic_form")
    return out


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_f64(t, shape, what):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise TypeError(f"{what} must be a contiguous float64 GPU tensor of shape {tuple(shape)}")


def rambo(sqrt_s, uniforms, stream=None):
    """Device RAMBO: sqrt_s [N], uniforms [N, n_final, 4] -> (momenta [N, n_final + 2, 4], weight [N])."""
    import torch
    n, nf = uniforms.shape[0], uniforms.shape[1]
    _dev_f64(sqrt_s, (n,), "sqrt_s")
    _dev_f64(uniforms, (n, nf, 4), "uniforms")
    mom = torch.empty((n, nf + 2, 4), dtype=torch.float64, device=uniforms.device)
    w = torch.empty(n, dtype=torch.float64, device=uniforms.device)
    _check(lib().heget_rambo(nf, n, sqrt_s.data_ptr(), uniforms.data_ptr(), mom.data_ptr(), w.data_ptr(),
                             _stream_ptr(stream)), "heget_rambo")
    return mom, w


def apply_cuts(momenta, pt_min: float, eta_max: float, delta_r_min: float, stream=None):
    """uint8 [N] pass flags of the jet cuts for momenta [N, n_ext, 4] on the GPU."""
    import torch
    n, n_ext = momenta.shape[0], momenta.shape[1]
    _dev_f64(momenta, (n, n_ext, 4), "momenta")
    out = torch.empty(n, dtype=torch.uint8, device=momenta.device)
    cuts = Cuts(pt_min, eta_max, delta_r_min)
    _check(lib().heget_apply_cuts(n_ext, n, momenta.data_ptr(), ctypes.byref(cuts), out.data_ptr(),
                                  _stream_ptr(stream)), "heget_apply_cuts")
    return out


def integrate_step(proc: Process, sqrt_s, uniforms, alpha_s: float, pt_min: float, eta_max: float,
                   delta_r_min: float, helicity=None, stream=None, out=None, noalloc: bool = False):
    """One device integration step; returns (momenta, me2, weight, sums[2]) GPU tensors.

    out: optional tuple of preallocated (momenta, me2, weight, sums) tensors to write.
    noalloc: call heget_integrate_step_noalloc (no device allocation inside the library)."""
    import torch
    n = uniforms.shape[0]
    _dev_f64(sqrt_s, (n,), "sqrt_s")
    _dev_f64(uniforms, (n, proc.n_ext - 2, 4), "uniforms")
    if helicity is not None and (helicity.dtype != torch.int32 or not helicity.is_cuda or helicity.shape != (n,)):
        raise TypeError("helicity must be an int32 GPU tensor [N]")
    dev = uniforms.device
    if out is None:
        mom = torch.empty((n, proc.n_ext, 4), dtype=torch.float64, device=dev)
        me2 = torch.empty(n, dtype=torch.float64, device=dev)
        w = torch.empty(n, dtype=torch.float64, device=dev)
        sums = torch.empty(2, dtype=torch.float64, device=dev)
    else:
        mom, me2, w, sums = out
        _dev_f64(mom, (n, proc.n_ext, 4), "momenta")
        _dev_f64(me2, (n,), "me2")
        _dev_f64(w, (n,), "weight")
        _dev_f64(sums, (2,), "sums")
    cuts = Cuts(pt_min, eta_max, delta_r_min)
    fn = lib().heget_integrate_step_noalloc if noalloc else lib().heget_integrate_step
    _check(fn(proc.handle, n, sqrt_s.data_ptr(), uniforms.data_ptr(),
              None if helicity is None else helicity.data_ptr(), alpha_s,
              ctypes.byref(cuts), mom.data_ptr(), me2.data_ptr(), w.data_ptr(),
              sums.data_ptr(), _stream_ptr(stream)),
           "heget_integrate_step_noalloc" if noalloc else "heget_integrate_step")
    return mom, me2, w, sums
