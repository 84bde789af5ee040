"""ctypes binding of libcsngf.so: the C ABI of include/csngf.h and include/csngf_debug.h.

Argument marshalling only - every step of the hot path runs in the HIP library.  Arrays may
be numpy arrays (host memory) or torch CUDA tensors (device memory, passed by pointer with
CSNGF_DEVICE_PTRS).  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcsngf.so")

OK = 0
E_INVALID_ARG = -1
E_UNSUPPORTED = -2
E_NO_DEVICE = -3
E_OUT_OF_MEMORY = -4
E_DEVICE = -5
E_NO_VALID_SHIFT = -6
DEVICE_PTRS = 1
UNSQUARED = 2
GRAPHS = 4
FP64 = 8

_NAMES = {0: "OK", -1: "E_INVALID_ARG", -2: "E_UNSUPPORTED", -3: "E_NO_DEVICE", -4: "E_OUT_OF_MEMORY",
          -5: "E_DEVICE", -6: "E_NO_VALID_SHIFT"}


class Dims(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("eps", C.c_float), ("gamma", C.c_double),
                ("pad", C.c_int32 * 3), ("batch", C.c_int32), ("flags", C.c_uint32),
                ("slices", C.c_int32), ("final_groups", C.c_int32), ("reserved", C.c_int32)]


class RotResult(C.Structure):
    _fields_ = [("score", C.c_float), ("shift", C.c_int32 * 3), ("overlap", C.c_int64),
                ("valid", C.c_int32), ("reserved", C.c_int32)]


class Best(C.Structure):
    _fields_ = [("score", C.c_float), ("rot_index", C.c_int32), ("shift", C.c_int32 * 3),
                ("reserved", C.c_int32), ("overlap", C.c_int64), ("R", C.c_double * 9)]


class Info(C.Structure):
    _fields_ = [("pad", C.c_int32 * 3), ("batch", C.c_int32), ("map_dims", C.c_int32 * 3),
                ("reserved", C.c_int32), ("count_a", C.c_int64), ("spectra_bytes", C.c_int64),
                ("workspace_bytes", C.c_int64)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


# name -> (restype, argtypes); this list is also what the CPU tests check is exported
SIGNATURES = {
    "csngf_default_params": (C.c_int, [C.POINTER(Params)]),
    "csngf_supported_length": (C.c_int, [C.c_int32]),
    "csngf_create": (C.c_int, [C.c_void_p, Dims, C.c_void_p, Dims, C.POINTER(Params), C.POINTER(C.c_void_p)]),
    "csngf_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "csngf_get_info": (C.c_int, [C.c_void_p, C.POINTER(Info)]),
    "csngf_evaluate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                 C.POINTER(RotResult), C.POINTER(Best)]),
    "csngf_evaluate_map": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "csngf_evaluate_async": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]),
    "csngf_query": (C.c_int, [C.c_void_p]),
    "csngf_wait": (C.c_int, [C.c_void_p, C.POINTER(RotResult), C.POINTER(Best)]),
    "csngf_autotune": (C.c_int, [C.c_void_p, Dims, C.c_void_p, Dims, C.POINTER(Params), C.c_int32,
                                 C.POINTER(Params), C.POINTER(C.c_double)]),
    "csngf_footprint": (C.c_int, [Dims, Dims, C.POINTER(Params), C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int32)]),
    "csngf_destroy": (C.c_int, [C.c_void_p]),
    "csngf_last_error": (C.c_char_p, []),
    "csngf_debug_fft": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "csngf_debug_fields": (C.c_int, [C.c_void_p, C.c_void_p, Dims, C.c_void_p, C.c_float, C.c_int32,
                                     C.c_void_p, C.c_void_p, C.c_uint32]),
    "csngf_smooth_downsample": (C.c_int, [C.c_void_p, Dims, C.c_float, C.c_int32, C.c_void_p, C.POINTER(Dims),
                                          C.c_uint32, C.c_void_p]),
    "csngf_smooth_downsample_noalloc": (C.c_int, [C.c_void_p, Dims, C.c_float, C.c_int32, C.c_void_p,
                                                  C.POINTER(Dims), C.c_void_p]),
    "csngf_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "csngf_profile_read": (C.c_int, [C.c_void_p, C.POINTER(KernelStat), C.c_int32, C.POINTER(C.c_int32)]),
    "csngf_profile_reset": (C.c_int, [C.c_void_p]),
    "csngf_profile_rows": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int64)]),
}

_lib = None


def lib():
    """Load libcsngf.so (raises if it has not been built; there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2110_10156_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class CsngfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise CsngfError(rc, lib().csngf_last_error().decode())
    return rc


def _ptr(a):
    """Data pointer of a numpy array or a torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _is_device(a):
    return a is not None and not isinstance(a, np.ndarray) and getattr(a, "is_cuda", False)


def dims_of(vol) -> Dims:
    nz, ny, nx = vol.shape
    return Dims(nx, ny, nz)


def default_params() -> Params:
    p = Params()
    _check(lib().csngf_default_params(C.byref(p)))
    return p


def supported_length(L: int) -> bool:
    return bool(lib().csngf_supported_length(L))


class Context:
    """Owns a csngf_ctx: A's resident spectra and the rotation workspaces."""

    def __init__(self, A, dims_b, *, mask_a=None, eps=1e-5, gamma=0.5, pad=(0, 0, 0), batch=0, stream=None,
                 measure="squared", graphs=False, fp64=False, slices=0, final_groups=0):
        """measure: "squared" (Eq. (2), CSNGF) or "unsquared" (Eq. (3), USNGF); graphs: replay
        each full batch from a recorded HIP graph; fp64: correlate in double precision
        (CSNGF_FP64); slices, final_groups: launch shapes (0 = automatic), as autotune returns."""
        if measure not in ("squared", "unsquared"):
            raise ValueError(f"unknown measure {measure!r}")
        self.device = _is_device(A)
        if not self.device:
            A = np.ascontiguousarray(A, dtype=np.float32)
            if mask_a is not None:
                mask_a = np.ascontiguousarray(mask_a, dtype=np.uint8)
        p = default_params()
        p.eps = eps
        p.gamma = gamma
        p.pad[:] = list(pad)
        p.batch = batch
        p.slices = slices
        p.final_groups = final_groups
        p.flags = ((DEVICE_PTRS if self.device else 0) | (UNSQUARED if measure == "unsquared" else 0)
                   | (GRAPHS if graphs else 0) | (FP64 if fp64 else 0))
        h = C.c_void_p()
        if isinstance(dims_b, tuple):
            dims_b = Dims(*dims_b)
        self._A = A
        _check(lib().csngf_create(_ptr(A), dims_of(A), _ptr(mask_a), dims_b, C.byref(p), C.byref(h)))
        self.h = h
        if stream is not None:
            self.set_stream(stream)

    def set_stream(self, stream):
        s = stream if isinstance(stream, int) else getattr(stream, "cuda_stream", stream)
        _check(lib().csngf_set_stream(self.h, C.c_void_p(s)))

    def info(self) -> Info:
        i = Info()
        _check(lib().csngf_get_info(self.h, C.byref(i)))
        return i

    def _b(self, B, mask_b):
        if self.device:
            return B, mask_b
        B = np.ascontiguousarray(B, dtype=np.float32)
        if mask_b is not None:
            mask_b = np.ascontiguousarray(mask_b, dtype=np.uint8)
        return B, mask_b

    def evaluate(self, B, rotations, mask_b=None, allow_no_valid=True):
        """Returns (per-rotation RotResult array, Best)."""
        B, mask_b = self._b(B, mask_b)
        R = np.ascontiguousarray(np.asarray(rotations, dtype=np.float64).reshape(-1, 9))
        n = R.shape[0]
        per = (RotResult * max(n, 1))()
        best = Best()
        rc = lib().csngf_evaluate(self.h, _ptr(B), _ptr(mask_b), R.ctypes.data if n else None, n, per,
                                  C.byref(best))
        if rc != OK and not (allow_no_valid and rc == E_NO_VALID_SHIFT):
            _check(rc)
        return per[:n], best

    def evaluate_async(self, B, rotations, mask_b=None):
        """Enqueue an evaluation; keep B alive and call wait() for the results."""
        B, mask_b = self._b(B, mask_b)
        R = np.ascontiguousarray(np.asarray(rotations, dtype=np.float64).reshape(-1, 9))
        self._inflight = (B, mask_b, R)
        _check(lib().csngf_evaluate_async(self.h, _ptr(B), _ptr(mask_b), R.ctypes.data if len(R) else None, len(R)))

    def done(self):
        return bool(_check_query(lib().csngf_query(self.h)))

    def wait(self, allow_no_valid=True):
        n = len(self._inflight[2]) if getattr(self, "_inflight", None) is not None else 0
        per = (RotResult * max(n, 1))()
        best = Best()
        rc = lib().csngf_wait(self.h, per, C.byref(best))
        self._inflight = None
        if rc != OK and not (allow_no_valid and rc == E_NO_VALID_SHIFT):
            _check(rc)
        return per[:n], best

    def evaluate_map(self, B, R, mask_b=None, with_overlap=True, out=None):
        """Full C map (-inf invalid) and N map for one rotation.  Host context: numpy arrays.
        Device context: written into ``out=(C, N)`` (float32 and int64 device tensors of the map
        shape, stream-ordered on the context's stream); without ``out`` they are allocated on
        B's device and the device is synchronised before they are returned."""
        B, mask_b = self._b(B, mask_b)
        R = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(9))
        i = self.info()
        W = (i.map_dims[2], i.map_dims[1], i.map_dims[0])
        if self.device:
            if out is None:
                import torch
                Cm = torch.empty(W, dtype=torch.float32, device=B.device)
                Nm = torch.empty(W, dtype=torch.int64, device=B.device) if with_overlap else None
                # the blocks belong to torch's current stream, where earlier work may still read
                # them; the library writes them on the context's stream, so let that work finish
                torch.cuda.current_stream(B.device).synchronize()
            else:
                Cm, Nm = out
            _check(lib().csngf_evaluate_map(self.h, _ptr(B), _ptr(mask_b), R.ctypes.data, _ptr(Cm), _ptr(Nm)))
            if out is None:
                torch.cuda.synchronize(B.device)
            return Cm, Nm
        Cm = np.empty(W, dtype=np.float32)
        Nm = np.empty(W, dtype=np.int64) if with_overlap else None
        _check(lib().csngf_evaluate_map(self.h, _ptr(B), _ptr(mask_b), R.ctypes.data, _ptr(Cm), _ptr(Nm)))
        return Cm, Nm

    def profile_enable(self, on=True):
        _check(lib().csngf_profile_enable(self.h, 1 if on else 0))

    def profile_reset(self):
        _check(lib().csngf_profile_reset(self.h))

    def profile_read(self):
        stats = (KernelStat * 16)()
        cnt = C.c_int32()
        _check(lib().csngf_profile_read(self.h, stats, 16, C.byref(cnt)))
        return {stats[i].name.decode(): (stats[i].launches, stats[i].total_ms) for i in range(min(cnt.value, 16))}

    def profile_rows(self):
        """(kept z-rows, kept rows, rotations) counted while profiling (minimum-overlap pruning)."""
        z, r, n = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().csngf_profile_rows(self.h, C.byref(z), C.byref(r), C.byref(n)))
        return z.value, r.value, n.value

    def close(self):
        if getattr(self, "h", None):
            lib().csngf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _check_query(rc):
    if rc < 0:
        _check(rc)
    return rc


def autotune(A, B, *, n_probe=64, measure="squared", gamma=0.5, eps=1e-5, graphs=False):
    """Fastest configuration for this pair's shapes; returns (dict(pad=..., batch=..., slices=...,
    final_groups=...), rotations/s), the dict's keys being Context keywords."""
    dev = _is_device(A)
    if not dev:
        A = np.ascontiguousarray(A, dtype=np.float32)
        B = np.ascontiguousarray(B, dtype=np.float32)
    p = default_params()
    p.eps, p.gamma = eps, gamma
    p.flags = ((DEVICE_PTRS if dev else 0) | (UNSQUARED if measure == "unsquared" else 0)
               | (GRAPHS if graphs else 0))
    out = Params()
    rate = C.c_double()
    _check(lib().csngf_autotune(_ptr(A), dims_of(A), _ptr(B), dims_of(B), C.byref(p), n_probe, C.byref(out),
                                C.byref(rate)))
    return ({"pad": tuple(out.pad), "batch": out.batch, "slices": out.slices, "final_groups": out.final_groups},
            rate.value)


def footprint(dims_a, dims_b, *, pad=(0, 0, 0), measure="squared"):
    """(spectra bytes, workspace bytes per rotation slot, FFT size) of a context, without allocating."""
    p = default_params()
    p.pad[:] = list(pad)
    p.flags = UNSQUARED if measure == "unsquared" else 0
    sb, wb = C.c_int64(), C.c_int64()
    P = (C.c_int32 * 3)()
    da = dims_a if isinstance(dims_a, Dims) else Dims(*dims_a)
    db = dims_b if isinstance(dims_b, Dims) else Dims(*dims_b)
    _check(lib().csngf_footprint(da, db, C.byref(p), C.byref(sb), C.byref(wb), P))
    return sb.value, wb.value, tuple(P)


def debug_fft(x_dev, inverse=False, out=None, stream=None):
    """Batched FFT along the last axis of a complex64 CUDA tensor [batch, L]."""
    batch, L = x_dev.shape
    out = x_dev if out is None else out
    _check(lib().csngf_debug_fft(_ptr(x_dev), _ptr(out), L, batch, 1 if inverse else 0, stream))
    return out


def debug_fields(vol, R=None, mask=None, eps=1e-5, Px=0, unsquared=False):
    """Separable fields (6 products, or the 3 NGF components with unsquared=True) as
    float32 (k, nz, ny, nx) and the eroded mask (nz, ny, nx) uint8 of the field stage."""
    vol = np.ascontiguousarray(vol, dtype=np.float32)
    prod = np.empty((3 if unsquared else 6,) + vol.shape, dtype=np.float32)
    m = np.empty(vol.shape, dtype=np.uint8)
    Rp = None
    if R is not None:
        Rr = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(9))
        Rp = Rr.ctypes.data
    mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    _check(lib().csngf_debug_fields(_ptr(vol), _ptr(mk), dims_of(vol), Rp, eps, Px, _ptr(prod), _ptr(m),
                                    UNSQUARED if unsquared else 0))
    return prod, m


def smooth_downsample(vol, sigma, factor, stream=None):
    """Gaussian blur (sigma voxels) then keep every factor-th voxel: numpy in -> numpy out,
    CUDA tensor in -> CUDA tensor out (on the given stream, else the current one)."""
    dev = _is_device(vol)
    if not dev:
        vol = np.ascontiguousarray(vol, dtype=np.float32)
    od = Dims()
    _check(lib().csngf_smooth_downsample(_ptr(vol), dims_of(vol), float(sigma), int(factor), None, C.byref(od),
                                         DEVICE_PTRS if dev else 0, None))
    shape = (od.nz, od.ny, od.nx)
    if dev:
        import torch
        out = torch.empty(shape, dtype=torch.float32, device=vol.device)
        s = stream if stream is not None else torch.cuda.current_stream(vol.device)
        _check(lib().csngf_smooth_downsample(_ptr(vol), dims_of(vol), float(sigma), int(factor), _ptr(out),
                                             C.byref(od), DEVICE_PTRS, C.c_void_p(s.cuda_stream)))
        return out
    out = np.empty(shape, dtype=np.float32)
    _check(lib().csngf_smooth_downsample(_ptr(vol), dims_of(vol), float(sigma), int(factor), _ptr(out), C.byref(od),
                                         0, None))
    return out


NOALLOC_SCRATCH_BYTES = 32 << 20


def smooth_downsample_noalloc(vol, sigma, factor, out=None, stream=None):
    """csngf_smooth_downsample_noalloc on a CUDA tensor: the library allocates nothing (its
    intermediates sit in a fixed per-device scratch array).  ``out`` (float32, the output
    shape) is allocated here by torch when omitted; the blur is enqueued on ``stream`` (else
    the current stream) and not synchronised."""
    import torch
    od = Dims()
    _check(lib().csngf_smooth_downsample_noalloc(_ptr(vol), dims_of(vol), float(sigma), int(factor), None,
                                                 C.byref(od), None))
    shape = (od.nz, od.ny, od.nx)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=vol.device)
    assert tuple(out.shape) == shape and out.dtype == torch.float32 and out.is_contiguous()
    s = stream if stream is not None else torch.cuda.current_stream(vol.device)
    _check(lib().csngf_smooth_downsample_noalloc(_ptr(vol), dims_of(vol), float(sigma), int(factor), _ptr(out),
                                                 C.byref(od), C.c_void_p(s.cuda_stream)))
    return out
