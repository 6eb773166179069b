"""Thin ctypes binding of libtvs (include/tvs.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Arrays are torch tensors on the GPU (float32 or float64,
contiguous); PyTorch provides device memory and streams.  If the library is
not built this module raises on import of the library, never falling back to
any other implementation.
"""
import ctypes
import os

import numpy as np

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtvs.so")

TVS_F32, TVS_F64 = 0, 1
TVS_OK, TVS_EINVAL, TVS_ENOMEM, TVS_EHIP, TVS_ENONFINITE, TVS_EBUSY = 0, -1, -2, -3, -4, -5
TVS_IRV2, TVS_IRV1 = 0, 1
TVS_LP_IMAGE, TVS_LP_BLOCKDCT = 0, 1


class Params(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("alpha", ctypes.c_double), ("t", ctypes.c_double),
                ("h", ctypes.c_double), ("eps", ctypes.c_double), ("variant", ctypes.c_int)]


class Layout(ctypes.Structure):
    _fields_ = [("M2", ctypes.c_int), ("M1", ctypes.c_int), ("s_y", ctypes.c_int),
                ("s_x", ctypes.c_int), ("alpha_hat", ctypes.c_double)]


class Iters(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int), ("inner", ctypes.c_int), ("tol", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("sweeps_done", ctypes.c_int), ("energy", ctypes.c_double),
                ("gap", ctypes.c_double), ("residual", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TvsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtvs error {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libtvs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.tvs_ctx_create.argtypes = [ci, ctypes.POINTER(vp)]
    lib.tvs_ctx_create.restype = ci
    lib.tvs_ctx_destroy.argtypes = [vp]
    lib.tvs_ctx_destroy.restype = None
    lib.tvs_last_error.argtypes = []
    lib.tvs_last_error.restype = ctypes.c_char_p
    lib.tvs_ctx_bytes.argtypes = [vp]
    lib.tvs_ctx_bytes.restype = ctypes.c_size_t
    P, L, I, S = (ctypes.POINTER(Params), ctypes.POINTER(Layout), ctypes.POINTER(Iters),
                  ctypes.POINTER(Stats))
    lib.tvs_step1.argtypes = [vp, vp, ci, ci, ci, P, L, I, vp, S, vp]
    lib.tvs_step1.restype = ci
    lib.tvs_step2.argtypes = [vp, vp, vp, ci, ci, ci, P, L, I, vp, S, vp]
    lib.tvs_step2.restype = ci
    lib.tvs_schwarz_solve.argtypes = [vp, vp, ci, ci, ci, P, L, I, vp, vp, S, vp]
    lib.tvs_schwarz_solve.restype = ci
    lib.tvs_project_div_free.argtypes = [vp, vp, ci, ci, ci, cd, vp, vp]
    lib.tvs_project_div_free.restype = ci
    lib.tvs_timing_enable.argtypes = [vp, ci]
    lib.tvs_timing_enable.restype = ci
    lib.tvs_timing_reset.argtypes = [vp]
    lib.tvs_timing_reset.restype = ci
    lib.tvs_timing_count.argtypes = [vp]
    lib.tvs_timing_count.restype = ci
    lib.tvs_timing_get.argtypes = [vp, ci, ctypes.c_char_p, ci, ctypes.POINTER(ctypes.c_longlong),
                                   ctypes.POINTER(cd), ctypes.POINTER(cd)]
    lib.tvs_timing_get.restype = ci
    sz = ctypes.c_size_t
    lib.tvs_job_footprint.argtypes = [ci, ci, ci, L, I, ctypes.POINTER(sz)]
    lib.tvs_job_footprint.restype = ci
    lib.tvs_job_create.argtypes = [vp, vp, ci, ci, ci, P, L, I, vp, ctypes.POINTER(vp)]
    lib.tvs_job_create.restype = ci
    lib.tvs_batch_sweep.argtypes = [vp, ctypes.POINTER(vp), ci, vp]
    lib.tvs_batch_sweep.restype = ci
    lib.tvs_job_status.argtypes = [vp, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.POINTER(ci)]
    lib.tvs_job_status.restype = ci
    lib.tvs_job_result.argtypes = [vp, vp, vp, vp, S, vp]
    lib.tvs_job_result.restype = ci
    lib.tvs_job_bytes.argtypes = [vp]
    lib.tvs_job_bytes.restype = sz
    lib.tvs_job_export_state.argtypes = [vp, vp, vp, sz, ctypes.POINTER(sz), vp]
    lib.tvs_job_export_state.restype = ci
    lib.tvs_job_import_state.argtypes = [vp, vp, sz, vp, ctypes.POINTER(vp)]
    lib.tvs_job_import_state.restype = ci
    lib.tvs_energy_history.argtypes = [vp, ctypes.POINTER(cd), ci, ctypes.POINTER(ci)]
    lib.tvs_energy_history.restype = ci
    lib.tvs_set_local_projection.argtypes = [vp, ci]
    lib.tvs_set_local_projection.restype = ci
    lib.tvs_set_block_groups.argtypes = [vp, ci, ci]
    lib.tvs_set_block_groups.restype = ci
    lib.tvs_tangent_field.argtypes = [vp, vp, ci, ci, ci, cd, vp, vp]
    lib.tvs_tangent_field.restype = ci
    lib.tvs_quality.argtypes = [vp, vp, vp, ci, ci, ci, ctypes.POINTER(cd), vp]
    lib.tvs_quality.restype = ci
    lib.tvs_set_tiles.argtypes = [vp, ci, ci, ci, ci, ci]
    lib.tvs_set_tiles.restype = ci
    lib.tvs_get_tiles.argtypes = [vp, ci, ci, ci, L, cd, ctypes.POINTER(ci)]
    lib.tvs_get_tiles.restype = ci
    lib.tvs_quality_noalloc.argtypes = [vp, vp, vp, ci, ci, ci, ctypes.POINTER(cd), vp]
    lib.tvs_quality_noalloc.restype = ci
    lib.tvs_job_destroy.argtypes = [vp]
    lib.tvs_job_destroy.restype = ci
    _lib = lib
    return lib


EXPORTED = ["tvs_ctx_create", "tvs_ctx_destroy", "tvs_last_error", "tvs_ctx_bytes", "tvs_step1",
            "tvs_step2", "tvs_schwarz_solve", "tvs_project_div_free", "tvs_timing_enable",
            "tvs_timing_reset", "tvs_timing_count", "tvs_timing_get", "tvs_job_footprint",
            "tvs_job_create", "tvs_batch_sweep", "tvs_job_status", "tvs_job_result",
            "tvs_job_bytes", "tvs_job_destroy", "tvs_job_export_state", "tvs_job_import_state",
            "tvs_tangent_field", "tvs_quality", "tvs_quality_noalloc", "tvs_set_local_projection",
            "tvs_set_block_groups", "tvs_set_tiles", "tvs_get_tiles",
            "tvs_energy_history"]


def _check(code):
    if code != 0:
        raise TvsError(code, load().tvs_last_error().decode())


def _dtype_code(t):
    if t.dtype == torch.float32:
        return TVS_F32
    if t.dtype == torch.float64:
        return TVS_F64
    raise TypeError("tensors must be float32 or float64")


def _dev(t, shape, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("all tensors must share one dtype")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_params(delta, alpha, t=0.125, h=1.0, eps=1e-3, variant=TVS_IRV2):
    return Params(float(delta), float(alpha), float(t), float(h), float(eps), int(variant))


def make_layout(m2=1, m1=1, s_y=0, s_x=0, alpha_hat=0.0):
    return Layout(int(m2), int(m1), int(s_y), int(s_x), float(alpha_hat))


def make_iters(sweeps, inner, tol=0.0):
    return Iters(int(sweeps), int(inner), float(tol))


class Context:
    """A libtvs context on one GPU (caches plans and work buffers)."""

    def __init__(self, device=0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.tvs_ctx_create(int(device), ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", int(device))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().tvs_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def bytes(self):
        return int(load().tvs_ctx_bytes(self._h))

    def synchronize(self):
        """Wait for the work enqueued on the device's current stream."""
        torch.cuda.current_stream(self.device).synchronize()

    def step1(self, d0, params, layout, iters, tau_out=None, stats=True):
        n2, n1 = d0.shape
        if tau_out is None:
            tau_out = torch.empty((2, n2 + 1, n1 + 1), dtype=d0.dtype, device=d0.device)
        st = Stats()
        _check(load().tvs_step1(self._h, _dev(d0, (n2, n1)), n2, n1, _dtype_code(d0),
                                ctypes.byref(params), ctypes.byref(layout), ctypes.byref(iters),
                                _dev(tau_out, (2, n2 + 1, n1 + 1), d0.dtype),
                                ctypes.byref(st) if stats else None, _stream(d0.device)))
        return tau_out, (st.as_dict() if stats else None)

    def step2(self, d0, tau, params, layout, iters, d_out=None, stats=True):
        n2, n1 = d0.shape
        if d_out is None:
            d_out = torch.empty_like(d0)
        st = Stats()
        _check(load().tvs_step2(self._h, _dev(d0, (n2, n1)), _dev(tau, (2, n2 + 1, n1 + 1), d0.dtype),
                                n2, n1, _dtype_code(d0), ctypes.byref(params), ctypes.byref(layout),
                                ctypes.byref(iters), _dev(d_out, (n2, n1), d0.dtype),
                                ctypes.byref(st) if stats else None, _stream(d0.device)))
        return d_out, (st.as_dict() if stats else None)

    def schwarz_solve(self, d0, params, layout, iters, d_out=None, tau_out=None, stats=True):
        n2, n1 = d0.shape
        if d_out is None:
            d_out = torch.empty_like(d0)
        st = (Stats * 2)()
        tau_p = None if tau_out is None else _dev(tau_out, (2, n2 + 1, n1 + 1), d0.dtype)
        _check(load().tvs_schwarz_solve(self._h, _dev(d0, (n2, n1)), n2, n1, _dtype_code(d0),
                                        ctypes.byref(params), ctypes.byref(layout),
                                        ctypes.byref(iters), _dev(d_out, (n2, n1), d0.dtype),
                                        tau_p, st if stats else None, _stream(d0.device)))
        return d_out, ([st[0].as_dict(), st[1].as_dict()] if stats else None)

    def timing(self, enable=True, every=1):
        """Switch kernel timing on or off (HIP events around one in `every`
        launches of each instrumented kernel class)."""
        if every < 1:
            raise ValueError("every must be >= 1")
        _check(load().tvs_timing_enable(self._h, int(every) if enable else 0))

    def timing_reset(self):
        _check(load().tvs_timing_reset(self._h))

    def timing_read(self):
        """{kernel class: (launches, total ms, total algorithmic bytes)}"""
        lib = load()
        n = lib.tvs_timing_count(self._h)
        if n < 0:
            _check(n)
        out = {}
        buf = ctypes.create_string_buffer(128)
        for i in range(n):
            la, ms, by = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
            _check(lib.tvs_timing_get(self._h, i, buf, 128, ctypes.byref(la), ctypes.byref(ms),
                                      ctypes.byref(by)))
            out[buf.value.decode()] = (la.value, ms.value, by.value)
        return out

    # -- jobs (resident state, one Schwarz sweep per batch call) -------------
    def job(self, d0, params, layout, iters):
        """Create a job solving d0 (a GPU tensor, copied) with both steps."""
        n2, n1 = d0.shape
        h = ctypes.c_void_p()
        _check(load().tvs_job_create(self._h, _dev(d0, (n2, n1)), n2, n1, _dtype_code(d0),
                                     ctypes.byref(params), ctypes.byref(layout), ctypes.byref(iters),
                                     _stream(d0.device), ctypes.byref(h)))
        return Job(self, h, n2, n1, d0.dtype)

    def import_job(self, state):
        """A job resumed from a blob of Job.export_state (bytes or a uint8
        array); its dtype and shape are the blob's."""
        buf = np.ascontiguousarray(np.frombuffer(state, dtype=np.uint8))
        h = ctypes.c_void_p()
        _check(load().tvs_job_import_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size,
                                           _stream(self.device), ctypes.byref(h)))
        # header: magic[8], u32 version, u32 header bytes, u64 total, i32 dtype, N2, N1
        code, n2, n1 = (int(x) for x in buf[24:36].view(np.int32))
        return Job(self, h, n2, n1, torch.float64 if code == TVS_F64 else torch.float32)

    def batch_sweep(self, jobs):
        """Advance every job in the list by one sweep of its current step."""
        arr = (ctypes.c_void_p * max(1, len(jobs)))(*[j._h.value for j in jobs])
        _check(load().tvs_batch_sweep(self._h, arr, len(jobs), _stream(self.device)))

    def energy_history(self):
        """FP64 dual energies per Schwarz sweep of the last one-shot step run
        with statistics on this context (a list)."""
        n = ctypes.c_int()
        _check(load().tvs_energy_history(self._h, None, 0, ctypes.byref(n)))
        out = (ctypes.c_double * max(1, n.value))()
        _check(load().tvs_energy_history(self._h, out, n.value, ctypes.byref(n)))
        return list(out[:n.value])

    def set_local_projection(self, kind):
        """TVS_LP_IMAGE (default) or TVS_LP_BLOCKDCT for the later one-shot
        Step-1 calls of this context."""
        _check(load().tvs_set_local_projection(self._h, int(kind)))

    def set_block_groups(self, g2=0, g1=0):
        """Frequency blocks per group (rows, columns) of the block-DCT plans
        built later in this context; 0 chooses automatically."""
        _check(load().tvs_set_block_groups(self._h, int(g2), int(g1)))

    def tangent_field(self, d, h=1.0, out=None):
        """tau_0 = (-D_y d, D_x d) with Neumann differences, 2 x (N2+1) x (N1+1)."""
        n2, n1 = d.shape
        if out is None:
            out = torch.empty((2, n2 + 1, n1 + 1), dtype=d.dtype, device=d.device)
        _check(load().tvs_tangent_field(self._h, _dev(d, (n2, n1)), n2, n1, _dtype_code(d), float(h),
                                        _dev(out, (2, n2 + 1, n1 + 1), d.dtype), _stream(d.device)))
        return out

    def quality(self, x, ref):
        """{"psnr", "mssim", "mse"} of x against ref (same shape and dtype)."""
        if x.dim() != 2:
            raise ValueError("expected a 2-D array")
        if x.shape != ref.shape:
            raise ValueError("x and ref must have the same shape")
        n2, n1 = x.shape
        out = (ctypes.c_double * 3)()
        _check(load().tvs_quality(self._h, _dev(x, (n2, n1)), _dev(ref, (n2, n1), x.dtype), n2, n1,
                                  _dtype_code(x), out, _stream(x.device)))
        return {"psnr": out[0], "mssim": out[1], "mse": out[2]}

    def set_tiles(self, run1=0, run1d=0, rows=0, cols=0, run2=0):
        """Force workgroup shapes for later calls and jobs (0 = the tuner's)."""
        _check(load().tvs_set_tiles(self._h, int(run1), int(run1d), int(rows), int(cols), int(run2)))

    def get_tiles(self, shape, dtype, layout, h=1.0):
        """The tuner's (run1, run1d, rows, cols, run2) for a problem shape,
        zeros if not tuned yet."""
        out = (ctypes.c_int * 5)()
        code = TVS_F32 if dtype == torch.float32 else TVS_F64
        _check(load().tvs_get_tiles(self._h, int(shape[0]), int(shape[1]), code, ctypes.byref(layout),
                                    float(h), out))
        return tuple(out)

    def quality_noalloc(self, x, ref):
        """As quality(), through tvs_quality_noalloc: the library allocates
        no device memory for it (its scratch is a static per-GPU array, shared
        by all calls on that GPU)."""
        if x.dim() != 2:
            raise ValueError("expected a 2-D array")
        if x.shape != ref.shape:
            raise ValueError("x and ref must have the same shape")
        n2, n1 = x.shape
        out = (ctypes.c_double * 3)()
        _check(load().tvs_quality_noalloc(self._h, _dev(x, (n2, n1)), _dev(ref, (n2, n1), x.dtype), n2, n1,
                                          _dtype_code(x), out, _stream(x.device)))
        return {"psnr": out[0], "mssim": out[1], "mse": out[2]}

    def project_div_free(self, u, h=1.0, out=None):
        _, n2, n1 = u.shape
        if out is None:
            out = torch.empty_like(u)
        _check(load().tvs_project_div_free(self._h, _dev(u, (2, n2, n1)), n2, n1, _dtype_code(u),
                                           float(h), _dev(out, (2, n2, n1), u.dtype),
                                           _stream(u.device)))
        return out


def job_footprint(shape, dtype, layout, iters):
    """Device bytes a job of this image shape needs (host-side estimate that
    equals the job's allocation plus its grid's Green-function table)."""
    n2, n1 = shape
    code = TVS_F32 if dtype == torch.float32 else TVS_F64 if dtype == torch.float64 else None
    if code is None:
        raise TypeError("dtype must be float32 or float64")
    out = ctypes.c_size_t()
    _check(load().tvs_job_footprint(int(n2), int(n1), code, ctypes.byref(layout), ctypes.byref(iters),
                                    ctypes.byref(out)))
    return int(out.value)


class Job:
    """One image's solve with resident device state (see tvs_job_* in tvs.h)."""

    def __init__(self, ctx, handle, n2, n1, dtype):
        self.ctx, self._h, self.shape, self.dtype = ctx, handle, (n2, n1), dtype

    def status(self):
        """(step, sweeps done in it, finished); step is -1 for a job that
        failed (non-finite statistics), which also counts as finished."""
        st, sw, dn = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(load().tvs_job_status(self._h, ctypes.byref(st), ctypes.byref(sw), ctypes.byref(dn)))
        return st.value, sw.value, bool(dn.value)

    @property
    def done(self):
        return self.status()[2]

    @property
    def failed(self):
        return self.status()[0] == -1

    def bytes(self):
        return int(load().tvs_job_bytes(self._h))

    def result(self, d_out=None, tau_out=None):
        """(d, tau, [stats step 1, stats step 2]); raises TvsError (TVS_EBUSY)
        before the job has finished, and the job's error if it failed."""
        n2, n1 = self.shape
        dev = self.ctx.device
        if d_out is None:
            d_out = torch.empty((n2, n1), dtype=self.dtype, device=dev)
        if tau_out is None:
            tau_out = torch.empty((2, n2 + 1, n1 + 1), dtype=self.dtype, device=dev)
        st = (Stats * 2)()
        _check(load().tvs_job_result(self.ctx._h, self._h, _dev(d_out, (n2, n1), self.dtype),
                                     _dev(tau_out, (2, n2 + 1, n1 + 1), self.dtype), st,
                                     _stream(dev)))
        return d_out, tau_out, [st[0].as_dict(), st[1].as_dict()]

    def export_state(self):
        """The job's state between sweeps as a host uint8 array (a checkpoint
        that Context.import_job resumes from)."""
        lib, dev = load(), self.ctx.device
        n = ctypes.c_size_t()
        _check(lib.tvs_job_export_state(self.ctx._h, self._h, None, 0, ctypes.byref(n), _stream(dev)))
        buf = np.empty(n.value, dtype=np.uint8)
        _check(lib.tvs_job_export_state(self.ctx._h, self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size,
                                        ctypes.byref(n), _stream(dev)))
        return buf

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(load().tvs_job_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
