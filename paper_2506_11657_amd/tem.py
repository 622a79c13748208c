"""Python binding of the C ABI in include/tem.h (argument marshalling only).

Every computation runs in libtem.so (HIP kernels for gfx950 and the host
RKFIT); this module converts NumPy/PyTorch buffers to pointers and raises on
error statuses.  There is no fallback: if the library is missing or a call
fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtem.so")

TEM_OK, TEM_EINVAL, TEM_ENOMEM, TEM_ENOCONV, TEM_EBREAKDOWN, TEM_EHIP, TEM_ESTATE = 0, -1, -2, -3, -4, -5, -6
TEM_SIGMA_LOG, TEM_DEVICE_PTR = 1, 2
TEM_MAX_SHIFTS = 64
STATUS_NAMES = {0: "TEM_OK", -1: "TEM_EINVAL", -2: "TEM_ENOMEM", -3: "TEM_ENOCONV",
                -4: "TEM_EBREAKDOWN", -5: "TEM_EHIP", -6: "TEM_ESTATE"}

EXPORTS = ["tem_setup_grid", "tem_set_conductivity", "tem_poles", "tem_forward", "tem_adjoint",
           "tem_solutions", "tem_apply", "tem_apply_noalloc", "tem_sizes", "tem_destroy", "tem_last_error",
           "tem_engine_create", "tem_attach_engine", "tem_engine_stats", "tem_engine_destroy",
           "tem_jacobian_apply", "tem_poles_single", "tem_forward_single"]


class tem_loop(C.Structure):
    _fields_ = [("i0", C.c_int), ("i1", C.c_int), ("j0", C.c_int), ("j1", C.c_int), ("current", C.c_double)]


class tem_receiver(C.Structure):
    _fields_ = [("i", C.c_int), ("j", C.c_int)]


class tem_solve_opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("rtol", C.c_double), ("max_iter", C.c_int), ("block", C.c_int),
                ("seed_shift", C.c_double), ("refine_max", C.c_int), ("keep_solutions", C.c_int),
                ("profile", C.c_int), ("method", C.c_int)]


class tem_stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("n_shifts", C.c_int),
                ("iters_per_shift", C.c_int * TEM_MAX_SHIFTS), ("est_res", C.c_double * TEM_MAX_SHIFTS),
                ("true_res", C.c_double * TEM_MAX_SHIFTS), ("refine_passes", C.c_int),
                ("seconds", C.c_double), ("unknown_updates", C.c_double),
                ("kernel_ms", C.c_double * 4), ("kernel_launches", C.c_longlong * 4)]

    def as_dict(self):
        J = self.n_shifts
        return {"iterations": self.iterations, "converged": bool(self.converged), "n_shifts": J,
                "iters_per_shift": list(self.iters_per_shift[:J]), "est_res": list(self.est_res[:J]),
                "true_res": list(self.true_res[:J]), "refine_passes": self.refine_passes,
                "seconds": self.seconds, "unknown_updates": self.unknown_updates,
                "kernel_ms": list(self.kernel_ms), "kernel_launches": list(self.kernel_launches)}


_lib = None


class TemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def lib():
    """Load libtem.so (built by paper_2506_11657_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libtem.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2506_11657_amd.build); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.tem_setup_grid.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int, dp, dp, dp, C.c_int,
                                     C.c_int, C.c_void_p]
        L.tem_set_conductivity.argtypes = [C.c_void_p, C.c_void_p, C.c_int]
        L.tem_poles.argtypes = [C.c_int, dp, dp, C.c_int, C.c_double, C.c_int, ip, dp, dp, dp]
        L.tem_forward.argtypes = [C.c_void_p, C.POINTER(tem_loop), C.c_int, C.POINTER(tem_receiver), C.c_int,
                                  C.c_int, C.c_int, dp, dp, C.POINTER(tem_solve_opts), dp, C.c_void_p,
                                  C.POINTER(tem_stats)]
        L.tem_poles_single.argtypes = [C.c_int, ip, dp, dp, dp, dp]
        L.tem_forward_single.argtypes = [C.c_void_p, C.POINTER(tem_loop), C.c_int, C.POINTER(tem_receiver),
                                         C.c_int, C.c_int, dp, C.c_int, dp, dp, C.c_double,
                                         C.POINTER(tem_solve_opts), dp, C.c_void_p, C.POINTER(tem_stats)]
        L.tem_adjoint.argtypes = [C.c_void_p, dp, dp, C.POINTER(tem_stats)]
        L.tem_jacobian_apply.argtypes = [C.c_void_p, dp, dp, C.POINTER(tem_stats)]
        L.tem_solutions.argtypes = [C.c_void_p, C.c_int, dp]
        L.tem_apply.argtypes = [C.c_void_p, C.c_double, C.c_double, dp, dp]
        L.tem_apply_noalloc.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p]
        L.tem_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]
        L.tem_destroy.argtypes = [C.c_void_p]
        L.tem_destroy.restype = None
        L.tem_engine_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_int]
        L.tem_attach_engine.argtypes = [C.c_void_p, C.c_void_p]
        L.tem_engine_stats.argtypes = [C.c_void_p, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong),
                                       C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.tem_engine_destroy.argtypes = [C.c_void_p]
        L.tem_last_error.argtypes = [C.c_void_p]
        L.tem_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("tem_destroy", "tem_last_error", "tem_engine_destroy"):
                getattr(L, name).restype = C.c_int
        L.tem_engine_destroy.restype = None
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _check(status, ctx=None, allow=()):
    if status != TEM_OK and status not in allow:
        raise TemError(status, lib().tem_last_error(ctx).decode())
    return status


def poles(t, degree=0, tol=1e-8, w=None, j_max=TEM_MAX_SHIFTS):
    """tem_poles: shared poles xi (J complex) and coefficients c (J x T complex,
    factor 2 of pairs folded in) and the per-channel errors err (T)."""
    t = _f64(t)
    T = len(t)
    wv = None if w is None else _f64(w)
    J = C.c_int(0)
    xi = np.zeros(2 * j_max)
    c = np.zeros(2 * j_max * T)
    err = np.zeros(T)
    _check(lib().tem_poles(T, _dptr(t), None if wv is None else _dptr(wv), int(degree), float(tol), j_max,
                           C.byref(J), _dptr(xi), _dptr(c), _dptr(err)))
    J = J.value
    xi_c = xi[:2 * J].view(np.complex128).copy()
    c_c = c[:2 * J * T].view(np.complex128).reshape(J, T).copy()
    return xi_c, c_c, err


def poles_single(m):
    """tem_poles_single: the type-[m/m] best approximation of exp(-x) on
    [0, inf): poles xi (ceil(m/2) complex, one per pair), residues a (factor
    2 of pairs folded in), the constant alpha0 and the uniform error."""
    J = C.c_int(0)
    xi = np.zeros(2 * 32)
    a = np.zeros(2 * 32)
    a0 = C.c_double(0.0)
    err = C.c_double(0.0)
    _check(lib().tem_poles_single(int(m), C.byref(J), _dptr(xi), _dptr(a), C.byref(a0), C.byref(err)))
    J = J.value
    return xi[:2 * J].view(np.complex128).copy(), a[:2 * J].view(np.complex128).copy(), a0.value, err.value


class Engine:
    """tem_engine_create: a solve engine on one device that batches the FP64
    multi-shift solves of every attached context into shared launches."""

    def __init__(self, device=0, max_jobs=0):
        h = C.c_void_p()
        _check(lib().tem_engine_create(C.byref(h), int(device), int(max_jobs)))
        self._h = h

    def stats(self):
        b, jb = C.c_longlong(), C.c_longlong()
        mj, mc = C.c_int(), C.c_int()
        _check(lib().tem_engine_stats(self._h, C.byref(b), C.byref(jb), C.byref(mj), C.byref(mc)))
        return {"blocks": b.value, "job_blocks": jb.value, "max_jobs": mj.value, "max_contexts": mc.value}

    def close(self):
        if getattr(self, "_h", None):
            lib().tem_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A grid on one device: tem_setup_grid / tem_set_conductivity / tem_forward ..."""

    def __init__(self, hx, hy, hz, k_surface, device=0, stream=None):
        self.hx, self.hy, self.hz = _f64(hx), _f64(hy), _f64(hz)
        self.shape = (len(self.hz), len(self.hy), len(self.hx))
        h = C.c_void_p()
        s = None if stream is None else C.c_void_p(int(stream))
        _check(lib().tem_setup_grid(C.byref(h), len(self.hx), len(self.hy), len(self.hz), _dptr(self.hx),
                                    _dptr(self.hy), _dptr(self.hz), int(k_surface), int(device), s))
        self._h = h
        ns, nu = C.c_longlong(), C.c_longlong()
        _check(lib().tem_sizes(h, C.byref(ns), C.byref(nu)), h)
        self.n_storage, self.n_unknowns = ns.value, nu.value
        self._n_src = 0
        self.generation = 0      # counts forward calls and conductivity changes

    @classmethod
    def from_workload(cls, wl, device=0, stream=None):
        ctx = cls(wl.hx, wl.hy, wl.hz, wl.k_s, device, stream)
        ctx.set_conductivity(wl.sigma)
        return ctx

    def attach(self, engine):
        """tem_attach_engine: route this context's FP64 solves through engine (None detaches)."""
        _check(lib().tem_attach_engine(self._h, None if engine is None else engine._h), self._h)
        self._engine = engine   # kept alive while attached

    def close(self):
        if getattr(self, "_h", None):
            lib().tem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_conductivity(self, sigma, log=False):
        """sigma (nz, ny, nx) S/m (or ln sigma with log=True); numpy or a torch tensor."""
        flags = TEM_SIGMA_LOG if log else 0
        self.generation += 1
        try:
            import torch
            if isinstance(sigma, torch.Tensor):
                if sigma.shape != self.shape:
                    raise ValueError("sigma must have shape %s" % (self.shape,))
                if sigma.is_cuda:
                    t = sigma.detach().to(torch.float64).contiguous()
                    _check(lib().tem_set_conductivity(self._h, C.c_void_p(t.data_ptr()), flags | TEM_DEVICE_PTR),
                           self._h)
                    return
                sigma = sigma.detach().cpu().numpy()
        except ImportError:
            pass
        a = _f64(sigma)
        if a.shape != self.shape:
            raise ValueError("sigma must have shape %s" % (self.shape,))
        _check(lib().tem_set_conductivity(self._h, a.ctypes.data_as(C.c_void_p), flags), self._h)

    def forward(self, loops, receivers, xi, c, fields=None, rtol=0.0, max_iter=0, block=0, seed_shift=0.0,
                precision=0, keep_solutions=False, refine_max=0, allow_noconv=False, profile=False, method=0):
        """tem_forward.  loops: list of (i0, i1, j0, j1, current) or objects with
        those attributes; receivers: list of (i, j); xi (J complex); c (J x T
        complex).  fields: optional device tensor (n_src, T, n_storage) float64.
        Returns (data (n_src, T, n_rx), stats dict)."""
        src = (tem_loop * len(loops))()
        for s, L in enumerate(loops):
            v = (L.i0, L.i1, L.j0, L.j1, L.current) if hasattr(L, "i0") else tuple(L)
            src[s] = tem_loop(int(v[0]), int(v[1]), int(v[2]), int(v[3]), float(v[4]))
        n_rx = len(receivers)
        rx = (tem_receiver * max(n_rx, 1))()
        for r, (i, j) in enumerate(receivers):
            rx[r] = tem_receiver(int(i), int(j))
        xi = np.ascontiguousarray(np.asarray(xi, np.complex128))
        c = np.ascontiguousarray(np.asarray(c, np.complex128))
        J, T = c.shape
        self._J = J
        if xi.shape != (J,):
            raise ValueError("xi must have one entry per row of c")
        xr = xi.view(np.float64)
        cr = c.view(np.float64)
        data = np.zeros((len(loops), T, max(n_rx, 1)))
        fptr = None
        if fields is not None:
            if tuple(fields.shape) != (len(loops), T, self.n_storage) or not fields.is_cuda:
                raise ValueError("fields must be a device tensor of shape (n_src, T, n_storage)")
            fptr = C.c_void_p(fields.data_ptr())
        opts = tem_solve_opts(int(precision), float(rtol), int(max_iter), int(block), float(seed_shift),
                              int(refine_max), 1 if keep_solutions else 0, 1 if profile else 0, int(method))
        st = tem_stats()
        self.generation += 1
        status = lib().tem_forward(self._h, src, len(loops), rx, n_rx, T, J, _dptr(xr), _dptr(cr), C.byref(opts),
                                   _dptr(data), fptr, C.byref(st))
        _check(status, self._h, allow=(TEM_ENOCONV,) if allow_noconv else ())
        self._n_src = len(loops)
        self._T, self._n_rx = T, n_rx
        out = st.as_dict()
        out["status"] = STATUS_NAMES[status]
        return data[:, :, :n_rx], out

    def forward_single(self, loops, receivers, t, xi, a, alpha0, fields=None, rtol=0.0, max_iter=0, block=0,
                       seed_shift=0.0, allow_noconv=False, profile=False):
        """tem_forward_single: eq. (rba) for every channel t (T) with the
        single-time approximant (xi, a, alpha0) of poles_single.  fields:
        optional device tensor (n_src, T, n_storage) float64.  Returns (data
        (n_src, T, n_rx), stats dict)."""
        src = (tem_loop * len(loops))()
        for s, L in enumerate(loops):
            v = (L.i0, L.i1, L.j0, L.j1, L.current) if hasattr(L, "i0") else tuple(L)
            src[s] = tem_loop(int(v[0]), int(v[1]), int(v[2]), int(v[3]), float(v[4]))
        n_rx = len(receivers)
        rx = (tem_receiver * max(n_rx, 1))()
        for r, (i, j) in enumerate(receivers):
            rx[r] = tem_receiver(int(i), int(j))
        t = _f64(t)
        T = len(t)
        xi = np.ascontiguousarray(np.asarray(xi, np.complex128))
        a = np.ascontiguousarray(np.asarray(a, np.complex128))
        if xi.shape != a.shape or xi.ndim != 1:
            raise ValueError("xi and a must be 1-D with one residue per pole")
        data = np.zeros((len(loops), T, max(n_rx, 1)))
        fptr = None
        if fields is not None:
            if tuple(fields.shape) != (len(loops), T, self.n_storage) or not fields.is_cuda:
                raise ValueError("fields must be a device tensor of shape (n_src, T, n_storage)")
            fptr = C.c_void_p(fields.data_ptr())
        opts = tem_solve_opts(0, float(rtol), int(max_iter), int(block), float(seed_shift), 0, 0,
                              1 if profile else 0, 0)
        st = tem_stats()
        self.generation += 1
        status = lib().tem_forward_single(self._h, src, len(loops), rx, n_rx, T, _dptr(t), len(xi),
                                          _dptr(xi.view(np.float64)), _dptr(a.view(np.float64)), float(alpha0),
                                          C.byref(opts), _dptr(data), fptr, C.byref(st))
        _check(status, self._h, allow=(TEM_ENOCONV,) if allow_noconv else ())
        out = st.as_dict()
        # per channel: the maxima over that channel's systems
        for key in ("iters_per_shift", "est_res", "true_res"):
            out[key] = out[key][:T]
        out["status"] = STATUS_NAMES[status]
        return data[:, :, :n_rx], out

    def solutions(self, s=0):
        """Stored x_j of source s in storage order: (J, n_storage) complex."""
        J = getattr(self, "_J", 0)
        if J == 0:
            raise RuntimeError("no forward run on this context")
        buf = np.zeros(2 * J * self.n_storage)
        _check(lib().tem_solutions(self._h, int(s), _dptr(buf)), self._h)
        return buf.view(np.complex128).reshape(J, self.n_storage)

    def apply(self, x, shift):
        """(K + shift M) x for a complex storage-order vector x."""
        x = np.ascontiguousarray(np.asarray(x, np.complex128))
        if x.shape != (self.n_storage,):
            raise ValueError("x must have length n_storage")
        y = np.zeros_like(x)
        _check(lib().tem_apply(self._h, float(np.real(shift)), float(np.imag(shift)), _dptr(x.view(np.float64)),
                               _dptr(y.view(np.float64))), self._h)
        return y

    def apply_noalloc(self, x, y, shift):
        """tem_apply_noalloc: y = (K + shift M) x with x, y complex128 device
        tensors of length n_storage (no device allocation by the library)."""
        import torch
        for v in (x, y):
            if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.complex128
                    and v.is_contiguous() and tuple(v.shape) == (self.n_storage,)):
                raise ValueError("x and y must be contiguous complex128 device tensors of length n_storage")
        _check(lib().tem_apply_noalloc(self._h, float(np.real(shift)), float(np.imag(shift)),
                                       C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr())), self._h)
        return y

    def jacobian_apply(self, dm):
        """tem_jacobian_apply: first-order change of the last forward's data
        (n_src, T, n_rx) for a change dm (nz, ny, nx) of ln sigma."""
        dm = _f64(dm)
        if dm.shape != self.shape:
            raise ValueError("dm must have shape %s" % (self.shape,))
        J = getattr(self, "_J", 0)
        if J == 0:
            raise RuntimeError("no forward run on this context")
        out = np.zeros((self._n_src, self._T, max(self._n_rx, 1)))
        st = tem_stats()
        _check(lib().tem_jacobian_apply(self._h, _dptr(dm), _dptr(out), C.byref(st)), self._h)
        return out[:, :, :self._n_rx], st.as_dict()

    def adjoint(self, w):
        """tem_adjoint: gradient (nz, ny, nx) of phi w.r.t. ln sigma given
        w = dphi/d data (n_src, T, n_rx) for the last forward."""
        w = _f64(w)
        grad = np.zeros(self.shape)
        st = tem_stats()
        _check(lib().tem_adjoint(self._h, _dptr(w), _dptr(grad), C.byref(st)), self._h)
        return grad, st.as_dict()
