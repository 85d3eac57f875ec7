"""ctypes binding of ``libsg.so`` (include/sg.h).  Argument marshalling only.

Tensors are torch ``complex128`` CUDA tensors used purely as device memory; the
stream is torch's current stream unless one is given.  Every call raises
``SGError`` on a negative status.  There is no fallback: if the native library is
missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsg.so")

SG_OK, SG_ENOTCONV, SG_FALLBACK_USED = 0, 1, 2
SG_PC_NONE, SG_PC_MEAN, SG_PC_CSL_MEAN, SG_PC_MEAN_NET = 0, 1, 2, 3
SG_PREC_F64, SG_PREC_F32, SG_PREC_BF16X3 = 0, 1, 2
SG_BC_ABSORBING = 0

PC = {"none": SG_PC_NONE, "mean": SG_PC_MEAN, "csl": SG_PC_CSL_MEAN, "net": SG_PC_MEAN_NET}
PREC = {"f64": SG_PREC_F64, "f32": SG_PREC_F32, "bf16x3": SG_PREC_BF16X3}
SIDE = {"right": 0, "left": 1}


class SGError(RuntimeError):
    pass


class C64(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int), ("bc", C.c_int), ("s", C.c_int), ("degree", C.c_int),
                ("k_fields", C.POINTER(C.c_double)), ("k_mean", C.c_double), ("csl_beta", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("maxit", C.c_int), ("precond", C.c_int), ("precision", C.c_int),
                ("tol", C.c_double), ("x0_zero", C.c_int), ("hist", C.POINTER(C.c_double)), ("hist_cap", C.c_int),
                ("side", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int), ("fallback", C.c_int),
                ("relres_true", C.c_double), ("relres_est", C.c_double), ("t_setup", C.c_double),
                ("t_precond", C.c_double), ("t_matvec", C.c_double), ("t_orth", C.c_double),
                ("t_total", C.c_double), ("relres_prec", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PRECOND_CB = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p)

_lib = None


def lib():
    """Load libsg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libsg.so not built: run `python -m paper_2209_14740_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded, so that the
    # process has one runtime (tensors, streams and the library's kernels share it)
    import torch  # noqa: F401
    L = C.CDLL(_LIB_PATH)
    vp, i, ll, d = C.c_void_p, C.c_int, C.c_longlong, C.c_double
    L.sg_setup.argtypes = [C.POINTER(Problem), vp, C.POINTER(vp)]
    L.sg_destroy.argtypes = [vp]
    L.sg_destroy.restype = None
    L.sg_basis.argtypes = [vp, C.POINTER(i), C.POINTER(i)]
    L.sg_size.argtypes = [vp]
    L.sg_size.restype = ll
    L.sg_rhs.argtypes = [vp, C.POINTER(d), vp, vp]
    L.sg_apply.argtypes = [vp, vp, vp, vp]
    L.sg_precond.argtypes = [vp, i, i, vp, vp, vp]
    L.sg_gmres.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveStats), vp]
    L.sg_fgmres.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), PRECOND_CB, vp, C.POINTER(SolveStats), vp]
    L.sg_stationary.argtypes = [vp, vp, vp, i, i, C.POINTER(d), vp]
    L.sg_set_operator_shift.argtypes = [vp, d]
    L.sg_moments.argtypes = [vp, vp, vp, vp, vp]
    L.sg_mean_solver.argtypes = [vp, C.POINTER(i), C.POINTER(d)]
    L.sg_setup_times.argtypes = [vp, C.POINTER(d)]
    L.sg_set_eigen_cond_limit.argtypes = [d]
    L.sg_set_orthogonalisation.argtypes = [vp, i]
    L.sg_last_basis.argtypes = [vp, C.POINTER(i), C.POINTER(vp)]
    L.sg_degree_magnitudes.argtypes = [vp, vp, C.POINTER(d), vp]
    L.sg_cgs2.argtypes = [ll, i, vp, vp, vp, vp]
    L.sg_cgs2_noalloc.argtypes = [ll, i, vp, vp, vp, vp]
    L.sg_norm.argtypes = [ll, vp, C.POINTER(d), vp]
    L.sg_axpby.argtypes = [ll, C64, vp, C64, vp, vp, vp]
    L.sg_gmres_batched.argtypes = [i, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(SolveOpts),
                                   C.POINTER(SolveStats), vp]
    L.sg_autotune.argtypes = [i, C.POINTER(vp), i, i, C.POINTER(d), vp]
    L.sg_batched_release.argtypes = []
    L.sg_tune_get.argtypes = [i, i, i]
    L.sg_tune_set.argtypes = [i, i, i, i]
    f = C.c_float
    L.sg_net_create.argtypes = [i, i, C.c_ulonglong, C.POINTER(vp)]
    L.sg_net_destroy.argtypes = [vp]
    L.sg_net_destroy.restype = None
    L.sg_net_num_params.argtypes = [vp]
    L.sg_net_num_params.restype = ll
    L.sg_net_get_params.argtypes = [vp, C.POINTER(f)]
    L.sg_net_set_params.argtypes = [vp, C.POINTER(f)]
    L.sg_net_forward_nhwc.argtypes = [vp, i, i, vp, vp, vp]
    L.sg_net_grad_nhwc.argtypes = [vp, i, i, vp, vp, C.POINTER(d), C.POINTER(f), vp]
    L.sg_net_adam_step.argtypes = [vp, f, vp]
    L.sg_net_train_pairs.argtypes = [vp, i, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), f, i, C.POINTER(d), vp]
    L.sg_net_save.argtypes = [vp, C.c_char_p]
    L.sg_net_load.argtypes = [vp, C.c_char_p]
    L.sg_attach_net.argtypes = [vp, vp]
    L.sg_set_profiling.argtypes = [vp, i]
    L.sg_profile_kinds.argtypes = [vp, C.c_uint]
    L.sg_kernel_times.argtypes = [vp, i, C.POINTER(d), C.POINTER(ll), C.POINTER(d)]
    L.sg_strerror.argtypes = [i]
    L.sg_strerror.restype = C.c_char_p
    L.sg_last_error.argtypes = []
    L.sg_last_error.restype = C.c_char_p
    for name in ("sg_setup", "sg_basis", "sg_rhs", "sg_apply", "sg_precond", "sg_gmres", "sg_fgmres",
                 "sg_stationary", "sg_set_operator_shift", "sg_moments", "sg_degree_magnitudes", "sg_mean_solver", "sg_setup_times", "sg_set_eigen_cond_limit", "sg_set_orthogonalisation", "sg_last_basis", "sg_cgs2",
                 "sg_cgs2_noalloc", "sg_norm", "sg_axpby", "sg_set_profiling",
                 "sg_kernel_times", "sg_gmres_batched", "sg_batched_release", "sg_autotune", "sg_tune_get", "sg_tune_set", "sg_net_create", "sg_net_get_params", "sg_net_set_params",
                 "sg_net_forward_nhwc", "sg_net_grad_nhwc", "sg_net_adam_step", "sg_net_train_pairs", "sg_net_save",
                 "sg_net_load", "sg_attach_net", "sg_profile_kinds"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc: int, what: str) -> int:
    if rc < 0:
        msg = lib().sg_last_error().decode(errors="replace")
        raise SGError("%s failed: %s (%s)" % (what, lib().sg_strerror(rc).decode(), msg))
    return rc


def _ptr(t) -> int:
    import torch
    if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise SGError("expected a contiguous complex128 CUDA tensor")
    return t.data_ptr()


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class SG:
    """One stochastic-Galerkin Helmholtz operator (a handle of the native library)."""

    def __init__(self, dim: int, n: int, s: int, degree: int, k_fields, k_mean: float, beta: float = 0.5,
                 stream=None):
        self._h = C.c_void_p()
        kf = np.ascontiguousarray(k_fields, dtype=np.float64)
        if kf.shape != (s + 1, n ** dim):
            raise SGError("k_fields must have shape (s+1, n**dim)")
        self._kf = kf
        prob = Problem(dim, n, SG_BC_ABSORBING, s, degree, kf.ctypes.data_as(C.POINTER(C.c_double)),
                       float(k_mean), float(beta))
        check(lib().sg_setup(C.byref(prob), C.c_void_p(_stream(stream)), C.byref(self._h)), "sg_setup")
        self.dim, self.n, self.s, self.degree = dim, n, s, degree
        q = C.c_int()
        check(lib().sg_basis(self._h, C.byref(q), None), "sg_basis")
        self.Q = q.value
        self.size = int(lib().sg_size(self._h))
        self._cb_keep = None
        self._net = None

    @classmethod
    def from_instance(cls, inst, stream=None):
        """Handle for a ``workloads.Instance``; a NaN k_mean (k_0 varies in space) selects the
        varying-mean block solves (k_mean = 0 at the ABI)."""
        km = inst.k_mean if np.isfinite(inst.k_mean) else 0.0
        return cls(inst.dim, inst.n, inst.s, inst.degree, inst.k_fields, km, inst.beta, stream)

    def close(self):
        if self._h:
            lib().sg_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def attach_net(self, net):
        """Attach a ``Net`` (or None) for pc="net"; the handle keeps a reference."""
        check(lib().sg_attach_net(self._h, net._h if net is not None else None), "sg_attach_net")
        self._net = net

    def basis(self) -> np.ndarray:
        q = C.c_int()
        out = (C.c_int * (self.Q * self.s))()
        check(lib().sg_basis(self._h, C.byref(q), out), "sg_basis")
        return np.frombuffer(out, dtype=np.int32).reshape(self.Q, self.s).copy()

    def empty(self):
        import torch
        return torch.empty(self.size, dtype=torch.complex128, device="cuda")

    def rhs(self, f, out=None, stream=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        b = self.empty() if out is None else out
        check(lib().sg_rhs(self._h, f.ctypes.data_as(C.POINTER(C.c_double)), C.c_void_p(_ptr(b)),
                           C.c_void_p(_stream(stream))), "sg_rhs")
        return b

    def apply(self, x, y=None, stream=None):
        y = self.empty() if y is None else y
        check(lib().sg_apply(self._h, C.c_void_p(_ptr(x)), C.c_void_p(_ptr(y)), C.c_void_p(_stream(stream))),
              "sg_apply")
        return y

    def precond(self, r, z=None, pc: str = "mean", precision: str = "f64", stream=None):
        z = self.empty() if z is None else z
        check(lib().sg_precond(self._h, PC[pc], PREC[precision], C.c_void_p(_ptr(r)), C.c_void_p(_ptr(z)),
                               C.c_void_p(_stream(stream))), "sg_precond")
        return z

    def set_orthogonalisation(self, kind: str):
        """"dcgs2" (default: delayed re-orthogonalisation) or "cgs2" (both passes in the same step)."""
        check(lib().sg_set_orthogonalisation(self._h, {"dcgs2": 0, "cgs2": 1}[kind]), "sg_set_orthogonalisation")

    def last_basis(self):
        """The orthonormal basis of the last delayed-CGS2 cycle as a (k, size) torch view."""
        k, p = C.c_int(), C.c_void_p()
        check(lib().sg_last_basis(self._h, C.byref(k), C.byref(p)), "sg_last_basis")
        return _wrap_device(p.value, k.value * self.size).view(k.value, self.size) if k.value else None

    def mean_solver(self):
        """("fd" | "line" | "line_fallback", estimated cond₂ of the eigenvector matrix)."""
        k, cv = C.c_int(), C.c_double()
        check(lib().sg_mean_solver(self._h, C.byref(k), C.byref(cv)), "sg_mean_solver")
        return ("fd", "line", "line_fallback")[k.value], cv.value

    def setup_times(self):
        """Milliseconds of this handle's setup: total, device allocations, uploads, stream creation."""
        ms = (C.c_double * 4)()
        check(lib().sg_setup_times(self._h, ms), "sg_setup_times")
        return {"total": ms[0], "alloc": ms[1], "upload": ms[2], "stream": ms[3]}

    def moments(self, x, stream=None):
        """(E[u], Var[Re u], Var[Im u]) of the SG solution x, as torch tensors on the device."""
        import torch
        mean = torch.empty(self.n ** self.dim, dtype=torch.complex128, device="cuda")
        var = torch.empty(2 * self.n ** self.dim, dtype=torch.float64, device="cuda")
        check(lib().sg_moments(self._h, C.c_void_p(_ptr(x)), C.c_void_p(_ptr(mean)), C.c_void_p(var.data_ptr()),
                               C.c_void_p(_stream(stream))), "sg_moments")
        P = self.n ** self.dim
        return mean, var[:P], var[P:]

    def degree_magnitudes(self, x, stream=None) -> np.ndarray:
        """γ_j = max ||V_i||_∞ over the basis polynomials of total degree j (j = 0..degree)."""
        out = (C.c_double * (self.degree + 1))()
        check(lib().sg_degree_magnitudes(self._h, C.c_void_p(_ptr(x)), out, C.c_void_p(_stream(stream))),
              "sg_degree_magnitudes")
        return np.array(out[:])

    def set_operator_shift(self, beta: float):
        """Operator of this handle: A (beta = 0) or M(beta) = A - i beta K."""
        check(lib().sg_set_operator_shift(self._h, float(beta)), "sg_set_operator_shift")

    def stationary(self, b, iters, x=None, pc: str = "mean", hist: bool = True, stream=None):
        """Stationary iteration x_{i+1} = x_i + B^{-1}(b - A x_i) from x_0 = B^{-1} b;
        returns (x, relative residual history of length iters+1, or None)."""
        x = self.empty() if x is None else x
        harr = (C.c_double * (iters + 1))() if hist else None
        check(lib().sg_stationary(self._h, C.c_void_p(_ptr(b)), C.c_void_p(_ptr(x)), PC[pc], iters,
                                  C.cast(harr, C.POINTER(C.c_double)) if harr is not None else None,
                                  C.c_void_p(_stream(stream))), "sg_stationary")
        return x, (list(harr) if hist else None)

    def _opts(self, restart, maxit, pc, precision, tol, x0_zero, hist, side="right"):
        harr = None
        if hist:
            harr = (C.c_double * maxit)()
        o = SolveOpts(restart, maxit, PC[pc], PREC[precision], tol, 1 if x0_zero else 0,
                      C.cast(harr, C.POINTER(C.c_double)) if harr is not None else None, maxit if hist else 0,
                      SIDE[side])
        return o, harr

    def gmres(self, b, x=None, restart=50, maxit=1000, pc="mean", precision="f64", tol=1e-8, x0_zero=True,
              hist=False, side="right", stream=None):
        """Restarted GMRES(m); side="left" preconditions from the left (tol then applies to the
        preconditioned residual, reported as info["relres_prec"])."""
        x = self.empty() if x is None else x
        o, harr = self._opts(restart, maxit, pc, precision, tol, x0_zero, hist, side)
        st = SolveStats()
        rc = check(lib().sg_gmres(self._h, C.c_void_p(_ptr(b)), C.c_void_p(_ptr(x)), C.byref(o), C.byref(st),
                                  C.c_void_p(_stream(stream))), "sg_gmres")
        info = st.as_dict()
        info["status"] = rc
        if hist:
            info["hist"] = list(harr)[: st.iters]
        return x, info

    def fgmres(self, b, x=None, restart=50, maxit=1000, pc="mean", precision="f64", tol=1e-8, x0_zero=True,
               hist=False, callback=None, stream=None):
        """Flexible GMRES; ``callback(r, z)`` (torch tensors) replaces the built-in preconditioner."""
        import torch
        x = self.empty() if x is None else x
        o, harr = self._opts(restart, maxit, pc, precision, tol, x0_zero, hist)
        st = SolveStats()
        cb = PRECOND_CB()
        if callback is not None:
            n = self.size

            def _tramp(user, r, z, s):
                try:
                    rt = _wrap_device(r, n)
                    zt = _wrap_device(z, n)
                    callback(rt, zt)
                    return 0
                except Exception:
                    return 1
            cb = PRECOND_CB(_tramp)
            self._cb_keep = cb
        rc = check(lib().sg_fgmres(self._h, C.c_void_p(_ptr(b)), C.c_void_p(_ptr(x)), C.byref(o), cb, None,
                                   C.byref(st), C.c_void_p(_stream(stream))), "sg_fgmres")
        info = st.as_dict()
        info["status"] = rc
        if hist:
            info["hist"] = list(harr)[: st.iters]
        return x, info


def _wrap_device(ptr, n):
    """View a raw device pointer of n complex128 values as a torch tensor (no copy)."""
    import torch

    class _Holder:
        pass

    h = _Holder()
    h.__cuda_array_interface__ = {"shape": (n,), "typestr": "<c16", "data": (ptr, False), "version": 2,
                                  "strides": None}
    return torch.as_tensor(h, device="cuda")


TILES = {"128x128": 0, "64x128": 1, "64x64": 2, "64x32": 3, "32x64": 4, "3m32x32": 5, "3m64x32": 6, "3m32x64": 7,
         "3m64x64": 8, "64x256": 9, "128x256": 10}


def set_eigen_cond_limit(limit: float):
    """Limit on cond₂ of the mean block's eigenvector matrix above which later setups use the
    line factorisation (default 1e4)."""
    check(lib().sg_set_eigen_cond_limit(float(limit)), "sg_set_eigen_cond_limit")


def gmres_batched(ops, bs, xs=None, restart=30, maxit=1000, pc="mean", precision="f32", tol=1e-8, stream=None):
    """Batched right-preconditioned GMRES over independent operators (``SG`` objects);
    returns (xs, status, [info per instance])."""
    cnt = len(ops)
    if len(bs) != cnt or (xs is not None and len(xs) != cnt):
        raise SGError("ops, bs and xs must have the same length")
    xs = [op.empty() for op in ops] if xs is None else xs
    for op, b, x in zip(ops, bs, xs):
        if b.numel() != op.size or x.numel() != op.size:
            raise SGError("vector length does not match its operator")
    H = (C.c_void_p * cnt)(*[op._h.value for op in ops])
    B = (C.c_void_p * cnt)(*[_ptr(b) for b in bs])
    X = (C.c_void_p * cnt)(*[_ptr(x) for x in xs])
    o = SolveOpts(restart, maxit, PC[pc], PREC[precision], tol, 1, None, 0, 0)
    st = (SolveStats * cnt)()
    rc = check(lib().sg_gmres_batched(cnt, H, B, X, C.byref(o), st, C.c_void_p(_stream(stream))),
               "sg_gmres_batched")
    return xs, rc, [st[i].as_dict() for i in range(cnt)]


def batched_release():
    """Free the batched solver's arena on the current device."""
    check(lib().sg_batched_release(), "sg_batched_release")


def autotune(ops, precision="f32", reps=5, stream=None) -> float:
    """Tile-shape autotuning of the preconditioner GEMMs for the shapes of ``ops``;
    returns the GPU milliseconds spent."""
    cnt = len(ops)
    H = (C.c_void_p * max(cnt, 1))(*[op._h.value for op in ops])
    ms = C.c_double()
    check(lib().sg_autotune(cnt, H, PREC[precision], reps, C.byref(ms), C.c_void_p(_stream(stream))), "sg_autotune")
    return ms.value


def tune_get(n, Q, precision="f32") -> int:
    return lib().sg_tune_get(n, Q, PREC[precision])


def tune_set(n, Q, precision, tile):
    check(lib().sg_tune_set(n, Q, PREC[precision], TILES.get(tile, tile)), "sg_tune_set")


class Net:
    """The learned correction network (``sg_net_*``)."""

    def __init__(self, Q: int, s: int, seed: int = 0):
        self._h = C.c_void_p()
        check(lib().sg_net_create(Q, s, seed, C.byref(self._h)), "sg_net_create")
        self.Q, self.s = Q, s
        self.c_in, self.c_out = 2 * Q + s + 1, 2 * Q
        self.num_params = int(lib().sg_net_num_params(self._h))

    def close(self):
        if self._h:
            lib().sg_net_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        check(lib().sg_net_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))), "sg_net_get_params")
        return out

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != self.num_params:
            raise SGError("expected %d parameters" % self.num_params)
        check(lib().sg_net_set_params(self._h, th.ctypes.data_as(C.POINTER(C.c_float))), "sg_net_set_params")

    @staticmethod
    def _f32(t, shape):
        import torch
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == shape):
            raise SGError("expected a contiguous float32 CUDA tensor of shape %s" % (shape,))
        return t.data_ptr()

    def forward_nhwc(self, x, stream=None):
        import torch
        B, H = x.shape[0], x.shape[1]
        y = torch.empty((B, H, H, self.c_out), dtype=torch.float32, device="cuda")
        check(lib().sg_net_forward_nhwc(self._h, B, H, C.c_void_p(self._f32(x, (B, H, H, self.c_in))),
                                        C.c_void_p(y.data_ptr()), C.c_void_p(_stream(stream))), "sg_net_forward_nhwc")
        return y

    def grad_nhwc(self, x, t, stream=None):
        B, H = x.shape[0], x.shape[1]
        loss = C.c_double()
        g = np.empty(self.num_params, dtype=np.float32)
        check(lib().sg_net_grad_nhwc(self._h, B, H, C.c_void_p(self._f32(x, (B, H, H, self.c_in))),
                                     C.c_void_p(self._f32(t, (B, H, H, self.c_out))), C.byref(loss),
                                     g.ctypes.data_as(C.POINTER(C.c_float)), C.c_void_p(_stream(stream))),
              "sg_net_grad_nhwc")
        return loss.value, g

    def adam_step(self, lr, stream=None):
        check(lib().sg_net_adam_step(self._h, float(lr), C.c_void_p(_stream(stream))), "sg_net_adam_step")

    def train_pairs(self, ops, rs, es, lr, precision="f64", stream=None) -> float:
        cnt = len(ops)
        H = (C.c_void_p * cnt)(*[op._h.value for op in ops])
        R = (C.c_void_p * cnt)(*[_ptr(r) for r in rs])
        E = (C.c_void_p * cnt)(*[_ptr(e) for e in es])
        loss = C.c_double()
        check(lib().sg_net_train_pairs(self._h, cnt, H, R, E, float(lr), PREC[precision], C.byref(loss),
                                       C.c_void_p(_stream(stream))), "sg_net_train_pairs")
        return loss.value

    def save(self, path):
        check(lib().sg_net_save(self._h, str(path).encode()), "sg_net_save")

    def load(self, path):
        check(lib().sg_net_load(self._h, str(path).encode()), "sg_net_load")


def cgs2(V, w, stream=None):
    """One CGS2 step against the orthonormal rows of V (nv × n); returns h (nv+1,) and normalises w."""
    nv, n = V.shape
    out = (C.c_double * (2 * (nv + 1)))()
    check(lib().sg_cgs2(n, nv, C.c_void_p(_ptr(V)), C.c_void_p(_ptr(w)), out, C.c_void_p(_stream(stream))),
          "sg_cgs2")
    a = np.frombuffer(out, dtype=np.float64)
    return a[0::2] + 1j * a[1::2]


def cgs2_noalloc(V, w, stream=None):
    """sg_cgs2 without any allocation (scratch in a fixed device array; nv <= 64)."""
    nv, n = V.shape
    out = (C.c_double * (2 * (nv + 1)))()
    check(lib().sg_cgs2_noalloc(n, nv, C.c_void_p(_ptr(V)), C.c_void_p(_ptr(w)), out, C.c_void_p(_stream(stream))),
          "sg_cgs2_noalloc")
    a = np.frombuffer(out, dtype=np.float64)
    return a[0::2] + 1j * a[1::2]


def axpby(alpha, x, beta=0.0, y=None, out=None, stream=None):
    """out = alpha x + beta y on the device (sg_axpby); out defaults to a new vector."""
    import torch
    out = torch.empty_like(x) if out is None else out
    a, bb = complex(alpha), complex(beta)
    check(lib().sg_axpby(x.numel(), C64(a.real, a.imag), C.c_void_p(_ptr(x)), C64(bb.real, bb.imag),
                         C.c_void_p(_ptr(y)) if y is not None else None, C.c_void_p(_ptr(out)),
                         C.c_void_p(_stream(stream))), "sg_axpby")
    return out


def norm(x, stream=None) -> float:
    out = C.c_double()
    check(lib().sg_norm(x.numel(), C.c_void_p(_ptr(x)), C.byref(out), C.c_void_p(_stream(stream))), "sg_norm")
    return out.value


EXPORTED = ["sg_setup", "sg_destroy", "sg_basis", "sg_size", "sg_rhs", "sg_apply", "sg_precond", "sg_gmres",
            "sg_fgmres", "sg_stationary", "sg_set_operator_shift", "sg_moments", "sg_degree_magnitudes", "sg_mean_solver",
            "sg_setup_times",
            "sg_set_eigen_cond_limit", "sg_set_orthogonalisation", "sg_last_basis", "sg_gmres_batched",
            "sg_batched_release", "sg_autotune", "sg_tune_get",
            "sg_tune_set", "sg_cgs2", "sg_cgs2_noalloc", "sg_norm", "sg_axpby",
            "sg_set_profiling", "sg_profile_kinds", "sg_kernel_times", "sg_net_create", "sg_net_destroy", "sg_net_num_params",
            "sg_net_get_params", "sg_net_set_params", "sg_net_forward_nhwc", "sg_net_grad_nhwc", "sg_net_adam_step",
            "sg_net_train_pairs", "sg_net_save", "sg_net_load", "sg_attach_net", "sg_strerror", "sg_last_error"]
