"""Thin ctypes binding of the C-ABI declared in include/fh.h and
include/fh_net.h.

Argument marshalling only: every step of the solver runs in libfh.so.  Device
arrays are passed as torch tensors on the context's device (their data
pointers go to the library); host arrays as numpy arrays.  Loading fails
loudly if libfh.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfh.so")

FH_OK, FH_NOT_CONVERGED = 0, 1
FH_EINVAL, FH_ENOMEM, FH_EDEVICE, FH_ENOTSPD, FH_ESTATE = -1, -2, -3, -4, -5
FH_SCALAR, FH_ELASTIC = 0, 1
FH_HEX8, FH_QUAD4, FH_TRI2, FH_TRI4 = 0, 1, 2, 3
FH_FP64, FH_FP32_REFINED = 0, 1
FH_MAX_LOADS = 32
FH_FLAG_TIME_KERNELS = 1
FH_FLAG_REBUILD = 2
FH_FLAG_WARM_START = 4
FH_FLAG_TIME_SAMPLED = 8
FH_FLAG_BATCH_SERIAL = 16
FH_FLAG_GRAPH = 32
FH_REF_MEAN, FH_REF_IDENTITY, FH_REF_BEST = 0, 1, 2
FH_MAX_INCREMENTS, FH_MAX_NEWTON = 64, 64
FH_NEWTON_REF_TANGENT, FH_NEWTON_REF_ELASTIC = 0, 1
NET_CLASSES = ["conv", "dgrad", "wgrad", "other"]
KERNEL_CLASSES = ["operator", "xfwd", "yfwd", "zsolve", "yinv", "xinv", "scalar", "other"]

ELEMENTS = {"hex8": FH_HEX8, "quad4": FH_QUAD4, "tri2": FH_TRI2, "tri4": FH_TRI4}
PROBLEMS = {"scalar": FH_SCALAR, "elastic": FH_ELASTIC}

EXPORTED = [
    "fh_create", "fh_destroy", "fh_last_error", "fh_set_stream", "fh_set_grid",
    "fh_set_phases", "fh_set_conductivity_field", "fh_set_reference", "fh_set_load",
    "fh_workspace_size", "fh_bind_workspace", "fh_batch_workspace_size", "fh_solve",
    "fh_get_fluctuation",
    "fh_get_homogenized", "fh_get_reference", "fh_get_history", "fh_apply_operator",
    "fh_apply_preconditioner", "fh_compute_rhs", "fh_compute_rhs_noalloc", "fh_get_symbol",
    "fh_solve_rhs",
    "fh_solve_batch", "fh_set_warm_start", "fh_eigen_bounds", "fh_choose_reference",
    "fh_set_plastic_phases", "fh_newton_solve", "fh_get_plastic_state",
    "fh_solve_strain_based", "fh_get_strain",
    "fh_net_param_count", "fh_net_create", "fh_net_destroy", "fh_net_last_error",
    "fh_net_set_stream", "fh_net_set_params", "fh_net_get_params", "fh_net_forward",
    "fh_net_gradient", "fh_net_adam", "fh_net_train", "fh_net_pack_target",
    "fh_net_set_timing", "fh_net_get_stats", "fh_net_guess", "fh_net_layer",
]


class fh_opts(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("itmax", ctypes.c_int),
                ("precision", ctypes.c_int), ("poll", ctypes.c_int),
                ("flags", ctypes.c_int), ("eta_inner", ctypes.c_double),
                ("guess_dev", ctypes.c_void_p)]


class fh_stats(ctypes.Structure):
    _fields_ = [("nload", ctypes.c_int),
                ("iterations", ctypes.c_int * FH_MAX_LOADS),
                ("status", ctypes.c_int * FH_MAX_LOADS),
                ("rel_res", ctypes.c_double * FH_MAX_LOADS),
                ("outer", ctypes.c_int * FH_MAX_LOADS),
                ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("chom_ms", ctypes.c_double), ("dof", ctypes.c_longlong),
                ("kernel_ms", ctypes.c_double * 8), ("kernel_launches", ctypes.c_longlong * 8),
                ("guess_used", ctypes.c_int * FH_MAX_LOADS),
                ("guess_res", ctypes.c_double * FH_MAX_LOADS), ("guess_ms", ctypes.c_double),
                ("kernel_issued", ctypes.c_longlong * 8),
                ("kernel_units", ctypes.c_double * 8)]

    def as_dict(self):
        n = self.nload
        return dict(nload=n, iterations=list(self.iterations[:n]), status=list(self.status[:n]),
                    rel_res=list(self.rel_res[:n]), outer=list(self.outer[:n]),
                    setup_ms=self.setup_ms, solve_ms=self.solve_ms, chom_ms=self.chom_ms,
                    dof=self.dof, kernel_ms=list(self.kernel_ms),
                    kernel_launches=list(self.kernel_launches),
                    kernel_issued=list(self.kernel_issued),
                    kernel_units=list(self.kernel_units),
                    guess_used=list(self.guess_used[:n]), guess_res=list(self.guess_res[:n]),
                    guess_ms=self.guess_ms)


class fh_system(ctypes.Structure):
    _fields_ = [("phase_dev", ctypes.c_void_p), ("n", ctypes.c_int * 3),
                ("nphase", ctypes.c_int), ("mat", ctypes.POINTER(ctypes.c_double)),
                ("u_dev", ctypes.c_void_p)]


class fh_adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double),
                ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("clip", ctypes.c_double)]


class fh_net_stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double * 4), ("kernel_launches", ctypes.c_longlong * 4),
                ("flops", ctypes.c_double * 4), ("adam_steps", ctypes.c_longlong)]

    def as_dict(self):
        return {k: dict(ms=self.kernel_ms[i], launches=self.kernel_launches[i],
                        flops=self.flops[i]) for i, k in enumerate(NET_CLASSES)} | \
            dict(adam_steps=self.adam_steps)


class fh_bounds(ctypes.Structure):
    _fields_ = [("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("kappa", ctypes.c_double), ("predicted_iterations", ctypes.c_int),
                ("pad", ctypes.c_int)]

    def as_dict(self):
        return dict(lambda_min=self.lambda_min, lambda_max=self.lambda_max, kappa=self.kappa,
                    predicted_iterations=self.predicted_iterations)


class fh_newton_opts(ctypes.Structure):
    _fields_ = [("eta_newton", ctypes.c_double), ("eta_cg", ctypes.c_double),
                ("itmax_newton", ctypes.c_int), ("itmax_cg", ctypes.c_int),
                ("nincrement", ctypes.c_int), ("ref_mode", ctypes.c_int)]


class fh_newton_stats(ctypes.Structure):
    _fields_ = [("nincrement", ctypes.c_int),
                ("newton_steps", ctypes.c_int * FH_MAX_INCREMENTS),
                ("converged", ctypes.c_int * FH_MAX_INCREMENTS),
                ("pcg_iterations", (ctypes.c_int * FH_MAX_NEWTON) * FH_MAX_INCREMENTS),
                ("du_ratio", (ctypes.c_double * FH_MAX_NEWTON) * FH_MAX_INCREMENTS),
                ("macro_stress", (ctypes.c_double * 6) * FH_MAX_INCREMENTS),
                ("plastic_fraction", ctypes.c_double * FH_MAX_INCREMENTS),
                ("total_pcg", ctypes.c_int), ("solve_ms", ctypes.c_double)]

    def as_dict(self):
        k = self.nincrement
        steps = list(self.newton_steps[:k])
        return dict(nincrement=k, newton_steps=steps, converged=list(self.converged[:k]),
                    pcg_iterations=[list(self.pcg_iterations[i][:steps[i]]) for i in range(k)],
                    du_ratio=[list(self.du_ratio[i][:steps[i]]) for i in range(k)],
                    macro_stress=[list(self.macro_stress[i]) for i in range(k)],
                    plastic_fraction=list(self.plastic_fraction[:k]),
                    total_pcg=self.total_pcg, solve_ms=self.solve_ms)


FH_MAX_GROUPS = 16


class fh_batch_report(ctypes.Structure):
    _fields_ = [("ngroups", ctypes.c_int), ("n", (ctypes.c_int * 3) * FH_MAX_GROUPS),
                ("nsys", ctypes.c_int * FH_MAX_GROUPS), ("kz", ctypes.c_int * FH_MAX_GROUPS),
                ("zb", ctypes.c_int * FH_MAX_GROUPS), ("kyb", ctypes.c_int * FH_MAX_GROUPS),
                ("tune_ms", ctypes.c_double * FH_MAX_GROUPS),
                ("setup_ms", ctypes.c_double * FH_MAX_GROUPS),
                ("solve_ms", ctypes.c_double * FH_MAX_GROUPS),
                ("xrows", ctypes.c_int * FH_MAX_GROUPS)]

    def as_dict(self):
        g = self.ngroups
        return [dict(n=list(self.n[i]), nsys=self.nsys[i], kz=self.kz[i], zb=self.zb[i],
                     kyb=self.kyb[i], xrows=self.xrows[i], tune_ms=self.tune_ms[i],
                     setup_ms=self.setup_ms[i], solve_ms=self.solve_ms[i]) for i in range(g)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfh.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libfh.so not found at {path}: run __graft_entry__.build() "
                           "or python paper_2203_02962_amd/build.py")
    # libfh.so links the HIP runtime.  PyTorch (which provides the device
    # memory and streams) ships its own copy; load it first so that both use
    # one runtime.  The other way round, torch then finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "fh_create": ([ctypes.POINTER(P), I], I),
        "fh_destroy": ([P], None),
        "fh_last_error": ([P], ctypes.c_char_p),
        "fh_set_stream": ([P, P], I),
        "fh_set_grid": ([P, I, ctypes.POINTER(I), ctypes.POINTER(D), I, I], I),
        "fh_set_phases": ([P, P, I, ctypes.POINTER(D)], I),
        "fh_set_conductivity_field": ([P, P], I),
        "fh_set_reference": ([P, ctypes.POINTER(D)], I),
        "fh_set_load": ([P, I, ctypes.POINTER(D)], I),
        "fh_workspace_size": ([P, ctypes.POINTER(ctypes.c_size_t)], I),
        "fh_bind_workspace": ([P, P, ctypes.c_size_t], I),
        "fh_batch_workspace_size": ([P, I, P, I, ctypes.POINTER(ctypes.c_size_t)], I),
        "fh_solve": ([P, ctypes.POINTER(fh_opts), ctypes.POINTER(fh_stats)], I),
        "fh_get_fluctuation": ([P, I, P], I),
        "fh_get_homogenized": ([P, ctypes.POINTER(D)], I),
        "fh_get_reference": ([P, ctypes.POINTER(D)], I),
        "fh_get_history": ([P, I, ctypes.POINTER(D), I, ctypes.POINTER(I)], I),
        "fh_apply_operator": ([P, P, P], I),
        "fh_apply_preconditioner": ([P, P, P], I),
        "fh_compute_rhs": ([P, ctypes.POINTER(D), P], I),
        "fh_compute_rhs_noalloc": ([P, ctypes.POINTER(D), P], I),
        "fh_get_symbol": ([P, P], I),
        "fh_solve_rhs": ([P, P, P, ctypes.POINTER(fh_opts), ctypes.POINTER(fh_stats)], I),
        "fh_solve_batch": ([P, I, ctypes.POINTER(fh_system), I, ctypes.POINTER(D),
                            ctypes.POINTER(fh_opts), ctypes.POINTER(D), ctypes.POINTER(fh_stats),
                            ctypes.POINTER(fh_batch_report)], I),
        "fh_set_warm_start": ([P, P], I),
        "fh_eigen_bounds": ([P, ctypes.POINTER(D), D, P, P, ctypes.POINTER(fh_bounds)], I),
        "fh_set_plastic_phases": ([P, P, I, ctypes.POINTER(D)], I),
        "fh_newton_solve": ([P, ctypes.POINTER(D), ctypes.POINTER(fh_newton_opts),
                             ctypes.POINTER(fh_newton_stats)], I),
        "fh_get_plastic_state": ([P, P, P, P], I),
        "fh_solve_strain_based": ([P, ctypes.POINTER(fh_opts), ctypes.POINTER(fh_stats)], I),
        "fh_get_strain": ([P, I, P], I),
        "fh_choose_reference": ([P, I, ctypes.POINTER(D), ctypes.POINTER(fh_bounds)], I),
        "fh_net_param_count": ([], ctypes.c_longlong),
        "fh_net_create": ([ctypes.POINTER(P), I, I, I], I),
        "fh_net_destroy": ([P], None),
        "fh_net_last_error": ([P], ctypes.c_char_p),
        "fh_net_set_stream": ([P, P], I),
        "fh_net_set_params": ([P, ctypes.POINTER(ctypes.c_float)], I),
        "fh_net_get_params": ([P, ctypes.POINTER(ctypes.c_float)], I),
        "fh_net_forward": ([P, I, P, ctypes.POINTER(ctypes.c_float), P], I),
        "fh_net_gradient": ([P, I, P, ctypes.POINTER(ctypes.c_float), P,
                             ctypes.POINTER(D), ctypes.POINTER(ctypes.c_float)], I),
        "fh_net_adam": ([P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(fh_adam)], I),
        "fh_net_train": ([P, I, P, ctypes.POINTER(ctypes.c_float), P, I, I,
                          ctypes.POINTER(I), ctypes.POINTER(fh_adam), ctypes.POINTER(D)], I),
        "fh_net_pack_target": ([P, P, D, P], I),
        "fh_net_set_timing": ([P, I], I),
        "fh_net_get_stats": ([P, ctypes.POINTER(fh_net_stats)], I),
        "fh_net_guess": ([P, P, ctypes.c_float, I, ctypes.POINTER(D), D, P], I),
        "fh_net_layer": ([P, I, I, I, P, P, P, P], I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


class FHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fh error {code}: {msg}")
        self.code = code


def _dptr(arr):
    # callers convert first, so the array outlives the call
    assert arr.dtype == np.float64 and arr.flags.c_contiguous
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _tptr(t, dtype=None, numel=None, device=None):
    """Data pointer of a contiguous device tensor, after checking what the
    library will read or write through it: `dtype` (a torch dtype or a tuple
    of them), at least `numel` elements and the context's device index.  A
    mismatch raises TypeError before any library call."""
    import torch  # device memory provider only
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or not t.is_contiguous():
        raise TypeError("expected a contiguous CUDA (HIP) tensor")
    if dtype is not None:
        ok = dtype if isinstance(dtype, tuple) else (dtype,)
        if t.dtype not in ok:
            raise TypeError(f"expected a tensor of dtype {ok}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise TypeError(f"tensor has {t.numel()} elements, the call needs at least {numel}")
    if device is not None and t.device.index != device:
        raise TypeError(f"tensor is on cuda:{t.device.index}, the context on cuda:{device}")
    return ctypes.c_void_p(t.data_ptr())


def _f64():
    import torch
    return torch.float64


def _U8():
    import torch
    return torch.uint8


def _BF16_CARRIERS():
    """16-bit storage the library reads as BF16 bit patterns."""
    import torch
    return (torch.int16, torch.bfloat16, torch.uint16) if hasattr(torch, "uint16") else \
        (torch.int16, torch.bfloat16)


class Context:
    """Owns one fh_ctx.  Method names follow the C functions (fh_ prefix
    dropped)."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.ptr = ctypes.c_void_p()
        rc = self.lib.fh_create(ctypes.byref(self.ptr), device)
        if rc != FH_OK:
            raise FHError(rc, f"fh_create(device={device}) failed")
        self.device = device
        self._keep = []      # device inputs that must outlive the call
        self._ws = None

    def _check(self, rc, allow_warning=False):
        if rc < 0 or (rc > 0 and not allow_warning):
            raise FHError(rc, self.lib.fh_last_error(self.ptr).decode())
        return rc

    def close(self):
        if self.ptr:
            self.lib.fh_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- setters
    def set_stream(self, stream):
        """stream: torch.cuda.Stream or a raw hipStream_t integer."""
        raw = getattr(stream, "cuda_stream", stream)
        return self._check(self.lib.fh_set_stream(self.ptr, ctypes.c_void_p(raw)))

    def set_grid(self, n, problem="elastic", element="hex8", l=None):
        n = list(n) + [1] * (3 - len(n))
        dim = 3 if element == "hex8" else 2
        narr = (ctypes.c_int * 3)(*[int(v) for v in n])
        larr = None if l is None else (ctypes.c_double * 3)(*(list(l) + [1.0] * (3 - len(l))))
        # fields per grid point: node sets x components (two node sets for
        # the two-node stencil)
        self.nd = (dim if problem == "elastic" else 1) * (2 if element == "tri4" else 1)
        self.element = element
        self.N = int(np.prod(n[:dim]))
        self.n = tuple(n[:dim])
        self.dim = dim
        self.m = dim * (dim + 1) // 2 if problem == "elastic" else dim
        return self._check(self.lib.fh_set_grid(self.ptr, dim, narr, larr,
                                                PROBLEMS[problem], ELEMENTS[element]))

    def set_phases(self, phase_dev, mat):
        mat = np.ascontiguousarray(mat, dtype=np.float64)
        import torch
        ptr = _tptr(phase_dev, torch.uint8, self.N, self.device)
        self._keep = [phase_dev]
        return self._check(self.lib.fh_set_phases(self.ptr, ptr, int(mat.shape[0]), _dptr(mat)))

    def set_conductivity_field(self, k_dev):
        ptr = _tptr(k_dev, _f64(), self.N, self.device)
        self._keep = [k_dev]
        return self._check(self.lib.fh_set_conductivity_field(self.ptr, ptr))

    def set_reference(self, Cref=None):
        if Cref is None:
            return self._check(self.lib.fh_set_reference(self.ptr, None))
        C = np.ascontiguousarray(Cref, dtype=np.float64)
        return self._check(self.lib.fh_set_reference(self.ptr, _dptr(C)))

    def set_load(self, E):
        E = np.ascontiguousarray(np.atleast_2d(E), dtype=np.float64)
        self.nload = E.shape[0]
        return self._check(self.lib.fh_set_load(self.ptr, E.shape[0], _dptr(E)))

    def workspace_size(self):
        b = ctypes.c_size_t()
        self._check(self.lib.fh_workspace_size(self.ptr, ctypes.byref(b)))
        return b.value

    def bind_workspace(self, buf=None):
        """Bind a torch uint8 CUDA tensor as the workspace (None: unbind)."""
        if buf is None:
            self._ws = None
            return self._check(self.lib.fh_bind_workspace(self.ptr, None, 0))
        import torch
        ptr = _tptr(buf, torch.uint8, None, self.device)
        self._ws = buf
        return self._check(self.lib.fh_bind_workspace(self.ptr, ptr, buf.numel()))

    # ----------------------------------------------------------------- solve
    @staticmethod
    def opts(eta=1e-10, itmax=10000, precision=FH_FP64, poll=0, eta_inner=0.0, flags=0):
        return fh_opts(eta, itmax, precision, poll, flags, eta_inner)

    def set_warm_start(self, net):
        """Attach a Net (None detaches) for solves with warm_start=True."""
        self._net = net
        return self._check(self.lib.fh_set_warm_start(self.ptr, net.ptr if net else None))

    def solve(self, eta=1e-10, itmax=10000, precision=FH_FP64, poll=0, eta_inner=0.0,
              time_kernels=False, rebuild=False, warm_start=False, guess_dev=None,
              time_sampled=False, graph=False):
        """graph: replay one captured PCG iteration from a hipGraph
        (FH_FLAG_GRAPH) instead of launching every kernel from the host."""
        flags = (FH_FLAG_TIME_KERNELS if time_kernels else 0) | \
            (FH_FLAG_REBUILD if rebuild else 0) | (FH_FLAG_WARM_START if warm_start else 0) | \
            (FH_FLAG_TIME_SAMPLED if time_sampled else 0) | (FH_FLAG_GRAPH if graph else 0)
        o = self.opts(eta, itmax, precision, poll, eta_inner, flags)
        if guess_dev is not None:
            o.guess_dev = _tptr(guess_dev, _f64(), self.nload * self.nd * self.N,
                                self.device).value
        st = fh_stats()
        rc = self._check(self.lib.fh_solve(self.ptr, ctypes.byref(o), ctypes.byref(st)),
                         allow_warning=True)
        return rc, st.as_dict()

    def get_fluctuation(self, load, out_dev):
        ptr = _tptr(out_dev, _f64(), self.nd * self.N, self.device)
        return self._check(self.lib.fh_get_fluctuation(self.ptr, load, ptr))

    def get_homogenized(self):
        H = np.zeros((self.nload, self.nload))
        self._check(self.lib.fh_get_homogenized(self.ptr, _dptr_out(H)))
        return H

    def get_reference(self):
        C = np.zeros((self.m, self.m))
        self._check(self.lib.fh_get_reference(self.ptr, _dptr_out(C)))
        return C

    def get_history(self, load):
        cnt = ctypes.c_int()
        self._check(self.lib.fh_get_history(self.ptr, load, None, 0, ctypes.byref(cnt)))
        h = np.zeros(max(cnt.value, 1))
        self._check(self.lib.fh_get_history(self.ptr, load, _dptr_out(h), cnt.value,
                                            ctypes.byref(cnt)))
        return h[:cnt.value]

    # ------------------------------------------------ strain-based scheme
    def solve_strain_based(self, eta=1e-10, itmax=10000):
        o = self.opts(eta, itmax, FH_FP64)
        st = fh_stats()
        rc = self._check(self.lib.fh_solve_strain_based(self.ptr, ctypes.byref(o),
                                                        ctypes.byref(st)), allow_warning=True)
        return rc, st.as_dict()

    def get_strain(self, load, eps_dev):
        ptr = _tptr(eps_dev, _f64(), 48 * self.N, self.device)
        return self._check(self.lib.fh_get_strain(self.ptr, int(load), ptr))

    # ------------------------------------------------ elasto-plastic Newton
    def set_plastic_phases(self, phase_dev, params):
        """params: (nphase, 4) = K, G, sy0, H per phase (fh_set_plastic_phases)."""
        import torch
        params = np.ascontiguousarray(params, dtype=np.float64)
        assert params.ndim == 2 and params.shape[1] == 4
        ptr = _tptr(phase_dev, torch.uint8, self.N, self.device)
        self._keep = [phase_dev]
        return self._check(self.lib.fh_set_plastic_phases(self.ptr, ptr, params.shape[0],
                                                          _dptr(params)))

    def newton_solve(self, E_final, nincrement=1, eta_newton=1e-8, eta_cg=1e-10,
                     itmax_newton=50, itmax_cg=10000, ref_mode=FH_NEWTON_REF_TANGENT):
        E = np.ascontiguousarray(E_final, dtype=np.float64)
        assert E.size == 6
        o = fh_newton_opts(eta_newton, eta_cg, itmax_newton, itmax_cg, nincrement, ref_mode)
        st = fh_newton_stats()
        rc = self._check(self.lib.fh_newton_solve(self.ptr, _dptr(E), ctypes.byref(o),
                                                  ctypes.byref(st)), allow_warning=True)
        return rc, st.as_dict()

    def get_plastic_state(self, u_dev=None, eps_p_dev=None, alpha_dev=None):
        N = self.N
        u = None if u_dev is None else _tptr(u_dev, _f64(), 3 * N, self.device)
        e = None if eps_p_dev is None else _tptr(eps_p_dev, _f64(), 48 * N, self.device)
        a = None if alpha_dev is None else _tptr(alpha_dev, _f64(), 8 * N, self.device)
        return self._check(self.lib.fh_get_plastic_state(self.ptr, u, e, a))

    # ---------------------------------------------------- eigenvalue bounds
    def eigen_bounds(self, Cref=None, eta=1e-6, lo_dev=None, hi_dev=None):
        """Guaranteed eigenvalue bounds (fh_eigen_bounds): dict with
        lambda_min, lambda_max, kappa and the predicted PCG iterations for
        eta; lo_dev / hi_dev (float64 tensors of N values, optional) receive
        the nodal bounds."""
        C = None if Cref is None else np.ascontiguousarray(Cref, dtype=np.float64)
        if C is not None:
            assert C.shape == (self.m, self.m)
        lo = None if lo_dev is None else _tptr(lo_dev, _f64(), self.N, self.device)
        hi = None if hi_dev is None else _tptr(hi_dev, _f64(), self.N, self.device)
        b = fh_bounds()
        self._check(self.lib.fh_eigen_bounds(self.ptr, None if C is None else _dptr(C),
                                             float(eta), lo, hi, ctypes.byref(b)))
        return b.as_dict()

    def choose_reference(self, strategy=FH_REF_BEST):
        """fh_choose_reference: returns (Cref, bounds dict); the choice
        becomes the context's reference."""
        C = np.zeros((self.m, self.m))
        b = fh_bounds()
        self._check(self.lib.fh_choose_reference(self.ptr, int(strategy), _dptr_out(C),
                                                 ctypes.byref(b)))
        return C, b.as_dict()

    # ----------------------------------------------------------- step hooks
    def _field(self, t):
        return _tptr(t, _f64(), self.nd * self.N, self.device)

    def apply_operator(self, u_dev, q_dev):
        return self._check(self.lib.fh_apply_operator(self.ptr, self._field(u_dev),
                                                      self._field(q_dev)))

    def apply_preconditioner(self, r_dev, z_dev):
        return self._check(self.lib.fh_apply_preconditioner(self.ptr, self._field(r_dev),
                                                            self._field(z_dev)))

    def compute_rhs(self, E, b_dev):
        E = np.ascontiguousarray(E, dtype=np.float64)
        assert E.size == self.m
        return self._check(self.lib.fh_compute_rhs(self.ptr, _dptr(E), self._field(b_dev)))

    def compute_rhs_noalloc(self, E, b_dev):
        """fh_compute_rhs without any device allocation (static staging)."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        assert E.size == self.m
        return self._check(self.lib.fh_compute_rhs_noalloc(self.ptr, _dptr(E),
                                                           self._field(b_dev)))

    def symbol_size(self):
        """Doubles written by get_symbol: nd(nd+1)/2 entries per frequency of
        the half spectrum (4 for the two-node stencil's Hermitian block)."""
        n = list(self.n) + [1] * (3 - len(self.n))
        nsym = 4 if self.element == "tri4" else self.nd * (self.nd + 1) // 2
        return nsym * (n[0] // 2 + 1) * n[1] * n[2]

    def get_symbol(self, kplus_dev):
        ptr = _tptr(kplus_dev, _f64(), self.symbol_size(), self.device)
        return self._check(self.lib.fh_get_symbol(self.ptr, ptr))

    def solve_rhs(self, b_dev, u_dev, eta=1e-10, itmax=10000, poll=0):
        o = self.opts(eta, itmax, FH_FP64, poll)
        st = fh_stats()
        rc = self._check(self.lib.fh_solve_rhs(self.ptr, self._field(b_dev), self._field(u_dev),
                                               ctypes.byref(o), ctypes.byref(st)),
                         allow_warning=True)
        return rc, st.as_dict()


    def _systems(self, systems, nload, u_out=None):
        mats = [np.ascontiguousarray(m, dtype=np.float64) for _, _, m in systems]
        arr = (fh_system * len(systems))()
        import torch
        for i, ((ph, n, _), m) in enumerate(zip(systems, mats)):
            arr[i].phase_dev = _tptr(ph, torch.uint8, int(np.prod(n)), self.device)
            arr[i].n = (ctypes.c_int * 3)(*[int(v) for v in n])
            arr[i].nphase = int(m.shape[0])
            arr[i].mat = _dptr(m)
            arr[i].u_dev = (_tptr(u_out[i], _f64(), nload * 3 * int(np.prod(n)),
                                  self.device).value
                            if u_out is not None and u_out[i] is not None else None)
        return arr, mats

    def batch_workspace_size(self, systems, nload):
        """fh_batch_workspace_size: device bytes fh_solve_batch takes from a
        bound workspace for these systems (list as for solve_batch)."""
        arr, _mats = self._systems(systems, nload)
        b = ctypes.c_size_t()
        self._check(self.lib.fh_batch_workspace_size(self.ptr, len(systems), arr, int(nload),
                                                     ctypes.byref(b)))
        return b.value

    def solve_batch(self, systems, E, eta=1e-6, itmax=10000, precision=FH_FP32_REFINED,
                    poll=0, eta_inner=0.0, u_out=None, serial=False):
        """systems: list of (phase_dev uint8 tensor, n (3,), mat (nphase, 6, 6)).
        u_out: optional list of float64 CUDA tensors (nload x 3 x N each) that
        receive the fluctuation fields.  serial: solve the grid-size groups
        one after another (FH_FLAG_BATCH_SERIAL) instead of concurrently.
        Returns (rc, chom (nsys, nload, nload), [stats dicts], [group reports])."""
        E = np.ascontiguousarray(np.atleast_2d(E), dtype=np.float64)
        nload = E.shape[0]
        arr, mats = self._systems(systems, nload, u_out)
        chom = np.zeros((len(systems), nload, nload))
        sts = (fh_stats * len(systems))()
        rep = fh_batch_report()
        o = self.opts(eta, itmax, precision, poll, eta_inner,
                      FH_FLAG_BATCH_SERIAL if serial else 0)
        rc = self._check(self.lib.fh_solve_batch(self.ptr, len(systems), arr, nload, _dptr(E),
                                                 ctypes.byref(o), _dptr_out(chom), sts,
                                                 ctypes.byref(rep)), allow_warning=True)
        return rc, chom, [x.as_dict() for x in sts], rep.as_dict()


def _dptr_out(arr):
    assert arr.dtype == np.float64 and arr.flags.c_contiguous
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# C-ABI names as module-level functions (same names as include/fh.h)
def fh_create(device=0):
    return Context(device)


class Net:
    """Owns one fh_net (learned warm start, include/fh_net.h)."""

    def __init__(self, n: int = 64, max_batch: int = 8, device: int = 0):
        self.lib = load_library()
        self.ptr = ctypes.c_void_p()
        rc = self.lib.fh_net_create(ctypes.byref(self.ptr), device, int(n), int(max_batch))
        if rc != FH_OK:
            raise FHError(rc, f"fh_net_create(n={n}, max_batch={max_batch}) failed")
        self.n, self.max_batch, self.device = n, max_batch, device
        self.P = int(self.lib.fh_net_param_count())

    def _check(self, rc):
        if rc != FH_OK:
            raise FHError(rc, self.lib.fh_net_last_error(self.ptr).decode())
        return rc

    def close(self):
        if self.ptr:
            self.lib.fh_net_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _f32(a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))

    def set_stream(self, stream):
        raw = getattr(stream, "cuda_stream", stream)
        return self._check(self.lib.fh_net_set_stream(self.ptr, ctypes.c_void_p(raw)))

    def set_params(self, params):
        a, p = self._f32(params)
        assert a.size == self.P
        return self._check(self.lib.fh_net_set_params(self.ptr, p))

    def get_params(self):
        a, p = self._f32(np.zeros(self.P))
        self._check(self.lib.fh_net_get_params(self.ptr, p))
        return a

    def forward(self, phase_dev, gamma, out_dev):
        g, gp = self._f32(gamma)
        import torch
        V, b = self.n ** 3, int(g.size)
        return self._check(self.lib.fh_net_forward(
            self.ptr, b, _tptr(phase_dev, torch.uint8, b * V, self.device), gp,
            _tptr(out_dev, torch.float32, b * 18 * V, self.device)))

    def gradient(self, phase_dev, gamma, target_dev):
        g, gp = self._f32(gamma)
        loss = ctypes.c_double()
        grad, grp = self._f32(np.zeros(self.P))
        import torch
        V, b = self.n ** 3, int(g.size)
        self._check(self.lib.fh_net_gradient(
            self.ptr, b, _tptr(phase_dev, torch.uint8, b * V, self.device), gp,
            _tptr(target_dev, _BF16_CARRIERS(), b * 18 * V, self.device), ctypes.byref(loss),
            grp))
        return loss.value, grad

    def adam(self, grad=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, clip=0.0):
        o = fh_adam(lr, beta1, beta2, eps, clip)
        if grad is None:
            return self._check(self.lib.fh_net_adam(self.ptr, None, ctypes.byref(o)))
        a, p = self._f32(grad)
        return self._check(self.lib.fh_net_adam(self.ptr, p, ctypes.byref(o)))

    def train(self, phase_dev, gamma, target_dev, order, batch, lr=1e-3, beta1=0.9,
              beta2=0.999, eps=1e-8, clip=0.0):
        """order: int array (steps, batch) of sample indices.  Returns the
        loss of every step."""
        order = np.ascontiguousarray(order, dtype=np.int32)
        steps = order.shape[0]
        g, gp = self._f32(gamma)
        loss = np.zeros(max(steps, 1))
        o = fh_adam(lr, beta1, beta2, eps, clip)
        self._check(self.lib.fh_net_train(
            self.ptr, int(g.size),
            _tptr(phase_dev, _U8(), int(g.size) * self.n ** 3, self.device), gp,
            _tptr(target_dev, _BF16_CARRIERS(), int(g.size) * 18 * self.n ** 3, self.device),
            int(batch),
            int(steps), order.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(o),
            _dptr_out(loss)))
        return loss[:steps]

    def guess(self, phase_dev, gamma, E, length, x_dev):
        E = np.ascontiguousarray(np.atleast_2d(E), dtype=np.float64)
        V = self.n ** 3
        return self._check(self.lib.fh_net_guess(
            self.ptr, _tptr(phase_dev, _U8(), V, self.device), float(gamma), E.shape[0],
            _dptr(E), float(length), _tptr(x_dev, _f64(), E.shape[0] * 3 * V, self.device)))

    def pack_target(self, u_dev, scale, target_dev):
        V = self.n ** 3
        return self._check(self.lib.fh_net_pack_target(
            self.ptr, _tptr(u_dev, _f64(), 18 * V, self.device), float(scale),
            _tptr(target_dev, _BF16_CARRIERS(), 18 * V, self.device)))

    LAYERS = [(3, 16, 0), (16, 16, 0), (16, 32, 1), (32, 32, 1), (32, 64, 2), (64, 64, 2),
              (64, 64, 3), (64, 64, 3), (128, 64, 2), (64, 64, 2), (96, 32, 1), (32, 32, 1),
              (48, 16, 0), (16, 16, 0)]  # (cin, cout, level), the header's layer order

    def layer(self, layer, op, batch, x=None, dz=None, mask=None, out=None):
        """fh_net_layer: op 0 forward, 1 input gradient, 2 weight gradient.
        BF16 tensors are torch int16/uint16 carriers (channels last)."""
        cin, cout, lev = self.LAYERS[layer]
        V = (self.n >> lev) ** 3
        cinp = (cin + 15) // 16 * 16
        need_out = {0: batch * V * cout, 1: batch * V * cinp, 2: 27 * cin * cout + cout}[op]
        import torch
        odt = torch.float32 if op == 2 else _BF16_CARRIERS()
        xp = None if x is None else _tptr(x, _BF16_CARRIERS(), batch * V * cinp, self.device)
        dp = None if dz is None else _tptr(dz, _BF16_CARRIERS(), batch * V * cout, self.device)
        mp = None if mask is None else _tptr(mask, _BF16_CARRIERS(), batch * V * cinp,
                                             self.device)
        op_ = _tptr(out, odt, need_out, self.device)
        return self._check(self.lib.fh_net_layer(self.ptr, int(layer), int(op), int(batch), xp, dp,
                                                 mp, op_))

    def set_timing(self, on=True):
        return self._check(self.lib.fh_net_set_timing(self.ptr, 1 if on else 0))

    def stats(self):
        st = fh_net_stats()
        self._check(self.lib.fh_net_get_stats(self.ptr, ctypes.byref(st)))
        return st.as_dict()
