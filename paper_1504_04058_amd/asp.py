"""Python binding of libasp.so (the C ABI of include/asp.h).

Argument marshalling only: every step of the method runs inside the HIP
library.  Functions carry the C names; device vectors are passed as torch
tensors (complex128, on the GPU) or raw device addresses.  torch is imported
first so that the library binds to the HIP runtime torch already loaded.
"""
import ctypes
import os
import re

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libasp.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "asp.h")

ASP_OK, ASP_ERR_ARG, ASP_ERR_OOM, ASP_ERR_STATE = 0, 1, 2, 3
ASP_ERR_BREAKDOWN, ASP_ERR_NOCONV, ASP_ERR_DEVICE = 4, 5, 6
ASP_PREC_FP64, ASP_PREC_FP32, ASP_PREC_BF16X3 = 0, 1, 2
ASP_SUB_M, ASP_SUB_R, ASP_SUB_L = 0, 1, 2
ASP_FACT3D_ND, ASP_FACT3D_BLOCKS, ASP_FACT3D_RECURSIVE = 0, 1, 2
ASP_SWEEP2D_MAPS, ASP_SWEEP2D_SEQUENTIAL = 0, 1
STATUS_NAMES = {0: "ASP_OK", 1: "ASP_ERR_ARG", 2: "ASP_ERR_OOM", 3: "ASP_ERR_STATE",
                4: "ASP_ERR_BREAKDOWN", 5: "ASP_ERR_NOCONV", 6: "ASP_ERR_DEVICE"}


class AspError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class asp_opts(ctypes.Structure):
    _fields_ = [("C", ctypes.c_double), ("prec", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("host_only", ctypes.c_int), ("pml_aux", ctypes.c_int),
                ("n_layers", ctypes.c_int), ("layer_widths", ctypes.POINTER(ctypes.c_int)),
                ("fact3d", ctypes.c_int), ("sweep2d", ctypes.c_int)]


class asp_plan_info(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("m", ctypes.c_int),
                ("n_sub", ctypes.c_int), ("max_lines", ctypes.c_int),
                ("factor_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
                ("factored", ctypes.c_int), ("factor_work_bytes", ctypes.c_size_t)]


_lib = None


def declared_functions():
    """Names of the functions include/asp.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(asp_[a-z_]+)\s*\(", text)))


def lib():
    """Load libasp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1504_04058_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, D, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, None
        sig = {
            "asp_default_opts": (V, [ctypes.POINTER(asp_opts)]),
            "asp_setup": (I, [ctypes.POINTER(P), I, P, D, I, I, I, ctypes.POINTER(asp_opts)]),
            "asp_factor": (I, [P]),
            "asp_apply": (I, [P, P, P, I]),
            "asp_apply_noalloc": (I, [P, P, P, I]),
            "asp_matvec": (I, [P, P, P, I]),
            "asp_gmres": (I, [P, P, P, I, D, I, I, P, P]),
            "asp_subsolve": (I, [P, I, I, P, P, I]),
            "asp_layers": (I, [P, P, P, P]),
            "asp_tables": (I, [P, I, P, P]),
            "asp_info": (I, [P, ctypes.POINTER(asp_plan_info)]),
            "asp_set_stream": (I, [P, P]),
            "asp_destroy": (V, [P]),
            "asp_last_error": (ctypes.c_char_p, [P]),
            "asp_timing_enable": (I, [P, I]),
            "asp_timing_read": (I, [P, I, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
            "asp_workspace_estimate": (I, [P, I, I, ctypes.POINTER(ctypes.c_size_t)]),
            "asp_release_workspace": (I, [P]),
            "asp_set_cache_limit": (ctypes.c_size_t, [ctypes.c_size_t]),
            "asp_cached_bytes": (ctypes.c_size_t, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(x):
    """Device address of a tensor (complex128, CUDA, contiguous) or an int."""
    if isinstance(x, torch.Tensor):
        if not x.is_cuda:
            raise ValueError("device vectors must be CUDA tensors")
        if x.dtype != torch.complex128:
            raise ValueError("device vectors must be complex128")
        if not x.is_contiguous():
            raise ValueError("device vectors must be contiguous")
        return ctypes.c_void_p(x.data_ptr())
    return ctypes.c_void_p(int(x))


def _check(plan, status):
    if status != ASP_OK:
        raise AspError(status, asp_last_error(plan))


def _current_stream():
    if torch.cuda.is_available():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(0)


# -- the C entry points --------------------------------------------------------------

def asp_setup(dim, c, omega, n, layer_b, pml_eta, C=25.0, prec=ASP_PREC_FP64, stream=None,
              host_only=False, pml_aux=0, nd3d=True, fact3d=None, sweep2d=ASP_SWEEP2D_MAPS):
    """Returns a plan handle (ctypes.c_void_p).  c: host array, n**dim velocities
    (column-major, i.e. numpy order='F' flattening of an (n,)*dim array).
    layer_b: lines per layer, or a sequence of physical lines per layer
    (arbitrary widths: opts.n_layers / opts.layer_widths).  fact3d: an
    ASP_FACT3D_* value; None takes nested dissection (nd3d) or the blocks."""
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(-1, order="F")
                             if np.asarray(c).ndim > 1 else np.asarray(c, dtype=np.float64))
    opts = asp_opts(C, prec, stream if stream is not None else
                    (ctypes.c_void_p(0) if host_only else _current_stream()), int(host_only),
                    int(pml_aux or 0), 0, None,
                    fact3d if fact3d is not None else (ASP_FACT3D_ND if nd3d else ASP_FACT3D_BLOCKS),
                    int(sweep2d))
    if not isinstance(layer_b, (int, np.integer)):
        widths = (ctypes.c_int * len(layer_b))(*[int(w) for w in layer_b])
        opts.n_layers = len(layer_b)
        opts.layer_widths = widths
        layer_b = 0
    plan = ctypes.c_void_p()
    st = lib().asp_setup(ctypes.byref(plan), dim, c.ctypes.data_as(ctypes.c_void_p), omega, n,
                         int(layer_b), pml_eta, ctypes.byref(opts))
    if st != ASP_OK:
        msg = asp_last_error(plan)
        asp_destroy(plan)
        raise AspError(st, msg)
    return plan


def asp_factor(plan):
    _check(plan, lib().asp_factor(plan))


def asp_apply(plan, r, z, nrhs):
    _check(plan, lib().asp_apply(plan, _ptr(r), _ptr(z), nrhs))


def asp_apply_noalloc(plan, r, z, nrhs):
    _check(plan, lib().asp_apply_noalloc(plan, _ptr(r), _ptr(z), nrhs))


def asp_matvec(plan, x, y, nrhs):
    _check(plan, lib().asp_matvec(plan, _ptr(x), _ptr(y), nrhs))


def asp_gmres(plan, f, u, nrhs, tol, restart, maxit):
    """Returns (status, iters[nrhs], relres[nrhs]); ASP_ERR_NOCONV is returned, not raised."""
    iters = np.zeros(nrhs, dtype=np.int32)
    relres = np.zeros(nrhs, dtype=np.float64)
    st = lib().asp_gmres(plan, _ptr(f), _ptr(u), nrhs, tol, restart, maxit,
                         iters.ctypes.data_as(ctypes.c_void_p), relres.ctypes.data_as(ctypes.c_void_p))
    if st not in (ASP_OK, ASP_ERR_NOCONV):
        raise AspError(st, asp_last_error(plan))
    return st, iters, relres


def asp_subsolve(plan, kind, p, inp, out, nrhs):
    _check(plan, lib().asp_subsolve(plan, kind, p, _ptr(inp), _ptr(out), nrhs))


def asp_layers(plan):
    """Returns (layers [m,2], subs [3m-2,6]) as int arrays."""
    m = ctypes.c_int()
    _check(plan, lib().asp_layers(plan, ctypes.byref(m), None, None))
    layers = np.zeros((m.value, 2), dtype=np.int32)
    subs = np.zeros((max(3 * m.value - 2, 0), 6), dtype=np.int32)
    _check(plan, lib().asp_layers(plan, ctypes.byref(m), layers.ctypes.data_as(ctypes.c_void_p),
                                  subs.ctypes.data_as(ctypes.c_void_p)))
    return layers, subs


def asp_tables(plan, sub, length):
    """(s_int[length], s_half[length+1]) complex arrays of one PML table."""
    s_int = np.zeros(2 * length, dtype=np.float64)
    s_half = np.zeros(2 * (length + 1), dtype=np.float64)
    _check(plan, lib().asp_tables(plan, sub, s_int.ctypes.data_as(ctypes.c_void_p),
                                  s_half.ctypes.data_as(ctypes.c_void_p)))
    return s_int.view(np.complex128), s_half.view(np.complex128)


def asp_info(plan):
    info = asp_plan_info()
    _check(plan, lib().asp_info(plan, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in asp_plan_info._fields_}


def asp_workspace_estimate(plan, nrhs, restart):
    b = ctypes.c_size_t()
    _check(plan, lib().asp_workspace_estimate(plan, nrhs, restart, ctypes.byref(b)))
    return b.value


def asp_release_workspace(plan):
    _check(plan, lib().asp_release_workspace(plan))


def asp_set_cache_limit(nbytes):
    """Device bytes the library may keep for reuse per device; returns the
    previous limit."""
    return int(lib().asp_set_cache_limit(int(nbytes)))


def asp_cached_bytes():
    return int(lib().asp_cached_bytes())


def asp_timing_enable(plan, enable):
    _check(plan, lib().asp_timing_enable(plan, int(enable)))


def asp_timing_read(plan, cls):
    """(launches, ms, bytes, flops) of one kernel class."""
    nl, ms = ctypes.c_int(), ctypes.c_double()
    by, fl = ctypes.c_double(), ctypes.c_double()
    _check(plan, lib().asp_timing_read(plan, cls, ctypes.byref(nl), ctypes.byref(ms),
                                       ctypes.byref(by), ctypes.byref(fl)))
    return nl.value, ms.value, by.value, fl.value


def asp_set_stream(plan, stream):
    _check(plan, lib().asp_set_stream(plan, ctypes.c_void_p(stream)))


def asp_destroy(plan):
    if plan is not None and plan.value:
        lib().asp_destroy(plan)


def asp_last_error(plan):
    msg = lib().asp_last_error(plan)
    return msg.decode() if msg else ""


class Plan:
    """Owning wrapper around a plan handle (destroyed with the object)."""

    def __init__(self, dim, c, omega, n, layer_b, pml_eta, C=25.0, prec=ASP_PREC_FP64,
                 host_only=False, pml_aux=0, nd3d=True, fact3d=None, sweep2d=ASP_SWEEP2D_MAPS):
        self.dim, self.n = dim, n
        self.N = n ** dim
        self.handle = asp_setup(dim, c, omega, n, layer_b, pml_eta, C=C, prec=prec,
                                host_only=host_only, pml_aux=pml_aux, nd3d=nd3d, fact3d=fact3d,
                                sweep2d=sweep2d)

    def close(self):
        if getattr(self, "handle", None) is not None:
            asp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def factor(self):
        asp_factor(self.handle)
        return self

    def apply(self, r):
        r = r.contiguous()
        z = torch.empty_like(r)
        asp_apply(self.handle, r, z, r.numel() // self.N)
        return z

    def apply_noalloc(self, r, z):
        """z = M^-1 r into the caller's z (same shape as r), allocating nothing."""
        asp_apply_noalloc(self.handle, r, z, r.numel() // self.N)
        return z

    def matvec(self, x):
        x = x.contiguous()
        y = torch.empty_like(x)
        asp_matvec(self.handle, x, y, x.numel() // self.N)
        return y

    def gmres(self, f, tol=1e-6, restart=20, maxit=200):
        f = f.contiguous()
        u = torch.empty_like(f)
        st, it, rr = asp_gmres(self.handle, f, u, f.numel() // self.N, tol, restart, maxit)
        return u, it, rr, st

    def subsolve(self, kind, p, inp, out_numel):
        nrhs = inp.shape[0] if inp.dim() > 1 else 1
        out = torch.empty(out_numel * nrhs, dtype=torch.complex128, device=inp.device)
        asp_subsolve(self.handle, kind, p, inp.contiguous(), out, nrhs)
        return out

    def layers(self):
        return asp_layers(self.handle)

    def info(self):
        return asp_info(self.handle)
