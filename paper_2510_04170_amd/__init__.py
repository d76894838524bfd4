"""Python binding of librfmnewton.so (C ABI in include/rfm.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Arrays may be numpy (host) arrays or torch device tensors; torch is
used only for device memory and stream handles.  The library must have been
built (``python -m paper_2510_04170_amd.build``); importing ``lib()`` without it
raises instead of falling back to anything else.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librfmnewton.so")

RFM_OK, RFM_EINVAL, RFM_ENOMEM, RFM_EDEVICE, RFM_ESINGULAR, RFM_ENUMERIC = 0, -1, -2, -3, -4, -5
RFM_ENOCONV, RFM_ESTALL = 1, 2
RFM_PDE, RFM_DIRICHLET, RFM_NEUMANN, RFM_CONTINUITY = 0, 1, 2, 3
RFM_IPN, RFM_AMIPN = 0, 1
RFM_PREC_F64, RFM_PREC_F32, RFM_PREC_BF16, RFM_PREC_FP8 = 0, 1, 2, 3
RFM_SKETCH_GAUSSIAN, RFM_SKETCH_COUNT = 0, 1
RFM_FN_COSH, RFM_FN_SINH, RFM_FN_EXP = 0, 1, 2
RFM_POU_INDICATOR, RFM_POU_SMOOTH = 0, 1
RFM_EVAL_VALUE, RFM_EVAL_GRAD = 0, 1
_FN_CODE = {"cosh": RFM_FN_COSH, "sinh": RFM_FN_SINH, "exp": RFM_FN_EXP}
RFM_MAX_STEPS = 64


class rfm_lin_term(C.Structure):
    _fields_ = [("eq", C.c_int32), ("comp", C.c_int32), ("coeff", C.c_double), ("deriv", C.c_int32)]


class rfm_poly_term(C.Structure):
    _fields_ = [("eq", C.c_int32), ("coeff", C.c_double), ("pow", C.c_int32 * 4)]


class rfm_fn_term(C.Structure):
    _fields_ = [("eq", C.c_int32), ("comp", C.c_int32), ("coeff", C.c_double), ("fn", C.c_int32)]


class rfm_factor(C.Structure):
    _fields_ = [("comp", C.c_int32), ("deriv", C.c_int32), ("pow", C.c_int32)]


class rfm_prod_term(C.Structure):
    _fields_ = [("eq", C.c_int32), ("coeff", C.c_double), ("nfac", C.c_int32), ("fac", rfm_factor * 4)]


class rfm_solve_opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("sketch_factor", C.c_double), ("sketch_seed", C.c_uint64),
                ("lsqr_tol", C.c_double), ("lsqr_max_iter", C.c_int32), ("outer_tol", C.c_double),
                ("max_outer", C.c_int32), ("m_max", C.c_int32), ("tau_rel", C.c_double),
                ("row_scale_c", C.c_double), ("gs_iters", C.c_int32), ("sketch_prec", C.c_int32),
                ("lsqr_prec", C.c_int32), ("sketch_pieces", C.c_int32), ("sketch_kind", C.c_int32),
                ("verbose", C.c_int32), ("sketch_rows_per_pass", C.c_int32), ("jac_index0", C.c_int32)]


class rfm_solve_stats(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("jac_evals", C.c_int32), ("lsqr_iters_total", C.c_int32),
                ("nsteps", C.c_int32), ("lsqr_iters", C.c_int32 * RFM_MAX_STEPS),
                ("alphas", C.c_double * RFM_MAX_STEPS), ("resnorms", C.c_double * RFM_MAX_STEPS),
                ("final_resnorm", C.c_double), ("t_assemble", C.c_double), ("t_sketch", C.c_double),
                ("t_qr", C.c_double), ("t_lsqr", C.c_double), ("t_linesearch", C.c_double),
                ("t_total", C.c_double), ("status_detail", C.c_int32), ("lsqr_fp64_fallback", C.c_int32),
                ("inner_steps", C.c_int32 * RFM_MAX_STEPS), ("flags", C.c_int32 * RFM_MAX_STEPS)]

    def as_dict(self) -> dict:
        k = min(self.nsteps, RFM_MAX_STEPS)
        ko = min(self.outer_iters, RFM_MAX_STEPS)
        return dict(outer_iters=self.outer_iters, jac_evals=self.jac_evals, lsqr_iters_total=self.lsqr_iters_total,
                    nsteps=self.nsteps, lsqr_iters=list(self.lsqr_iters[:k]), alphas=list(self.alphas[:k]),
                    resnorms=list(self.resnorms[:k]), final_resnorm=self.final_resnorm,
                    t_assemble=self.t_assemble, t_sketch=self.t_sketch, t_qr=self.t_qr, t_lsqr=self.t_lsqr,
                    t_linesearch=self.t_linesearch, t_total=self.t_total, status=self.status_detail,
                    lsqr_fp64_fallback=self.lsqr_fp64_fallback, inner_steps=list(self.inner_steps[:ko]),
                    flags=[bool(f) for f in self.flags[:ko]])


class rfm_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("seconds", C.c_double), ("flops", C.c_double),
                ("bytes", C.c_double)]


class rfm_train_opts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("lr_final", C.c_float), ("seed", C.c_uint64)]


class RfmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rfm status {status}: {msg}")
        self.status = status


_lib = None

_P = C.c_void_p
_D = C.c_void_p  # double* (host or device)
_SIGS = {
    "rfm_last_error": (C.c_char_p, []),
    "rfm_create": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, C.c_int32, C.c_void_p]),
    "rfm_destroy": (None, [_P]),
    "rfm_set_partition": (C.c_int, [_P, _D, _D, _D]),
    "rfm_set_features": (C.c_int, [_P, C.c_int32, _D, _D]),
    "rfm_add_points": (C.c_int, [_P, C.c_int32, C.c_int64, _D, C.c_int32, C.c_int32, _D, C.c_int32, C.c_int32, _D]),
    "rfm_set_operator": (C.c_int, [_P, C.POINTER(rfm_lin_term), C.c_int32, C.POINTER(rfm_poly_term), C.c_int32]),
    "rfm_set_fn_terms": (C.c_int, [_P, C.POINTER(rfm_fn_term), C.c_int32]),
    "rfm_set_prod_terms": (C.c_int, [_P, C.POINTER(rfm_prod_term), C.c_int32]),
    "rfm_set_partition_of_unity": (C.c_int, [_P, C.c_int32]),
    "rfm_finalize": (C.c_int, [_P]),
    "rfm_set_group_data": (C.c_int, [_P, C.c_int32, _D]),
    "rfm_num_unknowns": (C.c_int64, [_P]),
    "rfm_num_rows": (C.c_int64, [_P]),
    "rfm_num_jacobian_values": (C.c_int64, [_P]),
    "rfm_solve_opts_default": (None, [C.POINTER(rfm_solve_opts)]),
    "rfm_solve": (C.c_int, [_P, C.POINTER(rfm_solve_opts), _D, C.POINTER(rfm_solve_stats)]),
    "rfm_residual": (C.c_int, [_P, _D, _D, C.POINTER(C.c_double)]),
    "rfm_eval": (C.c_int, [_P, _D, C.c_int64, _D, _D, C.c_int32, _D]),
    "rfm_stage_assemble": (C.c_int, [_P, _D, C.c_double]),
    "rfm_get_scaled_residual": (C.c_int, [_P, _D]),
    "rfm_get_row_scale": (C.c_int, [_P, _D]),
    "rfm_get_jacobian_rows": (C.c_int, [_P, C.c_int64, C.c_int64, _D]),
    "rfm_jmul": (C.c_int, [_P, _D, _D]),
    "rfm_jtmul": (C.c_int, [_P, _D, _D]),
    "rfm_jtmul_noalloc": (C.c_int, [_P, _D, _D]),
    "rfm_stage_sketch": (C.c_int, [_P, C.c_double, C.c_uint64, C.c_uint64, C.c_int32, C.c_int32]),
    "rfm_sketch_table": (C.c_int, [C.c_int32, _D]),
    "rfm_stage_count_sketch": (C.c_int, [_P, C.c_double, C.c_uint64, C.c_uint64]),
    "rfm_sketch_operand_slots": (C.c_int64, [_P, C.c_int32]),
    "rfm_get_sketch_operand": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int64, C.c_int64, _D, C.c_void_p,
                                         C.c_void_p]),
    "rfm_get_sketch_cols": (C.c_int, [_P, C.c_int64, C.c_int64, _D]),
    "rfm_sketch_rows": (C.c_int64, [_P]),
    "rfm_stage_qr": (C.c_int, [_P]),
    "rfm_stage_sketch_qr_streamed": (C.c_int, [_P, C.c_double, C.c_uint64, C.c_uint64, C.c_int32, C.c_int32,
                                               C.c_int64]),
    "rfm_stage_count_sketch_qr_streamed": (C.c_int, [_P, C.c_double, C.c_uint64, C.c_uint64, C.c_int64]),
    "rfm_get_r_cols": (C.c_int, [_P, C.c_int64, C.c_int64, _D]),
    "rfm_r_solve": (C.c_int, [_P, _D, _D]),
    "rfm_rt_solve": (C.c_int, [_P, _D, _D]),
    "rfm_stage_lsqr": (C.c_int, [_P, _D, C.c_double, C.c_int32, C.c_int32, _D, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32)]),
    "rfm_stage_linesearch": (C.c_int, [_P, _D, _D, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "rfm_mlp_create": (C.c_int, [C.POINTER(_P), C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint64, C.c_int32,
                                 C.c_void_p]),
    "rfm_mlp_destroy": (None, [_P]),
    "rfm_mlp_num_params": (C.c_int64, [_P]),
    "rfm_mlp_get_params": (C.c_int, [_P, C.c_void_p]),
    "rfm_mlp_set_params": (C.c_int, [_P, C.c_void_p]),
    "rfm_mlp_set_precision": (C.c_int, [_P, C.c_int32]),
    "rfm_mlp_predict": (C.c_int, [_P, C.c_void_p, C.c_int64, C.c_void_p]),
    "rfm_mlp_loss_grad": (C.c_int, [_P, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_double), C.c_void_p]),
    "rfm_train_opts_default": (None, [C.POINTER(rfm_train_opts)]),
    "rfm_mlp_train": (C.c_int, [_P, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(rfm_train_opts), C.c_void_p]),
    "rfm_num_pde_points": (C.c_int64, [_P]),
    "rfm_get_pde_points": (C.c_int, [_P, _D, C.c_void_p]),
    "rfm_project": (C.c_int, [_P, C.POINTER(rfm_solve_opts), _D, _D, C.POINTER(C.c_double)]),
    "rfm_warm_inputs": (C.c_int, [_P, _D, _D, _D, C.c_int32, C.c_void_p]),
    "rfm_warm_start": (C.c_int, [_P, _P, C.POINTER(rfm_solve_opts), _D, _D, _D, C.c_int32, _D, _D]),
    "rfm_profile_enable": (C.c_int, [_P, C.c_int32]),
    "rfm_profile_read": (C.c_int32, [_P, C.POINTER(rfm_kernel_stat), C.c_int32]),
}


def lib():
    """Load librfmnewton.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2510_04170_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise RfmError(rc, lib().rfm_last_error().decode())
    return rc


def _ptr(a) -> Tuple[int, object]:
    """Pointer of a host numpy array (made float64/C-contiguous) or a torch tensor."""
    if a is None:
        return None, None
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), a
    return a.ctypes.data, a


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def sketch_table(prec: int) -> np.ndarray:
    """The 256 table values of the low-precision sketch (host only)."""
    out = np.zeros(256)
    _check(lib().rfm_sketch_table(prec, out.ctypes.data))
    return out


def train_opts(**kw) -> rfm_train_opts:
    o = rfm_train_opts()
    lib().rfm_train_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


# Handles still open when the interpreter exits are closed by an exit hook, while the HIP runtime is
# still up (finalizers that run later, during interpreter teardown, would destroy them after it).
_open_handles: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_open_handles():
    for obj in list(_open_handles):
        try:
            obj.close()
        except Exception:
            pass


class RfmMLP:
    """An rfm_mlp handle: in_dim -> width (tanh) x depth -> out_dim."""

    def __init__(self, in_dim: int, width: int, depth: int, out_dim: int, seed: int = 1, device: int = 0,
                 stream: Optional[int] = None):
        h = _P()
        _check(lib().rfm_mlp_create(C.byref(h), in_dim, width, depth, out_dim, seed, device, stream))
        self.h = h
        _open_handles.add(self)
        self.in_dim, self.width, self.depth, self.out_dim = in_dim, width, depth, out_dim

    def close(self):
        if getattr(self, "h", None):
            lib().rfm_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(lib().rfm_mlp_num_params(self.h))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.num_params, np.float32)
        _check(lib().rfm_mlp_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, p):
        p = _f32(p)
        assert p.size == self.num_params
        _check(lib().rfm_mlp_set_params(self.h, p.ctypes.data))

    def set_precision(self, prec: int):
        _check(lib().rfm_mlp_set_precision(self.h, prec))

    def predict(self, X) -> np.ndarray:
        X = _f32(X)
        Y = np.zeros((X.shape[0], self.out_dim), np.float32)
        _check(lib().rfm_mlp_predict(self.h, X.ctypes.data, X.shape[0], Y.ctypes.data))
        return Y

    def loss_grad(self, X, Y):
        X, Y = _f32(X), _f32(Y)
        loss = C.c_double()
        g = np.zeros(self.num_params, np.float32)
        _check(lib().rfm_mlp_loss_grad(self.h, X.ctypes.data, Y.ctypes.data, X.shape[0], C.byref(loss),
                                       g.ctypes.data))
        return loss.value, g

    def train(self, X, Y, **kw) -> np.ndarray:
        X, Y = _f32(X), _f32(Y)
        o = train_opts(**kw)
        log = np.zeros(max(o.steps, 1))
        _check(lib().rfm_mlp_train(self.h, X.ctypes.data, Y.ctypes.data, X.shape[0], C.byref(o), log.ctypes.data))
        return log[:o.steps]


def default_opts(**kw) -> rfm_solve_opts:
    o = rfm_solve_opts()
    lib().rfm_solve_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


class RfmProblem:
    """An rfm_problem handle; the library owns all device memory behind it."""

    def __init__(self, dim: int, ncomp: int, device: int = 0, stream: Optional[int] = None):
        h = _P()
        _check(lib().rfm_create(C.byref(h), dim, ncomp, device, stream))
        self.h = h
        _open_handles.add(self)
        self.dim, self.ncomp = dim, ncomp
        self.J = 0

    def close(self):
        if getattr(self, "h", None):
            lib().rfm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- description -------------------------------------------------------------
    def set_partition(self, lo, hi, nsub):
        lo, hi = _f64(lo), _f64(hi)
        ns = np.ascontiguousarray(nsub, dtype=np.int32)
        _check(lib().rfm_set_partition(self.h, lo.ctypes.data, hi.ctypes.data, ns.ctypes.data))

    def set_features(self, J: int, W, b):
        W, b = _f64(W), _f64(b)
        _check(lib().rfm_set_features(self.h, J, W.ctypes.data, b.ctypes.data))
        self.J = int(J)

    def add_points(self, kind, x, owner, neighbor=-1, normal=None, comp=-1, cont_order=1, data=None):
        x = _f64(x)
        nrm = None if normal is None else _f64(normal)
        dat = None if data is None else _f64(data)
        _check(lib().rfm_add_points(self.h, kind, x.shape[0], x.ctypes.data, int(owner), int(neighbor),
                                    None if nrm is None else nrm.ctypes.data, int(comp), int(cont_order),
                                    None if dat is None else dat.ctypes.data))

    def set_operator(self, lin_terms, poly_terms):
        L = (rfm_lin_term * max(1, len(lin_terms)))()
        for i, (eq, comp, coeff, deriv) in enumerate(lin_terms):
            L[i] = rfm_lin_term(eq, comp, coeff, deriv)
        Pt = (rfm_poly_term * max(1, len(poly_terms)))()
        for i, (eq, coeff, pw) in enumerate(poly_terms):
            p4 = (C.c_int32 * 4)(*(list(pw) + [0] * (4 - len(pw))))
            Pt[i] = rfm_poly_term(eq, coeff, p4)
        _check(lib().rfm_set_operator(self.h, L, len(lin_terms), Pt, len(poly_terms)))

    def set_fn_terms(self, fn_terms):
        """Pointwise terms (eq, comp, coeff, 'cosh' | 'sinh' | 'exp' or an RFM_FN_* code)."""
        T = (rfm_fn_term * max(1, len(fn_terms)))()
        for i, (eq, comp, coeff, fn) in enumerate(fn_terms):
            T[i] = rfm_fn_term(eq, comp, coeff, _FN_CODE[fn] if isinstance(fn, str) else int(fn))
        _check(lib().rfm_set_fn_terms(self.h, T, len(fn_terms)))

    def set_partition_of_unity(self, kind):
        """RFM_POU_INDICATOR (or "a") or RFM_POU_SMOOTH (or "b"); before finalize."""
        k = {"a": RFM_POU_INDICATOR, "b": RFM_POU_SMOOTH}.get(kind, kind)
        _check(lib().rfm_set_partition_of_unity(self.h, int(k)))

    def set_prod_terms(self, prod_terms):
        """Product terms (eq, coeff, ((comp, deriv, power), ...)) with 1..4 factors each."""
        T = (rfm_prod_term * max(1, len(prod_terms)))()
        for i, (eq, coeff, facs) in enumerate(prod_terms):
            if not 1 <= len(facs) <= 4:
                raise ValueError("a product term has 1..4 factors")
            fac = (rfm_factor * 4)(*[rfm_factor(int(c), int(d), int(p)) for (c, d, p) in facs])
            T[i] = rfm_prod_term(eq, coeff, len(facs), fac)
        _check(lib().rfm_set_prod_terms(self.h, T, len(prod_terms)))

    def finalize(self):
        _check(lib().rfm_finalize(self.h))

    def set_group_data(self, group: int, data):
        data = _f64(data)
        _check(lib().rfm_set_group_data(self.h, group, data.ctypes.data))

    def update_from(self, desc):
        """Take the operator and point data of another description with the same
        partition, features and points (a member of the same parameter family)."""
        self.set_operator(desc.lin_terms, desc.poly_terms)
        self.set_fn_terms(getattr(desc, "fn_terms", []))
        self.set_prod_terms(getattr(desc, "prod_terms", []))
        for i, g in enumerate(desc.groups):
            if g.data is not None and len(g.x):
                self.set_group_data(i, g.data)

    @property
    def n(self) -> int:
        return int(lib().rfm_num_unknowns(self.h))

    @property
    def m(self) -> int:
        return int(lib().rfm_num_rows(self.h))

    @property
    def nnz(self) -> int:
        """Values the block-sparse Jacobian stores (nnz(J))."""
        return int(lib().rfm_num_jacobian_values(self.h))

    # -- solver ------------------------------------------------------------------
    def solve(self, u0=None, opts: Optional[rfm_solve_opts] = None):
        """Returns (u, stats dict, status).  u0 may be a numpy array or a device tensor
        (updated in place); None means the zero guess."""
        o = opts or default_opts()
        u = np.zeros(self.n) if u0 is None else (u0 if hasattr(u0, "data_ptr") else _f64(u0).copy())
        st = rfm_solve_stats()
        rc = _check(lib().rfm_solve(self.h, C.byref(o), _ptr(u)[0], C.byref(st)))
        return u, st.as_dict(), rc

    def residual(self, u) -> Tuple[np.ndarray, float]:
        F = np.zeros(self.m)
        nrm = C.c_double()
        _check(lib().rfm_residual(self.h, _ptr(_f64(u) if not hasattr(u, "data_ptr") else u)[0], F.ctypes.data,
                                  C.byref(nrm)))
        return F, nrm.value

    def eval(self, u, x, owner) -> np.ndarray:
        """Field values [npts, ncomp]."""
        x = _f64(x)
        ow = np.ascontiguousarray(owner, dtype=np.int32)
        out = np.zeros((x.shape[0], self.ncomp))
        uu = u if hasattr(u, "data_ptr") else _f64(u)
        _check(lib().rfm_eval(self.h, _ptr(uu)[0], x.shape[0], x.ctypes.data, ow.ctypes.data, RFM_EVAL_VALUE,
                              out.ctypes.data))
        return out

    def eval_grad(self, u, x, owner) -> np.ndarray:
        """Field gradients [npts, ncomp, dim]."""
        x = _f64(x)
        ow = np.ascontiguousarray(owner, dtype=np.int32)
        out = np.zeros((x.shape[0], self.ncomp, self.dim))
        uu = u if hasattr(u, "data_ptr") else _f64(u)
        _check(lib().rfm_eval(self.h, _ptr(uu)[0], x.shape[0], x.ctypes.data, ow.ctypes.data, RFM_EVAL_GRAD,
                              out.ctypes.data))
        return out

    # -- stages ------------------------------------------------------------------
    def stage_assemble(self, u, c: float = 100.0):
        uu = u if hasattr(u, "data_ptr") else _f64(u)
        _check(lib().rfm_stage_assemble(self.h, _ptr(uu)[0], c))

    def get_scaled_residual(self) -> np.ndarray:
        out = np.zeros(self.m)
        _check(lib().rfm_get_scaled_residual(self.h, out.ctypes.data))
        return out

    def get_row_scale(self) -> np.ndarray:
        out = np.zeros(self.m)
        _check(lib().rfm_get_row_scale(self.h, out.ctypes.data))
        return out

    def get_jacobian_rows(self, r0: int, nrows: int) -> np.ndarray:
        out = np.zeros((nrows, self.n))
        _check(lib().rfm_get_jacobian_rows(self.h, r0, nrows, out.ctypes.data))
        return out

    def jmul(self, x) -> np.ndarray:
        x = _f64(x)
        y = np.zeros(self.m)
        _check(lib().rfm_jmul(self.h, x.ctypes.data, y.ctypes.data))
        return y

    def jtmul(self, y) -> np.ndarray:
        y = _f64(y)
        x = np.zeros(self.n)
        _check(lib().rfm_jtmul(self.h, y.ctypes.data, x.ctypes.data))
        return x

    def jtmul_noalloc(self, y, x):
        """x = (D J)^T y into the device tensor x from the device tensor y, without allocating (queued on
        the problem's stream; the caller synchronises)."""
        if not (hasattr(y, "data_ptr") and hasattr(x, "data_ptr")):
            raise ValueError("jtmul_noalloc takes device tensors")
        _check(lib().rfm_jtmul_noalloc(self.h, _ptr(y)[0], _ptr(x)[0]))

    def stage_sketch(self, gamma: float, seed: int, jac_index: int, prec: int = RFM_PREC_F64, pieces: int = 0):
        _check(lib().rfm_stage_sketch(self.h, gamma, seed, jac_index, prec, pieces))

    def stage_count_sketch(self, gamma: float, seed: int, jac_index: int):
        _check(lib().rfm_stage_count_sketch(self.h, gamma, seed, jac_index))

    def sketch_operand_slots(self, block: int) -> int:
        return int(lib().rfm_sketch_operand_slots(self.h, block))

    def get_sketch_operand(self, piece: int, block: int, slot0: int, nslots: int):
        """(values [nslots, J, 32], groups [nslots], scale exponents [nslots, J]) of one piece."""
        J = self.J
        out = np.zeros((nslots, J, 32))
        grp = np.zeros(nslots, np.int32)
        sc = np.zeros((nslots, J), np.int32)
        _check(lib().rfm_get_sketch_operand(self.h, piece, block, slot0, nslots, out.ctypes.data,
                                            grp.ctypes.data, sc.ctypes.data))
        return out, grp, sc

    @property
    def s(self) -> int:
        return int(lib().rfm_sketch_rows(self.h))

    def get_sketch_cols(self, c0: int, ncols: int) -> np.ndarray:
        """Columns [c0, c0+ncols) of B as an array [s, ncols]."""
        out = np.zeros((ncols, self.s))
        _check(lib().rfm_get_sketch_cols(self.h, c0, ncols, out.ctypes.data))
        return out.T

    def stage_qr(self):
        _check(lib().rfm_stage_qr(self.h))

    def stage_sketch_qr_streamed(self, gamma: float, seed: int, jac_index: int, prec: int = RFM_PREC_F64,
                                 pieces: int = 0, rows_per_pass: int = 0):
        _check(lib().rfm_stage_sketch_qr_streamed(self.h, gamma, seed, jac_index, prec, pieces, rows_per_pass))

    def stage_count_sketch_qr_streamed(self, gamma: float, seed: int, jac_index: int, rows_per_pass: int = 0):
        _check(lib().rfm_stage_count_sketch_qr_streamed(self.h, gamma, seed, jac_index, rows_per_pass))

    def get_r_cols(self, c0: int, ncols: int) -> np.ndarray:
        out = np.zeros((ncols, self.n))
        _check(lib().rfm_get_r_cols(self.h, c0, ncols, out.ctypes.data))
        return out.T

    def r_solve(self, y) -> np.ndarray:
        y = _f64(y)
        x = np.zeros(self.n)
        _check(lib().rfm_r_solve(self.h, y.ctypes.data, x.ctypes.data))
        return x

    def rt_solve(self, y) -> np.ndarray:
        y = _f64(y)
        x = np.zeros(self.n)
        _check(lib().rfm_rt_solve(self.h, y.ctypes.data, x.ctypes.data))
        return x

    def stage_lsqr(self, rhs, tol: float, max_iter: int = 500, prec: int = RFM_PREC_F64):
        rhs = _f64(rhs)
        y = np.zeros(self.n)
        it, istop = C.c_int32(), C.c_int32()
        _check(lib().rfm_stage_lsqr(self.h, rhs.ctypes.data, tol, max_iter, prec, y.ctypes.data, C.byref(it),
                                    C.byref(istop)))
        return y, it.value, istop.value

    # -- learned initial guess ---------------------------------------------------
    def pde_points(self):
        k = int(lib().rfm_num_pde_points(self.h))
        x = np.zeros((k, self.dim))
        ow = np.zeros(k, np.int32)
        _check(lib().rfm_get_pde_points(self.h, x.ctypes.data, ow.ctypes.data))
        return x, ow

    def project(self, values, opts=None):
        """Coefficients of the weighted least-squares fit of values [npde, ncomp] (and the residual norm)."""
        values = _f64(values)
        opts = opts or default_opts()
        u = np.zeros(self.n)
        rn = C.c_double()
        _check(lib().rfm_project(self.h, C.byref(opts), values.ctypes.data, u.ctypes.data, C.byref(rn)))
        return u, rn.value

    def warm_inputs(self, params, lo=None, hi=None) -> np.ndarray:
        """Network inputs [npde, nparam + dim] of one parameter draw (params encoded onto [-1, 1] over
        [lo, hi] when the ranges are given)."""
        params = _f64(params)
        lo = None if lo is None else _f64(lo)
        hi = None if hi is None else _f64(hi)
        k = int(lib().rfm_num_pde_points(self.h))
        X = np.zeros((k, params.size + self.dim), np.float32)
        _check(lib().rfm_warm_inputs(self.h, params.ctypes.data, None if lo is None else lo.ctypes.data,
                                     None if hi is None else hi.ctypes.data, params.size, X.ctypes.data))
        return X

    def warm_start(self, net: "RfmMLP", params, opts=None, lo=None, hi=None):
        """(u0, info): info = (||F(projection)||, ||F(0)||, kept)."""
        params = _f64(params)
        lo = None if lo is None else _f64(lo)
        hi = None if hi is None else _f64(hi)
        opts = opts or default_opts()
        u = np.zeros(self.n)
        info = np.zeros(3)
        _check(lib().rfm_warm_start(self.h, net.h, C.byref(opts), params.ctypes.data,
                                    None if lo is None else lo.ctypes.data, None if hi is None else hi.ctypes.data,
                                    params.size, u.ctypes.data, info.ctypes.data))
        return u, info

    def profile_enable(self, on: bool = True):
        _check(lib().rfm_profile_enable(self.h, 1 if on else 0))

    def profile_read(self) -> dict:
        """{kernel name: dict(launches, seconds, flops, bytes)} recorded since profile_enable."""
        buf = (rfm_kernel_stat * 64)()
        k = _check(lib().rfm_profile_read(self.h, buf, 64))
        return {buf[i].name.decode(): dict(launches=buf[i].launches, seconds=buf[i].seconds, flops=buf[i].flops,
                                           bytes=buf[i].bytes) for i in range(min(k, 64))}

    def stage_linesearch(self, u, du, gs_iters: int = 25):
        u, du = _f64(u), _f64(du)
        a, ph = C.c_double(), C.c_double()
        _check(lib().rfm_stage_linesearch(self.h, u.ctypes.data, du.ctypes.data, gs_iters, C.byref(a), C.byref(ph)))
        return a.value, ph.value


def from_description(desc, device: int = 0, stream: Optional[int] = None) -> RfmProblem:
    """Pass a problem description (attributes dim, ncomp, lo, hi, nsub, J, W, b,
    groups, lin_terms, poly_terms) to a new library problem, group by group."""
    p = RfmProblem(desc.dim, desc.ncomp, device, stream)
    p.set_partition(desc.lo, desc.hi, desc.nsub)
    if getattr(desc, "pou", "a") != "a":
        p.set_partition_of_unity(desc.pou)
    p.set_features(desc.J, desc.W, desc.b)
    for g in desc.groups:
        p.add_points(g.kind, g.x, g.owner, g.neighbor, g.normal, g.comp, g.cont_order, g.data)
    p.set_operator(desc.lin_terms, desc.poly_terms)
    if getattr(desc, "fn_terms", None):
        p.set_fn_terms(desc.fn_terms)
    if getattr(desc, "prod_terms", None):
        p.set_prod_terms(desc.prod_terms)
    p.finalize()
    return p
