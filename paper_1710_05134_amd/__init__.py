"""Python binding of libkth.so, the MI355X k-th eigenpair library.

Argument marshalling only: every numeric step runs in the library's HIP
kernels.  The names follow the C ABI of ``include/kth.h``.  PyTorch supplies
device memory and streams when a caller works with torch tensors
(``hip_stream`` / device pointers); numpy host arrays are accepted too.

Importing this module loads the in-tree ``libkth.so`` and raises if it is
missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkth.so")

KTH_OK, KTH_EINVAL, KTH_ENOMEM, KTH_EDEVICE, KTH_ENOTPD, KTH_ESINGULAR, KTH_ENOCONV, \
    KTH_ECLUSTER, KTH_ESTATE = range(9)
KTH_FP64, KTH_FP32_IR = 0, 1
KTH_DEVICE_PTRS, KTH_CHECK_SYMMETRY, KTH_SOLVE_UNREFINED = 1, 2, 4
ANALYZE_FIELDS = ("n", "nnz", "n_supervariables", "n_supernodes_fundamental", "n_supernodes",
                  "max_front", "max_pivot_block", "levels", "flops", "flops_padded", "nnz_l",
                  "nnz_l_padded", "front_pool_bytes", "factor_bytes", "t_order_s", "t_symbolic_s")


class KthError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


class kth_opts(C.Structure):
    _fields_ = [("m_max", C.c_int64), ("tau_res", C.c_double), ("tau_diff", C.c_double),
                ("tau_len", C.c_double), ("max_lanczos", C.c_int32), ("multisection", C.c_int32),
                ("seed", C.c_uint64), ("si_precision", C.c_int), ("start_vectors", C.c_void_p),
                ("warm_interval", C.c_void_p), ("warm_counts", C.c_void_p), ("ir_tol", C.c_double),
                ("batch_workers", C.c_int32), ("root_finder", C.c_int32), ("si_block", C.c_int32),
                ("n_start_vectors", C.c_int32), ("b_solver", C.c_int32)]


class kth_info(C.Structure):
    _fields_ = [("k_validated", C.c_int64), ("nu_lower", C.c_int64), ("nu_upper", C.c_int64),
                ("sigma_lower", C.c_double), ("sigma_upper", C.c_double), ("sigma_si", C.c_double),
                ("stage1_steps", C.c_int32), ("bisection_steps", C.c_int32),
                ("si_steps", C.c_int32), ("it_bound", C.c_int32), ("it_residual", C.c_int32),
                ("it_difference", C.c_int32), ("rel_residual", C.c_double),
                ("rel_residual_normA", C.c_double), ("eta", C.c_double),
                ("min_pivot_rel", C.c_double), ("n_factorizations", C.c_int64),
                ("flops_factor", C.c_double), ("t_task", C.c_double * 7),
                ("peak_device_bytes", C.c_double), ("n_sigmas", C.c_int32),
                ("sigmas", C.c_double * 128), ("nus", C.c_int64 * 128),
                ("si_precision", C.c_int32), ("ir_steps", C.c_int32), ("ir_fallback", C.c_int32),
                ("ir_max_berr", C.c_double), ("max_abs_l", C.c_double),
                ("weak_pivot_nudges", C.c_int32), ("weak_pivot_kept", C.c_int32),
                ("stage1_restarts", C.c_int32), ("si_block", C.c_int32), ("m_max_used", C.c_int64),
                ("b_cg_iterations", C.c_int32), ("pad1", C.c_int32)]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if name == "t_task":
                v = list(v)
            elif name in ("sigmas", "nus"):
                v = list(v)[: self.n_sigmas]
            d[name] = v
        return d


_lib = None


def lib() -> C.CDLL:
    """The loaded libkth.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1710_05134_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, p64, pi32, pd = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double)
    sig = {
        "kth_ctx_create": ([C.c_int, vp, vp, vp, vp, C.POINTER(vp)], C.c_int),
        "kth_ctx_destroy": ([vp], C.c_int),
        "kth_status_string": ([C.c_int], C.c_char_p),
        "kth_last_error": ([vp], C.c_char_p),
        "kth_analyze": ([C.c_int64, p64, pi32, C.c_uint32, pd, p64], C.c_int),
        "kth_pencil_create": ([vp, C.c_int64, p64, pi32, pd, p64, pi32, pd, C.c_uint32, C.POINTER(vp)],
                              C.c_int),
        "kth_pencil_set_values": ([vp, vp, vp, C.c_uint32], C.c_int),
        "kth_pencil_destroy": ([vp], C.c_int),
        "kth_inertia": ([vp, C.c_double, p64, p64], C.c_int),
        "kth_inertia_batch": ([vp, C.c_int32, pd, p64], C.c_int),
        "kth_factor": ([vp, C.c_double, C.c_int, C.POINTER(vp)], C.c_int),
        "kth_factor_inertia": ([vp, p64, p64, p64], C.c_int),
        "kth_solve": ([vp, C.c_int32, vp, C.c_int64, vp, C.c_int64, C.c_uint32], C.c_int),
        "kth_factor_destroy": ([vp], C.c_int),
        "kth_factor_stats": ([vp, p64, pd, pd], C.c_int),
        "kth_solve_noalloc": ([vp, C.c_int32, vp, C.c_int64, vp, C.c_int64, C.c_uint32], C.c_int),
        "kth_opts_default": ([C.POINTER(kth_opts)], None),
        "kth_eig": ([vp, C.c_int64, C.POINTER(kth_opts), pd, pd, C.POINTER(kth_info)], C.c_int),
        "kth_eig_batch": ([vp, C.c_int32, C.POINTER(vp), p64, C.POINTER(kth_opts), pd,
                           C.POINTER(pd), C.POINTER(kth_info), C.POINTER(C.c_int)], C.c_int),
        "kth_eig_backward": ([vp, C.c_double, pd, C.c_double, pd, pd], C.c_int),
        "kth_debug_mfma_probe": ([pd, pd, pd], C.c_int),
        "kth_profile_factor": ([vp, C.c_double, pd, C.c_int32], C.c_int),
        "kth_profile_solve": ([vp, C.c_int32, pd, C.c_int32], C.c_int),
        "kth_debug_mfma_probe_f32": ([C.POINTER(C.c_float)] * 3, C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _check(st: int, ctx=None):
    if st != KTH_OK:
        msg = lib().kth_last_error(ctx)
        raise KthError(st, (msg.decode() if msg else "") or lib().kth_status_string(st).decode())


def kth_analyze(rowptr, col, check_symmetry=False, want_perm=False):
    """Host-only ordering + symbolic statistics (dict); optionally the permutation."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    n = rowptr.size - 1
    stats = np.zeros(16)
    perm = np.zeros(n, dtype=np.int64) if want_perm else None
    st = lib().kth_analyze(n, _p(rowptr, C.c_int64), _p(col, C.c_int32),
                           KTH_CHECK_SYMMETRY if check_symmetry else 0, _p(stats, C.c_double),
                           _p(perm, C.c_int64) if want_perm else None)
    _check(st)
    d = dict(zip(ANALYZE_FIELDS, stats.tolist()))
    return (d, perm) if want_perm else d


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Context:
    """kth_ctx: device and stream (a raw hipStream_t, e.g. torch's
    ``torch.cuda.current_stream().cuda_stream``).  With ``torch_allocator=True`` the
    library's device memory comes from torch's caching allocator
    (``caching_allocator_alloc`` / ``caching_allocator_delete`` on that stream),
    through the allocator hooks of kth_ctx_create, and the context runs on torch's
    current stream unless ``hip_stream`` names another; torch must be imported first."""

    def __init__(self, device: int = 0, hip_stream: int | None = None, torch_allocator: bool = False):
        self._hooks = None
        alloc = free = None
        if torch_allocator:
            import torch
            dev = int(device)
            if hip_stream is None:   # run on torch's current stream: its pool's order
                hip_stream = torch.cuda.current_stream(dev).cuda_stream

            def _alloc(nbytes, _user):
                try:
                    return torch.cuda.caching_allocator_alloc(max(int(nbytes), 1), dev, hip_stream)
                except Exception:
                    return None   # the library reports KTH_ENOMEM

            def _free(ptr, _user):
                try:
                    torch.cuda.caching_allocator_delete(ptr)
                except Exception:
                    pass

            self._hooks = (_ALLOC_FN(_alloc), _FREE_FN(_free))   # kept alive with the context
            alloc, free = self._hooks
        h = C.c_void_p()
        _check(lib().kth_ctx_create(device, hip_stream, C.cast(alloc, C.c_void_p) if alloc else None,
                                    C.cast(free, C.c_void_p) if free else None, None, C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().kth_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pencil:
    """kth_pencil: A on (rowptr, col), B on (b_rowptr, b_col) -- by default the same
    pattern; both triangles stored."""

    def __init__(self, ctx: Context, rowptr, col, a_val, b_val, check_symmetry=False,
                 b_rowptr=None, b_col=None):
        self.ctx = ctx
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.b_rowptr = self.rowptr if b_rowptr is None else np.ascontiguousarray(b_rowptr, dtype=np.int64)
        self.b_col = self.col if b_col is None else np.ascontiguousarray(b_col, dtype=np.int32)
        self.n = self.rowptr.size - 1
        self.nnz = int(self.rowptr[-1])          # entries of A's pattern
        self.nnz_b = int(self.b_rowptr[-1])      # entries of B's pattern
        a = np.ascontiguousarray(a_val, dtype=np.float64)
        b = np.ascontiguousarray(b_val, dtype=np.float64)
        if a.size != self.nnz or b.size != self.nnz_b:
            raise ValueError("value arrays do not match their patterns")
        h = C.c_void_p()
        _check(lib().kth_pencil_create(ctx.h, self.n, _p(self.rowptr, C.c_int64),
                                       _p(self.col, C.c_int32), _p(a, C.c_double),
                                       _p(self.b_rowptr, C.c_int64), _p(self.b_col, C.c_int32),
                                       _p(b, C.c_double),
                                       KTH_CHECK_SYMMETRY if check_symmetry else 0, C.byref(h)),
               ctx.h)
        self.h = h

    @classmethod
    def from_pencilgen(cls, ctx, pen, **kw):
        return cls(ctx, pen.rowptr, pen.col, pen.a_val, pen.b_val, **kw)

    def set_values(self, a_val, b_val):
        a = np.ascontiguousarray(a_val, dtype=np.float64)
        b = np.ascontiguousarray(b_val, dtype=np.float64)
        _check(lib().kth_pencil_set_values(self.h, a.ctypes.data, b.ctypes.data, 0), self.ctx.h)

    def set_values_device(self, a_ptr: int, b_ptr: int):
        _check(lib().kth_pencil_set_values(self.h, a_ptr, b_ptr, KTH_DEVICE_PTRS), self.ctx.h)

    def inertia(self, sigma: float):
        """(nu, nzero); raises KthError(KTH_ESINGULAR) on an exactly zero pivot."""
        nu, nz = C.c_int64(), C.c_int64()
        st = lib().kth_inertia(self.h, float(sigma), C.byref(nu), C.byref(nz))
        if st == KTH_ESINGULAR:
            raise KthError(st, f"zero pivot at sigma={sigma!r} (nu={nu.value}, nzero={nz.value})")
        _check(st, self.ctx.h)
        return nu.value, nz.value

    def nu(self, sigma: float) -> int:
        return self.inertia(sigma)[0]

    def inertia_batch(self, sigmas):
        s = np.ascontiguousarray(sigmas, dtype=np.float64)
        out = np.zeros(s.size, dtype=np.int64)
        _check(lib().kth_inertia_batch(self.h, s.size, _p(s, C.c_double), _p(out, C.c_int64)),
               self.ctx.h)
        return out

    def profile_factor(self, sigma: float) -> dict:
        """One factorization with per-kernel-class event timing (see kth.h)."""
        out = np.zeros(32)
        _check(lib().kth_profile_factor(self.h, float(sigma), _p(out, C.c_double), 32), self.ctx.h)
        names = ("small", "assemble", "tile", "trsm", "gemm", "reduce")
        d = dict(total_s=out[0], flops=out[1], flops_padded=out[2], nu=int(out[27]))
        for c, nm in enumerate(names):
            d[nm] = dict(seconds=out[3 + 4 * c], flops=out[4 + 4 * c], launches=int(out[5 + 4 * c]),
                         bytes=out[6 + 4 * c])
        # the contribution-block launches' share of "gemm"
        d["gemm_cb"] = dict(seconds=out[28], flops=out[29], launches=int(out[30]), bytes=out[31])
        return d

    def factor(self, sigma: float, precision: int = KTH_FP64) -> "Factor":
        return Factor(self, sigma, precision)

    def eig(self, k: int, opts: kth_opts | None = None, want_x=True, **kw):
        """(lambda_k, x_k, info dict) by the three-stage algorithm."""
        o = default_opts(**kw) if opts is None else opts
        lam = C.c_double()
        x = np.zeros(self.n) if want_x else None
        info = kth_info()
        st = lib().kth_eig(self.h, int(k), C.byref(o), C.byref(lam),
                           _p(x, C.c_double) if want_x else None, C.byref(info))
        _check(st, self.ctx.h)
        return lam.value, x, info.as_dict()

    def backward(self, lam: float, x, g: float = 1.0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        ga = np.zeros(self.nnz)
        gb = np.zeros(self.nnz_b)
        _check(lib().kth_eig_backward(self.h, float(lam), _p(x, C.c_double), float(g),
                                      _p(ga, C.c_double), _p(gb, C.c_double)), self.ctx.h)
        return ga, gb

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().kth_pencil_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Factor:
    """kth_factor_t: kept numeric factor of A - sigma B."""

    def __init__(self, pencil: Pencil, sigma: float, precision: int = KTH_FP64):
        self.pencil = pencil
        h = C.c_void_p()
        _check(lib().kth_factor(pencil.h, float(sigma), precision, C.byref(h)), pencil.ctx.h)
        self.h = h

    def inertia(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().kth_factor_inertia(self.h, C.byref(a), C.byref(b), C.byref(c)),
               self.pencil.ctx.h)
        return a.value, b.value, c.value

    def stats(self) -> dict:
        """n2x2, min_pivot_rel, max_abs_l of the factor (see kth_factor_stats)."""
        n2, md, ml = C.c_int64(), C.c_double(), C.c_double()
        _check(lib().kth_factor_stats(self.h, C.byref(n2), C.byref(md), C.byref(ml)),
               self.pencil.ctx.h)
        return dict(n2x2=n2.value, min_pivot_rel=md.value, max_abs_l=ml.value)

    def profile_solve(self, reps: int = 10) -> dict:
        """Event timing of solves and SpMV (see kth_profile_solve)."""
        out = np.zeros(6)
        _check(lib().kth_profile_solve(self.h, int(reps), _p(out, C.c_double), 6),
               self.pencil.ctx.h)
        return dict(solve_s=out[0], solve_bytes=out[1], spmv_b_s=out[2], spmv_b_bytes=out[3],
                    spmv_ab_s=out[4], spmv_ab_bytes=out[5])

    def solve(self, r, refine: bool = True):
        """X = (A - sigma B)^{-1} R; refine=False applies an FP32 factor once."""
        r = np.asfortranarray(r, dtype=np.float64)
        one = r.ndim == 1
        R = r.reshape(self.pencil.n, -1, order="F")
        X = np.zeros_like(R, order="F")
        _check(lib().kth_solve(self.h, R.shape[1], R.ctypes.data, self.pencil.n, X.ctypes.data,
                               self.pencil.n, 0 if refine else KTH_SOLVE_UNREFINED),
               self.pencil.ctx.h)
        return X[:, 0] if one else X

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().kth_factor_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eig_batch(ctx: Context, pencils, ks, opts: kth_opts | None = None, want_x=True, **kw):
    """kth_eig_batch: list of (status, lambda, x, info dict), one per pencil."""
    o = default_opts(**kw) if opts is None else opts
    npen = len(pencils)
    hs = (C.c_void_p * npen)(*[p.h.value for p in pencils])
    kk = np.ascontiguousarray(ks, dtype=np.int64)
    lam = np.zeros(npen)
    xs = [np.zeros(p.n) for p in pencils] if want_x else None
    xptr = (C.POINTER(C.c_double) * npen)(*[_p(x, C.c_double) for x in xs]) if want_x else None
    infos = (kth_info * npen)()
    per = (C.c_int * npen)()
    _check(lib().kth_eig_batch(ctx.h, npen, hs, _p(kk, C.c_int64), C.byref(o), _p(lam, C.c_double),
                               xptr, infos, per), ctx.h)
    return [(int(per[i]), float(lam[i]), xs[i] if want_x else None, infos[i].as_dict())
            for i in range(npen)]


def default_opts(**kw) -> kth_opts:
    o = kth_opts()
    lib().kth_opts_default(C.byref(o))
    keep = kw.pop("_keep", None)
    for k, v in kw.items():
        if k == "start_vectors":
            arr = np.ascontiguousarray(v, dtype=np.float64)
            o._sv = arr
            o.start_vectors = arr.ctypes.data
            o.n_start_vectors = arr.shape[0] if arr.ndim == 2 else 1
        elif k == "warm_interval":
            arr = np.ascontiguousarray(v, dtype=np.float64)
            o._wi = arr
            o.warm_interval = arr.ctypes.data
        elif k == "warm_counts":
            arr = np.ascontiguousarray(v, dtype=np.int64)
            o._wc = arr
            o.warm_counts = arr.ctypes.data
        else:
            setattr(o, k, v)
    del keep
    return o


def kth_debug_mfma_probe_f32(A, B):
    A = np.ascontiguousarray(A, dtype=np.float32).reshape(-1)
    B = np.ascontiguousarray(B, dtype=np.float32).reshape(-1)
    D = np.zeros(256, dtype=np.float32)
    _check(lib().kth_debug_mfma_probe_f32(_p(A, C.c_float), _p(B, C.c_float), _p(D, C.c_float)))
    return D


def kth_debug_mfma_probe(A, B):
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(-1)
    B = np.ascontiguousarray(B, dtype=np.float64).reshape(-1)
    D = np.zeros(256)
    _check(lib().kth_debug_mfma_probe(_p(A, C.c_double), _p(B, C.c_double), _p(D, C.c_double)))
    return D


def eig_function():
    """torch.autograd.Function over (a_val, b_val) -> lambda_k: forward through kth_eig on
    the pencil's pattern(s), backward through kth_eig_backward (Hellmann-Feynman).
    float64 tensors on the host, or on the pencil's GPU: device values go to the
    library as device pointers (kth_pencil_set_values with KTH_DEVICE_PTRS, after
    torch's current stream is synchronised); lambda_k and the gradients come back on
    the values' device.  Usage:
        F = eig_function(); lam = F.apply(a, b, pencil, k, opts_or_None)"""
    import torch

    class KthEig(torch.autograd.Function):
        @staticmethod
        def forward(ctx, a_val, b_val, pencil, k, opts):
            dev = a_val.device
            if a_val.is_cuda:
                a = a_val.detach().to(torch.float64).contiguous()
                b = b_val.detach().to(device=dev, dtype=torch.float64).contiguous()
                torch.cuda.current_stream(dev).synchronize()
                pencil.set_values_device(a.data_ptr(), b.data_ptr())
            else:
                pencil.set_values(a_val.detach().to("cpu", torch.float64).numpy(),
                                  b_val.detach().to("cpu", torch.float64).numpy())
            lam, x, _ = pencil.eig(int(k), opts=opts)
            ctx.pencil, ctx.lam, ctx.x, ctx.dev = pencil, lam, x, dev
            return torch.tensor(lam, dtype=torch.float64, device=dev)

        @staticmethod
        def backward(ctx, g):
            ga, gb = ctx.pencil.backward(ctx.lam, ctx.x, float(g))
            return (torch.from_numpy(ga).to(ctx.dev), torch.from_numpy(gb).to(ctx.dev), None, None,
                    None)

    return KthEig
