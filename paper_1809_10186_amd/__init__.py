"""Python binding of libqcoll (the fast spectral collision operator on gfx950).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory and the stream.  The library must
be built in-tree (``python -m paper_1809_10186_amd.build``); importing this
package without it raises, there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqcoll.so")

QCOLL_FP64, QCOLL_FP32 = 0, 1
QCOLL_NYQ_SYMMETRIC, QCOLL_NYQ_LITERAL = 0, 1
STATUS = {0: "QCOLL_OK", 1: "QCOLL_EINVAL", 2: "QCOLL_ENOTSUP", 3: "QCOLL_ENOMEM",
          4: "QCOLL_EDEVICE", 5: "QCOLL_EWORKSPACE", 6: "QCOLL_ENONFINITE"}


class QcollError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("L", ctypes.c_double), ("N_rho", ctypes.c_int32),
                ("M", ctypes.c_int32), ("sphere", ctypes.POINTER(ctypes.c_double)),
                ("omega", ctypes.c_double), ("alpha", ctypes.c_double),
                ("prefactor", ctypes.c_double), ("svd_rank", ctypes.c_int32),
                ("svd_tol", ctypes.c_double), ("precision", ctypes.c_int32), ("nyquist", ctypes.c_int32)]


class Bc(ctypes.Structure):
    """One end of a 1-D domain: kind 0 periodic, 1 diffuse wall (u, T), 2 inflow (n, u, T)."""
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_double), ("u", ctypes.c_double * 3),
                ("T", ctypes.c_double)]

    def __init__(self, kind="periodic", n=1.0, u=(0.0, 0.0, 0.0), T=1.0):
        code = {"periodic": 0, "wall": 1, "inflow": 2}[kind] if isinstance(kind, str) else int(kind)
        super().__init__(code, float(n), (ctypes.c_double * 3)(*[float(x) for x in u]), float(T))


class Dg1dParams(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int32), ("faces", ctypes.POINTER(ctypes.c_double)),
                ("order", ctypes.c_int32), ("inv_kn", ctypes.c_double), ("coll_form", ctypes.c_int32),
                ("conserve", ctypes.c_int32), ("left", Bc), ("right", Bc)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("N_rho", ctypes.c_int32), ("M", ctypes.c_int32),
                ("rank", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("L", ctypes.c_double), ("R", ctypes.c_double), ("omega", ctypes.c_double),
                ("prefactor", ctypes.c_double), ("sigma_max", ctypes.c_double),
                ("sigma_min_kept", ctypes.c_double)]


_lib = None


def lib():
    """Load libqcoll.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1809_10186_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        sig = {
            "qcoll_params_check": ([ctypes.POINTER(Params)], i32),
            "qcoll_plan_create": ([ctypes.POINTER(Params), i32, ctypes.POINTER(vp)], i32),
            "qcoll_plan_destroy": ([vp], i32),
            "qcoll_plan_info": ([vp, ctypes.POINTER(PlanInfo)], i32),
            "qcoll_plan_radial": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], i32),
            "qcoll_plan_set_omega": ([vp, ctypes.c_double], i32),
            "qcoll_plan_table": ([vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t], i32),
            "qcoll_plan_set_schedule": ([vp, i32], i32),
            "qcoll_workspace_bytes": ([vp, i64, i32], ctypes.c_size_t),
            "qcoll_eval": ([vp, i64, dp, dp, vp, ctypes.c_size_t, vp], i32),
            "qcoll_eval_noalloc": ([vp, i64, dp, dp, vp], i32),
            "qcoll_conserve": ([vp, i64, dp, dp, vp], i32),
            "qcoll_moments": ([vp, i64, dp, dp, vp], i32),
            "qcoll_vjp": ([vp, i64, dp, dp, dp, dp, i32, vp, ctypes.c_size_t, vp], i32),
            "qcoll_poll": ([vp], i32),
            "qcoll_status_str": ([i32], ctypes.c_char_p),
            "qcoll_last_error": ([], ctypes.c_char_p),
            "qcoll_version": ([], i32),
            "qcoll_eval_bilinear": ([vp, i64, dp, dp, dp, vp, ctypes.c_size_t, vp], i32),
            "qcoll_dg_svd_workspace_bytes": ([vp, i64, i32, i32], ctypes.c_size_t),
            "qcoll_dg_collide_svd": ([vp, i64, i32, i32, dp, dp, dp, dp, dp, i32, vp, ctypes.c_size_t, vp], i32),
            "qcoll_dg_workspace_bytes": ([vp, i64, i32, i32], ctypes.c_size_t),
            "qcoll_dg_collocated_workspace_bytes": ([vp, i64, i32], ctypes.c_size_t),
            "qcoll_dg_collide_collocated": ([vp, i64, i32, ctypes.POINTER(ctypes.c_double), dp, dp, i32, vp,
                                             ctypes.c_size_t, vp], i32),
            "qcoll_dg_collide": ([vp, i64, i32, i32, dp, dp, dp, dp, i32, vp, ctypes.c_size_t, vp], i32),
            "qcoll_plan_set_chunk": ([vp, i32], i32),
            "qcoll_autotune_workspace_bytes": ([vp, i64], ctypes.c_size_t),
            "qcoll_autotune": ([vp, i64, dp, dp, vp, ctypes.c_size_t, vp, ctypes.POINTER(i32),
                                ctypes.POINTER(i32)], i32),
            "qcoll_group_create": ([ctypes.POINTER(vp), ctypes.POINTER(i64), i32, ctypes.POINTER(vp)], i32),
            "qcoll_group_destroy": ([vp], i32),
            "qcoll_group_workspace_bytes": ([vp, i32], ctypes.c_size_t),
            "qcoll_group_eval": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i32, vp, ctypes.c_size_t, vp, i32],
                                 i32),
            "qcoll_group_vjp": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                ctypes.POINTER(vp), i32, vp, ctypes.c_size_t, vp, i32], i32),
            "qcoll_group_autotune_workspace_bytes": ([vp], ctypes.c_size_t),
            "qcoll_group_autotune": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), vp, ctypes.c_size_t, vp], i32),
            "qcoll_dg1d_create": ([vp, ctypes.POINTER(Dg1dParams), ctypes.POINTER(vp)], i32),
            "qcoll_dg1d_destroy": ([vp], i32),
            "qcoll_dg1d_nodes": ([vp, ctypes.POINTER(ctypes.c_double)], i32),
            "qcoll_dg1d_workspace_bytes": ([vp, i32], ctypes.c_size_t),
            "qcoll_dg1d_rhs": ([vp, dp, dp, vp, ctypes.c_size_t, vp], i32),
            "qcoll_dg1d_step": ([vp, dp, ctypes.c_double, i32, vp, ctypes.c_size_t, vp], i32),
            "qcoll_timing_enable": ([i32], i32),
            "qcoll_timing_reset": ([], i32),
            "qcoll_timing_select": ([ctypes.c_char_p], i32),
            "qcoll_timing_read": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)], i32),
            "qcoll_timing_names": ([ctypes.c_char_p, ctypes.c_size_t], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise QcollError(code, lib().qcoll_last_error().decode())


def make_params(N, L, N_rho, sphere=None, omega=1.0, prefactor=None, svd_rank=-1, svd_tol=0.0,
                precision=QCOLL_FP64, alpha=1.0, nyquist="symmetric"):
    """Build a Params struct; sphere is (points [M,3], weights [M]) or None for the built-in M=6 rule.
    Returns (params, keepalive)."""
    keep = None
    p = Params()
    p.N, p.L, p.N_rho = int(N), float(L), int(N_rho)
    if sphere is None:
        p.M = 6
        p.sphere = None
    else:
        pts, w = sphere
        M = len(w)
        arr = (ctypes.c_double * (4 * M))()
        for q in range(M):
            arr[4 * q:4 * q + 3] = [float(x) for x in pts[q]]
            arr[4 * q + 3] = float(w[q])
        keep = arr
        p.M = M
        p.sphere = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
    p.omega = float(omega)
    p.alpha = float(alpha)
    p.prefactor = float("nan") if prefactor is None else float(prefactor)
    p.svd_rank = int(svd_rank)
    p.svd_tol = float(svd_tol)
    p.precision = int(precision)
    p.nyquist = {"symmetric": QCOLL_NYQ_SYMMETRIC, "literal": QCOLL_NYQ_LITERAL}[nyquist] \
        if isinstance(nyquist, str) else int(nyquist)
    return p, keep


def params_check(**kw):
    p, keep = make_params(**kw)
    code = lib().qcoll_params_check(ctypes.byref(p))
    del keep
    return code, lib().qcoll_last_error().decode()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _keep_for(t, stream):
    """A temporary allocated on the current stream but used by kernels enqueued
    on `stream`: tell the caching allocator not to reuse it before they finish."""
    if stream is not None and t is not None:
        t.record_stream(stream)


class Plan:
    """A plan for one velocity grid and kernel.  See include/qcoll.h."""

    def __init__(self, N, L, N_rho, sphere=None, omega=1.0, prefactor=None, svd_rank=-1,
                 svd_tol=0.0, precision=QCOLL_FP64, device=None, alpha=1.0, nyquist="symmetric"):
        """alpha: VSS scattering exponent (1 = VHS; (1, 2] = VSS, full table only).
        nyquist: "symmetric" (default) or "literal" shift at frequency -N/2."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("qcoll needs a ROCm GPU")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        p, keep = make_params(N, L, N_rho, sphere, omega, prefactor, svd_rank, svd_tol, precision, alpha, nyquist)
        h = ctypes.c_void_p()
        _check(lib().qcoll_plan_create(ctypes.byref(p), self.device.index, ctypes.byref(h)))
        del keep
        self._h = h
        self.N, self.L, self.N_rho = int(N), float(L), int(N_rho)
        self.precision = precision
        self._ws = {}

    def close(self):
        if getattr(self, "_h", None):
            import torch
            torch.cuda.synchronize(self.device)
            lib().qcoll_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = PlanInfo()
        _check(lib().qcoll_plan_info(self._h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in PlanInfo._fields_}

    def radial(self):
        n = self.N_rho
        r = (ctypes.c_double * n)()
        w = (ctypes.c_double * n)()
        _check(lib().qcoll_plan_radial(self._h, r, w))
        return list(r), list(w)

    def set_omega(self, omega):
        _check(lib().qcoll_plan_set_omega(self._h, float(omega)))

    def table(self, which):
        """Kernel-mode table as a float64 numpy array: "gain" [N_rho, N, N, N],
        "loss" [N, N, N] or "loss_nodes" [N_rho, N, N, N] (see include/qcoll.h)."""
        import numpy as np
        code = {"gain": 0, "loss": 1, "loss_nodes": 2}[which]
        n = self.N
        shape = (n, n, n) if code == 1 else (self.N_rho, n, n, n)
        out = np.empty(shape, dtype=np.float64)
        _check(lib().qcoll_plan_table(self._h, code, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      out.size))
        return out

    def set_schedule(self, schedule):
        """0 auto, 1 two-pass, 2 fused (see include/qcoll.h)."""
        _check(lib().qcoll_plan_set_schedule(self._h, int(schedule)))
        self._ws = {}

    def workspace_bytes(self, batch, op=0):
        return int(lib().qcoll_workspace_bytes(self._h, int(batch), int(op)))

    def workspace(self, batch, op=0, stream=None):
        """The plan's cached workspace for `stream` (one buffer per stream, so that
        calls on different streams never share scratch memory)."""
        import torch
        need = self.workspace_bytes(batch, op)
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        key = s.cuda_stream
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            with torch.cuda.stream(s):
                ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def _check_out(self, t, name, shape, batch=None):
        """An output buffer the library writes: float64, contiguous, on the plan's
        device, of exactly `shape` (the kernels trust these sizes)."""
        import torch
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def _check_f(self, t, name):
        import torch
        n = self.N
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device:
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if t.shape[-3:] != (n, n, n):
            raise ValueError(f"{name} must have trailing shape ({n}, {n}, {n})")
        return t.reshape(-1, n, n, n).shape[0]

    def eval(self, f, out=None, stream=None):
        import torch
        batch = self._check_f(f, "f")
        if out is None:
            out = torch.empty_like(f)
        else:
            self._check_out(out, "out", f.shape)
        ws = self.workspace(batch, 0, stream)
        _check(lib().qcoll_eval(self._h, batch, _ptr(f), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
        return out

    def eval_noalloc(self, f, out, stream=None):
        """qcoll_eval without a workspace and without any allocation (scratch in a
        fixed device array of the library; calls on one GPU must not overlap)."""
        batch = self._check_f(f, "f")
        self._check_out(out, "out", f.shape)
        _check(lib().qcoll_eval_noalloc(self._h, batch, _ptr(f), _ptr(out), _stream(stream)))
        return out

    def eval_bilinear(self, f, g, out=None, stream=None):
        """Bilinear Q(f, g) for every item (two-pass schedule)."""
        import torch
        batch = self._check_f(f, "f")
        if self._check_f(g, "g") != batch:
            raise ValueError("f and g batches differ")
        if out is None:
            out = torch.empty_like(f)
        else:
            self._check_out(out, "out", f.shape)
        need = self.workspace_bytes(batch, 2)
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        _check(lib().qcoll_eval_bilinear(self._h, batch, _ptr(f), _ptr(g), _ptr(out), _ptr(ws), ws.numel(),
                                         _stream(stream)))
        _keep_for(ws, stream)
        return out

    def conserve(self, Q, moments=None, stream=None):
        batch = self._check_f(Q, "Q")
        if moments is not None:
            self._check_out(moments, "moments", (batch, 5))
        _check(lib().qcoll_conserve(self._h, batch, _ptr(Q), _ptr(moments), _stream(stream)))
        return Q

    def moments(self, f, out=None, stream=None):
        import torch
        batch = self._check_f(f, "f")
        if out is None:
            out = torch.empty(f.shape[:-3] + (14,), dtype=torch.float64, device=self.device)
        else:
            self._check_out(out, "out", f.shape[:-3] + (14,))
        _check(lib().qcoll_moments(self._h, batch, _ptr(f), _ptr(out), _stream(stream)))
        return out

    def vjp(self, f, g, df=None, domega=None, through_conserve=False, want_df=True, want_domega=False,
            stream=None):
        import torch
        batch = self._check_f(f, "f")
        if self._check_f(g, "g") != batch:
            raise ValueError("f and g batches differ")
        if want_df:
            if df is None:
                df = torch.empty_like(f)
            else:
                self._check_out(df, "df", f.shape)
        if want_domega:
            if domega is None:
                domega = torch.empty(batch, dtype=torch.float64, device=self.device)
            else:
                self._check_out(domega, "domega", (batch,))
        ws = self.workspace(batch, 1, stream)
        _check(lib().qcoll_vjp(self._h, batch, _ptr(f), _ptr(g), _ptr(df if want_df else None),
                               _ptr(domega if want_domega else None), int(bool(through_conserve)),
                               _ptr(ws), ws.numel(), _stream(stream)))
        return df, domega

    def dg_collide(self, F, T, W, conserve=False, out=None, stream=None):
        """DG collision term C[e][m] = sum_r W[m][r] Q(sum_l T[r][l] F[e][l]).

        F: float64 [n_elem, K, N, N, N]; T: float64 [R, K]; W: float64 [K, R] (CUDA tensors)."""
        import torch
        n = self.N
        if F.dim() != 5 or F.shape[2:] != (n, n, n) or F.dtype != torch.float64 or not F.is_contiguous():
            raise ValueError("F must be a contiguous float64 tensor [n_elem, K, N, N, N]")
        E, K = F.shape[0], F.shape[1]
        R = T.shape[0]
        if T.shape != (R, K) or W.shape != (K, R):
            raise ValueError("T must be [R, K] and W [K, R]")
        if F.device != self.device:
            raise ValueError(f"F must be on {self.device}")
        T = T.to(device=self.device, dtype=torch.float64).contiguous()
        W = W.to(device=self.device, dtype=torch.float64).contiguous()
        if out is None:
            out = torch.empty_like(F)
        else:
            self._check_out(out, "out", F.shape)
        need = int(lib().qcoll_dg_workspace_bytes(self._h, E, K, R))
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        _check(lib().qcoll_dg_collide(self._h, E, K, R, _ptr(T), _ptr(W), _ptr(F), _ptr(out), int(bool(conserve)),
                                      _ptr(ws), ws.numel(), _stream(stream)))
        for t in (ws, T, W):
            _keep_for(t, stream)
        return out

    def dg_collide_collocated(self, F, weights, conserve=False, out=None, stream=None):
        """Collocated DG collision term C[e][m] = w_m Q(F[e][m]) (T = I, W = diag(w)).

        F: float64 [n_elem, K, N, N, N] CUDA tensor; weights: K host floats."""
        import numpy as np
        import torch
        n = self.N
        if F.dim() != 5 or F.shape[2:] != (n, n, n) or F.dtype != torch.float64 or not F.is_contiguous() \
                or F.device != self.device:
            raise ValueError(f"F must be a contiguous float64 tensor [n_elem, K, N, N, N] on {self.device}")
        E, K = F.shape[0], F.shape[1]
        w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
        if w.size != K:
            raise ValueError("weights must have K entries")
        if out is None:
            out = torch.empty_like(F)
        else:
            self._check_out(out, "out", F.shape)
        need = int(lib().qcoll_dg_collocated_workspace_bytes(self._h, E, K))
        key = ("colloc", torch.cuda.current_stream(self.device).cuda_stream if stream is None else stream.cuda_stream)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        _check(lib().qcoll_dg_collide_collocated(self._h, E, K, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 _ptr(F), _ptr(out), int(bool(conserve)), _ptr(ws), ws.numel(),
                                                 _stream(stream)))
        _keep_for(ws, stream)
        return out

    def dg_collide_svd(self, F, T1, T2, W, conserve=False, out=None, stream=None):
        """The paper's SVD form: C[e][m] = sum_r W[m][r] Q(T1_r . F[e], T2_r . F[e]) (bilinear Q)."""
        import torch
        n = self.N
        if F.dim() != 5 or F.shape[2:] != (n, n, n) or F.dtype != torch.float64 or not F.is_contiguous():
            raise ValueError("F must be a contiguous float64 tensor [n_elem, K, N, N, N]")
        E, K = F.shape[0], F.shape[1]
        R = T1.shape[0]
        if T1.shape != (R, K) or T2.shape != (R, K) or W.shape != (K, R):
            raise ValueError("T1, T2 must be [R, K] and W [K, R]")
        if F.device != self.device:
            raise ValueError(f"F must be on {self.device}")
        T1, T2, W = [x.to(device=self.device, dtype=torch.float64).contiguous() for x in (T1, T2, W)]
        if out is None:
            out = torch.empty_like(F)
        else:
            self._check_out(out, "out", F.shape)
        need = int(lib().qcoll_dg_svd_workspace_bytes(self._h, E, K, R))
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        _check(lib().qcoll_dg_collide_svd(self._h, E, K, R, _ptr(T1), _ptr(T2), _ptr(W), _ptr(F), _ptr(out),
                                          int(bool(conserve)), _ptr(ws), ws.numel(), _stream(stream)))
        for t in (ws, T1, T2, W):
            _keep_for(t, stream)
        return out

    def set_chunk(self, items):
        _check(lib().qcoll_plan_set_chunk(self._h, int(items)))
        self._ws = {}

    def autotune(self, f, Q=None, stream=None):
        """Time the candidate schedules on f and keep the fastest; returns (schedule, chunk)."""
        import torch
        batch = self._check_f(f, "f")
        if Q is None:
            Q = torch.empty_like(f)
        else:
            self._check_out(Q, "Q", f.shape)
        need = int(lib().qcoll_autotune_workspace_bytes(self._h, batch))
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.device)
        sch, ck = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().qcoll_autotune(self._h, batch, _ptr(f), _ptr(Q), _ptr(ws), ws.numel(), _stream(stream),
                                    ctypes.byref(sch), ctypes.byref(ck)))
        self._ws = {}
        return sch.value, ck.value

    def poll(self):
        _check(lib().qcoll_poll(self._h))



def timing_enable(on=True):
    _check(lib().qcoll_timing_enable(int(bool(on))))


def timing_select(name=None):
    """Time only the kernel role `name` (None: every role)."""
    _check(lib().qcoll_timing_select(name.encode() if name else None))


def timing_reset():
    _check(lib().qcoll_timing_reset())


def timing_read():
    """{kernel role: (total_ms, launches)} for every role launched since the last reset."""
    buf = ctypes.create_string_buffer(4096)
    _check(lib().qcoll_timing_names(buf, 4096))
    out = {}
    for name in filter(None, buf.value.decode().split("\n")):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().qcoll_timing_read(name.encode(), ctypes.byref(ms), ctypes.byref(n)))
        out[name] = (ms.value, n.value)
    return out


class Group:
    """Several plans with their item counts evaluated as one (graph) launch."""

    def __init__(self, plans, counts):
        self.plans = list(plans)
        self.counts = [int(c) for c in counts]
        n = len(self.plans)
        hp = (ctypes.c_void_p * n)(*[p._h for p in self.plans])
        hc = (ctypes.c_int64 * n)(*self.counts)
        h = ctypes.c_void_p()
        _check(lib().qcoll_group_create(hp, hc, n, ctypes.byref(h)))
        self._h = h
        self._ws = {}

    def close(self):
        if getattr(self, "_h", None):
            import torch
            torch.cuda.synchronize()
            lib().qcoll_group_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _workspace(self, op):
        import torch
        need = int(lib().qcoll_group_workspace_bytes(self._h, op))
        ws = self._ws.get(op)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.plans[0].device)
            self._ws[op] = ws
        return ws

    @staticmethod
    def _arr(ts):
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() if t is not None else None for t in ts])

    def eval(self, fs, Qs=None, conserve=True, use_graph=True, stream=None):
        import torch
        if Qs is None:
            Qs = [torch.empty_like(f) for f in fs]
        for p, f, q, c in zip(self.plans, fs, Qs, self.counts):
            if p._check_f(f, "f") != c or p._check_f(q, "Q") != c:
                raise ValueError("item counts differ from the group's")
        ws = self._workspace(0)
        _check(lib().qcoll_group_eval(self._h, self._arr(fs), self._arr(Qs), int(bool(conserve)), _ptr(ws),
                                      ws.numel(), _stream(stream), int(bool(use_graph))))
        return Qs

    def autotune(self, fs, Qs=None, stream=None):
        """Autotune every member plan on its inputs (before the first graph capture)."""
        import torch
        if Qs is None:
            Qs = [torch.empty_like(f) for f in fs]
        for p, f, q, c in zip(self.plans, fs, Qs, self.counts):
            if p._check_f(f, "f") != c or p._check_f(q, "Q") != c:
                raise ValueError("item counts differ from the group's")
        need = int(lib().qcoll_group_autotune_workspace_bytes(self._h))
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.plans[0].device)
        _check(lib().qcoll_group_autotune(self._h, self._arr(fs), self._arr(Qs), _ptr(ws), ws.numel(),
                                          _stream(stream)))
        for p in self.plans:
            p._ws = {}

    def vjp(self, fs, gs, dfs=None, domegas=None, through_conserve=True, use_graph=True, stream=None):
        import torch
        if dfs is None:
            dfs = [torch.empty_like(f) for f in fs]
        ws = self._workspace(1)
        dw = self._arr(domegas) if domegas is not None else None
        _check(lib().qcoll_group_vjp(self._h, self._arr(fs), self._arr(gs), self._arr(dfs), dw,
                                     int(bool(through_conserve)), _ptr(ws), ws.numel(), _stream(stream),
                                     int(bool(use_graph))))
        return dfs


class Dg1d:
    """1-D RKDG driver over a plan (see include/qcoll.h): state F [n_elem][K][N][N][N]."""

    def __init__(self, plan, faces, order, inv_kn, left=None, right=None, coll_form=0, conserve=True):
        import numpy as np
        self.plan = plan
        self.faces = np.ascontiguousarray(faces, dtype=np.float64)
        self.n_elem = len(self.faces) - 1
        self.K = int(order) + 1
        left = left if left is not None else Bc("periodic")
        right = right if right is not None else Bc("periodic")
        prm = Dg1dParams(self.n_elem, self.faces.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(order),
                         float(inv_kn), int(coll_form), int(bool(conserve)), left, right)
        h = ctypes.c_void_p()
        _check(lib().qcoll_dg1d_create(plan._h, ctypes.byref(prm), ctypes.byref(h)))
        self._h = h
        self._ws = {}

    def close(self):
        if getattr(self, "_h", None):
            import torch
            torch.cuda.synchronize()
            lib().qcoll_dg1d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nodes(self):
        import numpy as np
        x = np.zeros((self.n_elem, self.K))
        _check(lib().qcoll_dg1d_nodes(self._h, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return x

    def _workspace(self, rk):
        import torch
        need = int(lib().qcoll_dg1d_workspace_bytes(self._h, int(rk)))
        ws = self._ws.get(rk)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=self.plan.device)
            self._ws[rk] = ws
        return ws

    def _check_state(self, F):
        import torch
        N = self.plan.N
        if tuple(F.shape) != (self.n_elem, self.K, N, N, N) or F.dtype != torch.float64 \
                or not F.is_cuda or not F.is_contiguous():
            raise ValueError(f"state must be a contiguous float64 CUDA tensor {(self.n_elem, self.K, N, N, N)}")

    def rhs(self, F, R=None, stream=None):
        import torch
        self._check_state(F)
        if R is None:
            R = torch.empty_like(F)
        ws = self._workspace(0)
        _check(lib().qcoll_dg1d_rhs(self._h, _ptr(F), _ptr(R), _ptr(ws), ws.numel(), _stream(stream)))
        return R

    def step(self, F, dt, rk=3, stream=None):
        self._check_state(F)
        ws = self._workspace(rk)
        _check(lib().qcoll_dg1d_step(self._h, _ptr(F), float(dt), int(rk), _ptr(ws), ws.numel(), _stream(stream)))
        return F


def collide(f, plan, omega=None, conserve=True):
    """Differentiable Q(f,f) (optionally conservation-projected).

    f: float64 CUDA tensor [..., N, N, N].  omega: optional 0-d float64 tensor;
    when given (requires_grad allowed) the plan's omega is set to its value (and
    stays set for later calls) and its gradient is sum over the batch of
    g . dQ/d omega.  The backward pass calls qcoll_vjp (through the projection
    when conserve is True) at the omega the forward pass used: it is saved with
    the graph, so other calls that change the plan's omega in between do not
    affect this backward.
    """
    import torch

    class _Collide(torch.autograd.Function):
        @staticmethod
        def forward(ctx, f_, om_):
            if om_ is not None and abs(float(om_) - plan.info()["omega"]) > 0:
                plan.set_omega(float(om_))
            Q = plan.eval(f_.contiguous())
            if conserve:
                plan.conserve(Q)
            ctx.save_for_backward(f_)
            ctx.omega = plan.info()["omega"]
            return Q

        @staticmethod
        def backward(ctx, gQ):
            (f_,) = ctx.saved_tensors
            want_f = ctx.needs_input_grad[0]
            want_w = len(ctx.needs_input_grad) > 1 and ctx.needs_input_grad[1]
            now = plan.info()["omega"]
            if now != ctx.omega:
                plan.set_omega(ctx.omega)
            try:
                df, dw = plan.vjp(f_.contiguous(), gQ.contiguous(), through_conserve=conserve,
                                  want_df=want_f, want_domega=want_w)
            finally:
                if now != ctx.omega:
                    plan.set_omega(now)
            return (df if want_f else None), (dw.sum().reshape(()) if want_w else None)

    return _Collide.apply(f, omega)
