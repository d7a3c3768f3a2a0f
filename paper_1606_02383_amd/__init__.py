"""Python binding of libbemfmm (the MI355X FMM Burton-Miller BEM library).

Argument marshalling only: every numerical step runs in the HIP kernels of
``_lib/libbemfmm.so`` (built by ``paper_1606_02383_amd.build``).  PyTorch
supplies device memory and the current HIP stream.  Importing this module
does not touch the GPU; the first call loads the library and raises if it is
missing or was built without the GPU code.

Vectors are complex128 CUDA (HIP) tensors of length n_tri in the caller's
element order; the library reads and writes them in place on the current
stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

__all__ = ["Plan", "Problem", "GmresOptions", "ObjectiveJ", "FieldPoints", "Coupling",
           "topological_derivative", "BemError", "load_library", "LIB_PATH", "BEM_C128",
           "BEM_C64"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libbemfmm.so")
BEM_C128 = 0
BEM_C64 = 1

STATUS = {0: "BEM_OK", -1: "BEM_E_INVALID", -2: "BEM_E_OOM", -3: "BEM_E_HIP",
          -4: "BEM_E_NOCONV", -5: "BEM_E_BREAKDOWN", -6: "BEM_E_NAN"}

EXPORTS = ["bem_plan_create", "bem_plan_destroy", "bem_plan_get_stats", "bem_fmm_matvec",
           "bem_fmm_matvec_noalloc",
           "bem_fmm_matvec_adjoint", "bem_gmres_solve", "bem_gmres_solve_batch",
           "bem_plane_wave_rhs", "bem_point_source_rhs", "bem_eval_field",
           "bem_eval_field_adjoint", "bem_eval_field_grad", "bem_topological_derivative",
           "bem_field_points_create", "bem_field_points_destroy", "bem_field_points_get_stats",
           "bem_eval_field_grad_fmm",
           "bem_objective_grad", "bem_objective_forward",
           "bem_objective_backward", "bem_tree_export",
           "bem_leaves_export", "bem_lists_export", "bem_near_export", "bem_plan_set_tuning",
           "bem_profile_start", "bem_profile_serial_start",
           "bem_profile_leaf_m2l_start", "bem_profile_stop", "bem_coupling_create",
           "bem_coupling_destroy", "bem_coupling_get_matrix", "bem_coupling_apply",
           "bem_coupled_matvec",
           "bem_coupled_solve", "bem_last_error"]

STAGES = ["gather", "p2p", "p2m", "m2m", "m2l", "l2l", "finish", "m2l_reduce", "m2l_leaf",
          "m2l_leaf_reduce", "pt_l2p", "pt_p2p"]
PROFILE_SLOTS = 64


class _Problem(ctypes.Structure):
    _fields_ = [("vert", ctypes.POINTER(ctypes.c_double)), ("n_vert", ctypes.c_int64),
                ("tri", ctypes.POINTER(ctypes.c_int32)), ("n_tri", ctypes.c_int64),
                ("k", ctypes.c_double), ("alpha_re", ctypes.c_double),
                ("alpha_im", ctypes.c_double), ("near_eta", ctypes.c_double),
                ("leaf_cap", ctypes.c_int32), ("leaf_level", ctypes.c_int32),
                ("order64", ctypes.c_int32), ("order32", ctypes.c_int32),
                ("fmm_tol", ctypes.c_double), ("fmm_tol32", ctypes.c_double),
                ("p_max", ctypes.c_int32), ("m2l_rot", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("use_x0", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("matvec64", ctypes.c_int32),
                ("matvec32", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("resid", ctypes.c_double), ("converged", ctypes.c_int32),
                ("n_hist", ctypes.c_int32), ("hist", ctypes.c_double * 512)]

    def as_dict(self):
        return dict(iterations=self.iterations, matvec64=self.matvec64, matvec32=self.matvec32,
                    restarts=self.restarts, resid=self.resid, converged=bool(self.converged),
                    hist=list(self.hist[:self.n_hist]))


class _Material(ctypes.Structure):
    _fields_ = [("rho_f", ctypes.c_double), ("lam_f", ctypes.c_double),
                ("rho_s", ctypes.c_double), ("lam_s", ctypes.c_double),
                ("omega", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("n_tri", ctypes.c_int64), ("leaf_level", ctypes.c_int32),
                ("n_leaves", ctypes.c_int32), ("n_near", ctypes.c_int64),
                ("n_p2p_pairs", ctypes.c_int64), ("n_m2l", ctypes.c_int64 * 22),
                ("order64", ctypes.c_int32 * 22), ("order32", ctypes.c_int32 * 22),
                ("box_size", ctypes.c_double * 22), ("device_bytes", ctypes.c_int64),
                ("tuned_ms", ctypes.c_double), ("m2l_tile32", ctypes.c_int32 * 22),
                ("schedule", ctypes.c_int32 * 2), ("p2p_grid", ctypes.c_int32 * 2),
                ("m2l_grid", ctypes.c_int32 * 2), ("direct_depth", ctypes.c_int32 * 2),
                ("fmm_err64", ctypes.c_double), ("fmm_err32", ctypes.c_double),
                ("fmm_err64_smooth", ctypes.c_double), ("fmm_err32_smooth", ctypes.c_double),
                ("far_cut", ctypes.c_int32 * 2), ("n_m2l_far", ctypes.c_int64 * 22),
                ("m2l_rot64", ctypes.c_int32 * 22), ("m2l_rot32", ctypes.c_int32 * 22)]


class _PointStats(ctypes.Structure):
    _fields_ = [("n_pts", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("n_box", ctypes.c_int32 * 22), ("n_m2l", ctypes.c_int64 * 22),
                ("order", ctypes.c_int32 * 22), ("n_leaf", ctypes.c_int64),
                ("n_near_pairs", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("n_m2l_far", ctypes.c_int64 * 22), ("far_cut", ctypes.c_int32),
                ("m2l_rot", ctypes.c_int32 * 22)]


_LIB = None


def load_library(path: str = LIB_PATH):
    """Load libbemfmm.so (after torch, so that one HIP runtime is shared)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    import torch  # noqa: F401  (loads the HIP runtime first)
    if not os.path.exists(path):
        raise RuntimeError(f"libbemfmm.so not found at {path}; run paper_1606_02383_amd.build")
    lib = ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    lib.bem_plan_create.argtypes = [ctypes.POINTER(_Problem), i32, vp, ctypes.POINTER(vp)]
    lib.bem_plan_destroy.argtypes = [vp]
    lib.bem_plan_get_stats.argtypes = [vp, i32, ctypes.POINTER(_Stats)]
    lib.bem_fmm_matvec.argtypes = [vp, i32, i32, vp, vp, vp, i32, vp]
    lib.bem_fmm_matvec_noalloc.argtypes = [vp, i32, i32, vp, vp, vp, i32, vp]
    lib.bem_fmm_matvec_adjoint.argtypes = [vp, i32, i32, vp, vp, vp, i32, vp]
    lib.bem_gmres_solve.argtypes = [vp, i32, vp, i32, vp, vp, ctypes.POINTER(_Opts),
                                    ctypes.POINTER(_Info), vp]
    lib.bem_gmres_solve_batch.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(vp), ctypes.POINTER(vp),
                                          ctypes.POINTER(_Opts), ctypes.POINTER(_Info), vp]
    lib.bem_plane_wave_rhs.argtypes = [vp, i32, dp, vp, vp]
    lib.bem_point_source_rhs.argtypes = [vp, i32, vp, vp, i32, vp, vp]
    lib.bem_eval_field.argtypes = [vp, i32, vp, vp, vp, i32, dp, vp, vp]
    lib.bem_eval_field_adjoint.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp]
    lib.bem_eval_field_grad.argtypes = [vp, i32, vp, vp, vp, i32, dp, vp, vp, i32, vp, vp, vp]
    lib.bem_topological_derivative.argtypes = [i32, vp, vp, vp, vp, ctypes.POINTER(_Material),
                                               vp, vp]
    lib.bem_field_points_create.argtypes = [vp, i32, i32, dp, i64, vp, ctypes.POINTER(vp)]
    lib.bem_field_points_destroy.argtypes = [vp]
    lib.bem_field_points_get_stats.argtypes = [vp, ctypes.POINTER(_PointStats)]
    lib.bem_eval_field_grad_fmm.argtypes = [vp, vp, vp, dp, vp, vp, i32, vp, vp, vp]
    lib.bem_objective_grad.argtypes = [vp, i32, vp, dp, dp, i32, ctypes.POINTER(_Opts), dp, vp,
                                       vp, ctypes.POINTER(_Info), ctypes.POINTER(_Info), vp]
    lib.bem_objective_forward.argtypes = [vp, i32, vp, dp, dp, i32, ctypes.POINTER(_Opts), dp,
                                          vp, vp, ctypes.POINTER(_Info), vp]
    lib.bem_objective_backward.argtypes = [vp, i32, vp, vp, vp, dp, i32, ctypes.POINTER(_Opts),
                                           vp, ctypes.POINTER(_Info), vp]
    lib.bem_tree_export.argtypes = [vp, i32, vp, vp, vp]
    lib.bem_leaves_export.argtypes = [vp, i32, vp, vp, vp, vp]
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.bem_lists_export.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, i64p, i64p, i64p, vp]
    lib.bem_near_export.argtypes = [vp, i32, vp, vp, i64p, vp]
    lib.bem_plan_set_tuning.argtypes = [vp, i32, i32, i32, i32, i32, i32]
    lib.bem_profile_start.argtypes = [vp, i32]
    lib.bem_profile_serial_start.argtypes = [vp, i32]
    lib.bem_profile_leaf_m2l_start.argtypes = [vp, i32]
    lib.bem_profile_stop.argtypes = [vp, i32, dp, ctypes.POINTER(ctypes.c_int32)]
    ip = ctypes.POINTER(ctypes.c_int32)
    dd = ctypes.c_double
    lib.bem_coupling_create.argtypes = [vp, i32, dp, i64, ip, i64, ip, dd, dd, dd, dd, dd, vp,
                                        ctypes.POINTER(vp)]
    lib.bem_coupling_destroy.argtypes = [vp]
    lib.bem_coupling_get_matrix.argtypes = [vp, vp, vp]
    lib.bem_coupling_apply.argtypes = [vp, i32, vp, vp, vp]
    lib.bem_coupled_matvec.argtypes = [vp, i32, vp, vp, vp]
    lib.bem_coupled_solve.argtypes = [vp, i32, vp, vp, ctypes.POINTER(_Opts),
                                      ctypes.POINTER(_Info), vp]
    lib.bem_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "bem_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _LIB = lib
    return lib


class BemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _check(code):
    if code != 0:
        raise BemError(code, _LIB.bem_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Problem:
    """One mesh + wavenumber.  V (n_vert, 3) float64, T (n_tri, 3) int32,
    triangles counter-clockwise seen from the fluid."""
    V: np.ndarray
    T: np.ndarray
    k: float
    alpha: complex | None = None     # default i/k
    near_eta: float = 2.0
    leaf_cap: int = 64
    leaf_level: int = 0              # > 0 forced, < 0 tuned at plan creation
    order64: int = 0
    order32: int = 0
    fmm_tol: float = 1e-6            # float64 product error target (<= 0: level rule)
    fmm_tol32: float = 0.0           # float32: orders raised to meet it (<= 0: rule)
    p_max: int = 40
    m2l_rot: int = 0                 # M2L per level: 0 timed, 1 dense, 2 rotation-based


@dataclass
class GmresOptions:
    tol: float = 1e-6
    restart: int = 50
    max_iter: int = 2000
    mode: int = 0              # 0 float64, 1 float32 inner + float64 refinement
    inner_tol: float = 1e-3
    use_x0: bool = False

    def c(self):
        return _Opts(self.tol, self.restart, self.max_iter, self.mode, self.inner_tol,
                     int(self.use_x0))


class Plan:
    """A built plan (tree, lists, near field, operators) for one or more problems."""

    def __init__(self, problems):
        import torch
        lib = load_library()
        if isinstance(problems, Problem):
            problems = [problems]
        self._keep = []
        arr = (_Problem * len(problems))()
        for i, p in enumerate(problems):
            V = np.ascontiguousarray(p.V, dtype=np.float64)
            T = np.ascontiguousarray(p.T, dtype=np.int32)
            self._keep += [V, T]
            a = (1j / p.k if p.k else 0j) if p.alpha is None else complex(p.alpha)
            arr[i] = _Problem(V.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), V.shape[0],
                              T.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), T.shape[0],
                              float(p.k), a.real, a.imag, float(p.near_eta), int(p.leaf_cap),
                              int(p.leaf_level), int(p.order64), int(p.order32),
                              float(p.fmm_tol), float(p.fmm_tol32), int(p.p_max),
                              int(p.m2l_rot))
        self.problems = list(problems)
        self.n = [int(np.asarray(p.T).shape[0]) for p in problems]
        h = ctypes.c_void_p()
        _check(lib.bem_plan_create(arr, len(problems), _stream(), ctypes.byref(h)))
        self._h = h
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _LIB.bem_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- helpers
    def _vec(self, prob, nrhs=1):
        import torch
        shape = (self.n[prob],) if nrhs == 1 else (nrhs, self.n[prob])
        return torch.empty(shape, dtype=torch.complex128, device=self.device)

    def _in(self, t, prob):
        import torch
        if t is None:
            return None
        t = torch.as_tensor(t).to(device=self.device, dtype=torch.complex128).contiguous()
        if t.shape[-1] != self.n[prob]:
            raise ValueError(f"vector length {t.shape[-1]} != n_tri {self.n[prob]}")
        return t

    def stats(self, prob=0):
        st = _Stats()
        _check(_LIB.bem_plan_get_stats(self._h, prob, ctypes.byref(st)))
        L = st.leaf_level
        return dict(n_tri=st.n_tri, leaf_level=L, n_leaves=st.n_leaves, n_near=st.n_near,
                    n_p2p_pairs=st.n_p2p_pairs, n_m2l=list(st.n_m2l[:L + 1]),
                    order64=list(st.order64[:L + 1]), order32=list(st.order32[:L + 1]),
                    box_size=list(st.box_size[:L + 1]), device_bytes=st.device_bytes,
                    tuned_ms=st.tuned_ms, m2l_tile32=list(st.m2l_tile32[:L + 1]),
                    schedule=list(st.schedule), p2p_grid=list(st.p2p_grid),
                    m2l_grid=list(st.m2l_grid), direct_depth=list(st.direct_depth),
                    fmm_err64=st.fmm_err64, fmm_err32=st.fmm_err32,
                    fmm_err64_smooth=st.fmm_err64_smooth, fmm_err32_smooth=st.fmm_err32_smooth,
                    far_cut=list(st.far_cut), n_m2l_far=list(st.n_m2l_far)[:L + 1],
                    m2l_rot64=list(st.m2l_rot64)[:L + 1], m2l_rot32=list(st.m2l_rot32)[:L + 1])

    # ---- products
    def matvec(self, p, q=None, prec=BEM_C128, prob=0, out=None):
        """y = (I/2 - K - alpha H) p + (S + alpha K' + alpha/2 I) q."""
        p, q = self._in(p, prob), self._in(q, prob)
        nrhs = 1 if p.dim() == 1 else p.shape[0]
        y = out if out is not None else self._vec(prob, nrhs)
        _check(_LIB.bem_fmm_matvec(self._h, prob, prec, _ptr(p), _ptr(q), _ptr(y), nrhs, _stream()))
        return y

    def matvec_adjoint(self, y, prec=BEM_C128, prob=0, want_w=True):
        """(u, w) = ((I/2 - K - alpha H)^H y, (S + alpha K' + alpha/2 I)^H y);
        want_w=False asks for u alone (w is returned as None)."""
        y = self._in(y, prob)
        nrhs = 1 if y.dim() == 1 else y.shape[0]
        u = self._vec(prob, nrhs)
        w = self._vec(prob, nrhs) if want_w else None
        _check(_LIB.bem_fmm_matvec_adjoint(self._h, prob, prec, _ptr(y), _ptr(u), _ptr(w), nrhs,
                                           _stream()))
        return u, w

    def solve(self, b, sigma=None, adjoint=False, opts: GmresOptions | None = None, prob=0, x0=None):
        """GMRES on A(sigma) = (I/2 - K - alpha H) + (S + alpha K' + alpha/2 I) diag(sigma)."""
        opts = opts or GmresOptions()
        b, sigma = self._in(b, prob), self._in(sigma, prob)
        x = self._vec(prob) if x0 is None else self._in(x0, prob).clone()
        if x0 is not None:
            opts = GmresOptions(**{**opts.__dict__, "use_x0": True})
        info = _Info()
        o = opts.c()
        code = _LIB.bem_gmres_solve(self._h, prob, _ptr(sigma), int(adjoint), _ptr(b), _ptr(x),
                                    ctypes.byref(o), ctypes.byref(info), _stream())
        d = info.as_dict()
        if code not in (0, -4):
            _check(code)
        d["status"] = STATUS.get(code, code)
        return x, d

    def solve_batch(self, systems, opts: GmresOptions | None = None):
        """Lockstep batched solves.  systems: list of dicts with keys
        'prob', 'b' and optional 'sigma', 'adjoint'.  Returns (xs, infos)."""
        opts = opts or GmresOptions()
        ns = len(systems)
        probs = (ctypes.c_int32 * ns)()
        adj = (ctypes.c_int32 * ns)()
        sg = (ctypes.c_void_p * ns)()
        bs = (ctypes.c_void_p * ns)()
        xs_p = (ctypes.c_void_p * ns)()
        keep, xs = [], []
        for i, s in enumerate(systems):
            pr = int(s.get("prob", 0))
            b = self._in(s["b"], pr)
            sigma = self._in(s.get("sigma"), pr)
            x = self._vec(pr)
            keep += [b, sigma]
            xs.append(x)
            probs[i] = pr
            adj[i] = int(bool(s.get("adjoint", False)))
            sg[i] = sigma.data_ptr() if sigma is not None else None
            bs[i] = b.data_ptr()
            xs_p[i] = x.data_ptr()
        infos = (_Info * ns)()
        o = opts.c()
        code = _LIB.bem_gmres_solve_batch(self._h, ns, probs, sg, adj, bs, xs_p, ctypes.byref(o),
                                          infos, _stream())
        if code not in (0, -4):
            _check(code)
        return xs, [infos[i].as_dict() for i in range(ns)]

    def plane_wave_rhs(self, direction, prob=0):
        d = np.ascontiguousarray(direction, dtype=np.float64)
        b = self._vec(prob)
        _check(_LIB.bem_plane_wave_rhs(self._h, prob, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       _ptr(b), _stream()))
        return b

    def point_source_rhs(self, src, amp, prob=0):
        """b = p_inc + alpha dp_inc/dn for point sources (src (m, 3), amp (m,))."""
        import torch
        src = torch.as_tensor(np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3))
        src = src.to(self.device)
        amp = torch.as_tensor(np.asarray(amp, dtype=np.complex128).reshape(-1)).to(self.device)
        if amp.shape[0] != src.shape[0]:
            raise ValueError("src and amp differ in length")
        b = self._vec(prob)
        _check(_LIB.bem_point_source_rhs(self._h, prob, _ptr(src), _ptr(amp), src.shape[0],
                                         _ptr(b), _stream()))
        return b

    def eval_field(self, p, q, pts, direction=None, prob=0):
        import torch
        p, q = self._in(p, prob), self._in(q, prob)
        pts = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64)).to(self.device)
        out = torch.empty(pts.shape[0], dtype=torch.complex128, device=self.device)
        dptr = None
        if direction is not None:
            d = np.ascontiguousarray(direction, dtype=np.float64)
            self._keep.append(d)
            dptr = d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        _check(_LIB.bem_eval_field(self._h, prob, _ptr(p), _ptr(q),
                                   ctypes.cast(pts.data_ptr(), ctypes.POINTER(ctypes.c_double)),
                                   pts.shape[0], dptr, _ptr(out), _stream()))
        return out

    def eval_field_grad(self, p, q, pts, direction=None, src=None, amp=None, prob=0):
        """Total field (n_pts,) and its gradient (n_pts, 3) at exterior points:
        incident plane wave (direction) and/or point sources (src, amp) plus
        the representation of the boundary data p, q."""
        import torch
        p, q = self._in(p, prob), self._in(q, prob)
        pts = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3))
        pts = pts.to(self.device)
        n = pts.shape[0]
        out = torch.empty(n, dtype=torch.complex128, device=self.device)
        grad = torch.empty((n, 3), dtype=torch.complex128, device=self.device)
        dptr = None
        if direction is not None:
            d = np.ascontiguousarray(direction, dtype=np.float64)
            self._keep.append(d)
            dptr = d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s_t = a_t = None
        if src is not None:
            s_t = torch.as_tensor(np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3))
            s_t = s_t.to(self.device)
            a_t = torch.as_tensor(amp).to(device=self.device, dtype=torch.complex128)
            a_t = a_t.reshape(-1).contiguous()
        _check(_LIB.bem_eval_field_grad(self._h, prob, _ptr(p), _ptr(q), _ptr(pts), n, dptr,
                                        _ptr(s_t), _ptr(a_t), 0 if s_t is None else s_t.shape[0],
                                        _ptr(out), _ptr(grad), _stream()))
        return out, grad

    def eval_field_adjoint(self, pts, c, prob=0):
        import torch
        pts = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64)).to(self.device)
        c = torch.as_tensor(c).to(device=self.device, dtype=torch.complex128).contiguous()
        rp, rq = self._vec(prob), self._vec(prob)
        _check(_LIB.bem_eval_field_adjoint(self._h, prob,
                                           ctypes.cast(pts.data_ptr(), ctypes.POINTER(ctypes.c_double)),
                                           pts.shape[0], _ptr(c), _ptr(rp), _ptr(rq), _stream()))
        return rp, rq

    def objective_grad(self, beta, direction, pts, opts: GmresOptions | None = None, prob=0,
                       need_grad=True):
        """J = sum |p(x_m)|^2 for the admittance problem and dJ/dRe(beta) + i dJ/dIm(beta)."""
        opts = opts or GmresOptions(tol=1e-10)
        beta = self._in(beta, prob)
        d = np.ascontiguousarray(direction, dtype=np.float64)
        P = np.ascontiguousarray(pts, dtype=np.float64)
        J = ctypes.c_double()
        grad = self._vec(prob) if need_grad else None
        pout = self._vec(prob)
        fi, ai = _Info(), _Info()
        o = opts.c()
        _check(_LIB.bem_objective_grad(self._h, prob, _ptr(beta),
                                       d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), P.shape[0],
                                       ctypes.byref(o), ctypes.byref(J), _ptr(grad), _ptr(pout),
                                       ctypes.byref(fi), ctypes.byref(ai), _stream()))
        return J.value, grad, pout, fi.as_dict(), ai.as_dict()

    def objective_forward(self, beta, direction, pts, opts: GmresOptions | None = None, prob=0):
        """State solve and J = sum |p(x_m)|^2: returns (J, p, p_obs, info)."""
        import torch
        opts = opts or GmresOptions(tol=1e-10)
        beta = self._in(beta, prob)
        d = np.ascontiguousarray(direction, dtype=np.float64)
        P = np.ascontiguousarray(pts, dtype=np.float64)
        J = ctypes.c_double()
        p = self._vec(prob)
        pobs = torch.empty(P.shape[0], dtype=torch.complex128, device=self.device)
        fi = _Info()
        o = opts.c()
        _check(_LIB.bem_objective_forward(self._h, prob, _ptr(beta),
                                          d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          P.shape[0], ctypes.byref(o), ctypes.byref(J), _ptr(p),
                                          _ptr(pobs), ctypes.byref(fi), _stream()))
        return J.value, p, pobs, fi.as_dict()

    def objective_backward(self, beta, p, pobs, pts, opts: GmresOptions | None = None, prob=0):
        """Adjoint solve and dJ/dRe(beta) + i dJ/dIm(beta) from the forward
        half's p and p_obs: returns (grad, info)."""
        opts = opts or GmresOptions(tol=1e-10)
        beta, p = self._in(beta, prob), self._in(p, prob)
        import torch
        pobs = torch.as_tensor(pobs).to(device=self.device, dtype=torch.complex128).contiguous()
        P = np.ascontiguousarray(pts, dtype=np.float64)
        if pobs.shape[0] != P.shape[0]:
            raise ValueError("p_obs and pts differ in length")
        grad = self._vec(prob)
        ai = _Info()
        o = opts.c()
        _check(_LIB.bem_objective_backward(self._h, prob, _ptr(beta), _ptr(p), _ptr(pobs),
                                           P.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           P.shape[0], ctypes.byref(o), _ptr(grad),
                                           ctypes.byref(ai), _stream()))
        return grad, ai.as_dict()

    def set_tuning(self, prec=BEM_C128, prob=0, schedule=-1, p2p_grid=-1, m2l_grid=-1,
                   direct_depth=-1):
        """Override the choices timed at plan creation (negative: keep)."""
        _check(_LIB.bem_plan_set_tuning(self._h, prob, prec, int(schedule), int(p2p_grid),
                                        int(m2l_grid), int(direct_depth)))

    def profile_start(self, prob=0, leaf_m2l_only=False, serial=False):
        """Stage timing until profile_stop: every stage (event pairs on the
        streams), or only the leaf-level M2L with events attached to its
        launches (leaf_m2l_only; leaves the schedule of a timed region as is),
        or every stage alone on the GPU (serial: one stream, one stage after
        another)."""
        if leaf_m2l_only:
            _check(_LIB.bem_profile_leaf_m2l_start(self._h, prob))
        elif serial:
            _check(_LIB.bem_profile_serial_start(self._h, prob))
        else:
            _check(_LIB.bem_profile_start(self._h, prob))

    def profile_stop(self, prob=0):
        """{(stage, 'f64'|'f32', 'fwd'|'adj'): (total ms, executions)}"""
        ms = (ctypes.c_double * PROFILE_SLOTS)()
        calls = (ctypes.c_int32 * PROFILE_SLOTS)()
        _check(_LIB.bem_profile_stop(self._h, prob, ms, calls))
        out = {}
        for slot in range(PROFILE_SLOTS):
            if calls[slot]:
                st = STAGES[slot % 16] if slot % 16 < len(STAGES) else str(slot % 16)
                key = (st, "f32" if (slot // 16) % 2 else "f64", "adj" if slot >= 32 else "fwd")
                out[key] = (ms[slot], calls[slot])
        return out

    def tree_export(self, prob=0):
        import torch
        keys = torch.empty(self.n[prob], dtype=torch.int64, device=self.device)
        perm = torch.empty(self.n[prob], dtype=torch.int32, device=self.device)
        _check(_LIB.bem_tree_export(self._h, prob, _ptr(keys), _ptr(perm), _stream()))
        return keys, perm

    def leaves_export(self, prob=0):
        import torch
        nl = self.stats(prob)["n_leaves"]
        keys = torch.empty(nl, dtype=torch.int64, device=self.device)
        s = torch.empty(nl, dtype=torch.int32, device=self.device)
        e = torch.empty(nl, dtype=torch.int32, device=self.device)
        _check(_LIB.bem_leaves_export(self._h, prob, _ptr(keys), _ptr(s), _ptr(e), _stream()))
        return keys, s, e

    def lists_export(self, level, prob=0):
        """Box keys, V-list (destination, source) index pairs and, at the leaf
        level, the U lists (CSR) of tree level ``level``."""
        import torch
        nb, npr, nu = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_LIB.bem_lists_export(self._h, prob, int(level), None, None, None, None, None,
                                     ctypes.byref(nb), ctypes.byref(npr), ctypes.byref(nu),
                                     _stream()))
        dev = self.device
        keys = torch.empty(nb.value, dtype=torch.int64, device=dev)
        vd = torch.empty(max(npr.value, 1), dtype=torch.int32, device=dev)
        vs = torch.empty(max(npr.value, 1), dtype=torch.int32, device=dev)
        up = torch.empty(nb.value + 1, dtype=torch.int32, device=dev)
        ui = torch.empty(max(nu.value, 1), dtype=torch.int32, device=dev)
        _check(_LIB.bem_lists_export(self._h, prob, int(level), _ptr(keys), _ptr(vd), _ptr(vs),
                                     _ptr(up), _ptr(ui), None, None, None, _stream()))
        out = dict(keys=keys, v_dst=vd[:npr.value], v_src=vs[:npr.value])
        if nu.value:
            out.update(u_ptr=up, u_idx=ui[:nu.value])
        return out

    def near_export(self, prob=0):
        """Near-field pairs as CSR by target (sorted element order)."""
        import torch
        nn = ctypes.c_int64()
        _check(_LIB.bem_near_export(self._h, prob, None, None, ctypes.byref(nn), _stream()))
        ptr = torch.empty(self.n[prob] + 1, dtype=torch.int32, device=self.device)
        col = torch.empty(max(nn.value, 1), dtype=torch.int32, device=self.device)
        _check(_LIB.bem_near_export(self._h, prob, _ptr(ptr), _ptr(col), None, _stream()))
        return ptr, col[:nn.value]


class Coupling:
    """The BEM-FEM coupled operator of an elastic body (Sec. 2.3, Eqs.
    renritupu, kousokuu, GMRES) on one problem of a plan: a tetrahedral mesh
    (nodes n x 3, tets m x 4) whose boundary faces are the problem's
    triangles (tri, its element order, as node indices), isotropic material
    (lam, mu, rho_s), fluid density rho_f and angular frequency omega.  The
    device builds C = -rho_f omega^2 Tc (K - omega^2 M)^-1 N once; products
    and solves apply Mp + Mq C."""

    def __init__(self, plan, nodes, tets, tri, lam, mu, rho_s, rho_f, omega, prob=0):
        self._plan = plan  # keeps the plan alive while the coupling exists
        self.prob = prob
        self.n = plan.n[prob]
        nodes = np.ascontiguousarray(nodes, dtype=np.float64).reshape(-1, 3)
        tets = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
        tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
        if tri.shape[0] != self.n:
            raise ValueError("tri must hold the problem's triangles")
        ip = ctypes.POINTER(ctypes.c_int32)
        h = ctypes.c_void_p()
        _check(_LIB.bem_coupling_create(plan._h, prob,
                                        nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        nodes.shape[0], tets.ctypes.data_as(ip), tets.shape[0],
                                        tri.ctypes.data_as(ip), float(lam), float(mu),
                                        float(rho_s), float(rho_f), float(omega), _stream(),
                                        ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _LIB.bem_coupling_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matrix(self):
        """C (n x n float64, device)."""
        import torch
        C = torch.empty((self.n, self.n), dtype=torch.float64, device=self._plan.device)
        _check(_LIB.bem_coupling_get_matrix(self._h, _ptr(C), _stream()))
        return C

    def apply(self, v, transpose=False):
        """C v (or C^T v): the body's response dp/dn to the boundary pressure v."""
        v = self._plan._in(v, self.prob)
        out = self._plan._vec(self.prob)
        _check(_LIB.bem_coupling_apply(self._h, int(bool(transpose)), _ptr(v), _ptr(out),
                                       _stream()))
        return out

    def matvec(self, p, prec=BEM_C128):
        """y = Mp p + Mq C p."""
        p = self._plan._in(p, self.prob)
        y = self._plan._vec(self.prob)
        _check(_LIB.bem_coupled_matvec(self._h, int(prec), _ptr(p), _ptr(y), _stream()))
        return y

    def solve(self, b, adjoint=False, opts: GmresOptions | None = None):
        """GMRES on Mp + Mq C (or its conjugate transpose)."""
        opts = opts or GmresOptions()
        b = self._plan._in(b, self.prob)
        x = self._plan._vec(self.prob)
        info = _Info()
        o = opts.c()
        code = _LIB.bem_coupled_solve(self._h, int(adjoint), _ptr(b), _ptr(x), ctypes.byref(o),
                                      ctypes.byref(info), _stream())
        d = info.as_dict()
        if code not in (0, -4):
            _check(code)
        d["status"] = STATUS.get(code, code)
        return x, d


class FieldPoints:
    """A fixed set of evaluation points (e.g. the design-domain lattice) sorted
    into an octree on the grid of one problem of a plan, for FMM evaluation of
    the total field and its gradient (bem_eval_field_grad_fmm)."""

    def __init__(self, plan, pts, prec=BEM_C128, prob=0):
        self._plan = plan  # keeps the plan alive while the points exist
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        self.n = pts.shape[0]
        self.prob = prob
        h = ctypes.c_void_p()
        _check(_LIB.bem_field_points_create(plan._h, prob, int(prec),
                                            pts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            self.n, _stream(), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _LIB.bem_field_points_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self):
        st = _PointStats()
        _check(_LIB.bem_field_points_get_stats(self._h, ctypes.byref(st)))
        L = st.levels
        return dict(n_pts=st.n_pts, levels=L, n_box=list(st.n_box)[:L + 1],
                    n_m2l=list(st.n_m2l)[:L + 1], order=list(st.order)[:L + 1],
                    n_leaf=st.n_leaf, n_near_pairs=st.n_near_pairs,
                    device_bytes=st.device_bytes, n_m2l_far=list(st.n_m2l_far)[:L + 1],
                    far_cut=st.far_cut, m2l_rot=list(st.m2l_rot)[:L + 1])

    def eval_field_grad(self, p, q=None, direction=None, src=None, amp=None):
        """Total field (n,) and gradient (n, 3) at the points, as
        Plan.eval_field_grad, with the boundary sums by the FMM."""
        import torch
        plan = self._plan
        p, q = plan._in(p, self.prob), plan._in(q, self.prob)
        out = torch.empty(self.n, dtype=torch.complex128, device=plan.device)
        grad = torch.empty((self.n, 3), dtype=torch.complex128, device=plan.device)
        dptr = None
        if direction is not None:
            d = np.ascontiguousarray(direction, dtype=np.float64)
            plan._keep.append(d)
            dptr = d.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s_t = a_t = None
        if src is not None:
            s_t = torch.as_tensor(np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3))
            s_t = s_t.to(plan.device)
            a_t = torch.as_tensor(amp).to(device=plan.device, dtype=torch.complex128)
            a_t = a_t.reshape(-1).contiguous()
        _check(_LIB.bem_eval_field_grad_fmm(self._h, _ptr(p), _ptr(q), dptr, _ptr(s_t),
                                            _ptr(a_t), 0 if s_t is None else s_t.shape[0],
                                            _ptr(out), _ptr(grad), _stream()))
        return out, grad


def topological_derivative(p, grad_p, pt, grad_pt, rho_f=1.0, lam_f=1.0, rho_s=float("inf"),
                           lam_s=float("inf"), omega=1.0):
    """T_Omega at points (Eq. danseitpoderi) from the state and adjoint fields
    and their gradients (device tensors); infinite rho_s, lam_s: sound-hard."""
    import torch
    load_library()
    p, pt = p.contiguous(), pt.contiguous()
    grad_p, grad_pt = grad_p.contiguous(), grad_pt.contiguous()
    n = p.shape[0]
    T = torch.empty(n, dtype=torch.float64, device=p.device)
    m = _Material(rho_f, lam_f, rho_s, lam_s, omega)
    _check(_LIB.bem_topological_derivative(n, _ptr(p), _ptr(grad_p), _ptr(pt), _ptr(grad_pt),
                                           ctypes.byref(m), _ptr(T), _stream()))
    return T


def _objective_function():
    import torch

    class ObjectiveJ(torch.autograd.Function):
        """J(beta) = sum_m |p(x_m)|^2 for the plane-wave admittance problem;
        backward is the discrete adjoint (conjugate-transposed FMM solve)."""

        @staticmethod
        def forward(ctx, beta, plan, direction, pts, opts=None, prob=0):
            # the state solve only; the adjoint solve runs in backward
            b = beta.detach()
            J, p, pobs, _ = plan.objective_forward(b, direction, pts, opts, prob)
            ctx.save_for_backward(b, p, pobs)
            ctx.plan, ctx.pts, ctx.opts, ctx.prob = plan, pts, opts, prob
            return torch.tensor(J, dtype=torch.float64, device=beta.device)

        @staticmethod
        def backward(ctx, gout):
            b, p, pobs = ctx.saved_tensors
            grad, _ = ctx.plan.objective_backward(b, p, pobs, ctx.pts, ctx.opts, ctx.prob)
            return gout * grad, None, None, None, None, None

    return ObjectiveJ


class _Lazy:
    def __init__(self):
        self._cls = None

    def apply(self, *a, **k):
        if self._cls is None:
            self._cls = _objective_function()
        return self._cls.apply(*a, **k)


ObjectiveJ = _Lazy()
