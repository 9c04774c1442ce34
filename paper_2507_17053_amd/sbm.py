"""ctypes binding of libsbm.so (include/sbm.h).  Argument marshalling only.

Device vectors are torch tensors on a ROCm device (torch provides allocation and
streams); every step of the operator runs in the library's HIP kernels.  If the library
has not been built, importing this module raises ImportError: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
# torch ships its own HIP runtime under the same soname as /opt/rocm's; importing torch
# before loading libsbm.so makes the whole process use that one runtime.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsbm.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2507_17053_amd.build` "
                      "(or __graft_entry__.build()) first")
_lib = ctypes.CDLL(LIB_PATH)

SBM_OK, SBM_EINVAL, SBM_ENOMEM, SBM_EHIP, SBM_ENOCONV, SBM_EUNSUPPORTED = range(6)
SBM_CG, SBM_DG = 0, 1
SBM_F64, SBM_F32 = 0, 1
LS_KINDS = {"sphere": 0, "ellipsoid": 1, "torus": 2, "sphere_union": 3, "halfspace": 4, "callback": 5}
SOLVE_MODES = {"gmres": 0, "gmres_ir": 1, "cg": 2, "cg_ir": 3, "cg_rr": 4}
_STATUS = {0: "SBM_OK", 1: "SBM_EINVAL", 2: "SBM_ENOMEM", 3: "SBM_EHIP", 4: "SBM_ENOCONV",
           5: "SBM_EUNSUPPORTED"}


class SbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3)]


class _LevelSet(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("centre", ctypes.c_double * 3), ("radius", ctypes.c_double),
                ("semi_axes", ctypes.c_double * 3), ("R", ctypes.c_double), ("r", ctypes.c_double),
                ("normal", ctypes.c_double * 3), ("offset", ctypes.c_double),
                ("n_spheres", ctypes.c_int), ("centres", ctypes.c_void_p), ("radii", ctypes.c_void_p),
                ("phi", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("user", ctypes.c_void_p)]

_PHI_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)
_GRAD_FN = ctypes.CFUNCTYPE(None, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)


class _Options(ctypes.Structure):
    _fields_ = [("penalty_gamma", ctypes.c_double), ("dg_penalty_gamma", ctypes.c_double),
                ("shift_scale", ctypes.c_double), ("flags", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("outer_its", ctypes.c_int), ("inner_its", ctypes.c_int),
                ("applies_f64", ctypes.c_int), ("applies_f32", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_lib.sbm_setup.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_LevelSet), ctypes.c_int, ctypes.c_int,
                           ctypes.POINTER(_Options), ctypes.POINTER(_P)]
_lib.sbm_info.argtypes = [_P, _I64P, _I64P, _I64P, _I64P, ctypes.POINTER(ctypes.c_size_t)]
_lib.sbm_destroy.argtypes = [_P]
_lib.sbm_destroy.restype = None
_lib.sbm_last_error.restype = ctypes.c_char_p
_lib.sbm_apply.argtypes = [_P, _P, _P, ctypes.c_int, _P]
_lib.sbm_apply_parts.argtypes = [_P, _P, _P, ctypes.c_int, ctypes.c_int, _P]
_lib.sbm_apply_noalloc.argtypes = [_P, _P, _P, ctypes.c_int, _P]
_lib.sbm_apply_batch.argtypes = [ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                 ctypes.c_int, _P]
_lib.sbm_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_P)]
_lib.sbm_batch_run.argtypes = [_P, _P]
_lib.sbm_batch_destroy.argtypes = [_P]
_lib.sbm_dof_points.argtypes = [_P, _P]
_lib.sbm_rhs_points.argtypes = [_P, _P, _P]
_lib.sbm_rhs.argtypes = [_P, _P, _P, _P, _P]
_lib.sbm_solve.argtypes = [_P, _P, _P, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                           _P, ctypes.POINTER(SolveInfo)]
_lib.sbm_solve_batch.argtypes = [ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                 ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P,
                                 ctypes.POINTER(SolveInfo)]
_lib.sbm_diagonal.argtypes = [_P, _P, ctypes.c_int, _P]
_lib.sbm_l2_error.argtypes = [_P, _P, _P, ctypes.POINTER(ctypes.c_double)]
_lib.sbm_set_extension_order.argtypes = [_P, ctypes.c_int]
_lib.sbm_footprint_estimate.argtypes = [ctypes.POINTER(_Mesh), ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                        ctypes.c_int64]
_lib.sbm_footprint_estimate.restype = ctypes.c_size_t
for _n in ("sbm_export_cells", "sbm_export_sbm_faces", "sbm_export_face_xi", "sbm_export_cell_dofs"):
    getattr(_lib, _n).argtypes = [_P, _P]

PART_CELLS, PART_SBM_FACES, PART_ALL, PART_NO_ASSEMBLY, PART_REUSE_FACES = 2, 4, 6, 8, 16
_lib.sbm_layout_stats.argtypes = [_P, _I64P, _I64P, _I64P]
EXPORTED = ["sbm_setup", "sbm_info", "sbm_destroy", "sbm_last_error", "sbm_apply", "sbm_apply_noalloc",
            "sbm_apply_parts",
            "sbm_apply_batch", "sbm_batch_create", "sbm_batch_run", "sbm_batch_destroy", "sbm_layout_stats",
            "sbm_dof_points", "sbm_rhs_points", "sbm_rhs", "sbm_l2_error", "sbm_solve", "sbm_solve_batch", "sbm_diagonal",
            "sbm_footprint_estimate", "sbm_export_cells", "sbm_export_sbm_faces", "sbm_export_face_xi",
            "sbm_export_cell_dofs"]


def _check(status, what):
    if status != SBM_OK:
        raise SbmError(status, f"{what}: {_lib.sbm_last_error().decode()}")


def _mesh(d, n, lo, hi):
    m = _Mesh()
    m.dim = d
    nn = list(n) if np.ndim(n) else [n] * d
    lo_ = list(lo) if np.ndim(lo) else [lo] * d
    hi_ = list(hi) if np.ndim(hi) else [hi] * d
    for k in range(3):
        m.n[k] = int(nn[k]) if k < d else 1
        m.lo[k] = float(lo_[k]) if k < d else 0.0
        m.hi[k] = float(hi_[k]) if k < d else 1.0
    return m


def _levelset(ls: dict, keep: list):
    s = _LevelSet()
    s.kind = LS_KINDS[ls["kind"]]
    c = ls.get("centre", [0, 0, 0])
    for k in range(3):
        s.centre[k] = float(c[k]) if k < len(c) else 0.0
    s.radius = float(ls.get("radius", 0.0))
    ax = ls.get("semi_axes", [1, 1, 1])
    for k in range(3):
        s.semi_axes[k] = float(ax[k]) if k < len(ax) else 1.0
    s.R = float(ls.get("R", 0.0))
    s.r = float(ls.get("r", 0.0))
    nrm = ls.get("normal", [1, 0, 0])
    for k in range(3):
        s.normal[k] = float(nrm[k]) if k < len(nrm) else 0.0
    s.offset = float(ls.get("offset", 0.0))
    if ls["kind"] == "sphere_union":
        cs = np.asarray(ls["centres"], dtype=np.float64)
        c3 = np.zeros((cs.shape[0], 3))
        c3[:, : cs.shape[1]] = cs
        c3 = np.ascontiguousarray(c3)
        rs = np.ascontiguousarray(np.asarray(ls["radii"], dtype=np.float64))
        keep += [c3, rs]
        s.n_spheres = int(rs.shape[0])
        s.centres = c3.ctypes.data
        s.radii = rs.ctypes.data
    if ls["kind"] == "callback":
        d, fphi, fgrad = ls["dim"], ls["phi"], ls["grad"]

        def phi_c(x, _user):
            return float(fphi(np.array([[x[k] for k in range(d)]], dtype=np.float64))[0])

        def grad_c(x, g, _user):
            gv = fgrad(np.array([[x[k] for k in range(d)]], dtype=np.float64))[0]
            for k in range(d):
                g[k] = float(gv[k])

        # a missing function stays NULL (sbm_setup rejects it); the C side calls them during
        # sbm_setup only
        if fphi is not None:
            cp = _PHI_FN(phi_c)
            keep.append(cp)
            s.phi = ctypes.cast(cp, ctypes.c_void_p)
        if fgrad is not None:
            cg = _GRAD_FN(grad_c)
            keep.append(cg)
            s.grad = ctypes.cast(cg, ctypes.c_void_p)
    return s


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def footprint_estimate(d, n, lo, hi, p, disc, n_cells_hint, n_faces_hint):
    m = _mesh(d, n, lo, hi)
    return int(_lib.sbm_footprint_estimate(ctypes.byref(m), p, SBM_CG if disc == "cg" else SBM_DG,
                                           int(n_cells_hint), int(n_faces_hint)))


class Operator:
    """One SBM operator (sbm_setup handle)."""

    def __init__(self, d, n, lo, hi, levelset, p, disc="cg", gamma=10.0, gamma_dg=10.0, shift_scale=1.0,
                 host_only=False, taylor_order=None, host_build=False, solver_graphs=True):
        """taylor_order: None for the full extension (point value at the shifted point), m >= 0
        for the Taylor expansion kept to total order m (sbm_set_extension_order).  host_build:
        build the setup data on host threads (SBM_SETUP_HOST_BUILD) instead of the device."""
        self.d, self.p, self.disc = d, p, disc
        keep = []
        m = _mesh(d, n, lo, hi)
        ls = _levelset(levelset, keep)
        opt = _Options(gamma, gamma_dg, shift_scale,
                       (1 if host_only else 0) | (2 if host_build else 0) | (0 if solver_graphs else 4))
        h = _P()
        _check(_lib.sbm_setup(ctypes.byref(m), ctypes.byref(ls), int(p), SBM_CG if disc == "cg" else SBM_DG,
                              ctypes.byref(opt), ctypes.byref(h)), "sbm_setup")
        self._h = h
        nd, nc, nf, ni = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        nbytes = ctypes.c_size_t()
        _check(_lib.sbm_info(h, ctypes.byref(nd), ctypes.byref(nc), ctypes.byref(nf), ctypes.byref(ni),
                             ctypes.byref(nbytes)), "sbm_info")
        self.n_dofs, self.n_cells, self.n_sbm_faces, self.n_interior_faces = nd.value, nc.value, nf.value, ni.value
        self.nq_face = (p + 1) ** (d - 1)
        self.nb = (p + 1) ** d
        self.taylor_order = None
        if taylor_order is not None:
            self.set_extension_order(taylor_order)

    def set_extension_order(self, m):
        """sbm_set_extension_order: None or a negative m selects the full extension."""
        m = -1 if m is None else int(m)
        _check(_lib.sbm_set_extension_order(self._h, m), "sbm_set_extension_order")
        self.taylor_order = None if m < 0 else m

    @property
    def handle(self):
        return self._h

    @property
    def device_bytes(self):
        """Device bytes the handle holds now (sbm_info): operator data and scratch, plus the
        solver workspace once a solve has allocated it."""
        nbytes = ctypes.c_size_t()
        _check(_lib.sbm_info(self._h, None, None, None, None, ctypes.byref(nbytes)), "sbm_info")
        return nbytes.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.sbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- device work ----
    def apply(self, u, v, stream=None):
        """v = A u for torch device tensors (float64 -> FP64 apply, float32 -> FP32 apply)."""
        import torch
        prec = SBM_F64 if u.dtype == torch.float64 else SBM_F32
        if v.dtype != u.dtype:
            raise TypeError("u and v must have the same dtype")
        if u.numel() != self.n_dofs or v.numel() != self.n_dofs:
            raise ValueError("vector length must be n_dofs")
        if not (u.is_contiguous() and v.is_contiguous()):
            raise ValueError("vectors must be contiguous")
        _check(_lib.sbm_apply(self._h, _dptr(u), _dptr(v), prec, _stream_ptr(stream)), "sbm_apply")

    def apply_noalloc(self, u, v, stream=None):
        """sbm_apply_noalloc: v = A u with the library's static device scratch (no allocation)."""
        import torch
        prec = SBM_F64 if u.dtype == torch.float64 else SBM_F32
        if v.dtype != u.dtype:
            raise TypeError("u and v must have the same dtype")
        if u.numel() != self.n_dofs or v.numel() != self.n_dofs:
            raise ValueError("vector length must be n_dofs")
        if not (u.is_contiguous() and v.is_contiguous()):
            raise ValueError("vectors must be contiguous")
        _check(_lib.sbm_apply_noalloc(self._h, _dptr(u), _dptr(v), prec, _stream_ptr(stream)),
               "sbm_apply_noalloc")

    def apply_parts(self, u, v, parts, stream=None):
        """Diagnostic subset of the apply launches (see sbm_apply_parts)."""
        import torch
        prec = SBM_F64 if u.dtype == torch.float64 else SBM_F32
        _check(_lib.sbm_apply_parts(self._h, _dptr(u), _dptr(v), prec, int(parts), _stream_ptr(stream)),
               "sbm_apply_parts")

    def layout_stats(self):
        """(bricks, DoFs on brick boundaries, boundary slots) of the CG work decomposition."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.sbm_layout_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "sbm_layout_stats")
        return a.value, b.value, c.value

    def diagonal(self, out, stream=None):
        import torch
        prec = SBM_F64 if out.dtype == torch.float64 else SBM_F32
        _check(_lib.sbm_diagonal(self._h, _dptr(out), prec, _stream_ptr(stream)), "sbm_diagonal")

    def rhs(self, f_qp: np.ndarray, g_bp: np.ndarray, out, stream=None):
        f_qp = np.ascontiguousarray(f_qp, dtype=np.float64)
        g_bp = np.ascontiguousarray(g_bp, dtype=np.float64)
        _check(_lib.sbm_rhs(self._h, _hptr(f_qp), _hptr(g_bp), _dptr(out), _stream_ptr(stream)), "sbm_rhs")

    def l2_error(self, x, ustar_qp):
        """sbm_l2_error: ||u_h - u*|| for the FP64 device vector x, u* given at the cell Gauss
        points of rhs_points() (array n_cells x (p+1)^d)."""
        u = np.ascontiguousarray(ustar_qp, dtype=np.float64).reshape(-1)
        if u.size != self.n_cells * self.nb:
            raise ValueError("ustar_qp must have n_cells x (p+1)^d entries")
        out = ctypes.c_double()
        _check(_lib.sbm_l2_error(self._h, _dptr(x), _hptr(u), ctypes.byref(out)), "sbm_l2_error")
        return out.value

    def solve(self, b, x, rel_tol=1e-10, max_it=10000, mode="gmres", restart=50, jacobi=False, stream=None):
        """sbm_solve: A x = b to rel_tol from the initial x (FP64 device tensors of n_dofs).
        mode: "gmres" (FP64 GMRES(restart)), "gmres_ir" (FP64 refinement around FP32 GMRES),
        "cg" (FP64 CG), "cg_ir" (FP64 refinement around FP32 CG), "cg_rr" (FP32 CG with FP64
        residual replacement); the CG modes need a symmetric operator (shift_scale = 0).
        Returns the sbm_solve_info fields as a dict; ENOCONV is reported there, not raised."""
        info = SolveInfo()
        st = _lib.sbm_solve(self._h, _dptr(b), _dptr(x), float(rel_tol), int(max_it), SOLVE_MODES[mode],
                            int(restart), int(bool(jacobi)), _stream_ptr(stream), ctypes.byref(info))
        if st not in (SBM_OK, SBM_ENOCONV):
            _check(st, "sbm_solve")
        return info.as_dict()

    # ---- host-side data ----
    def dof_points(self):
        out = np.empty((self.n_dofs, self.d))
        _check(_lib.sbm_dof_points(self._h, _hptr(out)), "sbm_dof_points")
        return out

    def rhs_points(self, cells=True):
        """(cell Gauss points n_cells x (p+1)^d x d, true-boundary points n_faces x (p+1)^(d-1) x d);
        cells=False skips the cell points (returned as None)."""
        cq = np.empty((self.n_cells, self.nb, self.d)) if cells else None
        bp = np.empty((self.n_sbm_faces, self.nq_face, self.d))
        _check(_lib.sbm_rhs_points(self._h, _hptr(cq) if cells else None, _hptr(bp)), "sbm_rhs_points")
        return cq, bp

    def export_cells(self):
        out = np.empty((self.n_cells, self.d), dtype=np.int32)
        _check(_lib.sbm_export_cells(self._h, _hptr(out)), "sbm_export_cells")
        return out

    def export_sbm_faces(self):
        out = np.empty((self.n_sbm_faces, 3), dtype=np.int32)
        _check(_lib.sbm_export_sbm_faces(self._h, _hptr(out)), "sbm_export_sbm_faces")
        return out

    def export_face_xi(self):
        out = np.empty((self.n_sbm_faces, self.nq_face, self.d))
        _check(_lib.sbm_export_face_xi(self._h, _hptr(out)), "sbm_export_face_xi")
        return out

    def export_cell_dofs(self):
        out = np.empty((self.n_cells, self.nb), dtype=np.int64)
        _check(_lib.sbm_export_cell_dofs(self._h, _hptr(out)), "sbm_export_cell_dofs")
        return out


def _batch_args(ops, us, vs):
    import torch
    n = len(ops)
    if len(us) != n or len(vs) != n:
        raise ValueError("one input and one output per operator")
    dt = us[0].dtype if n else torch.float64
    for o, u, v in zip(ops, us, vs):
        if u.dtype != dt or v.dtype != dt or u.numel() != o.n_dofs or v.numel() != o.n_dofs:
            raise ValueError("vectors must have the operators' sizes and one dtype")
    hs = (_P * max(n, 1))(*[o.handle for o in ops])
    up = (_P * max(n, 1))(*[u.data_ptr() for u in us])
    vp = (_P * max(n, 1))(*[v.data_ptr() for v in vs])
    return n, hs, up, vp, (SBM_F64 if dt == torch.float64 else SBM_F32)


def apply_batch(ops, us, vs, stream=None):
    """v_i = A_i u_i for every i, the operators of one kernel instantiation in shared launches
    (sbm_apply_batch; asynchronous)."""
    n, hs, up, vp, prec = _batch_args(ops, us, vs)
    _check(_lib.sbm_apply_batch(n, hs, up, vp, prec, _stream_ptr(stream)), "sbm_apply_batch")


def solve_batch(ops, bs, xs, rel_tol=1e-10, max_it=1000, mode="gmres_ir", restart=50, stream=None):
    """Lockstep GMRES solves of several systems, their applies batched (sbm_solve_batch).
    bs, xs: FP64 device tensors (xs: initial guesses, overwritten).  Returns one info dict per
    system (status, outer_its, inner_its, applies_f64, applies_f32, rel_residual, seconds);
    does not raise when a system stops short of the tolerance (its status says so)."""
    import torch
    n = len(ops)
    if len(bs) != n or len(xs) != n:
        raise ValueError("one right-hand side and one solution per operator")
    for o, b, x in zip(ops, bs, xs):
        if b.dtype != torch.float64 or x.dtype != torch.float64 or b.numel() != o.n_dofs or x.numel() != o.n_dofs:
            raise ValueError("b and x must be FP64 vectors of the operators' sizes")
    hs = (_P * max(n, 1))(*[o.handle for o in ops])
    bp = (_P * max(n, 1))(*[b.data_ptr() for b in bs])
    xp = (_P * max(n, 1))(*[x.data_ptr() for x in xs])
    infos = (SolveInfo * max(n, 1))()
    st = _lib.sbm_solve_batch(n, hs, bp, xp, float(rel_tol), int(max_it), SOLVE_MODES[mode], int(restart),
                              _stream_ptr(stream), infos)
    if st not in (SBM_OK, SBM_ENOCONV):
        _check(st, "sbm_solve_batch")
    return [infos[i].as_dict() for i in range(n)]


class Batch:
    """A fixed batch of applies v_i = A_i u_i prepared once and run many times (sbm_batch_*):
    operators of one kernel instantiation share one launch per stage; with graph=True the first
    run (on a non-default stream) captures the batch into a HIP graph that later runs replay;
    streams > 1 spreads the groups over that many streams of the batch.  The operators and
    vectors must outlive the batch."""

    def __init__(self, ops, us, vs, graph=True, streams=4):
        n, hs, up, vp, prec = _batch_args(ops, us, vs)
        self._keep = (list(ops), list(us), list(vs))
        h = _P()
        _check(_lib.sbm_batch_create(n, hs, up, vp, prec, 1 if graph else 0, int(streams), ctypes.byref(h)),
               "sbm_batch_create")
        self._b = h

    def run(self, stream=None):
        if self._b is None:
            raise SbmError(SBM_EINVAL, "batch is closed")
        _check(_lib.sbm_batch_run(self._b, _stream_ptr(stream)), "sbm_batch_run")

    def close(self):
        if self._b is not None:
            b, self._b = self._b, None
            _check(_lib.sbm_batch_destroy(b), "sbm_batch_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def status_name(code):
    return _STATUS.get(code, str(code))
