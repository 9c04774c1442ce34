"""ctypes wrapper around the oracle's plain-C brute-force apply (apply_ref.c).

TEST INFRASTRUCTURE ONLY (see sbm_oracle.py).  build() compiles apply_ref.c with gcc and
OpenMP into oracle/liboracle_apply.so; apply() feeds it the oracle's own setup data.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import sbm_oracle as O

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "apply_ref.c")
_LIB = os.path.join(_HERE, "liboracle_apply.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc -O2 -fopenmp).  Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        _lib.oracle_apply.argtypes = [ctypes.c_int, ctypes.c_int, I64, I64, P, P, I64, P, P, P, P,
                                      I64, P, P, P, P, P, P, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, P, P, ctypes.c_int]
        _lib.oracle_apply.restype = ctypes.c_int
        _lib.oracle_max_threads.restype = ctypes.c_int
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


class NativeApply:
    """Holds the contiguous arrays the C apply needs for one oracle Problem."""

    def __init__(self, prob: O.Problem):
        self.prob = prob
        self.cell_dofs = np.ascontiguousarray(prob.cell_dofs, dtype=np.int64)
        self.cell_matrix = np.ascontiguousarray(O.cell_matrix(prob))
        f = prob.sbm_faces
        self.sbm_cell = np.ascontiguousarray(f[:, 0], dtype=np.int64)
        self.sbm_axis = np.ascontiguousarray(f[:, 1], dtype=np.int32)
        self.sbm_side = np.ascontiguousarray(f[:, 2], dtype=np.int32)
        self.sbm_xi = np.ascontiguousarray(prob.face_xi, dtype=np.float64)
        if prob.disc == "dg":
            fi = prob.interior_faces
        else:
            fi = np.zeros((0, 3), dtype=np.int64)
        self.int_k1 = np.ascontiguousarray(fi[:, 0], dtype=np.int64)
        self.int_k2 = np.ascontiguousarray(fi[:, 1], dtype=np.int64)
        self.int_axis = np.ascontiguousarray(fi[:, 2], dtype=np.int32)
        self.gll = np.ascontiguousarray(prob.nodes)
        gx, gw = O.gauss_rule(prob.p + 1)
        self.gx, self.gw = np.ascontiguousarray(gx), np.ascontiguousarray(gw)

    def __call__(self, u: np.ndarray, n_threads: int = 0, parts=("cell", "sbm", "dg")) -> np.ndarray:
        """v = A u with the terms named in parts: "cell" (Laplace cell term), "sbm"
        (surrogate-boundary faces), "dg" (SIPG interior faces, DG only).  A part left out is
        handed to the C code as zero entities (no faces, or a zero cell matrix)."""
        lib = _load()
        pr = self.prob
        u = np.ascontiguousarray(u, dtype=np.float64)
        v = np.empty(pr.n_dofs)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        cm = self.cell_matrix if "cell" in parts else np.zeros_like(self.cell_matrix)
        n_sbm = self.sbm_cell.shape[0] if "sbm" in parts else 0
        n_int = self.int_k1.shape[0] if "dg" in parts else 0
        rc = lib.oracle_apply(pr.d, pr.p, pr.n_dofs, self.cell_dofs.shape[0], ptr(self.cell_dofs),
                              ptr(cm), n_sbm, ptr(self.sbm_cell),
                              ptr(self.sbm_axis), ptr(self.sbm_side), ptr(self.sbm_xi),
                              n_int, ptr(self.int_k1), ptr(self.int_k2),
                              ptr(self.int_axis), ptr(self.gll), ptr(self.gx), ptr(self.gw),
                              pr.h, pr.sigma_gamma, pr.sigma_f, ptr(u), ptr(v), int(n_threads))
        if rc != 0:
            raise RuntimeError(f"oracle_apply failed with code {rc}")
        return v
