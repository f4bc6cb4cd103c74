"""ctypes front end of the CPU oracle.

TEST INFRASTRUCTURE ONLY: the oracle is the plain FP64 reference the HIP
library is checked against.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import it.  It imports nothing from the HIP package.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB
from .build import build as build_oracle


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """Wrapper over one build of fv_oracle.c (the default one, or a test copy)."""

    def __init__(self, path: str = LIB):
        L = ctypes.CDLL(path)
        i64, dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        L.oracle_face_flux.argtypes = [vp, vp, dbl, dbl, dbl, vp]
        L.oracle_face_flux.restype = None
        L.oracle_cell_residual.argtypes = [i64, vp, vp, vp, dbl, vp]
        L.oracle_cell_residual.restype = None
        L.oracle_step.argtypes = [i64, vp, vp, vp, dbl, dbl, i64, vp]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_step_threads.argtypes = [i64, vp, vp, vp, dbl, dbl, i64, vp, ctypes.c_int]
        L.oracle_step_threads.restype = ctypes.c_int
        L.oracle_cm_order.argtypes = [i64, vp, vp]
        L.oracle_cm_order.restype = ctypes.c_int
        L.oracle_am1_order.argtypes = [i64, vp, vp]
        L.oracle_am1_order.restype = ctypes.c_int
        L.oracle_am1_exact_sbw.argtypes = [i64, vp, vp, vp]
        L.oracle_am1_exact_sbw.restype = ctypes.c_int
        L.oracle_bandwidth.argtypes = [i64, vp, vp, vp]
        L.oracle_am1_bounded.argtypes = [i64, vp, i64, vp, vp, i64, vp, i64, vp, vp]
        L.oracle_am1_bounded.restype = ctypes.c_int
        L.oracle_bandwidth.restype = ctypes.c_int
        self.lib = L
        self.path = path

    def face_flux(self, UL, UR, nx: float, ny: float, gamma: float = 1.4) -> np.ndarray:
        """R_n F |n| for one face (x-y frame, times the face length)."""
        UL = np.ascontiguousarray(UL, dtype=np.float64)
        UR = np.ascontiguousarray(UR, dtype=np.float64)
        out = np.empty(4, dtype=np.float64)
        self.lib.oracle_face_flux(_p(UL), _p(UR), float(nx), float(ny), float(gamma), _p(out))
        return out

    def cell_residual(self, i: int, nbr, nrm, U, gamma: float = 1.4) -> np.ndarray:
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        nrm = np.ascontiguousarray(nrm, dtype=np.float64)
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.empty(4, dtype=np.float64)
        self.lib.oracle_cell_residual(int(i), _p(nbr), _p(nrm), _p(U), float(gamma), _p(out))
        return out

    def step(self, nbr, nrm, area, U, dt: float, n_steps: int, gamma: float = 1.4) -> np.ndarray:
        """U after n_steps forward-Euler Lax-Friedrichs steps (the input is not modified)."""
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        nrm = np.ascontiguousarray(nrm, dtype=np.float64)
        area = np.ascontiguousarray(area, dtype=np.float64)
        out = np.array(U, dtype=np.float64, order="C", copy=True)
        n = nbr.shape[0]
        if out.shape != (n, 4) or nrm.shape != (n, 3, 2) or area.shape != (n,):
            raise ValueError("shape mismatch")
        rc = self.lib.oracle_step(n, _p(nbr), _p(nrm), _p(area), float(gamma), float(dt),
                                  int(n_steps), _p(out))
        if rc != 0:
            raise RuntimeError("oracle_step failed")
        return out

    def step_threads(self, nbr, nrm, area, U, dt: float, n_steps: int, n_threads: int,
                     gamma: float = 1.4):
        """step() with each step's cell loop shared by n_threads OpenMP
        threads (bitwise the same result); returns (U, threads used)."""
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        nrm = np.ascontiguousarray(nrm, dtype=np.float64)
        area = np.ascontiguousarray(area, dtype=np.float64)
        out = np.array(U, dtype=np.float64, order="C", copy=True)
        n = nbr.shape[0]
        if out.shape != (n, 4) or nrm.shape != (n, 3, 2) or area.shape != (n,):
            raise ValueError("shape mismatch")
        used = self.lib.oracle_step_threads(n, _p(nbr), _p(nrm), _p(area), float(gamma),
                                            float(dt), int(n_steps), _p(out), int(n_threads))
        if used < 1:
            raise RuntimeError("oracle_step_threads failed")
        return out, int(used)

    def cm_order(self, nbr) -> np.ndarray:
        """Cuthill-McKee permutation, new label -> old id."""
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        perm = np.empty(nbr.shape[0], dtype=np.int32)
        if self.lib.oracle_cm_order(nbr.shape[0], _p(nbr), _p(perm)) != 0:
            raise RuntimeError("oracle_cm_order failed")
        return perm

    def am1_exact_sbw(self, nbr):
        """(AM1 order, per-position serial bandwidth by Eq. exact-sbw; -1 where
        undefined)."""
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        n = nbr.shape[0]
        perm = np.empty(n, dtype=np.int32)
        ex = np.empty(n, dtype=np.int64)
        if self.lib.oracle_am1_exact_sbw(n, _p(nbr), _p(perm), _p(ex)) != 0:
            raise RuntimeError("oracle_am1_exact_sbw failed")
        return perm, ex

    def am1_order(self, nbr) -> np.ndarray:
        """Amoeba1 permutation (section 4.2), new label -> old id."""
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        perm = np.empty(nbr.shape[0], dtype=np.int32)
        if self.lib.oracle_am1_order(nbr.shape[0], _p(nbr), _p(perm)) != 0:
            raise RuntimeError("oracle_am1_order failed")
        return perm

    def am1_bounded(self, nbr, bound: int, cap_factor: int = 16) -> dict:
        """Access pattern of serial bandwidth <= bound (section 4.3): idx
        (vertex of each load), ex (1 where that load executes it),
        part_begin (offsets of the parts), perfect (per vertex)."""
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        n = nbr.shape[0]
        cap = cap_factor * n
        idx = np.empty(cap, dtype=np.int32)
        ex = np.empty(cap, dtype=np.uint8)
        part_begin = np.empty(n + 1, dtype=np.int64)
        perfect = np.empty(n, dtype=np.uint8)
        counts = np.zeros(2, dtype=np.int64)
        rc = self.lib.oracle_am1_bounded(n, _p(nbr), int(bound), _p(idx), _p(ex), cap,
                                         _p(part_begin), n + 1, _p(perfect), _p(counts))
        if rc != 0:
            raise RuntimeError(f"oracle_am1_bounded failed ({rc})")
        m, parts = int(counts[0]), int(counts[1])
        return {"idx": idx[:m].copy(), "ex": ex[:m].copy(),
                "part_begin": part_begin[:parts + 1].copy(), "perfect": perfect.copy()}

    def bandwidth(self, nbr, label) -> dict:
        """B_f(G), C_BW and S_BW of the labelling label[old id] = new label."""
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        label = np.ascontiguousarray(label, dtype=np.int32)
        out = np.empty(3, dtype=np.int64)
        if self.lib.oracle_bandwidth(nbr.shape[0], _p(nbr), _p(label), _p(out)) != 0:
            raise RuntimeError("oracle_bandwidth failed")
        return {"B": int(out[0]), "C_BW": int(out[1]), "S_BW": int(out[2])}


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(LIB):
            build_oracle()
        _default = Oracle(LIB)
    return _default


def face_flux(*a, **k):
    return default().face_flux(*a, **k)


def cell_residual(*a, **k):
    return default().cell_residual(*a, **k)


def step(*a, **k):
    return default().step(*a, **k)


def step_threads(*a, **k):
    return default().step_threads(*a, **k)


def cm_order(*a, **k):
    return default().cm_order(*a, **k)


def am1_order(*a, **k):
    return default().am1_order(*a, **k)


def am1_exact_sbw(*a, **k):
    return default().am1_exact_sbw(*a, **k)


def bandwidth(*a, **k):
    return default().bandwidth(*a, **k)


def am1_bounded(*a, **k):
    return default().am1_bounded(*a, **k)
