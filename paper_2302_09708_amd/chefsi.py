"""ctypes binding of libchefsi.so (include/chefsi.h): argument marshalling only.

Every step of the CheFSI path runs in the library's HIP kernels and rocSOLVER;
this module only converts Python/NumPy/torch arguments to the C-ABI's plain
pointers and sizes and turns non-zero status codes into ``ChefsiError``.
Device blocks are torch tensors on a ROCm device (torch supplies device memory
and streams).  If the library is missing, loading fails loudly: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchefsi.so")

FP64 = 0
MIXED = 1

OK = 0
ERR_INVALID_ARG = 1
ERR_HIP = 2
ERR_WORKSPACE = 3
ERR_NOT_POSDEF = 4
ERR_EIG = 5
ERR_NONFINITE = 6
ERR_SOLVER = 7
ERR_OOM = 8

STATIC_SCRATCH_BYTES = 64 << 20  # CHEFSI_STATIC_SCRATCH_BYTES

PROF_HX, PROF_NL, PROF_GRAM, PROF_REDUCE, PROF_ROT, PROF_EIG, PROF_COPY, PROF_FALLBACK = range(8)

# every symbol include/chefsi.h declares
EXPORTS = (
    "chefsi_create", "chefsi_destroy", "chefsi_workspace_bytes", "chefsi_handle_bytes", "chefsi_spectral_bounds",
    "chefsi_apply_h", "chefsi_filter", "chefsi_project", "chefsi_eigh", "chefsi_rotate",
    "chefsi_step", "chefsi_solve", "chefsi_refine_fp64", "chefsi_profile_enable",
    "chefsi_profile_reset", "chefsi_profile_read", "chefsi_last_info", "chefsi_strerror",
    "chefsi_last_error", "chefsi_version", "chefsi_lanczos_workspace_bytes", "chefsi_lanczos_bound",
    "chefsi_update_veff", "chefsi_forces_workspace_bytes", "chefsi_nonlocal_forces",
    "chefsi_kinetic_stress", "chefsi_kpoint_create", "chefsi_kpoint_destroy", "chefsi_kpoint_last_error",
    "chefsi_kpoint_workspace_bytes", "chefsi_kpoint_apply_h", "chefsi_kpoint_step",
    "chefsi_kpoint_profile_enable", "chefsi_kpoint_profile_reset", "chefsi_kpoint_profile_read",
    "chefsi_set_stencil_tiling", "chefsi_get_stencil_tiling", "chefsi_nonlocal_stress",
    "chefsi_static_scratch_bytes", "chefsi_apply_h_static", "chefsi_set_projector_pass",
    "chefsi_autotune",
)


class ChefsiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"chefsi status {status}: {message}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("h", C.c_double * 3), ("bc", C.c_int32 * 3), ("fd_order", C.c_int32)]


class Nonlocal(C.Structure):
    _fields_ = [("n_atoms", C.c_int32),
                ("supp_ptr", C.POINTER(C.c_int64)),
                ("supp_idx", C.POINTER(C.c_int32)),
                ("nproj", C.POINTER(C.c_int32)),
                ("chi", C.POINTER(C.c_double)),
                ("gamma", C.POINTER(C.c_double))]


_lib = None


def load(path: str = LIB_PATH):
    """Load libchefsi.so and declare its signatures.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2302_09708_amd.build`")
    # PyTorch supplies device memory and streams; its HIP runtime must be the one in the
    # process before the library's own dependency on libamdhip64 is resolved
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, sz, i32, dbl = C.c_void_p, C.c_size_t, C.c_int32, C.c_double
    pd = C.POINTER(C.c_double)
    lib.chefsi_create.argtypes = [C.POINTER(Grid), pd, C.POINTER(Nonlocal), i32, i32, C.POINTER(vp)]
    lib.chefsi_destroy.argtypes = [vp]
    lib.chefsi_destroy.restype = None
    lib.chefsi_workspace_bytes.argtypes = [vp, i32, C.POINTER(sz)]
    lib.chefsi_handle_bytes.argtypes = [vp, C.POINTER(sz)]
    lib.chefsi_set_stencil_tiling.argtypes = [vp, i32, i32]
    lib.chefsi_set_projector_pass.argtypes = [vp, i32]
    lib.chefsi_autotune.argtypes = [vp, vp, i32, vp, sz, vp, C.POINTER(C.c_int32)]
    lib.chefsi_get_stencil_tiling.argtypes = [vp, C.POINTER(C.c_int32)]
    lib.chefsi_spectral_bounds.argtypes = [vp, pd, pd, pd]
    lib.chefsi_apply_h.argtypes = [vp, vp, vp, i32, vp, sz, vp]
    lib.chefsi_static_scratch_bytes.argtypes = [vp, i32, C.POINTER(sz)]
    lib.chefsi_apply_h_static.argtypes = [vp, vp, vp, i32, vp]
    lib.chefsi_update_veff.argtypes = [vp, pd, vp]
    lib.chefsi_forces_workspace_bytes.argtypes = [vp, i32, C.POINTER(sz)]
    lib.chefsi_nonlocal_forces.argtypes = [vp, vp, i32, pd, vp, sz, vp, pd]
    lib.chefsi_kinetic_stress.argtypes = [vp, vp, i32, pd, vp, sz, vp, pd]
    lib.chefsi_nonlocal_stress.argtypes = [vp, vp, i32, pd, pd, vp, sz, vp, pd]
    lib.chefsi_lanczos_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
    lib.chefsi_lanczos_bound.argtypes = [vp, vp, i32, vp, sz, vp, pd, pd, pd, pd]
    lib.chefsi_filter.argtypes = [vp, vp, i32, i32, dbl, dbl, dbl, vp, sz, vp]
    lib.chefsi_project.argtypes = [vp, vp, i32, vp, vp, vp, sz, vp]
    lib.chefsi_eigh.argtypes = [vp, vp, vp, vp, i32, vp, sz, vp]
    lib.chefsi_rotate.argtypes = [vp, vp, vp, i32, vp, sz, vp]
    lib.chefsi_step.argtypes = [vp, vp, i32, i32, dbl, dbl, dbl, vp, sz, vp, pd]
    lib.chefsi_solve.argtypes = [vp, vp, i32, i32, i32, dbl, dbl, dbl, vp, sz, vp, pd, pd, pd]
    lib.chefsi_refine_fp64.argtypes = [vp, vp, i32, i32, dbl, dbl, dbl, vp, sz, vp, pd]
    lib.chefsi_profile_enable.argtypes = [vp, i32]
    lib.chefsi_profile_reset.argtypes = [vp]
    lib.chefsi_profile_read.argtypes = [vp, i32, pd, C.POINTER(C.c_int64)]
    lib.chefsi_last_info.argtypes = [vp]
    lib.chefsi_strerror.argtypes = [C.c_int]
    lib.chefsi_strerror.restype = C.c_char_p
    lib.chefsi_last_error.argtypes = [vp]
    lib.chefsi_last_error.restype = C.c_char_p
    lib.chefsi_version.argtypes = []
    lib.chefsi_kpoint_create.argtypes = [C.POINTER(Grid), pd, C.POINTER(Nonlocal), C.POINTER(C.c_int32), pd, i32,
                                         C.POINTER(vp)]
    lib.chefsi_kpoint_destroy.argtypes = [vp]
    lib.chefsi_kpoint_destroy.restype = None
    lib.chefsi_kpoint_last_error.argtypes = [vp]
    lib.chefsi_kpoint_last_error.restype = C.c_char_p
    lib.chefsi_kpoint_workspace_bytes.argtypes = [vp, i32, C.POINTER(sz)]
    lib.chefsi_kpoint_apply_h.argtypes = [vp, vp, vp, i32, vp, sz, vp]
    lib.chefsi_kpoint_step.argtypes = [vp, vp, i32, i32, dbl, dbl, dbl, vp, sz, vp, pd]
    lib.chefsi_kpoint_profile_enable.argtypes = [vp, i32]
    lib.chefsi_kpoint_profile_reset.argtypes = [vp]
    lib.chefsi_kpoint_profile_read.argtypes = [vp, i32, pd, C.POINTER(C.c_int64)]
    _lib = lib
    return lib


def _ptr(t) -> int:
    """Device pointer of a torch tensor (or an int address)."""
    if t is None:
        return 0
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _marshal(problem):
    """(Grid, Nonlocal, veff array, arrays to keep alive) for a problem."""
    g = Grid()
    for d in range(3):
        g.n[d] = int(problem.n[d])
        g.h[d] = float(problem.h[d])
        g.bc[d] = int(problem.bc[d])
    g.fd_order = int(problem.fd_order)
    veff = np.ascontiguousarray(problem.veff, dtype=np.float64)
    keep = [veff]
    nl = Nonlocal()
    nl.n_atoms = int(len(problem.nproj))
    if nl.n_atoms > 0:
        arrs = [np.ascontiguousarray(problem.supp_ptr, dtype=np.int64),
                np.ascontiguousarray(problem.supp_idx, dtype=np.int32),
                np.ascontiguousarray(problem.nproj, dtype=np.int32),
                np.ascontiguousarray(problem.chi, dtype=np.float64),
                np.ascontiguousarray(problem.gamma, dtype=np.float64)]
        keep += arrs
        nl.supp_ptr = arrs[0].ctypes.data_as(C.POINTER(C.c_int64))
        nl.supp_idx = arrs[1].ctypes.data_as(C.POINTER(C.c_int32))
        nl.nproj = arrs[2].ctypes.data_as(C.POINTER(C.c_int32))
        nl.chi = arrs[3].ctypes.data_as(C.POINTER(C.c_double))
        nl.gamma = arrs[4].ctypes.data_as(C.POINTER(C.c_double))
    return g, nl, veff, keep


class KPoint:
    """One Hamiltonian at a Bloch wavevector k (chefsi_kpoint_create / _destroy); blocks
    are torch.complex128 tensors of shape (ns, Nd).  supp_img: (sum n_J, 3) int32 image
    of every support point."""

    def __init__(self, problem, k, supp_img, max_ns: int = 1):
        lib = load()
        self._lib = lib
        g, nl, veff, keep = _marshal(problem)
        img = np.ascontiguousarray(supp_img, dtype=np.int32).reshape(-1)
        kv = np.ascontiguousarray(k, dtype=np.float64).reshape(3)
        h = C.c_void_p()
        st = lib.chefsi_kpoint_create(C.byref(g), veff.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nl),
                                      img.ctypes.data_as(C.POINTER(C.c_int32)),
                                      kv.ctypes.data_as(C.POINTER(C.c_double)), int(max_ns), C.byref(h))
        del keep
        if st != OK:
            raise ChefsiError(st, lib.chefsi_strerror(st).decode())
        self.h = h
        self.nd = int(np.prod(problem.n))
        self.max_ns = int(max_ns)

    def _check(self, st: int):
        if st != OK:
            msg = self._lib.chefsi_kpoint_last_error(self.h).decode() or self._lib.chefsi_strerror(st).decode()
            raise ChefsiError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self._lib.chefsi_kpoint_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, ns: int) -> int:
        b = C.c_size_t()
        self._check(self._lib.chefsi_kpoint_workspace_bytes(self.h, int(ns), C.byref(b)))
        return int(b.value)

    def workspace(self, ns: int):
        import torch
        return torch.empty(self.workspace_bytes(ns), dtype=torch.uint8, device="cuda")

    def apply_h(self, X, Y, ns, ws, stream=None):
        self._check(self._lib.chefsi_kpoint_apply_h(self.h, _ptr(X), _ptr(Y), int(ns), _ptr(ws),
                                                     ws.numel() * ws.element_size(), _stream(stream)))

    def step(self, X, ns, degree, lam_lo, lam_cut, lam_hi, ws, stream=None) -> np.ndarray:
        d = np.zeros(int(ns), dtype=np.float64)
        self._check(self._lib.chefsi_kpoint_step(self.h, _ptr(X), int(ns), int(degree), float(lam_lo),
                                                  float(lam_cut), float(lam_hi), _ptr(ws),
                                                  ws.numel() * ws.element_size(), _stream(stream),
                                                  d.ctypes.data_as(C.POINTER(C.c_double))))
        return d

    def profile_enable(self, on: bool = True):
        self._check(self._lib.chefsi_kpoint_profile_enable(self.h, 1 if on else 0))

    def profile_reset(self):
        self._check(self._lib.chefsi_kpoint_profile_reset(self.h))

    def profile_read(self, kernel_id: int) -> Tuple[float, int]:
        ms, n = C.c_double(0.0), C.c_int64(0)
        self._check(self._lib.chefsi_kpoint_profile_read(self.h, int(kernel_id), C.byref(ms), C.byref(n)))
        return ms.value, n.value


class Handle:
    """One Hamiltonian on the current device (chefsi_create / chefsi_destroy)."""

    def __init__(self, problem, precision: int = FP64, max_ns: int = 1):
        lib = load()
        self._lib = lib
        g = Grid()
        for d in range(3):
            g.n[d] = int(problem.n[d])
            g.h[d] = float(problem.h[d])
            g.bc[d] = int(problem.bc[d])
        g.fd_order = int(problem.fd_order)
        self._keep = []
        veff = np.ascontiguousarray(problem.veff, dtype=np.float64)
        self._keep.append(veff)
        nl = Nonlocal()
        nl.n_atoms = int(len(problem.nproj))
        if nl.n_atoms > 0:
            arrs = [np.ascontiguousarray(problem.supp_ptr, dtype=np.int64),
                    np.ascontiguousarray(problem.supp_idx, dtype=np.int32),
                    np.ascontiguousarray(problem.nproj, dtype=np.int32),
                    np.ascontiguousarray(problem.chi, dtype=np.float64),
                    np.ascontiguousarray(problem.gamma, dtype=np.float64)]
            self._keep += arrs
            nl.supp_ptr = arrs[0].ctypes.data_as(C.POINTER(C.c_int64))
            nl.supp_idx = arrs[1].ctypes.data_as(C.POINTER(C.c_int32))
            nl.nproj = arrs[2].ctypes.data_as(C.POINTER(C.c_int32))
            nl.chi = arrs[3].ctypes.data_as(C.POINTER(C.c_double))
            nl.gamma = arrs[4].ctypes.data_as(C.POINTER(C.c_double))
        h = C.c_void_p()
        st = lib.chefsi_create(C.byref(g), veff.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nl),
                               int(precision), int(max_ns), C.byref(h))
        self._keep = []
        if st != OK:
            raise ChefsiError(st, lib.chefsi_strerror(st).decode())
        self.h = h
        self.precision = precision
        self.nd = int(np.prod(problem.n))
        self.n_atoms = int(len(problem.nproj))
        self.max_ns = int(max_ns)

    # -- helpers ---------------------------------------------------------------
    def _check(self, st: int):
        if st != OK:
            msg = self._lib.chefsi_last_error(self.h).decode() or self._lib.chefsi_strerror(st).decode()
            raise ChefsiError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self._lib.chefsi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C-ABI calls -------------------------------------------------------------
    def chefsi_workspace_bytes(self, ns: int) -> int:
        b = C.c_size_t()
        self._check(self._lib.chefsi_workspace_bytes(self.h, int(ns), C.byref(b)))
        return int(b.value)

    def chefsi_handle_bytes(self) -> int:
        b = C.c_size_t()
        self._check(self._lib.chefsi_handle_bytes(self.h, C.byref(b)))
        return int(b.value)

    def device_bytes(self) -> int:
        return self.chefsi_handle_bytes()

    def chefsi_set_stencil_tiling(self, rows_per_thread: int, row_groups: int) -> None:
        self._check(self._lib.chefsi_set_stencil_tiling(self.h, rows_per_thread, row_groups))

    def chefsi_set_projector_pass(self, in_stencil: bool) -> None:
        self._check(self._lib.chefsi_set_projector_pass(self.h, 1 if in_stencil else 0))

    def chefsi_autotune(self, X, ns, ws, ws_bytes=None, stream=None) -> Tuple[int, int, bool]:
        c = (C.c_int32 * 3)()
        self._check(self._lib.chefsi_autotune(self.h, _ptr(X), int(ns), _ptr(ws), self._wsb(ws, ws_bytes),
                                              _stream(stream), c))
        return int(c[0]), int(c[1]), bool(c[2])

    def chefsi_get_stencil_tiling(self) -> Tuple[int, int, int, int]:
        t = (C.c_int32 * 4)()
        self._check(self._lib.chefsi_get_stencil_tiling(self.h, t))
        return tuple(int(v) for v in t)

    def chefsi_spectral_bounds(self) -> Tuple[float, float, float]:
        lo, cut, hi = C.c_double(), C.c_double(), C.c_double()
        self._check(self._lib.chefsi_spectral_bounds(self.h, C.byref(lo), C.byref(cut), C.byref(hi)))
        return lo.value, cut.value, hi.value

    def chefsi_update_veff(self, veff, stream=None):
        v = np.ascontiguousarray(veff, dtype=np.float64).reshape(-1)
        if v.size != self.nd:
            raise ValueError(f"Veff has {v.size} values, the grid {self.nd}")
        self._check(self._lib.chefsi_update_veff(self.h, v.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))

    def chefsi_forces_workspace_bytes(self, ns: int) -> int:
        b = C.c_size_t()
        self._check(self._lib.chefsi_forces_workspace_bytes(self.h, int(ns), C.byref(b)))
        return int(b.value)

    def chefsi_nonlocal_forces(self, X, ns, occ, ws, ws_bytes=None, stream=None) -> np.ndarray:
        """(n_atoms, 3) nonlocal forces of the ns orbitals X with occupations occ."""
        g = np.ascontiguousarray(occ, dtype=np.float64).reshape(-1)
        if g.size != int(ns):
            raise ValueError("need one occupation per orbital")
        f = np.zeros((self.n_atoms, 3))
        self._check(self._lib.chefsi_nonlocal_forces(self.h, _ptr(X), int(ns), g.ctypes.data_as(C.POINTER(C.c_double)),
                                                     _ptr(ws), self._wsb(ws, ws_bytes), _stream(stream),
                                                     f.ctypes.data_as(C.POINTER(C.c_double))))
        return f

    def chefsi_kinetic_stress(self, X, ns, occ, ws, ws_bytes=None, stream=None) -> np.ndarray:
        """3 x 3 kinetic stress of the ns orbitals X with occupations occ."""
        g = np.ascontiguousarray(occ, dtype=np.float64).reshape(-1)
        if g.size != int(ns):
            raise ValueError("need one occupation per orbital")
        out = np.zeros(9)
        self._check(self._lib.chefsi_kinetic_stress(self.h, _ptr(X), int(ns), g.ctypes.data_as(C.POINTER(C.c_double)),
                                                    _ptr(ws), self._wsb(ws, ws_bytes), _stream(stream),
                                                    out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(3, 3)

    def chefsi_nonlocal_stress(self, X, ns, occ, disp, ws, ws_bytes=None, stream=None) -> np.ndarray:
        """3 x 3 nonlocal stress of the ns orbitals X with occupations occ; disp holds the
        (n_support, 3) displacements of the support points from their atoms."""
        g = np.ascontiguousarray(occ, dtype=np.float64).reshape(-1)
        if g.size != int(ns):
            raise ValueError("need one occupation per orbital")
        d = np.ascontiguousarray(disp, dtype=np.float64).reshape(-1)
        out = np.zeros(9)
        self._check(self._lib.chefsi_nonlocal_stress(self.h, _ptr(X), int(ns), g.ctypes.data_as(C.POINTER(C.c_double)),
                                                     d.ctypes.data_as(C.POINTER(C.c_double)), _ptr(ws),
                                                     self._wsb(ws, ws_bytes), _stream(stream),
                                                     out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(3, 3)

    def chefsi_lanczos_workspace_bytes(self) -> int:
        b = C.c_size_t()
        self._check(self._lib.chefsi_lanczos_workspace_bytes(self.h, C.byref(b)))
        return int(b.value)

    def chefsi_lanczos_bound(self, v0, steps, ws, ws_bytes=None, stream=None):
        """(lam_nd, theta, alphas, betas) of `steps` Lanczos steps from the device vector v0."""
        lam, th = C.c_double(), C.c_double()
        a = np.zeros(int(steps))
        b = np.zeros(int(steps))
        self._check(self._lib.chefsi_lanczos_bound(
            self.h, _ptr(v0), int(steps), _ptr(ws), self._wsb(ws, ws_bytes), _stream(stream), C.byref(lam),
            C.byref(th), a.ctypes.data_as(C.POINTER(C.c_double)), b.ctypes.data_as(C.POINTER(C.c_double))))
        return lam.value, th.value, a, b

    def chefsi_apply_h(self, X, Y, ns, ws, ws_bytes=None, stream=None):
        self._check(self._lib.chefsi_apply_h(self.h, _ptr(X), _ptr(Y), int(ns), _ptr(ws),
                                             self._wsb(ws, ws_bytes), _stream(stream)))

    def chefsi_static_scratch_bytes(self, ns):
        b = C.c_size_t()
        self._check(self._lib.chefsi_static_scratch_bytes(self.h, int(ns), C.byref(b)))
        return b.value

    def chefsi_apply_h_static(self, X, Y, ns, stream=None):
        self._check(self._lib.chefsi_apply_h_static(self.h, _ptr(X), _ptr(Y), int(ns), _stream(stream)))

    def chefsi_filter(self, X, ns, degree, lam_lo, lam_cut, lam_hi, ws, ws_bytes=None, stream=None):
        self._check(self._lib.chefsi_filter(self.h, _ptr(X), int(ns), int(degree), float(lam_lo), float(lam_cut),
                                            float(lam_hi), _ptr(ws), self._wsb(ws, ws_bytes), _stream(stream)))

    def chefsi_project(self, X, ns, Hs, Ms, ws, ws_bytes=None, stream=None):
        self._check(self._lib.chefsi_project(self.h, _ptr(X), int(ns), _ptr(Hs), _ptr(Ms), _ptr(ws),
                                             self._wsb(ws, ws_bytes), _stream(stream)))

    def chefsi_eigh(self, Hs, Ms, D, ns, ws, ws_bytes=None, stream=None):
        self._check(self._lib.chefsi_eigh(self.h, _ptr(Hs), _ptr(Ms), _ptr(D), int(ns), _ptr(ws),
                                          self._wsb(ws, ws_bytes), _stream(stream)))

    def chefsi_rotate(self, X, Z, ns, ws, ws_bytes=None, stream=None):
        self._check(self._lib.chefsi_rotate(self.h, _ptr(X), _ptr(Z), int(ns), _ptr(ws),
                                            self._wsb(ws, ws_bytes), _stream(stream)))

    def chefsi_step(self, X, ns, degree, lam_lo, lam_cut, lam_hi, ws, ws_bytes=None, stream=None) -> np.ndarray:
        ritz = np.zeros(int(ns))
        self._check(self._lib.chefsi_step(self.h, _ptr(X), int(ns), int(degree), float(lam_lo), float(lam_cut),
                                          float(lam_hi), _ptr(ws), self._wsb(ws, ws_bytes), _stream(stream),
                                          ritz.ctypes.data_as(C.POINTER(C.c_double))))
        return ritz

    def chefsi_solve(self, X, ns, degree, n_iter, lam_lo, lam_cut, lam_hi, ws, ws_bytes=None, stream=None):
        ritz = np.zeros(int(ns))
        lo, cut = C.c_double(), C.c_double()
        self._check(self._lib.chefsi_solve(self.h, _ptr(X), int(ns), int(degree), int(n_iter), float(lam_lo),
                                           float(lam_cut), float(lam_hi), _ptr(ws), self._wsb(ws, ws_bytes),
                                           _stream(stream), ritz.ctypes.data_as(C.POINTER(C.c_double)),
                                           C.byref(lo), C.byref(cut)))
        return ritz, lo.value, cut.value

    def chefsi_refine_fp64(self, X, ns, ws, degree=0, lam_lo=0.0, lam_cut=0.0, lam_hi=0.0, ws_bytes=None,
                           stream=None) -> np.ndarray:
        ritz = np.zeros(int(ns))
        self._check(self._lib.chefsi_refine_fp64(self.h, _ptr(X), int(ns), int(degree), float(lam_lo),
                                                 float(lam_cut), float(lam_hi), _ptr(ws), self._wsb(ws, ws_bytes),
                                                 _stream(stream), ritz.ctypes.data_as(C.POINTER(C.c_double))))
        return ritz

    def solve(self, X, ns, degree, n_iter, ws, bounds=None, stream=None):
        """n_iter CheFSI iterations with the bounds update lam_lo <- D_1, lam_cut <- D_ns.

        FP64 handle: n_iter chefsi_step calls.  Mixed handle: n_iter - 1 mixed steps,
        then chefsi_refine_fp64 with the same degree (filter + FP64 Rayleigh-Ritz), so
        both precisions apply the filter n_iter times.  Returns (ritz, lam_lo, lam_cut)."""
        lo, cut, hi = bounds if bounds is not None else self.chefsi_spectral_bounds()
        if self.precision == FP64:
            return self.chefsi_solve(X, ns, degree, n_iter, lo, cut, hi, ws, stream=stream)
        if n_iter > 1:
            _, lo, cut = self.chefsi_solve(X, ns, degree, n_iter - 1, lo, cut, hi, ws, stream=stream)
        ritz = self.chefsi_refine_fp64(X, ns, ws, degree, lo, cut, hi, stream=stream)
        return ritz, float(ritz[0]), float(ritz[-1])

    def chefsi_profile_enable(self, on: bool = True):
        self._check(self._lib.chefsi_profile_enable(self.h, 1 if on else 0))

    def chefsi_profile_reset(self):
        self._check(self._lib.chefsi_profile_reset(self.h))

    def chefsi_profile_read(self, kernel_id: int) -> Tuple[float, int]:
        ms, n = C.c_double(), C.c_int64()
        self._check(self._lib.chefsi_profile_read(self.h, int(kernel_id), C.byref(ms), C.byref(n)))
        return ms.value, int(n.value)

    def chefsi_last_info(self) -> int:
        return int(self._lib.chefsi_last_info(self.h))

    @staticmethod
    def _wsb(ws, ws_bytes: Optional[int]) -> int:
        if ws_bytes is not None:
            return int(ws_bytes)
        return int(ws.numel() * ws.element_size())


def workspace(handle: Handle, ns: int, device=None):
    """A torch uint8 device buffer of exactly chefsi_workspace_bytes(ns) bytes (caching allocator: 512-B aligned)."""
    import torch
    nbytes = handle.chefsi_workspace_bytes(ns)
    return torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")


def strerror(status: int) -> str:
    return load().chefsi_strerror(int(status)).decode()
