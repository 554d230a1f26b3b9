"""MI355X (gfx950) Schur-complement solver for the SMPM Poisson/Helmholtz-
Neumann problem with block-Jacobi + deflation preconditioned GMRES.

Thin ctypes binding over include/smpm_schur.h (argument marshalling only;
every step of the solve runs in the HIP library).  Device buffers are torch
CUDA tensors; PyTorch provides memory and streams.

Paper: Joshi, Thomsen & Diamessis, arXiv:1512.01756 (Algorithm 2, Sec. 3;
Fourier modes, Sec. 5).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmpm_schur.so")

OK, EINVAL, ENOMEM, EHIP, ESINGULAR, ENOTCONV, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32_IR, FP16S_IR = 0, 1, 2
METHOD_DBJ, METHOD_BJ, METHOD_SCHUR, METHOD_2LAS = 0, 1, 2, 3
FLAG_HOST_ONLY = 1
FLAG_NO_TUNE = 2
FLAG_ONE_KRYLOV = 4
FLAG_HOST_SETUP = 8
FLAG_DEVICE_SETUP = 16
_SETUP_FLAGS = {"auto": 0, "host": FLAG_HOST_SETUP, "device": FLAG_DEVICE_SETUP}
OP_SCHUR, OP_BJINV, OP_DEFLATE_P, OP_DEFLATE_Q, OP_AINV, OP_B, OP_SCHUR_RHS, OP_SCHUR_BJINV = range(8)
(TABLE_SCHUR_DENSE, TABLE_BJINV_DENSE, TABLE_COARSE_C, TABLE_U_S, TABLE_U_L, TABLE_U_C, TABLE_SZ,
 TABLE_SMINV_DENSE) = range(8)

STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", ESINGULAR: "ESINGULAR",
                ENOTCONV: "ENOTCONV", ENONFINITE: "ENONFINITE", EUNSUPPORTED: "EUNSUPPORTED"}


class SmpmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("mx", ctypes.c_int32), ("mz", ctypes.c_int32), ("order", ctypes.c_int32),
                ("xb", ctypes.POINTER(ctypes.c_double)), ("zb", ctypes.POINTER(ctypes.c_double))]


class Opts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("nrhs", ctypes.c_int32), ("precision", ctypes.c_int32), ("method", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_sweeps", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("zlabel", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("instances", ctypes.c_int32), ("converged", ctypes.c_int32), ("iters_total", ctypes.c_int32),
                ("iters_max", ctypes.c_int32), ("sweeps_max", ctypes.c_int32), ("schur_matvecs", ctypes.c_int32),
                ("rel_residual_max", ctypes.c_double), ("compat_defect_max", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("null_residual_max", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("mx", ctypes.c_int32), ("mz", ctypes.c_int32), ("nrhs", ctypes.c_int32),
                ("r", ctypes.c_int64), ("kS", ctypes.c_int64), ("d", ctypes.c_int32), ("kwave", ctypes.c_double),
                ("tau", ctypes.c_double), ("f_offset", ctypes.c_int64), ("g_offset", ctypes.c_int64),
                ("x_offset", ctypes.c_int64), ("unique_W", ctypes.c_int32), ("unique_M", ctypes.c_int32),
                ("bytes_W64", ctypes.c_int64), ("bytes_M64", ctypes.c_int64),
                ("gemm_sched", ctypes.c_int32 * 4), ("elem_sched", ctypes.c_int32 * 6),
                ("fused_op", ctypes.c_int32 * 3), ("setup_device", ctypes.c_int32),
                ("nnz_W_unique", ctypes.c_int64), ("nnz_W_total", ctypes.c_int64),
                ("nnz_M_unique", ctypes.c_int64), ("nnz_M_total", ctypes.c_int64),
                ("nnz_F_unique", ctypes.c_int64), ("nnz_F_total", ctypes.c_int64),
                ("strip_classes", ctypes.c_int32), ("elem_unique", ctypes.c_int32),
                ("fused_sched", ctypes.c_int32 * 3), ("rhs_gemm", ctypes.c_int32 * 2),
                ("gemm_list", ctypes.c_int32 * 4), ("elem_alt", ctypes.c_int32 * 3)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if isinstance(v, ctypes.Array) else v
        return out


EXPORTED = ["smpm_setup", "smpm_setup_batch", "smpm_setup_fourier", "smpm_save", "smpm_load", "smpm_solve",
            "smpm_solve_fourier", "smpm_transform_y",
            "smpm_apply", "smpm_schur_apply_all", "smpm_apply_all", "smpm_apply_noalloc", "smpm_query",
            "smpm_num_systems", "smpm_export", "smpm_destroy", "smpm_last_error"]

_lib = None


def load():
    """Load the HIP library; raise if it has not been built (there is no
    fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1512_01756_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.smpm_setup.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                               ctypes.POINTER(Opts), P, ctypes.POINTER(P)]
    lib.smpm_setup_batch.argtypes = lib.smpm_setup.argtypes
    lib.smpm_setup_fourier.argtypes = [ctypes.POINTER(Grid), ctypes.c_int32, ctypes.c_double, ctypes.POINTER(Opts),
                                       P, ctypes.POINTER(P)]
    lib.smpm_save.argtypes = [P, ctypes.c_char_p]
    lib.smpm_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(Opts), P, ctypes.POINTER(P)]
    lib.smpm_solve.argtypes = [P, P, P, P, P, ctypes.POINTER(Stats)]
    lib.smpm_solve_fourier.argtypes = lib.smpm_solve.argtypes
    lib.smpm_transform_y.argtypes = [P, ctypes.c_int32, P, P, P]
    lib.smpm_apply.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int32, P]
    lib.smpm_schur_apply_all.argtypes = [P, P, P, ctypes.c_int32, P]
    lib.smpm_apply_all.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int32, P]
    lib.smpm_apply_noalloc.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int32, P]
    lib.smpm_query.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Info)]
    lib.smpm_num_systems.argtypes = [P]
    lib.smpm_num_systems.restype = ctypes.c_int32
    lib.smpm_export.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int64]
    lib.smpm_destroy.argtypes = [P]
    lib.smpm_destroy.restype = None
    lib.smpm_last_error.restype = ctypes.c_char_p
    for name in ("smpm_setup", "smpm_setup_batch", "smpm_setup_fourier", "smpm_save", "smpm_load", "smpm_solve",
                 "smpm_solve_fourier", "smpm_transform_y",
                 "smpm_apply", "smpm_schur_apply_all", "smpm_apply_all", "smpm_apply_noalloc", "smpm_query",
                 "smpm_export"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status):
    if status != OK:
        raise SmpmError(status, load().smpm_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream)


class Solver:
    """One handle: one grid with several wavenumbers (`kwaves`), a batch of
    independent problems (`grids` list with one wavenumber each), or a 3-D
    problem periodic in y (`fourier=(m_y, l_y)`: modes k_m = 2 pi m / l_y,
    m = 0 .. m_y/2, Re and Im as two right-hand sides).  setup: where the
    large dense setup steps run on a GPU handle -- "auto" (the device from a
    few GFLOP of work on), "host" or "device" (always)."""

    def __init__(self, xb=None, zb=None, order=None, kwaves=(0.0,), grids=None, tau=0.0, tol=1e-10,
                 max_iter=300, nrhs=1, precision=FP64, method=METHOD_DBJ, inner_tol=0.0, max_sweeps=0,
                 host_only=False, tune=True, fourier=None, one_krylov=False, zlabel=0, load_path=None,
                 stream=None, setup="auto"):
        if fourier is not None:
            nrhs = 2
        lib = load()
        self._lib = lib
        self.host_only = host_only
        opts = Opts(tau, tol, max_iter, nrhs, precision, method, inner_tol, max_sweeps,
                    (FLAG_HOST_ONLY if host_only else 0) | (0 if tune else FLAG_NO_TUNE)
                    | (FLAG_ONE_KRYLOV if one_krylov else 0) | _SETUP_FLAGS[setup], zlabel)
        self.opts = opts
        self._keep = []
        h = ctypes.c_void_p()
        st = ctypes.c_void_p(0) if host_only else _stream(stream)
        self.fourier = fourier
        if load_path is not None:
            if nrhs == 1:
                opts.nrhs = 0          # the library default (2 for a saved Fourier handle)
            _check(lib.smpm_load(os.fsencode(load_path), ctypes.byref(opts), st, ctypes.byref(h)))
        elif fourier is not None:
            g = self._grid(xb, zb, order)
            _check(lib.smpm_setup_fourier(ctypes.byref(g), int(fourier[0]), float(fourier[1]), ctypes.byref(opts),
                                          st, ctypes.byref(h)))
        elif grids is None:
            g = self._grid(xb, zb, order)
            k = np.ascontiguousarray(np.asarray(kwaves, dtype=np.float64))
            self._keep.append(k)
            _check(lib.smpm_setup(ctypes.byref(g), k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  len(k), ctypes.byref(opts), st, ctypes.byref(h)))
        else:
            arr = (Grid * len(grids))(*[self._grid(*gg[:3]) for gg in grids])
            k = np.ascontiguousarray(np.array([gg[3] for gg in grids], dtype=np.float64))
            self._keep.append(k)
            _check(lib.smpm_setup_batch(arr, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        len(grids), ctypes.byref(opts), st, ctypes.byref(h)))
        self.h = h
        self.nsys = lib.smpm_num_systems(h)
        self.info = [self.query(s) for s in range(self.nsys)]
        self.nrhs = self.info[0]["nrhs"]

    def _grid(self, xb, zb, order):
        xb = np.ascontiguousarray(np.asarray(xb, dtype=np.float64))
        zb = np.ascontiguousarray(np.asarray(zb, dtype=np.float64))
        self._keep += [xb, zb]
        return Grid(len(xb) - 1, len(zb) - 1, int(order),
                    xb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    zb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    def query(self, s):
        info = Info()
        _check(self._lib.smpm_query(self.h, s, ctypes.byref(info)))
        return info.as_dict()

    @property
    def total_r(self):
        return sum(i["r"] for i in self.info) * self.nrhs

    @property
    def total_kS(self):
        return sum(i["kS"] for i in self.info) * self.nrhs

    @property
    def total_g(self):
        return sum(2 * i["n"] * (i["mx"] + i["mz"]) for i in self.info) * self.nrhs

    def solve(self, f, g=None, u=None, stream=None, check=True):
        """f, g, u: torch float64 CUDA tensors in the batched layouts."""
        import torch
        if u is None:
            u = torch.empty_like(f)
        stats = Stats()
        status = self._lib.smpm_solve(self.h, _ptr(f), _ptr(g), _ptr(u), _stream(stream), ctypes.byref(stats))
        if check:
            _check(status)
        return u, stats.as_dict(), status

    def save(self, path):
        """Write the handle's host tables (smpm_save); Solver(load_path=path)
        rebuilds an equal handle without the setup."""
        _check(self._lib.smpm_save(self.h, os.fsencode(path)))

    def solve_fourier(self, f, g=None, u=None, stream=None, check=True):
        """Physical-space 3-D solve: f, u torch float64 CUDA tensors [m_y, r];
        g None or [m_y, 2 n (m_x + m_z)]."""
        import torch
        if u is None:
            u = torch.empty_like(f)
        stats = Stats()
        status = self._lib.smpm_solve_fourier(self.h, _ptr(f), _ptr(g), _ptr(u), _stream(stream), ctypes.byref(stats))
        if check:
            _check(status)
        return u, stats.as_dict(), status

    def transform_y(self, x, y, inverse=False, stream=None):
        """smpm_transform_y: planes [m_y, r] <-> modes [m_y/2 + 1, 2, r]."""
        _check(self._lib.smpm_transform_y(self.h, 1 if inverse else 0, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def apply(self, op, sys, x, y, precision=FP64, stream=None):
        _check(self._lib.smpm_apply(self.h, op, sys, _ptr(x), _ptr(y), precision, _stream(stream)))
        return y

    def schur_apply_all(self, x, y, precision=FP64, stream=None):
        _check(self._lib.smpm_schur_apply_all(self.h, _ptr(x), _ptr(y), precision, _stream(stream)))
        return y

    def apply_noalloc(self, op, sys, x, y, precision=FP64, stream=None):
        """smpm_apply_noalloc: no allocation, no synchronization."""
        _check(self._lib.smpm_apply_noalloc(self.h, op, sys, _ptr(x), _ptr(y), precision, _stream(stream)))
        return y

    def apply_all(self, op, x, y, precision=FP64, stream=None):
        _check(self._lib.smpm_apply_all(self.h, op, _ptr(x), _ptr(y), precision, _stream(stream)))
        return y

    def export(self, table, sys=0):
        i = self.info[sys]
        sizes = {TABLE_SCHUR_DENSE: i["kS"] ** 2, TABLE_BJINV_DENSE: i["kS"] ** 2, TABLE_COARSE_C: i["d"] ** 2,
                 TABLE_U_S: i["kS"], TABLE_U_L: i["r"], TABLE_U_C: i["d"], TABLE_SZ: i["kS"] * i["d"],
                 TABLE_SMINV_DENSE: i["kS"] ** 2}
        n = sizes[table]
        out = np.empty(n, dtype=np.float64)
        _check(self._lib.smpm_export(self.h, table, sys, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n))
        return out

    def close(self):
        if getattr(self, "h", None):
            self._lib.smpm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack_g(problem_g, info_list, nrhs):
    """Flatten per-side Neumann data dicts {side: (nk, nrhs, m, n)} into the
    batched g layout [system][rhs][S | N | W | E]."""
    parts = []
    for s, info in enumerate(info_list):
        for q in range(nrhs):
            for side in ("S", "N", "W", "E"):
                m = info["mx"] if side in ("S", "N") else info["mz"]
                if side in problem_g:
                    parts.append(np.asarray(problem_g[side][s, q], dtype=np.float64).reshape(m * info["n"]))
                else:
                    parts.append(np.zeros(m * info["n"]))
    return np.concatenate(parts)
