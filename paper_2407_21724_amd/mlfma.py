"""Python binding of libmlfma.so (argument marshalling only).

Every entry point has the name of the C function it calls (without the
``mlfma_`` prefix).  Device buffers are torch tensors (complex64 for the
MLFMA_C64 context precision, complex128 for MLFMA_C128) of shape
[R, P, 2N], contiguous, on the current HIP device; streams are torch
streams.  Nothing here computes any part of the method: if the library is
missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libmlfma.so")

OK, EINVAL, ENOMEM, EHIP, ENOTREADY, ENONFINITE, NOT_CONVERGED = 0, -1, -2, -3, -4, -5, 1
C64, C128, C64_BF16 = 0, 1, 2
PART_NEAR, PART_FAR, PART_ALL = 1, 2, 3
SOLVE_USE_X0 = 1
SOLVE_ALWAYS_REORTH = 2
SOLVE_FP32_BASIS = 4


class MlfmaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mlfma error {code}: {msg}")
        self.code = code


class Problem(C.Structure):
    _fields_ = [("n_particles", C.c_int32), ("centers", C.POINTER(C.c_double)),
                ("class_id", C.POINTER(C.c_int32)), ("n_classes", C.c_int32),
                ("eps_bg_re", C.c_double), ("eps_bg_im", C.c_double)]


class TreeParams(C.Structure):
    _fields_ = [("leaf_size", C.c_double), ("L_leaf", C.c_int32), ("L_rule", C.c_int32),
                ("digits", C.c_double), ("interp_order", C.c_int32), ("precision", C.c_int32),
                ("outer_levels", C.c_int32), ("near_rule", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("L", C.c_int32 * 16), ("K", C.c_int32 * 16),
                ("nx", C.c_int32 * 16), ("ny", C.c_int32 * 16), ("n_unknowns", C.c_int64),
                ("n_modes", C.c_int32), ("device_bytes", C.c_int64)]


class StageTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("total_ms", C.c_double), ("launches", C.c_int64),
                ("bytes_per_launch", C.c_double), ("flops_per_launch", C.c_double),
                ("kernel", C.c_char * 96)]


class Tuning(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("agg_rows", C.c_int32 * 16), ("dis_rows", C.c_int32 * 16),
                ("gemm_rows_near", C.c_int32), ("gemm_rows_receive", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("true_rel_res", C.c_double), ("time_s", C.c_double),
                ("converged", C.c_int32), ("reorth", C.c_int32), ("cycles", C.c_int32)]


EXPORTS = [
    "mlfma_default_params", "mlfma_build_tree", "mlfma_static_modes", "mlfma_set_static_modes",
    "mlfma_prepare", "mlfma_plane_wave_rhs", "mlfma_matvec", "mlfma_matvec_parts", "mlfma_matvec_noalloc",
    "mlfma_precondition", "mlfma_gmres_solve", "mlfma_fields", "mlfma_info", "mlfma_destroy", "mlfma_last_error",
    "mlfma_debug_near_block", "mlfma_debug_pair_block_device", "mlfma_debug_leaf_pattern", "mlfma_debug_level_grid",
    "mlfma_debug_translation", "mlfma_debug_interpolate", "mlfma_profile", "mlfma_profile_read", "mlfma_share_setup",
    "mlfma_mlp_create", "mlfma_mlp_destroy", "mlfma_mlp_last_error", "mlfma_mlp_num_params",
    "mlfma_mlp_get_params", "mlfma_mlp_set_params", "mlfma_mlp_forward", "mlfma_mlp_loss_grad",
    "mlfma_mlp_train_step", "mlfma_learned_guess", "mlfma_guess_features", "mlfma_set_tuning",
    "mlfma_get_tuning",
]


def load_library(path: str = _LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2407_21724_amd.build`")
    lib = C.CDLL(path)
    dp, ip, vp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_void_p
    ctxp = C.c_void_p
    sig = {
        "mlfma_default_params": (None, [C.POINTER(TreeParams)]),
        "mlfma_build_tree": (C.c_int, [C.POINTER(Problem), C.POINTER(TreeParams), C.POINTER(C.c_void_p)]),
        "mlfma_static_modes": (C.c_int, [C.c_int32, dp, C.c_int32, ip, C.c_int32, ip, C.c_int32, C.c_int32, dp, dp]),
        "mlfma_set_static_modes": (C.c_int, [ctxp, C.c_int32, C.c_int32, dp, C.c_int32, ip, C.c_int32, ip,
                                             C.c_int32, C.c_int32, dp, C.c_double, C.c_double]),
        "mlfma_prepare": (C.c_int, [ctxp]),
        "mlfma_plane_wave_rhs": (C.c_int, [ctxp, C.c_int32, dp, dp, vp, vp]),
        "mlfma_matvec": (C.c_int, [ctxp, vp, vp, C.c_int32, vp]),
        "mlfma_matvec_noalloc": (C.c_int, [ctxp, vp, vp, C.c_int32, vp]),
        "mlfma_matvec_parts": (C.c_int, [ctxp, vp, vp, C.c_int32, C.c_int32, vp]),
        "mlfma_precondition": (C.c_int, [ctxp, vp, vp, C.c_int32, vp]),
        "mlfma_fields": (C.c_int, [ctxp, vp, C.c_int32, C.c_int32, dp, vp, vp]),
        "mlfma_gmres_solve": (C.c_int, [ctxp, vp, vp, C.c_int32, C.c_double, C.c_int32, C.c_int32, C.c_int32,
                                        C.POINTER(SolveStats), vp]),
        "mlfma_info": (C.c_int, [ctxp, C.POINTER(Info)]),
        "mlfma_profile": (C.c_int, [ctxp, C.c_int32]),
        "mlfma_profile_read": (C.c_int, [ctxp, C.c_int32, C.POINTER(StageTime), C.POINTER(C.c_int32)]),
        "mlfma_destroy": (None, [ctxp]),
        "mlfma_last_error": (C.c_char_p, [ctxp]),
        "mlfma_debug_near_block": (C.c_int, [ctxp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, dp]),
        "mlfma_debug_pair_block_device": (C.c_int, [ctxp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, dp]),
        "mlfma_debug_leaf_pattern": (C.c_int, [ctxp, C.c_int32, dp]),
        "mlfma_debug_level_grid": (C.c_int, [ctxp, C.c_int32, dp, dp]),
        "mlfma_debug_translation": (C.c_int, [ctxp, C.c_int32, C.c_int32, C.c_int32, dp]),
        "mlfma_debug_interpolate": (C.c_int, [ctxp, C.c_int32, dp, dp]),
        "mlfma_share_setup": (C.c_int, [ctxp, ctxp]),
        "mlfma_set_tuning": (C.c_int, [ctxp, C.POINTER(Tuning)]),
        "mlfma_get_tuning": (C.c_int, [ctxp, C.POINTER(Tuning)]),
        "mlfma_mlp_create": (C.c_int, [C.c_int32, ip, C.c_uint64, C.POINTER(C.c_void_p)]),
        "mlfma_mlp_destroy": (None, [vp]),
        "mlfma_mlp_last_error": (C.c_char_p, [vp]),
        "mlfma_mlp_num_params": (C.c_int64, [vp]),
        "mlfma_mlp_get_params": (C.c_int, [vp, C.POINTER(C.c_float)]),
        "mlfma_mlp_set_params": (C.c_int, [vp, C.POINTER(C.c_float)]),
        "mlfma_mlp_forward": (C.c_int, [vp, vp, C.c_int32, vp, vp]),
        "mlfma_mlp_loss_grad": (C.c_int, [vp, vp, vp, C.c_int32, dp, C.POINTER(C.c_float), vp]),
        "mlfma_mlp_train_step": (C.c_int, [vp, vp, vp, C.c_int32, C.c_float, dp, vp]),
        "mlfma_learned_guess": (C.c_int, [ctxp, vp, dp, C.c_double, C.c_int32, dp, vp, vp]),
        "mlfma_guess_features": (C.c_int, [ctxp, dp, C.c_double, C.c_int32, dp, C.POINTER(C.c_float)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def default_params(**kw) -> TreeParams:
    tp = TreeParams()
    lib().mlfma_default_params(C.byref(tp))
    for k, v in kw.items():
        setattr(tp, k, v)
    return tp


def static_modes(verts, tris, edges, n_perp: int, n_par: int):
    """mlfma_static_modes: returns (M [(n_perp+n_par)][ne], gamma)."""
    v = np.ascontiguousarray(verts, np.float64)
    t = np.ascontiguousarray(tris, np.int32)
    e = np.ascontiguousarray(edges, np.int32)
    N = n_perp + n_par
    M = np.zeros((N, len(e)))
    g = np.zeros(N)
    rc = lib().mlfma_static_modes(len(v), _dptr(v), len(t), _iptr(t), len(e), _iptr(e), n_perp, n_par,
                                  _dptr(M), _dptr(g))
    if rc != OK:
        raise MlfmaError(rc, "static_modes failed")
    return M, g


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Context:
    """An mlfma_ctx: tree, classes and device tables of one particle array."""

    def __init__(self, centers, class_id, n_classes: int, params: TreeParams | None = None, eps_bg=1.0):
        self._centers = np.ascontiguousarray(centers, np.float64)
        self._cls = np.ascontiguousarray(class_id, np.int32)
        eb = complex(eps_bg)
        pb = Problem(len(self._centers), _dptr(self._centers), _iptr(self._cls), n_classes, eb.real, eb.imag)
        self.params = params or default_params()
        h = C.c_void_p()
        rc = lib().mlfma_build_tree(C.byref(pb), C.byref(self.params), C.byref(h))
        if rc != OK:
            raise MlfmaError(rc, "build_tree rejected the problem")
        self._h = h
        self.n_particles = len(self._centers)
        self.n_classes = int(n_classes)
        self.n_modes = None

    @property
    def dtype(self):
        import torch
        return torch.complex128 if self.params.precision == C128 else torch.complex64

    def _check(self, rc, what):
        if rc < 0:
            raise MlfmaError(rc, f"{what}: {lib().mlfma_last_error(self._h).decode()}")
        return rc

    def close(self):
        if getattr(self, "_h", None):
            lib().mlfma_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_tuning(self):
        """(agg_rows, dis_rows): interpolation strip heights per level."""
        t = Tuning()
        self._check(lib().mlfma_get_tuning(self._h, C.byref(t)), "get_tuning")
        return list(t.agg_rows[:t.n_levels]), list(t.dis_rows[:t.n_levels])

    def get_gemm_tiles(self):
        """(near+projection, receive) 16-row MFMA tiles per block."""
        t = Tuning()
        self._check(lib().mlfma_get_tuning(self._h, C.byref(t)), "get_tuning")
        return int(t.gemm_rows_near), int(t.gemm_rows_receive)

    def set_tuning(self, agg_rows, dis_rows, gemm_rows=None):
        t = Tuning()
        t.n_levels = len(agg_rows)
        for i, (a, d) in enumerate(zip(agg_rows, dis_rows)):
            t.agg_rows[i] = int(a)
            t.dis_rows[i] = int(d)
        t.gemm_rows_near, t.gemm_rows_receive = gemm_rows if gemm_rows is not None else self.get_gemm_tiles()
        self._check(lib().mlfma_set_tuning(self._h, C.byref(t)), "set_tuning")

    def share_setup(self, src: "Context"):
        """Use src's per-class setup and neighbour-block cache (mlfma_share_setup)."""
        self._check(lib().mlfma_share_setup(self._h, src._h), "share_setup")
        self.n_modes = src.n_modes
        self._shared_from = src          # keeps the source alive for readability; the data is refcounted

    def guess_features(self, class_param, scale, khat):
        """Network inputs [R][P][n_classes + 11] of mlfma_learned_guess (host)."""
        khat = np.ascontiguousarray(np.atleast_2d(khat), np.float64)
        cp = np.ascontiguousarray(class_param, np.float64)
        if len(cp) != self.n_classes:
            raise ValueError("class_param needs one entry per class")
        out = np.zeros((len(khat), self.n_particles, self.n_classes + 11), np.float32)
        self._check(lib().mlfma_guess_features(self._h, _dptr(cp), float(scale), len(khat), _dptr(khat),
                                               out.ctypes.data_as(C.POINTER(C.c_float))), "guess_features")
        return out

    def learned_guess(self, net: "Mlp", class_param, scale, khat, out=None, stream=None):
        """x0 [R][P][2N] predicted by `net` for directions khat [R][3]."""
        import torch
        khat = np.ascontiguousarray(np.atleast_2d(khat), np.float64)
        cp = np.ascontiguousarray(class_param, np.float64)
        if len(cp) != self.n_classes:
            raise ValueError("class_param needs one entry per class")
        R = len(khat)
        if out is None:
            out = torch.empty(self._shape(R), dtype=self.dtype, device="cuda")
        self._check(lib().mlfma_learned_guess(self._h, net._h, _dptr(cp), float(scale), R, _dptr(khat),
                                              self._dev(out, R), _stream_ptr(stream)), "learned_guess")
        return out

    def set_static_modes(self, class_id, verts, tris, edges, n_perp, n_par, M, eps):
        v = np.ascontiguousarray(verts, np.float64)
        t = np.ascontiguousarray(tris, np.int32)
        e = np.ascontiguousarray(edges, np.int32)
        Mm = np.ascontiguousarray(M, np.float64)
        eps = complex(eps)
        self._check(lib().mlfma_set_static_modes(self._h, class_id, len(v), _dptr(v), len(t), _iptr(t), len(e),
                                                 _iptr(e), n_perp, n_par, _dptr(Mm), eps.real, eps.imag),
                    "set_static_modes")
        self.n_modes = n_perp + n_par

    def prepare(self):
        self._check(lib().mlfma_prepare(self._h), "prepare")

    def _shape(self, R):
        return (R, self.n_particles, 2 * self.n_modes)

    def _dev(self, t, R):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == self.dtype and t.is_contiguous()
                and tuple(t.shape) == self._shape(R)):
            raise ValueError(f"expected a contiguous {self.dtype} device tensor of shape {self._shape(R)}")
        return C.c_void_p(t.data_ptr())

    def plane_wave_rhs(self, khat, pol, out=None, stream=None):
        import torch
        khat = np.ascontiguousarray(np.atleast_2d(khat), np.float64)
        pol = np.atleast_2d(np.asarray(pol, complex))
        R = len(khat)
        polri = np.ascontiguousarray(np.stack([pol.real, pol.imag], -1).reshape(R, 6), np.float64)
        if out is None:
            out = torch.empty(self._shape(R), dtype=self.dtype, device="cuda")
        self._check(lib().mlfma_plane_wave_rhs(self._h, R, _dptr(khat), _dptr(polri), self._dev(out, R),
                                               _stream_ptr(stream)), "plane_wave_rhs")
        return out

    def matvec_parts(self, x, parts=PART_ALL, out=None, stream=None):
        import torch
        R = x.shape[0]
        if out is None:
            out = torch.empty_like(x)
        self._check(lib().mlfma_matvec_parts(self._h, self._dev(x, R), self._dev(out, R), R, parts,
                                             _stream_ptr(stream)), "matvec")
        return out

    def matvec(self, x, out=None, stream=None):
        import torch
        R = x.shape[0]
        if out is None:
            out = torch.empty_like(x)
        self._check(lib().mlfma_matvec(self._h, self._dev(x, R), self._dev(out, R), R, _stream_ptr(stream)),
                    "matvec")
        return out

    def matvec_noalloc(self, x, out, stream=None):
        """mlfma_matvec_noalloc: the product with the library's static
        scratch (the context must be prepared; `out` is caller-allocated)."""
        R = x.shape[0]
        self._check(lib().mlfma_matvec_noalloc(self._h, self._dev(x, R), self._dev(out, R), R,
                                               _stream_ptr(stream)), "matvec_noalloc")
        return out

    def precondition(self, x, out=None, stream=None):
        import torch
        R = x.shape[0]
        if out is None:
            out = torch.empty_like(x)
        self._check(lib().mlfma_precondition(self._h, self._dev(x, R), self._dev(out, R), R, _stream_ptr(stream)),
                    "precondition")
        return out

    def fields(self, x, points, stream=None):
        """Scattered E at host points [n][3] from currents x [R][P][2N]
        (mlfma_fields): device tensor [R][n][3] in the context dtype."""
        import torch
        R = x.shape[0]
        pts = np.ascontiguousarray(np.atleast_2d(points), np.float64)
        if pts.ndim != 2 or pts.shape[1] != 3:
            raise ValueError("points must be [n][3]")
        out = torch.empty((R, len(pts), 3), dtype=self.dtype, device=x.device)
        self._check(lib().mlfma_fields(self._h, self._dev(x, R), R, len(pts), _dptr(pts), out.data_ptr(),
                                       _stream_ptr(stream)), "fields")
        return out

    def gmres_solve(self, b, x=None, rtol=1e-4, max_iter=1000, restart=100, use_x0=False, always_reorth=False,
                    fp32_basis=False, stream=None):
        import torch
        R = b.shape[0]
        if x is None:
            x = torch.zeros_like(b)
        stats = (SolveStats * R)()
        rc = self._check(lib().mlfma_gmres_solve(self._h, self._dev(b, R), self._dev(x, R), R, rtol, max_iter,
                                                 restart, (SOLVE_USE_X0 if use_x0 else 0)
                                                 | (SOLVE_ALWAYS_REORTH if always_reorth else 0)
                                                 | (SOLVE_FP32_BASIS if fp32_basis else 0), stats,
                                                 _stream_ptr(stream)), "gmres_solve")
        out = [dict(iterations=s.iterations, true_rel_res=s.true_rel_res, time_s=s.time_s,
                    converged=bool(s.converged), reorth=s.reorth, cycles=s.cycles) for s in stats]
        return x, out, rc

    def profile(self, enable: bool):
        self._check(lib().mlfma_profile(self._h, 1 if enable else 0), "profile")

    def profile_read(self):
        arr = (StageTime * 128)()
        cnt = C.c_int32()
        self._check(lib().mlfma_profile_read(self._h, 128, arr, C.byref(cnt)), "profile_read")
        return [dict(name=a.name.decode(), total_ms=a.total_ms, launches=a.launches,
                     bytes_per_launch=a.bytes_per_launch, flops_per_launch=a.flops_per_launch,
                     kernel=a.kernel.decode())
                for a in arr[: cnt.value]]

    def info(self) -> dict:
        inf = Info()
        self._check(lib().mlfma_info(self._h, C.byref(inf)), "info")
        n = inf.n_levels
        return dict(n_levels=n, L=list(inf.L[:n]), K=list(inf.K[:n]), nx=list(inf.nx[:n]), ny=list(inf.ny[:n]),
                    n_unknowns=inf.n_unknowns, n_modes=inf.n_modes, device_bytes=inf.device_bytes)

    # ---- diagnostics (host-side tables) ----
    def debug_near_block(self, cp, cq, dx, dy):
        if self.n_modes is None:
            raise MlfmaError(ENOTREADY, "no class has static modes")
        n = 2 * self.n_modes
        out = np.zeros((n, n), complex)
        self._check(lib().mlfma_debug_near_block(self._h, cp, cq, dx, dy, out.ctypes.data_as(C.POINTER(C.c_double))),
                    "debug_near_block")
        return out

    def debug_pair_block_device(self, cp, cq, dx, dy):
        if self.n_modes is None:
            raise MlfmaError(ENOTREADY, "no class has static modes")
        n = 2 * self.n_modes
        out = np.zeros((n, n), complex)
        self._check(lib().mlfma_debug_pair_block_device(self._h, cp, cq, dx, dy,
                                                        out.ctypes.data_as(C.POINTER(C.c_double))),
                    "debug_pair_block_device")
        return out

    def debug_leaf_pattern(self, c):
        K = self.info()["K"][0]
        out = np.zeros((K, 2, self.n_modes), complex)
        self._check(lib().mlfma_debug_leaf_pattern(self._h, c, out.ctypes.data_as(C.POINTER(C.c_double))),
                    "debug_leaf_pattern")
        return out

    def debug_level_grid(self, level):
        K = self.info()["K"][level]
        kh = np.zeros((K, 3))
        w = np.zeros(K)
        self._check(lib().mlfma_debug_level_grid(self._h, level, _dptr(kh), _dptr(w)), "debug_level_grid")
        return kh, w

    def debug_interpolate(self, level, pattern):
        """pattern: [K_{level-1}][2] complex (theta, phi) -> [K_level][2]."""
        K = self.info()["K"]
        u = np.ascontiguousarray(pattern, complex)
        if u.shape != (K[level - 1], 2):
            raise ValueError(f"expected a pattern of shape {(K[level - 1], 2)}")
        out = np.zeros((K[level], 2), complex)
        self._check(lib().mlfma_debug_interpolate(self._h, level, u.ctypes.data_as(C.POINTER(C.c_double)),
                                                  out.ctypes.data_as(C.POINTER(C.c_double))), "debug_interpolate")
        return out

    def debug_translation(self, level, dx, dy):
        K = self.info()["K"][level]
        out = np.zeros(K, complex)
        self._check(lib().mlfma_debug_translation(self._h, level, dx, dy, out.ctypes.data_as(C.POINTER(C.c_double))),
                    "debug_translation")
        return out


class Mlp:
    """The learned initial guess's network (mlfma_mlp_*): FP32 on the GPU."""

    def __init__(self, sizes, seed: int = 0):
        arr = np.ascontiguousarray(sizes, np.int32)
        h = C.c_void_p()
        rc = lib().mlfma_mlp_create(len(arr) - 1, _iptr(arr), C.c_uint64(seed), C.byref(h))
        if rc != OK:
            raise MlfmaError(rc, "mlp_create rejected the sizes")
        self._h = h
        self.sizes = [int(v) for v in arr]

    def _check(self, rc, what):
        if rc < 0:
            raise MlfmaError(rc, f"{what}: {lib().mlfma_mlp_last_error(self._h).decode()}")
        return rc

    def close(self):
        if getattr(self, "_h", None):
            lib().mlfma_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(lib().mlfma_mlp_num_params(self._h))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.num_params, np.float32)
        self._check(lib().mlfma_mlp_get_params(self._h, out.ctypes.data_as(C.POINTER(C.c_float))), "get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        if p.size != self.num_params:
            raise ValueError("parameter vector size")
        self._check(lib().mlfma_mlp_set_params(self._h, p.ctypes.data_as(C.POINTER(C.c_float))), "set_params")

    def layers(self, p=None):
        """Split a flat parameter vector into [(W [out][in], b [out]), ...]."""
        p = self.get_params() if p is None else p
        out, o = [], 0
        for i, j in zip(self.sizes[:-1], self.sizes[1:]):
            W = p[o:o + i * j].reshape(j, i)
            o += i * j
            b = p[o:o + j]
            o += j
            out.append((W, b))
        return out

    def forward(self, X, out=None, stream=None):
        import torch
        n = X.shape[0]
        if out is None:
            out = torch.empty((n, self.sizes[-1]), dtype=torch.float32, device=X.device)
        self._check(lib().mlfma_mlp_forward(self._h, C.c_void_p(X.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                            _stream_ptr(stream)), "forward")
        return out

    def loss_grad(self, X, T, stream=None):
        loss = C.c_double()
        g = np.zeros(self.num_params, np.float32)
        self._check(lib().mlfma_mlp_loss_grad(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                              X.shape[0], C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_float)),
                                              _stream_ptr(stream)), "loss_grad")
        return loss.value, g

    def train_step(self, X, T, lr, stream=None):
        loss = C.c_double()
        self._check(lib().mlfma_mlp_train_step(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()),
                                               X.shape[0], C.c_float(lr), C.byref(loss), _stream_ptr(stream)),
                    "train_step")
        return loss.value
