"""ctypes binding of libpeifem (the C ABI declared in include/peifem.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch supplies device memory (tensor data pointers) and the
HIP stream; if the library is missing this module raises instead of falling
back to anything else.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
# PEIFEM_LIB selects another build of the same library (the host-sanitizer
# build); there is no other implementation behind this binding
LIB_PATH = os.environ.get("PEIFEM_LIB") or os.path.join(HERE, "libpeifem.so")

PE_OK = 0
PE_E_ARG = -1
PE_E_HIP = -2
PE_E_WORKSPACE = -3
PE_E_NUMERIC = -4
PE_E_UNSUPPORTED = -5
PE_MAX_DIM = 3
PE_MAX_STAGES = 8
PE_MAX_TERMS = 64
PE_MAX_ITERS = 64
PE_NOALLOC_MAX_DOF = 1 << 25
PE_FP64 = 0
PE_SPLIT_BF16 = 1
PE_TRANSFORM_DENSE = 0
PE_TRANSFORM_FFT = 1

EXPORTS = [
    "pe_init_grid", "pe_init_grid_periodic", "pe_free_grid", "pe_set_transform", "pe_set_fusion",
    "pe_set_forcing", "pe_set_boundary",
    "pe_set_moving_sources",
    "pe_phi_tables", "pe_project_workspace_bytes", "pe_project", "pe_project_state",
    "pe_fine_workspace_bytes",
    "pe_fine_propagate", "pe_coarse_workspace_bytes", "pe_coarse_sweep", "pe_coarse_sweep_noalloc",
    "pe_solve_workspace_bytes", "pe_parareal_solve", "pe_grid_dof",
    "pe_grid_precision", "pe_last_error", "pe_set_timing", "pe_get_timing",
    "pe_mlp_create", "pe_mlp_free", "pe_mlp_get_params", "pe_mlp_set_params", "pe_mlp_forward",
    "pe_mlp_train_step", "pe_learned_samples_workspace_bytes", "pe_learned_samples",
    "pe_learned_rows_workspace_bytes", "pe_learned_rows",
    "pe_learned_correction_workspace_bytes", "pe_learned_correction",
]
PE_MLP_INPUTS, PE_MLP_WIDTH, PE_MLP_PARAMS, PE_MLP_SAMPLES = 12, 64, 9217, 8
(PE_K_DST_LAST, PE_K_DST_MID, PE_K_LOAD, PE_K_UPDATE, PE_K_SWEEP, PE_K_MID_UPDATE,
 PE_K_COARSE_FORCING, PE_K_COUNT) = 0, 1, 2, 3, 4, 5, 6, 7
KERNEL_CLASSES = ("dst_last", "dst_mid", "load", "update", "sweep", "mid_update",
                  "coarse_forcing")


class PeifemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"peifem error {status}: {msg}")
        self.status = status


class SpaceFactor(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("phase", ctypes.c_double),
                ("poly", ctypes.c_double * 3)]


class TimeFactor(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("omega", ctypes.c_double),
                ("phase", ctypes.c_double), ("poly", ctypes.c_double * 4)]


class Term(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_double), ("time", TimeFactor),
                ("space", SpaceFactor * PE_MAX_DIM)]


class MovingHat(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_double), ("axis", ctypes.c_int32), ("width", ctypes.c_double),
                ("c0", ctypes.c_double), ("c1", ctypes.c_double), ("omega", ctypes.c_double),
                ("phase", ctypes.c_double), ("time", TimeFactor),
                ("space", SpaceFactor * PE_MAX_DIM)]


class KernelStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class SolveParams(ctypes.Structure):
    _fields_ = [("t0", ctypes.c_double), ("T", ctypes.c_double), ("N", ctypes.c_int32),
                ("J", ctypes.c_int32), ("p", ctypes.c_int32), ("q", ctypes.c_int32),
                ("cG", ctypes.c_double * PE_MAX_STAGES), ("cF", ctypes.c_double * PE_MAX_STAGES),
                ("K_max", ctypes.c_int32), ("tol", ctypes.c_double),
                ("d_corr", ctypes.c_void_p), ("mlp", ctypes.c_void_p)]


class SolveReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("jumps", ctypes.c_double * PE_MAX_ITERS), ("ms_tables", ctypes.c_double),
                ("ms_coarse", ctypes.c_double), ("ms_fine", ctypes.c_double),
                ("ms_sweep", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_learned", ctypes.c_double), ("fallback", ctypes.c_int32),
                ("residuals", ctypes.c_double * PE_MAX_ITERS)]


_lib = None


def load_library():
    """Load libpeifem.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    dp = ctypes.POINTER(ctypes.c_double)
    L.pe_init_grid.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i32), dp, dp, dbl, i32, i32, vp]
    L.pe_init_grid_periodic.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i32), dp, dp, dbl, i32,
                                        i32, ctypes.POINTER(i32), vp]
    L.pe_free_grid.argtypes = [vp]
    L.pe_free_grid.restype = None
    L.pe_set_transform.argtypes = [vp, i32]
    L.pe_set_fusion.argtypes = [vp, i32]
    L.pe_set_forcing.argtypes = [vp, i32, ctypes.POINTER(Term), vp]
    L.pe_set_boundary.argtypes = [vp, i32, ctypes.POINTER(Term), vp]
    L.pe_set_moving_sources.argtypes = [vp, i32, ctypes.POINTER(MovingHat), vp]
    L.pe_project_state.argtypes = [vp, i32, ctypes.POINTER(Term), dbl, vp, vp, sz, vp]
    L.pe_phi_tables.argtypes = [vp, dbl, i32, dp, vp, vp, vp]
    L.pe_project_workspace_bytes.argtypes = [vp]
    L.pe_project_workspace_bytes.restype = sz
    L.pe_project.argtypes = [vp, i32, ctypes.POINTER(Term), vp, vp, sz, vp]
    L.pe_fine_workspace_bytes.argtypes = [vp, i64]
    L.pe_fine_workspace_bytes.restype = sz
    L.pe_fine_propagate.argtypes = [vp, i32, dbl, dbl, i32, i32, dp, vp, vp, vp, vp, vp, sz, vp]
    L.pe_coarse_workspace_bytes.argtypes = [vp, i32, i32]
    L.pe_coarse_workspace_bytes.restype = sz
    L.pe_coarse_sweep.argtypes = [vp, i32, dbl, dbl, i32, dp, vp, vp, i32, vp, vp, vp, vp, vp, vp,
                                  vp, sz, vp]
    L.pe_coarse_sweep_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.pe_solve_workspace_bytes.argtypes = [vp, ctypes.POINTER(SolveParams)]
    L.pe_solve_workspace_bytes.restype = sz
    L.pe_parareal_solve.argtypes = [vp, ctypes.POINTER(SolveParams), vp, vp, vp, sz,
                                    ctypes.POINTER(SolveReport), vp]
    L.pe_grid_dof.argtypes = [vp]
    L.pe_grid_dof.restype = i64
    L.pe_grid_precision.argtypes = [vp]
    L.pe_grid_precision.restype = i32
    L.pe_set_timing.argtypes = [vp, i32]
    L.pe_get_timing.argtypes = [vp, ctypes.POINTER(KernelStat)]
    fp = ctypes.POINTER(ctypes.c_float)
    L.pe_mlp_create.argtypes = [ctypes.POINTER(vp), fp, vp]
    L.pe_mlp_free.argtypes = [vp]
    L.pe_mlp_free.restype = None
    L.pe_mlp_get_params.argtypes = [vp, fp, vp]
    L.pe_mlp_set_params.argtypes = [vp, fp, vp]
    L.pe_mlp_forward.argtypes = [vp, i64, vp, vp, vp]
    L.pe_mlp_train_step.argtypes = [vp, i64, vp, vp, ctypes.c_float, i32, vp, vp, vp]
    L.pe_learned_samples_workspace_bytes.argtypes = [vp, i32]
    L.pe_learned_samples_workspace_bytes.restype = sz
    L.pe_learned_samples.argtypes = [vp, i32, dbl, dbl, vp, vp, sz, vp]
    L.pe_learned_rows_workspace_bytes.argtypes = [vp, i32]
    L.pe_learned_rows_workspace_bytes.restype = sz
    L.pe_learned_rows.argtypes = [vp, i32, dbl, dbl, vp, vp, dbl, vp, vp, vp, i64,
                                  ctypes.POINTER(ctypes.c_int64), vp, sz, vp]
    L.pe_learned_correction_workspace_bytes.argtypes = [vp, i32]
    L.pe_learned_correction_workspace_bytes.restype = sz
    L.pe_learned_correction.argtypes = [vp, vp, i32, dbl, dbl, vp, ctypes.POINTER(ctypes.c_int32),
                                        vp, sz, vp]
    L.pe_last_error.argtypes = []
    L.pe_last_error.restype = ctypes.c_char_p
    for name in ("pe_init_grid", "pe_init_grid_periodic", "pe_set_transform", "pe_set_fusion",
                 "pe_set_forcing", "pe_set_boundary",
                 "pe_set_moving_sources",
                 "pe_project_state", "pe_phi_tables", "pe_project",
                 "pe_fine_propagate", "pe_coarse_sweep", "pe_coarse_sweep_noalloc",
                 "pe_parareal_solve", "pe_set_timing",
                 "pe_get_timing", "pe_mlp_create", "pe_mlp_get_params", "pe_mlp_set_params",
                 "pe_mlp_forward", "pe_mlp_train_step", "pe_learned_samples", "pe_learned_rows",
                 "pe_learned_correction"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def _check(status: int):
    if status != PE_OK:
        msg = load_library().pe_last_error().decode(errors="replace")
        raise PeifemError(status, msg)


def _dbl_array(vals: Sequence[float]):
    arr = (ctypes.c_double * max(1, len(vals)))(*[float(v) for v in vals])
    return arr


def to_c_terms(terms) -> Tuple[ctypes.Array, int]:
    """Separable descriptors (objects with amp / time / space attributes, as
    in the workloads module) -> a ctypes pe_term array."""
    terms = list(terms)
    if len(terms) > PE_MAX_TERMS:
        raise ValueError(f"at most {PE_MAX_TERMS} terms")
    arr = (Term * max(1, len(terms)))()
    for i, t in enumerate(terms):
        arr[i].amp = t.amp
        tf = t.time
        arr[i].time.alpha = tf.alpha
        arr[i].time.omega = tf.omega
        arr[i].time.phase = tf.phase
        for j in range(4):
            arr[i].time.poly[j] = tf.poly[j]
        for a, sf in enumerate(t.space):
            arr[i].space[a].kappa = sf.kappa
            arr[i].space[a].phase = sf.phase
            for j in range(3):
                arr[i].space[a].poly[j] = sf.poly[j]
        for a in range(len(t.space), PE_MAX_DIM):
            arr[i].space[a].kappa = 0.0
            arr[i].space[a].phase = math.pi / 2
            arr[i].space[a].poly[0] = 1.0
    return arr, len(terms)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Grid:
    """A pe_grid handle plus its forcing."""

    def __init__(self, n: Sequence[int], lo: Sequence[float], hi: Sequence[float], D: float,
                 precision: str = "fp64", quad_q: int = 3, device: str = "cuda:0", stream=None,
                 transform: str = "dense", periodic: Optional[Sequence[bool]] = None):
        import torch
        self.L = load_library()
        self.device = torch.device(device)
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        self.precision = precision
        prec = {"fp64": PE_FP64, "split_bf16": PE_SPLIT_BF16}[precision]
        self.state_dtype = torch.float64 if prec == PE_FP64 else torch.float32
        self.stream = stream
        handle = ctypes.c_void_p()
        nn = (ctypes.c_int32 * len(self.n))(*self.n)
        self.periodic = tuple(bool(p) for p in periodic) if periodic else (False,) * self.dim
        with torch.cuda.device(self.device):
            if any(self.periodic):
                per = (ctypes.c_int32 * self.dim)(*[int(p) for p in self.periodic])
                _check(self.L.pe_init_grid_periodic(ctypes.byref(handle), self.dim, nn,
                                                    _dbl_array(lo), _dbl_array(hi), float(D), prec,
                                                    int(quad_q), per, _stream(stream)))
            else:
                _check(self.L.pe_init_grid(ctypes.byref(handle), self.dim, nn, _dbl_array(lo),
                                           _dbl_array(hi), float(D), prec, int(quad_q),
                                           _stream(stream)))
        self.h = handle
        self.dof = int(self.L.pe_grid_dof(self.h))
        self.transform = "fft" if any(self.periodic) else "dense"
        if transform != "dense" and transform != self.transform:
            self.set_transform(transform)

    @classmethod
    def from_problem(cls, prob, quad_q: int = 3, device: str = "cuda:0", stream=None,
                     transform: str = "dense") -> "Grid":
        g = cls(prob.n, prob.lo, prob.hi, prob.D, prob.precision, quad_q, device, stream,
                transform, getattr(prob, "periodic", None) or None)
        g.set_forcing(prob.forcing)
        if getattr(prob, "boundary", None):
            g.set_boundary(prob.boundary)
        if getattr(prob, "moving", None):
            g.set_moving_sources(prob.moving)
        return g

    def set_fusion(self, enable: bool):
        """Generating and middle-axis passes as one kernel on 3D split-bf16
        grids (the default) or as two passes."""
        _check(self.L.pe_set_fusion(self.h, 1 if enable else 0))

    def set_transform(self, kind: str):
        """"dense" (matrix-core products) or "fft" (LDS FFT of the odd extension)."""
        import torch
        code = {"dense": PE_TRANSFORM_DENSE, "fft": PE_TRANSFORM_FFT}[kind]
        with torch.cuda.device(self.device):
            _check(self.L.pe_set_transform(self.h, code))
        self.transform = kind

    def close(self):
        if getattr(self, "h", None):
            self.L.pe_free_grid(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers --------------------------------------------------------
    def empty_states(self, count: int):
        import torch
        return torch.empty((count,) + self.n, dtype=self.state_dtype, device=self.device)

    def workspace(self, nbytes: int):
        import torch
        return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=self.device)

    # -- instrumentation --------------------------------------------------
    def set_timing(self, enable: bool):
        _check(self.L.pe_set_timing(self.h, 1 if enable else 0))

    def get_timing(self) -> dict:
        arr = (KernelStat * PE_K_COUNT)()
        _check(self.L.pe_get_timing(self.h, arr))
        return {name: dict(launches=int(arr[i].launches), ms=float(arr[i].ms),
                           flops=float(arr[i].flops), bytes=float(arr[i].bytes))
                for i, name in enumerate(KERNEL_CLASSES)}

    # -- calls ----------------------------------------------------------
    def set_forcing(self, terms):
        arr, m = to_c_terms(terms)
        _check(self.L.pe_set_forcing(self.h, m, arr, _stream(self.stream)))

    def set_moving_sources(self, hats):
        """Moving hat sources (objects with the workloads.MovingHat fields)."""
        hats = list(hats)
        arr = (MovingHat * max(1, len(hats)))()
        for i, h in enumerate(hats):
            arr[i].amp, arr[i].axis, arr[i].width = h.amp, h.axis, h.width
            arr[i].c0, arr[i].c1, arr[i].omega, arr[i].phase = h.c0, h.c1, h.omega, h.phase
            tf = h.time
            arr[i].time.alpha, arr[i].time.omega, arr[i].time.phase = tf.alpha, tf.omega, tf.phase
            for j in range(4):
                arr[i].time.poly[j] = tf.poly[j]
            for a in range(PE_MAX_DIM):
                sf = h.space[a] if a < len(h.space) else None
                arr[i].space[a].kappa = sf.kappa if sf else 0.0
                arr[i].space[a].phase = sf.phase if sf else math.pi / 2
                for j in range(3):
                    arr[i].space[a].poly[j] = sf.poly[j] if sf else (1.0 if j == 0 else 0.0)
        _check(self.L.pe_set_moving_sources(self.h, len(hats), arr, _stream(self.stream)))

    def set_boundary(self, terms):
        """Dirichlet data g (separable terms); [] for homogeneous data."""
        arr, m = to_c_terms(terms)
        _check(self.L.pe_set_boundary(self.h, m, arr, _stream(self.stream)))

    def project_state(self, terms, t: float):
        """Interior state whose boundary values are the Dirichlet data at t and
        which is otherwise the L2 projection of `terms`."""
        arr, m = to_c_terms(terms)
        W = self.empty_states(1)[0]
        nb = self.L.pe_project_workspace_bytes(self.h)
        work = self.workspace(nb)
        _check(self.L.pe_project_state(self.h, m, arr, float(t), _ptr(W), _ptr(work), nb,
                                       _stream(self.stream)))
        return W

    def phi_tables(self, h: float, c: Sequence[float]):
        import torch
        s = len(c)
        E = torch.empty(self.n, dtype=torch.float64, device=self.device)
        B = torch.empty((s,) + self.n, dtype=torch.float64, device=self.device)
        _check(self.L.pe_phi_tables(self.h, float(h), s, _dbl_array(c), _ptr(E), _ptr(B),
                                    _stream(self.stream)))
        return E, B

    def project(self, terms):
        arr, m = to_c_terms(terms)
        W = self.empty_states(1)[0]
        nb = self.L.pe_project_workspace_bytes(self.h)
        work = self.workspace(nb)
        _check(self.L.pe_project(self.h, m, arr, _ptr(W), _ptr(work), nb, _stream(self.stream)))
        return W

    def fine_workspace_bytes(self, fields: int) -> int:
        return int(self.L.pe_fine_workspace_bytes(self.h, int(fields)))

    def fine_propagate(self, Uin, t0: float, dT: float, J: int, c: Sequence[float], E, B,
                       Uout=None, work=None):
        n_slices = Uin.shape[0]
        if Uout is None:
            Uout = self.empty_states(n_slices)
        if work is None:
            work = self.workspace(self.fine_workspace_bytes(n_slices * J * len(c)))
        _check(self.L.pe_fine_propagate(self.h, n_slices, float(t0), float(dT), int(J), len(c),
                                        _dbl_array(c), _ptr(E), _ptr(B), _ptr(Uin), _ptr(Uout),
                                        _ptr(work), work.numel(), _stream(self.stream)))
        return Uout

    def coarse_sweep(self, U, t0: float, dT: float, c: Sequence[float], E, B, r, compute_r=True,
                     corr=None, Uprev=None, Fout=None, norms=None, work=None):
        N = U.shape[0] - 1
        if norms is not None and norms.numel() < 3:
            raise ValueError("norms must hold 3 doubles (jump, norm, residual)")
        if work is None:
            work = self.workspace(self.L.pe_coarse_workspace_bytes(self.h, N, len(c)))
        _check(self.L.pe_coarse_sweep(self.h, N, float(t0), float(dT), len(c), _dbl_array(c),
                                      _ptr(E), _ptr(B), 1 if compute_r else 0, _ptr(r),
                                      _ptr(corr), _ptr(Uprev), _ptr(Fout), _ptr(U), _ptr(norms),
                                      _ptr(work), work.numel(), _stream(self.stream)))
        return U

    def coarse_sweep_noalloc(self, U, E, r, corr=None, Uprev=None, Fout=None, norms=None):
        """pe_coarse_sweep with r given, no workspace (static norm partials)."""
        N = U.shape[0] - 1
        if norms is not None and norms.numel() < 3:
            raise ValueError("norms must hold 3 doubles (jump, norm, residual)")
        _check(self.L.pe_coarse_sweep_noalloc(self.h, N, _ptr(E), _ptr(r), _ptr(corr),
                                              _ptr(Uprev), _ptr(Fout), _ptr(U), _ptr(norms),
                                              _stream(self.stream)))
        return U

    def learned_samples(self, N: int, t0: float, dT: float, out=None, work=None):
        """Spectral forcing at T_n + s dT/7, s = 0..7, for every slice: [8N, *grid]."""
        if out is None:
            out = self.empty_states(PE_MLP_SAMPLES * N)
        if work is None:
            work = self.workspace(self.L.pe_learned_samples_workspace_bytes(self.h, N))
        _check(self.L.pe_learned_samples(self.h, N, float(t0), float(dT), _ptr(out), _ptr(work),
                                         work.numel(), _stream(self.stream)))
        return out

    def learned_rows(self, R, r, t0: float, dT: float, rel_thresh: float = 1e-9,
                     max_rows: Optional[int] = None, want_scale: bool = False):
        """Training rows (x [rows, 12], target [rows], count) of the slices
        starting at t0 + n dT whose forcing samples have a part of degree >= 4
        (R = F^J(0), r = G(0) per slice); with want_scale the rows' output
        scales s [rows] come third."""
        import torch
        N = R.shape[0]
        if max_rows is None:
            max_rows = N * self.dof
        x = torch.empty((max(max_rows, 1), PE_MLP_INPUTS), dtype=torch.float32, device=self.device)
        t = torch.empty(max(max_rows, 1), dtype=torch.float32, device=self.device)
        sc = (torch.empty(max(max_rows, 1), dtype=torch.float32, device=self.device)
              if want_scale else None)
        work = self.workspace(self.L.pe_learned_rows_workspace_bytes(self.h, N))
        cnt = ctypes.c_int64(0)
        _check(self.L.pe_learned_rows(self.h, N, float(t0), float(dT), _ptr(R), _ptr(r),
                                      float(rel_thresh), _ptr(x), _ptr(t), _ptr(sc),
                                      int(max_rows), ctypes.byref(cnt), _ptr(work), work.numel(),
                                      _stream(self.stream)))
        n = min(int(cnt.value), max_rows)
        if want_scale:
            return x[:n], t[:n], sc[:n], int(cnt.value)
        return x[:n], t[:n], int(cnt.value)

    def learned_correction(self, mlp: "Mlp", N: int, t0: float, dT: float, out=None, work=None):
        """delta_n for slices starting at t0 + n dT: ([N, *grid], fallback)."""
        if out is None:
            out = self.empty_states(N)
        if work is None:
            work = self.workspace(self.L.pe_learned_correction_workspace_bytes(self.h, N))
        fb = ctypes.c_int32(0)
        _check(self.L.pe_learned_correction(self.h, mlp.h, N, float(t0), float(dT), _ptr(out),
                                            ctypes.byref(fb), _ptr(work), work.numel(),
                                            _stream(self.stream)))
        return out, bool(fb.value)

    def solve_params(self, t0, T, N, J, cG, cF, K_max, tol, corr=None, mlp=None) -> SolveParams:
        P = SolveParams()
        P.t0, P.T, P.N, P.J = float(t0), float(T), int(N), int(J)
        P.p, P.q = len(cG), len(cF)
        for i, v in enumerate(cG):
            P.cG[i] = v
        for i, v in enumerate(cF):
            P.cF[i] = v
        P.K_max, P.tol = int(K_max), float(tol)
        P.d_corr = _ptr(corr)
        P.mlp = mlp.h if mlp is not None else None
        return P

    def solve_workspace_bytes(self, P: SolveParams) -> int:
        return int(self.L.pe_solve_workspace_bytes(self.h, ctypes.byref(P)))

    def parareal_solve(self, P: SolveParams, U0=None, U=None, work=None):
        if U is None:
            U = self.empty_states(P.N + 1)
        if work is None:
            work = self.workspace(self.solve_workspace_bytes(P))
        rep = SolveReport()
        _check(self.L.pe_parareal_solve(self.h, ctypes.byref(P), _ptr(U0), _ptr(U), _ptr(work),
                                        work.numel(), ctypes.byref(rep), _stream(self.stream)))
        return U, rep


class Mlp:
    """A pe_mlp handle (the learned coarse correction network)."""

    def __init__(self, params, stream=None):
        import numpy as np
        self.L = load_library()
        self.stream = stream
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        if p.size != PE_MLP_PARAMS:
            raise ValueError(f"expected {PE_MLP_PARAMS} parameters")
        h = ctypes.c_void_p()
        _check(self.L.pe_mlp_create(ctypes.byref(h), p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                    _stream(stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.pe_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np
        p = np.empty(PE_MLP_PARAMS, dtype=np.float32)
        _check(self.L.pe_mlp_get_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                        _stream(self.stream)))
        return p

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        _check(self.L.pe_mlp_set_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                        _stream(self.stream)))

    def forward(self, x):
        import torch
        y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _check(self.L.pe_mlp_forward(self.h, x.shape[0], _ptr(x), _ptr(y), _stream(self.stream)))
        return y

    def train_step(self, x, t, lr: float, apply: bool = True, want_grad: bool = False):
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        grad = torch.empty(PE_MLP_PARAMS, dtype=torch.float32, device=x.device) if want_grad else None
        _check(self.L.pe_mlp_train_step(self.h, x.shape[0], _ptr(x), _ptr(t), float(lr),
                                        1 if apply else 0, _ptr(loss), _ptr(grad),
                                        _stream(self.stream)))
        return loss, grad


def solve_problem(prob, K_max: Optional[int] = None, tol: Optional[float] = None,
                  corr=None, device: str = "cuda:0", mlp: Optional[Mlp] = None,
                  transform: str = "dense"):
    """Grid + forcing + P_h u0 + Algorithm 1 for a workloads.Problem."""
    g = Grid.from_problem(prob, device=device, transform=transform)
    if getattr(prob, "boundary", None):
        U0 = g.project_state(prob.u0, prob.t0)
    else:
        U0 = g.project(prob.u0) if prob.u0 else None
    P = g.solve_params(prob.t0, prob.T, prob.N, prob.J, prob.c_coarse, prob.c_fine,
                       prob.K_max if K_max is None else K_max, prob.tol if tol is None else tol, corr,
                       mlp)
    U, rep = g.parareal_solve(P, U0=U0)
    return g, U, rep
