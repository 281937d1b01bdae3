"""ctypes binding of libsf.so (the C ABI in include/sf.h).

Argument marshalling only: every step of the SF runs in the library's HIP
kernels.  torch supplies device memory (tensors, the workspace) and the
current stream.  There is no CPU fallback: if the library is missing or a call
fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
from pathlib import Path
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

LIB_PATH = Path(__file__).resolve().parent / "libsf.so"

SF_SAVE_FOR_BACKWARD = 1
SF_PLAIN = 2
SF_GRAPH = 4
SF_UNFUSED = 8

_ERRORS = {0: "SF_OK", -1: "SF_ERR_INVALID_ARG", -2: "SF_ERR_SHAPE",
           -3: "SF_ERR_WORKSPACE_SMALL", -4: "SF_ERR_NOT_SAVED", -5: "SF_ERR_HIP",
           -6: "SF_ERR_NONFINITE"}

EXPORTED = ("sf_setup", "sf_project", "sf_project_backward", "sf_destroy",
            "sf_error_string", "sf_last_error_detail", "sf_plan_threads", "sf_set_early_exit",
            "sf_project_iterations")


class SFError(RuntimeError):
    def __init__(self, code: int, detail: str):
        super().__init__(f"{_ERRORS.get(code, code)}: {detail}")
        self.code = code
        self.detail = detail


class SFConfigC(ctypes.Structure):
    _fields_ = [("n_dim", ctypes.c_int32), ("n_coef", ctypes.c_int32),
                ("n_steps", ctypes.c_int32), ("checkpoint_every", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("rho", ctypes.c_double)]


_lib = None


def load_library(path: Optional[Path] = None) -> ctypes.CDLL:
    """Load libsf.so (built by paper_2510_09204_amd.build); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path is not None else LIB_PATH
    if not p.exists():
        raise RuntimeError(f"SF library not built: {p} is missing "
                           "(run python -m paper_2510_09204_amd.build)")
    lib = ctypes.CDLL(str(p))
    vp, i32, f32p = ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p
    lib.sf_setup.argtypes = [ctypes.POINTER(SFConfigC), i32, vp, vp, vp, vp, vp,
                             ctypes.POINTER(ctypes.c_size_t), vp, ctypes.POINTER(vp)]
    lib.sf_setup.restype = ctypes.c_int
    lib.sf_project.argtypes = [vp, vp, f32p, f32p, f32p, f32p, f32p, i32, i32, f32p, f32p,
                               f32p, vp]
    lib.sf_project.restype = ctypes.c_int
    lib.sf_project_backward.argtypes = [vp, vp, f32p, f32p, f32p, ctypes.c_float, f32p, f32p,
                                        f32p, vp]
    lib.sf_project_backward.restype = ctypes.c_int
    lib.sf_destroy.argtypes = [vp]
    lib.sf_destroy.restype = None
    lib.sf_error_string.argtypes = [ctypes.c_int]
    lib.sf_error_string.restype = ctypes.c_char_p
    lib.sf_last_error_detail.argtypes = []
    lib.sf_last_error_detail.restype = ctypes.c_char_p
    lib.sf_plan_threads.argtypes = [vp]
    lib.sf_plan_threads.restype = ctypes.c_int
    lib.sf_set_early_exit.argtypes = [vp, ctypes.c_float, i32]
    lib.sf_set_early_exit.restype = ctypes.c_int
    lib.sf_project_iterations.argtypes = [vp, vp, vp, vp]
    lib.sf_project_iterations.restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _check(lib, rc: int) -> None:
    if rc != 0:
        raise SFError(rc, lib.sf_last_error_detail().decode())


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


class SFPlan:
    """A batch of SF problems sharing (n_coef, n_steps, rho) and its workspace.

    n_robots, n_obs, robot_a and box ([B][2][2] = p_min, p_max) describe each
    problem; the FP64 KKT factors are built on the host and the workspace is a
    torch uint8 tensor on `device`."""

    def __init__(self, n_robots: Sequence[int], n_obs: Sequence[int],
                 robot_a: Sequence[float], box, n_coef: int, n_steps: int, rho: float,
                 checkpoint_every: int = 1, max_iters: int = 0, threads: int = 0,
                 device="cuda"):
        self.lib = load_library()
        dev = torch.device(device)
        if dev.type == "cuda" and dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.n_robots = _host(n_robots, np.int32)
        self.n_obs = _host(n_obs, np.int32)
        self.robot_a = _host(robot_a, np.float32)
        self.box = _host(box, np.float32).reshape(-1, 2, 2)
        self.B = int(self.n_robots.size)
        self.n_coef, self.n_steps, self.rho = int(n_coef), int(n_steps), float(rho)
        self.cfg = SFConfigC(2, self.n_coef, self.n_steps, int(checkpoint_every),
                             int(max_iters), int(threads), self.rho)
        self.coef_size = int(2 * self.n_robots.astype(np.int64).sum() * self.n_coef)
        self.n_rob_total = int(self.n_robots.sum())
        self.n_obs_total = int(self.n_obs.sum())
        nbytes = ctypes.c_size_t(0)
        args = (ctypes.byref(self.cfg), self.B, self.n_robots.ctypes.data,
                self.n_obs.ctypes.data, self.robot_a.ctypes.data, self.box.ctypes.data)
        _check(self.lib, self.lib.sf_setup(*args, None, ctypes.byref(nbytes), None, None))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % 256:
            raise SFError(-1, "torch workspace allocation is not 256-byte aligned")
        plan = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(self.lib, self.lib.sf_setup(*args, ctypes.c_void_p(self.workspace.data_ptr()),
                                           ctypes.byref(nbytes), ctypes.c_void_p(stream),
                                           ctypes.byref(plan)))
        self._plan = plan

    @property
    def threads(self) -> int:
        return int(self.lib.sf_plan_threads(self._plan))

    def set_early_exit(self, tol: float, check_every: int) -> None:
        """sf_set_early_exit: stop a problem once its residual is <= tol at a
        check every `check_every` iterations (0 = off)."""
        _check(self.lib, self.lib.sf_set_early_exit(self._plan, float(tol), int(check_every)))

    def iterations(self) -> torch.Tensor:
        """sf_project_iterations: iterations each problem ran in the last
        project call, int32[B] on the device (on the current stream)."""
        out = torch.empty(self.B, dtype=torch.int32, device=self.device)
        _check(self.lib, self.lib.sf_project_iterations(
            self._plan, ctypes.c_void_p(self.workspace.data_ptr()), out.data_ptr(),
            self._stream()))
        return out

    def close(self) -> None:
        if getattr(self, "_plan", None):
            self.lib.sf_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _coef(self, t: torch.Tensor, name: str) -> torch.Tensor:
        if t.device != self.device or t.dtype != torch.float32 or not t.is_contiguous():
            raise SFError(-1, f"{name} must be a contiguous float32 tensor on {self.device}")
        if t.numel() != self.coef_size:
            raise SFError(-2, f"{name} has {t.numel()} elements, expected {self.coef_size}")
        return t

    def _stream(self) -> ctypes.c_void_p:
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def project(self, xi, xi0, lam0, boundary, obstacles, n_iters: int, save: bool = False,
                plain: bool = False, graph: bool = False, unfused: bool = False,
                out: Optional[Tuple[torch.Tensor, torch.Tensor, torch.Tensor]] = None):
        """Run sf_project; returns (xi_out, lam_out, residual[B][4])."""
        for t, name in ((xi, "xi"), (xi0, "xi0"), (lam0, "lam0")):
            self._coef(t, name)
        if boundary.numel() != self.n_rob_total * 4 or boundary.dtype != torch.float32 \
                or not boundary.is_contiguous() or boundary.device != self.device:
            raise SFError(-2, "boundary must be contiguous float32 [sum n][2][2] on device")
        if self.n_obs_total:
            if obstacles is None or obstacles.numel() != self.n_obs_total * 3 \
                    or obstacles.dtype != torch.float32 or not obstacles.is_contiguous() \
                    or obstacles.device != self.device:
                raise SFError(-2, "obstacles must be contiguous float32 [sum M][3] on device")
        if out is None:
            xi_out = torch.empty_like(xi)
            lam_out = torch.empty_like(xi)
            res = torch.empty((self.B, 4), dtype=torch.float32, device=self.device)
        else:
            xi_out, lam_out, res = out
        flags = (SF_SAVE_FOR_BACKWARD if save else 0) | (SF_PLAIN if plain else 0) | \
                (SF_GRAPH if graph else 0) | (SF_UNFUSED if unfused else 0)
        _check(self.lib, self.lib.sf_project(
            self._plan, ctypes.c_void_p(self.workspace.data_ptr()), xi.data_ptr(),
            xi0.data_ptr(), lam0.data_ptr(), boundary.data_ptr(),
            _ptr(obstacles) if self.n_obs_total else None, int(n_iters), flags,
            xi_out.data_ptr(), lam_out.data_ptr(), res.data_ptr(), self._stream()))
        return xi_out, lam_out, res

    def backward(self, g_xi_out=None, g_lam_out=None, g_residual=None, fp_weight: float = 0.0,
                 need=(True, True, True)):
        """Run sf_project_backward; returns (g_xi, g_xi0, g_lam0) (None where not needed)."""
        for t, name in ((g_xi_out, "g_xi_out"), (g_lam_out, "g_lam_out")):
            if t is not None:
                self._coef(t, name)
        if g_residual is not None and (g_residual.numel() != self.B * 4
                                       or g_residual.dtype != torch.float32
                                       or not g_residual.is_contiguous()):
            raise SFError(-2, "g_residual must be contiguous float32 [B][4]")
        outs = [torch.empty(self.coef_size, dtype=torch.float32, device=self.device)
                if need[q] else None for q in range(3)]
        _check(self.lib, self.lib.sf_project_backward(
            self._plan, ctypes.c_void_p(self.workspace.data_ptr()), _ptr(g_xi_out),
            _ptr(g_lam_out), _ptr(g_residual), float(fp_weight), _ptr(outs[0]),
            _ptr(outs[1]), _ptr(outs[2]), self._stream()))
        return tuple(outs)


class SFProject(torch.autograd.Function):
    """(xi, xi0, lam0) -> (xi_bar^L, lambda^L, residual[B][4]) through L unrolled SF
    iterations, with the hand-written adjoint of sf_project_backward.  The
    plan must have max_iters >= n_iters.  fp_weight adds fp_weight * sum_l L_FP^l
    (the fixed-point residual terms of the warm-start loss) to the loss being
    differentiated: its gradient is included in the backward."""

    @staticmethod
    def forward(ctx, xi, xi0, lam0, boundary, obstacles, plan: SFPlan, n_iters: int,
                fp_weight: float = 0.0):
        xi_out, lam_out, res = plan.project(xi.contiguous(), xi0.contiguous(),
                                            lam0.contiguous(), boundary, obstacles, n_iters,
                                            save=True)
        ctx.plan = plan
        ctx.fp_weight = float(fp_weight)
        return xi_out, lam_out, res

    @staticmethod
    def backward(ctx, g_xi_out, g_lam_out, g_res):
        need = ctx.needs_input_grad[:3]
        g_res = None if g_res is None else g_res.contiguous()
        g = ctx.plan.backward(None if g_xi_out is None else g_xi_out.contiguous(),
                              None if g_lam_out is None else g_lam_out.contiguous(),
                              g_res, ctx.fp_weight, need=tuple(bool(x) for x in need))
        return g[0], g[1], g[2], None, None, None, None, None


def to_device(packed, device="cuda"):
    """Move a workloads.PackedBatch's arrays to torch tensors on `device`."""
    def t(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return dict(xi=t(packed.xi), xi0=t(packed.xi0), lam0=t(packed.lam0),
                boundary=t(packed.boundary),
                obstacles=t(packed.obstacles) if packed.obstacles.size else None)
