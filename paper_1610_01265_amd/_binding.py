"""ctypes binding of libsts.so (include/sts.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.  PyTorch
supplies device memory and the current HIP stream."""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsts.so")

STS_OK, STS_NOT_CONVERGED = 0, 1
STS_EINVAL, STS_EHIP, STS_ENOMEM, STS_BREAKDOWN = -1, -2, -3, -4
SPHERICAL, CARTESIAN = 0, 1
BC_ZEROFLUX, BC_DIRICHLET, BC_PERIODIC = 0, 1, 2
PC_JACOBI, PC_BLOCK_ILU0, PC_FACTOR = 0, 1, 2
DEBUG_WG_REVERSE = 1
DEBUG_SEPARATE_FINALIZE = 2
SHELL_BC = (BC_DIRICHLET, BC_ZEROFLUX, BC_ZEROFLUX, BC_ZEROFLUX, BC_PERIODIC, BC_PERIODIC)

_STATUS = {0: "STS_OK", 1: "STS_NOT_CONVERGED", -1: "STS_EINVAL", -2: "STS_EHIP",
           -3: "STS_ENOMEM", -4: "STS_BREAKDOWN"}

_lib = None


class StsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


def load():
    """Load libsts.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1610_01265_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P, D, I = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    PI, PD = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    sig = {
        "sts_create": (I, [ctypes.POINTER(P), I, I, I, I, PD, PD, PD, PI, P]),
        "sts_destroy": (I, [P]),
        "sts_set_stream": (I, [P, P]),
        "sts_last_error": (ctypes.c_char_p, [P]),
        "sts_num_cells": (ctypes.c_longlong, [P]),
        "sts_set_spitzer": (I, [P, P, D, P, P, P]),
        "sts_set_isotropic": (I, [P, D]),
        "sts_set_spitzer_f32": (I, [P, P, D, P, P, P]),
        "sts_set_isotropic_f32": (I, [P, D]),
        "sts_set_dirichlet": (I, [P, I, P, D]),
        "sts_dt_euler": (I, [P, PD]),
        "apply_F": (I, [P, P, P, I]),
        "rkl2_step": (I, [P, P, I, D, I, PI]),
        "rkl2_step_noalloc": (I, [P, P, I, D, I, PI]),
        "rkl_step": (I, [P, P, I, D, I, I, I, I, D, D, PI]),
        "apply_F_nonlinear": (I, [P, P, P, D, P, P, P]),
        "rkl2_step_nonlinear": (I, [P, P, D, D, P, P, P, I, PI]),
        "sts_set_resistivity": (I, [P, D]),
        "sts_resistivity_sizes": (I, [P, ctypes.POINTER(ctypes.c_longlong)]),
        "apply_F_resistivity": (I, [P, P, P]),
        "resistivity_dt_euler": (I, [P, PD]),
        "resistivity_be_pcg_solve": (I, [P, P, P, D, D, I, PI, PD]),
        "be_pcg_solve": (I, [P, P, P, D, I, PI, D, I, PI, PD]),
        "sts_be_residual": (I, [P, P, P, D, PD]),
        "cnn_create": (I, [ctypes.POINTER(P), P, I, I]),
        "cnn_destroy": (I, [P]),
        "cnn_num_params": (ctypes.c_longlong, [P]),
        "cnn_set_weights": (I, [P, P, ctypes.c_longlong]),
        "cnn_get_weights": (I, [P, P, ctypes.c_longlong]),
        "cnn_state_size": (ctypes.c_longlong, [P]),
        "cnn_get_state": (I, [P, P, ctypes.c_longlong, P]),
        "cnn_set_state": (I, [P, P, ctypes.c_longlong, P]),
        "cnn_set_norm": (I, [P, D, D, D, D]),
        "cnn_moments": (I, [P, P, P, D, PD]),
        "cnn_pack_input": (I, [P, P, D, P, P]),
        "cnn_conv": (I, [P, I, I, P, P, P]),
        "cnn_weight_grad": (I, [P, I, P, P, P]),
        "cnn_forward": (I, [P, P, D, P, P]),
        "cnn_train_step": (I, [P, P, D, P, P, ctypes.c_float, PD]),
        "cnn_set_adam": (I, [P, D, D, D]),
        "cnn_adam_step": (I, [P, P, ctypes.c_float]),
        "cnn_guess": (I, [P, P, D, P, PI, PD]),
        "sts_set_pc_factor": (I, [P, P]),
        "sts_apply_pc_factor": (I, [P, P, P]),
        "sts_pc_objective": (I, [P, D, P, PD, P]),
        "cnn_create_pc": (I, [ctypes.POINTER(P), P, I, I]),
        "cnn_pc_set_norm": (I, [P, D, D]),
        "cnn_pc_factor": (I, [P, P, D, PI]),
        "cnn_pc_train_step": (I, [P, P, D, P, ctypes.c_float, PD]),
        "cnn_pc_grad": (I, [P, P, D, P, P, PD]),
        "sts_set_profile": (I, [P, I]),
        "sts_profile_summary": (I, [P, ctypes.c_char_p, ctypes.c_longlong, I]),
        "sts_set_debug": (I, [P, I]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return ["sts_create", "sts_destroy", "sts_set_stream", "sts_last_error", "sts_num_cells",
            "sts_set_spitzer", "sts_set_isotropic", "sts_set_spitzer_f32", "sts_set_isotropic_f32",
            "sts_set_dirichlet", "sts_dt_euler", "apply_F", "rkl2_step", "rkl2_step_noalloc",
            "rkl_step", "apply_F_nonlinear", "rkl2_step_nonlinear", "sts_set_resistivity",
            "sts_resistivity_sizes", "apply_F_resistivity", "resistivity_dt_euler",
            "resistivity_be_pcg_solve", "be_pcg_solve",
            "sts_be_residual", "cnn_create", "cnn_destroy", "cnn_num_params", "cnn_set_weights",
            "cnn_get_weights", "cnn_state_size", "cnn_get_state", "cnn_set_state", "cnn_set_norm", "cnn_moments", "cnn_pack_input", "cnn_conv",
            "cnn_weight_grad", "cnn_forward", "cnn_train_step", "cnn_set_adam", "cnn_adam_step",
            "cnn_guess", "sts_set_pc_factor", "sts_apply_pc_factor", "sts_pc_objective",
            "cnn_create_pc", "cnn_pc_set_norm", "cnn_pc_factor", "cnn_pc_train_step",
            "cnn_pc_grad", "sts_set_profile", "sts_profile_summary", "sts_set_debug"]


def _ptr(t: torch.Tensor | None, ncell: int, name: str, ncomp: int | None = 1,
         dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if ncomp is not None and t.numel() != ncell * ncomp:
        raise ValueError(f"{name} has {t.numel()} elements, expected {ncell * ncomp}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _d(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Context:
    """One grid + one operator (sts_ctx)."""

    def __init__(self, coord, f0, f1, f2, bc=SHELL_BC):
        lib = load()
        self._lib = lib
        a0, p0 = _d(f0)
        a1, p1 = _d(f1)
        a2, p2 = _d(f2)
        self.shape = (len(a0) - 1, len(a1) - 1, len(a2) - 1)
        self.ncell = self.shape[0] * self.shape[1] * self.shape[2]
        bcs = (ctypes.c_int * 6)(*bc)
        h = ctypes.c_void_p()
        st = lib.sts_create(ctypes.byref(h), int(coord), *self.shape, p0, p1, p2, bcs, _stream())
        if st != STS_OK:
            raise StsError(st, "sts_create failed (see stderr)")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sts_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, ok=(STS_OK,)):
        if st not in ok:
            raise StsError(st, self._lib.sts_last_error(self._h).decode())
        return st

    def _sync_stream(self):
        self._lib.sts_set_stream(self._h, _stream())

    def set_spitzer(self, T, kappa0, b0, b1, b2):
        self._sync_stream()
        n = self.ncell
        self._check(self._lib.sts_set_spitzer(self._h, _ptr(T, n, "T"), float(kappa0),
                                              _ptr(b0, n, "b0"), _ptr(b1, n, "b1"),
                                              _ptr(b2, n, "b2")))

    def set_isotropic(self, nu):
        self._sync_stream()
        self._check(self._lib.sts_set_isotropic(self._h, float(nu)))

    def set_spitzer_f32(self, T, kappa0, b0, b1, b2):
        """Precision form: T, b are float32 device tensors."""
        self._sync_stream()
        n, f = self.ncell, torch.float32
        self._check(self._lib.sts_set_spitzer_f32(
            self._h, _ptr(T, n, "T", dtype=f), float(kappa0), _ptr(b0, n, "b0", dtype=f),
            _ptr(b1, n, "b1", dtype=f), _ptr(b2, n, "b2", dtype=f)))

    def set_isotropic_f32(self, nu):
        self._sync_stream()
        self._check(self._lib.sts_set_isotropic_f32(self._h, float(nu)))

    def set_dirichlet(self, side, values=None, value=0.0):
        self._sync_stream()
        nb = self.shape[1] * self.shape[2]
        self._check(self._lib.sts_set_dirichlet(self._h, int(side), _ptr(values, nb, "values"),
                                                float(value)))

    def dt_euler(self) -> float:
        self._sync_stream()
        out = ctypes.c_double()
        self._check(self._lib.sts_dt_euler(self._h, ctypes.byref(out)))
        return out.value

    def _ncomp(self, u):
        nc = u.numel() // self.ncell
        if nc * self.ncell != u.numel():
            raise ValueError("field size is not a multiple of the cell count")
        return nc

    def apply_F(self, u, out=None):
        self._sync_stream()
        nc = self._ncomp(u)
        if out is None:
            out = torch.empty_like(u)
        self._check(self._lib.apply_F(self._h, _ptr(u, self.ncell, "u", nc),
                                      _ptr(out, self.ncell, "out", nc), nc))
        return out

    def rkl2_step(self, u, dt, s=0) -> int:
        self._sync_stream()
        nc = self._ncomp(u)
        used = ctypes.c_int()
        self._check(self._lib.rkl2_step(self._h, _ptr(u, self.ncell, "u", nc), nc, float(dt),
                                        int(s), ctypes.byref(used)))
        return used.value

    def rkl2_step_noalloc(self, u, dt, s=0) -> int:
        """rkl2_step with its stage buffers in the library's static device
        scratch (no device allocation; see include/sts.h for the limits)."""
        self._sync_stream()
        nc = self._ncomp(u)
        used = ctypes.c_int()
        self._check(self._lib.rkl2_step_noalloc(self._h, _ptr(u, self.ncell, "u", nc), nc,
                                                float(dt), int(s), ctypes.byref(used)))
        return used.value

    def rkl_step(self, u, dt, scheme=2, extra=0, odd=False, nsub=1, euler_fraction=0.0,
                 euler_cfl=0.5) -> int:
        """Super-step variants (see include/sts.h); returns the operator evaluations."""
        self._sync_stream()
        nc = self._ncomp(u)
        n = ctypes.c_int()
        self._check(self._lib.rkl_step(self._h, _ptr(u, self.ncell, "u", nc), nc, float(dt),
                                       int(scheme), int(extra), int(bool(odd)), int(nsub),
                                       float(euler_fraction), float(euler_cfl), ctypes.byref(n)))
        return n.value

    def apply_F_nonlinear(self, u, kappa0, b0, b1, b2, out=None):
        """F(u) with kappa = kappa0 max(u, 0)^{5/2} taken from u (no lagging)."""
        self._sync_stream()
        n = self.ncell
        if out is None:
            out = torch.empty_like(u)
        self._check(self._lib.apply_F_nonlinear(
            self._h, _ptr(u, n, "u"), _ptr(out, n, "out"), float(kappa0), _ptr(b0, n, "b0"),
            _ptr(b1, n, "b1"), _ptr(b2, n, "b2")))
        return out

    def rkl2_step_nonlinear(self, u, dt, kappa0, b0, b1, b2, s=0) -> int:
        """RKL2 super-step with kappa taken from every stage value; returns s."""
        self._sync_stream()
        n = self.ncell
        used = ctypes.c_int()
        self._check(self._lib.rkl2_step_nonlinear(
            self._h, _ptr(u, n, "u"), float(dt), float(kappa0), _ptr(b0, n, "b0"),
            _ptr(b1, n, "b1"), _ptr(b2, n, "b2"), int(s), ctypes.byref(used)))
        return used.value

    def set_resistivity(self, eta):
        """Resistive diffusion of A on cell edges (see include/sts.h)."""
        self._sync_stream()
        self._check(self._lib.sts_set_resistivity(self._h, float(eta)))

    def resistivity_sizes(self):
        out = (ctypes.c_longlong * 3)()
        self._check(self._lib.sts_resistivity_sizes(self._h, out))
        return tuple(int(v) for v in out)

    def _nedge(self):
        return sum(self.resistivity_sizes())

    def apply_F_resistivity(self, E, out=None):
        self._sync_stream()
        n = self._nedge()
        if out is None:
            out = torch.empty_like(E)
        self._check(self._lib.apply_F_resistivity(self._h, _ptr(E, n, "E"), _ptr(out, n, "out")))
        return out

    def resistivity_dt_euler(self) -> float:
        self._sync_stream()
        v = ctypes.c_double()
        self._check(self._lib.resistivity_dt_euler(self._h, ctypes.byref(v)))
        return v.value

    def resistivity_be_pcg_solve(self, E_n, E, dt, rtol=1e-8, maxit=10000,
                                 allow_not_converged=False):
        self._sync_stream()
        n = self._nedge()
        it = ctypes.c_int()
        rel = ctypes.c_double()
        st = self._lib.resistivity_be_pcg_solve(self._h, _ptr(E_n, n, "E_n"), _ptr(E, n, "E"),
                                                float(dt), float(rtol), int(maxit),
                                                ctypes.byref(it), ctypes.byref(rel))
        self._check(st, (STS_OK, STS_NOT_CONVERGED) if allow_not_converged else (STS_OK,))
        return it.value, rel.value, st

    def be_pcg_solve(self, u_n, x, dt, pc=PC_JACOBI, block=(8, 8, 8), rtol=1e-8, maxit=10000,
                     allow_not_converged=False):
        self._sync_stream()
        n = self.ncell
        blk = (ctypes.c_int * 3)(*block)
        it = ctypes.c_int()
        rel = ctypes.c_double()
        st = self._lib.be_pcg_solve(self._h, _ptr(u_n, n, "u_n"), _ptr(x, n, "x"), float(dt),
                                    int(pc), blk, float(rtol), int(maxit), ctypes.byref(it),
                                    ctypes.byref(rel))
        self._check(st, (STS_OK, STS_NOT_CONVERGED) if allow_not_converged else (STS_OK,))
        return it.value, rel.value, st

    def set_profile(self, on=True):
        self._check(self._lib.sts_set_profile(self._h, 1 if on else 0))

    def profile_summary(self, reset=True, cap=1 << 16):
        """Per-launcher timing table: {name: (calls, total_ms, avg_us, min_us, max_us)}."""
        self._sync_stream()
        buf = ctypes.create_string_buffer(cap)
        self._check(self._lib.sts_profile_summary(self._h, buf, cap, 1 if reset else 0))
        out = {}
        for line in buf.value.decode().splitlines()[1:]:
            f = line.split()
            out[f[5]] = (int(f[0]), float(f[1]), float(f[2]), float(f[3]), float(f[4]))
        return out

    def set_debug(self, flags):
        self._check(self._lib.sts_set_debug(self._h, int(flags)))

    def set_pc_factor(self, g):
        """The STS_PC_FACTOR factor from a device FP32 tensor [4, n0, n1, n2] (stored rounded
        to BF16)."""
        self._sync_stream()
        self._check(self._lib.sts_set_pc_factor(self._h, _ptr(g, self.ncell, "g", 4,
                                                              dtype=torch.float32)))

    def apply_pc_factor(self, r, out=None):
        """z = G (G^T r) with the context's factor."""
        self._sync_stream()
        if out is None:
            out = torch.empty_like(r)
        self._check(self._lib.sts_apply_pc_factor(self._h, _ptr(r, self.ncell, "r"),
                                                  _ptr(out, self.ncell, "out")))
        return out

    def pc_objective(self, dt, z, want_grad=True):
        """(L, dL/dG as a device FP64 tensor [4, n0, n1, n2] or None)."""
        self._sync_stream()
        loss = ctypes.c_double()
        dg = torch.empty((4,) + tuple(z.shape), dtype=torch.float64, device=z.device) \
            if want_grad else None
        self._check(self._lib.sts_pc_objective(self._h, float(dt), _ptr(z, self.ncell, "z"),
                                               ctypes.byref(loss),
                                               _ptr(dg, self.ncell, "dg", 4)))
        return loss.value, dg

    def be_residual(self, u_n, x, dt) -> float:
        self._sync_stream()
        n = self.ncell
        rel = ctypes.c_double()
        self._check(self._lib.sts_be_residual(self._h, _ptr(u_n, n, "u_n"), _ptr(x, n, "x"),
                                              float(dt), ctypes.byref(rel)))
        return rel.value


CNN_RELU, CNN_LINEAR, CNN_INPUT_GRAD, CNN_F32, CNN_INPUT_GRAD_F32, CNN_OUT4 = 0, 1, 2, 3, 4, 5
CNN_PADDED_PARAMS = 16 * 16 * 27 + 16  # per layer, cnn_weight_grad's output


class Cnn:
    """Learned initial guess (sts_cnn): a 3D CNN on the context's grid.
    Activations are bfloat16 tensors of shape [cells, 16]."""

    _create = "cnn_create"

    def __init__(self, ctx: Context, layers=4, channels=16):
        self.ctx = ctx
        self._lib = ctx._lib
        h = ctypes.c_void_p()
        ctx._sync_stream()
        ctx._check(getattr(self._lib, self._create)(ctypes.byref(h), ctx._h, int(layers),
                                                    int(channels)))
        self._h = h
        self.layers = layers
        self.nparam = self._lib.cnn_num_params(h)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        return self.ctx._check(st)

    def _act(self, t, name, dtype=torch.bfloat16, width=16):
        return _ptr(t, self.ctx.ncell, name, width, dtype=dtype)

    def set_weights(self, w):
        import numpy as np
        self.ctx._sync_stream()
        a = np.ascontiguousarray(w, dtype=np.float32)
        self._chk(self._lib.cnn_set_weights(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size))

    def get_weights(self):
        import numpy as np
        self.ctx._sync_stream()
        a = np.empty(self.nparam, np.float32)
        self._chk(self._lib.cnn_get_weights(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size))
        return a

    def get_state(self):
        """The training state: {"buf": FP32 [3 x layers x 6928] (master parameters, Adam
        moments), "meta": FP64 [8] (step, four scalings, beta1, beta2, eps)}."""
        import numpy as np
        self.ctx._sync_stream()
        n = self._lib.cnn_state_size(self._h)
        buf = np.empty(n, np.float32)
        meta = np.empty(8, np.float64)
        self._chk(self._lib.cnn_get_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), n,
                                          meta.ctypes.data_as(ctypes.c_void_p)))
        return {"buf": buf, "meta": meta}

    def set_state(self, state):
        import numpy as np
        self.ctx._sync_stream()
        buf = np.ascontiguousarray(state["buf"], dtype=np.float32)
        meta = np.ascontiguousarray(state["meta"], dtype=np.float64)
        if meta.size != 8:
            raise ValueError("meta must hold 8 values")
        self._chk(self._lib.cnn_set_state(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size,
                                          meta.ctypes.data_as(ctypes.c_void_p)))

    def set_norm(self, rhs_scale, T_shift, T_scale, delta_scale):
        self._chk(self._lib.cnn_set_norm(self._h, float(rhs_scale), float(T_shift),
                                         float(T_scale), float(delta_scale)))

    def moments(self, x, y=None, scale=1.0):
        self.ctx._sync_stream()
        n = self.ctx.ncell
        out = (ctypes.c_double * 2)()
        self._chk(self._lib.cnn_moments(self._h, _ptr(x, n, "x"), _ptr(y, n, "y"), float(scale),
                                        out))
        return out[0], out[1]

    def pack_input(self, F_prev, dt, T_prev, out=None):
        self.ctx._sync_stream()
        n = self.ctx.ncell
        if out is None:
            out = torch.empty((n, 16), dtype=torch.bfloat16, device=T_prev.device)
        self._chk(self._lib.cnn_pack_input(self._h, _ptr(F_prev, n, "F_prev"), float(dt),
                                           _ptr(T_prev, n, "T_prev"), self._act(out, "out")))
        return out

    def conv(self, layer, kind, x, mask=None, out=None):
        self.ctx._sync_stream()
        n = self.ctx.ncell
        if out is None:
            if kind in (CNN_RELU, CNN_INPUT_GRAD):
                out = torch.empty((n, 16), dtype=torch.bfloat16, device=x.device)
            elif kind == CNN_LINEAR:
                out = torch.empty(n, dtype=torch.float32, device=x.device)
            elif kind == CNN_OUT4:
                out = torch.empty((n, 4), dtype=torch.float32, device=x.device)
            else:
                out = torch.empty((n, 16), dtype=torch.float32, device=x.device)
        if kind in (CNN_RELU, CNN_INPUT_GRAD):
            po = self._act(out, "out")
        elif kind == CNN_LINEAR:
            po = _ptr(out, n, "out", 1, dtype=torch.float32)
        elif kind == CNN_OUT4:
            po = _ptr(out, n, "out", 4, dtype=torch.float32)
        else:
            po = _ptr(out, n, "out", 16, dtype=torch.float32)
        self._chk(self._lib.cnn_conv(self._h, int(layer), int(kind), self._act(x, "x"),
                                     self._act(mask, "mask"), po))
        return out

    def weight_grad(self, layer, act, dout, out=None):
        self.ctx._sync_stream()
        if out is None:
            out = torch.empty(CNN_PADDED_PARAMS, dtype=torch.float32, device=act.device)
        self._chk(self._lib.cnn_weight_grad(self._h, int(layer), self._act(act, "act"),
                                            self._act(dout, "dout"),
                                            _ptr(out, CNN_PADDED_PARAMS, "out", 1,
                                                 dtype=torch.float32)))
        return out

    def forward(self, F_prev, dt, T_prev, x0=None):
        self.ctx._sync_stream()
        n = self.ctx.ncell
        if x0 is None:
            x0 = torch.empty_like(T_prev)
        self._chk(self._lib.cnn_forward(self._h, _ptr(F_prev, n, "F_prev"), float(dt),
                                        _ptr(T_prev, n, "T_prev"), _ptr(x0, n, "x0")))
        return x0

    def train_step(self, F_prev, dt, T_prev, x_star, lr, want_loss=True):
        self.ctx._sync_stream()
        n = self.ctx.ncell
        loss = ctypes.c_double()
        self._chk(self._lib.cnn_train_step(self._h, _ptr(F_prev, n, "F_prev"), float(dt),
                                           _ptr(T_prev, n, "T_prev"), _ptr(x_star, n, "x_star"),
                                           float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def set_adam(self, beta1=0.9, beta2=0.999, eps=1e-8):
        self._chk(self._lib.cnn_set_adam(self._h, float(beta1), float(beta2), float(eps)))

    def adam_step(self, grad, lr):
        """One Adam step with a device FP32 gradient of layers * 6928 values."""
        self.ctx._sync_stream()
        n = self.layers * CNN_PADDED_PARAMS
        self._chk(self._lib.cnn_adam_step(self._h, _ptr(grad, n, "grad", 1, dtype=torch.float32),
                                          float(lr)))

    def guess(self, T_prev, dt, x0=None):
        """Returns (x0, used_net, (relres_net, relres_prev))."""
        self.ctx._sync_stream()
        n = self.ctx.ncell
        if x0 is None:
            x0 = torch.empty_like(T_prev)
        used = ctypes.c_int()
        rel = (ctypes.c_double * 2)()
        self._chk(self._lib.cnn_guess(self._h, _ptr(T_prev, n, "T_prev"), float(dt),
                                      _ptr(x0, n, "x0"), ctypes.byref(used), rel))
        return x0, bool(used.value), (rel[0], rel[1])


class CnnPC(Cnn):
    """The factor network (cnn_create_pc): 4 output channels giving the
    factor G of the STS_PC_FACTOR preconditioner M^-1 = G G^T."""

    _create = "cnn_create_pc"

    def set_norm(self, T_shift, T_scale):
        self._chk(self._lib.cnn_pc_set_norm(self._h, float(T_shift), float(T_scale)))

    def factor(self, T, dt) -> bool:
        """The network's factor for the context's operator at dt, set as the
        context's factor; False if it fell back to point Jacobi."""
        self.ctx._sync_stream()
        used = ctypes.c_int()
        self._chk(self._lib.cnn_pc_factor(self._h, _ptr(T, self.ctx.ncell, "T"), float(dt),
                                          ctypes.byref(used)))
        return bool(used.value)

    def grad(self, T, dt, z, out=None):
        """(loss, gradient as a device FP32 tensor of layers * 6928 values)."""
        self.ctx._sync_stream()
        n = self.ctx.ncell
        if out is None:
            out = torch.empty(self.layers * CNN_PADDED_PARAMS, dtype=torch.float32,
                              device=T.device)
        loss = ctypes.c_double()
        self._chk(self._lib.cnn_pc_grad(self._h, _ptr(T, n, "T"), float(dt), _ptr(z, n, "z"),
                                        _ptr(out, self.layers * CNN_PADDED_PARAMS, "grad", 1,
                                             dtype=torch.float32), ctypes.byref(loss)))
        return loss.value, out

    def train_step(self, T, dt, z, lr, want_loss=True):
        self.ctx._sync_stream()
        n = self.ctx.ncell
        loss = ctypes.c_double()
        self._chk(self._lib.cnn_pc_train_step(self._h, _ptr(T, n, "T"), float(dt),
                                              _ptr(z, n, "z"), float(lr),
                                              ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None


# Module-level names of the C ABI (same names, Python arguments).
def sts_create(coord, f0, f1, f2, bc=SHELL_BC) -> Context:
    return Context(coord, f0, f1, f2, bc)


def sts_destroy(ctx: Context):
    ctx.close()


def sts_set_spitzer(ctx: Context, T, kappa0, b0, b1, b2):
    ctx.set_spitzer(T, kappa0, b0, b1, b2)


def sts_set_isotropic(ctx: Context, nu):
    ctx.set_isotropic(nu)


def sts_set_spitzer_f32(ctx: Context, T, kappa0, b0, b1, b2):
    ctx.set_spitzer_f32(T, kappa0, b0, b1, b2)


def sts_set_isotropic_f32(ctx: Context, nu):
    ctx.set_isotropic_f32(nu)


def sts_set_dirichlet(ctx: Context, side, values=None, value=0.0):
    ctx.set_dirichlet(side, values, value)


def sts_dt_euler(ctx: Context) -> float:
    return ctx.dt_euler()


def apply_F(ctx: Context, u, out=None):
    return ctx.apply_F(u, out)


def rkl2_step(ctx: Context, u, dt, s=0) -> int:
    return ctx.rkl2_step(u, dt, s)


def rkl2_step_noalloc(ctx: Context, u, dt, s=0) -> int:
    return ctx.rkl2_step_noalloc(u, dt, s)


def apply_F_nonlinear(ctx: Context, u, kappa0, b0, b1, b2, out=None):
    return ctx.apply_F_nonlinear(u, kappa0, b0, b1, b2, out)


def rkl2_step_nonlinear(ctx: Context, u, dt, kappa0, b0, b1, b2, s=0) -> int:
    return ctx.rkl2_step_nonlinear(u, dt, kappa0, b0, b1, b2, s)


def rkl_step(ctx: Context, u, dt, scheme=2, extra=0, odd=False, nsub=1, euler_fraction=0.0,
             euler_cfl=0.5) -> int:
    return ctx.rkl_step(u, dt, scheme, extra, odd, nsub, euler_fraction, euler_cfl)


def be_pcg_solve(ctx: Context, u_n, x, dt, pc=PC_JACOBI, block=(8, 8, 8), rtol=1e-8,
                 maxit=10000, allow_not_converged=False):
    return ctx.be_pcg_solve(u_n, x, dt, pc, block, rtol, maxit, allow_not_converged)


def sts_be_residual(ctx: Context, u_n, x, dt) -> float:
    return ctx.be_residual(u_n, x, dt)


def cnn_create(ctx: Context, layers=4, channels=16) -> Cnn:
    return Cnn(ctx, layers, channels)


def cnn_create_pc(ctx: Context, layers=4, channels=16) -> CnnPC:
    return CnnPC(ctx, layers, channels)


def cnn_pc_set_norm(net: CnnPC, T_shift, T_scale):
    net.set_norm(T_shift, T_scale)


def cnn_pc_factor(net: CnnPC, T, dt) -> bool:
    return net.factor(T, dt)


def cnn_pc_train_step(net: CnnPC, T, dt, z, lr, want_loss=True):
    return net.train_step(T, dt, z, lr, want_loss)


def cnn_pc_grad(net: CnnPC, T, dt, z, out=None):
    return net.grad(T, dt, z, out)


def sts_set_profile(ctx: Context, on=True):
    ctx.set_profile(on)


def sts_profile_summary(ctx: Context, reset=True):
    return ctx.profile_summary(reset)


def sts_set_debug(ctx: Context, flags):
    ctx.set_debug(flags)


def sts_set_pc_factor(ctx: Context, g):
    ctx.set_pc_factor(g)


def sts_apply_pc_factor(ctx: Context, r, out=None):
    return ctx.apply_pc_factor(r, out)


def sts_pc_objective(ctx: Context, dt, z, want_grad=True):
    return ctx.pc_objective(dt, z, want_grad)


def cnn_destroy(net: Cnn):
    net.close()


def cnn_num_params(net: Cnn) -> int:
    return net.nparam


def cnn_set_weights(net: Cnn, w):
    net.set_weights(w)


def cnn_get_weights(net: Cnn):
    return net.get_weights()


def cnn_set_norm(net: Cnn, rhs_scale, T_shift, T_scale, delta_scale):
    net.set_norm(rhs_scale, T_shift, T_scale, delta_scale)


def cnn_moments(net: Cnn, x, y=None, scale=1.0):
    return net.moments(x, y, scale)


def cnn_pack_input(net: Cnn, F_prev, dt, T_prev, out=None):
    return net.pack_input(F_prev, dt, T_prev, out)


def cnn_conv(net: Cnn, layer, kind, x, mask=None, out=None):
    return net.conv(layer, kind, x, mask, out)


def cnn_weight_grad(net: Cnn, layer, act, dout, out=None):
    return net.weight_grad(layer, act, dout, out)


def cnn_forward(net: Cnn, F_prev, dt, T_prev, x0=None):
    return net.forward(F_prev, dt, T_prev, x0)


def cnn_train_step(net: Cnn, F_prev, dt, T_prev, x_star, lr, want_loss=True):
    return net.train_step(F_prev, dt, T_prev, x_star, lr, want_loss)


def cnn_set_adam(net: Cnn, beta1=0.9, beta2=0.999, eps=1e-8):
    return net.set_adam(beta1, beta2, eps)


def cnn_adam_step(net: Cnn, grad, lr):
    return net.adam_step(grad, lr)


def cnn_guess(net: Cnn, T_prev, dt, x0=None):
    return net.guess(T_prev, dt, x0)
