"""tgexp: split exponential Euler on MI355X (gfx950) -- Python binding.

Thin ctypes layer over ``libtgexp.so`` (C interface in ``include/tgexp.h``).
It only marshals arguments: every step of the method runs in the HIP
library.  PyTorch supplies device memory and streams.  Importing this
package raises if the compiled library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtgexp.so")

GEOMETRY = {"disk": 0, "sphere": 1, "ball": 2, "cylinder": 3, "disk_lambda": 4}
PRECISION = {"fp64": 0, "fp32": 1, "bf16x2": 2, "bf16x3": 3}
REACTION = {"none": 0, "schnakenberg": 1, "ais3": 2, "schnakenberg_scaled": 3, "linear": 4, "dib": 5}
APPLY = {"F": 0, "diffusion": 1, "reaction": 2}
NDIM = {"disk": 2, "sphere": 2, "ball": 3, "cylinder": 3, "disk_lambda": 2}
ROUTES = {"fused": 0, "generic": 1, "fused_stencil_apart": 2, "per_slice": 3, "resident": 4}

_c_int = ctypes.c_int32
_c_i64 = ctypes.c_int64
_p = ctypes.c_void_p
_pd = ctypes.POINTER(ctypes.c_double)
_pi = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)

_SIGNATURES = {
    "tg_last_error": (ctypes.c_char_p, []),
    "tg_version": (ctypes.c_int, []),
    "tg_grid_create": (ctypes.c_int, [_c_int, _pi, _pd, ctypes.POINTER(_p)]),
    "tg_grid_destroy": (ctypes.c_int, [_p]),
    "tg_grid_dims": (ctypes.c_int, [_p, _pi, _pi]),
    "tg_grid_coords": (ctypes.c_int, [_p, _c_int, _pd]),
    "tg_grid_operator": (ctypes.c_int, [_p, _c_int, _pd, _pd, _pd]),
    "tg_grid_eig": (ctypes.c_int, [_p, _c_int, _pd, _pd, _pd]),
    "tg_grid_phi1": (ctypes.c_int, [_p, _c_int, ctypes.c_double, _pd]),
    "tg_plan_create": (ctypes.c_int, [_p, _c_int, _c_int, _pd, _c_int, _c_int, _pd, _pd,
                                      ctypes.c_double, _c_int, ctypes.POINTER(_p)]),
    "tg_plan_destroy": (ctypes.c_int, [_p]),
    "tg_plan_state_size": (ctypes.c_int, [_p, _pi64, _pi]),
    "tg_plan_reference": (ctypes.c_int, [_p, _pd]),
    "tg_step": (ctypes.c_int, [_p, _p, _p]),
    "tg_run": (ctypes.c_int, [_p, _p, _c_i64, _p]),
    "tg_run_history": (ctypes.c_int, [_p, _p, _c_i64, _p, ctypes.c_int32, _p]),
    "tg_run_prepare": (ctypes.c_int, [_p, _p]),
    "tg_step_diag_noalloc": (ctypes.c_int, [_p, _p, _p, _p]),
    "tg_step_diag": (ctypes.c_int, [_p, _p, _p, _p]),
    "tg_sync_status": (ctypes.c_int, [_p, _p]),
    "tg_coupled_step": (ctypes.c_int, [_p, _p, _p, _p, _pd, _p]),
    "tg_coupled_run": (ctypes.c_int, [_p, _p, _p, _p, _pd, _c_i64, _p]),
    "tg_run_diag": (ctypes.c_int, [_p, _p, _c_i64, _c_int, _p, _p]),
    "tg_apply_operator": (ctypes.c_int, [_p, _p, _p, _c_int, _p]),
    "tg_apply_split_phi1": (ctypes.c_int, [_p, _p, _p, _p]),
    "tg_plan_chain": (ctypes.c_int, [_p, _pi, _pi, _pd]),
    "tg_apply_chain_op": (ctypes.c_int, [_p, _c_int, _p, _p, _p]),
    "tg_plan_set_route": (ctypes.c_int, [_p, _c_int]),
    "tg_adjoint_step": (ctypes.c_int, [_p, _p, _p, _p, _p]),
    "tg_plan_route": (ctypes.c_int, [_p, _pi]),
    "tg_group_run": (ctypes.c_int, [ctypes.POINTER(_p), _c_int, ctypes.POINTER(_p), _c_i64, _p]),
    "tg_group_info": (ctypes.c_int, [ctypes.POINTER(_p), _c_int, ctypes.POINTER(_p), _pi, _pi]),
    "tg_plan_autotune": (ctypes.c_int, [_p, _p, _c_int, _p, _pd]),
    "tg_plan_tiles": (ctypes.c_int, [_p, _pi, _pi]),
    "tg_run_timed": (ctypes.c_int, [_p, _p, _c_i64, _p, _c_int, _pi, _pd]),
    "tg_plan_set_tiles": (ctypes.c_int, [_p, _c_int, _pi]),
    "tg_group_autotune": (ctypes.c_int, [ctypes.POINTER(_p), _c_int, ctypes.POINTER(_p), _c_int, _p, _pd]),
}

_lib = None


class TGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tgexp error {code}: {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2604_11558_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != 0:
        raise TGError(rc, lib().tg_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_pd)


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


class Grid:
    """Grid and 1D operators of one geometry (host, FP64)."""

    def __init__(self, geometry: str, n: Sequence[int], extent=(1.0, 1.0)):
        self.geometry = geometry
        self.n = tuple(int(x) for x in n)
        if len(self.n) != NDIM[geometry]:
            raise ValueError(f"{geometry} needs {NDIM[geometry]} sizes")
        h = _p()
        narr = (ctypes.c_int32 * 3)(*(list(self.n) + [1] * (3 - len(self.n))))
        ext = (ctypes.c_double * 2)(*extent)
        _check(lib().tg_grid_create(GEOMETRY[geometry], narr, ext, ctypes.byref(h)))
        self._h = h
        self.extent = tuple(float(e) for e in extent)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.tg_grid_destroy(h)
            self._h = None

    def coords(self, mode: int) -> np.ndarray:
        out = np.empty(self.n[mode - 1])
        _check(lib().tg_grid_coords(self._h, mode, _dptr(out)))
        return out

    def operator(self, mode: int):
        n = self.n[mode - 1]
        lo, dg, up = np.empty(n), np.empty(n), np.empty(n)
        _check(lib().tg_grid_operator(self._h, mode, _dptr(lo), _dptr(dg), _dptr(up)))
        return lo, dg, up

    def dense_operator(self, mode: int) -> np.ndarray:
        lo, dg, up = self.operator(mode)
        n = dg.size
        A = np.diag(dg) + np.diag(up[:-1], 1) + np.diag(lo[1:], -1)
        A[0, n - 1] += lo[0]
        A[n - 1, 0] += up[n - 1]
        return A

    def eig(self, mode: int):
        n = self.n[mode - 1]
        lam, V, Vi = np.empty(n), np.empty((n, n)), np.empty((n, n))
        _check(lib().tg_grid_eig(self._h, mode, _dptr(lam), _dptr(V), _dptr(Vi)))
        return lam, V, Vi

    def phi1(self, mode: int, c: float) -> np.ndarray:
        n = self.n[mode - 1]
        out = np.empty((n, n))
        _check(lib().tg_grid_phi1(self._h, mode, float(c), _dptr(out)))
        return out


class Plan:
    """Split exponential Euler plan: factors on the device, step / run.

    ``diff``: [batch][n_species] (or [n_species], broadcast); ``params``:
    [batch][n_params] (or [n_params]).  The state is a device tensor of
    shape ``state_shape`` holding deviations from ``reference``.
    """

    def __init__(self, grid: Grid, diff, reaction: str = "schnakenberg", params=(),
                 tau: float = 1e-2, precision: str = "fp64", batch: int = 1, w_ref=None):
        self.grid = grid
        diff = np.atleast_2d(np.asarray(diff, dtype=np.float64))
        if diff.shape[0] == 1 and batch > 1:
            diff = np.repeat(diff, batch, axis=0)
        self.batch = batch
        self.n_species = diff.shape[1]
        params = np.asarray(params, dtype=np.float64)
        if params.ndim == 1:
            params = np.repeat(params[None, :], batch, axis=0) if params.size else np.zeros((batch, 0))
        self.precision = precision
        self.tau = float(tau)
        self.reaction = reaction
        diff = np.ascontiguousarray(diff)
        params = np.ascontiguousarray(params)
        wref = None if w_ref is None else np.ascontiguousarray(np.broadcast_to(
            np.asarray(w_ref, dtype=np.float64), (batch, self.n_species)))
        h = _p()
        _check(lib().tg_plan_create(grid._h, self.n_species, batch, _dptr(diff), REACTION[reaction],
                                    params.shape[1], _dptr(params) if params.size else None,
                                    _dptr(wref) if wref is not None else None, self.tau,
                                    PRECISION[precision], ctypes.byref(h)))
        self._h = h
        elems, esize = ctypes.c_int64(), ctypes.c_int32()
        _check(lib().tg_plan_state_size(h, ctypes.byref(elems), ctypes.byref(esize)))
        self.state_elems = elems.value
        self.elem_bytes = esize.value
        ref = np.empty((batch, self.n_species))
        _check(lib().tg_plan_reference(h, _dptr(ref)))
        self.reference = ref

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.tg_plan_destroy(h)
            self._h = None

    @property
    def state_shape(self):
        return (self.batch, self.n_species) + tuple(reversed(self.grid.n))

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.elem_bytes == 8 else torch.float32

    def _check_tensor(self, t):
        if not t.is_cuda or not t.is_contiguous() or t.dtype != self.dtype or t.numel() != self.state_elems:
            raise ValueError(f"expected contiguous {self.dtype} device tensor of {self.state_elems} elements")

    def state_from_deviation(self, dev: np.ndarray):
        """Device state tensor from a host deviation array (any of the state shapes)."""
        import torch
        arr = np.asarray(dev, dtype=np.float64).reshape(self.state_shape)
        return torch.from_numpy(arr).to(device="cuda", dtype=self.dtype).contiguous()

    def step(self, state, stream=None):
        self._check_tensor(state)
        _check(lib().tg_step(self._h, state.data_ptr(), _stream_ptr(stream)))

    def run(self, state, n_steps: int, stream=None):
        self._check_tensor(state)
        _check(lib().tg_run(self._h, state.data_ptr(), int(n_steps), _stream_ptr(stream)))

    def run_history(self, state, n_steps: int, history, stream=None):
        """``n_steps`` steps keeping the state before each in ``history[k]``
        (a device tensor of shape (n_steps,) + state shape, in the plan's
        dtype, or float64 for an FP32-storage plan: the values widened)."""
        import torch
        self._check_tensor(state)
        fp64 = history.dtype == torch.float64 and self.dtype != torch.float64
        if (not history.is_cuda or not history.is_contiguous() or (history.dtype != self.dtype and not fp64)
                or tuple(history.shape) != (int(n_steps),) + tuple(state.shape)):
            raise ValueError("history must be a contiguous device tensor of shape (n_steps,) + state shape "
                             "in the plan's dtype or float64")
        _check(lib().tg_run_history(self._h, state.data_ptr(), int(n_steps), history.data_ptr(), int(fp64),
                                    _stream_ptr(stream)))

    def prepare_run(self, state):
        """Capture the graphs ``run`` replays on this state (no steps run)."""
        self._check_tensor(state)
        _check(lib().tg_run_prepare(self._h, state.data_ptr()))

    def sync_status(self, stream=None):
        """Synchronise the stream; raise TGError if a step wrote a non-finite value."""
        _check(lib().tg_sync_status(self._h, _stream_ptr(stream)))

    def step_diag(self, state, stream=None):
        """One step; returns a [batch, n_species, 2] float64 device tensor of
        (integral mean, L2 norm of the increment)."""
        self._check_tensor(state)
        import torch
        out = torch.empty((self.batch, self.n_species, 2), dtype=torch.float64, device=state.device)
        _check(lib().tg_step_diag(self._h, state.data_ptr(), out.data_ptr(), _stream_ptr(stream)))
        return out

    def step_diag_noalloc(self, state, out, stream=None):
        """``step_diag`` into a caller-given [batch, n_species, 2] float64 device
        tensor, with the partial sums in the library's static scratch (the call
        allocates nothing)."""
        self._check_tensor(state)
        import torch
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() \
                or out.numel() != 2 * self.batch * self.n_species:
            raise ValueError("out must be a contiguous cuda float64 tensor of 2 * batch * n_species entries")
        _check(lib().tg_step_diag_noalloc(self._h, state.data_ptr(), out.data_ptr(), _stream_ptr(stream)))

    def run_diag(self, state, n_steps: int, every: int = 1, stream=None):
        """``n_steps`` steps; the indicators of steps every, 2 every, ... as a
        [n_steps // every, batch, n_species, 2] float64 device tensor."""
        self._check_tensor(state)
        import torch
        out = torch.empty((int(n_steps) // int(every), self.batch, self.n_species, 2), dtype=torch.float64,
                          device=state.device)
        _check(lib().tg_run_diag(self._h, state.data_ptr(), int(n_steps), int(every), out.data_ptr(),
                                 _stream_ptr(stream)))
        return out

    def run_timed(self, state, n_steps: int, stream=None):
        """``n_steps`` direct-launch steps; average microseconds of each launch of a step."""
        self._check_tensor(state)
        n = ctypes.c_int32()
        us = (ctypes.c_double * 32)()
        _check(lib().tg_run_timed(self._h, state.data_ptr(), int(n_steps), _stream_ptr(stream), 32,
                                  ctypes.byref(n), us))
        return [us[i] for i in range(n.value)]

    def apply_operator(self, x, out, what: str = "F", stream=None):
        self._check_tensor(x)
        self._check_tensor(out)
        _check(lib().tg_apply_operator(self._h, x.data_ptr(), out.data_ptr(), APPLY[what],
                                       _stream_ptr(stream)))

    def set_route(self, route: str):
        """'fused' (default), 'fused_stencil_apart', 'generic', 'per_slice'
        (ball and cylinder: the scaled mode by per-slice dense factors) or
        'resident' (disk: one workgroup per instance runs many steps with the
        states in LDS)."""
        _check(lib().tg_plan_set_route(self._h, ROUTES[route]))

    @property
    def route(self) -> str:
        r = ctypes.c_int32()
        _check(lib().tg_plan_route(self._h, ctypes.byref(r)))
        return {v: k for k, v in ROUTES.items()}[r.value]

    def chain(self):
        """[(mode, flops)] of each launch of the active route's split chain."""
        n = ctypes.c_int32()
        modes = (ctypes.c_int32 * 16)()
        flops = (ctypes.c_double * 16)()
        _check(lib().tg_plan_chain(self._h, ctypes.byref(n), modes, flops))
        return [(modes[i], flops[i]) for i in range(n.value)]

    def chain_modes(self):
        return [m for m, _ in self.chain()]

    def apply_chain_op(self, op: int, x, out, stream=None):
        self._check_tensor(x)
        self._check_tensor(out)
        _check(lib().tg_apply_chain_op(self._h, int(op), x.data_ptr(), out.data_ptr(),
                                       _stream_ptr(stream)))

    def adjoint_step(self, state_n, lam, grad, stream=None):
        """lam <- dL/dW_n from dL/dW_{n+1}; grad (cuda float64, 2 * batch * species) accumulates."""
        import torch
        self._check_tensor(state_n)
        self._check_tensor(lam)
        if grad.dtype != torch.float64 or not grad.is_cuda or grad.numel() != 2 * self.batch * self.n_species:
            raise ValueError("grad must be a cuda float64 tensor of 2 * batch * n_species entries")
        _check(lib().tg_adjoint_step(self._h, state_n.data_ptr(), lam.data_ptr(), grad.data_ptr(),
                                     _stream_ptr(stream)))

    def split_phi1(self, x, out, stream=None):
        self._check_tensor(x)
        self._check_tensor(out)
        _check(lib().tg_apply_split_phi1(self._h, x.data_ptr(), out.data_ptr(), _stream_ptr(stream)))

    def tiles(self):
        """Tile width of each fused launch (columns / rows)."""
        n = ctypes.c_int32()
        t = (ctypes.c_int32 * 16)()
        _check(lib().tg_plan_tiles(self._h, ctypes.byref(n), t))
        return [t[i] for i in range(n.value)]

    def set_tiles(self, tiles):
        t = (ctypes.c_int32 * len(tiles))(*[int(v) for v in tiles])
        _check(lib().tg_plan_set_tiles(self._h, len(tiles), t))

    def autotune(self, state, iters: int = 20, stream=None) -> dict:
        """Time the launch configurations on a copy of ``state``; keep the fastest."""
        self._check_tensor(state)
        best = ctypes.c_double()
        _check(lib().tg_plan_autotune(self._h, state.data_ptr(), int(iters), _stream_ptr(stream),
                                      ctypes.byref(best)))
        return {"route": self.route, "tiles": self.tiles(), "us_per_step": best.value}


def _group_args(plans, states):
    if len(plans) != len(states):
        raise ValueError("one state per plan")
    for p, s in zip(plans, states):
        p._check_tensor(s)
    hp = (_p * len(plans))(*[p._h.value if isinstance(p._h, _p) else p._h for p in plans])
    hs = (_p * len(states))(*[s.data_ptr() for s in states])
    return hp, hs


def _coupling(coupling):
    """The five coupling constants (fewer are padded with zeros)."""
    c = np.zeros(5)
    v = np.asarray(coupling, dtype=np.float64).ravel()
    if v.size > 5:
        raise ValueError("at most five coupling constants")
    c[:v.size] = v
    return c, _dptr(c)


def coupled_step(bulk, surface, bulk_state, surface_state, coupling, stream=None):
    """One bulk-surface step: a ball plan + sphere plan with coupling =
    (zeta1, zeta2, zeta3, eta1, eta2) (Section 5.5), or a cylinder plan +
    bottom-disk plan with coupling = (alpha3, beta3) (Section 5.6)."""
    bulk._check_tensor(bulk_state)
    surface._check_tensor(surface_state)
    c, cp = _coupling(coupling)
    _check(lib().tg_coupled_step(bulk._h, surface._h, bulk_state.data_ptr(), surface_state.data_ptr(), cp,
                                 _stream_ptr(stream)))


def coupled_run(bulk, surface, bulk_state, surface_state, coupling, n_steps: int, stream=None):
    """``n_steps`` bulk-surface steps (graph replays)."""
    bulk._check_tensor(bulk_state)
    surface._check_tensor(surface_state)
    c, cp = _coupling(coupling)
    _check(lib().tg_coupled_run(bulk._h, surface._h, bulk_state.data_ptr(), surface_state.data_ptr(), cp,
                                int(n_steps), _stream_ptr(stream)))


def group_run(plans, states, n_steps: int, stream=None):
    """``n_steps`` steps of every plan; fused launches shared across plans when possible."""
    hp, hs = _group_args(plans, states)
    _check(lib().tg_group_run(hp, len(plans), hs, int(n_steps), _stream_ptr(stream)))


def group_autotune(plans, states, iters: int = 10, stream=None) -> float:
    """Pick the route (0 or 2) of a grouped run on copies of the states; microseconds per step."""
    hp, hs = _group_args(plans, states)
    best = ctypes.c_double()
    _check(lib().tg_group_autotune(hp, len(plans), hs, int(iters), _stream_ptr(stream), ctypes.byref(best)))
    return best.value


def group_info(plans, states) -> dict:
    hp, hs = _group_args(plans, states)
    g, n = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().tg_group_info(hp, len(plans), hs, ctypes.byref(g), ctypes.byref(n)))
    return {"grouped": bool(g.value), "launches_per_step": n.value}


__all__ = ["Grid", "Plan", "TGError", "lib", "group_run", "group_info", "group_autotune", "GEOMETRY", "PRECISION",
           "REACTION"]
