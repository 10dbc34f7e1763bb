"""Thin ctypes binding of libslhjb (include/slhjb.h): argument marshalling only.

Device arrays are torch tensors on the context's device; every step of the method runs in
the library's HIP kernels. The library is built in-tree by ``paper_1502_01629_amd.build``;
if it is missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import sys

# kept at import: during interpreter shutdown the sys module itself may be gone
_is_finalizing = sys.is_finalizing

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslhjb.so")

OK, NOT_CONVERGED, E_INVALID_ARG, E_UNSUPPORTED, E_HIP, E_NOMEM, E_NONFINITE = 0, 1, -1, -2, -3, -4, -5
DIFF_NONE, DIFF_ISO, DIFF_RANK1 = 0, 1, 2
SL2, SL3 = 0, 1
FREE, TARGET, OBSTACLE = 0, 1, 2


class SlhjbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"slhjb status {status}: {message}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("x_lo", ctypes.c_float),
        ("x_hi", ctypes.c_float),
        ("h", ctypes.c_float),
        ("lam", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("diffusion", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("n_controls", ctypes.c_int32),
        ("controls", ctypes.c_void_p),
        ("speed", ctypes.c_void_p),
        ("speed_const", ctypes.c_float),
        ("running_cost", ctypes.c_float),
        ("node_class", ctypes.c_void_p),
        ("target_value", ctypes.c_float),
        ("v_out", ctypes.c_float),
        ("drift", ctypes.c_void_p),
        ("running_cost_field", ctypes.c_void_p),
        ("control_cost", ctypes.c_void_p),
        ("eps_field", ctypes.c_void_p),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_int64),
        ("converged_sweep", ctypes.c_int64),
        ("node_updates", ctypes.c_int64),
        ("residual", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("sweep_seconds", ctypes.c_double),
        ("sweep_launches", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("kernel_path", ctypes.c_int32),
        ("halo", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("policy_updates", ctypes.c_int64),
        ("check_sweeps", ctypes.c_int64),
        ("check_seconds", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class TileOpts(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("label", ctypes.c_void_p),
        ("key_slack", ctypes.c_float),
        ("max_inner", ctypes.c_int32),
        ("tile_shape", ctypes.c_int32),
        ("persistent", ctypes.c_int32),
        ("max_workgroups", ctypes.c_int32),
        ("collect_kernel_time", ctypes.c_int32),
        ("policy_sweeps", ctypes.c_int32),
    ]


ORDER_NONE, ORDER_KEYS = 0, 1
# tile shapes of the active-tile solver (slhjb_tile_opts.tile_shape)
TILE_32x16, TILE_16x16, TILE_8x8_SPLIT4, TILE_16x16_SPLIT4, TILE_16x16_SPLIT2 = 0, 1, 2, 3, 4
PATCHY_TRANSMISSION, PATCHY_INDEPENDENT, PATCHY_STATIC = 0, 1, 2


class PatchyOpts(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32),
        ("n_patches", ctypes.c_int32),
        ("source_patch", ctypes.c_void_p),
        ("tol", ctypes.c_double),
        ("tol_coarse", ctypes.c_double),
        ("max_passes", ctypes.c_int64),
        ("key_window", ctypes.c_float),
        ("tile_shape", ctypes.c_int32),
        ("collect_kernel_time", ctypes.c_int32),
        ("policy_sweeps", ctypes.c_int32),
    ]


class PatchyStats(ctypes.Structure):
    _fields_ = [
        ("t_coarse", ctypes.c_double),
        ("t_upsample", ctypes.c_double),
        ("t_synthesize", ctypes.c_double),
        ("t_label", ctypes.c_double),
        ("t_solve", ctypes.c_double),
        ("t_total", ctypes.c_double),
        ("t_visit", ctypes.c_double),
        ("coarse_passes", ctypes.c_int64),
        ("node_updates_coarse", ctypes.c_int64),
        ("label_passes", ctypes.c_int64),
        ("passes", ctypes.c_int64),
        ("node_updates", ctypes.c_int64),
        ("policy_updates", ctypes.c_int64),
        ("residual", ctypes.c_double),
        ("status", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("check_sweeps", ctypes.c_int64),
        ("t_check_visit", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


MODE_TRANSMISSION, MODE_INDEPENDENT = 0, 1

# tile shapes of the batched solve (slhjb_batch_opts.tile_shapes)
BATCH_TILE_64x16, BATCH_TILE_64x8, BATCH_TILE_32x16, BATCH_TILE_32x8 = 0, 1, 2, 3
BATCH_TILE_SHAPES = {BATCH_TILE_64x16: (64, 16), BATCH_TILE_64x8: (64, 8), BATCH_TILE_32x16: (32, 16),
                     BATCH_TILE_32x8: (32, 8)}


class BatchOpts(ctypes.Structure):
    _fields_ = [
        ("check_every", ctypes.c_int32),
        ("batches_per_graph", ctypes.c_int32),
        ("tile_shapes", ctypes.c_void_p),
        ("max_workgroups", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


class BatchStats(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_int64),
        ("node_updates", ctypes.c_int64),
        ("tiles_swept", ctypes.c_int64),
        ("replays", ctypes.c_int64),
        ("seconds", ctypes.c_double),
        ("converged", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class NetConfig(ctypes.Structure):
    _fields_ = [
        ("layers", ctypes.c_int32),
        ("channels", ctypes.c_int32),
        ("dilation", ctypes.c_int32 * 12),
        ("arch", ctypes.c_int32),
    ]


NET_DILATED, NET_UNET = 0, 1


class NetSample(ctypes.Structure):
    _fields_ = [
        ("v_hat", ctypes.c_void_p),
        ("v_star", ctypes.c_void_p),
        ("speed", ctypes.c_void_p),
        ("node_class", ctypes.c_void_p),
        ("speed_const", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("n", ctypes.c_int32),
        ("x0", ctypes.c_int32),
        ("y0", ctypes.c_int32),
    ]


class Regime(ctypes.Structure):
    _fields_ = [
        ("omega", ctypes.c_double),
        ("upsilon", ctypes.c_double),
        ("alpha_lower", ctypes.c_double),
        ("alpha_upper", ctypes.c_double),
        ("alpha_opt", ctypes.c_double),
        ("tau_dx", ctypes.c_double),
        ("h_alpha", ctypes.c_double),
        ("h_upper", ctypes.c_double),
        ("hyperbolic", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


# name -> (restype, argtypes); every symbol include/slhjb.h declares
_vp, _i32, _i64, _f64, _f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
_PP = ctypes.POINTER(Problem)
SIGNATURES = {
    "slhjb_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "slhjb_version": (ctypes.c_int, []),
    "slhjb_source_hash": (ctypes.c_char_p, []),
    "slhjb_ctx_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _vp]),
    "slhjb_ctx_destroy": (ctypes.c_int, [_vp]),
    "slhjb_last_hip_error": (ctypes.c_int, [_vp]),
    "slhjb_last_error_message": (ctypes.c_char_p, [_vp]),
    "slhjb_sweep": (ctypes.c_int, [_vp, _PP, _vp, _vp, ctypes.POINTER(_f64)]),
    "slhjb_solve": (ctypes.c_int, [_vp, _PP, _vp, _f64, _i64, _i32, ctypes.POINTER(Stats)]),
    "slhjb_solve_noalloc": (ctypes.c_int, [_vp, _PP, _vp, _f64, _i64, _i32, ctypes.POINTER(Stats)]),
    "slhjb_solve_tiles": (ctypes.c_int, [_vp, _PP, _vp, _f64, _i64, ctypes.POINTER(TileOpts), ctypes.POINTER(Stats)]),
    "slhjb_solve_patchy": (ctypes.c_int, [_vp, _PP, _PP, ctypes.POINTER(PatchyOpts), _vp, _vp,
                                          ctypes.POINTER(PatchyStats)]),
    "slhjb_solve_batch": (ctypes.c_int, [_vp, _PP, _i32, ctypes.POINTER(_vp), _f64, _i64, ctypes.POINTER(BatchOpts),
                                         ctypes.POINTER(Stats), ctypes.POINTER(BatchStats)]),
    "slhjb_solve_tiles_batch": (ctypes.c_int, [_vp, _PP, _i32, ctypes.POINTER(_vp), _f64, _i64, ctypes.POINTER(TileOpts),
                                               ctypes.POINTER(Stats), ctypes.POINTER(BatchStats)]),
    "slhjb_tiles_batch_create": (ctypes.c_int, [_vp, _PP, _i32, ctypes.POINTER(_vp), ctypes.POINTER(TileOpts),
                                                ctypes.POINTER(_vp)]),
    "slhjb_tiles_batch_run": (ctypes.c_int, [_vp, _f64, _i64, ctypes.POINTER(Stats), ctypes.POINTER(BatchStats)]),
    "slhjb_tiles_batch_destroy": (ctypes.c_int, [_vp]),
    "slhjb_balance_sources": (ctypes.c_int, [_vp, _PP, _vp, _vp, _i32, _i32, _vp, ctypes.POINTER(_i64), _vp,
                                             ctypes.POINTER(_i32)]),
    "slhjb_net_create": (ctypes.c_int, [_vp, ctypes.POINTER(NetConfig), ctypes.POINTER(_vp)]),
    "slhjb_net_destroy": (ctypes.c_int, [_vp]),
    "slhjb_net_param_count": (_i64, [_vp]),
    "slhjb_net_set_params": (ctypes.c_int, [_vp, _vp]),
    "slhjb_net_get_params": (ctypes.c_int, [_vp, _vp]),
    "slhjb_net_get_grads": (ctypes.c_int, [_vp, _vp]),
    "slhjb_net_forward": (ctypes.c_int, [_vp, ctypes.POINTER(NetSample), _i32, _i32, _vp]),
    "slhjb_net_loss_grad": (ctypes.c_int, [_vp, ctypes.POINTER(NetSample), _i32, _i32, ctypes.POINTER(_f64)]),
    "slhjb_net_adam_step": (ctypes.c_int, [_vp, _f32]),
    "slhjb_net_warm_start": (ctypes.c_int, [_vp, _PP, _vp, _vp]),
    "slhjb_upsample": (ctypes.c_int, [_vp, _i32, _vp, _i32, _vp]),
    "slhjb_upsample_bicubic": (ctypes.c_int, [_vp, _i32, _vp, _i32, _vp]),
    "slhjb_synthesize": (ctypes.c_int, [_vp, _PP, _vp, _vp]),
    "slhjb_partition_sources": (ctypes.c_int, [_i32, _vp, _i32, _vp, ctypes.POINTER(_i32)]),
    "slhjb_label": (ctypes.c_int, [_vp, _PP, _vp, _vp, _vp, _i32, ctypes.c_uint16, _vp, _vp, _vp,
                                   ctypes.POINTER(_i64)]),
    "slhjb_regime_analyze": (ctypes.c_int, [_f64, _f64, _f64, _f64, ctypes.POINTER(Regime)]),
    "slhjb_foot_reach": (_f64, [_PP, _f32]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1502_01629_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        built = L.slhjb_source_hash().decode()
        if os.path.isdir(os.path.join(HERE, "csrc")):
            from . import build as _build

            now = _build.source_hash()
            if built != now:
                raise RuntimeError(f"{LIB_PATH} was built from other sources (hash {built}, sources {now}): "
                                   "rebuild it with `python -m paper_1502_01629_amd.build`")
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().slhjb_status_string(status).decode()


def regime(f_min: float, f_max: float, sigma_inf: float, dx: float) -> dict:
    out = Regime()
    st = lib().slhjb_regime_analyze(f_min, f_max, sigma_inf, dx, ctypes.byref(out))
    if st != OK:
        raise SlhjbError(st, "invalid regime arguments")
    return out.as_dict()


def _ptr(t) -> int:
    return int(t.data_ptr())


def partition_sources(node_class: np.ndarray, n_patches: int):
    """Host-side split of the TARGET nodes into n_patches source sets (see include/slhjb.h)."""
    cls = np.ascontiguousarray(node_class, dtype=np.uint8)
    n = int(cls.shape[0])
    out = np.empty(n * n, dtype=np.int16)
    nt = ctypes.c_int32()
    st = lib().slhjb_partition_sources(n, cls.ctypes.data, n_patches, out.ctypes.data, ctypes.byref(nt))
    if st != OK:
        raise SlhjbError(st, "slhjb_partition_sources failed")
    return out.reshape(n, n), nt.value


class DeviceProblem:
    """Device-resident arrays of a problem instance plus the ctypes struct pointing at them."""

    def __init__(self, inst, scheme: int = SL3, device="cuda"):
        import torch

        self.inst = inst
        self.controls = np.ascontiguousarray(inst.controls, dtype=np.float32).reshape(-1)
        self.speed = torch.from_numpy(np.ascontiguousarray(inst.speed, dtype=np.float32).reshape(-1)).to(device)
        self.node_class = torch.from_numpy(np.ascontiguousarray(inst.node_class, dtype=np.uint8).reshape(-1)).to(device)
        drift = getattr(inst, "drift", None)
        self.drift = None if drift is None else \
            torch.from_numpy(np.ascontiguousarray(drift, dtype=np.float32).reshape(-1)).to(device)
        dev = lambda a: None if a is None else \
            torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).reshape(-1)).to(device)
        self.running_cost_field = dev(getattr(inst, "running_cost_field", None))
        self.eps_field = dev(getattr(inst, "eps_field", None))
        cc = getattr(inst, "control_cost", None)
        self.control_cost = None if cc is None else np.ascontiguousarray(cc, dtype=np.float32).reshape(-1)
        self.scheme = scheme
        self.struct = self._make()

    @staticmethod
    def host_struct(inst, scheme: int = SL3) -> Problem:
        """The problem struct with no device arrays (for the host-only calls such as
        slhjb_foot_reach); the controls array is kept alive on the struct."""
        controls = np.ascontiguousarray(inst.controls, dtype=np.float32).reshape(-1)
        p = Problem(n=inst.n, x_lo=float(inst.x_lo), x_hi=float(inst.x_hi), h=float(inst.h), lam=float(inst.lam),
                    eps=float(inst.eps), diffusion=int(inst.diffusion), scheme=int(scheme),
                    n_controls=int(controls.size // 2), controls=controls.ctypes.data, speed=None, speed_const=1.0,
                    running_cost=float(inst.running_cost), node_class=None, target_value=float(inst.target_value),
                    v_out=float(inst.v_out))
        p._keep = controls
        return p

    def _make(self) -> Problem:
        inst = self.inst
        return Problem(
            n=inst.n, x_lo=float(inst.x_lo), x_hi=float(inst.x_hi), h=float(inst.h), lam=float(inst.lam),
            eps=float(inst.eps), diffusion=int(inst.diffusion), scheme=int(self.scheme),
            n_controls=int(self.controls.size // 2), controls=self.controls.ctypes.data, speed=_ptr(self.speed),
            speed_const=1.0, running_cost=float(inst.running_cost), node_class=_ptr(self.node_class),
            target_value=float(inst.target_value), v_out=float(inst.v_out),
            drift=_ptr(self.drift) if self.drift is not None else None,
            running_cost_field=_ptr(self.running_cost_field) if self.running_cost_field is not None else None,
            control_cost=self.control_cost.ctypes.data if self.control_cost is not None else None,
            eps_field=_ptr(self.eps_field) if self.eps_field is not None else None)

    def with_scheme(self, scheme: int) -> "DeviceProblem":
        self.scheme = scheme
        self.struct = self._make()
        return self


class Context:
    """A library context bound to a device and a HIP stream (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = ctypes.c_void_p()
        st = lib().slhjb_ctx_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != OK:
            raise SlhjbError(st, "slhjb_ctx_create failed")
        self.handle = h

    def close(self):
        if self.handle:
            lib().slhjb_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        # during interpreter shutdown the HIP runtime may already be gone: leave the memory to the
        # process exit instead of calling into it
        if _is_finalizing is None or _is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, allow=(OK,)) -> int:
        if st not in allow:
            msg = lib().slhjb_last_error_message(self.handle).decode()
            raise SlhjbError(st, msg or status_string(st))
        return st

    def sweep(self, prob: DeviceProblem, v_in, v_out) -> float:
        r = ctypes.c_double()
        self._check(lib().slhjb_sweep(self.handle, ctypes.byref(prob.struct), _ptr(v_in), _ptr(v_out), ctypes.byref(r)))
        return r.value

    def solve_tiles(self, prob: DeviceProblem, v, tol: float = 1e-6, max_passes: int = 1_000_000,
                    order: int = ORDER_NONE, mode: int = MODE_TRANSMISSION, label=None, key_slack: float = -1.0,
                    max_inner: int = 0, tile_shape: int = TILE_16x16_SPLIT2, persistent: int = 0, max_workgroups: int = 0,
                    collect_kernel_time: int = 0, policy_sweeps: int = 0):
        opts = TileOpts(order, mode, _ptr(label) if label is not None else None, key_slack, max_inner, tile_shape,
                        persistent, max_workgroups, collect_kernel_time, policy_sweeps)
        stats = Stats()
        st = lib().slhjb_solve_tiles(self.handle, ctypes.byref(prob.struct), _ptr(v), tol, max_passes,
                                     ctypes.byref(opts), ctypes.byref(stats))
        self._check(st, allow=(OK, NOT_CONVERGED))
        return stats.as_dict()

    def solve_patchy(self, fine: DeviceProblem, coarse: DeviceProblem | None, v, mode: int = PATCHY_TRANSMISSION,
                     tol: float = 1e-6, tol_coarse: float = 1e-7, source_patch=None, n_patches: int = 0,
                     label_out=None, max_passes: int = 1_000_000, key_window: float = -1.0, tile_shape: int = TILE_16x16_SPLIT2,
                     collect_kernel_time: int = 0, policy_sweeps: int = 0):
        opts = PatchyOpts(mode, n_patches, _ptr(source_patch) if source_patch is not None else None, tol, tol_coarse,
                          max_passes, key_window, tile_shape, collect_kernel_time, policy_sweeps)
        stats = PatchyStats()
        st = lib().slhjb_solve_patchy(self.handle, ctypes.byref(fine.struct),
                                      ctypes.byref(coarse.struct) if coarse is not None else None,
                                      ctypes.byref(opts), _ptr(v), _ptr(label_out) if label_out is not None else None,
                                      ctypes.byref(stats))
        self._check(st, allow=(OK, NOT_CONVERGED))
        return stats.as_dict()

    def upsample(self, v_c, n_c: int, v_f, n_f: int):
        self._check(lib().slhjb_upsample(self.handle, n_c, _ptr(v_c), n_f, _ptr(v_f)))

    def upsample_bicubic(self, v_c, n_c: int, v_f, n_f: int):
        self._check(lib().slhjb_upsample_bicubic(self.handle, n_c, _ptr(v_c), n_f, _ptr(v_f)))

    def synthesize(self, prob: DeviceProblem, v_hat, ctrl_out):
        self._check(lib().slhjb_synthesize(self.handle, ctypes.byref(prob.struct), _ptr(v_hat), _ptr(ctrl_out)))

    def label(self, prob: DeviceProblem, ctrl, source_patch, n_patches: int, label_out, tau_q15: int = 0,
              overlap_out=None, phi_out=None, v_hat=None) -> int:
        passes = ctypes.c_int64()
        self._check(lib().slhjb_label(self.handle, ctypes.byref(prob.struct), _ptr(ctrl),
                                      _ptr(v_hat) if v_hat is not None else None, _ptr(source_patch),
                                      n_patches, tau_q15, _ptr(label_out),
                                      _ptr(overlap_out) if overlap_out is not None else None,
                                      _ptr(phi_out) if phi_out is not None else None, ctypes.byref(passes)))
        return passes.value

    def balance_sources(self, prob: DeviceProblem, ctrl, source_patch, n_patches: int, iterations: int,
                        v_hat=None, label_out=None) -> np.ndarray:
        """slhjb_balance_sources: `iterations` rounds of re-dividing the sources (source_patch, a
        device int16 tensor, receives the best balanced subdivision visited). Returns (the patch
        sizes of every subdivision visited, int64[iterations + 1, n_patches], the kept round)."""
        sizes = np.zeros((iterations + 1) * n_patches, dtype=np.int64)
        best = ctypes.c_int32(-1)
        self._check(lib().slhjb_balance_sources(self.handle, ctypes.byref(prob.struct), _ptr(ctrl),
                                                _ptr(v_hat) if v_hat is not None else None, n_patches, iterations,
                                                _ptr(source_patch), sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                                _ptr(label_out) if label_out is not None else None, ctypes.byref(best)))
        return sizes.reshape(iterations + 1, n_patches), best.value

    def solve_batch(self, probs, vs, tol: float = 1e-6, max_sweeps: int = 1_000_000, check_every: int = 16,
                    batches_per_graph: int = 0, tile_shapes=None, max_workgroups: int = 0):
        """Jacobi value iteration of independent instances in shared launches (slhjb_solve_batch).
        Returns (per-instance stats dicts, totals dict)."""
        count = len(probs)
        if len(vs) != count:
            raise ValueError("one iterate per problem")
        arr = (Problem * count)(*[p.struct for p in probs])
        ptrs = (_vp * count)(*[_ptr(v) for v in vs])
        shapes = None
        if tile_shapes is not None:
            shapes = np.ascontiguousarray(tile_shapes, dtype=np.int8)
            if shapes.size != count:
                raise ValueError("one tile shape per problem")
        opts = BatchOpts(check_every, batches_per_graph, shapes.ctypes.data if shapes is not None else None,
                         max_workgroups, 0)
        stats = (Stats * count)()
        tot = BatchStats()
        st = lib().slhjb_solve_batch(self.handle, arr, count, ptrs, tol, max_sweeps, ctypes.byref(opts), stats,
                                     ctypes.byref(tot))
        self._check(st, allow=(OK, NOT_CONVERGED))
        return [s.as_dict() for s in stats], tot.as_dict()

    def solve_tiles_batch(self, probs, vs, tol: float = 1e-6, max_passes: int = 1_000_000, order: int = ORDER_NONE,
                          key_slack: float = -1.0, max_inner: int = 0, tile_shape: int = TILE_16x16_SPLIT2,
                          policy_sweeps: int = 0):
        """The active-tile solve of independent instances in shared launches (slhjb_solve_tiles_batch).
        Returns (per-instance stats dicts, totals dict)."""
        count = len(probs)
        if len(vs) != count:
            raise ValueError("one iterate per problem")
        arr = (Problem * count)(*[p.struct for p in probs])
        ptrs = (_vp * count)(*[_ptr(v) for v in vs])
        opts = TileOpts(order, MODE_TRANSMISSION, None, key_slack, max_inner, tile_shape, 0, 0, 0, policy_sweeps)
        stats = (Stats * count)()
        tot = BatchStats()
        st = lib().slhjb_solve_tiles_batch(self.handle, arr, count, ptrs, tol, max_passes, ctypes.byref(opts), stats,
                                           ctypes.byref(tot))
        self._check(st, allow=(OK, NOT_CONVERGED))
        return [s.as_dict() for s in stats], tot.as_dict()

    def solve(self, prob: DeviceProblem, v, tol: float = 1e-6, max_sweeps: int = 1_000_000, check_every: int = 0):
        stats = Stats()
        st = lib().slhjb_solve(self.handle, ctypes.byref(prob.struct), _ptr(v), tol, max_sweeps, check_every,
                               ctypes.byref(stats))
        self._check(st, allow=(OK, NOT_CONVERGED))
        return stats.as_dict()


    def solve_noalloc(self, prob: DeviceProblem, v, tol: float = 1e-6, max_sweeps: int = 1_000_000,
                      check_every: int = 0):
        """slhjb_solve_noalloc: slhjb_solve with the library's static scratch (no allocation)."""
        stats = Stats()
        st = lib().slhjb_solve_noalloc(self.handle, ctypes.byref(prob.struct), _ptr(v), tol, max_sweeps, check_every,
                                       ctypes.byref(stats))
        self._check(st, allow=(OK, NOT_CONVERGED))
        return stats.as_dict()


class TilesBatch:
    """A reusable batched active-tile solve (slhjb_tiles_batch_*): the problems and the iterate
    tensors are fixed at creation; run() solves from whatever the tensors hold."""

    def __init__(self, ctx: "Context", probs, vs, order: int = ORDER_NONE, key_slack: float = -1.0,
                 max_inner: int = 0, tile_shape: int = TILE_16x16_SPLIT2, policy_sweeps: int = 0):
        if len(vs) != len(probs):
            raise ValueError("one iterate per problem")
        self.ctx = ctx
        self.count = len(probs)
        self._keep = (list(probs), list(vs))  # the object holds their device pointers
        arr = (Problem * self.count)(*[p.struct for p in probs])
        ptrs = (_vp * self.count)(*[_ptr(v) for v in vs])
        opts = TileOpts(order, MODE_TRANSMISSION, None, key_slack, max_inner, tile_shape, 0, 0, 0, policy_sweeps)
        h = ctypes.c_void_p()
        ctx._check(lib().slhjb_tiles_batch_create(ctx.handle, arr, self.count, ptrs, ctypes.byref(opts),
                                                  ctypes.byref(h)))
        self.handle = h

    def run(self, tol: float = 1e-6, max_passes: int = 1_000_000):
        stats = (Stats * self.count)()
        tot = BatchStats()
        st = lib().slhjb_tiles_batch_run(self.handle, tol, max_passes, stats, ctypes.byref(tot))
        self.ctx._check(st, allow=(OK, NOT_CONVERGED))
        return [s.as_dict() for s in stats], tot.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            lib().slhjb_tiles_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        # during interpreter shutdown the HIP runtime may already be gone: leave the memory to the
        # process exit instead of calling into it
        if _is_finalizing is None or _is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Net:
    """The learned warm-start network of a context (slhjb_net_*): parameters live on the device."""

    def __init__(self, ctx: "Context", layers: int = 6, channels: int = 32, dilations=(1, 2, 4, 8, 16, 1),
                 arch: int = NET_DILATED):
        if arch == NET_DILATED and len(dilations) != layers:
            raise ValueError("one dilation per layer")
        self.ctx = ctx
        self.arch = arch
        self.layers, self.channels, self.dilations = layers, channels, tuple(int(d) for d in dilations)
        cfg = NetConfig(layers, channels, (ctypes.c_int32 * 12)(*self.dilations[:12]), arch)
        h = ctypes.c_void_p()
        ctx._check(lib().slhjb_net_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().slhjb_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        # during interpreter shutdown the HIP runtime may already be gone: leave the memory to the
        # process exit instead of calling into it
        if _is_finalizing is None or _is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    @property
    def param_count(self) -> int:
        return int(lib().slhjb_net_param_count(self.handle))

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.param_count:
            raise ValueError("wrong parameter count")
        self.ctx._check(lib().slhjb_net_set_params(self.handle, p.ctypes.data))

    def get_params(self) -> np.ndarray:
        out = np.empty(self.param_count, dtype=np.float32)
        self.ctx._check(lib().slhjb_net_get_params(self.handle, out.ctypes.data))
        return out

    def get_grads(self) -> np.ndarray:
        out = np.empty(self.param_count, dtype=np.float32)
        self.ctx._check(lib().slhjb_net_get_grads(self.handle, out.ctypes.data))
        return out

    @staticmethod
    def samples(items) -> "ctypes.Array":
        """items: (v_hat, v_star or None, DeviceProblem, x0, y0) tuples."""
        arr = (NetSample * len(items))()
        for k, (vh, vs, dp, x0, y0) in enumerate(items):
            st = dp.struct
            arr[k] = NetSample(_ptr(vh), _ptr(vs) if vs is not None else None, st.speed, st.node_class,
                               st.speed_const, st.eps, st.n, x0, y0)
        return arr

    def forward(self, items, crop: int, out):
        arr = self.samples(items)
        self.ctx._check(lib().slhjb_net_forward(self.handle, arr, len(items), crop, _ptr(out)))
        return out

    def loss_grad(self, items, crop: int) -> float:
        arr = self.samples(items)
        loss = ctypes.c_double()
        self.ctx._check(lib().slhjb_net_loss_grad(self.handle, arr, len(items), crop, ctypes.byref(loss)))
        return loss.value

    def adam_step(self, lr: float):
        self.ctx._check(lib().slhjb_net_adam_step(self.handle, lr))

    def warm_start(self, dp: DeviceProblem, v_hat, v_out):
        self.ctx._check(lib().slhjb_net_warm_start(self.handle, ctypes.byref(dp.struct), _ptr(v_hat), _ptr(v_out)))
        return v_out
