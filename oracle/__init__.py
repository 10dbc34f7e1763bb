"""FP64 CPU oracle for the semi-Lagrangian Markov-chain scheme (arXiv 1502.01629).

TEST INFRASTRUCTURE ONLY. The plain, slow reference the GPU library is checked against.
Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import it. It shares no code with the GPU package: the C source next to this file is
compiled with gcc into ``liboracle.so`` and driven through ctypes.

Inputs are the FP32 arrays of a problem instance promoted exactly to float64, so the oracle
and the GPU solve the same discrete problem and parity measures arithmetic only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slhjb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FREE, TARGET, OBSTACLE = 0, 1, 2
DIFF_NONE, DIFF_ISO, DIFF_RANK1 = 0, 1, 2
SL2, SL3 = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("x_lo", ctypes.c_double),
        ("x_hi", ctypes.c_double),
        ("h", ctypes.c_double),
        ("lam", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("diffusion", ctypes.c_int32),
        ("scheme", ctypes.c_int32),
        ("n_controls", ctypes.c_int32),
        ("controls", ctypes.c_void_p),
        ("speed", ctypes.c_void_p),
        ("running_cost", ctypes.c_double),
        ("node_class", ctypes.c_void_p),
        ("target_value", ctypes.c_double),
        ("v_out", ctypes.c_double),
        ("drift", ctypes.c_void_p),
        ("running_cost_field", ctypes.c_void_p),
        ("control_cost", ctypes.c_void_p),
        ("eps_field", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_Problem)
        vp = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "or_beta": (f64, [P]),
            "or_rho": (f64, [P]),
            "or_rho_at": (f64, [P, i32, i32]),
            "or_feet": (i32, [P, i32, i32, i32, vp]),
            "or_interp_weights": (i32, [P, f64, f64, vp, vp]),
            "or_interp": (f64, [P, vp, f64, f64]),
            "or_one_step_mean": (f64, [P, vp, i32, i32]),
            "or_candidate": (f64, [P, vp, i32, i32]),
            "or_bellman": (f64, [P, vp, i32, vp]),
            "or_jacobi_sweep": (f64, [P, vp, vp, i32]),
            "or_solve": (i64, [P, vp, f64, i64, i32, vp, i32, vp, vp, i64]),
            "or_transitions": (i32, [P, i32, i32, vp, vp, vp]),
            "or_synthesize": (None, [P, vp, vp, vp]),
            "or_policy_chain": (None, [P, vp, vp, vp, vp, i32]),
            "or_policy_improve": (i64, [P, vp, vp, i32]),
            "or_rho_policy": (None, [P, vp, vp]),
            "or_upsample_bilinear": (None, [i32, vp, i32, vp]),
            "or_upsample_bicubic": (None, [i32, vp, i32, vp]),
            "or_displacement": (None, [i32, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp, vp, vp, vp]),
            "or_label": (i64, [i32, vp, vp, vp, i32, i32, vp, vp]),
            "or_sweep_independent": (f64, [P, vp, vp, vp, i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class Problem:
    """A discrete problem on the n x n grid of [x_lo, x_hi]^2 (node (i,j) stored at j*n+i),
    dynamics f(x,a) = c(x) (d(x) + a) with the drift d absent (0) unless given. Arrays are held
    as float64/uint8 copies owned by this object."""

    n: int
    x_lo: float
    x_hi: float
    h: float
    lam: float
    eps: float
    diffusion: int
    scheme: int
    controls: np.ndarray  # (N_A, 2)
    speed: np.ndarray  # (n, n) or (n*n,)
    node_class: np.ndarray  # (n, n) uint8
    running_cost: float = 1.0
    target_value: float = 0.0
    v_out: float = 1.0
    drift: np.ndarray | None = None  # (n, n, 2) or None
    running_cost_field: np.ndarray | None = None  # (n, n): l_x per node, or None = running_cost
    control_cost: np.ndarray | None = None  # (N_A,): l_a per control, or None = 0
    eps_field: np.ndarray | None = None  # (n, n): eps(x) per node, or None = eps

    def __post_init__(self):
        self.controls = np.ascontiguousarray(self.controls, dtype=np.float64).reshape(-1, 2)
        if self.drift is not None:
            self.drift = np.ascontiguousarray(self.drift, dtype=np.float64).reshape(-1)
            assert self.drift.size == 2 * self.n * self.n
        for name, size in (("running_cost_field", self.n * self.n), ("control_cost", self.controls.shape[0]),
                           ("eps_field", self.n * self.n)):
            a = getattr(self, name)
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
                assert a.size == size, name
                setattr(self, name, a)
        self.speed = np.ascontiguousarray(self.speed, dtype=np.float64).reshape(-1)
        self.node_class = np.ascontiguousarray(self.node_class, dtype=np.uint8).reshape(-1)
        assert self.speed.size == self.n * self.n and self.node_class.size == self.n * self.n

    def c_struct(self) -> _Problem:
        return _Problem(self.n, self.x_lo, self.x_hi, self.h, self.lam, self.eps, self.diffusion,
                        self.scheme, self.controls.shape[0], _ptr(self.controls), _ptr(self.speed),
                        self.running_cost, _ptr(self.node_class), self.target_value, self.v_out,
                        _ptr(self.drift) if self.drift is not None else None,
                        *[_ptr(a) if a is not None else None
                          for a in (self.running_cost_field, self.control_cost, self.eps_field)])

    @classmethod
    def from_instance(cls, inst, scheme: int = SL3) -> "Problem":
        """Promote an FP32 instance (paper_1502_01629_amd.instances.Instance) exactly to float64."""
        return cls(n=inst.n, x_lo=float(inst.x_lo), x_hi=float(inst.x_hi), h=float(inst.h),
                   lam=float(inst.lam), eps=float(inst.eps), diffusion=int(inst.diffusion), scheme=scheme,
                   controls=inst.controls.astype(np.float64), speed=inst.speed.astype(np.float64),
                   node_class=inst.node_class, running_cost=float(inst.running_cost),
                   target_value=float(inst.target_value), v_out=float(inst.v_out),
                   drift=None if getattr(inst, "drift", None) is None else inst.drift.astype(np.float64),
                   **{k: (None if getattr(inst, k, None) is None else getattr(inst, k).astype(np.float64))
                      for k in ("running_cost_field", "control_cost", "eps_field")})

    # ---- thin wrappers -------------------------------------------------------------------
    def beta(self) -> float:
        s = self.c_struct()
        return lib().or_beta(ctypes.byref(s))

    def rho(self) -> float:
        s = self.c_struct()
        return lib().or_rho(ctypes.byref(s))

    def rho_table(self) -> np.ndarray:
        """(N, N_A) running cost of one step at every node under every control (eq. SLscheme2:
        (1-beta) l / lambda, or h l for lambda = 0, with l = l_x(x) + l_a(a))."""
        s = self.c_struct()
        N, NA = self.n * self.n, self.controls.shape[0]
        if self.running_cost_field is None and self.control_cost is None:
            return np.full((N, NA), lib().or_rho(ctypes.byref(s)))
        out = np.empty((N, NA))
        for node in range(N):
            for m in range(NA):
                out[node, m] = lib().or_rho_at(ctypes.byref(s), node, m)
        return out

    def initial(self, free_value: float = 1.0) -> np.ndarray:
        v = np.full(self.n * self.n, free_value, dtype=np.float64)
        v[self.node_class == TARGET] = self.target_value
        v[self.node_class == OBSTACLE] = self.v_out
        return v

    def feet(self, i: int, j: int, m: int) -> np.ndarray:
        s = self.c_struct()
        y = np.zeros(8, dtype=np.float64)
        K = lib().or_feet(ctypes.byref(s), i, j, m, _ptr(y))
        return y[: 2 * K].reshape(K, 2)

    def interp(self, v: np.ndarray, y1: float, y2: float) -> float:
        s = self.c_struct()
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        return lib().or_interp(ctypes.byref(s), _ptr(v), y1, y2)

    def one_step_mean(self, v: np.ndarray, node: int, m: int) -> float:
        s = self.c_struct()
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        return lib().or_one_step_mean(ctypes.byref(s), _ptr(v), node, m)

    def candidate(self, v: np.ndarray, node: int, m: int) -> float:
        s = self.c_struct()
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        return lib().or_candidate(ctypes.byref(s), _ptr(v), node, m)

    def bellman(self, v: np.ndarray, node: int):
        s = self.c_struct()
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        am = np.zeros(1, dtype=np.int32)
        val = lib().or_bellman(ctypes.byref(s), _ptr(v), node, _ptr(am))
        return val, int(am[0])

    def sweep(self, v: np.ndarray, threads: int = 1):
        s = self.c_struct()
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        out = np.empty_like(v)
        r = lib().or_jacobi_sweep(ctypes.byref(s), _ptr(v), _ptr(out), threads)
        return out, r

    def sweep_independent(self, label: np.ndarray, v: np.ndarray, threads: int = 1):
        s = self.c_struct()
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        lab = np.ascontiguousarray(label, dtype=np.int16).reshape(-1)
        out = np.empty_like(v)
        r = lib().or_sweep_independent(ctypes.byref(s), _ptr(lab), _ptr(v), _ptr(out), threads)
        return out, r

    def solve(self, v0: np.ndarray | None = None, tol: float = 1e-10, max_sweeps: int = 1_000_000,
              gauss_seidel: bool = False, order: np.ndarray | None = None, threads: int = 1,
              history: int = 0):
        """Value iteration to sup-norm change <= tol. Returns (v, sweeps, residual, history)."""
        s = self.c_struct()
        v = self.initial() if v0 is None else np.array(v0, dtype=np.float64).reshape(-1)
        hist = np.zeros(max(history, 1), dtype=np.float64)
        r = np.zeros(1, dtype=np.float64)
        o = None
        if order is not None:
            o = np.ascontiguousarray(order, dtype=np.int32)
        sweeps = lib().or_solve(ctypes.byref(s), _ptr(v), tol, max_sweeps, int(gauss_seidel),
                                _ptr(o) if o is not None else None, threads, _ptr(r), _ptr(hist), history)
        if sweeps < 0:
            raise MemoryError("oracle solve: allocation failed")
        return v, int(sweeps), float(r[0]), hist[: min(history, sweeps)]

    def transitions(self, node: int, m: int):
        s = self.c_struct()
        idx = np.zeros(16, dtype=np.int32)
        w = np.zeros(16, dtype=np.float64)
        wo = np.zeros(1, dtype=np.float64)
        cnt = lib().or_transitions(ctypes.byref(s), node, m, _ptr(idx), _ptr(w), _ptr(wo))
        return idx[:cnt].copy(), w[:cnt].copy(), float(wo[0])

    def policy_chain(self, policy: np.ndarray, threads: int = 1):
        """Per node the chain of control policy[node]: (index[N,16] with -1 padding, weight[N,16],
        weight of feet outside the box[N])."""
        s = self.c_struct()
        N = self.n * self.n
        pol = np.ascontiguousarray(policy, dtype=np.int32).reshape(-1)
        idx = np.empty((N, 16), dtype=np.int32)
        w = np.empty((N, 16), dtype=np.float64)
        wo = np.empty(N, dtype=np.float64)
        lib().or_policy_chain(ctypes.byref(s), _ptr(pol), _ptr(idx), _ptr(w), _ptr(wo), threads)
        return idx, w, wo

    def rho_policy(self, policy: np.ndarray) -> np.ndarray:
        """Step cost of every node under its control policy[node] (0 off the FREE nodes)."""
        s = self.c_struct()
        pol = np.ascontiguousarray(policy, dtype=np.int32).reshape(-1)
        out = np.empty(self.n * self.n, dtype=np.float64)
        lib().or_rho_policy(ctypes.byref(s), _ptr(pol), _ptr(out))
        return out

    def policy_improve(self, v: np.ndarray, policy: np.ndarray, threads: int = 1) -> int:
        """Greedy improvement of policy (int32[N], changed in place) at v; returns the changes."""
        s = self.c_struct()
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        assert policy.dtype == np.int32 and policy.flags.c_contiguous
        return int(lib().or_policy_improve(ctypes.byref(s), _ptr(v), _ptr(policy), threads))

    def synthesize(self, v_hat: np.ndarray):
        s = self.c_struct()
        v = np.ascontiguousarray(v_hat, dtype=np.float64).reshape(-1)
        ctrl = np.zeros(self.n * self.n, dtype=np.int32)
        gap = np.zeros(self.n * self.n, dtype=np.float64)
        lib().or_synthesize(ctypes.byref(s), _ptr(v), _ptr(ctrl), _ptr(gap))
        return ctrl, gap


def upsample_bilinear(v_c: np.ndarray, n_f: int) -> np.ndarray:
    n_c = int(round(np.sqrt(v_c.size)))
    vc = np.ascontiguousarray(v_c, dtype=np.float64).reshape(-1)
    out = np.zeros(n_f * n_f, dtype=np.float64)
    lib().or_upsample_bilinear(n_c, _ptr(vc), n_f, _ptr(out))
    return out


def upsample_bicubic(v_c: np.ndarray, n_f: int) -> np.ndarray:
    """Keys (a = -1/2) bicubic interpolation with edge replication (see the C source)."""
    n_c = int(round(np.sqrt(v_c.size)))
    vc = np.ascontiguousarray(v_c, dtype=np.float64).reshape(-1)
    out = np.zeros(n_f * n_f, dtype=np.float64)
    lib().or_upsample_bicubic(n_c, _ptr(vc), n_f, _ptr(out))
    return out


def displacement(n: int, x_lo: float, x_hi: float, h: float, speed: np.ndarray, controls: np.ndarray,
                 ctrl: np.ndarray) -> np.ndarray:
    """Q.8 foot displacement of the synthesized field, computed in float (see the C source)."""
    sp = np.ascontiguousarray(speed, dtype=np.float32).reshape(-1)
    ct = np.ascontiguousarray(controls, dtype=np.float32).reshape(-1)
    cl = np.ascontiguousarray(ctrl, dtype=np.int32).reshape(-1)
    out = np.zeros(2 * n * n, dtype=np.int32)
    lib().or_displacement(n, float(np.float32(x_lo)), float(np.float32(x_hi)), float(np.float32(h)),
                          _ptr(sp), _ptr(ct), _ptr(cl), _ptr(out))
    return out.reshape(n * n, 2)


def label(n: int, node_class: np.ndarray, disp_q8: np.ndarray, source_patch: np.ndarray, n_patches: int,
          order_mode: int = 0):
    """Integer patch labeling. Returns (label int16[n*n], phi uint16[n*n, P], passes)."""
    cl = np.ascontiguousarray(node_class, dtype=np.uint8).reshape(-1)
    d = np.ascontiguousarray(disp_q8, dtype=np.int32).reshape(-1)
    sp = np.ascontiguousarray(source_patch, dtype=np.int16).reshape(-1)
    phi = np.zeros(n * n * n_patches, dtype=np.uint16)
    lab = np.zeros(n * n, dtype=np.int16)
    passes = lib().or_label(n, _ptr(cl), _ptr(d), _ptr(sp), n_patches, order_mode, _ptr(phi), _ptr(lab))
    if passes < 0:
        raise MemoryError("oracle label: allocation failed")
    return lab, phi.reshape(n * n, n_patches), int(passes)
