"""ctypes wrapper of the FP64 CPU oracle (``liblbref.so``).

TEST INFRASTRUCTURE ONLY.  The oracle is the independent checker of the GPU
path: only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import this module.  It does not import the GPU package and the GPU
package does not import it.

The wrapped library implements one time step of the coupled lattice Boltzmann
freezing scheme of Huang, Chai, Liu, Huang (arXiv 2511.09422), Sec. 3, in
plain FP64 loops; see ``lbref.c`` for the step and its readings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbref.so")

PARAM_DOUBLES = (
    "rho_l", "rho_g", "rho_s", "nu", "tau_phi", "tau_h", "tau_c", "eps",
    "sigma0", "sigma_T", "sigma_c", "T_ref", "c_ref", "cp_l", "cp_s", "cp_g",
    "rhoc_ref", "latent", "T_sol", "T_liq", "k_p", "Ds_over_Dl", "T_lo", "T_hi",
    "T_lo_amp",
)
PARAM_INTS = ("dim", "nx", "ny", "nz", "walls", "t_lo_dirichlet", "t_hi_dirichlet",
              "surface_tension_mode", "threads")


class LbrefParams(ctypes.Structure):
    _fields_ = ([(k, ctypes.c_int32) for k in PARAM_INTS]
                + [(k, ctypes.c_double) for k in PARAM_DOUBLES]
                + [("body_force", ctypes.c_double * 3)])


class LbrefParamsSingle(ctypes.Structure):
    _fields_ = ([(k, ctypes.c_int32) for k in PARAM_INTS]
                + [(k, ctypes.c_float) for k in PARAM_DOUBLES]
                + [("body_force", ctypes.c_float * 3)])


# Variants of the oracle built from the same source, for the tests that
# compare against them: name -> gcc defines.  "hard_cutoff" switches one
# reading (the interface normal); "single" is the same source with every
# double made a float (and single-precision constants), the scheme evaluated
# in FP32 arithmetic and storage, as a measure of what FP32 alone does to a
# trajectory; "single_cw" the same with weights that sum to one in FP32: each
# rest weight the complement of the moving ones (as the GPU kernels' rest
# equilibria, the complements of the moving ones, are), and the D3Q7 set,
# which has no rest weight, with its +-z pair one ulp below fl(1/6) (as the
# GPU's 3D phase-field and solute collisions take it).
VARIANTS = {"hard_cutoff": ["-DLBREF_HARD_NORMAL_CUTOFF"],
            "single": ["-fsingle-precision-constant"],
            "single_cw": ["-fsingle-precision-constant", "-DLBREF_REST_WEIGHT_COMPLEMENT"]}


SINGLE = ("single", "single_cw")   # the FP32 builds (float ABI)


def _lib_path(variant=None) -> str:
    return _LIB_PATH if variant is None else os.path.join(_HERE, f"liblbref_{variant}.so")


def build(force: bool = False, variant=None) -> str:
    """Compile ``lbref.c`` with gcc (-O2, no fast-math, OpenMP for loops)."""
    import re
    import shutil
    import tempfile
    src = os.path.join(_HERE, "lbref.c")
    path = _lib_path(variant)
    if force or not os.path.exists(path) or (os.path.getmtime(path) < os.path.getmtime(src)):
        tmp = path + ".tmp"
        work = None
        if variant in SINGLE:
            # the same source with double -> float, built in a scratch folder
            work = tempfile.mkdtemp(prefix="lbref_single_")
            for name in ("lbref.c", "lbref.h"):
                with open(os.path.join(_HERE, name)) as fh:
                    text = re.sub(r"\bdouble\b", "float", fh.read())
                with open(os.path.join(work, name), "w") as fh:
                    fh.write(text)
            src = os.path.join(work, "lbref.c")
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
               "-fopenmp", "-Wall", "-Wno-unknown-pragmas"]
        cmd += VARIANTS[variant] if variant is not None else []
        cmd += ["-o", tmp, src, "-lm"]
        try:
            subprocess.check_call(cmd, cwd=_HERE)
        finally:
            if work:
                shutil.rmtree(work, ignore_errors=True)
        os.replace(tmp, path)
    return path


_libs = {}


def lib(variant=None):
    if variant not in _libs:
        path = _lib_path(variant)
        if variant is not None or not os.path.exists(path):
            build(variant=variant)
        L = ctypes.CDLL(path)
        single = variant in SINGLE
        dp = ctypes.POINTER(ctypes.c_float if single else ctypes.c_double)
        pp = ctypes.POINTER(LbrefParamsSingle if single else LbrefParams)
        L.lbref_create.argtypes = [pp, dp, dp, dp, ctypes.c_void_p, ctypes.c_void_p]
        L.lbref_create.restype = ctypes.c_int
        L.lbref_destroy.argtypes = [ctypes.c_void_p]
        L.lbref_destroy.restype = None
        L.lbref_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.lbref_step.restype = ctypes.c_int
        L.lbref_fields.argtypes = [ctypes.c_void_p] + [dp] * 9
        L.lbref_fields.restype = ctypes.c_int
        L.lbref_totals.argtypes = [ctypes.c_void_p, dp]
        L.lbref_totals.restype = ctypes.c_int
        for nm in ("lbref_get_pops", "lbref_set_pops", "lbref_get_state", "lbref_set_state"):
            getattr(L, nm).argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
            getattr(L, nm).restype = ctypes.c_int
        L.lbref_q.argtypes = [ctypes.c_int, ctypes.c_int]
        L.lbref_q.restype = ctypes.c_int
        L.lbref_enthalpy_map.argtypes = [pp, (ctypes.c_float if single else ctypes.c_double), (ctypes.c_float if single else ctypes.c_double), dp, dp, dp]
        L.lbref_enthalpy_map.restype = None
        L.lbref_feq_g.argtypes = [ctypes.c_int, (ctypes.c_float if single else ctypes.c_double), (ctypes.c_float if single else ctypes.c_double), dp, dp]
        L.lbref_feq_g.restype = None
        L.lbref_src_g.argtypes = [ctypes.c_int, (ctypes.c_float if single else ctypes.c_double), dp, dp, dp, dp]
        L.lbref_src_g.restype = None
        L.lbref_heq.argtypes = [pp, (ctypes.c_float if single else ctypes.c_double), (ctypes.c_float if single else ctypes.c_double), (ctypes.c_float if single else ctypes.c_double), dp, dp]
        L.lbref_heq.restype = None
        L.lbref_grad_lap.argtypes = [pp, dp, ctypes.c_int, dp, dp]
        L.lbref_grad_lap.restype = None
        ip = ctypes.POINTER(ctypes.c_int)
        L.lbref_lattice.argtypes = [ctypes.c_int, ctypes.c_int, ip, dp, ip]
        L.lbref_lattice.restype = ctypes.c_int
        _libs[variant] = L
    return _libs[variant]


def _dptr(a: np.ndarray):
    ct = ctypes.c_float if a.dtype == np.float32 else ctypes.c_double
    return a.ctypes.data_as(ctypes.POINTER(ct))


def make_params(cfg: dict, threads: int = 1, single: bool = False):
    P = LbrefParamsSingle() if single else LbrefParams()
    for k in PARAM_INTS:
        setattr(P, k, int(cfg.get(k, 0)))
    if P.dim == 2:
        P.nz = 1
    P.threads = int(threads)
    for k in PARAM_DOUBLES:
        setattr(P, k, float(cfg[k]))
    bf = cfg.get("body_force", (0.0, 0.0, 0.0))
    for a in range(3):
        P.body_force[a] = float(bf[a])
    return P


class Oracle:
    """One FP64 oracle instance: create from initial (phi, T, C[, mask])."""

    def __init__(self, cfg: dict, phi, T, C, mask=None, threads: int = 1, variant=None):
        self._L = lib(variant)
        self._ft = np.float32 if variant in SINGLE else np.float64
        self.cfg = dict(cfg)
        self.P = make_params(cfg, threads, single=variant in SINGLE)
        self.shape = (self.P.nz, self.P.ny, self.P.nx) if self.P.dim == 3 else (self.P.ny, self.P.nx)
        self.N = self.P.nx * self.P.ny * self.P.nz
        phi = np.ascontiguousarray(phi, dtype=self._ft).reshape(-1)
        T = np.ascontiguousarray(T, dtype=self._ft).reshape(-1)
        C = np.ascontiguousarray(C, dtype=self._ft).reshape(-1)
        for a in (phi, T, C):
            if a.size != self.N:
                raise ValueError("initial field size does not match the grid")
        mptr = None
        self._mask = None
        if mask is not None:
            self._mask = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
            mptr = self._mask.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        rc = self._L.lbref_create(ctypes.byref(self.P), _dptr(phi), _dptr(T), _dptr(C), mptr,
                                ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"lbref_create failed with code {rc}")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.lbref_destroy(h)
            self._h = None

    def step(self, n: int = 1):
        rc = self._L.lbref_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError(f"lbref_step failed with code {rc}")

    def fields(self) -> dict:
        names = ("phi", "fl", "T", "C", "ux", "uy", "uz", "p", "rho")
        out = {k: np.empty(self.N, self._ft) for k in names}
        rc = self._L.lbref_fields(self._h, *[_dptr(out[k]) for k in names])
        if rc != 0:
            raise RuntimeError("lbref_fields failed")
        return {k: v.reshape(self.shape).astype(np.float64, copy=False) for k, v in out.items()}

    def totals(self) -> dict:
        out = np.empty(9, self._ft)
        self._L.lbref_totals(self._h, _dptr(out))
        keys = ("sum_f", "sum_l", "sum_h", "mpc", "vol_solid", "vol_sl", "step", "nonfinite",
                "qsum")
        return dict(zip(keys, out.astype(np.float64, copy=False).tolist()))

    def q(self, which: int) -> int:
        return self._L.lbref_q(self.P.dim, which)

    def get_pops(self, which: int) -> np.ndarray:
        out = np.empty(self.q(which) * self.N, self._ft)
        self._L.lbref_get_pops(self._h, which, _dptr(out))
        return out.reshape((self.q(which),) + self.shape).astype(np.float64, copy=False)

    def set_pops(self, which: int, arr) -> None:
        a = np.ascontiguousarray(arr, dtype=self._ft).reshape(-1)
        assert a.size == self.q(which) * self.N
        self._L.lbref_set_pops(self._h, which, _dptr(a))

    def get_state(self, which: int) -> np.ndarray:
        out = np.empty(self.N, self._ft)
        self._L.lbref_get_state(self._h, which, _dptr(out))
        return out.reshape(self.shape).astype(np.float64, copy=False)

    def set_state(self, which: int, arr) -> None:
        a = np.ascontiguousarray(arr, dtype=self._ft).reshape(-1)
        assert a.size == self.N
        self._L.lbref_set_state(self._h, which, _dptr(a))


def enthalpy_map(cfg: dict, E: float, psi: float):
    P = make_params(cfg)
    T, fl, fs = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().lbref_enthalpy_map(ctypes.byref(P), float(E), float(psi), ctypes.byref(T),
                             ctypes.byref(fl), ctypes.byref(fs))
    return T.value, fl.value, fs.value


def feq_g(dim: int, p: float, rho: float, u) -> np.ndarray:
    u3 = np.zeros(3)
    u3[: len(u)] = u
    out = np.empty(19)
    lib().lbref_feq_g(dim, float(p), float(rho), _dptr(u3), _dptr(out))
    return out[: lib().lbref_q(dim, 1)].copy()


def src_g(dim: int, S: float, Ff, u, Ft) -> np.ndarray:
    def v3(a):
        r = np.zeros(3)
        r[: len(a)] = a
        return r
    a, b, c = v3(Ff), v3(u), v3(Ft)
    out = np.empty(19)
    lib().lbref_src_g(dim, float(S), _dptr(a), _dptr(b), _dptr(c), _dptr(out))
    return out[: lib().lbref_q(dim, 1)].copy()


def heq(cfg: dict, E: float, T: float, rhocp: float, u) -> np.ndarray:
    P = make_params(cfg)
    u3 = np.zeros(3)
    u3[: len(u)] = u
    out = np.empty(19)
    lib().lbref_heq(ctypes.byref(P), float(E), float(T), float(rhocp), _dptr(u3), _dptr(out))
    return out[: lib().lbref_q(P.dim, 0)].copy()


def grad_lap(cfg: dict, field: np.ndarray, kind: int = 0):
    P = make_params(cfg)
    f = np.ascontiguousarray(field, dtype=np.float64).reshape(-1)
    N = P.nx * P.ny * P.nz
    assert f.size == N
    g = np.empty(3 * N)
    lp = np.empty(N)
    lib().lbref_grad_lap(ctypes.byref(P), _dptr(f), int(kind), _dptr(g), _dptr(lp))
    shape = (P.nz, P.ny, P.nx) if P.dim == 3 else (P.ny, P.nx)
    return g.reshape((3,) + shape), lp.reshape(shape)


def lattice(dim: int, which: int):
    """(c [q,3] int, w [q], opp [q]) of the oracle's flow (which=1) or scalar lattice."""
    c = np.zeros(19 * 3, dtype=np.int32)
    w = np.zeros(19)
    o = np.zeros(19, dtype=np.int32)
    q = lib().lbref_lattice(dim, which, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dptr(w),
                            o.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return c[: 3 * q].reshape(q, 3).copy(), w[:q].copy(), o[:q].copy()
