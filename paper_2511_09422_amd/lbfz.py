"""Thin ctypes binding of the C ABI in ``include/lbfz.h`` (``liblbfz.so``).

Argument marshalling only: every step of the scheme runs in the HIP kernels
of the shared library.  PyTorch provides the device workspace and the stream.
The functions keep the C names (``lbfz_create``, ``lbfz_step``,
``lbfz_fields``, ``lbfz_totals``, ...); :class:`Solver` bundles them.

The library must have been built (``python -m paper_2511_09422_amd.build``);
there is no fallback of any kind: a missing or unloadable library raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbfz.so")

LBFZ_OK, LBFZ_EINVAL, LBFZ_ENOMEM, LBFZ_EHIP, LBFZ_ENONFINITE, LBFZ_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
FIELDS = ("phi", "fl", "T", "C", "ux", "uy", "uz", "p", "rho")

_INTS = ("dim", "nx", "ny", "nz", "walls", "t_lo_dirichlet", "t_hi_dirichlet",
         "surface_tension_mode", "storage", "contact_angle_deg")
_DOUBLES = ("rho_l", "rho_g", "rho_s", "nu", "tau_phi", "tau_h", "tau_c", "eps", "sigma0",
            "sigma_T", "sigma_c", "T_ref", "c_ref", "cp_l", "cp_s", "cp_g", "rhoc_ref", "latent",
            "T_sol", "T_liq", "k_p", "Ds_over_Dl", "T_lo", "T_hi", "T_lo_amp")


class lbfz_params(ctypes.Structure):
    _fields_ = ([(k, ctypes.c_int32) for k in _INTS] + [(k, ctypes.c_double) for k in _DOUBLES]
                + [("body_force", ctypes.c_double * 3)])


class lbfz_totals_t(ctypes.Structure):
    _fields_ = [("sum_f", ctypes.c_double), ("sum_l", ctypes.c_double),
                ("sum_h", ctypes.c_double), ("mpc", ctypes.c_double),
                ("vol_solid", ctypes.c_double), ("vol_sl", ctypes.c_double),
                ("step", ctypes.c_int64), ("nonfinite", ctypes.c_int64)]


class LbfzError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {lbfz_strerror(code)} (code {code})")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load ``liblbfz.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2511_09422_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(lbfz_params)
        L.lbfz_workspace_bytes.argtypes = [pp, ctypes.POINTER(ctypes.c_size_t)]
        L.lbfz_create.argtypes = [pp, dp, dp, dp, vp, vp, ctypes.c_size_t, vp,
                                  ctypes.POINTER(vp)]
        L.lbfz_step.argtypes = [vp, ctypes.c_int64]
        L.lbfz_fields.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p),
                                  ctypes.c_int]
        L.lbfz_totals.argtypes = [vp, ctypes.POINTER(lbfz_totals_t)]
        L.lbfz_sync.argtypes = [vp]
        L.lbfz_state_floats.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.lbfz_get_state.argtypes = [vp, ctypes.c_void_p]
        L.lbfz_set_state.argtypes = [vp, ctypes.c_void_p]
        L.lbfz_destroy.argtypes = [vp]
        L.lbfz_destroy.restype = None
        L.lbfz_strerror.argtypes = [ctypes.c_int]
        L.lbfz_strerror.restype = ctypes.c_char_p
        L.lbfz_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.lbfz_stream_planes.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_long,
                                         vp]
        L.lbfz_stream_planes3d.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_long, ctypes.c_int32,
                                           ctypes.c_int32, vp]
        ip = ctypes.POINTER(ctypes.c_int32)
        dpp = ctypes.POINTER(dp)
        L.lbfz_batch_workspace_bytes.argtypes = [ctypes.c_int32, pp,
                                                 ctypes.POINTER(ctypes.c_size_t)]
        L.lbfz_batch_create.argtypes = [ctypes.c_int32, pp, dpp, dpp, dpp, vp, ctypes.c_size_t,
                                        vp, ctypes.POINTER(vp)]
        L.lbfz_batch_tune.argtypes = [vp, ctypes.c_int32]
        L.lbfz_batch_step.argtypes = [vp, ctypes.c_int64]
        L.lbfz_batch_step_sequential.argtypes = [vp, ctypes.c_int64]
        L.lbfz_batch_groups.argtypes = [vp]
        L.lbfz_batch_group_config.argtypes = [vp, ctypes.c_int32, ip, ip, ip, ip, ip]
        L.lbfz_batch_fields.argtypes = [vp, ctypes.c_int32, ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
        L.lbfz_batch_totals.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(lbfz_totals_t)]
        L.lbfz_batch_destroy.argtypes = [vp]
        L.lbfz_batch_destroy.restype = None
        vpp = ctypes.POINTER(ctypes.c_void_p)
        L.lbfz_restart_fields.argtypes = [vp, vpp]
        L.lbfz_batch_select.argtypes = [vp, ctypes.c_int32, ip]
        L.lbfz_batch_restart_fields.argtypes = [vp, ctypes.c_int32, vpp]
        L.lbfz_batch_fields_all.argtypes = [vp, ctypes.c_uint32, vp, ctypes.c_int64]
        L.lbfz_batch_restart_many.argtypes = [vp, ctypes.c_int32, ip, vpp,
                                              ctypes.POINTER(ctypes.c_int64)]
        for nm in ("lbfz_workspace_bytes", "lbfz_create", "lbfz_step", "lbfz_fields",
                   "lbfz_totals", "lbfz_sync", "lbfz_state_floats", "lbfz_get_state",
                   "lbfz_set_state", "lbfz_batch_workspace_bytes", "lbfz_batch_create",
                   "lbfz_batch_tune", "lbfz_batch_step", "lbfz_batch_step_sequential",
                   "lbfz_batch_groups", "lbfz_batch_group_config", "lbfz_batch_fields",
                   "lbfz_batch_totals", "lbfz_restart_fields", "lbfz_batch_select",
                   "lbfz_batch_restart_fields", "lbfz_batch_fields_all",
                   "lbfz_batch_restart_many"):
            getattr(L, nm).restype = ctypes.c_int
        _lib = L
    return _lib


def lbfz_strerror(code: int) -> str:
    return lib().lbfz_strerror(int(code)).decode()


def make_params(cfg: dict, storage: str = "f32") -> lbfz_params:
    P = lbfz_params()
    for k in _INTS:
        setattr(P, k, int(cfg.get(k, 0)))
    if P.dim == 2:
        P.nz = 1
    P.storage = STORAGE[storage]
    P.contact_angle_deg = int(cfg.get("contact_angle_deg", 90))
    for k in _DOUBLES:
        setattr(P, k, float(cfg[k]))
    bf = cfg.get("body_force", (0.0, 0.0, 0.0))
    for a in range(3):
        P.body_force[a] = float(bf[a])
    return P


def _check(rc: int, where: str):
    if rc != LBFZ_OK:
        raise LbfzError(rc, where)


def lbfz_workspace_bytes(cfg: dict, storage: str = "f32") -> int:
    P = make_params(cfg, storage)
    n = ctypes.c_size_t()
    _check(lib().lbfz_workspace_bytes(ctypes.byref(P), ctypes.byref(n)), "lbfz_workspace_bytes")
    return n.value


def lbfz_create(cfg, phi, T, C, mask, ws_ptr: int, ws_bytes: int, stream_ptr: int,
                storage: str = "f32") -> ctypes.c_void_p:
    P = make_params(cfg, storage)
    arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (phi, T, C)]
    dp = ctypes.POINTER(ctypes.c_double)
    mptr = None
    if mask is not None:
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        mptr = m.ctypes.data_as(ctypes.c_void_p)
    h = ctypes.c_void_p()
    rc = lib().lbfz_create(ctypes.byref(P), *[a.ctypes.data_as(dp) for a in arrs], mptr,
                           ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes),
                           ctypes.c_void_p(stream_ptr), ctypes.byref(h))
    _check(rc, "lbfz_create")
    return h


def lbfz_step(h, nsteps: int):
    _check(lib().lbfz_step(h, int(nsteps)), "lbfz_step")


def lbfz_fields(h, mask_bits: int, ptrs, dst_is_device: bool):
    arr = (ctypes.c_void_p * len(FIELDS))(*[ctypes.c_void_p(p) for p in ptrs])
    _check(lib().lbfz_fields(h, ctypes.c_uint32(mask_bits), arr, int(dst_is_device)),
           "lbfz_fields")


def lbfz_totals(h) -> dict:
    t = lbfz_totals_t()
    _check(lib().lbfz_totals(h, ctypes.byref(t)), "lbfz_totals")
    return {k: getattr(t, k) for k, _ in lbfz_totals_t._fields_}


def lbfz_state_floats(h) -> int:
    n = ctypes.c_size_t()
    _check(lib().lbfz_state_floats(h, ctypes.byref(n)), "lbfz_state_floats")
    return n.value


def lbfz_get_state(h) -> np.ndarray:
    out = np.empty(lbfz_state_floats(h), dtype=np.float32)
    _check(lib().lbfz_get_state(h, out.ctypes.data_as(ctypes.c_void_p)), "lbfz_get_state")
    return out


def lbfz_set_state(h, arr) -> None:
    a = np.ascontiguousarray(arr, dtype=np.float32).reshape(-1)
    if a.size != lbfz_state_floats(h):
        raise ValueError("state size does not match the solver")
    _check(lib().lbfz_set_state(h, a.ctypes.data_as(ctypes.c_void_p)), "lbfz_set_state")


RESTART_FIELDS = ("phi", "fl", "T", "C", "ux", "uy", "p")


def _field_ptrs(planes):
    if len(planes) != len(RESTART_FIELDS):
        raise ValueError(f"restart takes {len(RESTART_FIELDS)} planes {RESTART_FIELDS}")
    return (ctypes.c_void_p * len(planes))(*[t.data_ptr() for t in planes])


def lbfz_restart_fields(h, planes) -> None:
    """planes: device tensors (FP32, N values each) in RESTART_FIELDS order."""
    _check(lib().lbfz_restart_fields(h, _field_ptrs(planes)), "lbfz_restart_fields")


def lbfz_stream_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream_ptr: int) -> None:
    _check(lib().lbfz_stream_copy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr),
                                  int(nbytes), ctypes.c_void_p(stream_ptr)), "lbfz_stream_copy")


def lbfz_stream_planes(dst_ptr: int, src_ptr: int, nx: int, ny: int, plane_stride: int,
                       stream_ptr: int) -> None:
    _check(lib().lbfz_stream_planes(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), nx, ny,
                                    int(plane_stride), ctypes.c_void_p(stream_ptr)),
           "lbfz_stream_planes")


def lbfz_stream_planes3d(dst_ptr: int, src_ptr: int, nx: int, ny: int, nz: int,
                         plane_stride: int, nread: int, nwrite: int, stream_ptr: int) -> None:
    _check(lib().lbfz_stream_planes3d(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), nx, ny,
                                      nz, int(plane_stride), nread, nwrite,
                                      ctypes.c_void_p(stream_ptr)), "lbfz_stream_planes3d")


def lbfz_sync(h):
    _check(lib().lbfz_sync(h), "lbfz_sync")


def lbfz_destroy(h):
    lib().lbfz_destroy(h)


class Solver:
    """A solver state on one GPU.  ``cfg`` is a parameter dictionary (see
    ``workloads.base_params``), phi/T/C the initial fields (C-order)."""

    def __init__(self, cfg: dict, phi, T, C, mask=None, device: int = 0, storage: str = "f32",
                 stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the lbfz solver runs on the GPU only")
        self.cfg = dict(cfg)
        self.device = torch.device("cuda", device)
        self.storage = storage
        nbytes = lbfz_workspace_bytes(cfg, storage)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.shape = ((cfg["nz"], cfg["ny"], cfg["nx"]) if cfg["dim"] == 3
                      else (cfg["ny"], cfg["nx"]))
        self.N = int(np.prod(self.shape))
        self._h = lbfz_create(cfg, phi, T, C, mask, self.workspace.data_ptr(), nbytes,
                              self.stream.cuda_stream, storage)

    def close(self, _destroy=lbfz_destroy):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter exit: the library may be unloaded already
            pass

    def step(self, n: int = 1):
        lbfz_step(self._h, n)

    def sync(self):
        lbfz_sync(self._h)

    def fields(self, names=FIELDS, device: bool = False) -> dict:
        """Macroscopic fields at the current time level (FP32).  device=True
        returns torch tensors on the GPU (no host copy)."""
        import torch
        bits = 0
        out = {}
        ptrs = [0] * len(FIELDS)
        for k, nm in enumerate(FIELDS):
            if nm in names:
                bits |= 1 << k
                if device:
                    t = torch.empty(self.shape, dtype=torch.float32, device=self.device)
                else:
                    t = np.empty(self.shape, dtype=np.float32)
                out[nm] = t
                ptrs[k] = t.data_ptr() if device else t.ctypes.data
        lbfz_fields(self._h, bits, ptrs, device)
        return out

    def totals(self) -> dict:
        return lbfz_totals(self._h)

    def get_state(self) -> np.ndarray:
        """Raw state as (planes, *shape) FP32, in the order of lbfz.h."""
        return lbfz_get_state(self._h).reshape((-1,) + self.shape)

    def set_state(self, arr) -> None:
        lbfz_set_state(self._h, arr)

    def restart_fields(self, planes) -> None:
        """Equilibrium restart from device planes (RESTART_FIELDS order)."""
        lbfz_restart_fields(self._h, planes)


# --------------------------------------------------------------------------
# batched sweep

def lbfz_batch_workspace_bytes(cfgs, storage: str = "f32") -> int:
    P = (lbfz_params * len(cfgs))(*[make_params(c, storage) for c in cfgs])
    n = ctypes.c_size_t()
    _check(lib().lbfz_batch_workspace_bytes(len(cfgs), P, ctypes.byref(n)),
           "lbfz_batch_workspace_bytes")
    return n.value


def lbfz_batch_create(cfgs, fields, ws_ptr: int, ws_bytes: int, stream_ptr: int,
                      storage: str = "f32") -> ctypes.c_void_p:
    """fields: one (phi, T, C) triple per grid."""
    n = len(cfgs)
    P = (lbfz_params * n)(*[make_params(c, storage) for c in cfgs])
    dp = ctypes.POINTER(ctypes.c_double)
    keep = [[np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in f] for f in fields]
    ptrs = [(dp * n)(*[keep[i][k].ctypes.data_as(dp) for i in range(n)]) for k in range(3)]
    b = ctypes.c_void_p()
    rc = lib().lbfz_batch_create(n, P, ptrs[0], ptrs[1], ptrs[2], ctypes.c_void_p(ws_ptr),
                                 ctypes.c_size_t(ws_bytes), ctypes.c_void_p(stream_ptr),
                                 ctypes.byref(b))
    _check(rc, "lbfz_batch_create")
    return b


def lbfz_batch_tune(b, trial_steps: int):
    _check(lib().lbfz_batch_tune(b, int(trial_steps)), "lbfz_batch_tune")


def lbfz_batch_step(b, nsteps: int):
    _check(lib().lbfz_batch_step(b, int(nsteps)), "lbfz_batch_step")


def lbfz_batch_step_sequential(b, nsteps: int):
    _check(lib().lbfz_batch_step_sequential(b, int(nsteps)), "lbfz_batch_step_sequential")


def lbfz_batch_groups(b) -> list:
    n = lib().lbfz_batch_groups(b)
    if n < 0:
        raise LbfzError(n, "lbfz_batch_groups")
    out = []
    for g in range(n):
        v = [ctypes.c_int32() for _ in range(5)]
        _check(lib().lbfz_batch_group_config(b, g, *[ctypes.byref(x) for x in v]),
               "lbfz_batch_group_config")
        out.append(dict(zip(("nx", "ny", "ncases", "tile_rows", "grid_blocks"),
                            [x.value for x in v])))
    return out


def lbfz_batch_fields(b, i: int, mask_bits: int, ptrs, dst_is_device: bool):
    arr = (ctypes.c_void_p * len(FIELDS))(*[ctypes.c_void_p(p) for p in ptrs])
    _check(lib().lbfz_batch_fields(b, int(i), ctypes.c_uint32(mask_bits), arr,
                                   int(dst_is_device)), "lbfz_batch_fields")


def lbfz_batch_totals(b, i: int) -> dict:
    t = lbfz_totals_t()
    _check(lib().lbfz_batch_totals(b, int(i), ctypes.byref(t)), "lbfz_batch_totals")
    return {k: getattr(t, k) for k, _ in lbfz_totals_t._fields_}


def lbfz_batch_select(b, idx) -> None:
    idx = [int(i) for i in idx]
    arr = (ctypes.c_int32 * max(len(idx), 1))(*idx)
    _check(lib().lbfz_batch_select(b, len(idx), arr), "lbfz_batch_select")


def lbfz_batch_restart_fields(b, i: int, planes) -> None:
    _check(lib().lbfz_batch_restart_fields(b, int(i), _field_ptrs(planes)),
           "lbfz_batch_restart_fields")


def lbfz_batch_destroy(b):
    lib().lbfz_batch_destroy(b)


class Batch:
    """Many independent 2D grids on one GPU, advanced together (the batched
    sweep).  ``cases``: a list of (params, phi, T, C)."""

    def __init__(self, cases, device: int = 0, storage: str = "f32", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the lbfz solver runs on the GPU only")
        self.cfgs = [dict(c[0]) for c in cases]
        self.shapes = [(c["ny"], c["nx"]) for c in self.cfgs]
        self.device = torch.device("cuda", device)
        nbytes = lbfz_batch_workspace_bytes(self.cfgs, storage)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._b = lbfz_batch_create(self.cfgs, [c[1:] for c in cases],
                                    self.workspace.data_ptr(), nbytes, self.stream.cuda_stream,
                                    storage)

    def close(self, _destroy=lbfz_batch_destroy):
        b = getattr(self, "_b", None)
        if b is not None and b.value:
            _destroy(b)
        self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter exit: the library may be unloaded already
            pass

    def tune(self, trial_steps: int = 8):
        lbfz_batch_tune(self._b, trial_steps)

    def step(self, n: int = 1):
        lbfz_batch_step(self._b, n)

    def step_sequential(self, n: int = 1):
        lbfz_batch_step_sequential(self._b, n)

    def groups(self) -> list:
        return lbfz_batch_groups(self._b)

    def fields(self, i: int, names=FIELDS) -> dict:
        bits = 0
        out = {}
        ptrs = [0] * len(FIELDS)
        for k, nm in enumerate(FIELDS):
            if nm in names:
                bits |= 1 << k
                t = np.empty(self.shapes[i], dtype=np.float32)
                out[nm] = t
                ptrs[k] = t.ctypes.data
        lbfz_batch_fields(self._b, i, bits, ptrs, False)
        return out

    def fields_to_device(self, i: int, planes) -> None:
        """The first len(planes) fields of grid i (order FIELDS) into the given
        device tensors (asynchronous on the stream)."""
        bits = 0
        ptrs = [0] * len(FIELDS)
        for k, t in enumerate(planes):
            bits |= 1 << k
            ptrs[k] = t.data_ptr()
        lbfz_batch_fields(self._b, i, bits, ptrs, True)

    def totals(self, i: int) -> dict:
        return lbfz_batch_totals(self._b, i)

    def restart_many(self, idx, planes, strides) -> None:
        """Equilibrium restart of the grids idx: field m (RESTART_FIELDS) of
        grid i at planes[m] (a device tensor) + i * strides[m] floats."""
        idx = [int(i) for i in idx]
        if not idx:
            return
        arr = (ctypes.c_int32 * len(idx))(*idx)
        ptrs = (ctypes.c_void_p * 7)(*[t.data_ptr() for t in planes])
        st = (ctypes.c_int64 * 7)(*[int(v) for v in strides])
        _check(lib().lbfz_batch_restart_many(self._b, len(idx), arr, ptrs, st),
               "lbfz_batch_restart_many")

    def fields_all_to_device(self, nfields: int, dst, case_stride: int = 0) -> None:
        """The first nfields fields (order FIELDS) of every grid into device
        memory at dst (a tensor or a view of one; asynchronous): grid i's
        planes at dst + i * case_stride floats (default: dst is
        [grids][nfields][...] and the stride its per-grid size)."""
        per = case_stride or dst.numel() // dst.shape[0]
        _check(lib().lbfz_batch_fields_all(self._b, (1 << nfields) - 1, dst.data_ptr(), per),
               "lbfz_batch_fields_all")

    def select(self, idx=()) -> None:
        """Later steps advance only the grids in idx (empty: all)."""
        lbfz_batch_select(self._b, idx)

    def restart_fields(self, i: int, planes) -> None:
        """Equilibrium restart of grid i from device planes (RESTART_FIELDS)."""
        lbfz_batch_restart_fields(self._b, i, planes)
