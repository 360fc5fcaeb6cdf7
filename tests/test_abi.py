"""The C-ABI library loads, exports every symbol include/lbfz.h declares, and
rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2511_09422_amd import lbfz
from paper_2511_09422_amd.workloads import base_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(lbfz_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_exports_every_declared_symbol():
    L = lbfz.lib()
    names = _declared()
    assert {"lbfz_create", "lbfz_step", "lbfz_fields", "lbfz_totals"} <= set(names)
    for nm in names:
        assert hasattr(L, nm), nm


def test_params_struct_matches_header():
    # the ctypes mirror lists the header's fields in order
    txt = open(os.path.join(ROOT, "include", "lbfz.h")).read()
    body = txt[txt.index("typedef struct lbfz_params"):txt.index("} lbfz_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S).split("{", 1)[1]
    fields = re.findall(r"\b([a-zA-Z_][a-zA-Z0-9_]*)\s*(?:\[3\])?\s*[,;]", body)
    assert fields == [f for f, _ in lbfz.lbfz_params._fields_]


def test_conv_args_struct_matches_header():
    from paper_2511_09422_amd import surrogate
    txt = open(os.path.join(ROOT, "include", "lbfz_nn.h")).read()
    body = txt[txt.index("typedef struct lbfz_conv_args"):txt.index("} lbfz_conv_args;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S).split("{", 1)[1]
    fields = re.findall(r"\b([a-zA-Z_][a-zA-Z0-9_]*)\s*[,;]", body)
    mirror = [f.rstrip("_") for f, _ in surrogate.lbfz_conv_args._fields_]
    assert fields == mirror
    surrogate.nnlib()   # every kernel entry point binds


def test_strerror_and_workspace_errors():
    assert lbfz.lbfz_strerror(0) == "ok"
    assert "workspace" in lbfz.lbfz_strerror(lbfz.LBFZ_ENOMEM)
    cfg = base_params(nx=64, ny=64)
    assert lbfz.lbfz_workspace_bytes(cfg) > 64 * 64 * 24 * 4 * 2
    for bad in (dict(tau_phi=0.5), dict(nu=0.0), dict(eps=0.0), dict(nx=1),
                dict(contact_angle_deg=60)):
        with pytest.raises(lbfz.LbfzError) as e:
            lbfz.lbfz_workspace_bytes(base_params(**bad))
        assert e.value.code == lbfz.LBFZ_EINVAL


def test_create_rejects_bad_inputs_before_device_work():
    cfg = base_params(nx=16, ny=8)
    phi = np.zeros((8, 16))
    T = np.zeros((8, 16))
    C = np.zeros((8, 16))
    need = lbfz.lbfz_workspace_bytes(cfg)
    fake = 1 << 20          # never dereferenced: every check below fails first
    with pytest.raises(lbfz.LbfzError) as e:
        lbfz.lbfz_create(cfg, phi, T, C, None, fake, need - 256, 0)
    assert e.value.code == lbfz.LBFZ_ENOMEM
    with pytest.raises(lbfz.LbfzError) as e:
        lbfz.lbfz_create(cfg, phi, T, C, None, fake + 4, need, 0)
    assert e.value.code == lbfz.LBFZ_ENOMEM
    bad = T.copy()
    bad[3, 4] = np.nan
    with pytest.raises(lbfz.LbfzError) as e:
        lbfz.lbfz_create(cfg, phi, bad, C, None, fake, need, 0)
    assert e.value.code == lbfz.LBFZ_ENONFINITE
    with pytest.raises(lbfz.LbfzError) as e:
        lbfz.lbfz_create(cfg, phi, T, C, np.zeros((8, 16), np.uint8), fake, need, 0)
    assert e.value.code == lbfz.LBFZ_EINVAL
    with pytest.raises(lbfz.LbfzError) as e:
        lbfz.lbfz_create(base_params(nx=16, ny=8, tau_h=0.4), phi, T, C, None, fake, need, 0)
    assert e.value.code == lbfz.LBFZ_EINVAL


def test_tail_args_struct_and_conv_tail_rejections():
    """lbfz_tail_args mirrors the header, and lbfz_nn_conv_tail rejects each
    invalid argument before any launch (fake pointers, never dereferenced)."""
    from paper_2511_09422_amd import surrogate as sg
    txt = open(os.path.join(ROOT, "include", "lbfz_nn.h")).read()
    body = txt[txt.index("typedef struct lbfz_tail_args"):txt.index("} lbfz_tail_args;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S).split("{", 1)[1]
    fields = re.findall(r"\b([a-zA-Z_][a-zA-Z0-9_]*)\s*[,;]", body)
    assert fields == [f for f, _ in sg.lbfz_tail_args._fields_]
    L = sg.nnlib()
    fake = 1 << 20

    def args(**over):
        a = sg.lbfz_conv_args()
        a.in_, a.in_cs, a.in_co, a.Cin = fake, 32, 0, 32
        a.w, a.N, a.bias, a.out = fake, 32, fake, None
        a.out_cs, a.out_co, a.relu, a.sign = 32, 0, 1, 1
        a.B, a.H, a.W, a.taps, a.up = 2, 16, 16, 9, 0
        t = sg.lbfz_tail_args()
        t.head_w, t.head_b, t.nh, t.nf = fake, fake, 8, 6
        t.before, t.before_stride = fake, 6 * 256
        t.shift = t.scale = t.resid = fake
        t.pred, t.pred_stride = fake, 6 * 256
        for k, v in over.items():
            setattr(t if hasattr(t, k) else a, k, v)
        return a, t

    for bad in (dict(N=64), dict(Cin=48), dict(taps=1), dict(sign=-1), dict(up=1),
                dict(out_f32=1), dict(pool=fake), dict(nf=9), dict(nh=33), dict(nf=0),
                dict(before_stride=6 * 256 - 1), dict(pred_stride=100), dict(head_w=None),
                dict(pred=None), dict(in_=None), dict(out=fake, out_co=8)):
        a, t = args(**bad)
        assert L.lbfz_nn_conv_tail(ctypes.byref(a), ctypes.byref(t), None) == sg.LBFZ_NN_EINVAL, bad


def test_descriptor_range_limits_grid_size():
    """Every access goes through a buffer descriptor with a 32-bit byte range:
    a 3D FP32 grid whose 19-plane flow set spans 2^32 bytes or more (384^3:
    76 B x 56.6 M nodes) is rejected, the same grid with 16-bit storage (36 B
    per node in its widest set) is accepted, as is the largest 2D grid."""
    big = dict(dim=3, nx=384, ny=384, nz=384)
    with pytest.raises(lbfz.LbfzError) as e:
        lbfz.lbfz_workspace_bytes(base_params(**big))
    assert e.value.code == lbfz.LBFZ_EINVAL
    assert lbfz.lbfz_workspace_bytes(base_params(**big), "f16") > 0
    assert lbfz.lbfz_workspace_bytes(base_params(dim=3, nx=320, ny=320, nz=320)) > 0
    assert lbfz.lbfz_workspace_bytes(base_params(nx=8192, ny=8192)) > 0
