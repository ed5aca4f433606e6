"""MI355X-native surface flux transport (HipFT method) behind a C ABI.

``Ensemble`` marshals numpy arrays / torch device tensors to the functions of
``include/sft.h``; the HIP library does all the work.  torch is used only for
device memory and the HIP stream.
"""
from __future__ import annotations

import ctypes
from typing import Iterable, Optional

import numpy as np

from . import _abi
from ._abi import *  # noqa: F401,F403  (constants and structures)
from ._abi import check, load

__all__ = ["Ensemble", "load", "make_params", "make_options"]


def make_options(**kw) -> _abi.sft_options:
    o = _abi.sft_options()
    check(load().sft_options_default(ctypes.byref(o)), None, "sft_options_default")
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def make_params(r) -> _abi.sft_params:
    """sft_params from any object with the realization attributes (km^2/s, m/s)."""
    p = _abi.sft_params()
    for name in ("nu_km2_s", "d0", "d2", "d4", "m1", "m3", "m5", "alpha_mu", "mu_lim", "lat_lim_deg"):
        setattr(p, name, float(getattr(r, name)))
    p.flux_balance = int(getattr(r, "flux_balance", 0))
    p.att_b0 = float(getattr(r, "att_b0", 0.0))
    p.nu_grid_alpha = float(getattr(r, "nu_grid_alpha", 0.0))
    return p


def _ptr(a):
    """(pointer, dtype code, on_device) of a numpy array or torch tensor."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            if not a.is_contiguous():
                raise ValueError("tensor must be contiguous")
            code = {torch.float64: _abi.SFT_DTYPE_F64, torch.float32: _abi.SFT_DTYPE_F32}[a.dtype]
            return ctypes.c_void_p(a.data_ptr()), code, int(a.is_cuda)
    except ImportError:
        pass
    if not (isinstance(a, np.ndarray) and a.flags["C_CONTIGUOUS"]):
        raise ValueError("expected a C-contiguous numpy array or torch tensor")
    code = {np.dtype(np.float64): _abi.SFT_DTYPE_F64, np.dtype(np.float32): _abi.SFT_DTYPE_F32}[a.dtype]
    return ctypes.c_void_p(a.ctypes.data), code, 0


class Ensemble:
    """One library context: grid classes with realizations, advanced together."""

    def __init__(self, options: Optional[_abi.sft_options] = None, stream=None, **kw):
        self.L = load()
        self.opt = options if options is not None else make_options(**kw)
        # stream=None: the library creates its own blocking stream, ordered
        # with the null stream (torch's default stream)
        self.ctx = ctypes.c_void_p()
        check(self.L.sft_create(ctypes.byref(self.ctx), ctypes.byref(self.opt),
                                ctypes.c_void_p(stream or 0)), None, "sft_create")
        self.grids = []      # (nt, np, first_id, R)

    def _chk(self, st, what):
        return check(st, self.ctx, what)

    def add_grid(self, nt: int, np_: int, realizations: Iterable) -> int:
        gid = ctypes.c_int32()
        self._chk(self.L.sft_add_grid(self.ctx, nt, np_, ctypes.byref(gid)), "sft_add_grid")
        rs = list(realizations)
        arr = (_abi.sft_params * len(rs))(*[make_params(r) for r in rs])
        first = ctypes.c_int32()
        self._chk(self.L.sft_add_realizations(self.ctx, gid.value, len(rs), arr, ctypes.byref(first)),
                  "sft_add_realizations")
        self.grids.append((nt, np_, first.value, len(rs)))
        return gid.value

    def set_state(self, rid: int, br):
        p, code, dev = _ptr(br)
        self._chk(self.L.sft_set_state(self.ctx, rid, p, code, dev), "sft_set_state")

    def get_state(self, rid: int, out):
        p, code, dev = _ptr(out)
        self._chk(self.L.sft_get_state(self.ctx, rid, p, code, dev), "sft_get_state")
        return out

    def set_states(self, gid: int, br):
        p, code, dev = _ptr(br)
        self._chk(self.L.sft_set_states(self.ctx, gid, p, code, dev), "sft_set_states")

    def get_states(self, gid: int, out=None):
        if out is None:
            nt, np_, _, R = self.grids[gid]
            out = np.empty((R, nt, np_))
        p, code, dev = _ptr(out)
        self._chk(self.L.sft_get_states(self.ctx, gid, p, code, dev), "sft_get_states")
        return out

    def advance(self, t_end: float):
        self._chk(self.L.sft_advance(self.ctx, float(t_end)), "sft_advance")

    def assimilate(self, gid: int, data, weight=None, kind: int = _abi.SFT_WEIGHT_DISK,
                   b0_deg: float = 0.0, l0_deg: float = 0.0):
        p, code, dev = _ptr(data)
        if weight is not None:
            w, wcode, wdev = _ptr(weight)
            if wcode != code or wdev != dev:
                raise ValueError("data and weight must share dtype and device")
        else:
            w = ctypes.c_void_p(0)
        self._chk(self.L.sft_assimilate(self.ctx, gid, p, w, code, kind, float(b0_deg), float(l0_deg),
                                        dev), "sft_assimilate")

    def assimilate_noalloc(self, gid: int, data, weight=None, kind: int = _abi.SFT_WEIGHT_DISK,
                           b0_deg: float = 0.0, l0_deg: float = 0.0):
        """sft_assimilate_noalloc: device arrays only; allocates nothing."""
        p, code, dev = _ptr(data)
        if not dev:
            raise ValueError("sft_assimilate_noalloc takes device arrays")
        if weight is not None:
            w, wcode, wdev = _ptr(weight)
            if wcode != code or not wdev:
                raise ValueError("data and weight must share dtype and device")
        else:
            w = ctypes.c_void_p(0)
        self._chk(self.L.sft_assimilate_noalloc(self.ctx, gid, p, w, code, kind, float(b0_deg),
                                                float(l0_deg)), "sft_assimilate_noalloc")

    def diagnostics(self, rid: int) -> dict:
        d = _abi.sft_diag()
        st = self.L.sft_diagnostics(self.ctx, rid, ctypes.byref(d))
        out = {name: getattr(d, name) for name, _ in _abi.sft_diag._fields_ if name != "pad"}
        out["status"] = st
        if st not in (_abi.SFT_OK, _abi.SFT_ERR_NOT_FINITE):
            self._chk(st, "sft_diagnostics")
        return out

    def time(self) -> float:
        t = ctypes.c_double()
        self._chk(self.L.sft_time(self.ctx, ctypes.byref(t)), "sft_time")
        return t.value

    def set_time(self, t: float):
        self._chk(self.L.sft_set_time(self.ctx, float(t)), "sft_set_time")

    def sync(self):
        self._chk(self.L.sft_sync(self.ctx), "sft_sync")

    def counts(self, rid: int) -> dict:
        v = [ctypes.c_int64() for _ in range(4)]
        self._chk(self.L.sft_counts(self.ctx, rid, *[ctypes.byref(x) for x in v]), "sft_counts")
        return dict(zip(("steps", "stages", "adv_stages", "assim"), [x.value for x in v]))

    def set_timing(self, on: bool):
        self._chk(self.L.sft_set_timing(self.ctx, int(bool(on))), "sft_set_timing")

    def timing(self) -> dict:
        out = {}
        for fam, name in enumerate(_abi.KFAM_NAMES):
            ms, n, b, mb = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            self._chk(self.L.sft_get_timing(self.ctx, fam, ctypes.byref(ms), ctypes.byref(n),
                                            ctypes.byref(b), ctypes.byref(mb)), "sft_get_timing")
            out[name] = {"ms": ms.value, "launches": n.value, "bytes": b.value, "min_bytes": mb.value}
        return out

    def tile_choice(self, gid: int) -> int:
        v = ctypes.c_int32()
        self._chk(self.L.sft_tile_choice(self.ctx, gid, ctypes.byref(v)), "sft_tile_choice")
        return v.value

    def set_class_tile(self, gid: int, index: int):
        self._chk(self.L.sft_set_class_tile(self.ctx, gid, int(index)), "sft_set_class_tile")

    def close(self):
        if self.ctx:
            self.L.sft_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tile_info(precision: int, index: int):
    """(tx, ty, k, nthreads) of a blocked tile shape, or None past the table."""
    v = [ctypes.c_int32() for _ in range(4)]
    st = load().sft_tile_info(precision, index, *[ctypes.byref(x) for x in v])
    return tuple(x.value for x in v) if st == _abi.SFT_OK else None


class Net:
    """The CNN surrogate network (marshalling to the sft_net_* functions).

    Device arrays are torch CUDA tensors; host arrays numpy."""

    def __init__(self, nt: int, np_: int, max_batch: int, stream=None):
        self.L = load()
        self.h = ctypes.c_void_p()
        check(self.L.sft_net_create(ctypes.byref(self.h), nt, np_, max_batch,
                                    ctypes.c_void_p(stream or 0)), None, "sft_net_create")
        n = ctypes.c_int64()
        check(self.L.sft_net_param_count(self.h, ctypes.byref(n)), None, "sft_net_param_count")
        self.n = n.value
        self.nt, self.np, self.max_batch = nt, np_, max_batch

    def set_params(self, params):
        p, code, dev = _ptr(params)
        count = params.numel() if hasattr(params, "numel") else params.size
        if code != _abi.SFT_DTYPE_F32 or count != self.n:
            raise ValueError(f"expected {self.n} float32 parameters")
        check(self.L.sft_net_set_params(self.h, p, dev), None, "sft_net_set_params")

    def get_params(self, out=None):
        out = np.empty(self.n, np.float32) if out is None else out
        p, _, dev = _ptr(out)
        check(self.L.sft_net_get_params(self.h, p, dev), None, "sft_net_get_params")
        return out

    def get_grads(self, out=None):
        out = np.empty(self.n, np.float32) if out is None else out
        p, _, dev = _ptr(out)
        check(self.L.sft_net_get_grads(self.h, p, dev), None, "sft_net_get_grads")
        return out

    def forward(self, b_in, feats, y=None):
        p, code, _ = _ptr(b_in)
        f, _, _ = _ptr(feats)
        yp = _ptr(y)[0] if y is not None else ctypes.c_void_p(0)
        check(self.L.sft_net_forward(self.h, b_in.shape[0], p, code, f, yp), None, "sft_net_forward")
        return y

    def predict(self, b_in, feats, y=None):
        """Inference only (sft_net_predict): the same y as forward, without
        keeping the last hidden layer's activations."""
        p, code, _ = _ptr(b_in)
        f, _, _ = _ptr(feats)
        yp = _ptr(y)[0] if y is not None else ctypes.c_void_p(0)
        check(self.L.sft_net_predict(self.h, b_in.shape[0], p, code, f, yp), None, "sft_net_predict")
        return y

    def activation(self, layer: int, out):
        """Copies bf16 activations into a torch CUDA tensor (int16 storage)."""
        check(self.L.sft_net_get_activation(self.h, layer, ctypes.c_void_p(out.data_ptr())), None,
              "sft_net_get_activation")
        return out

    def train_step(self, b_in, b_target, feats, lr: float, apply: bool = True,
                   want_loss: bool = True) -> float:
        """One training step; returns the loss (and waits for it) if want_loss."""
        p, code, _ = _ptr(b_in)
        t, tcode, _ = _ptr(b_target)
        if tcode != code:
            raise ValueError("b_in and b_target must share dtype")
        f, _, _ = _ptr(feats)
        loss = ctypes.c_double(float("nan"))
        check(self.L.sft_net_train_step(self.h, b_in.shape[0], p, t, code, f, float(lr), int(apply),
                                        ctypes.byref(loss) if want_loss else None),
              None, "sft_net_train_step")
        return loss.value

    def set_grid_limit(self, max_blocks: int):
        """sft_net_set_grid_limit: at most max_blocks blocks per persistent launch (0: default)."""
        check(self.L.sft_net_set_grid_limit(self.h, int(max_blocks)), None, "sft_net_set_grid_limit")

    def sync(self):
        check(self.L.sft_net_sync(self.h), None, "sft_net_sync")

    def close(self):
        if self.h:
            self.L.sft_net_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def surrogate_advance(ens: "Ensemble", gid: int, net: Net, feats: np.ndarray, t_end: float, tol: float,
                      check_: int = 1):
    """sft_surrogate_advance (check_: 0 none, 1 every interval, K >= 2 every
    K-th interval per realization with escalation after a rejection); returns
    the per-realization relative L2 distances (-1 where not checked)."""
    feats = np.ascontiguousarray(feats, dtype=np.float32)
    R = ens.grids[gid][3]
    err = np.zeros(R)
    check(ens.L.sft_surrogate_advance(ens.ctx, gid, net.h, feats.ctypes.data_as(ctypes.c_void_p),
                                      float(t_end), float(tol), int(check_),
                                      err.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
          ens.ctx, "sft_surrogate_advance")
    return err


def surrogate_counts(ens: "Ensemble", rid: int) -> dict:
    """sft_surrogate_counts: accepted, rejected and unchecked surrogate
    intervals of a realization, and whether it is escalated."""
    v = [ctypes.c_int64() for _ in range(3)]
    esc = ctypes.c_int32()
    check(ens.L.sft_surrogate_counts(ens.ctx, rid, *[ctypes.byref(x) for x in v], ctypes.byref(esc)),
          ens.ctx, "sft_surrogate_counts")
    return {"accepted": v[0].value, "rejected": v[1].value, "unchecked": v[2].value, "escalated": esc.value}
