"""ctypes marshalling for include/tn.h (no arithmetic happens here)."""
from __future__ import annotations

import collections.abc as _abc
import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libtn.so")

if not os.path.exists(library_path):
    raise ImportError(
        f"{library_path} is missing: build it with `python paper_1908_08553_amd/build.py`")

# PyTorch bundles its own HIP runtime under the same soname
# (libamdhip64.so.7).  Loading torch first makes libtn.so bind to that
# already-loaded runtime, so the process holds exactly one HIP runtime and the
# library sees the same devices, streams and allocations as torch.
import torch  # noqa: E402,F401

lib = C.CDLL(library_path)

TN_OK, TN_PENDING = 0, 1
TN_EINVAL, TN_ENOMEM, TN_EBUSY, TN_EDEVICE = -1, -2, -3, -4
TN_ENOTFOUND, TN_ENONFINITE, TN_EOVERFLOW = -5, -6, -7
TN_ORDER_COLSWEEP, TN_ORDER_QUADRANT, TN_ORDER_HEURISTIC, TN_ORDER_SWEEP_AUTO = 0, 1, 2, 3
TN_ORDER_ROWS, TN_ORDER_ROWS_T = 4, 5
TN_PREC_F64, TN_PREC_F32, TN_PREC_BF16X3 = 0, 1, 2

_ORDERS = {"colsweep": 0, "quadrant": 1, "heuristic": 2, "sweep_auto": 3, "rows": 4,
           "rows_t": 5}
_PRECS = {"f64": 0, "f32": 1, "bf16x3": 2}


class tn_grid(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("D", C.c_int32),
                ("hdim", C.POINTER(C.c_int32)), ("vdim", C.POINTER(C.c_int32))]


class tn_result(C.Structure):
    _fields_ = [("sign", C.c_int32), ("status", C.c_int32), ("log_abs", C.c_double),
                ("value", C.c_double), ("mantissa", C.c_double), ("exp2_sum", C.c_int64)]


class tn_plan_info(C.Structure):
    _fields_ = [("order", C.c_int32), ("transpose", C.c_int32), ("quad_h", C.c_int32),
                ("quad_w", C.c_int32), ("n_steps", C.c_int32), ("n_units", C.c_int32),
                ("n_slots", C.c_int32), ("n_links", C.c_int32),
                ("peak_entries", C.c_int64), ("flops", C.c_int64),
                ("moved_entries", C.c_int64), ("workspace_bytes", C.c_int64 * 3),
                ("hbm_bytes", C.c_int64 * 3), ("ring_slices", C.c_int32 * 3),
                ("reserved2", C.c_int32), ("buffer_entries", C.c_int64)]


_P = C.c_void_p
lib.tn_last_error.restype = C.c_char_p
lib.tn_last_error.argtypes = []
lib.tn_plan_grid.restype = C.c_int32
lib.tn_plan_grid.argtypes = [C.POINTER(tn_grid), C.c_int32, C.c_int32, C.c_int32, C.POINTER(_P)]
lib.tn_plan_grid_budget.restype = C.c_int32
lib.tn_plan_grid_budget.argtypes = [C.POINTER(tn_grid), C.c_int32, C.c_int32, C.c_int32,
                                    C.c_int64, C.POINTER(_P)]
lib.tn_plan_stats.restype = C.c_int32
lib.tn_plan_stats.argtypes = [_P, C.POINTER(tn_plan_info)]
lib.tn_plan_text.restype = C.c_int32
lib.tn_plan_text.argtypes = [_P, C.c_char_p, C.POINTER(C.c_size_t)]
lib.tn_plan_free.restype = None
lib.tn_plan_free.argtypes = [_P]
lib.tn_set_option.restype = C.c_int32
lib.tn_set_option.argtypes = [C.c_int32, C.c_int64]
lib.tn_profile_enable.restype = C.c_int32
lib.tn_profile_enable.argtypes = [C.c_int32]
class tn_batch_config(C.Structure):
    _fields_ = [("threads", C.c_int32), ("split", C.c_int32)]


lib.tn_batch_workspace.restype = C.c_int32
lib.tn_batch_workspace.argtypes = [C.POINTER(_P), C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
lib.tn_batch_create.restype = C.c_int32
lib.tn_batch_create.argtypes = [C.POINTER(_P), C.c_int32, C.c_int32, C.POINTER(tn_batch_config),
                                _P, C.c_size_t, C.POINTER(_P)]
lib.tn_batch_run.restype = C.c_int32
lib.tn_batch_run.argtypes = [_P, C.POINTER(C.POINTER(C.c_void_p)), _P, C.POINTER(tn_result)]
lib.tn_batch_destroy.restype = C.c_int32
lib.tn_batch_destroy.argtypes = [_P]
lib.tn_contract_batch.restype = C.c_int32
lib.tn_contract_batch.argtypes = [C.POINTER(_P), C.POINTER(C.POINTER(C.c_void_p)), C.c_int32,
                                  C.c_int32, _P, C.c_size_t, _P, C.POINTER(tn_result)]
lib.tn_contract_grid.restype = C.c_int32
lib.tn_contract_grid.argtypes = [_P, C.POINTER(C.c_void_p), C.c_int32, C.c_int32, _P,
                                 C.c_size_t, _P, C.POINTER(tn_result)]
lib.tn_contract_grid_static.restype = C.c_int32
lib.tn_contract_grid_static.argtypes = [_P, C.POINTER(C.c_void_p), C.c_int32, C.c_int32, _P,
                                        C.POINTER(tn_result)]
TN_STATIC_SCRATCH_BYTES = 160 << 20


class tn_double_layer_site(C.Structure):
    _fields_ = [("A", C.c_void_p), ("op", C.c_void_p), ("E", C.c_void_p), ("d", C.c_int32),
                ("rank", C.c_int32), ("dims", C.c_int32 * 4), ("perm", C.c_int32 * 4)]


lib.tn_double_layer.restype = C.c_int32
lib.tn_double_layer.argtypes = [C.POINTER(tn_double_layer_site), C.c_int32, _P]
lib.tn_observables.restype = C.c_int32
lib.tn_observables.argtypes = [C.POINTER(tn_result), C.c_int32, C.c_int32,
                               C.POINTER(C.c_double), C.POINTER(C.c_double),
                               C.POINTER(C.c_double)]


class TnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"tn status {status}: {msg}")
        self.status = status


def _check(status: int) -> int:
    if status < 0:
        raise TnError(status, lib.tn_last_error().decode())
    return status


@dataclass
class Result:
    sign: int
    status: int
    log_abs: float
    value: float
    mantissa: float
    exp2_sum: int

    @classmethod
    def from_c(cls, r: tn_result) -> "Result":
        return cls(r.sign, r.status, r.log_abs, r.value, r.mantissa, r.exp2_sum)


class Results(_abc.Sequence):
    """The records of a batch of contractions, in the C array the library
    wrote: one numpy array per field (``.log_abs``, ``.mantissa``, ...) and a
    Result per index, built when it is read."""

    _DT = None

    def __init__(self, outs):
        import numpy as np
        if Results._DT is None:
            Results._DT = np.dtype([("sign", np.int32), ("status", np.int32),
                                    ("log_abs", np.float64), ("value", np.float64),
                                    ("mantissa", np.float64), ("exp2_sum", np.int64)])
            assert Results._DT.itemsize == C.sizeof(tn_result)
        self._outs = outs
        self._a = np.frombuffer(outs, dtype=Results._DT)

    def __len__(self):
        return len(self._a)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[j] for j in range(*i.indices(len(self)))]
        r = self._a[i]
        return Result(int(r["sign"]), int(r["status"]), float(r["log_abs"]), float(r["value"]),
                      float(r["mantissa"]), int(r["exp2_sum"]))

    def __getattr__(self, name):
        if name in ("sign", "status", "log_abs", "value", "mantissa", "exp2_sum"):
            return self._a[name]
        raise AttributeError(name)


def _int_array(v) -> Optional[C.Array]:
    if v is None:
        return None
    import numpy as np
    flat = [int(x) for x in np.asarray(v, dtype=np.int64).reshape(-1)]
    return (C.c_int32 * max(len(flat), 1))(*flat)


class Plan:
    """Owns a tn_plan*; freed when garbage-collected."""

    def __init__(self, handle: int, grid_keepalive=None):
        self._h = C.c_void_p(handle)
        self._keep = grid_keepalive

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.tn_plan_free(self._h)
            self._h = None

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def info(self) -> dict:
        return tn_plan_stats(self)

    def text(self) -> str:
        return tn_plan_text(self)


def tn_plan_grid(rows: int, cols: int, D: int = 2, hdim=None, vdim=None,
                 order=TN_ORDER_COLSWEEP, quad_h: int = 0, quad_w: int = 0,
                 budget: int = 0) -> Plan:
    """tn_plan_grid, or tn_plan_grid_budget when ``budget`` (the most entries
    of intermediate storage) is positive."""
    if isinstance(order, str):
        order = _ORDERS[order]
    h = _int_array(hdim)
    v = _int_array(vdim)
    g = tn_grid(rows, cols, D,
                C.cast(h, C.POINTER(C.c_int32)) if h is not None else None,
                C.cast(v, C.POINTER(C.c_int32)) if v is not None else None)
    out = C.c_void_p()
    if budget > 0:
        _check(lib.tn_plan_grid_budget(C.byref(g), order, quad_h, quad_w, int(budget),
                                       C.byref(out)))
    else:
        _check(lib.tn_plan_grid(C.byref(g), order, quad_h, quad_w, C.byref(out)))
    return Plan(out.value)


def tn_plan_stats(plan: Plan) -> dict:
    info = tn_plan_info()
    _check(lib.tn_plan_stats(plan.handle, C.byref(info)))
    return {"order": info.order, "transpose": info.transpose,
            "quad": (info.quad_h, info.quad_w), "n_steps": info.n_steps,
            "n_units": info.n_units, "n_slots": info.n_slots, "n_links": info.n_links,
            "buffer_entries": info.buffer_entries,
            "peak_entries": info.peak_entries, "flops": info.flops,
            "moved_entries": info.moved_entries,
            "workspace_bytes": list(info.workspace_bytes),
            "hbm_bytes": list(info.hbm_bytes),
            "ring_slices": list(info.ring_slices)}


def tn_plan_text(plan: Plan) -> str:
    n = C.c_size_t(0)
    lib.tn_plan_text(plan.handle, None, C.byref(n))
    buf = C.create_string_buffer(n.value)
    _check(lib.tn_plan_text(plan.handle, buf, C.byref(n)))
    return buf.value.decode()


def tn_contract_grid(plan: Plan, site_ptrs, sites_on_device: bool,
                     precision: int, workspace_ptr: int, ws_bytes: int,
                     stream_ptr: int) -> Result:
    arr = site_ptrs if isinstance(site_ptrs, C.Array) else (C.c_void_p * len(site_ptrs))(*site_ptrs)
    out = tn_result()
    status = lib.tn_contract_grid(plan.handle, arr, 1 if sites_on_device else 0, precision,
                                  C.c_void_p(workspace_ptr), ws_bytes, C.c_void_p(stream_ptr),
                                  C.byref(out))
    if status == TN_ENONFINITE:
        return Result.from_c(out)
    _check(status)
    return Result.from_c(out)


def tn_contract_grid_static(plan: Plan, site_ptrs, sites_on_device: bool, precision: int,
                            stream_ptr: int) -> Result:
    """tn_contract_grid in the library's static device workspace (no
    allocation by the library or here)."""
    arr = site_ptrs if isinstance(site_ptrs, C.Array) else (C.c_void_p * len(site_ptrs))(*site_ptrs)
    out = tn_result()
    status = lib.tn_contract_grid_static(plan.handle, arr, 1 if sites_on_device else 0,
                                         precision, C.c_void_p(stream_ptr), C.byref(out))
    if status == TN_ENONFINITE:
        return Result.from_c(out)
    _check(status)
    return Result.from_c(out)


TN_OPT_KERNEL_IMPL = 0
TN_OPT_BATCH_THREADS = 1
TN_OPT_FUSE_STEPS = 2
TN_OPT_CHUNK_SCHEDULE = 3
TN_OPT_QUADRANT_STREAMS = 4
TN_OPT_CHAIN_STEPS = 5
TN_OPT_ENV_STREAMS = 6
TN_OPT_ENV_ROWS = 7
TN_OPT_ENV_SITES = 8
TN_OPT_RING_OPERAND_SCALE = 9
TN_OPT_CHUNK_STREAM = 10


class tn_kernel_stat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double)]


lib.tn_profile_read.restype = C.c_int32
lib.tn_profile_read.argtypes = [C.POINTER(tn_kernel_stat), C.c_int32, C.POINTER(C.c_int32)]


def tn_profile_enable(on: bool) -> None:
    _check(lib.tn_profile_enable(1 if on else 0))


def tn_profile_read(cap: int = 64):
    """Per-kernel totals recorded since tn_profile_enable(True), as dicts."""
    arr = (tn_kernel_stat * cap)()
    n = C.c_int32(0)
    _check(lib.tn_profile_read(arr, cap, C.byref(n)))
    return [{"name": arr[i].name.decode(), "launches": arr[i].launches,
             "total_ms": arr[i].total_ms, "bytes": arr[i].bytes, "flops": arr[i].flops}
            for i in range(min(n.value, cap))]


def tn_set_option(option: int, value: int) -> None:
    _check(lib.tn_set_option(option, value))


# ------------------------------------------------------------ conveniences

plan_grid = tn_plan_grid


def device_sites(sites, device="cuda"):
    """Copy float64 site arrays to the GPU as contiguous torch tensors."""
    import torch
    return [torch.as_tensor(s, dtype=torch.float64).contiguous().to(device) for s in sites]


def workspace_for(plan: Plan, precision: int, device="cuda"):
    import torch
    nbytes = plan.info()["workspace_bytes"][precision]
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


class Sites:
    """Device sites checked once, with their pointer table, for repeated
    contractions over the same tensors (keeps them alive)."""

    def __init__(self, sites):
        import torch
        self.keep = list(sites)
        for t in self.keep:
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                    and t.is_contiguous()):
                raise ValueError("device sites must be contiguous float64 device tensors")
        self.table = (C.c_void_p * len(self.keep))(*[t.data_ptr() for t in self.keep])

    def __len__(self):
        return len(self.keep)


def prepare_sites(sites) -> Sites:
    return Sites(sites)


def contract_grid(plan: Plan, sites, precision="f64", workspace=None, stream=None) -> Result:
    """Contract with device-resident torch sites (a list, or prepare_sites'
    Sites) or host numpy arrays."""
    import torch
    if isinstance(precision, str):
        precision = _PRECS[precision]
    if isinstance(sites, Sites):
        if workspace is None:
            workspace = workspace_for(plan, precision)
        if stream is None:
            stream = torch.cuda.current_stream()
        return tn_contract_grid(plan, sites.table, True, precision, workspace.data_ptr(),
                                workspace.numel() * workspace.element_size(), stream.cuda_stream)
    on_device = all(isinstance(s, torch.Tensor) and s.is_cuda for s in sites)
    if on_device:
        for s in sites:
            if s.dtype != torch.float64 or not s.is_contiguous():
                raise ValueError("device sites must be contiguous float64 tensors")
        ptrs = [s.data_ptr() for s in sites]
        keep = sites
    else:
        import numpy as np
        keep = [np.ascontiguousarray(np.asarray(s, dtype=np.float64)) for s in sites]
        ptrs = [a.ctypes.data for a in keep]
    if workspace is None:
        workspace = workspace_for(plan, precision)
    if stream is None:
        stream = torch.cuda.current_stream()
    res = tn_contract_grid(plan, ptrs, on_device, precision, workspace.data_ptr(),
                           workspace.numel() * workspace.element_size(), stream.cuda_stream)
    del keep
    return res


# ------------------------------------------------------------------ batches

def _plan_array(plans):
    return (C.c_void_p * len(plans))(*[p.handle.value for p in plans])


def _site_table(site_lists):
    rows = [(C.c_void_p * len(sl))(*[t.data_ptr() for t in sl]) for sl in site_lists]
    table = (C.POINTER(C.c_void_p) * len(rows))(*[C.cast(r, C.POINTER(C.c_void_p)) for r in rows])
    return table, rows


def tn_batch_workspace(plans, precision) -> int:
    if isinstance(precision, str):
        precision = _PRECS[precision]
    n = C.c_size_t(0)
    _check(lib.tn_batch_workspace(_plan_array(plans), len(plans), precision, C.byref(n)))
    return n.value


class Batch:
    """A tn_batch: device tables + captured launch graph for a fixed list of
    column-sweep plans.  `threads` of 0 uses the library default (see
    tn_set_option); the `split` costliest lattices run in lock-step across
    the GPU."""

    def __init__(self, plans, precision="f32", threads=0, device="cuda", split=0):
        import torch
        if isinstance(precision, str):
            precision = _PRECS[precision]
        self.plans = list(plans)
        self.precision = precision
        nbytes = tn_batch_workspace(self.plans, precision)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        cfg = tn_batch_config(threads, split)
        h = C.c_void_p()
        _check(lib.tn_batch_create(_plan_array(self.plans), len(self.plans), precision,
                                   C.byref(cfg), C.c_void_p(self.workspace.data_ptr()),
                                   self.workspace.numel(), C.byref(h)))
        self._h = h

    def prepare(self, site_lists):
        """Pointer tables of `site_lists` for repeated runs over the same tensors."""
        if len(site_lists) != len(self.plans):
            raise ValueError("one site list per plan")
        return _site_table(site_lists) + (site_lists,)

    def run(self, site_lists, stream=None, prepared=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        table, keep = prepared[:2] if prepared is not None else _site_table(site_lists)
        outs = (tn_result * len(self.plans))()
        status = lib.tn_batch_run(self._h, table, C.c_void_p(stream.cuda_stream), outs)
        if status not in (TN_OK, TN_ENONFINITE):
            _check(status)
        del keep
        return Results(outs)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.tn_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def tn_contract_batch(plans, site_lists, precision="f32", workspace=None, stream=None):
    import torch
    if isinstance(precision, str):
        precision = _PRECS[precision]
    if workspace is None:
        workspace = torch.empty(max(tn_batch_workspace(plans, precision), 256),
                                dtype=torch.uint8, device="cuda")
    if stream is None:
        stream = torch.cuda.current_stream()
    table, keep = _site_table(site_lists)
    outs = (tn_result * len(plans))()
    status = lib.tn_contract_batch(_plan_array(plans), table, len(plans), precision,
                                   C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                   C.c_void_p(stream.cuda_stream), outs)
    if status not in (TN_OK, TN_ENONFINITE):
        _check(status)
    del keep
    return Results(outs)


# ------------------------------------------------------- cached environments
lib.tn_envset_workspace.argtypes = [C.POINTER(tn_grid), C.c_int32, C.c_int32,
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_size_t)]
lib.tn_envset_workspace.restype = C.c_int32
lib.tn_envset_create.argtypes = [C.POINTER(tn_grid), C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                 C.POINTER(C.c_int32), _P, C.c_size_t, C.POINTER(_P)]
lib.tn_envset_create.restype = C.c_int32
lib.tn_envset_run.argtypes = [_P, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), _P,
                              C.POINTER(tn_result)]
lib.tn_envset_run.restype = C.c_int32
lib.tn_envset_destroy.argtypes = [_P]
lib.tn_envset_destroy.restype = C.c_int32


class EnvSet:
    """A tn_envset: networks equal to a base network except at a few sites,
    contracted with cached left and right column environments.

    networks: one list of row-major site indices per network (the sites it
    replaces).  run(base, subst) takes the base network's rows*cols device
    sites and, per network, the replacing device sites in the same order;
    it returns [base result] + one result per network."""

    def __init__(self, rows, cols, D=2, hdim=None, vdim=None, networks=(), precision="f64",
                 device="cuda"):
        import torch
        if isinstance(precision, str):
            precision = _PRECS[precision]
        self.rows, self.cols, self.precision = rows, cols, precision
        self.networks = [list(map(int, n)) for n in networks]
        h = _int_array(hdim)
        v = _int_array(vdim)
        self._dims = (h, v)
        self._grid = tn_grid(rows, cols, D,
                             C.cast(h, C.POINTER(C.c_int32)) if h is not None else None,
                             C.cast(v, C.POINTER(C.c_int32)) if v is not None else None)
        counts = [len(n) for n in self.networks]
        flat = [i for n in self.networks for i in n]
        self._counts = (C.c_int32 * max(len(counts), 1))(*counts)
        self._flat = (C.c_int32 * max(len(flat), 1))(*flat)
        self.n_subst = len(flat)
        nbytes = C.c_size_t()
        _check(lib.tn_envset_workspace(C.byref(self._grid), precision, len(counts), self._counts,
                                       self._flat, C.byref(nbytes)))
        self.workspace = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=device)
        hd = C.c_void_p()
        _check(lib.tn_envset_create(C.byref(self._grid), precision, len(counts), self._counts,
                                    self._flat, C.c_void_p(self.workspace.data_ptr()),
                                    self.workspace.numel(), C.byref(hd)))
        self._h = hd

    def prepare(self, base, subst):
        """Pointer tables of (base, subst) for repeated runs over the same
        tensors (keeps them alive)."""
        import torch
        base, subst = list(base), list(subst)
        if len(base) != self.rows * self.cols:
            raise ValueError("one base site per lattice site")
        if len(subst) != self.n_subst:
            raise ValueError("one replacing site per substitution")
        for t in base + subst:
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                    and t.is_contiguous()):
                raise ValueError("sites must be contiguous float64 device tensors")
        b = (C.c_void_p * len(base))(*[t.data_ptr() for t in base])
        s = (C.c_void_p * max(len(subst), 1))(*[t.data_ptr() for t in subst])
        return b, s, (base, subst)

    def run(self, base=None, subst=None, stream=None, prepared=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        b, s, keep = prepared if prepared is not None else self.prepare(base, subst)
        outs = (tn_result * (len(self.networks) + 1))()
        status = lib.tn_envset_run(self._h, b, s, C.c_void_p(stream.cuda_stream), outs)
        if status not in (TN_OK, TN_ENONFINITE):
            _check(status)
        del keep
        return Results(outs)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.tn_envset_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


# ------------------------------------------------------------------ PEPS
def tn_double_layer_prepare(pairs):
    """Checked descriptor array of (A, op, E) or (A, op, E, perm) entries for
    repeated calls over the same tensors (it keeps them alive); perm lists
    which of A's bond legs each of E's bond legs is (default: the same)."""
    import torch
    arr = (tn_double_layer_site * max(len(pairs), 1))()
    for i, item in enumerate(pairs):
        A, op, E = item[:3]
        for t in (A, E) + ((op,) if op is not None else ()):
            if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("double-layer tensors must be contiguous float64 device tensors")
        dims = list(A.shape[1:])
        perm = list(item[3]) if len(item) > 3 else list(range(len(dims)))
        if len(dims) > 4 or sorted(perm) != list(range(len(dims))) or \
                tuple(E.shape) != tuple(dims[a] * dims[a] for a in perm):
            raise ValueError("E must have shape dims^2 of A's bond legs in perm order (at most 4)")
        arr[i] = tn_double_layer_site(A.data_ptr(), op.data_ptr() if op is not None else None,
                                      E.data_ptr(), A.shape[0], len(dims),
                                      (C.c_int32 * 4)(*(dims + [1] * (4 - len(dims)))),
                                      (C.c_int32 * 4)(*(perm + list(range(len(perm), 4)))))
    return arr, len(pairs), list(pairs)


def tn_double_layer(pairs, stream=None, prepared=None):
    """pairs: (A, op, E) device float64 tensors (op may be None): A [d][dims...],
    op [d][d], E [dims^2...] preallocated.  One asynchronous library call on
    `stream` (default: torch's current stream)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    arr, n, _ = prepared if prepared is not None else tn_double_layer_prepare(pairs)
    _check(lib.tn_double_layer(arr, n, C.c_void_p(stream.cuda_stream)))


def tn_observables(results, rows: int, cols: int):
    """(mx, mz, czz) lists from the results of a state's networks in the order
    tn.h documents (norm, S^x per site, S^z per site, S^z S^z per pair)."""
    n = rows * cols
    pairs = rows * (cols - 1) + (rows - 1) * cols
    if len(results) != 1 + 2 * n + pairs:
        raise ValueError("need 1 + 2 rows cols + pairs results")
    if isinstance(results, Results):
        res = results._outs
    else:
        res = (tn_result * len(results))()
        for i, r in enumerate(results):
            res[i] = tn_result(r.sign, r.status, r.log_abs, r.value, r.mantissa, r.exp2_sum)
    mx = (C.c_double * n)()
    mz = (C.c_double * n)()
    czz = (C.c_double * max(pairs, 1))()
    _check(lib.tn_observables(res, rows, cols, mx, mz, czz))
    return list(mx), list(mz), list(czz)[:pairs]


# ------------------------------------------------------------------ serving

class tn_server_info(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("queued", C.c_int64),
                ("active", C.c_int64), ("arena_bytes", C.c_int64), ("arena_in_use", C.c_int64),
                ("peak_arena_in_use", C.c_int64), ("peak_active", C.c_int64)]


lib.tn_server_create.restype = C.c_int32
lib.tn_server_create.argtypes = [_P, C.c_size_t, C.c_int32, C.c_int32, C.POINTER(_P)]
lib.tn_submit.restype = C.c_int32
lib.tn_submit.argtypes = [_P, C.POINTER(tn_grid), C.c_int32, C.c_int32,
                          C.POINTER(C.c_void_p), C.POINTER(C.c_uint64)]
lib.tn_poll_ex.restype = C.c_int32
lib.tn_poll_ex.argtypes = [_P, C.c_uint64, C.POINTER(tn_result), C.POINTER(C.c_int64)]
lib.tn_poll.restype = C.c_int32
lib.tn_poll.argtypes = [_P, C.c_uint64, C.POINTER(tn_result)]
lib.tn_server_stats.restype = C.c_int32
lib.tn_server_stats.argtypes = [_P, C.POINTER(tn_server_info)]
lib.tn_server_destroy.restype = C.c_int32
lib.tn_server_destroy.argtypes = [_P]


class Server:
    """A tn_server over a torch-allocated arena of `arena_bytes` bytes."""

    def __init__(self, arena_bytes: int, max_slots: int = 4, queue_depth: int = 4096,
                 device="cuda"):
        import torch
        self.arena = torch.empty(max(int(arena_bytes), 256), dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(lib.tn_server_create(C.c_void_p(self.arena.data_ptr()), self.arena.numel(),
                                    max_slots, queue_depth, C.byref(h)))
        self._h = h

    def submit(self, rows, cols, sites, D=2, hdim=None, vdim=None, order=TN_ORDER_HEURISTIC,
               precision="f64") -> int:
        import numpy as np
        if isinstance(order, str):
            order = _ORDERS[order]
        if isinstance(precision, str):
            precision = _PRECS[precision]
        h = _int_array(hdim)
        v = _int_array(vdim)
        g = tn_grid(rows, cols, D,
                    C.cast(h, C.POINTER(C.c_int32)) if h is not None else None,
                    C.cast(v, C.POINTER(C.c_int32)) if v is not None else None)
        keep = [np.ascontiguousarray(np.asarray(s, dtype=np.float64)) for s in sites]
        ptrs = (C.c_void_p * len(keep))(*[a.ctypes.data for a in keep])
        t = C.c_uint64(0)
        _check(lib.tn_submit(self._h, C.byref(g), order, precision, ptrs, C.byref(t)))
        return t.value

    def poll(self, ticket: int):
        """(status, Result or None, (t_submit, t_admit, t_done) ns)."""
        out = tn_result()
        times = (C.c_int64 * 3)()
        st = lib.tn_poll_ex(self._h, ticket, C.byref(out), times)
        if st == TN_PENDING:
            return st, None, None
        if st not in (TN_OK, TN_ENONFINITE):
            _check(st)
        return st, Result.from_c(out), tuple(times)

    def wait(self, ticket: int, timeout: float = 120.0):
        import time
        t0 = time.monotonic()
        while True:
            st, res, times = self.poll(ticket)
            if st != TN_PENDING:
                return res, times
            if time.monotonic() - t0 > timeout:
                raise TimeoutError(f"ticket {ticket} still pending after {timeout} s")
            time.sleep(50e-6)

    def stats(self) -> dict:
        i = tn_server_info()
        _check(lib.tn_server_stats(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in tn_server_info._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.tn_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


# ------------------------------------------------------------ imaginary time
class tn_ite_config(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("chi_max", C.c_int32),
                ("reserved", C.c_int32), ("J", C.c_double), ("gamma", C.c_double),
                ("eps", C.c_double)]


lib.tn_ite_workspace.restype = C.c_int32
lib.tn_ite_workspace.argtypes = [C.POINTER(tn_ite_config), C.POINTER(C.c_size_t)]
lib.tn_ite_create.restype = C.c_int32
lib.tn_ite_create.argtypes = [C.POINTER(tn_ite_config), _P, C.c_size_t, _P, C.POINTER(_P)]
lib.tn_ite_step.restype = C.c_int32
lib.tn_ite_step.argtypes = [_P, C.c_double, C.c_int32]
lib.tn_ite_energy.restype = C.c_int32
lib.tn_ite_energy.argtypes = [_P, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(C.c_double), C.POINTER(C.c_double)]
lib.tn_ite_sites.restype = C.c_int32
lib.tn_ite_sites.argtypes = [_P, C.POINTER(C.c_void_p)]
lib.tn_ite_destroy.restype = C.c_int32
lib.tn_ite_destroy.argtypes = [_P]


class Ite:
    """tn_ite over a torch-allocated workspace: imaginary-time evolution of a
    rows x cols PEPS for H = -J sum S^z S^z - gamma sum S^x (S = Pauli)."""

    def __init__(self, rows: int, cols: int, chi_max: int, J: float, gamma: float,
                 eps: float = 0.01, device="cuda"):
        import torch
        self.rows, self.cols, self.chi = rows, cols, chi_max
        self.cfg = tn_ite_config(rows, cols, chi_max, 0, J, gamma, eps)
        n = C.c_size_t(0)
        _check(lib.tn_ite_workspace(C.byref(self.cfg), C.byref(n)))
        self.ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib.tn_ite_create(C.byref(self.cfg), C.c_void_p(self.ws.data_ptr()),
                                 self.ws.numel(), C.c_void_p(self.stream.cuda_stream),
                                 C.byref(h)))
        self._h = h

    def step(self, dtau: float, n: int = 1):
        _check(lib.tn_ite_step(self._h, dtau, n))

    def energy(self):
        """(E, mx, mz, czz) of the current state."""
        n = self.rows * self.cols
        nb = self.rows * (self.cols - 1) + (self.rows - 1) * self.cols
        e = C.c_double()
        mx, mz, cz = (C.c_double * n)(), (C.c_double * n)(), (C.c_double * max(nb, 1))()
        _check(lib.tn_ite_energy(self._h, C.byref(e), mx, mz, cz))
        return e.value, list(mx), list(mz), list(cz)[:nb]

    def site_views(self):
        """The current site tensors as float64 torch views of the workspace
        (canonical shapes [2][chi]..[chi]); writing them sets the state."""
        import torch
        n = self.rows * self.cols
        ptrs = (C.c_void_p * n)()
        _check(lib.tn_ite_sites(self._h, ptrs))
        base = self.ws.data_ptr()
        out = []
        for k in range(n):
            r, c = divmod(k, self.cols)
            rank = (c > 0) + (r > 0) + (c < self.cols - 1) + (r < self.rows - 1)
            shape = (2,) + (self.chi,) * rank
            cnt = 2 * self.chi ** rank
            off = ptrs[k] - base
            out.append(self.ws[off:off + 8 * cnt].view(torch.float64).reshape(shape))
        return out

    def evolve(self, tau: float, steps: int, energy_every: int = 2):
        """`steps` Trotter steps of dtau = tau / steps; [(step, energy)] every
        `energy_every` steps (the paper's monitoring, §5)."""
        dtau = tau / steps
        out = []
        done = 0
        while done < steps:
            k = min(energy_every, steps - done) if energy_every else steps - done
            self.step(dtau, k)
            done += k
            if energy_every and done % energy_every == 0:
                out.append((done, self.energy()[0]))
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.tn_ite_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover
            pass
