"""Python binding of the C ABI in ``include/qtn.h``, same names, marshalling only.

Arrays are converted with numpy; device workspaces are torch uint8 tensors on
the current HIP device and streams are torch streams.  Nothing here computes
any part of the energy: every call goes to ``libqtn.so``.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _capi
from ._capi import (QTN_C128, QTN_C64, QTN_MIXED, QtnError, check, lib, qtn_bucket_info,
                    qtn_batch_tune_report, qtn_config,
                    qtn_launch_rec, qtn_plan_stats, qtn_timing, qtn_tune_pick, qtn_tune_rec,
                    qtn_tune_report)

__all__ = [
    "QTN_C128", "QTN_C64", "QTN_MIXED", "QtnError", "qtn_network_build", "qtn_network_info",
    "qtn_order_minfill", "qtn_plan", "qtn_set_angles", "qtn_contract",
    "qtn_contract_timed", "qtn_contract_batch", "qtn_batch_workspace", "qtn_autotune_batch",
    "qtn_get_plan_stats", "qtn_bucket_widths", "qtn_slice_vars", "qtn_network_free",
    "qtn_last_error", "qtn_launch_log", "qtn_plan_order", "qtn_autotune",
    "qtn_autotune_angles", "qtn_tune_angles_workspace", "qtn_tune_log",
    "qtn_tune_picks", "qtn_set_tune_picks", "qtn_angles_workspace", "qtn_contract_angles",
    "qtn_gradient_workspace", "qtn_energy_gradient",
    "Network", "CostModel", "qtn_apply_costmodel", "workspace", "stream_handle",
    "qtn_bucket_plan", "qtn_bucket_get_info", "qtn_bucket_contract",
    "qtn_bucket_contract_noalloc", "qtn_bucket_contract_timed", "qtn_bucket_free",
    "Bucket",
]

_pi32 = ctypes.POINTER(ctypes.c_int32)
_pd = ctypes.POINTER(ctypes.c_double)


def _i32(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.int32).ravel())
    return a, a.ctypes.data_as(_pi32)


def _f64(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    return a, a.ctypes.data_as(_pd)


def qtn_last_error() -> str:
    return lib().qtn_last_error().decode()


def qtn_network_build(n_vertices, edges, gamma, beta, max_levels=0,
                      small_width=0, max_width=0, n_streams=0, eager=False,
                      lane_sum_bits=0, variant=0, order_trials=0, executor=0,
                      spin_limit=0, mixed_width=0, slice_width=0, order_weight=0,
                      hybrid_width=0):
    """Returns an opaque handle (int)."""
    e, ep = _i32(edges)
    g, gp = _f64(gamma)
    b, bp = _f64(beta)
    if len(g) != len(b):
        raise ValueError("gamma and beta differ in length")
    cfg = qtn_config(max_levels, small_width, max_width, n_streams, int(eager),
                     lane_sum_bits, variant, order_trials, executor, spin_limit,
                     mixed_width, slice_width, order_weight, hybrid_width)
    h = ctypes.c_void_p()
    check(lib().qtn_network_build(int(n_vertices), len(e) // 2, ep, len(g), gp,
                                  bp, ctypes.byref(cfg), ctypes.byref(h)))
    return h.value


def qtn_network_info(net, edge):
    nv, nt, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().qtn_network_info(net, edge, ctypes.byref(nv), ctypes.byref(nt),
                                 ctypes.byref(w)))
    return nv.value, nt.value, w.value


def qtn_order_minfill(net, edge):
    nv, _, _ = qtn_network_info(net, edge)
    out, op = _i32(np.zeros(nv))
    check(lib().qtn_order_minfill(net, edge, op))
    return out


def qtn_plan(net, orders=None, precision=QTN_C128):
    """orders: None or a list (one entry per edge) of None / permutations."""
    ws = ctypes.c_size_t()
    keep = []
    if orders is None:
        arr = None
    else:
        arr = (_pi32 * len(orders))()
        for i, o in enumerate(orders):
            if o is None:
                arr[i] = _pi32()
            else:
                a, ap = _i32(o)
                keep.append(a)
                arr[i] = ap
    check(lib().qtn_plan(net, arr, int(precision), ctypes.byref(ws)))
    return ws.value


def qtn_set_angles(net, gamma, beta):
    g, gp = _f64(gamma)
    b, bp = _f64(beta)
    check(lib().qtn_set_angles(net, gp, bp))


def stream_handle(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def workspace(nbytes, device=None):
    """Caller-owned device workspace (256-byte aligned by the allocator)."""
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8,
                    device=device or "cuda")
    if t.data_ptr() % 256:
        raise RuntimeError("workspace is not 256-byte aligned")
    return t


def qtn_contract(net, n_edges, ws, stream=None):
    """Returns (zz real [n_edges], zz imag [n_edges], energy)."""
    zz = np.zeros(n_edges)
    zi = np.zeros(n_edges)
    en = ctypes.c_double()
    check(lib().qtn_contract(net, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                             stream_handle(stream), zz.ctypes.data_as(_pd),
                             zi.ctypes.data_as(_pd), ctypes.byref(en)))
    return zz, zi, en.value


def qtn_contract_timed(net, n_edges, ws, stream=None):
    """Returns (zz real, energy, timing dict)."""
    zz = np.zeros(n_edges)
    en = ctypes.c_double()
    t = qtn_timing()
    check(lib().qtn_contract_timed(net, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   stream_handle(stream), zz.ctypes.data_as(_pd),
                                   ctypes.byref(en), ctypes.byref(t)))
    return zz, en.value, _timing_dict(t)


def _net_array(nets):
    arr = (ctypes.c_void_p * len(nets))(*nets)
    return arr


def qtn_batch_workspace(nets):
    ws = ctypes.c_size_t()
    check(lib().qtn_batch_workspace(_net_array(nets), len(nets), ctypes.byref(ws)))
    return ws.value


def qtn_contract_batch(nets, total_edges, ws, stream=None):
    """Returns (zz real concatenated over networks, energies [n])."""
    zz = np.zeros(total_edges)
    en = np.zeros(len(nets))
    check(lib().qtn_contract_batch(_net_array(nets), len(nets),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   stream_handle(stream), zz.ctypes.data_as(_pd),
                                   en.ctypes.data_as(_pd)))
    return zz, en


def qtn_autotune_batch(nets, ws, stream=None):
    """Persistent grid and step item order of the batched call; returns the
    measured configurations and the one kept."""
    r = qtn_batch_tune_report()
    check(lib().qtn_autotune_batch(_net_array(nets), len(nets), ctypes.c_void_p(ws.data_ptr()),
                                   ws.numel(), stream_handle(stream), ctypes.byref(r)))
    n = r.n_candidates
    return {"n_candidates": n, "pick": r.pick, "grid_blocks": list(r.grid_blocks[:n]),
            "item_order": list(r.item_order[:n]), "ms": list(r.ms[:n])}


def qtn_get_plan_stats(net):
    s = qtn_plan_stats()
    check(lib().qtn_get_plan_stats(net, ctypes.byref(s)))
    return {"n_buckets": s.n_buckets, "n_groups": s.n_groups, "n_wide": s.n_wide,
            "max_width": s.max_width, "width_hist": list(s.width_hist),
            "bytes": s.bytes, "flops": s.flops, "paper_flops": s.paper_flops,
            "workspace": s.workspace, "n_matrix": s.n_matrix,
            "n_cell": s.n_cell, "n_stream": s.n_stream, "n_over4g": s.n_over4g,
            "n_over4g_generic": s.n_over4g_generic, "n_sliced": s.n_sliced,
            "n_slices": s.n_slices}


def qtn_plan_order(net, edge):
    nv, _, _ = qtn_network_info(net, edge)
    out, op = _i32(np.zeros(nv))
    check(lib().qtn_plan_order(net, edge, op))
    return out


def qtn_bucket_widths(net, edge):
    nv, _, _ = qtn_network_info(net, edge)
    out, op = _i32(np.zeros(nv))
    check(lib().qtn_bucket_widths(net, edge, op))
    return out


def qtn_slice_vars(net, edge):
    """Variables fixed by index slicing in one light cone (slice bit order)."""
    out, op = _i32(np.zeros(16))
    n = ctypes.c_int32()
    check(lib().qtn_slice_vars(net, edge, 16, op, ctypes.byref(n)))
    return out[:n.value]


def qtn_launch_log(net):
    """Per-launch records of the last timed evaluation, as dicts."""
    n = ctypes.c_int64()
    check(lib().qtn_launch_log(net, 0, None, ctypes.byref(n)))
    arr = (qtn_launch_rec * max(1, n.value))()
    check(lib().qtn_launch_log(net, n.value, arr, ctypes.byref(n)))
    return [{f: getattr(r, f) for f, _ in qtn_launch_rec._fields_} for r in arr[:n.value]]


def qtn_autotune(net, ws, stream=None):
    """Measure each candidate kernel configuration and keep the fastest per
    group.  Returns the report as a dict."""
    r = qtn_tune_report()
    check(lib().qtn_autotune(net, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                             stream_handle(stream), ctypes.byref(r)))
    nc = r.n_candidates
    return {"n_groups": r.n_groups, "n_candidates": nc,
            "cand_ms": list(r.cand_ms[:nc]), "tuned_ms": r.tuned_ms,
            "picks": list(r.picks[:nc])}


def qtn_tune_angles_workspace(net, n_sets):
    b = ctypes.c_size_t()
    check(lib().qtn_tune_angles_workspace(net, int(n_sets), ctypes.byref(b)))
    return b.value


def qtn_autotune_angles(net, ws, n_sets, stream=None):
    """The autotuner with every candidate run over n_sets copies of the
    network's angles in one pass.  Returns the report as a dict."""
    r = qtn_tune_report()
    check(lib().qtn_autotune_angles(net, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    stream_handle(stream), int(n_sets), ctypes.byref(r)))
    nc = r.n_candidates
    return {"n_groups": r.n_groups, "n_candidates": nc,
            "cand_ms": list(r.cand_ms[:nc]), "tuned_ms": r.tuned_ms,
            "picks": list(r.picks[:nc]), "n_sets": int(n_sets)}


def qtn_angles_workspace(net, n_sets):
    b = ctypes.c_size_t()
    check(lib().qtn_angles_workspace(net, int(n_sets), ctypes.byref(b)))
    return b.value


def qtn_gradient_workspace(net):
    b = ctypes.c_size_t()
    check(lib().qtn_gradient_workspace(net, ctypes.byref(b)))
    return b.value


def qtn_energy_gradient(net, p, gamma, beta, ws, step, stream=None):
    """Energy and its central-difference gradient in gamma and beta (one
    batched pass over 4p + 1 angle sets).  Returns (E, dE/dgamma, dE/dbeta)."""
    import numpy as np
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    if g.shape != (p,) or b.shape != (p,):
        raise ValueError(f"gamma and beta must have shape ({p},)")
    e = ctypes.c_double()
    dg = np.empty(p, dtype=np.float64)
    db = np.empty(p, dtype=np.float64)
    pd = ctypes.POINTER(ctypes.c_double)
    check(lib().qtn_energy_gradient(net, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    stream_handle(stream), g.ctypes.data_as(pd),
                                    b.ctypes.data_as(pd), float(step), ctypes.byref(e),
                                    dg.ctypes.data_as(pd), db.ctypes.data_as(pd)))
    return e.value, dg, db


def _timing_dict(t):
    return {name: {"ms": t.ms[k], "launches": int(t.launches[k]),
                   "bytes": t.bytes[k], "flops": t.flops[k]}
            for k, name in enumerate(_capi.KERNEL_NAMES)}


def qtn_contract_angles(net, n_edges, gammas, betas, ws, stream=None, timed=False):
    """gammas, betas: [n_sets][p].  Returns (zz [n_sets, n_edges], energies
    [n_sets]), plus the timing dict when timed (launches serialized)."""
    g = np.ascontiguousarray(np.asarray(gammas, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
    if g.ndim != 2 or g.shape != b.shape:
        raise ValueError("gammas and betas must both be [n_sets][p]")
    n_sets = g.shape[0]
    zz = np.zeros((n_sets, n_edges))
    en = np.zeros(n_sets)
    t = qtn_timing()
    check(lib().qtn_contract_angles(net, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    stream_handle(stream), n_sets, g.ctypes.data_as(_pd),
                                    b.ctypes.data_as(_pd), zz.ctypes.data_as(_pd),
                                    en.ctypes.data_as(_pd), ctypes.byref(t) if timed else None))
    return (zz, en, _timing_dict(t)) if timed else (zz, en)


def qtn_tune_picks(net):
    """Kernel choice per group: list of (edge, group, place, variant, rls, shape)."""
    n = ctypes.c_int64()
    check(lib().qtn_tune_picks(net, 0, None, ctypes.byref(n)))
    arr = (qtn_tune_pick * max(1, n.value))()
    check(lib().qtn_tune_picks(net, n.value, arr, ctypes.byref(n)))
    return [(r.edge, r.group, r.place, r.variant, r.rls, r.shape) for r in arr[:n.value]]


def qtn_set_tune_picks(net, picks):
    """Apply picks as returned by qtn_tune_picks."""
    arr = (qtn_tune_pick * max(1, len(picks)))()
    for k, (e, g, pl, v, r, sh) in enumerate(picks):
        arr[k] = qtn_tune_pick(int(e), int(g), int(pl), int(v), int(r), 0, int(sh))
    check(lib().qtn_set_tune_picks(net, arr, len(picks)))


def qtn_tune_log(net):
    """(features [n, 16] float32, ms [n, 4] float64) from the last autotune."""
    n = ctypes.c_int64()
    check(lib().qtn_tune_log(net, 0, None, ctypes.byref(n)))
    arr = (qtn_tune_rec * max(1, n.value))()
    check(lib().qtn_tune_log(net, n.value, arr, ctypes.byref(n)))
    feats = np.array([list(r.features) for r in arr[:n.value]], dtype=np.float32)
    ms = np.array([list(r.ms) for r in arr[:n.value]], dtype=np.float64)
    return feats.reshape(-1, 16), ms.reshape(-1, 4)


def qtn_network_free(net):
    lib().qtn_network_free(net)


class Network:
    """Owning wrapper around one qtn_network handle."""

    def __init__(self, n_vertices, edges, gamma, beta, **cfg):
        self.n = int(n_vertices)
        self.edges = [tuple(map(int, e)) for e in edges]
        self.m = len(self.edges)
        self.p = len(gamma)
        self.h = qtn_network_build(self.n, self.edges, gamma, beta, **cfg)
        self.ws_bytes = None
        self._ws = None
        self._aws = None

    def info(self, edge):
        return qtn_network_info(self.h, edge)

    def order_minfill(self, edge):
        return qtn_order_minfill(self.h, edge)

    def plan(self, precision=QTN_C128, orders=None):
        self.ws_bytes = qtn_plan(self.h, orders, precision)
        return self.ws_bytes

    def set_angles(self, gamma, beta):
        qtn_set_angles(self.h, gamma, beta)

    def workspace(self):
        if self._ws is None or self._ws.numel() < self.ws_bytes:
            self._ws = None
            self._ws = workspace(self.ws_bytes)
        return self._ws

    def contract(self, ws=None, stream=None):
        return qtn_contract(self.h, self.m, ws if ws is not None else self.workspace(),
                            stream)

    def contract_timed(self, ws=None, stream=None):
        return qtn_contract_timed(self.h, self.m,
                                  ws if ws is not None else self.workspace(), stream)

    def stats(self):
        return qtn_get_plan_stats(self.h)

    def launch_log(self):
        return qtn_launch_log(self.h)

    def autotune(self, ws=None, stream=None, n_sets=1):
        """Measure every candidate kernel configuration and keep the fastest
        per group; n_sets > 1 measures angle batches of that size."""
        if n_sets == 1:
            return qtn_autotune(self.h, ws if ws is not None else self.workspace(), stream)
        if ws is None:
            ws = workspace(qtn_tune_angles_workspace(self.h, n_sets))
        return qtn_autotune_angles(self.h, ws, n_sets, stream)

    def tune_log(self):
        return qtn_tune_log(self.h)

    def angles_workspace(self, n_sets):
        return qtn_angles_workspace(self.h, n_sets)

    def contract_angles(self, gammas, betas, ws=None, stream=None, timed=False):
        """Energies of several angle sets in one pass over the plan."""
        if ws is None:
            need = qtn_angles_workspace(self.h, len(gammas))
            if self._aws is None or self._aws.numel() < need:
                self._aws = None
                self._aws = workspace(need)
            ws = self._aws
        return qtn_contract_angles(self.h, self.m, gammas, betas, ws, stream, timed)

    def energy_gradient(self, gamma, beta, step=1e-4, ws=None, stream=None):
        """Energy at (gamma, beta) and its gradient, by central differences
        evaluated in one angle-batched pass."""
        if ws is None:
            need = qtn_gradient_workspace(self.h)
            if self._aws is None or self._aws.numel() < need:
                self._aws = None
                self._aws = workspace(need)
            ws = self._aws
        return qtn_energy_gradient(self.h, self.p, gamma, beta, ws, step, stream)

    def tune_picks(self):
        return qtn_tune_picks(self.h)

    def set_tune_picks(self, picks):
        qtn_set_tune_picks(self.h, picks)

    def plan_order(self, edge):
        return qtn_plan_order(self.h, edge)

    def slice_vars(self, edge):
        return qtn_slice_vars(self.h, edge)

    def bucket_widths(self, edge):
        return qtn_bucket_widths(self.h, edge)

    def close(self):
        if self.h:
            qtn_network_free(self.h)
            self.h = None
        self._ws = None
        self._aws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_pf = ctypes.POINTER(ctypes.c_float)


def _f32(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32).ravel())
    return a, a.ctypes.data_as(_pf)


class CostModel:
    """Owning wrapper of a qtn_costmodel (16-64-64-4 perceptron)."""

    n_params = _capi.MLP_PARAMS
    n_out = _capi.MLP_OUT

    def __init__(self, params):
        p, pp = _f32(params)
        if len(p) != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        h = ctypes.c_void_p()
        check(lib().qtn_costmodel_create(pp, ctypes.byref(h)))
        self.h = h.value

    @staticmethod
    def workspace(n):
        b = ctypes.c_size_t()
        check(lib().qtn_costmodel_workspace(int(n), ctypes.byref(b)))
        return workspace(b.value)

    def params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        check(lib().qtn_costmodel_params(self.h, out.ctypes.data_as(_pf)))
        return out

    def normalization(self):
        mu = np.zeros(16, dtype=np.float32)
        inv = np.zeros(16, dtype=np.float32)
        check(lib().qtn_costmodel_normalization(self.h, mu.ctypes.data_as(_pf),
                                                inv.ctypes.data_as(_pf)))
        return mu, inv

    def train(self, x, ms, epochs, lr, stream=None):
        x, xp = _f32(x)
        n = len(x) // 16
        m, mp = _f64(ms)
        if len(x) != 16 * n or len(m) != self.n_out * n:
            raise ValueError(f"expected x [n, 16] and ms [n, {self.n_out}]")
        ws = self.workspace(n)
        hist = np.zeros(epochs, dtype=np.float32)
        check(lib().qtn_costmodel_train(self.h, xp, mp, n, int(epochs), float(lr),
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                        stream_handle(stream), hist.ctypes.data_as(_pf)))
        return hist

    def predict(self, x, stream=None):
        x, xp = _f32(x)
        n = len(x) // 16
        if len(x) != 16 * n:
            raise ValueError("expected x [n, 16]")
        ws = self.workspace(n)
        y = np.zeros(n * self.n_out, dtype=np.float32)
        check(lib().qtn_costmodel_predict(self.h, xp, n, ctypes.c_void_p(ws.data_ptr()),
                                          ws.numel(), stream_handle(stream),
                                          y.ctypes.data_as(_pf)))
        return y.reshape(n, self.n_out)

    def grad(self, x, t, m, stream=None):
        x, xp = _f32(x)
        t, tp = _f32(t)
        m, mp = _f32(m)
        n = len(x) // 16
        if len(x) != 16 * n or len(t) != self.n_out * n or len(m) != self.n_out * n:
            raise ValueError(f"expected x [n, 16], t and m [n, {self.n_out}]")
        ws = self.workspace(n)
        loss = ctypes.c_float()
        g = np.zeros(self.n_params, dtype=np.float32)
        check(lib().qtn_costmodel_grad(self.h, xp, tp, mp, n, ctypes.c_void_p(ws.data_ptr()),
                                       ws.numel(), stream_handle(stream), ctypes.byref(loss),
                                       g.ctypes.data_as(_pf)))
        return loss.value, g

    def adam_step(self, grad, lr, stream=None):
        g, gp = _f32(grad)
        if len(g) != self.n_params:
            raise ValueError(f"expected {self.n_params} gradient entries")
        ws = self.workspace(1)
        check(lib().qtn_costmodel_adam_step(self.h, gp, float(lr),
                                            ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                            stream_handle(stream)))

    def close(self):
        if self.h:
            lib().qtn_costmodel_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qtn_apply_costmodel(net, cm, stream=None):
    """Variant per group from the cost model; returns groups per variant
    (workgroup, streaming, generic, matrix form)."""
    n_groups = qtn_get_plan_stats(net)["n_groups"]
    ws = CostModel.workspace(max(1, n_groups))
    counts = np.zeros(4, dtype=np.int32)
    check(lib().qtn_apply_costmodel(net, cm.h, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    stream_handle(stream), counts.ctypes.data_as(_pi32)))
    return counts


# ------------------------------------------------------------ single bucket

def qtn_bucket_plan(operands, offsets, out_labels, out_offset, precision=QTN_C128, variant=0,
                    knob=0):
    """operands: list of label lists (each in union order); offsets: byte
    offsets of the operands in the data buffer.  Returns the bucket handle."""
    ranks, rp = _i32([len(o) for o in operands])
    labs, lp = _i32([x for o in operands for x in o] or [0])
    offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    outl, olp = _i32(list(out_labels) or [0])
    h = ctypes.c_void_p()
    check(lib().qtn_bucket_plan(len(operands), rp, lp,
                                offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                len(out_labels), olp, int(out_offset), precision, variant, knob,
                                ctypes.byref(h)))
    return h


def qtn_bucket_get_info(b):
    r = qtn_bucket_info()
    check(lib().qtn_bucket_get_info(b, ctypes.byref(r)))
    return {f: getattr(r, f) for f, _ in qtn_bucket_info._fields_}


def qtn_bucket_contract(b, data, ws, stream=None):
    check(lib().qtn_bucket_contract(b, ctypes.c_void_p(data.data_ptr()), data.numel(),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    stream_handle(stream)))


def qtn_bucket_contract_timed(b, data, ws, stream=None):
    """Runs the bucket and returns its kernel's duration in milliseconds."""
    ms = ctypes.c_double()
    check(lib().qtn_bucket_contract_timed(b, ctypes.c_void_p(data.data_ptr()), data.numel(),
                                          ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                          stream_handle(stream), ctypes.byref(ms)))
    return ms.value


def qtn_bucket_contract_noalloc(b, data, stream=None):
    check(lib().qtn_bucket_contract_noalloc(b, ctypes.c_void_p(data.data_ptr()), data.numel(),
                                            stream_handle(stream)))


def qtn_bucket_free(b):
    lib().qtn_bucket_free(b)


class Bucket:
    """One bucket contraction of caller-given tensors (qtn_bucket_*).  The
    tensors share one device buffer: operand k at offsets[k], the output at
    out_offset (packed at 256-byte boundaries in operand order when not
    given)."""

    def __init__(self, operands, out_labels, precision=QTN_C128, variant=0, knob=0,
                 offsets=None, out_offset=None):
        es = 8 if precision == QTN_C64 else 16
        self.operands = [list(o) for o in operands]
        self.out_labels = list(out_labels)
        self.precision = precision
        if offsets is None:
            offsets, pos = [], 0
            for o in self.operands:
                offsets.append(pos)
                pos += ((es << len(o)) + 255) // 256 * 256
            out_offset = pos
        self.offsets = list(offsets)
        self.out_offset = int(out_offset)
        self.h = qtn_bucket_plan(self.operands, self.offsets, self.out_labels, self.out_offset,
                                 precision, variant, knob)
        self._ws = None

    def info(self):
        return qtn_bucket_get_info(self.h)

    def workspace(self):
        if self._ws is None:
            self._ws = workspace(self.info()["workspace_bytes"])
        return self._ws

    def contract(self, data, ws=None, stream=None):
        """Queue the contraction on the stream (asynchronous)."""
        qtn_bucket_contract(self.h, data, self.workspace() if ws is None else ws, stream)

    def contract_timed(self, data, ws=None, stream=None):
        """Run once and return the kernel's duration in milliseconds."""
        return qtn_bucket_contract_timed(self.h, data, self.workspace() if ws is None else ws,
                                         stream)

    def contract_noalloc(self, data, stream=None):
        """Queue the contraction with the descriptors in the library's fixed
        device array (no workspace, no allocation)."""
        qtn_bucket_contract_noalloc(self.h, data, stream)

    def close(self):
        if self.h:
            qtn_bucket_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
