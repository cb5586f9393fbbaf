"""MI355X (gfx950) barycentric Lagrange treecode.

Thin Python binding over the C ABI of ``include/bltc.h`` (libbltc.so): it only
checks and marshals arguments.  Every step of the evaluation runs in the HIP
kernels of ``csrc/``; PyTorch supplies device memory and the current stream.

Coordinates are passed structure-of-arrays: a float64 tensor of shape (3, n)
(rows x, y, z).  Charges are (n,) or (m, n); potentials come back with the same
leading shape, in the caller's target order.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _capi
from ._capi import BLTCError, InvalidArgument  # noqa: F401

__all__ = ["params", "Plan", "Batch", "batch_potential", "autotune", "potential", "direct",
           "BLTCError", "InvalidArgument", "library_path", "version"]

_KERNELS = {"coulomb": _capi.COULOMB, "yukawa": _capi.YUKAWA, "regularized": _capi.REGULARIZED}
_PRECISIONS = {"fp64": _capi.FP64, "fp32_mixed": _capi.FP32_MIXED, "mixed": _capi.FP32_MIXED}
# "bltc": the paper's particle-cluster treecode (sources interpolated);
# "cp": cluster-particle (targets interpolated); "cc": cluster-cluster (both);
# "hermite": particle-cluster with the barycentric Hermite interpolant
_METHODS = {"bltc": _capi.PARTICLE_CLUSTER, "particle_cluster": _capi.PARTICLE_CLUSTER,
            "cp": _capi.CLUSTER_PARTICLE, "cluster_particle": _capi.CLUSTER_PARTICLE,
            "cc": _capi.CLUSTER_CLUSTER, "cluster_cluster": _capi.CLUSTER_CLUSTER,
            "hermite": _capi.HERMITE}


def library_path() -> str:
    return _capi.LIB_PATH


def version() -> str:
    return _capi.load().bltc_version().decode()


def params(kernel="coulomb", kappa=0.0, theta=0.7, degree=8, leaf_size=2000, batch_size=2000,
           precision="fp64", threads_per_target=1, method="bltc", delta=0.0,
           symmetry=True, workspace_limit=0) -> _capi.Params:
    """bltc_params: leaf_size = batch_size = 0 and threads_per_target = 0 leave the
    choice to the library's tuner (plans from device coordinates); workspace_limit
    caps the device bytes a plan holds (0: none)."""
    p = _capi.Params()
    _capi.load().bltc_params_default(ctypes.byref(p))
    p.kernel = _KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    p.precision = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.kappa = float(kappa)
    p.theta = float(theta)
    p.degree = int(degree)
    p.leaf_size = int(leaf_size)
    p.batch_size = int(batch_size)
    p.threads_per_target = int(threads_per_target)
    p.method = _METHODS[method] if isinstance(method, str) else int(method)
    p.delta = float(delta)
    p.no_symmetry = 0 if symmetry else 1
    p.workspace_limit = int(workspace_limit)
    return p


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _coords_device(a, name):
    torch = _torch()
    if not isinstance(a, torch.Tensor) or not a.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if a.dtype != torch.float64 or a.dim() != 2 or a.shape[0] != 3 or not a.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor of shape (3, n)")
    n = a.shape[1]
    base = a.data_ptr()
    return n, [ctypes.c_void_p(base + 8 * n * r) for r in range(3)]


def _coords_host(a, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] != 3:
        raise ValueError(f"{name} must have shape (3, n)")
    n = a.shape[1]
    return a, n, [a[r].ctypes.data_as(ctypes.c_void_p) for r in range(3)]


def _charges_device(q, ns):
    torch = _torch()
    if not isinstance(q, torch.Tensor) or not q.is_cuda or q.dtype != torch.float64:
        raise TypeError("charges must be a float64 CUDA (HIP) tensor")
    one = q.dim() == 1
    q2 = q.unsqueeze(0) if one else q
    if q2.dim() != 2 or q2.shape[1] != ns or q2.stride(1) != 1:
        raise ValueError("charges must have shape (n,) or (m, n) with unit inner stride")
    return q2, one


class Plan:
    """Geometry fixed once (trees, batches, interaction lists, device tables);
    charges vary between executions (`bltc_plan_create` / `bltc_plan_execute`)."""

    def __init__(self, targets, sources, *, max_q=1, stream=None, host=False, **kw):
        lib = _capi.load()
        self._lib = lib
        self.params = params(**kw)
        self._h = ctypes.c_void_p()
        self.max_q = int(max_q)
        if host:
            self._hold = []
            t, self.nt, tp = _coords_host(targets, "targets")
            if sources is targets:
                s, self.ns, sp = t, self.nt, tp
            else:
                s, self.ns, sp = _coords_host(sources, "sources")
            self._hold = [t, s]
            rc = lib.bltc_plan_create_host(ctypes.byref(self._h), ctypes.byref(self.params),
                                           self.nt, *tp, self.ns, *sp, self.max_q)
        else:
            self.nt, tp = _coords_device(targets, "targets")
            self.ns, sp = _coords_device(sources, "sources")
            rc = lib.bltc_plan_create(ctypes.byref(self._h), ctypes.byref(self.params),
                                      self.nt, *tp, self.ns, *sp, self.max_q,
                                      _stream_handle(stream))
        _capi.check(rc)
        self.device = None if host else targets.device

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.bltc_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def execute(self, charges, out=None, stream=None):
        """Potentials at all targets for the given charges (device tensors)."""
        torch = _torch()
        q2, one = _charges_device(charges, self.ns)
        m = q2.shape[0]
        if out is None:
            out = torch.empty((m, self.nt), dtype=torch.float64, device=q2.device)
        o2 = out.unsqueeze(0) if out.dim() == 1 else out
        if o2.shape != (m, self.nt) or o2.dtype != torch.float64 or o2.stride(1) != 1:
            raise ValueError("out must be float64 of shape (m, nt)")
        rc = self._lib.bltc_plan_execute(self._h, ctypes.c_void_p(q2.data_ptr()), m,
                                         q2.stride(0) if m > 1 else self.ns,
                                         ctypes.c_void_p(o2.data_ptr()),
                                         o2.stride(0) if m > 1 else self.nt,
                                         _stream_handle(stream))
        _capi.check(rc)
        return out[0] if (one and out.dim() == 2) else out

    def stats(self) -> dict:
        st = _capi.Stats()
        _capi.check(self._lib.bltc_plan_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in _capi.Stats._fields_}

    def set_timing(self, enable=True):
        _capi.check(self._lib.bltc_plan_set_timing(self._h, 1 if enable else 0))

    def phase_times(self) -> dict:
        """Device milliseconds of the last execution's phases (timing must be on)."""
        ms = (ctypes.c_double * 5)()
        _capi.check(self._lib.bltc_plan_phase_times(self._h, ms))
        return {"gather": ms[0], "upward": ms[1], "interact": ms[2], "total": ms[3],
                "mutual_pairs": ms[4]}

    def view(self) -> dict:
        """Copies of the plan's host-side structure (numpy arrays)."""
        v = _capi.PlanView()
        _capi.check(self._lib.bltc_plan_view_get(self._h, ctypes.byref(v)))

        def arr(ptr, n, dt):
            if n == 0:
                return np.zeros(0, dtype=dt)
            return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dt, copy=True)

        nc, nb, ni = v.n_clusters, v.n_batches, v.n_items
        return {
            "source_order": arr(v.source_order, v.ns, np.int64),
            "target_order": arr(v.target_order, v.nt, np.int64),
            "cluster_begin": arr(v.cluster_begin, nc, np.int64),
            "cluster_count": arr(v.cluster_count, nc, np.int64),
            "cluster_lo": arr(v.cluster_lo, 3 * nc, np.float64).reshape(nc, 3),
            "cluster_hi": arr(v.cluster_hi, 3 * nc, np.float64).reshape(nc, 3),
            "cluster_first_child": arr(v.cluster_first_child, nc, np.int32),
            "cluster_nchild": arr(v.cluster_nchild, nc, np.int32),
            "cluster_level": arr(v.cluster_level, nc, np.int32),
            "batch_begin": arr(v.batch_begin, nb, np.int64),
            "batch_count": arr(v.batch_count, nb, np.int64),
            "batch_lo": arr(v.batch_lo, 3 * nb, np.float64).reshape(nb, 3),
            "batch_hi": arr(v.batch_hi, 3 * nb, np.float64).reshape(nb, 3),
            "item_batch": arr(v.item_batch, ni, np.int32),
            "item_cluster": arr(v.item_cluster, ni, np.int32),
            "item_kind": arr(v.item_kind, ni, np.int32),
        }

    def modified_charges(self, cluster, qi=0, stream=None):
        """Modified charges the last execution formed for a cluster: (n+1, n+1, n+1); for
        the Hermite method (8, n+1, n+1, n+1), first index a = 4 a1 + 2 a2 + a3."""
        n1 = self.params.degree + 1
        hermite = self.params.method == _capi.HERMITE
        out = np.zeros(n1 ** 3 * (8 if hermite else 1))
        rc = self._lib.bltc_plan_modified_charges(self._h, int(cluster), int(qi),
                                                  out.ctypes.data_as(ctypes.c_void_p),
                                                  _stream_handle(stream))
        _capi.check(rc)
        if hermite:
            return np.ascontiguousarray(np.moveaxis(out.reshape(n1, n1, n1, 8), -1, 0))
        return out.reshape(n1, n1, n1)


class Batch:
    """Many systems evaluated together (`bltc_batch_create` / `bltc_batch_execute`): one
    persistent work-queue launch over all systems, replayed from a hipGraph.  The plans
    must be created with max_q >= 2 and outlive the batch."""

    def __init__(self, plans, stream=None):
        lib = _capi.load()
        self._lib = lib
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        self._h = ctypes.c_void_p()
        _capi.check(lib.bltc_batch_create(ctypes.byref(self._h), arr, len(self.plans),
                                          _stream_handle(stream)))

    def set_graph(self, enable=True):
        _capi.check(self._lib.bltc_batch_set_graph(self._h, 1 if enable else 0))

    def info(self) -> dict:
        inf = _capi.BatchInfo()
        _capi.check(self._lib.bltc_batch_info_get(self._h, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in _capi.BatchInfo._fields_}

    def execute(self, charges, outs=None, stream=None):
        """charges: one (m_i, ns_i) float64 device tensor per system; returns (m_i, nt_i) tensors."""
        return _batch_call(self.plans, charges, outs, stream,
                           lambda *a: self._lib.bltc_batch_execute(self._h, *a))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.bltc_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch_call(plans, charges, outs, stream, call):
    torch = _torch()
    n = len(plans)
    if len(charges) != n:
        raise ValueError("one charge tensor per system")
    qs, outs2 = [], []
    for i, (p, q) in enumerate(zip(plans, charges)):
        q2, _ = _charges_device(q, p.ns)
        qs.append(q2)
        if outs is None:
            o = torch.empty((q2.shape[0], p.nt), dtype=torch.float64, device=q2.device)
        else:
            o = outs[i]
            o = o.unsqueeze(0) if o.dim() == 1 else o
        outs2.append(o)
    qp = (ctypes.c_void_p * n)(*[q.data_ptr() for q in qs])
    nq = (ctypes.c_int32 * n)(*[q.shape[0] for q in qs])
    ql = (ctypes.c_int64 * n)(*[q.stride(0) if q.shape[0] > 1 else p.ns for q, p in zip(qs, plans)])
    op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs2])
    ol = (ctypes.c_int64 * n)(*[o.stride(0) if o.shape[0] > 1 else p.nt for o, p in zip(outs2, plans)])
    _capi.check(call(qp, nq, ql, op, ol, _stream_handle(stream)))
    return outs2


def batch_potential(plans, charges, outs=None, stream=None):
    """One evaluation of many systems over a list of plans (`bltc_batch_potential`):
    the work-queue launch of a Batch, built and freed in the call; synchronises."""
    lib = _capi.load()
    arr = (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])
    return _batch_call(plans, charges, outs, stream,
                       lambda *a: lib.bltc_batch_potential(arr, len(plans), *a))


def autotune(targets, sources, candidates=(1000, 2000, 3000, 4000), *, num_q=1, use_cache=True,
             stream=None, full=False, **kw):
    """Leaf/batch size chosen by timing each candidate on the GPU (`bltc_autotune`);
    with threads_per_target=0 (the default) for a one-vector BLTC problem, also the
    threads per target (1, 2 or 4).

    Returns (size, milliseconds of one evaluation), or with full=True
    (size, threads per target, milliseconds)."""
    lib = _capi.load()
    kw.setdefault("threads_per_target", 0)   # searched unless fixed by the caller
    p = params(**kw)
    nt, tp = _coords_device(targets, "targets")
    ns, sp = _coords_device(sources, "sources")
    cand = (ctypes.c_int32 * len(candidates))(*[int(c) for c in candidates])
    out = _capi.Params()
    ms = ctypes.c_double()
    _capi.check(lib.bltc_autotune(ctypes.byref(p), nt, *tp, ns, *sp, int(num_q), cand, len(candidates),
                                  1 if use_cache else 0, ctypes.byref(out), ctypes.byref(ms),
                                  _stream_handle(stream)))
    if full:
        return out.leaf_size, max(1, out.threads_per_target), ms.value
    return out.leaf_size, ms.value


def potential(targets, sources, charges, *, stream=None, out=None, **kw):
    """One-shot treecode evaluation (`bltc_potential`); synchronises the stream."""
    torch = _torch()
    lib = _capi.load()
    p = params(**kw)
    nt, tp = _coords_device(targets, "targets")
    ns, sp = _coords_device(sources, "sources")
    q2, one = _charges_device(charges, ns)
    m = q2.shape[0]
    if out is None:
        out = torch.empty((m, nt), dtype=torch.float64, device=q2.device)
    o2 = out.unsqueeze(0) if out.dim() == 1 else out
    rc = lib.bltc_potential(ctypes.byref(p), nt, *tp, ns, *sp, ctypes.c_void_p(q2.data_ptr()), m,
                            q2.stride(0) if m > 1 else ns, ctypes.c_void_p(o2.data_ptr()),
                            o2.stride(0) if m > 1 else nt, _stream_handle(stream))
    _capi.check(rc)
    return out[0] if (one and out.dim() == 2) else out


def direct(targets, sources, charges, *, stream=None, out=None, kernel="coulomb", kappa=0.0,
           delta=0.0, noalloc=False):
    """GPU FP64 direct sum of eq. (1) (`bltc_direct`); with noalloc=True the variant
    that allocates no device memory (`bltc_direct_noalloc`, at most 2^20 sources;
    pass `out` to keep the call free of allocations here too)."""
    torch = _torch()
    lib = _capi.load()
    p = params(kernel=kernel, kappa=kappa, delta=delta)
    nt, tp = _coords_device(targets, "targets")
    ns, sp = _coords_device(sources, "sources")
    q2, one = _charges_device(charges, ns)
    m = q2.shape[0]
    if out is None:
        out = torch.empty((m, nt), dtype=torch.float64, device=q2.device)
    o2 = out.unsqueeze(0) if out.dim() == 1 else out
    fn = lib.bltc_direct_noalloc if noalloc else lib.bltc_direct
    rc = fn(ctypes.byref(p), nt, *tp, ns, *sp, ctypes.c_void_p(q2.data_ptr()), m,
            q2.stride(0) if m > 1 else ns, ctypes.c_void_p(o2.data_ptr()),
            o2.stride(0) if m > 1 else nt, _stream_handle(stream))
    _capi.check(rc)
    return out[0] if (one and out.dim() == 2) else out
