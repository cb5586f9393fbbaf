"""CPU oracle for the barycentric Lagrange treecode -- TEST INFRASTRUCTURE ONLY.

Plain FP64 C code (``bltc_oracle.c``) behind a ctypes wrapper.  It computes the
direct sum of eq. (1) and the treecode of Alg. 1 (tree of source clusters,
target batches, two-part MAC of eq. (13), modified charges of eq. (12) with the
removable-singularity rule of eq. (5), approximation eq. (11) and direct sum
eq. (9)) of Vaughn, Wilson and Krasny (2020), and the cluster-particle variant
(the same interpolation in the target variable) and the cluster-cluster
variant (both sides interpolated) that the paper's outlook names.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the GPU library and never
consumes anything the GPU library produced.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bltc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

COULOMB = 0
YUKAWA = 1
# regularized Coulomb 1/sqrt(r^2 + delta^2): delta is passed as `kappa` (the
# kernel parameter) to every function of this module
REGULARIZED = 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    d, i32, i64, vp = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_direct.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, vp, i32, i64, i32, d, vp, i64]
    lib.oracle_direct.restype = None
    lib.oracle_chebyshev.argtypes = [i32, d, d, vp, vp]
    lib.oracle_lagrange.argtypes = [i32, vp, vp, d, vp]
    lib.oracle_tc_create.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, d, i32, i64, i64]
    lib.oracle_tc_create.restype = vp
    lib.oracle_tc_destroy.argtypes = [vp]
    lib.oracle_tc_sizes.argtypes = [vp, vp]
    lib.oracle_tc_source_node.argtypes = [vp, i64, vp, vp, vp, vp]
    lib.oracle_tc_source_order.argtypes = [vp, vp]
    lib.oracle_tc_target_order.argtypes = [vp, vp]
    lib.oracle_tc_batch.argtypes = [vp, i64, vp, vp, vp]
    lib.oracle_tc_items.argtypes = [vp, vp, vp, vp]
    lib.oracle_tc_cluster_nodes.argtypes = [vp, i32, vp]
    lib.oracle_tc_modified_charges.argtypes = [vp, i32, vp, i32, i64, vp]
    lib.oracle_tc_potential.argtypes = [vp, vp, i32, i64, i32, d, i64, vp, vp, i64, vp]
    lib.oracle_tc_potential.restype = ctypes.c_int
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_cp_create.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, d, i32, i64, i64]
    lib.oracle_cp_create.restype = vp
    lib.oracle_cp_destroy.argtypes = [vp]
    lib.oracle_cp_sizes.argtypes = [vp, vp]
    lib.oracle_cp_target_order.argtypes = [vp, vp]
    lib.oracle_cp_source_order.argtypes = [vp, vp]
    lib.oracle_cp_cluster.argtypes = [vp, i64, vp, vp, vp, vp]
    lib.oracle_cp_batch.argtypes = [vp, i64, vp]
    lib.oracle_cp_items.argtypes = [vp, vp, vp, vp]
    lib.oracle_cp_proxy_potentials.argtypes = [vp, i32, vp, i32, d, vp]
    lib.oracle_cp_potential.argtypes = [vp, vp, i32, d, i64, vp, vp, vp]
    lib.oracle_cp_potential.restype = ctypes.c_int
    lib.oracle_kernel_derivatives.argtypes = [d, i32, d, vp]
    lib.oracle_hermite_basis.argtypes = [i32, vp, vp, d, vp, vp]
    lib.oracle_tc_create_hermite.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, d, i32, i64, i64]
    lib.oracle_tc_create_hermite.restype = vp
    lib.oracle_tc_hermite_charges.argtypes = [vp, i32, vp, vp]
    lib.oracle_tc_hermite_potential.argtypes = [vp, vp, i32, d, i64, vp, vp, vp]
    lib.oracle_tc_hermite_potential.restype = ctypes.c_int
    lib.oracle_cc_create.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, d, i32, i64, i64]
    lib.oracle_cc_create.restype = vp
    lib.oracle_cc_destroy.argtypes = [vp]
    lib.oracle_cc_sizes.argtypes = [vp, vp]
    lib.oracle_cc_orders.argtypes = [vp, vp, vp]
    lib.oracle_cc_node.argtypes = [vp, i32, i64, vp, vp, vp]
    lib.oracle_cc_pairs.argtypes = [vp, vp, vp, vp]
    lib.oracle_cc_proxy_potentials.argtypes = [vp, i32, vp, i32, d, vp]
    lib.oracle_cc_potential.argtypes = [vp, vp, i32, d, i64, vp, vp, vp]
    lib.oracle_cc_potential.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_load().oracle_max_threads())


def _charges_2d(q):
    q = _f64(q)
    if q.ndim == 1:
        q = q[None, :]
    if q.shape[0] > 64:
        raise ValueError("the oracle supports at most 64 charge vectors")
    return np.ascontiguousarray(q)


def direct(targets, sources, charges, kernel=COULOMB, kappa=0.0):
    """Direct sum, eq. (1); pairs at zero distance are skipped.

    targets (nt, 3), sources (ns, 3), charges (ns,) or (m, ns) -> phi (nt,) or (m, nt).
    """
    lib = _load()
    t = _f64(targets)
    s = _f64(sources)
    q = _charges_2d(charges)
    one = np.asarray(charges).ndim == 1
    tx, ty, tz = (np.ascontiguousarray(t[:, c]) for c in range(3))
    sx, sy, sz = (np.ascontiguousarray(s[:, c]) for c in range(3))
    m, ns = q.shape
    nt = t.shape[0]
    phi = np.zeros((m, nt))
    lib.oracle_direct(nt, _ptr(tx), _ptr(ty), _ptr(tz), ns, _ptr(sx), _ptr(sy), _ptr(sz),
                      _ptr(q), m, ns, int(kernel), float(kappa), _ptr(phi), nt)
    return phi[0] if one else phi


def chebyshev(n, a=-1.0, b=1.0):
    """Chebyshev points of the 2nd kind on [a, b] and barycentric weights, eqs. (6)-(7)."""
    s = np.zeros(n + 1)
    w = np.zeros(n + 1)
    _load().oracle_chebyshev(int(n), float(a), float(b), _ptr(s), _ptr(w))
    return s, w


def lagrange(n, s, w, x):
    """L_k(x), k = 0..n, barycentric form eq. (4) with the rule of eq. (5)."""
    s = _f64(s)
    w = _f64(w)
    L = np.zeros(n + 1)
    _load().oracle_lagrange(int(n), _ptr(s), _ptr(w), float(x), _ptr(L))
    return L


def kernel_derivatives(r, kernel=COULOMB, kappa=0.0):
    """G(r) and g1 = G'/r, g2 = g1'/r, g3 = g2'/r of a radial kernel at r > 0."""
    g = np.zeros(4)
    _load().oracle_kernel_derivatives(float(r), int(kernel), float(kappa), _ptr(g))
    return g


def hermite_basis(n, s, w, x):
    """Hermite basis A_k(x), B_k(x), k = 0..n, on the nodes s with weights w."""
    s = _f64(s)
    w = _f64(w)
    A = np.zeros(n + 1)
    B = np.zeros(n + 1)
    _load().oracle_hermite_basis(int(n), _ptr(s), _ptr(w), float(x), _ptr(A), _ptr(B))
    return A, B


class Treecode:
    """Oracle BLTC (Alg. 1): trees, batches and interaction lists are built here;
    modified charges and potentials on demand.  hermite=True: the barycentric
    Hermite treecode (8 (n+1)^3 modified charges per cluster, kernel
    derivatives in the approximation, size test against 8 (n+1)^3)."""

    def __init__(self, targets, sources, theta, degree, leaf_size, batch_size, hermite=False):
        lib = _load()
        self._t = _f64(targets)
        self._s = _f64(sources)
        self._tc_cols = [np.ascontiguousarray(self._t[:, c]) for c in range(3)]
        self._sc_cols = [np.ascontiguousarray(self._s[:, c]) for c in range(3)]
        self.nt = self._t.shape[0]
        self.ns = self._s.shape[0]
        self.degree = int(degree)
        if not (1 <= self.degree <= 60):
            raise ValueError("degree out of range")
        tx, ty, tz = self._tc_cols
        sx, sy, sz = self._sc_cols
        self.hermite = bool(hermite)
        create = lib.oracle_tc_create_hermite if self.hermite else lib.oracle_tc_create
        self._h = create(self.nt, _ptr(tx), _ptr(ty), _ptr(tz), self.ns, _ptr(sx), _ptr(sy),
                         _ptr(sz), float(theta), self.degree, int(leaf_size), int(batch_size))
        if not self._h:
            raise RuntimeError("oracle treecode creation failed")
        sizes = np.zeros(5, dtype=np.int64)
        lib.oracle_tc_sizes(self._h, _ptr(sizes))
        self.n_clusters, self.n_batches, self.n_items = (int(v) for v in sizes[:3])
        self.t_setup = float(sizes[4]) * 1e-9

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().oracle_tc_destroy(h)
            self._h = None

    # ---- structure --------------------------------------------------------
    def source_order(self):
        out = np.zeros(self.ns, dtype=np.int64)
        _load().oracle_tc_source_order(self._h, _ptr(out))
        return out

    def target_order(self):
        out = np.zeros(self.nt, dtype=np.int64)
        _load().oracle_tc_target_order(self._h, _ptr(out))
        return out

    def cluster(self, i):
        lo = np.zeros(3)
        hi = np.zeros(3)
        bc = np.zeros(2, dtype=np.int64)
        ncl = np.zeros(10, dtype=np.int32)
        _load().oracle_tc_source_node(self._h, int(i), _ptr(lo), _ptr(hi), _ptr(bc), _ptr(ncl))
        nch = int(ncl[0])
        return {"lo": lo, "hi": hi, "begin": int(bc[0]), "count": int(bc[1]),
                "children": [int(c) for c in ncl[1:1 + nch]], "level": int(ncl[9])}

    def batch(self, b):
        lo = np.zeros(3)
        hi = np.zeros(3)
        bc = np.zeros(2, dtype=np.int64)
        _load().oracle_tc_batch(self._h, int(b), _ptr(lo), _ptr(hi), _ptr(bc))
        return {"lo": lo, "hi": hi, "begin": int(bc[0]), "count": int(bc[1])}

    def items(self):
        """(batch, cluster, kind) for every interaction; kind 0 = approx, 1 = direct."""
        b = np.zeros(self.n_items, dtype=np.int64)
        c = np.zeros(self.n_items, dtype=np.int32)
        k = np.zeros(self.n_items, dtype=np.int32)
        _load().oracle_tc_items(self._h, _ptr(b), _ptr(c), _ptr(k))
        return b, c, k

    def cluster_nodes(self, c):
        out = np.zeros(3 * (self.degree + 1))
        _load().oracle_tc_cluster_nodes(self._h, int(c), _ptr(out))
        return out.reshape(3, self.degree + 1)

    def cluster_members(self, c):
        """Original source indices of cluster c."""
        info = self.cluster(c)
        order = self.source_order()
        return order[info["begin"]:info["begin"] + info["count"]]

    # ---- numerics ---------------------------------------------------------
    def modified_charges(self, c, charges):
        """qhat of cluster c, eq. (12): array (m, n+1, n+1, n+1) or (n+1,)*3 for 1-D charges."""
        q = _charges_2d(charges)
        one = np.asarray(charges).ndim == 1
        m = q.shape[0]
        np1 = self.degree + 1
        out = np.zeros(np1 ** 3 * m)
        _load().oracle_tc_modified_charges(self._h, int(c), _ptr(q), m, q.shape[1], _ptr(out))
        out = out.reshape(np1, np1, np1, m).transpose(3, 0, 1, 2)
        return out[0] if one else out

    def hermite_charges(self, c, charges):
        """Hermite modified charges of cluster c: (8, n+1, n+1, n+1), component
        4 a1 + 2 a2 + a3 for the derivative orders (a1, a2, a3)."""
        q = _f64(charges)
        np1 = self.degree + 1
        out = np.zeros(8 * np1 ** 3)
        _load().oracle_tc_hermite_charges(self._h, int(c), _ptr(q), _ptr(out))
        return out.reshape(8, np1, np1, np1)

    def potential(self, charges, kernel=COULOMB, kappa=0.0, sample=None, return_times=False):
        """Treecode potential at all targets (caller order), or at `sample` (indices)."""
        if self.hermite:
            return self._hermite_potential(charges, kernel, kappa, sample, return_times)
        q = _charges_2d(charges)
        one = np.asarray(charges).ndim == 1
        m = q.shape[0]
        if q.shape[1] != self.ns:
            raise ValueError("charges must have one value per source")
        if sample is None:
            ns_eval, sp = self.nt, None
        else:
            smp = np.ascontiguousarray(sample, dtype=np.int64)
            ns_eval, sp = smp.shape[0], _ptr(smp)
        phi = np.zeros((m, ns_eval))
        times = np.zeros(2)
        rc = _load().oracle_tc_potential(self._h, _ptr(q), m, q.shape[1], int(kernel),
                                         float(kappa), ns_eval, sp, _ptr(phi), ns_eval,
                                         _ptr(times))
        if rc != 0:
            raise ValueError("sample index out of range")
        res = phi[0] if one else phi
        if return_times:
            return res, {"upward": float(times[0]), "eval": float(times[1])}
        return res


def _hermite_potential_impl(tc, charges, kernel, kappa, sample, return_times):
    q = _f64(charges)
    if q.ndim != 1 or q.shape[0] != tc.ns:
        raise ValueError("the Hermite treecode takes one charge vector")
    if sample is None:
        n_eval, sp = tc.nt, None
    else:
        smp = np.ascontiguousarray(sample, dtype=np.int64)
        n_eval, sp = smp.shape[0], _ptr(smp)
    phi = np.zeros(n_eval)
    times = np.zeros(2)
    rc = _load().oracle_tc_hermite_potential(tc._h, _ptr(q), int(kernel), float(kappa), n_eval, sp,
                                             _ptr(phi), _ptr(times))
    if rc != 0:
        raise ValueError("sample index out of range")
    if return_times:
        return phi, {"upward": float(times[0]), "eval": float(times[1])}
    return phi


Treecode._hermite_potential = _hermite_potential_impl


class ClusterParticle:
    """Oracle barycentric cluster-particle treecode: the interpolation of the
    BLTC applied to the target variable.  Targets form the cluster tree
    (capacity leaf_size), the leaves of the source tree (capacity batch_size)
    are the source batches; each source batch walks the target tree with the
    MAC of eq. (13).  Single charge vector."""

    def __init__(self, targets, sources, theta, degree, leaf_size, batch_size):
        lib = _load()
        self._t = _f64(targets)
        self._s = _f64(sources)
        self._tc_cols = [np.ascontiguousarray(self._t[:, c]) for c in range(3)]
        self._sc_cols = [np.ascontiguousarray(self._s[:, c]) for c in range(3)]
        self.nt = self._t.shape[0]
        self.ns = self._s.shape[0]
        self.degree = int(degree)
        if not (1 <= self.degree <= 60):
            raise ValueError("degree out of range")
        tx, ty, tz = self._tc_cols
        sx, sy, sz = self._sc_cols
        self._h = lib.oracle_cp_create(self.nt, _ptr(tx), _ptr(ty), _ptr(tz),
                                       self.ns, _ptr(sx), _ptr(sy), _ptr(sz),
                                       float(theta), self.degree, int(leaf_size), int(batch_size))
        if not self._h:
            raise RuntimeError("oracle treecode creation failed")
        sizes = np.zeros(4, dtype=np.int64)
        lib.oracle_cp_sizes(self._h, _ptr(sizes))
        self.n_clusters, self.n_batches, self.n_items, self.n_source_nodes = (int(v) for v in sizes)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().oracle_cp_destroy(h)
            self._h = None

    def target_order(self):
        out = np.zeros(self.nt, dtype=np.int64)
        _load().oracle_cp_target_order(self._h, _ptr(out))
        return out

    def source_order(self):
        out = np.zeros(self.ns, dtype=np.int64)
        _load().oracle_cp_source_order(self._h, _ptr(out))
        return out

    def cluster(self, i):
        """Target cluster i (range in target tree order)."""
        lo = np.zeros(3)
        hi = np.zeros(3)
        bc = np.zeros(2, dtype=np.int64)
        ncl = np.zeros(10, dtype=np.int32)
        _load().oracle_cp_cluster(self._h, int(i), _ptr(lo), _ptr(hi), _ptr(bc), _ptr(ncl))
        nch = int(ncl[0])
        return {"lo": lo, "hi": hi, "begin": int(bc[0]), "count": int(bc[1]),
                "children": [int(c) for c in ncl[1:1 + nch]], "level": int(ncl[9])}

    def batch(self, b):
        """Source batch b (range in source tree order)."""
        bc = np.zeros(2, dtype=np.int64)
        _load().oracle_cp_batch(self._h, int(b), _ptr(bc))
        return {"begin": int(bc[0]), "count": int(bc[1])}

    def items(self):
        """(source batch, target cluster, kind) for every interaction; kind 0 = approx."""
        b = np.zeros(self.n_items, dtype=np.int64)
        c = np.zeros(self.n_items, dtype=np.int32)
        k = np.zeros(self.n_items, dtype=np.int32)
        _load().oracle_cp_items(self._h, _ptr(b), _ptr(c), _ptr(k))
        return b, c, k

    def proxy_potentials(self, c, charges, kernel=COULOMB, kappa=0.0):
        """Potentials at target cluster c's Chebyshev grid: (n+1, n+1, n+1)."""
        q = _f64(charges)
        if q.ndim != 1 or q.shape[0] != self.ns:
            raise ValueError("charges must have one value per source")
        np1 = self.degree + 1
        out = np.zeros(np1 ** 3)
        _load().oracle_cp_proxy_potentials(self._h, int(c), _ptr(q), int(kernel), float(kappa),
                                           _ptr(out))
        return out.reshape(np1, np1, np1)

    def potential(self, charges, kernel=COULOMB, kappa=0.0, sample=None, return_times=False):
        """Potential at all targets (caller order), or at `sample` (indices)."""
        q = _f64(charges)
        if q.ndim != 1 or q.shape[0] != self.ns:
            raise ValueError("charges must have one value per source")
        if sample is None:
            n_eval, sp = self.nt, None
        else:
            smp = np.ascontiguousarray(sample, dtype=np.int64)
            n_eval, sp = smp.shape[0], _ptr(smp)
        phi = np.zeros(n_eval)
        times = np.zeros(2)
        rc = _load().oracle_cp_potential(self._h, _ptr(q), int(kernel), float(kappa), n_eval, sp,
                                         _ptr(phi), _ptr(times))
        if rc != 0:
            raise ValueError("sample index out of range")
        if return_times:
            return phi, {"proxy": float(times[0]), "eval": float(times[1])}
        return phi


class ClusterCluster:
    """Oracle barycentric cluster-cluster treecode: source tree (capacity
    leaf_size) with modified charges, target tree (capacity batch_size) with
    proxy potentials, a dual walk from the roots choosing per accepted pair
    cluster-cluster, particle-cluster, cluster-particle or direct by the
    (n+1)^3 size test on each side.  Single charge vector."""

    KINDS = ("cc", "pc", "cp", "direct")

    def __init__(self, targets, sources, theta, degree, leaf_size, batch_size):
        lib = _load()
        self._t = _f64(targets)
        self._s = _f64(sources)
        self._tc_cols = [np.ascontiguousarray(self._t[:, c]) for c in range(3)]
        self._sc_cols = [np.ascontiguousarray(self._s[:, c]) for c in range(3)]
        self.nt = self._t.shape[0]
        self.ns = self._s.shape[0]
        self.degree = int(degree)
        if not (1 <= self.degree <= 60):
            raise ValueError("degree out of range")
        tx, ty, tz = self._tc_cols
        sx, sy, sz = self._sc_cols
        self._h = lib.oracle_cc_create(self.nt, _ptr(tx), _ptr(ty), _ptr(tz),
                                       self.ns, _ptr(sx), _ptr(sy), _ptr(sz),
                                       float(theta), self.degree, int(leaf_size), int(batch_size))
        if not self._h:
            raise RuntimeError("oracle treecode creation failed")
        sizes = np.zeros(3, dtype=np.int64)
        lib.oracle_cc_sizes(self._h, _ptr(sizes))
        self.n_target_nodes, self.n_source_nodes, self.n_pairs = (int(v) for v in sizes)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().oracle_cc_destroy(h)
            self._h = None

    def orders(self):
        """(target order, source order): original index at each tree position."""
        t = np.zeros(self.nt, dtype=np.int64)
        s = np.zeros(self.ns, dtype=np.int64)
        _load().oracle_cc_orders(self._h, _ptr(t), _ptr(s))
        return t, s

    def node(self, side, i):
        """Node i of the target (side 0) or source (side 1) tree."""
        lo = np.zeros(3)
        hi = np.zeros(3)
        bc = np.zeros(2, dtype=np.int64)
        _load().oracle_cc_node(self._h, int(side), int(i), _ptr(lo), _ptr(hi), _ptr(bc))
        return {"lo": lo, "hi": hi, "begin": int(bc[0]), "count": int(bc[1])}

    def pairs(self):
        """(target node, source node, kind) in walk order; kind 0 cc, 1 pc, 2 cp, 3 direct."""
        t = np.zeros(self.n_pairs, dtype=np.int32)
        s = np.zeros(self.n_pairs, dtype=np.int32)
        k = np.zeros(self.n_pairs, dtype=np.int32)
        _load().oracle_cc_pairs(self._h, _ptr(t), _ptr(s), _ptr(k))
        return t, s, k

    def proxy_potentials(self, c, charges, kernel=COULOMB, kappa=0.0):
        q = _f64(charges)
        if q.ndim != 1 or q.shape[0] != self.ns:
            raise ValueError("charges must have one value per source")
        np1 = self.degree + 1
        out = np.zeros(np1 ** 3)
        _load().oracle_cc_proxy_potentials(self._h, int(c), _ptr(q), int(kernel), float(kappa),
                                           _ptr(out))
        return out.reshape(np1, np1, np1)

    def potential(self, charges, kernel=COULOMB, kappa=0.0, sample=None, return_times=False):
        q = _f64(charges)
        if q.ndim != 1 or q.shape[0] != self.ns:
            raise ValueError("charges must have one value per source")
        if sample is None:
            n_eval, sp = self.nt, None
        else:
            smp = np.ascontiguousarray(sample, dtype=np.int64)
            n_eval, sp = smp.shape[0], _ptr(smp)
        phi = np.zeros(n_eval)
        times = np.zeros(2)
        rc = _load().oracle_cc_potential(self._h, _ptr(q), int(kernel), float(kappa), n_eval, sp,
                                         _ptr(phi), _ptr(times))
        if rc != 0:
            raise ValueError("sample index out of range")
        if return_times:
            return phi, {"proxy": float(times[0]), "eval": float(times[1])}
        return phi


def rel_l2(ref, approx):
    """Relative 2-norm error, eq. (16)."""
    ref = np.asarray(ref, dtype=np.float64)
    approx = np.asarray(approx, dtype=np.float64)
    den = float(np.sum(ref * ref))
    num = float(np.sum((ref - approx) ** 2))
    return (num / den) ** 0.5 if den > 0 else num ** 0.5
