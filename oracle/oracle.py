"""ctypes front end of the CPU FP64 oracle (``liboracle.so``) plus the paper's
error and balance metrics written out in numpy.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``; the GPU solver never imports it.
"""
import ctypes as C
import os

import numpy as np

from .build import ensure_built

UC, TC, TCO = 0, 1, 2
MAX_LEVEL = 21

_lib = None


def lib():
    global _lib
    if _lib is None:
        # a planted-mistake copy of the oracle can be loaded in its place
        path = os.environ.get("AMFMM_ORACLE_LIB") or ensure_built()
        L = C.CDLL(path)
        P = C.c_void_p
        d = C.POINTER(C.c_double)
        i32 = C.POINTER(C.c_int32)
        i64 = C.POINTER(C.c_int64)
        u64 = C.POINTER(C.c_uint64)
        L.orc_build_tree.restype = P
        L.orc_build_tree.argtypes = [C.c_int64, d, d, d, d, C.c_int32, C.c_int32, i32]
        L.orc_free.argtypes = [P]
        L.orc_num_cells.restype = C.c_int64
        L.orc_num_cells.argtypes = [P]
        L.orc_depth.restype = C.c_int32
        L.orc_depth.argtypes = [P]
        L.orc_get_cube.argtypes = [P, d, d, d]
        L.orc_get_keys.argtypes = [P, u64, i64]
        L.orc_get_cells.argtypes = [P, i32, i64, i64, i32, i32, i32]
        L.orc_compute_moments.restype = C.c_int32
        L.orc_compute_moments.argtypes = [P]
        L.orc_get_moments.argtypes = [P, d]
        L.orc_walk.restype = C.c_int32
        L.orc_walk.argtypes = [P, C.c_double]
        L.orc_walk_field.restype = C.c_int32
        L.orc_walk_field.argtypes = [P, C.c_double, C.c_double, d]
        L.orc_walk_multipole.restype = C.c_int32
        L.orc_walk_multipole.argtypes = [P, C.c_double, C.c_double, d]
        L.orc_multipole_levels.argtypes = [P, i32, i32]
        L.orc_num_m2l.restype = C.c_int64
        L.orc_num_m2l.argtypes = [P]
        L.orc_num_p2p.restype = C.c_int64
        L.orc_num_p2p.argtypes = [P]
        L.orc_get_lists.argtypes = [P, i32, i32]
        L.orc_evaluate.restype = C.c_int32
        L.orc_evaluate.argtypes = [P, C.c_int32, C.c_double, d, d, d, d]
        L.orc_evaluate_targets.restype = C.c_int32
        L.orc_evaluate_targets.argtypes = [P, C.c_int32, C.c_double, d, d, d, d]
        L.orc_num_threads.restype = C.c_int32
        L.orc_num_threads.argtypes = []
        L.orc_evaluate_sample.restype = C.c_int32
        L.orc_evaluate_sample.argtypes = [P, C.c_int32, C.c_double, C.c_int64, i64, d, d, d, d]
        L.orc_num_coincident.restype = C.c_int64
        L.orc_num_coincident.argtypes = [P]
        L.orc_solve.restype = C.c_int32
        L.orc_solve.argtypes = [C.c_int64, d, d, d, d, C.c_double, C.c_int32, C.c_int32,
                                C.c_double, d, d, d, d]
        L.orc_direct.restype = C.c_int32
        L.orc_direct.argtypes = [C.c_int64, d, d, d, d, C.c_int64, i64, C.c_double,
                                 d, d, d, d, d]
        L.orc_greens.argtypes = [d, d, d, d, d, d, d]
        L.orc_greens_softened.argtypes = [d, C.c_double, d, d, d, d, d, d]
        L.orc_set_softening.restype = C.c_int32
        L.orc_set_softening.argtypes = [P, C.c_double]
        L.orc_set_order.restype = C.c_int32
        L.orc_set_order.argtypes = [P, C.c_int32]
        L.orc_set_order_form.restype = C.c_int32
        L.orc_set_order_form.argtypes = [P, C.c_int32, C.c_int32]
        L.orc_num_multi_indices.restype = C.c_int32
        L.orc_num_multi_indices.argtypes = [C.c_int32]
        L.orc_multi_indices.argtypes = [C.c_int32, i32]
        L.orc_greens_general.argtypes = [d, C.c_double, C.c_int32, d]
        L.orc_pair_far_order.argtypes = [C.c_int32, C.c_int32, C.c_int64, d, d, d, d, C.c_int64, d, d, d, d, C.c_int32,
                                         d, d, d, d]
        L.orc_direct_softened.restype = C.c_int32
        L.orc_direct_softened.argtypes = [C.c_int64, d, d, d, d, C.c_int64, i64, C.c_double, C.c_double,
                                          d, d, d, d, d]
        L.orc_cluster_moments.argtypes = [C.c_int64, d, d, d, d, d]
        L.orc_pair_far.argtypes = [C.c_int64, d, d, d, d, C.c_int64, d, d, d, d, C.c_int32,
                                   d, d, d, d]
        f = C.POINTER(C.c_float)
        L.orc_walk_learned.restype = C.c_int32
        L.orc_walk_learned.argtypes = [P, C.c_double, C.c_double, C.c_double, d, f, C.c_int64]
        L.orc_pair_features.argtypes = [P, C.c_int64, i32, f]
        L.orc_pair_labels.restype = C.c_int32
        L.orc_pair_labels.argtypes = [P, C.c_int32, C.c_int64, i32, d]
        L.orc_pair_errors.restype = C.c_int32
        L.orc_pair_errors.argtypes = [P, C.c_int32, C.c_int64, i32, d]
        L.orc_multipole_weights.argtypes = [d]
        L.orc_bf16_round.restype = C.c_float
        L.orc_bf16_round.argtypes = [C.c_float]
        L.orc_plog2.restype = C.c_double
        L.orc_plog2.argtypes = [C.c_double]
        L.orc_mlp_predict.argtypes = [f, C.c_int64, f, f]
        L.orc_mlp_grad.restype = C.c_double
        L.orc_mlp_grad.argtypes = [f, C.c_int64, f, f, C.c_double, C.c_int32, d]
        L.orc_mlp_adam.argtypes = [f, f, f, f, C.c_int64, C.c_double, C.c_double, C.c_double,
                                   C.c_double]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def multipole_weights():
    """The multipole error estimate's weights (w1..w5)."""
    w = np.zeros(5)
    lib().orc_multipole_weights(_d(w))
    return w


class Tree:
    """Octree of the oracle: build (a1-a4), moments (a5), walk (a6), evaluate."""

    def __init__(self, x, y, z, m, n_crit=25, max_level=MAX_LEVEL, softening=0.0, order=3):
        self._keep = [_f64(v) for v in (x, y, z, m)]
        x, y, z, m = self._keep
        st = C.c_int32(0)
        self.n = len(x)
        self._t = lib().orc_build_tree(self.n, _d(x), _d(y), _d(z), _d(m), n_crit, max_level,
                                       C.byref(st))
        if not self._t:
            raise OracleError(st.value)
        if softening:
            self.set_softening(softening)
        if order != 3:
            self.set_order(order)

    def set_order(self, P, general=None):
        """Expansion order P of every later evaluation (3: the printed
        equations; others, or general=True: the appendix's general form, UC
        and TC)."""
        g = (P != 3) if general is None else bool(general)
        st = lib().orc_set_order_form(self._t, int(P), int(g))
        if st:
            raise OracleError(st)

    def set_softening(self, eps):
        """Plummer softening length of every later evaluation (0 = plain 1/R)."""
        st = lib().orc_set_softening(self._t, float(eps))
        if st:
            raise OracleError(st)

    def __del__(self):
        if getattr(self, "_t", None):
            lib().orc_free(self._t)
            self._t = None

    @property
    def num_cells(self):
        return lib().orc_num_cells(self._t)

    @property
    def depth(self):
        return lib().orc_depth(self._t)

    def cube(self):
        lo = np.zeros(3)
        side = C.c_double()
        scale = C.c_double()
        lib().orc_get_cube(self._t, _d(lo), C.byref(side), C.byref(scale))
        return lo, side.value, scale.value

    def keys(self):
        k = np.zeros(self.n, np.uint64)
        p = np.zeros(self.n, np.int64)
        lib().orc_get_keys(self._t, k.ctypes.data_as(C.POINTER(C.c_uint64)),
                           p.ctypes.data_as(C.POINTER(C.c_int64)))
        return k, p

    def cells(self):
        nc = self.num_cells
        out = dict(level=np.zeros(nc, np.int32), begin=np.zeros(nc, np.int64),
                   count=np.zeros(nc, np.int64), parent=np.zeros(nc, np.int32),
                   child0=np.zeros(nc, np.int32), nchild=np.zeros(nc, np.int32))
        ptr = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32 if a.dtype == np.int32 else C.c_int64))
        lib().orc_get_cells(self._t, ptr(out["level"]), ptr(out["begin"]), ptr(out["count"]),
                            ptr(out["parent"]), ptr(out["child0"]), ptr(out["nchild"]))
        return out

    def compute_moments(self):
        st = lib().orc_compute_moments(self._t)
        if st:
            raise OracleError(st)

    def moments(self):
        out = np.zeros((self.num_cells, 21))
        lib().orc_get_moments(self._t, _d(out))
        return out

    def walk(self, theta):
        st = lib().orc_walk(self._t, float(theta))
        if st:
            raise OracleError(st)

    def walk_field(self, eps, theta_max, gmag):
        """Walk with the error-estimate criterion against per-particle |g|."""
        g = _f64(gmag)
        st = lib().orc_walk_field(self._t, float(eps), float(theta_max), _d(g))
        if st:
            raise OracleError(st)

    def walk_learned(self, eps, theta_max, theta, gmag, model, min_work=1 << 18):
        """Walk whose accept decision asks the network (model: MLP_MODEL floats,
        or None for the opening-angle walk) for pairs with N_A N_B >= min_work."""
        g = _f64(gmag)
        mp = None
        if model is not None:
            model = _f32(model)
            assert model.size == MLP_MODEL
            mp = _fp(model)
        st = lib().orc_walk_learned(self._t, float(eps), float(theta_max), float(theta), _d(g), mp, int(min_work))
        if st:
            raise OracleError(st)

    def pair_features(self, pairs):
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        out = np.zeros((len(pairs), 8), np.float32)
        lib().orc_pair_features(self._t, len(pairs), pairs.ctypes.data_as(C.POINTER(C.c_int32)), _fp(out))
        return out

    def pair_labels(self, pairs, variant=TC):
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        out = np.zeros(len(pairs))
        st = lib().orc_pair_labels(self._t, variant, len(pairs), pairs.ctypes.data_as(C.POINTER(C.c_int32)),
                                   _d(out))
        if st:
            raise OracleError(st)
        return out

    def pair_errors(self, pairs, variant=TC):
        """The method's largest error from each pair alone on its first and
        on its second cell (n x 2)."""
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        out = np.zeros((len(pairs), 2))
        st = lib().orc_pair_errors(self._t, variant, len(pairs), pairs.ctypes.data_as(C.POINTER(C.c_int32)),
                                   _d(out))
        if st:
            raise OracleError(st)
        return out

    def walk_multipole(self, eps, theta_max, gmag):
        """Walk with the multipole error estimate against per-particle |g|."""
        g = _f64(gmag)
        st = lib().orc_walk_multipole(self._t, float(eps), float(theta_max), _d(g))
        if st:
            raise OracleError(st)

    def multipole_levels(self):
        k2 = np.zeros(self.num_cells, np.int32)
        k3 = np.zeros(self.num_cells, np.int32)
        lib().orc_multipole_levels(self._t, k2.ctypes.data_as(C.POINTER(C.c_int32)),
                                   k3.ctypes.data_as(C.POINTER(C.c_int32)))
        return k2, k3

    def lists(self):
        nm = lib().orc_num_m2l(self._t)
        npp = lib().orc_num_p2p(self._t)
        m2l = np.zeros((nm, 2), np.int32)
        p2p = np.zeros((npp, 2), np.int32)
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        lib().orc_get_lists(self._t, ip(m2l), ip(p2p))
        return m2l, p2p

    def evaluate(self, variant=TC, G=1.0):
        n = self.n
        ax, ay, az, pot = (np.zeros(n) for _ in range(4))
        st = lib().orc_evaluate(self._t, variant, float(G), _d(ax), _d(ay), _d(az), _d(pot))
        if st:
            raise OracleError(st)
        return np.stack([ax, ay, az]), pot

    def evaluate_targets(self, variant=TC, G=1.0):
        """The same evaluation organised by target (all host cores in the
        OpenMP build); equal to evaluate() up to summation order."""
        n = self.n
        ax, ay, az, pot = (np.zeros(n) for _ in range(4))
        st = lib().orc_evaluate_targets(self._t, variant, float(G), _d(ax), _d(ay), _d(az), _d(pot))
        if st:
            raise OracleError(st)
        return np.stack([ax, ay, az]), pot

    def evaluate_sample(self, idx, variant=TC, G=1.0):
        """Same evaluation at the caller indices idx only."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        k = len(idx)
        ax, ay, az, pot = (np.zeros(k) for _ in range(4))
        st = lib().orc_evaluate_sample(self._t, variant, float(G), k,
                                       idx.ctypes.data_as(C.POINTER(C.c_int64)),
                                       _d(ax), _d(ay), _d(az), _d(pot))
        if st:
            raise OracleError(st)
        return np.stack([ax, ay, az]), pot

    @property
    def coincident(self):
        return lib().orc_num_coincident(self._t)


def num_threads():
    """Threads the loaded oracle library's target-ordered evaluation uses."""
    return lib().orc_num_threads()


def use_openmp_build():
    """Load the OpenMP build of the oracle in place of the serial one (the
    benchmark's CPU baseline; call before any other oracle call)."""
    from .build import ensure_built_omp
    global _lib
    if _lib is None:
        os.environ["AMFMM_ORACLE_LIB"] = ensure_built_omp()


def solve(x, y, z, m, theta=0.5, n_crit=25, variant=TC, G=1.0, softening=0.0, order=3):
    """Whole FMM solve; returns (acc[3,n], pot[n]) in caller order."""
    if softening or order != 3:
        t = Tree(x, y, z, m, n_crit=n_crit, softening=softening, order=order)
        t.compute_moments()
        t.walk(theta)
        a, p = t.evaluate(variant, G)
        return a, p
    x, y, z, m = (_f64(v) for v in (x, y, z, m))
    n = len(x)
    ax, ay, az, pot = (np.zeros(n) for _ in range(4))
    st = lib().orc_solve(n, _d(x), _d(y), _d(z), _d(m), float(theta), n_crit, variant, float(G),
                         _d(ax), _d(ay), _d(az), _d(pot))
    if st:
        raise OracleError(st)
    return np.stack([ax, ay, az]), pot


def leapfrog(x, y, z, vx, vy, vz, m, theta, dt, steps, n_crit=25, variant=TC, G=1.0, acc=None, softening=0.0):
    """Uniform-step kick-drift-kick leapfrog with the oracle's forces (Sec. 1
    and Sec. 4 ask for one time step for every particle): per step
    v += (dt/2) a, x += dt v, a = solve(x), v += (dt/2) a.  acc: the
    accelerations at the starting positions ([3, n]; solved when None).
    Returns the new (x, y, z, vx, vy, vz, acc) as float64 copies."""
    pos = np.stack([_f64(x), _f64(y), _f64(z)]).copy()
    vel = np.stack([_f64(vx), _f64(vy), _f64(vz)]).copy()
    m = _f64(m)
    if acc is None:
        acc, _ = solve(pos[0], pos[1], pos[2], m, theta, n_crit, variant, G, softening)
    acc = np.array(acc, dtype=np.float64)
    for _ in range(steps):
        vel += (0.5 * dt) * acc
        pos += dt * vel
        acc, _ = solve(pos[0], pos[1], pos[2], m, theta, n_crit, variant, G, softening)
        vel += (0.5 * dt) * acc
    return pos[0], pos[1], pos[2], vel[0], vel[1], vel[2], acc


def direct(x, y, z, m, targets=None, G=1.0, softening=0.0):
    """Exact direct sum; returns (acc[3,t], pot[t], gabs[t]) for the targets
    (softened Green's function when softening > 0)."""
    x, y, z, m = (_f64(v) for v in (x, y, z, m))
    n = len(x)
    if targets is None:
        nt = n
        tp = None
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        nt = len(targets)
        tp = targets.ctypes.data_as(C.POINTER(C.c_int64))
    ax, ay, az, pot, gabs = (np.zeros(nt) for _ in range(5))
    st = lib().orc_direct_softened(n, _d(x), _d(y), _d(z), _d(m), nt, tp, float(G), float(softening),
                                   _d(ax), _d(ay), _d(az), _d(pot), _d(gabs))
    if st:
        raise OracleError(st)
    return np.stack([ax, ay, az]), pot, gabs


def greens_softened(R, eps):
    """D0..D4 and D'_ijkl of the softened g = -1/sqrt(R^2 + eps^2) as full tensors."""
    R = _f64(R)
    D0 = np.zeros(1)
    D1 = np.zeros(3)
    D2 = np.zeros((3, 3))
    D3 = np.zeros((3, 3, 3))
    D4 = np.zeros((3, 3, 3, 3))
    D4p = np.zeros((3, 3, 3, 3))
    lib().orc_greens_softened(_d(R), float(eps), _d(D0), _d(D1), _d(D2), _d(D3), _d(D4), _d(D4p))
    return D0[0], D1, D2, D3, D4, D4p


def greens(R):
    R = _f64(R)
    D0 = np.zeros(1)
    D1 = np.zeros(3)
    D2 = np.zeros((3, 3))
    D3 = np.zeros((3, 3, 3))
    D4 = np.zeros((3, 3, 3, 3))
    D4p = np.zeros((3, 3, 3, 3))
    lib().orc_greens(_d(R), _d(D0), _d(D1), _d(D2), _d(D3), _d(D4), _d(D4p))
    return D0[0], D1, D2, D3, D4, D4p


# ------------------------------------------------- learned pair selection --
MLP_PARAMS = 4801
MLP_MODEL = 4833


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def bf16_round(v):
    return float(lib().orc_bf16_round(float(v)))


def plog2(x):
    return float(lib().orc_plog2(float(x)))


def mlp_predict(model, feats):
    model, feats = _f32(model), _f32(feats).reshape(-1, 8)
    y = np.zeros(len(feats), np.float32)
    lib().orc_mlp_predict(_fp(model), len(feats), _fp(feats), _fp(y))
    return y


def mlp_grad(model, feats, labels, tau=0.9, round=True):
    """(mean pinball loss, gradient over the MLP_PARAMS trainable entries)."""
    model, feats, labels = _f32(model), _f32(feats).reshape(-1, 8), _f32(labels)
    g = np.zeros(MLP_PARAMS)
    loss = lib().orc_mlp_grad(_fp(model), len(feats), _fp(feats), _fp(labels), float(tau), int(bool(round)), _d(g))
    return loss, g


def mlp_adam(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; params, m, v (float32) are updated in place."""
    for a in (params, m, v):
        assert a.dtype == np.float32 and a.flags.c_contiguous
    g = _f32(grad)
    lib().orc_mlp_adam(_fp(params), _fp(g), _fp(m), _fp(v), int(t), float(lr), float(beta1), float(beta2),
                       float(eps))


def cluster_moments(x, y, z, m):
    x, y, z, m = (_f64(v) for v in (x, y, z, m))
    out = np.zeros(21)
    lib().orc_cluster_moments(len(x), _d(x), _d(y), _d(z), _d(m), _d(out))
    return out


def multi_indices(n):
    """Multi-indices (a, b, c) of order <= n, graded ([k, 3] int array)."""
    k = lib().orc_num_multi_indices(int(n))
    out = np.zeros((k, 3), np.int32)
    lib().orc_multi_indices(int(n), out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out


def greens_general(R, n, eps=0.0):
    """D_alpha(R) for |alpha| <= n in the order of multi_indices(n)."""
    R = _f64(R)
    out = np.zeros(lib().orc_num_multi_indices(int(n)))
    lib().orc_greens_general(_d(R), float(eps), int(n), _d(out))
    return out


def pair_far(A, B, variant=TC, order=3, general=False):
    """A, B: (x, y, z, m) tuples.  Far-field accelerations [n,3] and potentials."""
    xa, ya, za, ma = (_f64(v) for v in A)
    xb, yb, zb, mb = (_f64(v) for v in B)
    na, nb = len(xa), len(xb)
    gA = np.zeros((na, 3))
    gB = np.zeros((nb, 3))
    pA = np.zeros(na)
    pB = np.zeros(nb)
    lib().orc_pair_far_order(int(order), int(general), na, _d(xa), _d(ya), _d(za), _d(ma), nb, _d(xb), _d(yb), _d(zb), _d(mb),
                             variant, _d(gA), _d(pA), _d(gB), _d(pB))
    return gA, pA, gB, pB


# ----------------------------------------------------------------- metrics --
def balance(m, A):
    """Net balance of Sec. 3: sqrt(sum_d (sum_n m_n A_nd)^2 / sum_d (sum_n m_n |A_nd|)^2).

    A is [3, n] (linear accelerations, or X x g for the angular ones).  Sums are
    taken with math.fsum so that the metric itself adds no round-off."""
    import math
    num = sum(math.fsum(m * A[d]) ** 2 for d in range(3))
    den = sum(math.fsum(m * np.abs(A[d])) ** 2 for d in range(3))
    return math.sqrt(num / den)


def angular(pos, acc):
    """X x g for every particle (pos, acc as [3, n])."""
    return np.cross(pos.T, acc.T).T


def rel_force_error(acc, acc_true):
    """epsilon_n = |g_n - g_PP,n| / |g_PP,n| (Sec. 3), skipping zero truths."""
    num = np.linalg.norm(acc - acc_true, axis=0)
    den = np.linalg.norm(acc_true, axis=0)
    ok = den > 0
    return num[ok] / den[ok]


def rel_torque_error(pos, acc, acc_true):
    """Same with X x g about the coordinate origin (Sec. 3)."""
    t = angular(pos, acc)
    tt = angular(pos, acc_true)
    num = np.linalg.norm(t - tt, axis=0)
    den = np.linalg.norm(tt, axis=0)
    ok = den > 0
    return num[ok] / den[ok]
