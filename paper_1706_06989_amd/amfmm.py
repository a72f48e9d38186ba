"""Python binding of libamfmm_hip.so (ctypes; argument marshalling only).

Every call goes straight to the C ABI declared in ``include/amfmm.h``; all
work runs in the library's HIP kernels.  Tensors are torch CUDA (ROCm)
float64 tensors used only as device memory; the library enqueues on the
current torch stream of the context.  Importing this module fails loudly when
the native library is missing: there is no fallback.
"""
import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamfmm_hip.so")

OK, E_INVALID, E_NONFINITE, E_OOM, E_HIP, E_STATE = 0, -1, -2, -3, -4, -5
UC, TC, TCO = 0, 1, 2
FP64, MIXED = 0, 1
GEOMETRIC, ESTIMATE, LEARNED, MULTIPOLE = 0, 1, 2, 3
MLP_PARAMS, MLP_MODEL = 4801, 4833
PHASES = ["validate+bbox", "keys+sort", "tree", "moments", "walk", "far", "push-down",
          "near+eval", "total", "walk-pass"]


class amfmm_options(C.Structure):
    _fields_ = [("n_crit", C.c_int32), ("variant", C.c_int32), ("precision", C.c_int32),
                ("criterion", C.c_int32), ("G", C.c_double), ("error_tol", C.c_double),
                ("theta_max", C.c_double), ("max_bytes", C.c_int64), ("list_bytes", C.c_int64),
                ("learned_min_work", C.c_int64), ("softening", C.c_double), ("order", C.c_int32)]


_lib = None


def lib():
    """Load libamfmm_hip.so and declare every exported symbol."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(there is no non-HIP fallback)")
    L = C.CDLL(LIB_PATH)
    P, d, i64, i32, u64 = (C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.c_int32,
                           C.POINTER(C.c_uint64))
    pd = C.c_void_p  # device pointers are passed as integers
    sig = {
        "amfmm_default_options": (C.c_int, [C.POINTER(amfmm_options)]),
        "amfmm_create": (C.c_int, [C.POINTER(amfmm_options), P, C.POINTER(P)]),
        "amfmm_destroy": (C.c_int, [P]),
        "amfmm_set_stream": (C.c_int, [P, P]),
        "amfmm_set_field_estimate": (C.c_int, [P, pd, pd, pd]),
        "amfmm_build_tree": (C.c_int, [P, i64, pd, pd, pd, pd]),
        "amfmm_compute_moments": (C.c_int, [P]),
        "amfmm_walk": (C.c_int, [P, C.c_double]),
        "amfmm_evaluate": (C.c_int, [P, pd, pd, pd, pd]),
        "amfmm_solve_gravity": (C.c_int, [P, i64, pd, pd, pd, pd, C.c_double, pd, pd, pd, pd]),
        "amfmm_solve_gravity_noalloc": (C.c_int, [P, i64, pd, pd, pd, pd, C.c_double, pd, pd, pd, pd]),
        "amfmm_leapfrog": (C.c_int, [P, i64, pd, pd, pd, pd, pd, pd, pd, C.c_double, C.c_double, i32,
                                     pd, pd, pd]),
        "amfmm_direct": (C.c_int, [P, i64, pd, pd, pd, pd, i64, pd, pd, pd, pd, pd, pd]),
        "amfmm_balance": (C.c_int, [P, i64, pd, pd, pd, pd, pd, pd, pd, d]),
        "amfmm_get_counts": (C.c_int, [P, C.POINTER(C.c_int64)]),
        "amfmm_get_tree": (C.c_int, [P, u64, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)]),
        "amfmm_get_moments": (C.c_int, [P, d]),
        "amfmm_get_lists": (C.c_int, [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "amfmm_get_phase_times": (C.c_int, [P, d, i32]),
        "amfmm_set_model": (C.c_int, [P, C.POINTER(C.c_float)]),
        "amfmm_pair_features": (C.c_int, [P, i64, pd, pd]),
        "amfmm_pair_labels": (C.c_int, [P, i32, i64, pd, pd]),
        "amfmm_mlp_predict": (C.c_int, [P, i64, pd, pd, pd]),
        "amfmm_mlp_grad": (C.c_int, [P, i64, pd, pd, pd, C.c_double, pd, d]),
        "amfmm_mlp_train": (C.c_int, [P, i64, pd, pd, pd, pd, pd, i64, i32, i32, C.c_double,
                                      C.c_double, d]),
        "amfmm_status_string": (C.c_char_p, [C.c_int]),
        "amfmm_last_error": (C.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = ["amfmm_default_options", "amfmm_create", "amfmm_destroy", "amfmm_set_stream",
            "amfmm_set_field_estimate",
            "amfmm_build_tree", "amfmm_compute_moments", "amfmm_walk", "amfmm_evaluate",
            "amfmm_solve_gravity", "amfmm_solve_gravity_noalloc", "amfmm_leapfrog", "amfmm_direct", "amfmm_balance", "amfmm_get_counts",
            "amfmm_get_tree", "amfmm_get_moments", "amfmm_get_lists", "amfmm_get_phase_times",
            "amfmm_set_model", "amfmm_pair_features", "amfmm_pair_labels", "amfmm_mlp_predict",
            "amfmm_mlp_grad", "amfmm_mlp_train", "amfmm_status_string", "amfmm_last_error"]


class AmfmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"amfmm status {code}: {msg}")
        self.code = code


def _dev(t, name, n=None):
    """Device pointer of a contiguous float64 CUDA tensor holding exactly n
    elements (when n is given): the library reads n elements through it."""
    return _devt(t, name, torch.float64, n)


def _devt(t, name, dtype, n=None):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (ROCm) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, {n} expected")
    return C.c_void_p(t.data_ptr())


def _rows(t, name, width):
    """Rows of a [rows, width] tensor (checked: the library reads rows x width)."""
    if not isinstance(t, torch.Tensor) or t.dim() != 2 or t.shape[1] != width:
        raise ValueError(f"{name} must be a [rows, {width}] tensor")
    return t.shape[0]


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class Solver:
    """One amfmm context.  Method names follow the C ABI without the prefix."""

    def __init__(self, n_crit=25, variant=TC, precision=FP64, criterion=GEOMETRIC, G=1.0,
                 error_tol=1e-4, theta_max=1.0, max_bytes=0, list_bytes=0, learned_min_work=1 << 18,
                 stream=None, softening=0.0, order=3):
        L = lib()
        o = amfmm_options()
        L.amfmm_default_options(C.byref(o))
        o.n_crit, o.variant, o.precision, o.criterion = n_crit, variant, precision, criterion
        o.G, o.error_tol, o.theta_max, o.max_bytes = G, error_tol, theta_max, max_bytes
        o.list_bytes = list_bytes
        o.learned_min_work = learned_min_work
        o.softening = softening
        o.order = order
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        st = L.amfmm_create(C.byref(o), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st:
            raise AmfmmError(st, L.amfmm_status_string(st).decode())
        self._h = h
        self.n = 0

    def close(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.amfmm_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st < 0:
            raise AmfmmError(st, lib().amfmm_last_error(self._h).decode())
        return st

    def set_field_estimate(self, gx, gy=None, gz=None):
        """Per-particle field estimates (CUDA float64, caller order) for the
        error-estimate criteria (ESTIMATE, MULTIPOLE, LEARNED): magnitudes (gx only) or the three
        components; None clears them.  The tensors are kept alive by the
        solver until replaced."""
        self._field = (gx, gy, gz)
        d = lambda t, nm: _dev(t, nm) if t is not None else None
        self._check(lib().amfmm_set_field_estimate(self._h, d(gx, "gx"), d(gy, "gy"), d(gz, "gz")))

    def set_model(self, model):
        """Install a network (AMFMM_MLP_MODEL floats, host array or None)."""
        if model is None:
            self._check(lib().amfmm_set_model(self._h, None))
            return
        m = np.ascontiguousarray(model, dtype=np.float32)
        if m.size != MLP_MODEL:
            raise ValueError(f"a model has {MLP_MODEL} floats")
        self._check(lib().amfmm_set_model(self._h, _ptr(m, C.c_float)))

    def pair_features(self, pairs):
        """pairs: CUDA int32 tensor [np, 2] of cells of the current tree."""
        np_ = _rows(pairs, "pairs", 2)
        out = torch.empty((np_, 8), dtype=torch.float32, device=pairs.device)
        self._check(lib().amfmm_pair_features(self._h, np_, _devt(pairs, "pairs", torch.int32),
                                              _devt(out, "feats", torch.float32)))
        return out

    def pair_labels(self, pairs, variant=TC):
        np_ = _rows(pairs, "pairs", 2)
        out = torch.empty(np_, dtype=torch.float64, device=pairs.device)
        self._check(lib().amfmm_pair_labels(self._h, variant, np_, _devt(pairs, "pairs", torch.int32),
                                            _devt(out, "labels", torch.float64)))
        return out

    def mlp_predict(self, model, feats):
        """model: CUDA float32 [MLP_MODEL]; feats: CUDA float32 [n, 8]."""
        n = _rows(feats, "feats", 8)
        y = torch.empty(n, dtype=torch.float32, device=feats.device)
        self._check(lib().amfmm_mlp_predict(self._h, n, _devt(model, "model", torch.float32, MLP_MODEL),
                                            _devt(feats, "feats", torch.float32), _devt(y, "y", torch.float32)))
        return y

    def mlp_grad(self, model, feats, labels, tau=0.9):
        n = _rows(feats, "feats", 8)
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feats.device)
        loss = np.zeros(1)
        self._check(lib().amfmm_mlp_grad(self._h, n, _devt(model, "model", torch.float32, MLP_MODEL),
                                         _devt(feats, "feats", torch.float32),
                                         _devt(labels, "labels", torch.float32, n), float(tau),
                                         _devt(g, "grad", torch.float32), _ptr(loss, C.c_double)))
        return float(loss[0]), g

    def mlp_train(self, feats, labels, model, adam_m, adam_v, step0, steps, batch, lr, tau=0.9):
        """Adam steps on the pinball loss; model, adam_m, adam_v updated in place."""
        n = _rows(feats, "feats", 8)
        loss = np.zeros(1)
        self._check(lib().amfmm_mlp_train(self._h, n, _devt(feats, "feats", torch.float32),
                                          _devt(labels, "labels", torch.float32, n),
                                          _devt(model, "model", torch.float32, MLP_MODEL),
                                          _devt(adam_m, "adam_m", torch.float32, MLP_PARAMS),
                                          _devt(adam_v, "adam_v", torch.float32, MLP_PARAMS), int(step0),
                                          int(steps), int(batch), float(lr), float(tau), _ptr(loss, C.c_double)))
        return float(loss[0])

    def build_tree(self, x, y, z, m):
        n = x.numel()
        self._check(lib().amfmm_build_tree(self._h, n, _dev(x, "x", n), _dev(y, "y", n),
                                           _dev(z, "z", n), _dev(m, "m", n)))
        self.n = n

    def compute_moments(self):
        self._check(lib().amfmm_compute_moments(self._h))

    def walk(self, theta):
        self._check_field(self.n)
        self._check(lib().amfmm_walk(self._h, float(theta)))

    def _outputs(self, n, pot):
        dev = torch.device("cuda", torch.cuda.current_device())
        ax, ay, az = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
        p = torch.empty(n, dtype=torch.float64, device=dev) if pot else None
        return ax, ay, az, p

    def evaluate(self, out=None, pot=True):
        n = self.n
        ax, ay, az, p = out if out is not None else self._outputs(n, pot)
        self._check_field(n)
        self._check(lib().amfmm_evaluate(self._h, _dev(ax, "ax", n), _dev(ay, "ay", n), _dev(az, "az", n),
                                         _dev(p, "pot", n) if p is not None else None))
        return ax, ay, az, p

    def _check_field(self, n):
        # the library reads n elements of each installed field estimate
        for t, nm in zip(getattr(self, "_field", (None, None, None)), ("gx", "gy", "gz")):
            if t is not None and t.numel() != n:
                raise ValueError(f"field estimate {nm} has {t.numel()} elements, {n} expected")

    def solve_gravity(self, x, y, z, m, theta, out=None, pot=True):
        n = x.numel()
        ax, ay, az, p = out if out is not None else self._outputs(n, pot)
        self._check_field(n)
        args = (_dev(x, "x", n), _dev(y, "y", n), _dev(z, "z", n), _dev(m, "m", n), float(theta),
                _dev(ax, "ax", n), _dev(ay, "ay", n), _dev(az, "az", n),
                _dev(p, "pot", n) if p is not None else None)
        self.n = n
        self._check(lib().amfmm_solve_gravity(self._h, n, *args))
        return ax, ay, az, p

    def solve_gravity_noalloc(self, x, y, z, m, theta, out):
        """amfmm_solve_gravity_noalloc: the solve without device allocation
        (scratch in the library's static array); out = (ax, ay, az, pot or
        None), preallocated by the caller."""
        n = x.numel()
        ax, ay, az, p = out
        self._check_field(n)
        args = (_dev(x, "x", n), _dev(y, "y", n), _dev(z, "z", n), _dev(m, "m", n), float(theta),
                _dev(ax, "ax", n), _dev(ay, "ay", n), _dev(az, "az", n),
                _dev(p, "pot", n) if p is not None else None)
        self.n = n
        self._check(lib().amfmm_solve_gravity_noalloc(self._h, n, *args))
        return ax, ay, az, p

    def leapfrog(self, x, y, z, vx, vy, vz, m, theta, dt, steps, acc):
        """amfmm_leapfrog: `steps` kick-drift-kick steps of dt in place on the
        positions and velocities; acc = (ax, ay, az) holds the accelerations at
        the positions on entry and at the new ones on return."""
        n = x.numel()
        ax, ay, az = acc
        self._check_field(n)
        self._check(lib().amfmm_leapfrog(self._h, n, _dev(x, "x", n), _dev(y, "y", n), _dev(z, "z", n),
                                         _dev(vx, "vx", n), _dev(vy, "vy", n), _dev(vz, "vz", n),
                                         _dev(m, "m", n), float(theta), float(dt), int(steps),
                                         _dev(ax, "ax", n), _dev(ay, "ay", n), _dev(az, "az", n)))
        self.n = n
        return acc

    def direct(self, x, y, z, m, targets=None, pot=True, gabs=True):
        n = x.numel()
        nt = n if targets is None else targets.numel()
        if targets is not None and (targets.dtype != torch.int64 or targets.device.type != "cuda"):
            raise TypeError("targets must be a CUDA int64 tensor")
        if targets is not None and not targets.is_contiguous():
            raise TypeError("targets must be contiguous")
        ax, ay, az, p = self._outputs(nt, pot)
        g = torch.empty(nt, dtype=torch.float64, device=x.device) if gabs else None
        tp = C.c_void_p(targets.data_ptr()) if targets is not None else None
        self._check(lib().amfmm_direct(self._h, n, _dev(x, "x", n), _dev(y, "y", n), _dev(z, "z", n),
                                       _dev(m, "m", n), nt, tp, _dev(ax, "ax"), _dev(ay, "ay"),
                                       _dev(az, "az"), _dev(p, "pot") if p is not None else None,
                                       _dev(g, "gabs") if g is not None else None))
        return ax, ay, az, p, g

    def balance(self, x, y, z, m, ax, ay, az):
        n = x.numel()
        out = np.zeros(2)
        self._check(lib().amfmm_balance(self._h, n, _dev(x, "x", n), _dev(y, "y", n),
                                        _dev(z, "z", n), _dev(m, "m", n), _dev(ax, "ax", n),
                                        _dev(ay, "ay", n), _dev(az, "az", n), _ptr(out, C.c_double)))
        return float(out[0]), float(out[1])

    def get_counts(self):
        c = np.zeros(12, np.int64)
        self._check(lib().amfmm_get_counts(self._h, _ptr(c, C.c_int64)))
        keys = ["cells", "depth", "far_pairs", "near_pairs", "leaves", "particles",
                "near_interactions", "far_evaluations", "far_launches", "near_launches",
                "walk_candidates", "walk_pass_launches"]
        return dict(zip(keys, (int(v) for v in c)))

    def get_tree(self):
        cnt = self.get_counts()
        n, nc = cnt["particles"], cnt["cells"]
        keys = np.zeros(n, np.uint64)
        perm = np.zeros(n, np.int64)
        level = np.zeros(nc, np.int32)
        begin = np.zeros(nc, np.int64)
        count = np.zeros(nc, np.int64)
        parent = np.zeros(nc, np.int32)
        child0 = np.zeros(nc, np.int32)
        nchild = np.zeros(nc, np.int32)
        self._check(lib().amfmm_get_tree(self._h, _ptr(keys, C.c_uint64), _ptr(perm, C.c_int64),
                                         _ptr(level, C.c_int32), _ptr(begin, C.c_int64),
                                         _ptr(count, C.c_int64), _ptr(parent, C.c_int32),
                                         _ptr(child0, C.c_int32), _ptr(nchild, C.c_int32)))
        return dict(keys=keys, perm=perm, level=level, begin=begin, count=count, parent=parent,
                    child0=child0, nchild=nchild)

    def get_moments(self):
        nc = self.get_counts()["cells"]
        out = np.zeros((nc, 21))
        self._check(lib().amfmm_get_moments(self._h, _ptr(out, C.c_double)))
        return out

    def get_lists(self):
        cnt = self.get_counts()
        far = np.zeros((cnt["far_pairs"], 2), np.int32)
        near = np.zeros((cnt["near_pairs"], 2), np.int32)
        self._check(lib().amfmm_get_lists(self._h, _ptr(far, C.c_int32), _ptr(near, C.c_int32)))
        return far, near

    def get_phase_times(self):
        ms = np.zeros(len(PHASES))
        k = self._check(lib().amfmm_get_phase_times(self._h, _ptr(ms, C.c_double), len(PHASES)))
        return dict(zip(PHASES[:k], ms[:k].tolist()))
