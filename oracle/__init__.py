"""ctypes wrapper of the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports this package.

Coordinates are numpy float64 arrays in structure-of-arrays order, shape (3, N)
for one walker or (W, 3, N) for several.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))


class System(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("order", C.c_int32),
        ("L", C.c_double),
        ("b", C.c_double),
        ("hbar2_over_m", C.c_double),
        ("step_sigma", C.c_double),
        ("seed", C.c_uint64),
        ("fp32_coords", C.c_int32),
    ]


WALKER_FIELDS = [
    ("u_run", C.c_double), ("v_run", C.c_double),
    ("sum_e", C.c_double), ("c_e", C.c_double),
    ("sum_e2", C.c_double), ("c_e2", C.c_double),
    ("sum_v", C.c_double), ("c_v", C.c_double),
    ("sum_tpb", C.c_double), ("c_tpb", C.c_double),
    ("sum_tjf", C.c_double), ("c_tjf", C.c_double),
    ("sum_tf", C.c_double), ("c_tf", C.c_double),
    ("sum_vs", C.c_double), ("c_vs", C.c_double),
    ("n_samples", C.c_int64), ("n_sweeps_meas", C.c_int64),
    ("n_acc", C.c_int64), ("n_try", C.c_int64),
]


class Walker(C.Structure):
    _fields_ = WALKER_FIELDS


WALKER_DTYPE = np.dtype([(n, np.float64 if t is C.c_double else np.int64) for n, t in WALKER_FIELDS])

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        sp = C.POINTER(System)
        wp = C.POINTER(Walker)
        L.or_box_side.argtypes = [C.c_int32, C.c_double, C.c_int32]
        L.or_box_side.restype = C.c_double
        L.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.or_draw_move.argtypes = [sp, C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(C.c_int32), dp, dp]
        for name in ("or_f", "or_u"):
            getattr(L, name).argtypes = [sp, C.c_double]
            getattr(L, name).restype = C.c_double
        L.or_u_derivs.argtypes = [sp, C.c_double, dp, dp, dp]
        L.or_aziz.argtypes = [C.c_double]
        L.or_aziz.restype = C.c_double
        L.or_aziz_deriv.argtypes = [C.c_double]
        L.or_aziz_deriv.restype = C.c_double
        L.or_min_image.argtypes = [C.c_double, C.c_double]
        L.or_min_image.restype = C.c_double
        L.or_totals.argtypes = [sp, dp, dp, dp]
        L.or_trial_position.argtypes = [sp, dp, C.c_int32, dp, dp]
        L.or_delta.argtypes = [sp, dp, C.c_int32, dp, dp, dp, dp, dp]
        L.or_delta_slopes.argtypes = [sp, dp, C.c_int32, dp, dp, dp]
        L.or_local_energy.argtypes = [sp, dp, dp, dp, dp, dp]
        L.or_fcc_start.argtypes = [sp, C.c_uint32, dp]
        u64p = C.POINTER(C.c_uint64)
        L.or_pair_histogram.argtypes = [sp, dp, C.c_int32, u64p, u64p, C.c_double]
        L.or_walker_init.argtypes = [sp, dp, wp]
        L.or_run_walker.argtypes = [sp, C.c_uint32, dp, wp, C.c_uint32, C.c_int32, C.c_uint32,
                                    C.c_int32, dp, C.POINTER(C.c_int64)]
        L.or_metropolis_accept.argtypes = [C.c_double, C.c_double]
        L.or_metropolis_accept.restype = C.c_int
        L.or_run_walker_log.argtypes = [sp, C.c_uint32, dp, wp, C.c_uint32, C.c_int32, C.c_uint32,
                                        C.c_int32, dp, C.c_int64]
        L.or_run_walkers.argtypes = [sp, C.c_uint32, C.c_int32, dp, wp, C.c_uint32, C.c_int32,
                                     C.c_uint32, C.c_int32, C.c_int32]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def system(n, L, b, hbar2_over_m=12.1194, step_sigma=1.0, seed=1, order=0, fp32_coords=False):
    """fp32_coords: keep every stored position rounded to FP32 (the precision
    form's coordinates; use box_side(..., fp32=True) for L)."""
    return System(int(n), int(order), float(L), float(b), float(hbar2_over_m), float(step_sigma), int(seed),
                  int(bool(fp32_coords)))


def box_side(n, density, fp32=False):
    return lib().or_box_side(int(n), float(density), int(bool(fp32)))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return tuple(int(x) for x in o)


def draw_move(sys_, k, t, w):
    s = C.c_int32()
    xi = C.c_double()
    d = (C.c_double * 3)()
    lib().or_draw_move(C.byref(sys_), k, t, w, C.byref(s), C.byref(xi), d)
    return s.value, xi.value, np.array(d[:])


def f(sys_, r):
    return lib().or_f(C.byref(sys_), float(r))


def u(sys_, r):
    return lib().or_u(C.byref(sys_), float(r))


def u_derivs(sys_, r):
    a, b_, c = C.c_double(), C.c_double(), C.c_double()
    lib().or_u_derivs(C.byref(sys_), float(r), C.byref(a), C.byref(b_), C.byref(c))
    return a.value, b_.value, c.value


def aziz(r):
    return lib().or_aziz(float(r))


def aziz_deriv(r):
    return lib().or_aziz_deriv(float(r))


def min_image(d, L):
    return lib().or_min_image(float(d), float(L))


def totals(sys_, xyz):
    x = _f64(xyz, (3, sys_.n))
    U, V = C.c_double(), C.c_double()
    lib().or_totals(C.byref(sys_), _dp(x), C.byref(U), C.byref(V))
    return U.value, V.value


def trial_position(sys_, xyz, s, delta):
    x = _f64(xyz, (3, sys_.n))
    d = _f64(delta, (3,))
    out = np.zeros(3)
    lib().or_trial_position(C.byref(sys_), _dp(x), int(s), _dp(d), _dp(out))
    return out


def delta(sys_, xyz, s, rnew):
    """Eq. (7) sums for moving atom s to rnew: (dU, dV, scale_u, scale_v)."""
    x = _f64(xyz, (3, sys_.n))
    rn = _f64(rnew, (3,))
    vals = [C.c_double() for _ in range(4)]
    lib().or_delta(C.byref(sys_), _dp(x), int(s), _dp(rn), *[C.byref(v) for v in vals])
    return tuple(v.value for v in vals)


def delta_slopes(sys_, xyz, s, rnew):
    """Tolerance slopes of a move: (sum |u'|, sum |dV/dr|) over the old and
    the trial distances of atom s to every other atom."""
    x = _f64(xyz, (3, sys_.n))
    rn = _f64(rnew, (3,))
    a, b_ = C.c_double(), C.c_double()
    lib().or_delta_slopes(C.byref(sys_), _dp(x), int(s), _dp(rn), C.byref(a), C.byref(b_))
    return a.value, b_.value


def local_energy(sys_, xyz, want_derivs=False):
    """Returns (out, scale[, grad, lap]); out = [E_L, V, T_PB, T_JF, T_F, U]."""
    x = _f64(xyz, (3, sys_.n))
    out = np.zeros(6)
    scale = C.c_double()
    if want_derivs:
        g = np.zeros((3, sys_.n))
        lp = np.zeros(sys_.n)
        lib().or_local_energy(C.byref(sys_), _dp(x), _dp(out), C.byref(scale), _dp(g), _dp(lp))
        return out, scale.value, g, lp
    lib().or_local_energy(C.byref(sys_), _dp(x), _dp(out), C.byref(scale), None, None)
    return out, scale.value


def pair_histogram(sys_, xyz, nb, rel_window=0.0):
    """(counts[nb], edge[nb+1]) of unordered pair distances in nb equal bins
    over [0, L/2]; edge[b] counts pairs within rel_window of bin edge b."""
    x = _f64(xyz, (3, sys_.n))
    counts = np.zeros(nb, dtype=np.uint64)
    edge = np.zeros(nb + 1, dtype=np.uint64)
    u64p = C.POINTER(C.c_uint64)
    lib().or_pair_histogram(C.byref(sys_), _dp(x), int(nb), counts.ctypes.data_as(u64p),
                            edge.ctypes.data_as(u64p), float(rel_window))
    return counts, edge


def fcc_start(sys_, w):
    out = np.zeros((3, sys_.n))
    lib().or_fcc_start(C.byref(sys_), int(w), _dp(out))
    return out


def walker_init(sys_, xyz):
    x = _f64(xyz, (3, sys_.n))
    acc = Walker()
    lib().or_walker_init(C.byref(sys_), _dp(x), C.byref(acc))
    return acc


def walker_to_dict(acc):
    return {name: getattr(acc, name) for name, _ in WALKER_FIELDS}


def run_walker(sys_, w, xyz, acc, t0, n_sweeps, measure_start, m, record_el=False):
    """Advance one walker in place (xyz is modified).  Returns the E_L samples
    if record_el, else None."""
    if xyz.dtype != np.float64 or not xyz.flags.c_contiguous or xyz.shape != (3, sys_.n):
        raise ValueError("xyz must be a C-contiguous float64 (3, N) array")
    el = None
    n_el = C.c_int64(0)
    if record_el:
        cap = n_sweeps // m + 1 if m > 0 else 1
        el = np.zeros(cap)
    lib().or_run_walker(C.byref(sys_), int(w), _dp(xyz), C.byref(acc), int(t0), int(n_sweeps),
                        int(measure_start), int(m), _dp(el) if record_el else None, C.byref(n_el))
    return el[: n_el.value] if record_el else None


def metropolis_accept(du, xi):
    """Eq. (5) decision for a move with Eq. (7) sum du and uniform xi."""
    return bool(lib().or_metropolis_accept(float(du), float(xi)))


MOVE_LOG_FIELDS = ("s", "accepted", "du", "dv", "scale_u", "scale_v", "slope_u", "slope_v")


def run_walker_log(sys_, w, xyz, acc, t0, n_sweeps, measure_start, m, cap=None):
    """run_walker that returns the record of every micro-update, an array of
    shape (moves, 8): (s, accepted, dU, dV, scale_u, scale_v, slope_u,
    slope_v), dU and dV the Eq. (7) sums at the configuration each move was
    proposed in, the slopes those of delta_slopes there."""
    if xyz.dtype != np.float64 or not xyz.flags.c_contiguous or xyz.shape != (3, sys_.n):
        raise ValueError("xyz must be a C-contiguous float64 (3, N) array")
    cap = n_sweeps * sys_.n if cap is None else cap
    log = np.zeros((cap, len(MOVE_LOG_FIELDS)))
    lib().or_run_walker_log(C.byref(sys_), int(w), _dp(xyz), C.byref(acc), int(t0), int(n_sweeps),
                            int(measure_start), int(m), _dp(log), int(cap))
    return log


def run_walkers(sys_, w0, xyz, accs, t0, n_sweeps, measure_start, m, n_threads):
    """Advance walkers w0.. in place; xyz (W, 3, N) float64, accs a ctypes
    array of Walker of length W."""
    W = xyz.shape[0]
    if xyz.dtype != np.float64 or not xyz.flags.c_contiguous or xyz.shape[1:] != (3, sys_.n):
        raise ValueError("xyz must be a C-contiguous float64 (W, 3, N) array")
    lib().or_run_walkers(C.byref(sys_), int(w0), int(W), _dp(xyz), accs, int(t0), int(n_sweeps),
                         int(measure_start), int(m), int(n_threads))
