"""ctypes binding of libhevmc (include/hevmc.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts torch
tensors to device pointers and streams and turns error codes into exceptions.
There is no fallback: if libhevmc.so is missing or the call fails, it raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhevmc.so")

FP64 = 0
FP32 = 1
SELECT_RANDOM = 0
SELECT_SEQUENTIAL = 1
VARIANT_AUTO = 0
VARIANT_PLAIN = 1
VARIANT_ROWS = 2
NO_MEASURE = 0xFFFFFFFF

STATUS = {0: "HEVMC_OK", -1: "HEVMC_EINVAL", -2: "HEVMC_ENOMEM", -3: "HEVMC_ENOFIT",
          -4: "HEVMC_EDEVICE", -5: "HEVMC_ESTATE", -6: "HEVMC_EBUSY"}


class HevmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("n_walkers", C.c_int32),
        ("precision", C.c_int32),
        ("order", C.c_int32),
        ("density", C.c_double),
        ("b", C.c_double),
        ("hbar2_over_m", C.c_double),
        ("step_sigma", C.c_double),
        ("seed", C.c_uint64),
        ("walker_id_base", C.c_uint32),
        ("threads", C.c_int32),
        ("variant", C.c_int32),
    ]


MAX_BATCH = 16


class Request(C.Structure):
    _fields_ = [
        ("params", Params),
        ("sweep0", C.c_uint32),
        ("measure_start", C.c_uint32),
        ("energy_every", C.c_int32),
        ("reserved", C.c_int32),
    ]


ACC_FIELDS = [
    "u_run", "v_run", "sum_e", "c_e", "sum_e2", "c_e2", "sum_v", "c_v", "sum_tpb", "c_tpb",
    "sum_tjf", "c_tjf", "sum_tf", "c_tf", "sum_vs", "c_vs",
]
ACC_INT_FIELDS = ["n_samples", "n_sweeps_meas", "n_acc", "n_try"]
ACC_DTYPE = np.dtype([(f, np.float64) for f in ACC_FIELDS] + [(f, np.int64) for f in ACC_INT_FIELDS])
ACC_BYTES = ACC_DTYPE.itemsize   # 160


class WalkerAcc(C.Structure):
    _fields_ = [(f, C.c_double) for f in ACC_FIELDS] + [(f, C.c_int64) for f in ACC_INT_FIELDS]


assert C.sizeof(WalkerAcc) == ACC_BYTES

class Plan(C.Structure):
    _fields_ = [
        ("threads", C.c_int32),
        ("variant", C.c_int32),
        ("spatial_order", C.c_int32),
        ("walkers_per_cu", C.c_int32),
        ("lds_per_walker", C.c_uint64),
        ("lds_per_group", C.c_uint64),
        ("slices", C.c_int32),
        ("reserved", C.c_int32),
    ]


EXPORTS = [
    "hevmc_plan_launch", "hevmc_box", "hevmc_footprint", "hevmc_init_walkers", "hevmc_sweep", "hevmc_sweep_gr",
    "hevmc_pair_histogram", "hevmc_sweep_trace", "hevmc_sweep_log", "hevmc_local_energy",
    "hevmc_move_delta", "hevmc_draw_moves", "hevmc_sweep_batch", "hevmc_create", "hevmc_create_on", "hevmc_run",
    "hevmc_sync", "hevmc_get_acc", "hevmc_get_coords", "hevmc_get_sweep", "hevmc_destroy",
    "hevmc_eval_config", "hevmc_eval_config_noalloc", "hevmc_last_error",
]

NOALLOC_MAX_N = 8192   # HEVMC_NOALLOC_MAX_N

_lib = None


def lib():
    """Load libhevmc.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(Params)
        vp = C.c_void_p
        st = C.c_int
        sig = {
            "hevmc_plan_launch": [P, C.POINTER(Plan)],
            "hevmc_box": [P, C.POINTER(C.c_double)],
            "hevmc_footprint": [P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)],
            "hevmc_init_walkers": [P, vp, vp, vp, C.c_int32, vp],
            "hevmc_sweep": [P, vp, vp, vp, C.c_uint32, C.c_int32, C.c_uint32, C.c_int32, vp],
            "hevmc_sweep_gr": [P, vp, vp, vp, vp, C.c_int32, C.c_uint32, C.c_int32, C.c_uint32, C.c_int32, vp],
            "hevmc_pair_histogram": [P, vp, C.c_int32, vp, vp],
            "hevmc_sweep_trace": [P, vp, vp, vp, vp, C.c_int32, C.c_uint32, C.c_int32, C.c_uint32, C.c_int32, vp],
            "hevmc_sweep_log": [P, vp, vp, vp, vp, C.c_int32, C.c_int64, C.c_uint32, C.c_int32, C.c_uint32,
                                C.c_int32, vp],
            "hevmc_local_energy": [P, vp, vp, vp],
            "hevmc_move_delta": [P, vp, vp, vp, vp, vp],
            "hevmc_draw_moves": [P, C.c_uint32, vp, vp, vp, vp],
            "hevmc_sweep_batch": [C.c_int32, C.POINTER(Request), vp, C.c_int32, vp, vp, vp, C.c_int32, vp],
            "hevmc_create": [P, vp, vp, C.POINTER(vp)],
            "hevmc_create_on": [P, vp, vp, vp, C.POINTER(vp)],
            "hevmc_run": [vp, C.c_int32, C.c_int32, C.c_int32],
            "hevmc_sync": [vp],
            "hevmc_get_acc": [vp, vp],
            "hevmc_get_coords": [vp, vp],
            "hevmc_get_sweep": [vp, C.POINTER(C.c_uint32)],
            "hevmc_destroy": [vp],
            "hevmc_eval_config": [P, vp, C.c_int32, vp, C.POINTER(C.c_double), C.POINTER(C.c_double), vp],
            "hevmc_eval_config_noalloc": [P, vp, C.c_int32, vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = st
        L.hevmc_last_error.argtypes = []
        L.hevmc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise HevmcError(code, lib().hevmc_last_error().decode())


def make_params(n, n_walkers, precision=FP64, density=0.02186, b=1.15 * 2.556, hbar2_over_m=12.1194,
                step_sigma=0.63, seed=1, walker_id_base=0, threads=0, order=SELECT_RANDOM, variant=VARIANT_AUTO):
    return Params(int(n), int(n_walkers), int(precision), int(order), float(density), float(b),
                  float(hbar2_over_m), float(step_sigma), int(seed), int(walker_id_base), int(threads),
                  int(variant))


def params_for(workload, **over):
    """Params of a configs.Workload (keyword overrides allowed)."""
    kw = dict(n=workload.n, n_walkers=workload.walkers, precision=workload.precision,
              density=workload.density, b=workload.b, step_sigma=workload.step_sigma, seed=workload.seed)
    kw.update(over)
    return make_params(**kw)


def box(p):
    L = C.c_double()
    _check(lib().hevmc_box(C.byref(p), C.byref(L)))
    return L.value


def footprint(p):
    lds, hbm = C.c_size_t(), C.c_size_t()
    _check(lib().hevmc_footprint(C.byref(p), C.byref(lds), C.byref(hbm)))
    return lds.value, hbm.value


def plan_launch(p):
    """The library's launch plan for a sweep of p, as a dict."""
    out = Plan()
    _check(lib().hevmc_plan_launch(C.byref(p), C.byref(out)))
    return {f: getattr(out, f) for f, _ in Plan._fields_}


def plan_uses_rows(p):
    """True if the library runs the row-sum variant of the sweep for p."""
    return plan_launch(p)["variant"] == VARIANT_ROWS


# ---- torch-facing helpers -------------------------------------------------

def _torch():
    import torch
    return torch


def _ptr(t, dtype=None, shape=None, what="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def coord_dtype(p):
    torch = _torch()
    return torch.float32 if p.precision == FP32 else torch.float64


def alloc_state(p, device="cuda"):
    """Device buffers for an ensemble: coords [W,3,N] and acc [W,160 bytes]."""
    torch = _torch()
    coords = torch.zeros((p.n_walkers, 3, p.n), dtype=coord_dtype(p), device=device)
    acc = torch.zeros((p.n_walkers, ACC_BYTES), dtype=torch.uint8, device=device)
    return coords, acc


def alloc_rows(p, device="cuda"):
    """Device buffer [W,N] float64 for the per-atom row sums kept between sweeps."""
    torch = _torch()
    return torch.zeros((p.n_walkers, p.n), dtype=torch.float64, device=device)


def _rows_ptr(p, rows):
    if rows is None:
        return None
    return _ptr(rows, _torch().float64, (p.n_walkers, p.n), "rows")


def init_walkers(p, coords, acc, fcc_start=True, stream=None, rows=None):
    _check(lib().hevmc_init_walkers(C.byref(p), _ptr(coords, coord_dtype(p), (p.n_walkers, 3, p.n), "coords"),
                                    _ptr(acc, None, (p.n_walkers, ACC_BYTES), "acc"), _rows_ptr(p, rows),
                                    int(bool(fcc_start)), _stream(stream)))


def sweep(p, coords, acc, sweep0, n_sweeps, measure_start=NO_MEASURE, energy_every=0, stream=None, rows=None,
          gr=None, trace=None, movelog=None):
    """hevmc_sweep; hevmc_sweep_gr when gr (int64 [W][bins], device) is given;
    hevmc_sweep_trace when trace (float64 [W][cap][6], device) is given;
    hevmc_sweep_log when movelog (float64 [log_walkers][cap][4], device) is
    given (records (s, accepted, dU, dV) of every micro-update of the first
    log_walkers walkers)."""
    cp = _ptr(coords, coord_dtype(p), (p.n_walkers, 3, p.n), "coords")
    ap = _ptr(acc, None, (p.n_walkers, ACC_BYTES), "acc")
    if sum(x is not None for x in (gr, trace, movelog)) > 1:
        raise ValueError("one of gr, trace and movelog per call")
    if movelog is not None:
        lw, cap = int(movelog.shape[0]), int(movelog.shape[1])
        lp = _ptr(movelog, _torch().float64, (lw, cap, 4), "movelog")
        _check(lib().hevmc_sweep_log(C.byref(p), cp, ap, _rows_ptr(p, rows), lp, lw, cap, int(sweep0),
                                     int(n_sweeps), int(measure_start), int(energy_every), _stream(stream)))
    elif trace is not None:
        cap = int(trace.shape[1])
        tp = _ptr(trace, _torch().float64, (p.n_walkers, cap, 6), "trace")
        _check(lib().hevmc_sweep_trace(C.byref(p), cp, ap, _rows_ptr(p, rows), tp, cap, int(sweep0),
                                       int(n_sweeps), int(measure_start), int(energy_every), _stream(stream)))
    elif gr is None:
        _check(lib().hevmc_sweep(C.byref(p), cp, ap, _rows_ptr(p, rows), int(sweep0), int(n_sweeps),
                                 int(measure_start), int(energy_every), _stream(stream)))
    else:
        bins = int(gr.shape[-1])
        gp = _ptr(gr, _torch().int64, (p.n_walkers, bins), "gr")
        _check(lib().hevmc_sweep_gr(C.byref(p), cp, ap, _rows_ptr(p, rows), gp, bins, int(sweep0), int(n_sweeps),
                                    int(measure_start), int(energy_every), _stream(stream)))


def pair_histogram(p, coords, counts, stream=None):
    """hevmc_pair_histogram: counts (int64 [W][bins], device) is overwritten."""
    bins = int(counts.shape[-1])
    _check(lib().hevmc_pair_histogram(C.byref(p), _ptr(coords, coord_dtype(p), (p.n_walkers, 3, p.n), "coords"),
                                      bins, _ptr(counts, _torch().int64, (p.n_walkers, bins), "counts"),
                                      _stream(stream)))


def local_energy(p, coords, out, stream=None):
    torch = _torch()
    _check(lib().hevmc_local_energy(C.byref(p), _ptr(coords, coord_dtype(p), (p.n_walkers, 3, p.n), "coords"),
                                    _ptr(out, torch.float64, (p.n_walkers, 6), "out"), _stream(stream)))


def move_delta(p, coords, s, delta, out, stream=None):
    torch = _torch()
    W = p.n_walkers
    _check(lib().hevmc_move_delta(C.byref(p), _ptr(coords, coord_dtype(p), (W, 3, p.n), "coords"),
                                  _ptr(s, torch.int32, (W,), "s"), _ptr(delta, torch.float64, (W, 3), "delta"),
                                  _ptr(out, torch.float64, (W, 2), "out"), _stream(stream)))


def draw_moves(p, t, s_out, xi_out, delta_out, stream=None):
    torch = _torch()
    W, n = p.n_walkers, p.n
    _check(lib().hevmc_draw_moves(C.byref(p), int(t), _ptr(s_out, torch.int32, (W, n), "s_out"),
                                  _ptr(xi_out, torch.float64, (W, n), "xi_out"),
                                  _ptr(delta_out, torch.float64, (W, n, 3), "delta_out"), _stream(stream)))


def sweep_batch(requests, walker_map, coords, acc, rows, n_sweeps, stream=None):
    """hevmc_sweep_batch: requests is a ctypes array of Request sharing N and
    precision; walker_map a [slots, 2] int32 device tensor (request index or
    -1, Philox walker id); coords/acc/rows the class's slot buffers."""
    torch = _torch()
    p0 = requests[0].params
    slots = walker_map.shape[0]
    _check(lib().hevmc_sweep_batch(len(requests), requests, _ptr(walker_map, torch.int32, (slots, 2), "map"), slots,
                                   _ptr(coords, coord_dtype(p0), (slots, 3, p0.n), "coords"),
                                   _ptr(acc, None, (slots, ACC_BYTES), "acc"),
                                   _ptr(rows, torch.float64, (slots, p0.n), "rows") if rows is not None else None,
                                   int(n_sweeps), _stream(stream)))


def acc_to_numpy(acc):
    """[W,160] uint8 device or host tensor -> numpy structured array (ACC_DTYPE)."""
    a = acc.detach().cpu().numpy()
    return np.ascontiguousarray(a).view(ACC_DTYPE).reshape(a.shape[0])


def eval_config(p, xyz, s, delta, noalloc=False):
    """Host-buffer parity entry: returns (dU, dV, [E_L, V, T_PB, T_JF, T_F, U]).
    noalloc: through hevmc_eval_config_noalloc (no device allocation)."""
    x = np.ascontiguousarray(xyz, dtype=np.float64)
    if x.shape != (3, p.n):
        raise ValueError(f"xyz must have shape (3, {p.n})")
    d = np.ascontiguousarray(delta, dtype=np.float64)
    du, dv = C.c_double(), C.c_double()
    out = np.zeros(6)
    fn = lib().hevmc_eval_config_noalloc if noalloc else lib().hevmc_eval_config
    _check(fn(C.byref(p), x.ctypes.data_as(C.c_void_p), int(s), d.ctypes.data_as(C.c_void_p),
              C.byref(du), C.byref(dv), out.ctypes.data_as(C.c_void_p)))
    return du.value, dv.value, out


class Ensemble:
    """Owning ensemble (hevmc_create): device state kept between calls."""

    def __init__(self, p, init_xyz=None, stream=None):
        self.p = p
        self._h = C.c_void_p()
        self._stream = _stream(stream)
        buf = None
        if init_xyz is not None:
            buf = np.ascontiguousarray(init_xyz, dtype=np.float64)
            if buf.shape != (p.n_walkers, 3, p.n):
                raise ValueError("init_xyz must have shape (W, 3, N)")
        _check(lib().hevmc_create(C.byref(p), buf.ctypes.data_as(C.c_void_p) if buf is not None else None,
                                  self._stream, C.byref(self._h)))

    def run(self, n_sweeps, energy_every=0, measure=False):
        _check(lib().hevmc_run(self._h, int(n_sweeps), int(energy_every), int(bool(measure))))

    def sync(self):
        _check(lib().hevmc_sync(self._h))

    def acc(self):
        out = np.zeros(self.p.n_walkers, dtype=ACC_DTYPE)
        _check(lib().hevmc_get_acc(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def coords(self):
        out = np.zeros((self.p.n_walkers, 3, self.p.n))
        _check(lib().hevmc_get_coords(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def sweep_index(self):
        s = C.c_uint32()
        _check(lib().hevmc_get_sweep(self._h, C.byref(s)))
        return s.value

    def close(self):
        if self._h:
            _check(lib().hevmc_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
