"""Python binding of libpphd (include/pphd.h, include/pphd_mlp.h): argument
marshalling only.

Every function here has the name of the C entry point it calls and does no
computation of its own; each stage of the filter runs in the library's HIP
kernels.  PyTorch is used for device memory (the workspace) and for the
stream handle.  If the built library is missing this module raises on first
use -- there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpphd.so")
_LIB = None

PPHD_OK, PPHD_EINVAL, PPHD_ENOMEM, PPHD_ECAPACITY, PPHD_EDEVICE, PPHD_ESTATE = 0, -1, -2, -3, -4, -5
PPHD_FP64, PPHD_FP32 = 0, 1
PHASE_READY, PHASE_PREDICTED, PHASE_UPDATED, PHASE_RESAMPLED = 1, 2, 3, 4
KERNEL_CLASSES = ["predict", "cz", "cz_combine", "weight", "finalize", "fuse", "rs_tiles", "rs_expand",
                  "xchg_gather", "xchg_scatter", "init", "wmax", "geom", "wfinal", "birth_meas",
                  "mlp_infer", "birth_mix", "zprep", "rs_order", "birth_order"]
MLP_HIDDEN, MLP_OUTPUTS, MLP_PARAMS = 128, 36, 38052
K_COUNT = len(KERNEL_CLASSES)


class PphdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pphd error {code}: {msg}")
        self.code = code


class pphd_model(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("partitions", ctypes.c_int32),
        ("births_per_step", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("T", ctypes.c_double), ("sigma_a", ctypes.c_double),
        ("sensor_x", ctypes.c_double), ("sensor_y", ctypes.c_double),
        ("sigma_r", ctypes.c_double), ("sigma_theta", ctypes.c_double),
        ("p_S", ctypes.c_double), ("p_D", ctypes.c_double),
        ("clutter_rate", ctypes.c_double),
        ("r_min", ctypes.c_double), ("r_max", ctypes.c_double),
        ("th_min", ctypes.c_double), ("th_max", ctypes.c_double),
        ("birth_mass", ctypes.c_double), ("region", ctypes.c_double * 4),
        ("birth_sigma_v", ctypes.c_double), ("init_mass", ctypes.c_double),
        ("particles_per_target", ctypes.c_double), ("exchange_fraction", ctypes.c_double),
        ("birth_proposal", ctypes.c_int32), ("global_cz", ctypes.c_int32), ("birth_alpha", ctypes.c_double),
        ("birth_density", ctypes.c_int32), ("reserved2", ctypes.c_int32),
        ("birth_mean", ctypes.c_double * 4), ("birth_std", ctypes.c_double * 4),
        ("sigma_w", ctypes.c_double), ("birth_sigma_w", ctypes.c_double),
    ]


class pphd_run_desc(ctypes.Structure):
    _fields_ = [("partitions", ctypes.c_int32), ("births_per_step", ctypes.c_int32),
                ("clutter_rate", ctypes.c_double), ("particles_per_target", ctypes.c_double),
                ("run_id", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class pphd_mlp_config(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("dataset", ctypes.c_int32), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double)]


class pphd_estimate(ctypes.Structure):
    _fields_ = [("state", ctypes.c_double * 4), ("label", ctypes.c_int32), ("votes", ctypes.c_int32)]


ESTIMATE_DTYPE = np.dtype([("state", np.float64, (4,)), ("label", np.int32), ("votes", np.int32)])

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_I32, _I64, _U32, _U64, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
_MP = ctypes.POINTER(pphd_model)
SIGNATURES = {
    "pphd_workspace_size": (_I32, [_MP, _I64, _I32, ctypes.POINTER(_SZ)]),
    "pphd_create": (_I32, [_MP, _I64, _I32, _P, _SZ, _U64, _U32, _P, ctypes.POINTER(_P)]),
    "pphd_init": (_I32, [_P]),
    "pphd_predict": (_I32, [_P, _U32]),
    "pphd_update": (_I32, [_P, _P, _I32, _I32]),
    "pphd_update_noalloc": (_I32, [_P, _P, _I32, _I32]),
    "pphd_extract": (_I32, [_P, _P, _I32, ctypes.POINTER(_I32), _P]),
    "pphd_extract_device": (_I32, [_P, _P, _I32, _P]),
    "pphd_resample": (_I32, [_P, _U32]),
    "pphd_exchange": (_I32, [_P, _U32]),
    "pphd_destroy": (_I32, [_P]),
    "pphd_last_error": (ctypes.c_char_p, []),
    "pphd_read_state": (_I32, [_P, _P, _P, _P]),
    "pphd_write_state": (_I32, [_P, _P, _P, _P, _I32]),
    "pphd_read_update": (_I32, [_P, _P, _P, _P, _P]),
    "pphd_read_local": (_I32, [_P, _P, _P]),
    "pphd_set_record_counts": (_I32, [_P, _I32]),
    "pphd_set_tuning": (_I32, [_P, _I32, _I32, _I32]),
    "pphd_set_launch_shape": (_I32, [_P, _I32, _I32]),
    "pphd_read_resample": (_I32, [_P, _P, _P, ctypes.POINTER(_I64)]),
    "pphd_set_timing": (_I32, [_P, _I32]),
    "pphd_read_timing": (_I32, [_P, _P, _P]),
    "pphd_kernel_name": (ctypes.c_char_p, [_I32]),
    "pphd_mlp_workspace_size": (_I32, [ctypes.POINTER(pphd_mlp_config), ctypes.POINTER(_SZ)]),
    "pphd_mlp_create": (_I32, [_MP, ctypes.POINTER(pphd_mlp_config), _P, _SZ, _U64, _P, ctypes.POINTER(_P)]),
    "pphd_mlp_init_params": (_I32, [_P, _U32]),
    "pphd_mlp_set_params": (_I32, [_P, _P, _I32]),
    "pphd_mlp_get_params": (_I32, [_P, _P, _I32]),
    "pphd_mlp_simulate": (_I32, [_P, _U32]),
    "pphd_mlp_read_dataset": (_I32, [_P, _I32, _I32, _P, _P]),
    "pphd_mlp_loss_grad": (_I32, [_P, _P, _P, _I32, _I32, _P, ctypes.POINTER(ctypes.c_double)]),
    "pphd_mlp_train": (_I32, [_P, _I32, ctypes.c_double, _P]),
    "pphd_mlp_forward": (_I32, [_P, _P, _I32, _I32, _P]),
    "pphd_mlp_steps": (_I32, [_P, ctypes.POINTER(_I64)]),
    "pphd_mlp_destroy": (_I32, [_P]),
    "pphd_attach_mlp": (_I32, [_P, _P]),
    "pphd_batch_workspace_size": (_I32, [_MP, _P, _I32, _I64, _I32, ctypes.POINTER(_SZ)]),
    "pphd_batch_create": (_I32, [_MP, _P, _I32, _I64, _I32, _P, _SZ, _U64, _P, ctypes.POINTER(_P)]),
    "pphd_batch_update": (_I32, [_P, _P, _I32, _P, _I32]),
    "pphd_batch_extract": (_I32, [_P, _P, _I32, _P, _P]),
    "pphd_batch_extract_device": (_I32, [_P, _P, _I32, _P]),
    "pphd_batch_capture": (_I32, [_P, _P, _I32, _P, _P, _I32, _P, _U32]),
    "pphd_batch_launch": (_I32, [_P]),
    "pphd_set_birth_mixture": (_I32, [_P, _P, _I32, _I32]),
}


def lib():
    """Loads libpphd.so (raises if it was not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _chk(rc):
    if rc != PPHD_OK:
        raise PphdError(rc, lib().pphd_last_error().decode())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


def model_struct(p: dict, precision: int) -> pphd_model:
    m = pphd_model()
    m.dim = int(p.get("dim", 4))
    m.partitions = int(p["partitions"])
    m.births_per_step = int(p["births_per_step"])
    m.precision = int(precision)
    for k in ("T", "sigma_a", "sensor_x", "sensor_y", "sigma_r", "sigma_theta", "p_S", "p_D",
              "clutter_rate", "r_min", "r_max", "th_min", "th_max", "birth_mass",
              "birth_sigma_v", "init_mass", "particles_per_target", "exchange_fraction"):
        setattr(m, k, float(p[k]))
    for i in range(4):
        m.region[i] = float(p["region"][i])
    m.birth_proposal = int(p.get("birth_proposal", 0))
    m.global_cz = int(p.get("global_cz", 0))
    m.birth_alpha = float(p.get("birth_alpha", 1.0))
    m.birth_density = int(p.get("birth_density", 0))
    for i in range(4):
        m.birth_mean[i] = float(p.get("birth_mean", (0.0,) * 4)[i])
        m.birth_std[i] = float(p.get("birth_std", (1.0,) * 4)[i])
    m.sigma_w = float(p.get("sigma_w", 0.0))
    m.birth_sigma_w = float(p.get("birth_sigma_w", 0.0))
    return m


# ---- one wrapper per entry point -------------------------------------------

def pphd_workspace_size(model: pphd_model, cap: int, max_meas: int) -> int:
    n = _SZ(0)
    _chk(lib().pphd_workspace_size(ctypes.byref(model), cap, max_meas, ctypes.byref(n)))
    return int(n.value)


def pphd_create(model, cap, max_meas, workspace_ptr, workspace_bytes, seed, run_id, stream_ptr):
    h = _P()
    _chk(lib().pphd_create(ctypes.byref(model), cap, max_meas, workspace_ptr, workspace_bytes,
                           seed, run_id, stream_ptr, ctypes.byref(h)))
    return h


def pphd_init(h):
    _chk(lib().pphd_init(h))


def pphd_predict(h, step):
    _chk(lib().pphd_predict(h, step))


def pphd_update(h, z, m, z_on_device):
    _chk(lib().pphd_update(h, z, m, z_on_device))


def pphd_update_noalloc(h, z, m, z_on_device):
    _chk(lib().pphd_update_noalloc(h, z, m, z_on_device))


def pphd_extract(h, out_ptr, cap, mass_ptr=None):
    n = _I32(0)
    _chk(lib().pphd_extract(h, out_ptr, cap, ctypes.byref(n), mass_ptr))
    return int(n.value)


def pphd_extract_device(h, d_out_ptr, cap, d_n_ptr):
    _chk(lib().pphd_extract_device(h, d_out_ptr, cap, d_n_ptr))


def pphd_resample(h, step):
    _chk(lib().pphd_resample(h, step))


def pphd_exchange(h, step):
    _chk(lib().pphd_exchange(h, step))


def pphd_destroy(h):
    _chk(lib().pphd_destroy(h))


def pphd_read_state(h, x_ptr, w_ptr, count_ptr):
    _chk(lib().pphd_read_state(h, x_ptr, w_ptr, count_ptr))


def pphd_write_state(h, x_ptr, w_ptr, count_ptr, phase):
    _chk(lib().pphd_write_state(h, x_ptr, w_ptr, count_ptr, phase))


def pphd_read_update(h, C_ptr, dW_ptr, mass_ptr, LT_ptr):
    _chk(lib().pphd_read_update(h, C_ptr, dW_ptr, mass_ptr, LT_ptr))


def pphd_read_local(h, sel_ptr, zeta_ptr):
    _chk(lib().pphd_read_local(h, sel_ptr, zeta_ptr))


def pphd_set_launch_shape(h, pass_workgroups, rs_tiles):
    _chk(lib().pphd_set_launch_shape(h, pass_workgroups, rs_tiles))


def pphd_set_tuning(h, pt_cz, pt_weight, meas_per_wave):
    _chk(lib().pphd_set_tuning(h, int(pt_cz), int(pt_weight), int(meas_per_wave)))


def pphd_set_record_counts(h, enable):
    _chk(lib().pphd_set_record_counts(h, int(enable)))


def pphd_read_resample(h, counts_ptr, massq_ptr):
    c = _I64(0)
    _chk(lib().pphd_read_resample(h, counts_ptr, massq_ptr, ctypes.byref(c)))
    return int(c.value)


def pphd_set_timing(h, enable):
    _chk(lib().pphd_set_timing(h, int(enable)))


def pphd_read_timing(h, ms_ptr, launches_ptr):
    _chk(lib().pphd_read_timing(h, ms_ptr, launches_ptr))


def pphd_mlp_workspace_size(cfg):
    n = _SZ(0)
    _chk(lib().pphd_mlp_workspace_size(ctypes.byref(cfg), ctypes.byref(n)))
    return int(n.value)


def pphd_mlp_create(model, cfg, workspace_ptr, workspace_bytes, seed, stream_ptr):
    h = _P()
    _chk(lib().pphd_mlp_create(ctypes.byref(model), ctypes.byref(cfg), workspace_ptr, workspace_bytes, seed,
                               stream_ptr, ctypes.byref(h)))
    return h


def pphd_mlp_init_params(h, init_id):
    _chk(lib().pphd_mlp_init_params(h, int(init_id)))


def pphd_mlp_set_params(h, params_ptr, on_device):
    _chk(lib().pphd_mlp_set_params(h, params_ptr, int(on_device)))


def pphd_mlp_get_params(h, params_ptr, on_device):
    _chk(lib().pphd_mlp_get_params(h, params_ptr, int(on_device)))


def pphd_mlp_simulate(h, run):
    _chk(lib().pphd_mlp_simulate(h, int(run)))


def pphd_mlp_read_dataset(h, first, n, z_ptr, x_ptr):
    _chk(lib().pphd_mlp_read_dataset(h, int(first), int(n), z_ptr, x_ptr))


def pphd_mlp_loss_grad(h, z_ptr, x_ptr, n, on_device, grad_ptr):
    loss = ctypes.c_double(0.0)
    _chk(lib().pphd_mlp_loss_grad(h, z_ptr, x_ptr, int(n), int(on_device), grad_ptr, ctypes.byref(loss)))
    return float(loss.value)


def pphd_mlp_train(h, steps, lr, loss_ptr):
    _chk(lib().pphd_mlp_train(h, int(steps), float(lr), loss_ptr))


def pphd_mlp_forward(h, z_ptr, n, on_device, out_ptr):
    _chk(lib().pphd_mlp_forward(h, z_ptr, int(n), int(on_device), out_ptr))


def pphd_mlp_steps(h):
    n = _I64(0)
    _chk(lib().pphd_mlp_steps(h, ctypes.byref(n)))
    return int(n.value)


def pphd_mlp_destroy(h):
    _chk(lib().pphd_mlp_destroy(h))


def pphd_attach_mlp(f, h):
    _chk(lib().pphd_attach_mlp(f, h))


def pphd_set_birth_mixture(f, raw_ptr, m, on_device):
    _chk(lib().pphd_set_birth_mixture(f, raw_ptr, int(m), int(on_device)))


def pphd_batch_workspace_size(model, runs_ptr, nruns, cap, max_meas):
    n = _SZ(0)
    _chk(lib().pphd_batch_workspace_size(ctypes.byref(model), runs_ptr, int(nruns), int(cap), int(max_meas),
                                         ctypes.byref(n)))
    return int(n.value)


def pphd_batch_create(model, runs_ptr, nruns, cap, max_meas, workspace_ptr, workspace_bytes, seed, stream_ptr):
    h = _P()
    _chk(lib().pphd_batch_create(ctypes.byref(model), runs_ptr, int(nruns), int(cap), int(max_meas), workspace_ptr,
                                 workspace_bytes, seed, stream_ptr, ctypes.byref(h)))
    return h


def pphd_batch_update(h, z_ptr, z_count, windows_ptr, on_device):
    _chk(lib().pphd_batch_update(h, z_ptr, int(z_count), windows_ptr, int(on_device)))


def pphd_batch_extract(h, out_ptr, cap, n_ptr, mass_ptr=None):
    _chk(lib().pphd_batch_extract(h, out_ptr, int(cap), n_ptr, mass_ptr))


def pphd_batch_extract_device(h, d_out_ptr, cap, d_n_ptr):
    _chk(lib().pphd_batch_extract_device(h, d_out_ptr, int(cap), d_n_ptr))


def pphd_batch_capture(h, d_z_ptr, z_count, d_windows_ptr, d_out_ptr, cap, d_n_ptr, first_step):
    _chk(lib().pphd_batch_capture(h, d_z_ptr, int(z_count), d_windows_ptr, d_out_ptr, int(cap), d_n_ptr,
                                  int(first_step)))


def pphd_batch_launch(h):
    _chk(lib().pphd_batch_launch(h))


def pphd_last_error():
    return lib().pphd_last_error().decode()


def pphd_kernel_name(c):
    r = lib().pphd_kernel_name(c)
    return r.decode() if r else None


TUNING_PATH = os.path.join(_HERE, "tuning.json")


def load_tuning():
    """The autotuner's table (autotune.py): launch shapes keyed by bucket."""
    import json
    if os.path.exists(TUNING_PATH):
        with open(TUNING_PATH) as fh:
            return json.load(fh)
    return {}


def tuning_bucket(precision: int, batch: bool, groups: int, cap: int, measurements: float) -> str:
    """Key of the autotuner's table: storage precision, single filter or batch,
    and the rounded base-2 logarithms of the groups over all runs, of the
    slots per group (the capacity, which sizes every grid) and of the expected
    measurements per run (clutter rate plus ten)."""
    import math

    def lg(v):
        return int(round(math.log2(max(v, 1))))
    kind = ("fp64" if precision == PPHD_FP64 else "fp32") + ("_batch" if batch else "")
    return f"{kind}/g{lg(groups)}/cap{lg(cap)}/m{lg(measurements)}"


def lookup_tuning(precision: int, batch: bool, groups: int, cap: int, measurements: float):
    """The tuned shape of this bucket, else of the nearest bucket of the same
    kind (precision, single or batch), else None (the library's defaults)."""
    import re
    table = load_tuning()
    key = tuning_bucket(precision, batch, groups, cap, measurements)
    if key in table:
        return table[key]
    kind = key.split("/")[0]
    want = [int(v) for v in re.findall(r"-?\d+", key.split("/", 1)[1])]
    best, dist = None, None
    for k, v in table.items():
        parts = k.split("/")
        if len(parts) != 4 or parts[0] != kind:
            continue
        have = [int(x) for x in re.findall(r"-?\d+", k.split("/", 1)[1])]
        d = sum(abs(a - b) for a, b in zip(have, want))
        if dist is None or d < dist:
            best, dist = v, d
    return best


def apply_tuning_to(h, t):
    if t:
        pphd_set_tuning(h, t["pt_cz"], t["pt_weight"], t.get("meas_per_wave", 16))
        pphd_set_launch_shape(h, t.get("pass_workgroups", 0), t.get("rs_tiles", 0))


# ---- convenience object (allocation through torch, arrays through numpy) ---

class Filter:
    """One filter run on the current torch device and stream.

    The workspace is a torch uint8 tensor; host-side results come back as
    numpy arrays.  Methods map one-to-one onto the C entry points."""

    def __init__(self, params: dict, precision: int, cap: int, max_meas: int, seed: int, run_id: int = 0,
                 stream=None, apply_tuning: bool = True):
        import torch
        self.torch = torch
        self.params = params
        self.K = int(params["partitions"])
        self.cap = int(cap)
        self.max_meas = int(max_meas)
        self.precision = int(precision)
        self.dim = int(params.get("dim", 4))
        self.model = model_struct(params, precision)
        nbytes = pphd_workspace_size(self.model, self.cap, self.max_meas)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = pphd_create(self.model, self.cap, self.max_meas, aligned, nbytes, int(seed), int(run_id),
                             self.stream.cuda_stream)
        self.last_m = 0
        self.tuning = None
        if apply_tuning:
            self.tuning = lookup_tuning(self.precision, False, self.K, self.cap, float(params["clutter_rate"]) + 10.0)
            apply_tuning_to(self.h, self.tuning)

    def close(self):
        if getattr(self, "h", None) is not None:
            pphd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # stages
    def init(self):
        pphd_init(self.h)

    def predict(self, step):
        pphd_predict(self.h, int(step))

    def update(self, Z):
        """Z: numpy array [m, 2] (host) or a torch CUDA float64 tensor [m, 2]."""
        if isinstance(Z, np.ndarray):
            Z = np.ascontiguousarray(Z, dtype=np.float64).reshape(-1, 2)
            m = Z.shape[0]
            pphd_update(self.h, Z.ctypes.data if m > 0 else None, m, 0)
        else:
            assert Z.is_cuda and Z.dtype == self.torch.float64 and Z.is_contiguous()
            m = Z.shape[0]
            pphd_update(self.h, Z.data_ptr() if m > 0 else None, m, 1)
        self.last_m = m

    def extract(self):
        cap = max(self.max_meas, 1)
        out = np.zeros(cap, dtype=ESTIMATE_DTYPE)
        mass = np.zeros(self.K)
        n = pphd_extract(self.h, out.ctypes.data, cap, mass.ctypes.data)
        return out[:n].copy(), mass

    def extract_device(self, d_out, d_n, cap):
        pphd_extract_device(self.h, d_out.data_ptr(), cap, d_n.data_ptr())

    def resample(self, step):
        pphd_resample(self.h, int(step))

    def exchange(self, step):
        pphd_exchange(self.h, int(step))

    # state access
    def read_state(self):
        KC = self.K * self.cap
        X = np.zeros((self.dim, KC))
        W = np.zeros(KC)
        n = np.zeros(self.K, dtype=np.int32)
        pphd_read_state(self.h, X.ctypes.data, W.ctypes.data, n.ctypes.data)
        return X, W, n

    def read_counts(self):
        n = np.zeros(self.K, dtype=np.int32)
        pphd_read_state(self.h, None, None, n.ctypes.data)
        return n

    def write_state(self, X, W, n, phase):
        X = np.ascontiguousarray(X, dtype=np.float64)
        W = np.ascontiguousarray(W, dtype=np.float64)
        n = np.ascontiguousarray(n, dtype=np.int32)
        assert X.shape == (self.dim, self.K * self.cap) and W.shape == (self.K * self.cap,) and n.shape == (self.K,)
        pphd_write_state(self.h, X.ctypes.data, W.ctypes.data, n.ctypes.data, int(phase))

    def read_update(self):
        M = self.last_m
        C = np.zeros(max(self.K * M, 1))
        dW = np.zeros(max(self.K * M, 1))
        mass = np.zeros(self.K)
        LT = np.zeros(self.K, dtype=np.int32)
        pphd_read_update(self.h, C.ctypes.data, dW.ctypes.data, mass.ctypes.data, LT.ctypes.data)
        return dict(C=C[:self.K * M].reshape(self.K, M), dW=dW[:self.K * M].reshape(self.K, M), mass=mass, LT=LT)

    def read_local(self):
        M = self.last_m
        sel = np.zeros(max(self.K * M, 1), dtype=np.int32)
        zeta = np.zeros(max(self.K * M * 4, 1))
        pphd_read_local(self.h, sel.ctypes.data, zeta.ctypes.data)
        return dict(sel=sel[:self.K * M].reshape(self.K, M), zeta=zeta[:self.K * M * 4].reshape(self.K, M, 4))

    def set_tuning(self, pt_cz, pt_weight, meas_per_wave):
        pphd_set_tuning(self.h, pt_cz, pt_weight, meas_per_wave)

    def set_launch_shape(self, pass_workgroups, rs_tiles):
        pphd_set_launch_shape(self.h, pass_workgroups, rs_tiles)

    def attach_mlp(self, mlp):
        """Network whose mixtures the births of birth_proposal 2 draw from."""
        pphd_attach_mlp(self.h, mlp.h if mlp is not None else None)
        self.mlp = mlp  # keeps the network alive while the filter uses it

    def set_birth_mixture(self, raw):
        """Network outputs float32 [m, 36] (host) for the next update."""
        raw = np.ascontiguousarray(raw, dtype=np.float32).reshape(-1, MLP_OUTPUTS)
        m = raw.shape[0]
        pphd_set_birth_mixture(self.h, raw.ctypes.data if m > 0 else None, m, 0)

    def set_record_counts(self, enable=True):
        pphd_set_record_counts(self.h, enable)

    def read_resample(self):
        counts = np.zeros(self.K * self.cap, dtype=np.int32)
        mq = np.zeros(self.K)
        clamped = pphd_read_resample(self.h, counts.ctypes.data, mq.ctypes.data)
        return counts, mq, clamped

    def set_timing(self, enable=True):
        pphd_set_timing(self.h, enable)

    def read_timing(self):
        ms = np.zeros(K_COUNT)
        n = np.zeros(K_COUNT, dtype=np.int64)
        pphd_read_timing(self.h, ms.ctypes.data, n.ctypes.data)
        return {KERNEL_CLASSES[i]: (float(ms[i]), int(n[i])) for i in range(K_COUNT)}


def run_table(runs):
    """ctypes array of pphd_run_desc from dicts (partitions, births_per_step,
    clutter_rate, particles_per_target, run_id)."""
    arr = (pphd_run_desc * len(runs))()
    for i, r in enumerate(runs):
        arr[i].partitions = int(r["partitions"])
        arr[i].births_per_step = int(r["births_per_step"])
        arr[i].clutter_rate = float(r["clutter_rate"])
        arr[i].particles_per_target = float(r["particles_per_target"])
        arr[i].run_id = int(r["run_id"])
        arr[i].reserved = 0
    return arr


class Batch(Filter):
    """Independent runs of one model in one set of launches per stage
    (pphd_batch_*).  Inherits the state, tuning and timing methods; the
    update and extraction take every run's measurements at once."""

    def __init__(self, params: dict, runs, precision: int, cap: int, max_meas: int, seed: int, stream=None,
                 apply_tuning: bool = True):
        import torch
        self.torch = torch
        self.params = params
        self.runs = [dict(r) for r in runs]
        self.nruns = len(runs)
        self.K = int(sum(int(r["partitions"]) for r in runs))
        self.run_g0 = np.concatenate([[0], np.cumsum([int(r["partitions"]) for r in runs])])[:-1].astype(int)
        self.cap = int(cap)
        self.max_meas = int(max_meas)
        self.precision = int(precision)
        self.dim = int(params.get("dim", 4))
        self.model = model_struct(dict(params, partitions=1, births_per_step=0, clutter_rate=0.0,
                                       particles_per_target=1.0), precision)
        self._table = run_table(runs)
        nbytes = pphd_batch_workspace_size(self.model, ctypes.addressof(self._table), self.nruns, self.cap,
                                           self.max_meas)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = pphd_batch_create(self.model, ctypes.addressof(self._table), self.nruns, self.cap, self.max_meas,
                                   aligned, nbytes, int(seed), self.stream.cuda_stream)
        self.last_m = 0
        self.tuning = None
        if apply_tuning:
            lam = float(np.mean([float(r["clutter_rate"]) for r in runs]))
            self.tuning = lookup_tuning(self.precision, True, self.K, self.cap, lam + 10.0)
            apply_tuning_to(self.h, self.tuning)

    @staticmethod
    def pack(Zs):
        """Concatenated sets and (offset, count) windows of a list of [m_r, 2] arrays."""
        counts = np.array([np.asarray(z).reshape(-1, 2).shape[0] for z in Zs], dtype=np.int32)
        offs = np.concatenate([[0], np.cumsum(counts)])[:-1].astype(np.int32)
        z = np.concatenate([np.asarray(z, dtype=np.float64).reshape(-1, 2) for z in Zs]) if counts.sum() else \
            np.zeros((0, 2))
        return np.ascontiguousarray(z), np.ascontiguousarray(np.stack([offs, counts], axis=1))

    def update(self, Zs):
        """Zs: list of [m_r, 2] host arrays (one per run)."""
        z, win = self.pack(Zs)
        pphd_batch_update(self.h, z.ctypes.data if z.shape[0] else None, z.shape[0], win.ctypes.data, 0)

    def update_device(self, dz, z_count, dwin):
        pphd_batch_update(self.h, dz.data_ptr(), z_count, dwin.data_ptr(), 1)

    def extract(self):
        """List (per run) of estimate record arrays, and every group's mass."""
        cap = max(self.max_meas, 1)
        out = np.zeros(self.nruns * cap, dtype=ESTIMATE_DTYPE)
        n = np.zeros(self.nruns, dtype=np.int32)
        mass = np.zeros(self.K)
        pphd_batch_extract(self.h, out.ctypes.data, cap, n.ctypes.data, mass.ctypes.data)
        return [out[r * cap:r * cap + int(n[r])].copy() for r in range(self.nruns)], mass

    def extract_device(self, d_out, d_n, cap):
        pphd_batch_extract_device(self.h, d_out.data_ptr(), cap, d_n.data_ptr())

    def capture(self, dz, z_count, dwin, d_out, cap, d_n, first_step):
        pphd_batch_capture(self.h, dz.data_ptr(), z_count, dwin.data_ptr(), d_out.data_ptr(), cap, d_n.data_ptr(),
                           first_step)

    def launch(self):
        pphd_batch_launch(self.h)


class Mlp:
    """The learned birth proposal's network (include/pphd_mlp.h) on the current
    torch device and stream; host arrays are numpy."""

    def __init__(self, params: dict, batch=4096, dataset=1 << 20, seed=0, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8, stream=None):
        import torch
        self.cfg = pphd_mlp_config(int(batch), int(dataset), float(lr), float(beta1), float(beta2), float(eps))
        nbytes = pphd_mlp_workspace_size(self.cfg)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        aligned = (self.workspace.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = pphd_mlp_create(model_struct(params, PPHD_FP32), self.cfg, aligned, nbytes, int(seed),
                                 self.stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None) is not None:
            pphd_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_params(self, init_id=0):
        pphd_mlp_init_params(self.h, init_id)

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32).reshape(MLP_PARAMS)
        pphd_mlp_set_params(self.h, theta.ctypes.data, 0)

    def get_params(self):
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        pphd_mlp_get_params(self.h, out.ctypes.data, 0)
        return out

    def simulate(self, run=0):
        pphd_mlp_simulate(self.h, run)

    def read_dataset(self, first, n):
        z = np.zeros((max(n, 1), 2), dtype=np.float32)
        x = np.zeros((max(n, 1), 4), dtype=np.float32)
        pphd_mlp_read_dataset(self.h, first, n, z.ctypes.data, x.ctypes.data)
        return z[:n], x[:n]

    def loss_grad(self, z, x):
        z = np.ascontiguousarray(z, dtype=np.float32).reshape(-1, 2)
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 4)
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = pphd_mlp_loss_grad(self.h, z.ctypes.data, x.ctypes.data, z.shape[0], 0, g.ctypes.data)
        return loss, g

    def train(self, steps, lr=0.0, record_loss=True):
        loss = np.zeros(max(int(steps), 1), dtype=np.float32) if record_loss else None
        pphd_mlp_train(self.h, steps, lr, loss.ctypes.data if record_loss else None)
        return loss[:steps] if record_loss else None

    def forward(self, z):
        z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1, 2)
        out = np.zeros((max(z.shape[0], 1), MLP_OUTPUTS), dtype=np.float32)
        pphd_mlp_forward(self.h, z.ctypes.data, z.shape[0], 0, out.ctypes.data)
        return out[:z.shape[0]]

    def steps(self):
        return pphd_mlp_steps(self.h)
