"""Oracle for the distributed particle PHD filter -- TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation (``pphd_oracle.c``) of the per-step recursion of
the distributed computation particle PHD filter (Wang et al., arXiv 1503.03769):
prediction and births (Eqs 5-6), the grouped update (Eqs 10-15), local
estimation (Eqs 16-18), central fusion (section 3.1, Step 4), group-local
resampling (Step 5) and the ring exchange (Step 6), plus the textbook single-set
filter of section 2.2 for cross-checking, and the births of a learned
proposal.  This module only marshals numpy arrays into it; ``oracle.mlp`` holds
the FP64 network of the learned proposal.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

PURPOSE_INIT, PURPOSE_PREDICT, PURPOSE_BIRTH, PURPOSE_RESAMPLE, PURPOSE_EXCHANGE, PURPOSE_PAIRS = 1, 2, 3, 4, 5, 6


class OrcModel(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("partitions", ctypes.c_int32),
        ("births_per_step", ctypes.c_int32), ("global_cz", ctypes.c_int32),
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
        ("birth_proposal", ctypes.c_int32), ("reserved2", ctypes.c_int32), ("birth_alpha", ctypes.c_double),
        ("birth_density", ctypes.c_int32), ("reserved3", ctypes.c_int32),
        ("birth_mean", ctypes.c_double * 4), ("birth_std", ctypes.c_double * 4),
        ("sigma_w", ctypes.c_double), ("birth_sigma_w", ctypes.c_double),
    ]


def model_struct(p: dict) -> OrcModel:
    m = OrcModel()
    m.dim = int(p.get("dim", 4))
    m.partitions = int(p["partitions"])
    m.births_per_step = int(p["births_per_step"])
    m.global_cz = int(p.get("global_cz", 0))
    for k in ("T", "sigma_a", "sensor_x", "sensor_y", "sigma_r", "sigma_theta", "p_S", "p_D",
              "clutter_rate", "r_min", "r_max", "th_min", "th_max", "birth_mass",
              "birth_sigma_v", "init_mass", "particles_per_target", "exchange_fraction"):
        setattr(m, k, float(p[k]))
    for i in range(4):
        m.region[i] = float(p["region"][i])
    m.birth_proposal = int(p.get("birth_proposal", 0))
    m.birth_alpha = float(p.get("birth_alpha", 1.0))
    m.birth_density = int(p.get("birth_density", 0))
    for i in range(4):
        m.birth_mean[i] = float(p.get("birth_mean", (0.0,) * 4)[i])
        m.birth_std[i] = float(p.get("birth_std", (1.0,) * 4)[i])
    m.sigma_w = float(p.get("sigma_w", 0.0))
    m.birth_sigma_w = float(p.get("birth_sigma_w", 0.0))
    return m


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        src = os.path.join(_HERE, "pphd_oracle.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        L = ctypes.CDLL(path)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.POINTER(ctypes.c_int32)
        U = ctypes.POINTER(ctypes.c_uint32)
        M = ctypes.POINTER(OrcModel)
        c_int, u32, u64 = ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64
        L.orc_philox4x32_10.argtypes = [U, U, U]
        L.orc_set_threads.argtypes = [c_int]
        L.orc_threads.restype = c_int
        L.orc_u53.argtypes = [u32, u32]
        L.orc_u53.restype = ctypes.c_double
        L.orc_kappa.argtypes = [M]
        L.orc_kappa.restype = ctypes.c_double
        L.orc_likelihood.argtypes = [M] + [ctypes.c_double] * 4
        L.orc_likelihood.restype = ctypes.c_double
        L.orc_births_in_partition.argtypes = [M, c_int]
        L.orc_init.argtypes = [M, c_int, u64, u32, D, D, I]
        L.orc_predict.argtypes = [M, c_int, u32, u64, u32, D, D, I]
        L.orc_update.argtypes = [M, c_int, D, c_int, D, D, I, D, D, D, D, D]
        L.orc_birth_proposal_density.argtypes = [M, D, c_int, ctypes.c_double, ctypes.c_double]
        L.orc_birth_proposal_density.restype = ctypes.c_double
        L.orc_birth_from_measurements.argtypes = [M, c_int, u32, u64, u32, D, c_int, D, D, I]
        L.orc_bearing_bucket.argtypes = [M, ctypes.c_double, ctypes.c_double]
        L.orc_sort_by_bucket.argtypes = [M, ctypes.c_size_t, D, D, ctypes.c_size_t, c_int]
        L.orc_mixture_proposal_density.argtypes = [M, D, c_int, D]
        L.orc_mixture_proposal_density.restype = ctypes.c_double
        L.orc_birth_from_mixture.argtypes = [M, c_int, u32, u64, u32, D, c_int, D, D, I]
        L.orc_simulate_pairs.argtypes = [M, u64, u32, c_int, c_int, D, D]
        L.orc_extract.argtypes = [M, c_int, D, D, D, I, I, D]
        L.orc_fuse.argtypes = [M, c_int, I, D, D, I, I, I]
        L.orc_resample.argtypes = [M, c_int, u32, u64, u32, D, D, I, D, D, I, I, D]
        L.orc_exchange.argtypes = [M, c_int, u32, u64, u32, D, D, I]
        L.orc_textbook_step.argtypes = [M, c_int, u32, u64, u32, D, c_int, D, D, I, D, D, D, I]
        _LIB = L
    return _LIB


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def set_threads(n):
    """Threads of the per-group loops (the results do not depend on it)."""
    lib().orc_set_threads(int(n))


def threads():
    return int(lib().orc_threads())


def u53(a, b):
    return lib().orc_u53(int(a), int(b))


def kappa(p):
    return lib().orc_kappa(ctypes.byref(model_struct(p)))


def likelihood(p, zr, zth, x, y):
    return lib().orc_likelihood(ctypes.byref(model_struct(p)), zr, zth, x, y)


def births_in_partition(p, j):
    return lib().orc_births_in_partition(ctypes.byref(model_struct(p)), j)


class State:
    """Particle state in the oracle layout: X[dim][K*cap], W[K*cap], n[K]."""

    def __init__(self, K, cap, dim=4):
        self.K, self.cap = K, cap
        self.X = np.zeros((dim, K * cap), dtype=np.float64)
        self.W = np.zeros(K * cap, dtype=np.float64)
        self.n = np.zeros(K, dtype=np.int32)

    def copy(self):
        s = State(self.K, self.cap, self.X.shape[0])
        s.X[:] = self.X
        s.W[:] = self.W
        s.n[:] = self.n
        return s

    def particles(self, j):
        """(states [n_j, 4], weights [n_j]) of partition j."""
        a, b = j * self.cap, j * self.cap + int(self.n[j])
        return self.X[:, a:b].T.copy(), self.W[a:b].copy()


def init(p, st, seed, run):
    _check(lib().orc_init(ctypes.byref(model_struct(p)), st.cap, seed, run, _d(st.X), _d(st.W), _i(st.n)), "init")


def predict(p, st, step, seed, run):
    _check(lib().orc_predict(ctypes.byref(model_struct(p)), st.cap, step, seed, run,
                             _d(st.X), _d(st.W), _i(st.n)), "predict")


def _zbuf(Z):
    Z = np.ascontiguousarray(np.asarray(Z, dtype=np.float64).reshape(-1, 2))
    return Z, (Z.reshape(-1) if Z.shape[0] > 0 else np.zeros(2))


def birth_proposal_density(p, Z, x, y):
    Z, Zb = _zbuf(Z)
    return lib().orc_birth_proposal_density(ctypes.byref(model_struct(p)), _d(Zb), Z.shape[0], x, y)


def birth_from_measurements(p, st, step, seed, run, Z):
    """Fills the J_j reserved birth slots of every group (measurement-driven proposal)."""
    Z, Zb = _zbuf(Z)
    _check(lib().orc_birth_from_measurements(ctypes.byref(model_struct(p)), st.cap, step, seed, run, _d(Zb),
                                              Z.shape[0], _d(st.X), _d(st.W), _i(st.n)), "birth_from_measurements")


def bearing_bucket(p, x, y):
    """Bearing bucket (0..63) the resampling orders parents by."""
    return lib().orc_bearing_bucket(ctypes.byref(model_struct(p)), float(x), float(y))


def sort_by_bucket(p, st, base, count):
    """Stable bearing-bucket order of the slots [base, base + count) of st
    (the order births take once drawn)."""
    _check(lib().orc_sort_by_bucket(ctypes.byref(model_struct(dict(p, dim=st.X.shape[0]))), st.K * st.cap, _d(st.X),
                                    _d(st.W), int(base), int(count)), "sort_by_bucket")


def _table(table, M):
    t = np.ascontiguousarray(np.asarray(table, dtype=np.float64).reshape(-1))
    assert t.size == M * 36, (t.size, M)
    return t if M > 0 else np.zeros(36)


def mixture_proposal_density(p, table, x):
    """Proposal density (learned mixtures, birth_proposal 2) at state x."""
    t = np.asarray(table, dtype=np.float64).reshape(-1, 4, 9)
    M = t.shape[0]
    xs = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(4))
    return lib().orc_mixture_proposal_density(ctypes.byref(model_struct(p)), _d(_table(t, M)), M, _d(xs))


def birth_from_mixture(p, st, step, seed, run, table):
    """Fills the J_j reserved birth slots of every group from the learned
    proposal; table [M, 4, 9] as made by oracle.mlp.mixture_table."""
    t = np.asarray(table, dtype=np.float64).reshape(-1, 4, 9)
    M = t.shape[0]
    _check(lib().orc_birth_from_mixture(ctypes.byref(model_struct(p)), st.cap, step, seed, run, _d(_table(t, M)),
                                         M, _d(st.X), _d(st.W), _i(st.n)), "birth_from_mixture")


def simulate_pairs(p, seed, run, first, n):
    """Training pairs (z [n,2], x [n,4]) of the learned proposal."""
    z = np.zeros((max(n, 1), 2))
    x = np.zeros((max(n, 1), 4))
    _check(lib().orc_simulate_pairs(ctypes.byref(model_struct(p)), seed, run, first, n, _d(z), _d(x)),
           "simulate_pairs")
    return z[:n], x[:n]


def update(p, st, Z):
    """Updates st.W in place.  Returns dict with C, dW [K,M], dW0 [K], zeta_num [K,M,4], mass [K]."""
    Z = np.ascontiguousarray(np.asarray(Z, dtype=np.float64).reshape(-1, 2))
    M = Z.shape[0]
    K = st.K
    C = np.zeros(max(K * M, 1))
    dW = np.zeros(max(K * M, 1))
    dW0 = np.zeros(K)
    zn = np.zeros(max(K * M * 4, 1))
    mass = np.zeros(K)
    Zb = Z.reshape(-1) if M > 0 else np.zeros(2)
    _check(lib().orc_update(ctypes.byref(model_struct(p)), st.cap, _d(np.ascontiguousarray(Zb)), M,
                            _d(st.X), _d(st.W), _i(st.n), _d(C), _d(dW), _d(dW0), _d(zn), _d(mass)), "update")
    return dict(C=C[:K * M].reshape(K, M), dW=dW[:K * M].reshape(K, M), dW0=dW0,
                zeta_num=zn[:K * M * 4].reshape(K, M, 4), mass=mass)


def extract(p, M, upd):
    K = int(p["partitions"])
    LT = np.zeros(K, dtype=np.int32)
    sel = np.zeros(max(K * M, 1), dtype=np.int32)
    zeta = np.zeros(max(K * M * 4, 1))
    dW = np.ascontiguousarray(upd["dW"].reshape(-1)) if M > 0 else np.zeros(1)
    zn = np.ascontiguousarray(upd["zeta_num"].reshape(-1)) if M > 0 else np.zeros(1)
    _check(lib().orc_extract(ctypes.byref(model_struct(p)), M, _d(dW), _d(zn),
                             _d(np.ascontiguousarray(upd["mass"])), _i(LT), _i(sel), _d(zeta)), "extract")
    return dict(LT=LT, sel=sel[:K * M].reshape(K, M), zeta=zeta[:K * M * 4].reshape(K, M, 4))


def fuse(p, M, ext):
    K = int(p["partitions"])
    cap = max(M, 1)
    est = np.zeros(cap * 4)
    lab = np.zeros(cap, dtype=np.int32)
    votes = np.zeros(cap, dtype=np.int32)
    n = np.zeros(1, dtype=np.int32)
    sel = np.ascontiguousarray(ext["sel"].reshape(-1)) if M > 0 else np.zeros(K, dtype=np.int32)
    zeta = np.ascontiguousarray(ext["zeta"].reshape(-1)) if M > 0 else np.zeros(4 * K)
    _check(lib().orc_fuse(ctypes.byref(model_struct(p)), M, _i(sel), _d(zeta), _d(est), _i(lab), _i(votes), _i(n)),
           "fuse")
    k = int(n[0])
    return dict(state=est[:4 * k].reshape(k, 4), label=lab[:k].copy(), votes=votes[:k].copy())


def resample(p, st, step, seed, run):
    """Returns (new State, counts [K*cap], mass_q [K])."""
    out = State(st.K, st.cap, st.X.shape[0])
    counts = np.zeros(st.K * st.cap, dtype=np.int32)
    mq = np.zeros(st.K)
    _check(lib().orc_resample(ctypes.byref(model_struct(p)), st.cap, step, seed, run,
                              _d(st.X), _d(st.W), _i(st.n), _d(out.X), _d(out.W), _i(out.n), _i(counts), _d(mq)),
           "resample")
    return out, counts, mq


def exchange(p, st, step, seed, run):
    _check(lib().orc_exchange(ctypes.byref(model_struct(p)), st.cap, step, seed, run,
                              _d(st.X), _d(st.W), _i(st.n)), "exchange")


def textbook_step(p, st, step, seed, run, Z):
    """One step of the single-set filter of section 2.2 (K must be 1).

    st is predicted in place (X, W hold the predicted particles, n the predicted
    count).  Returns (Wupd, resampled State)."""
    Z = np.ascontiguousarray(np.asarray(Z, dtype=np.float64).reshape(-1))
    M = Z.size // 2
    Wupd = np.zeros(st.cap)
    out = State(1, st.cap)
    nout = np.zeros(1, dtype=np.int32)
    Zb = Z if M > 0 else np.zeros(2)
    _check(lib().orc_textbook_step(ctypes.byref(model_struct(p)), st.cap, step, seed, run, _d(Zb), M,
                                   _d(st.X), _d(st.W), _i(st.n), _d(Wupd), _d(out.X), _d(out.W), _i(nout)),
           "textbook_step")
    out.n[0] = nout[0]
    return Wupd, out


class OracleFilter:
    """One run of the grouped filter, step by step, in the paper's order
    (predict, update, extract, fuse, resample, exchange)."""

    def __init__(self, p, cap, seed, run, mlp_theta=None, mlp_hidden=128):
        self.p, self.seed, self.run = p, seed, run
        self.mlp_theta, self.mlp_hidden = mlp_theta, mlp_hidden
        self.st = State(int(p["partitions"]), cap, int(p.get("dim", 4)))
        init(p, self.st, seed, run)

    def step(self, k, Z):
        p = self.p
        predict(p, self.st, k, self.seed, self.run)
        Z = np.asarray(Z, dtype=np.float64).reshape(-1, 2)
        if int(p.get("birth_proposal", 0)) == 1:
            birth_from_measurements(p, self.st, k, self.seed, self.run, Z)
        elif int(p.get("birth_proposal", 0)) == 2:
            from . import mlp
            o, _ = mlp.forward(self.mlp_theta, mlp.features(p, Z), self.mlp_hidden)
            birth_from_mixture(p, self.st, k, self.seed, self.run, mlp.mixture_table(p, Z, o))
        n_pred = self.st.n.copy()
        upd = update(p, self.st, Z)
        ext = extract(p, Z.shape[0], upd)
        est = fuse(p, Z.shape[0], ext)
        self.st, counts, mq = resample(p, self.st, k, self.seed, self.run)
        exchange(p, self.st, k, self.seed, self.run)
        return dict(upd=upd, ext=ext, est=est, counts=counts, mass_q=mq, n_pred=n_pred)
