"""pphd_update_noalloc (the update whose first-pass partial sums live in the
library's static device array) against pphd_update on identical filters:
particles, weights, C(z), Delta W, masses, LT, label sets and fused
estimates bit for bit, on two calls in a row, the second with a smaller
input (fewer groups, particles and measurements; measurements already on the
device), and the size limit of the static array."""
import numpy as np
import pytest

from paper_1503_03769_amd import pphd
from paper_1503_03769_amd.scenario import BASE_MODEL, WORKLOADS, make_scenario
from tests import parity as P

pytestmark = pytest.mark.gpu

CALLS = [
    # prec, K, count range, lambda, targets, max_meas, z on device
    ("fp32", 64, (14000, 17000), 50.0, 10, 512, False),
    ("fp32", 8, (2000, 3000), 20.0, 4, 64, True),
    ("fp64", 3, (500, 900), 10.0, 3, 64, False),
]


def _twin(prec, K, rng_c, lam, ntg, maxm, seed):
    p = dict(BASE_MODEL, partitions=K, clutter_rate=lam, births_per_step=0)
    truth, Zs = make_scenario(p, ntg, 6, seed)
    k = max(range(1, 7), key=lambda i: len(truth[i]))
    counts = [int(c) for c in np.random.default_rng(seed).integers(rng_c[0], rng_c[1], K)]
    cap = max(counts) + 256
    X, W, n = P.cloud(K, cap, counts, seed + 1, truth[k], prec)
    fa = P.make_filter(p, prec, cap, max_meas=maxm)
    fb = P.make_filter(p, prec, cap, max_meas=maxm)
    for f in (fa, fb):
        f.write_state(X, W, n, pphd.PHASE_PREDICTED)
    return fa, fb, np.ascontiguousarray(Zs[k])


def test_noalloc_update_equals_update(gpu):
    import torch
    for i, (prec, K, rng_c, lam, ntg, maxm, on_dev) in enumerate(CALLS):
        print(f"call {i + 1}: {prec}, {K} groups, lambda {lam}, z on device {on_dev}", flush=True)
        fa, fb, Z = _twin(prec, K, rng_c, lam, ntg, maxm, 600 + i)
        m = Z.shape[0]
        fa.update(Z)
        if on_dev:
            dz = torch.from_numpy(Z).cuda()
            pphd.pphd_update_noalloc(fb.h, dz.data_ptr() if m else None, m, 1)
        else:
            pphd.pphd_update_noalloc(fb.h, Z.ctypes.data if m else None, m, 0)
        fb.last_m = m
        Xa, Wa, na = fa.read_state()
        Xb, Wb, nb = fb.read_state()
        assert np.array_equal(na, nb)
        for j in range(K):
            sl = slice(j * fa.cap, j * fa.cap + int(na[j]))
            assert np.array_equal(Wa[sl], Wb[sl]), j
            assert np.array_equal(Xa[:, sl], Xb[:, sl]), j
        ua, ub = fa.read_update(), fb.read_update()
        for key in ("C", "dW", "mass", "LT"):
            assert np.array_equal(ua[key], ub[key]), key
        la, lb = fa.read_local(), fb.read_local()
        assert np.array_equal(la["sel"], lb["sel"]) and np.array_equal(la["zeta"], lb["zeta"])
        ea, _ = fa.extract()
        eb, _ = fb.extract()
        assert ea.tobytes() == eb.tobytes()
        print(f"  M = {m}, particles {int(na.sum())}, fused {len(ea)}: equal", flush=True)
        fa.close()
        fb.close()


def test_noalloc_size_limit(gpu):
    """A filter whose first-pass partials exceed the static array is refused
    (16 groups x 512 wave tiles x 1024 measurements: about 100 MB)."""
    p = dict(BASE_MODEL, partitions=16, births_per_step=0, particles_per_target=16000.0)
    f = P.make_filter(p, "fp32", 131072, max_meas=1024)
    X, W, n = P.cloud(16, 131072, [1000] * 16, 3, np.zeros((1, 4)), "fp32")
    f.write_state(X, W, n, pphd.PHASE_PREDICTED)
    Z = np.array([[500.0, 0.3]])
    with pytest.raises(pphd.PphdError) as e:
        pphd.pphd_update_noalloc(f.h, Z.ctypes.data, 1, 0)
    assert e.value.code == pphd.PPHD_EINVAL
    f.update(Z)  # the filter is unchanged and still usable
    f.close()
