"""Pins of the oracle's random streams.

Philox-4x32-10 is checked against an independent implementation: the
header-only engine of rocRAND, compiled here for the host and run (nothing of
it is copied).  The uniform and Box-Muller mappings are checked against their
closed forms and moments."""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROCRAND_PROBE = r"""
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  // reads lines "c0 c1 c2 c3 k0 k1" (hex), prints the Philox-4x32-10 block
  unsigned c[4], k[2];
  while (scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
    unsigned long long seed = ((unsigned long long)k[1] << 32) | k[0];
    unsigned long long subseq = ((unsigned long long)c[3] << 32) | c[2];
    // counter words 0-1 are reached with discard(): each unit of the 64-bit
    // low counter is four outputs (split so that no offset overflows)
    rocrand_device::philox4x32_10_engine e(seed, subseq, 4ull * c[0]);
    for (int i = 0; i < 4; ++i) e.discard((unsigned long long)c[1] << 32);
    uint4 r = e.next4();
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_probe():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "probe.cpp")
    exe = os.path.join(d, "probe")
    with open(src, "w") as f:
        f.write(ROCRAND_PROBE)
    subprocess.run([hipcc, "-O1", src, "-o", exe], check=True, capture_output=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_rocrand(orc, rocrand_probe):
    rng = np.random.default_rng(12345)
    cases = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 2, 3, 4, 5, 6)]
    for _ in range(2000):
        cases.append(tuple(int(v) for v in rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)))
    # counters of the shape the filter uses (slot, step, purpose*16+sub, run)
    for slot in (0, 1, 4095, 1 << 20):
        for purpose in (1, 2, 3, 4, 5):
            cases.append((slot, 7, purpose * 16 + 1, 3, 0x5EED0001, 0))
    inp = "\n".join(" ".join(f"{v:08x}" for v in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for c, line in zip(cases, out):
        want = [int(t, 16) for t in line.split()]
        got = orc.philox(c[:4], c[4:])
        assert got == want, (c, got, want)


def test_u53_closed_form(orc):
    assert orc.u53(0, 0) == 2.0 ** -53
    assert orc.u53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0
    assert orc.u53(0, 0x7FF) == 2.0 ** -53          # low 11 bits of b are dropped
    assert orc.u53(0, 0x800) == 2.0 * 2.0 ** -53
    assert orc.u53(1, 0) == (2 ** 21 + 1) * 2.0 ** -53
    a, b = 0x12345678, 0x9ABCDEF0
    assert orc.u53(a, b) == ((a << 21 | b >> 11) + 1) / 2.0 ** 53


def test_predict_noise_moments(orc):
    """With T = 1, sigma_a = 1 and a zero state, the velocity after predict is
    exactly the drawn standard normal; its moments must match N(0, 1)."""
    from paper_1503_03769_amd.scenario import BASE_MODEL
    p = dict(BASE_MODEL, sigma_a=1.0, T=1.0, partitions=1, births_per_step=0)
    n = 200000
    st = orc.State(1, n)
    st.n[0] = n
    st.W[:] = 1.0
    orc.predict(p, st, 3, 99, 0)
    v = np.concatenate([st.X[1, :n], st.X[3, :n]])
    N = v.size
    assert abs(v.mean()) < 5 / math.sqrt(N)
    assert abs(v.var() - 1.0) < 5 * math.sqrt(2.0 / N)
    assert abs(np.mean(v ** 3)) < 5 * math.sqrt(15.0 / N)
    assert abs(np.mean(v ** 4) - 3.0) < 5 * math.sqrt(96.0 / N)
    # x and y noise are independent
    assert abs(np.mean(st.X[1, :n] * st.X[3, :n])) < 5 / math.sqrt(n)
