"""Host-side check of the lower-envelope code the ESDF y and z passes use
(paper_2410_21149_amd/csrc/edt_envelope.h, compiled for the host with
hipcc): on random lines the envelope value at every position equals the
brute-force minimum over all parabolas f(q) + (y - q)^2."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_21149_amd", "csrc")

HARNESS = r'''
#include <cstdio>
#include <vector>
#include "edt_envelope.h"
using namespace covox;
int main() {
    int n; 
    while (scanf("%d", &n) == 1) {
        std::vector<int> f(n);
        for (int i = 0; i < n; ++i) scanf("%d", &f[i]);
        std::vector<uint8_t> stk(256);
        auto getf = [&](int q) { return f[q]; };
        Envelope e; env_clear(e);
        for (int q = 0; q < n; ++q) if (f[q] >= 0) env_push(e, stk.data(), 1, 0, q, f[q], getf);
        Walker w;
        if (e.k >= 0) walk_init(w, e, stk.data(), 1, 0, getf);
        for (int y = 0; y < n; ++y) printf("%d ", e.k >= 0 ? walk_at(w, e, stk.data(), 1, 0, y, getf) : -1);
        printf("\n");
    }
    return 0;
}
'''


@pytest.fixture(scope="module")
def harness():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "h.cpp")
    open(src, "w").write(HARNESS)
    exe = os.path.join(d, "h")
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-I", CSRC, src, "-o", exe],
                          stderr=subprocess.DEVNULL)
    return exe


def test_envelope_matches_brute_force(harness):
    rng = np.random.default_rng(0)
    lines = []
    for t in range(400):
        n = int(rng.integers(1, 257))
        R = int(rng.integers(1, 57))
        f = rng.integers(0, R + 1, size=n) ** 2
        f[rng.uniform(size=n) < rng.uniform(0, 1)] = -1  # no site on this position
        if t % 7 == 0:
            f[:] = -1
            f[rng.integers(0, n)] = 0
        if t % 11 == 0:
            f[:] = rng.integers(0, 3) ** 2  # many ties
        lines.append(f)
    inp = "".join("%d %s\n" % (len(f), " ".join(map(str, f))) for f in lines)
    out = subprocess.run([harness], input=inp, capture_output=True, text=True, check=True).stdout.splitlines()
    assert len(out) == len(lines)
    for f, o in zip(lines, out):
        got = np.array(list(map(int, o.split())))
        q = np.nonzero(f >= 0)[0]
        if len(q) == 0:
            assert np.all(got == -1)
            continue
        y = np.arange(len(f))
        want = np.min(f[q][None, :] + (y[:, None] - q[None, :]) ** 2, axis=1)
        assert np.array_equal(got, want)
