"""Pins for the oracle's random-number layer and elementary functions.

* Philox4x32-10 is checked against two independent implementations: PyTorch's C++
  PhiloxRNGEngine header and rocRAND's Philox4x32-10 header, each compiled here into a tiny
  helper.
* The uniform map u = (2*(x>>9)+1) 2^-24 is checked exhaustively over its 2^23 classes.
* The fp32 log/log1p/exp/expm1 written from their series are checked against fp64
  numpy on dense grids to a stated ulp bound.
"""
import os
import subprocess
import tempfile

import numpy as np
import pytest
import torch

import oracle

ATEN_SRC = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned c0,c1,c2,c3,k0,k1;
  while (scanf("%u %u %u %u %u %u", &c0,&c1,&c2,&c3,&k0,&k1) == 6) {
    uint64_t seed = ((uint64_t)k1 << 32) | k0;
    uint64_t sub = ((uint64_t)c3 << 32) | c2;
    at::philox_engine e(seed, sub, 0);
    e.set_offset(((uint64_t)c1 << 32) | c0);
    unsigned a = e(), b = e(), c = e(), d = e();
    printf("%u %u %u %u\n", a, b, c, d);
  }
}
"""


@pytest.fixture(scope="module")
def aten_philox():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "px.cpp")
    exe = os.path.join(d, "px")
    open(src, "w").write(ATEN_SRC)
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I" + inc, "-o", exe, src], check=True)
    return exe


def test_philox_matches_independent_implementation(aten_philox):
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2**32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(2000, 2), dtype=np.uint64).astype(np.uint32)
    # include the counters the simulator actually uses (small rep/station/step, substream<<24|block)
    ctr[:8] = [[0, 0, 0, 0], [1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1],
               [5, 3, 999, (2 << 24) | 7], [4095, 999, 19999, 1 << 24], [0xFFFFFFFF] * 4]
    key[:8] = [[0, 0]] * 8
    lines = "\n".join(" ".join(str(int(v)) for v in (*c, *k)) for c, k in zip(ctr, key))
    res = subprocess.run([aten_philox], input=lines, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t) for t in ln.split()] for ln in res.strip().splitlines()], dtype=np.uint32)
    got = oracle.philox(ctr, key)
    assert np.array_equal(got, ref)


ROCRAND_SRC = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
// rocRAND's own ten-round Philox4x32 block function on a given counter and key
struct Block : rocrand_device::philox4x32_10_engine {
  uint4 at(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  Block b;
  while (scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint4 c; c.x = c0; c.y = c1; c.z = c2; c.w = c3;
    uint2 k; k.x = k0; k.y = k1;
    uint4 r = b.at(c, k);
    printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
}
"""


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc for rocRAND's header")
def test_philox_matches_rocrand(tmp_path):
    """A second independent implementation: rocRAND's Philox4x32-10 block function (its source
    header, compiled here for the host), on random counters and keys and on the counters the
    simulator uses."""
    src, exe = str(tmp_path / "rr.cpp"), str(tmp_path / "rr")
    open(src, "w").write(ROCRAND_SRC)
    subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-o", exe, src], check=True, capture_output=True)
    rng = np.random.default_rng(13)
    ctr = rng.integers(0, 2**32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(2000, 2), dtype=np.uint64).astype(np.uint32)
    ctr[:4] = [[0, 0, 0, 0], [3, 7, 19999, (2 << 24) | 5], [4095, 999, 0, 1 << 24], [0xFFFFFFFF] * 4]
    lines = "\n".join(" ".join(str(int(v)) for v in (*c, *k)) for c, k in zip(ctr, key))
    res = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t) for t in ln.split()] for ln in res.strip().splitlines()], dtype=np.uint32)
    assert np.array_equal(oracle.philox(ctr, key), ref)


def test_uniform_map_exhaustive():
    j = np.arange(2**23, dtype=np.uint32)
    x = j << np.uint32(9)                       # every class x>>9 = j, low bits zero
    u = oracle.u01(x)
    # low 9 bits must not matter
    assert np.array_equal(u, oracle.u01(x | np.uint32(0x1FF)))
    expect = (2.0 * j.astype(np.float64) + 1.0) * 2.0 ** -24
    assert np.array_equal(u.astype(np.float64), expect)          # exact
    assert u.min() == np.float32(2.0 ** -24) and u.max() == np.float32(1 - 2.0 ** -24)
    assert np.all(np.diff(u) > 0)                                # strictly increasing, never 0 or 1
    # the C function the samplers call, on the same words and with random low bits
    low = np.random.default_rng(5).integers(0, 512, size=j.size, dtype=np.uint32)
    for words in (x, x | low):
        assert np.array_equal(oracle.math_fn(4, words.view(np.float32)).astype(np.float64), expect)


def _ulp_err(got32, ref64):
    got = got32.astype(np.float64)
    ulp = np.spacing(np.abs(ref64).astype(np.float32)).astype(np.float64)
    return np.abs(got - ref64) / ulp


def test_logf_accuracy():
    rng = np.random.default_rng(1)
    x = np.concatenate([
        np.exp(rng.uniform(np.log(1.2e-38), np.log(3e38), 400000)),
        rng.uniform(0.5, 2.0, 400000),
        1.0 + rng.uniform(-1e-3, 1e-3, 100000),
        np.array([2.0 ** -24, 1 - 2.0 ** -24, 1.0, 2.0, 0.5, np.sqrt(2.0)]),
    ]).astype(np.float32)
    y = oracle.math_fn(0, x)
    ref = np.log(x.astype(np.float64))
    err = _ulp_err(y, ref)
    err[ref == 0] = np.abs(y[ref == 0])
    assert err.max() <= 2.0, err.max()


def test_log1pf_accuracy():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(-0.999, 3.0, 400000), rng.uniform(-0.3, 0.3, 400000),
                        np.sign(rng.uniform(-1, 1, 100000)) * np.exp(rng.uniform(-80, -2, 100000))]).astype(np.float32)
    y = oracle.math_fn(1, x)
    ref = np.log1p(x.astype(np.float64))
    err = _ulp_err(y, ref)
    assert err.max() <= 2.5, err.max()


def test_expf_accuracy():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-86.0, 88.0, 800000), rng.uniform(-1, 1, 200000)]).astype(np.float32)
    y = oracle.math_fn(2, x)
    ref = np.exp(x.astype(np.float64))
    assert _ulp_err(y, ref).max() <= 2.0
    assert oracle.math_fn(2, np.array([-90.0], np.float32))[0] == 0.0


def test_expm1f_accuracy():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.uniform(-20.0, 5.0, 500000), rng.uniform(-0.4, 0.4, 400000),
                        -np.exp(rng.uniform(-60, -1, 100000))]).astype(np.float32)
    y = oracle.math_fn(3, x)
    ref = np.expm1(x.astype(np.float64))
    assert _ulp_err(y, ref).max() <= 2.0


def test_sampler_tables():
    inv, fc = oracle.sampler_tables()
    k = np.arange(1, 256)
    assert len(inv) == 256 and inv[0] == 0
    assert np.array_equal(inv[1:], (np.float32(1.0) / k.astype(np.float32)))
    from math import lgamma, log, pi
    for j in range(10):
        exact = lgamma(j + 1) - ((j + 0.5) * log(j + 1) - (j + 1) + 0.5 * log(2 * pi))
        assert abs(fc[j] - exact) < 1e-8
