"""The device's elementary functions against the oracle's on every fp32 input of the domain
the samplers use them on: log on all positive floats, log1p on x > -1, exp and expm1 on all
finite floats; and the map from a Philox output word to a uniform on all 2^32 words.  Outputs
must be bit-identical (NaN compared as NaN)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

POS = (0x00000000, 0x7F800000)          # +0 .. largest finite
NEG_TO_M1 = (0x80000000, 0xBF800000)    # -0 .. -(1 - 2^-24)
NEG = (0x80000000, 0xFF800000)          # -0 .. most negative finite
DOMAINS = {0: [(0x00000001, 0x7F800000)], 1: [POS, NEG_TO_M1], 2: [POS, NEG], 3: [POS, NEG],
           4: [(0x00000000, 0x100000000)]}
NAMES = {0: "log", 1: "log1p", 2: "exp", 3: "expm1", 4: "uniform"}
CHUNK = 1 << 28


@pytest.fixture(scope="module")
def eb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_13259_amd import binding
    return binding


@pytest.mark.parametrize("kind", [0, 1, 2, 3, 4])
def test_math_exhaustive(eb, kind):
    import torch
    workers = min(16, os.cpu_count() or 1)
    oracle.lib()                      # load once before the worker threads use it
    checked = 0
    with ThreadPoolExecutor(workers) as pool:
        for lo, hi in DOMAINS[kind]:
            for a in range(lo, hi, CHUNK):
                b = min(a + CHUNK, hi)
                xg = torch.arange(a, b, dtype=torch.int64, device="cuda").to(torch.int32).view(torch.float32)
                yg = eb.selftest_math(kind, xg).cpu().numpy()
                del xg
                x = np.arange(a, b, dtype=np.uint32).view(np.float32)
                yc = np.concatenate(list(pool.map(lambda p: oracle.math_fn(kind, p), np.array_split(x, 4 * workers))))
                same = yg.view(np.uint32) == yc.view(np.uint32)
                if not same.all():
                    bad = ~same & ~(np.isnan(yg) & np.isnan(yc))
                    idx = np.flatnonzero(bad)
                    assert idx.size == 0, (NAMES[kind], hex(a + int(idx[0])), yg[idx[0]], yc[idx[0]], idx.size)
                checked += b - a
    print(f"{NAMES[kind]}: {checked} inputs bit-identical", flush=True)
