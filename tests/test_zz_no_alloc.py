"""The allocation-free run entry point (eq_sim_run_noalloc) against eq_sim_run on the GPU,
through the C ABI: bit-identical states and tile sums on two calls in a row, the second with a
smaller input (fewer replications, the other scheme) reusing the same static scratch; the
refusals (tables not built, a run needing more scratch than the static array) happen on the
host before any launch."""
import ctypes as C

import numpy as np
import pytest

import netgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_13259_amd import binding
    return binding


def noalloc(eb, net, d):
    import torch
    st = torch.empty((net.n, d.reps), dtype=torch.int32, device="cuda")
    sums = torch.empty((3, net.n, eb.n_tiles(d.reps)), dtype=torch.int64, device="cuda")
    rc = eb.eq_sim_run_noalloc(net.handle, C.byref(d), None, st.data_ptr(), sums.data_ptr(),
                               torch.cuda.current_stream().cuda_stream)
    return rc, st, sums


def test_noalloc_equals_sim_run(eb):
    import torch
    w = netgen.config3()
    net = eb.Net(w.net)
    K = 300
    first = eb.make_desc(0, w.dt, K, w.reps, 13)              # 4096 replications: 32 MiB of slots
    rc, _, _ = noalloc(eb, net, first)
    assert rc == eb.EQ_EINVAL and b"tables" in eb.eq_last_error()
    second = eb.make_desc(1, w.dt, K, 1000, 13)               # smaller: 1000 replications, forward
    for d in (first, second):
        ref = eb.simulate(net, d.scheme, w.dt, K, d.reps, 13)
        torch.cuda.synchronize()
        rc, st, sums = noalloc(eb, net, d)
        assert rc == 0, eb.eq_last_error()
        eb._check(eb.eq_sim_check(net.handle, None))
        torch.cuda.synchronize()
        assert torch.equal(st, ref.state) and torch.equal(sums, ref.sums), (d.scheme, d.reps)
    # the second call's first replications against the oracle as well
    o = oracle.run(w.net, 1, w.dt, K, 13, np.arange(3))
    assert np.array_equal(st.cpu().numpy().T[:3], o["final"])


def test_noalloc_refuses_oversize(eb):
    import torch
    w = netgen.config3()
    net = eb.Net(w.net)
    eb.simulate(net, 1, w.dt, 2, 64, 0)
    torch.cuda.synchronize()
    d = eb.make_desc(1, w.dt, 2, 4096, 0)                     # forward rings: 141 MB > 64 MiB
    st = torch.empty((net.n, 4096), dtype=torch.int32, device="cuda")
    assert eb.eq_sim_run_noalloc(net.handle, C.byref(d), None, st.data_ptr(), None, None) == eb.EQ_EINVAL
    assert b"bytes of scratch" in eb.eq_last_error()
