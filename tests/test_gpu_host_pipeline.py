"""GPU: lp_batch_solve_host -- batches in host memory streamed through the
device in chunks (three rotating chunk buffers, upload / solve / download
streams).  Results must match the oracle (status exact, objective 1e-9) and be
the same bits as the device-resident solve of the same batch (every chunk runs
the same kernels on the same LPs)."""
import numpy as np
import pytest

from helpers import assert_parity, oracle_solve
from paper_1802_08557_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1802_08557_amd import lpbatch
    c = lpbatch.Context(0)
    yield c
    c.close()


def device_solve(ctx, batch, **kw):
    import torch
    from paper_1802_08557_amd.lpbatch import DeviceBatch
    sol = ctx.solve(DeviceBatch.from_host(batch), **kw)
    torch.cuda.synchronize()
    return sol.status.cpu().numpy(), sol.x.cpu().numpy(), sol.obj.cpu().numpy()


def host_solve(ctx, batch, **kw):
    print(f"[gpu] host solve {batch.name} N={batch.num_lps} {kw}", flush=True)
    return ctx.solve_host(batch.A, batch.b, batch.c, batch.sense, batch.m, batch.n, **kw)


@pytest.mark.parametrize("chunk", [1, 7, 64, 0])
def test_pageable_chunks_match_oracle_and_device(ctx, chunk):
    # Mixed sizes (wavefront and workgroup kernels), two-phase LPs, and chunk
    # counts from one LP per chunk (every buffer set reused many times) to the
    # automatic choice (a single chunk here).
    bt = W.uneven_batch(150, seed=31, lo=4, hi=70)
    st, x, obj = host_solve(ctx, bt, chunk_lps=chunk)
    assert_parity(bt, st, obj, x, oracle_solve(bt))
    dst, dx, dobj = device_solve(ctx, bt)
    np.testing.assert_array_equal(st, dst)
    np.testing.assert_array_equal(obj, dobj)
    np.testing.assert_array_equal(x, dx)


def test_pinned_inputs_and_outputs(ctx):
    import torch
    bt = W.uneven_batch(120, seed=32, lo=3, hi=40)
    pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
    A, b, c, s = pin(bt.A), pin(bt.b), pin(bt.c), pin(bt.sense)
    out = (torch.empty(bt.num_lps, dtype=torch.int32).pin_memory(),
           torch.empty(int(bt.n.sum()), dtype=torch.float64).pin_memory(),
           torch.empty(bt.num_lps, dtype=torch.float64).pin_memory())
    print("[gpu] host solve pinned", flush=True)
    ctx.solve_host(A, b, c, s, bt.m, bt.n, chunk_lps=11, out=out)
    st, x, obj = (t.numpy() for t in out)
    assert_parity(bt, st, obj, x, oracle_solve(bt))
    dst, dx, dobj = device_solve(ctx, bt)
    np.testing.assert_array_equal(obj, dobj)
    np.testing.assert_array_equal(x, dx)


def test_mixed_pinned_and_pageable(ctx):
    # Pinned inputs, pageable outputs: each array takes its own route.
    import torch
    bt = W.uniform_batch(300, 12, 9, seed=33)
    A = torch.from_numpy(bt.A).pin_memory()
    st, x, obj = ctx.solve_host(A, bt.b, bt.c, bt.sense, bt.m, bt.n, chunk_lps=50)
    assert_parity(bt, st, obj, x, oracle_solve(bt))


def test_fp32_certified_through_host_path(ctx):
    from paper_1802_08557_amd import lpbatch
    bt = W.uniform_batch(400, 30, 30, seed=34)
    st, x, obj = host_solve(ctx, bt, chunk_lps=90, precision=lpbatch.PREC_FP32_CERT64)
    assert_parity(bt, st, obj, x, oracle_solve(bt))


def test_default_chunking_of_a_larger_uniform_batch(ctx):
    # 9000 LPs: the automatic chunk is max(4096, ceil(N / 8)) = 4096 -> three
    # chunks, the last one partial.
    bt = W.uniform_batch(9000, 20, 20, seed=35)
    st, x, obj = host_solve(ctx, bt)
    ref = oracle_solve(bt)
    assert_parity(bt, st, obj, x, ref)


def test_empty_batch_and_argument_errors(ctx):
    from paper_1802_08557_amd import lpbatch
    e = np.zeros(0)
    st, x, obj = ctx.solve_host(e, e, e, np.zeros(0, np.int8), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert st.size == 0 and x.size == 0 and obj.size == 0
    bt = W.uniform_batch(4, 3, 3, seed=36)
    with pytest.raises(lpbatch.LPBatchError) as ei:
        ctx.solve_host(bt.A, bt.b, bt.c, bt.sense, bt.m, bt.n, chunk_lps=-1)
    assert ei.value.code == lpbatch.LP_ERR_ARG
    bad_m = bt.m.copy()
    bad_m[2] = 0
    with pytest.raises(lpbatch.LPBatchError) as ei:
        ctx.solve_host(bt.A, bt.b, bt.c, bt.sense, bad_m, bt.n)
    assert ei.value.code == lpbatch.LP_ERR_ARG
