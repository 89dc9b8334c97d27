"""Serving path (continuous batching through tfmm_submit / tfmm_poll / tfmm_wait).

Jobs on several operators arrive while others run; the scheduler coalesces
jobs on the same operator into one launch.  Each job's result must be
bitwise the same as the job run alone (every RHS is computed independently
and the restored operator does not depend on the batch), and equal to the
oracle within the arithmetic tolerance.
"""
import numpy as np
import pytest

import oracle as O
import synth
from factor_layout import random_factors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2010_00520_amd as P

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return P


def make_ops(ctx):
    specs = [("tucker3d", (8, 8, 8), 3, None), ("tt4d", (12, 12, 12), 3, (9, 17, 12)), ("full", (4, 8, 8), 3, None),
             ("htucker4d", (16, 8, 8), 2, (6, 5, 5, 7, 11, 10))]
    ops = []
    for i, (fmt, K, L, ranks) in enumerate(specs):
        n = tuple(2 * k for k in K)
        ndir = (L + 1) * 2 * (L + 1)
        rk, data, comp = random_factors(fmt, n, ndir, np.random.default_rng(100 + i), ranks)
        ops.append((ctx.import_factors(K, L, fmt, rk, data), K, ndir, comp))
    return ops


def test_mixed_stream_equals_alone(P):
    ctx = P.Context(0)
    ops = make_ops(ctx)
    rng = np.random.default_rng(7)
    jobs = []
    for j in range(40):
        oi = int(rng.integers(len(ops)))
        op, K, ndir, comp = ops[oi]
        nrhs = int(rng.integers(1, 5))
        A = torch.from_numpy(synth.gaussian_patterns((nrhs, ndir) + K, 1000 + j)).cuda()
        B = torch.zeros_like(A)
        jobs.append((oi, A, B))
    torch.cuda.synchronize()
    tickets = [ctx.submit(ops[oi][0], A, B) for oi, A, B in jobs]
    lats = []
    for t in tickets:
        st, lat = ctx.wait(t)
        assert st == 0
        lats.append(lat)
    assert all(l > 0 for l in lats)
    for j, (oi, A, B) in enumerate(jobs):
        Balone = torch.zeros_like(A)
        ctx.translate(ops[oi][0], A, Balone)
        torch.cuda.synchronize()
        assert torch.equal(B, Balone), f"job {j} differs from its solo run"
    # a few jobs against the oracle as well
    for j in (0, 7, 23):
        oi, A, B = jobs[j]
        ref = O.translate_compressed(A.cpu().numpy(), ops[oi][3])
        assert O.rel_l2(B.cpu().numpy().astype(np.complex128), ref) < 2e-5
    for op, *_ in ops:
        op.release()
    ctx.close()


def test_poll_reports_completion_and_retires_ticket(P):
    ctx = P.Context(0)
    op, K, ndir, _ = make_ops(ctx)[0]
    A = torch.from_numpy(synth.gaussian_patterns((2, ndir) + K, 3)).cuda()
    B = torch.zeros_like(A)
    t = ctx.submit(op, A, B)
    import time

    deadline = time.time() + 60
    done = False
    while not done and time.time() < deadline:
        done, st, lat = ctx.poll(t)
        time.sleep(0.001)
    assert done and st == 0 and lat > 0
    with pytest.raises(P.TfmmError) as e:
        ctx.poll(t)
    assert e.value.status == 7
    ctx.close()


def test_budget_rejects_operator_that_does_not_fit(P):
    ctx = P.Context(0, budget_bytes=1 << 20)
    with pytest.raises(P.TfmmError) as e:
        ctx.setup(K=(16, 16, 16), box=0.5, L=4, fmt="full")
    assert e.value.status == 3
    used, budget = ctx.memory()
    assert used <= budget == 1 << 20
    ctx.close()


def test_release_after_jobs_complete(P):
    ctx = P.Context(0)
    op, K, ndir, _ = make_ops(ctx)[1]
    A = torch.from_numpy(synth.gaussian_patterns((1, ndir) + K, 4)).cuda()
    B = torch.zeros_like(A)
    ts = [ctx.submit(op, A, B) for _ in range(8)]
    try:
        op.release()
        released = True
    except P.TfmmError as e:  # still referenced by queued jobs
        assert e.status == 6
        released = False
    for t in ts:
        ctx.wait(t)
    if not released:
        op.release()
    ctx.close()


def test_jobs_park_for_memory_and_match_solo(P):
    """Memory-based admission: with a budget that holds the operator and one
    job's A and B (not two), jobs submitted together wait for memory at the head
    of the queue instead of failing, complete in order, and each result is
    bitwise the result of the job run alone.  A job that cannot fit even with
    nothing else running fails with TFMM_ERR_BUDGET and leaves the queue moving.
    The operator takes the fused path (16^3 FFT grid), which needs no
    translation scratch, so a job's charge is exactly its A and B."""
    fmt, K, L = "tucker3d", (8, 8, 8), 3
    n = tuple(2 * k for k in K)
    ndir = (L + 1) * 2 * (L + 1)
    rk, data, _ = random_factors(fmt, n, ndir, np.random.default_rng(5))
    nrhs = 4
    jobs = [torch.from_numpy(synth.gaussian_patterns((nrhs, ndir) + K, 300 + j)).cuda() for j in range(6)]
    io = 2 * jobs[0].numel() * 8
    # solo results and the memory the operator takes, in a context with the default budget
    with P.Context(0) as big:
        op = big.import_factors(K, L, fmt, rk, data)
        assert op.plan()["fused"] and op.info()["bytes_scratch"] == 0
        u0, _ = big.memory()
        solo = []
        for A in jobs:
            B = torch.zeros_like(A)
            big.translate(op, A, B)
            solo.append(B)
        torch.cuda.synchronize()
        op.release()
    with P.Context(0, budget_bytes=u0 + int(1.5 * io)) as ctx:
        op = ctx.import_factors(K, L, fmt, rk, data)
        outs = [torch.zeros_like(A) for A in jobs]
        torch.cuda.synchronize()
        tickets = [ctx.submit(op, A, B) for A, B in zip(jobs, outs)]
        # a job four times as large can never fit next to the operator
        Abig = torch.cat([jobs[0]] * 4)
        tbig = ctx.submit(op, Abig, torch.zeros_like(Abig))
        tafter = ctx.submit(op, jobs[1], torch.zeros_like(jobs[1]))
        for t in tickets:
            st, lat = ctx.wait(t)
            assert st == 0 and lat > 0
        st_big, _ = ctx.wait(tbig)
        st_after, _ = ctx.wait(tafter)
        stats = ctx.sched_stats()
        assert (st_big, st_after) == (3, 0), (st_big, st_after, stats)
        assert stats["memory_waits"] >= 1 and stats["failed"] == 1 and stats["done"] == 7, stats
        used, budget = ctx.memory()
        assert used <= budget
        for j, (B, R) in enumerate(zip(outs, solo)):
            assert torch.equal(B, R), f"parked job {j} differs from its solo run"
        op.release()
