"""Batched form on the GPU: every member of a batch must match its own
single-problem solve and the oracle; the captured graph must re-read values
on every replay; the autotuner's plan must be valid and cacheable."""

import json

import numpy as np
import pytest

import gen
import oracle
from gen.problems import rgg_one, rgg_sizes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_02995_amd import api

    c = api.Context(0)
    yield c
    c.close()


def _small_members(k=6, seed_offset=0):
    sizes = rgg_sizes()
    idx = [int(i) for i in np.argsort(sizes)[seed_offset:seed_offset + k]]
    return [rgg_one(b, sizes[b]) for b in idx]


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_single_and_oracle(ctx, precision):
    from paper_2208_02995_amd import api

    inps = _small_members(6)
    probs = [api.Problem.from_input(ctx, p, precision=precision) for p in inps]
    print(f"[batch] {precision} sizes={[p.n for p in inps]}", flush=True)
    batch = api.Batch(ctx, probs)
    plan = json.loads(batch.plan())
    assert plan["chosen"] in [c["plan"] for c in plan["candidates"]]
    outs, status, stats = batch.solve()
    for p, inp, out, st in zip(probs, inps, outs, stats):
        single = p.solve()[0][: p.nnz].cpu().numpy()
        got = out[: p.nnz].cpu().numpy()
        st_o, res = oracle.solve(inp)
        assert st.iterations == res.iterations == inp.maxit
        if precision == "fp64":
            assert _rel(got, single) < 1e-12
            assert _rel(got, res.P) < 1e-10
            dE = np.array(res.dE)
            assert abs(st.dE_first - dE[0]) < 1e-9 * dE[0]
        else:
            assert _rel(got, res.P) < 1e-4
            E = oracle.energy(inp.A, st_o.rowptr, st_o.colind, got, inp.nc)
            E_o = oracle.energy(inp.A, st_o.rowptr, st_o.colind, res.P, inp.nc)
            assert abs(E - E_o) <= 1e-6 * E_o
        from oracle import rcg as orc
        assert orc.constraint_error(st_o.rowptr, st_o.colind, got, inp.B, inp.Bc) < 1e-12
    batch.close()
    for p in probs:
        p.close()


def test_batch_replay_rereads_values(ctx):
    """Change one member's A values between replays: the batched result must
    follow (the graph gathers values at every launch)."""
    import torch

    from paper_2208_02995_amd import api

    inps = _small_members(4, seed_offset=10)
    probs = [api.Problem.from_input(ctx, p) for p in inps]
    batch = api.Batch(ctx, probs)
    o1 = [t[: p.nnz].cpu().numpy().copy() for t, p in zip(batch.solve()[0], probs)]
    o1b = [t[: p.nnz].cpu().numpy().copy() for t, p in zip(batch.solve()[0], probs)]
    for a, b in zip(o1, o1b):
        assert np.array_equal(a, b)  # replay is deterministic
    # new values for member 2: A + 0.5 I (same structure)
    inp = inps[2]
    A2 = inp.A.copy()
    d = np.array([A2.indptr[i] + list(A2.indices[A2.indptr[i]:A2.indptr[i + 1]]).index(i)
                  for i in range(inp.n)])
    A2.data[d] += 0.5
    probs[2].A.vals.copy_(torch.tensor(A2.data, device="cuda"))
    o2 = [t[: p.nnz].cpu().numpy().copy() for t, p in zip(batch.solve()[0], probs)]
    inp.A = A2
    _, res = oracle.solve(inp)
    assert _rel(o2[2], res.P) < 1e-10
    assert np.array_equal(o2[0], o1[0])
    batch.close()
    for p in probs:
        p.close()


def test_batch_tune_cache(ctx, tmp_path):
    from paper_2208_02995_amd import api

    inps = _small_members(3, seed_offset=20)
    probs = [api.Problem.from_input(ctx, p) for p in inps]
    cache = str(tmp_path / "tune.txt")
    b1 = api.Batch(ctx, probs, tune_cache=cache)
    p1 = json.loads(b1.plan())
    assert not p1["from_cache"]
    b2 = api.Batch(ctx, probs, tune_cache=cache)
    p2 = json.loads(b2.plan())
    assert p2["from_cache"] and p2["chosen"] == p1["chosen"]
    r1 = [t[: p.nnz].cpu().numpy() for t, p in zip(b1.solve()[0], probs)]
    r2 = [t[: p.nnz].cpu().numpy() for t, p in zip(b2.solve()[0], probs)]
    for a, b in zip(r1, r2):
        assert _rel(a, b) < 1e-14
    b1.close()
    b2.close()
    for p in probs:
        p.close()


def test_batch_full_256_sampled(ctx):
    """The full 256-matrix workload in the configuration the benchmark times
    (mixed precision, 15 iterations, one graph): three sampled members are
    checked against the oracle; every member against the constraint."""
    from paper_2208_02995_amd import api

    inps = gen.rgg_batch(256)
    probs = [api.Problem.from_input(ctx, p, precision="mixed") for p in inps]
    print(f"[batch256] rows={sum(p.n for p in inps)}", flush=True)
    batch = api.Batch(ctx, probs)
    outs, status, stats = batch.solve()
    assert all(s.iterations == 15 for s in stats)
    for b in (0, 128, 255):
        inp = inps[b]
        st_o, res = oracle.solve(inp)
        got = outs[b][: probs[b].nnz].cpu().numpy()
        E = oracle.energy(inp.A, st_o.rowptr, st_o.colind, got, inp.nc)
        E_o = oracle.energy(inp.A, st_o.rowptr, st_o.colind, res.P, inp.nc)
        print(f"  member {b}: rel={_rel(got, res.P):.2e} dE/E={abs(E - E_o) / E_o:.2e}", flush=True)
        assert _rel(got, res.P) < 1e-4
        assert abs(E - E_o) <= 1e-6 * E_o
    for p, out in zip(probs, outs):
        assert p.constraint_error(out) < 1e-12
    batch.close()
    for p in probs:
        p.close()
