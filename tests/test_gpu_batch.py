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


def test_batch_every_plan(ctx, tmp_path):
    """Every candidate bucket plan of the autotuner, forced through the tune
    cache, against the oracle (FP64): each plan's kernels, not only the one
    the timing picks, meet the bar."""
    from paper_2208_02995_amd import api

    inps = _small_members(6)
    refs = [oracle.solve(inp)[1] for inp in inps]
    probs = [api.Problem.from_input(ctx, p, precision="fp64") for p in inps]
    b0 = api.Batch(ctx, probs)
    plan = json.loads(b0.plan())
    b0.close()
    names = [c["plan"] for c in plan["candidates"]]
    assert "wide-one" in names and "wide-one-rest1" in names
    for name in names:
        cache = tmp_path / f"{name}.txt"
        cache.write_text(f"{plan['signature']} {name}\n")
        print(f"[plan] {name}", flush=True)
        b = api.Batch(ctx, probs, tune_cache=str(cache))
        forced = json.loads(b.plan())
        assert forced["from_cache"] and forced["chosen"] == name
        outs, status, stats = b.solve()
        for p, out, res in zip(probs, outs, refs):
            assert _rel(out[: p.nnz].cpu().numpy(), res.P) < 1e-10, name
        b.close()
    for p in probs:
        p.close()


@pytest.mark.timeout(900)
def test_batch_full_256(ctx):
    """The full 256-matrix workload in the configuration the benchmark times
    (mixed precision, 15 iterations, one graph): every member element by
    element against the oracle (computed in worker processes) and against the
    constraint."""
    from paper_2208_02995_amd import api
    from tests import oracle_pool

    inps = gen.rgg_batch(256)
    print(f"[batch256] rows={sum(p.n for p in inps)}; oracle in "
          f"{oracle_pool.workers()} processes", flush=True)
    ref = oracle_pool.rgg_members(range(256))
    probs = [api.Problem.from_input(ctx, p, precision="mixed") for p in inps]
    batch = api.Batch(ctx, probs)
    outs, status, stats = batch.solve()
    assert all(s.iterations == 15 for s in stats)
    worst_rel, worst_dE = 0.0, 0.0
    for b, inp in enumerate(inps):
        P_o, it_o, _, _, E_o = ref[b]
        assert it_o == 15
        got = outs[b][: probs[b].nnz].cpu().numpy()
        rel = _rel(got, P_o)
        E = oracle.energy(inp.A, *oracle.pattern_expand(inp.A, inp.P0, 1), got, inp.nc)
        dE = abs(E - E_o) / E_o
        worst_rel, worst_dE = max(worst_rel, rel), max(worst_dE, dE)
        assert rel < 1e-4, f"member {b}: rel {rel:.2e}"
        assert dE <= 1e-6, f"member {b}: energy {dE:.2e}"
        assert probs[b].constraint_error(outs[b]) < 1e-12
    print(f"  worst rel={worst_rel:.2e} worst dE/E={worst_dE:.2e}", flush=True)
    batch.close()
    for p in probs:
        p.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_tau_stop(ctx, precision):
    """Energy-monitor stop inside the captured graph (Sec. 3.3, eq. relRed):
    every member stops on its own when its dE_k falls below tau dE_1, the
    update of that iteration is skipped, and the other members go on.  Each
    member against the oracle's tau stop."""
    from paper_2208_02995_amd import api, emin

    inps = _small_members(8, seed_offset=30)
    # a tau no member's ratio dE_k / dE_1 comes within 2 % of, that makes the
    # members stop at different iterations
    full = [oracle.solve(p)[1] for p in inps]
    ratios = [np.array(r.dE) / r.dE[0] for r in full]
    tau = None
    for cand in np.geomspace(0.5, 1e-3, 60):
        if all(np.min(np.abs(np.log(q / cand))) > 0.02 for q in ratios):
            stops = {int(np.argmax(q < cand)) if np.any(q < cand) else 99 for q in ratios}
            if len(stops) >= 2 and 99 not in stops:
                tau = float(cand)
                break
    assert tau is not None
    probs = [api.Problem.from_input(ctx, p, precision=precision, tau=tau) for p in inps]
    batch = api.Batch(ctx, probs)
    outs, status, stats = batch.solve()
    its = []
    for p, inp, out, st in zip(probs, inps, outs, stats):
        st_o, res = oracle.solve(inp, tau=tau)
        assert res.status == "tau"
        assert st.stop == emin.EMIN_STOP_TAU
        assert st.iterations == res.iterations
        its.append(st.iterations)
        got = out[: p.nnz].cpu().numpy()
        assert _rel(got, res.P) < (1e-10 if precision == "fp64" else 1e-4)
    print(f"  tau={tau:.4g} stop iterations {its}", flush=True)
    assert len(set(its)) >= 2
    batch.close()
    for p in probs:
        p.close()


def test_batch_rank_counts_per_member(ctx):
    """A member whose B_c is zero has no constraint direction on any row
    (rank(G_i) = 0 everywhere): the batch reports those rows on that member
    only, and the member still matches the oracle (its SVD branch)."""
    from paper_2208_02995_amd import api, emin

    inps = _small_members(4, seed_offset=40)
    inps[2].Bc = np.zeros_like(inps[2].Bc)
    probs = [api.Problem.from_input(ctx, p) for p in inps]
    batch = api.Batch(ctx, probs)
    outs, status, stats = batch.solve()
    assert status == emin.EMIN_WARN_RANK
    assert [s.rank_deficient_rows for s in stats] == [0, 0, inps[2].n, 0]
    st_o, res = oracle.solve(inps[2])
    assert int(np.sum(st_o.rank < 1)) == inps[2].n
    assert _rel(outs[2][: probs[2].nnz].cpu().numpy(), res.P) < 1e-10
    batch.close()
    for p in probs:
        p.close()
