"""GPU checks of the batched solver and of hipGraph replay.

Batch: every problem must follow exactly the algorithm of a single solve
(same stop test, same cycle count, iterates within 1e-12 of the FP64 oracle
run on that problem alone), whatever the other problems in the batch do.
Graph replay must give the same bits as eager launches, on every replay.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1208_4247_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_4247_amd import capi

    capi.lib()
    oracle.build()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def levels_of(m):
    return int(np.log2(m + 1))


def run_batch(problems, rhs, flags=0, rtol=1e-10, maxit=60):
    from paper_1208_4247_amd.solver import BatchPlan

    plan = BatchPlan([(d, levels_of(m)) for d, m in problems], flags=flags)
    fs = [dev(f) for f in rhs]
    us = [torch.zeros_like(f) for f in fs]
    s, its, rels, sts = plan.solve(us, fs, rtol=rtol, maxit=maxit)
    return plan, [host(u) for u in us], its, rels, sts


SMALL = [(2, 3), (3, 7), (2, 63), (3, 31), (2, 255), (3, 15), (2, 127), (3, 63), (2, 63), (3, 31),
         (2, 1023), (3, 127)]


def test_batch_matches_single_oracle_solves():
    rhs = [wl.batch_rhs(11, q, d, m) for q, (d, m) in enumerate(SMALL)]
    _, us, its, rels, sts = run_batch(SMALL, rhs)
    for q, (d, m) in enumerate(SMALL):
        u_ref, it_ref, rel_ref, st_ref, _ = oracle.solve(rhs[q], rtol=1e-10)
        assert (sts[q], its[q]) == (st_ref, it_ref), (q, d, m, its[q], it_ref)
        assert rel2(us[q], u_ref) <= 1e-12, (q, d, m)
        assert rels[q] <= 1e-10


@pytest.mark.parametrize("post_forward", [False, True])
def test_batch_equals_single_plans_bitwise(post_forward):
    """A batch runs every level through table-driven launches shared by all
    its problems, a single-problem plan through launches of its own (tiles
    tuned per plan): every half-sweep is the same per-point expression, so
    both give the same cycle count and the same bits."""
    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import Plan

    probs = [(3, 63), (2, 255), (3, 31), (3, 127), (2, 511)]
    flags = capi.GMG_POST_FORWARD if post_forward else 0
    rhs = [wl.batch_rhs(17, q, d, m) for q, (d, m) in enumerate(probs)]
    _, us, its, _, sts = run_batch(probs, rhs, flags=flags)
    for q, (d, m) in enumerate(probs):
        plan = Plan(d, levels_of(m), flags=flags)
        ud = torch.zeros((m,) * d, dtype=torch.float64, device="cuda")
        st, it, _ = plan.solve(ud, dev(rhs[q]), rtol=1e-10)
        assert (sts[q], its[q]) == (st, it), (q, d, m)
        assert np.array_equal(us[q], host(ud)), (q, d, m)
        plan.close()


@pytest.mark.parametrize("smoother,nu1,nu2", [("wj", 2, 2), ("rbgs", 1, 1), ("rbgs", 1, 2),
                                              ("rbgs", 3, 3)])
def test_batch_smoothers_and_sweep_counts(smoother, nu1, nu2):
    """Weighted Jacobi and other sweep counts through the batch's tables
    and its two concurrent branches: every problem gives the bits and cycle
    count of its own single-problem plan (for V(1,1) that plan runs the
    cross-cycle schedule), and one problem of each dimension those of the
    oracle's solve to 1e-12."""
    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import BatchPlan, Plan

    probs = [(3, 31), (2, 127), (3, 63), (2, 255)]
    rhs = [wl.batch_rhs(23, q, d, m) for q, (d, m) in enumerate(probs)]
    plan = BatchPlan([(d, levels_of(m)) for d, m in probs], smoother=smoother, nu1=nu1, nu2=nu2,
                     flags=capi.GMG_USE_GRAPH)
    fs = [dev(f) for f in rhs]
    us = [torch.zeros_like(f) for f in fs]
    s, its, rels, sts = plan.solve(us, fs, rtol=1e-10, maxit=80)
    for q, (d, m) in enumerate(probs):
        single = Plan(d, levels_of(m), smoother=smoother, nu1=nu1, nu2=nu2)
        ud = torch.zeros_like(fs[q])
        st, it, _ = single.solve(ud, fs[q], rtol=1e-10, maxit=80)
        assert (sts[q], its[q]) == (st, it) == (0, it), (q, d, m)
        assert np.array_equal(host(us[q]), host(ud)), (q, d, m)
        single.close()
    wj = smoother == "wj"
    for q in (0, 1):
        d = probs[q][0]
        u_ref, it_ref, _, st_ref, _ = oracle.solve(
            rhs[q], nu1=nu1, nu2=nu2, smoother=oracle.WJ if wj else oracle.RBGS,
            omega=(6.0 / 7.0 if d == 3 else 0.8), rtol=1e-10, maxit=80)
        assert (sts[q], its[q]) == (st_ref, it_ref), (q, its[q], it_ref)
        assert rel2(host(us[q]), u_ref) <= 1e-12


def test_batch_per_problem_stop_tests():
    """A zero RHS stops at once, an easy RHS early, the rest later; the
    batch result of each equals its own solve."""
    probs = [(2, 127), (3, 31), (2, 127), (3, 63)]
    rhs = [np.zeros((127, 127)), wl.rhs_sine(3, 31), wl.batch_rhs(12, 2, 2, 127),
           wl.batch_rhs(12, 3, 3, 63)]
    _, us, its, rels, sts = run_batch(probs, rhs)
    assert its[0] == 0 and sts[0] == 0 and np.all(us[0] == 0)
    for q in range(1, 4):
        u_ref, it_ref, *_ = oracle.solve(rhs[q], rtol=1e-10)
        assert its[q] == it_ref
        assert rel2(us[q], u_ref) <= 1e-12


def test_batch_graph_replay_bitwise():
    from paper_1208_4247_amd import capi

    probs = SMALL[:8]
    rhs = [wl.batch_rhs(13, q, d, m) for q, (d, m) in enumerate(probs)]
    _, us_e, its_e, _, _ = run_batch(probs, rhs)
    plan, us_g, its_g, _, _ = run_batch(probs, rhs, flags=capi.GMG_USE_GRAPH)
    assert its_e == its_g
    for a, b in zip(us_e, us_g):
        assert np.array_equal(a, b)
    # replay the captured graph again, with eager work in between
    fs = [dev(f) for f in rhs]
    for rep in range(3):
        us = [torch.zeros_like(f) for f in fs]
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
        s, its, rels, sts = plan.solve(us, fs, rtol=1e-10)
        assert its == its_e
        for a, b in zip(us, us_e):
            assert np.array_equal(host(a), b)


@pytest.mark.parametrize("graph", [False, True])
def test_batch_two_branches_equal_one_stream(graph):
    """A batch of 2D and 3D problems runs them as two concurrent branches
    (the 2D launches on a side stream); with GMG_BATCH_ONE_STREAM every
    launch runs in order on one stream.  Same launches, so the same bits and
    cycle counts, on every replay of a captured cycle."""
    from paper_1208_4247_amd import capi

    probs = SMALL
    rhs = [wl.batch_rhs(19, q, d, m) for q, (d, m) in enumerate(probs)]
    g = capi.GMG_USE_GRAPH if graph else 0
    _, us_1, its_1, rels_1, _ = run_batch(probs, rhs, flags=g | capi.GMG_BATCH_ONE_STREAM)
    plan, us_2, its_2, rels_2, _ = run_batch(probs, rhs, flags=g)
    assert its_1 == its_2 and rels_1 == rels_2
    for a, b in zip(us_1, us_2):
        assert np.array_equal(a, b)
    fs = [dev(f) for f in rhs]
    for rep in range(2):
        us = [torch.zeros_like(f) for f in fs]
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
        s, its, rels, sts = plan.solve(us, fs, rtol=1e-10)
        assert its == its_1
        for a, b in zip(us, us_1):
            assert np.array_equal(host(a), b)


def test_single_problem_graph_replay_bitwise():
    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import Plan

    f = dev(wl.rhs_uniform(3, 127, seed=14))
    ref = None
    for flags in (0, capi.GMG_USE_GRAPH):
        plan = Plan(3, 7, flags=flags)
        for rep in range(3):
            u = torch.zeros_like(f)
            st, it, rel = plan.solve(u, f, rtol=1e-10)
            _ = torch.ones(10, device="cuda").sum().item()
            got = host(u)
            if ref is None:
                ref = (it, got)
            assert it == ref[0] and np.array_equal(got, ref[1])
    # the graph also serves gmg_vcycle (ungated variant)
    plan = Plan(3, 7, flags=capi.GMG_USE_GRAPH)
    u0 = wl.rhs_uniform(3, 127, seed=15) * 1e-3
    ud = dev(u0)
    plan.vcycle(ud, f)
    want = oracle.vcycle(u0, host(f))
    assert float(np.max(np.abs(host(ud) - want))) <= 1e-12 * float(np.max(np.abs(want)))


def test_batch_uneven_256_problems():
    """The uneven batch: 128 2D problems with side 2^k-1, k in 6..10 and 128
    3D problems with k in 5..7, U[-1,1] right-hand sides.  Every problem
    converges to 1e-10 on its own stop test; a sample spanning every size is
    compared with the oracle (same cycle count, iterates to 1e-12)."""
    probs = wl.batch_problems(4)
    rhs = [wl.batch_rhs(4, q, d, m) for q, (d, m) in enumerate(probs)]
    _, us, its, rels, sts = run_batch(probs, rhs)
    assert all(s == 0 for s in sts)
    assert max(rels) <= 1e-10
    seen = {}
    for q, (d, m) in enumerate(probs):
        seen.setdefault((d, m), q)
    for (d, m), q in sorted(seen.items()):
        u_ref, it_ref, *_ = oracle.solve(rhs[q], rtol=1e-10)
        assert its[q] == it_ref, (q, d, m)
        assert rel2(us[q], u_ref) <= 1e-12, (q, d, m)


def test_batch_autotuned_matches_oracle_and_replays():
    """With the autotuner the first batch solve tunes one problem of each
    shape and rebuilds the launch tables; results still follow each
    problem's own algorithm, and the graph replays give the same bits."""
    from paper_1208_4247_amd import capi

    probs = SMALL[:10]
    rhs = [wl.batch_rhs(17, q, d, m) for q, (d, m) in enumerate(probs)]
    plan, us, its, rels, sts = run_batch(probs, rhs, flags=capi.GMG_AUTOTUNE | capi.GMG_USE_GRAPH)
    for q, (d, m) in enumerate(probs):
        u_ref, it_ref, *_ = oracle.solve(rhs[q], rtol=1e-10)
        assert its[q] == it_ref, (q, d, m)
        assert rel2(us[q], u_ref) <= 1e-12, (q, d, m)
    fs = [dev(f) for f in rhs]
    for rep in range(2):
        u2 = [torch.zeros_like(f) for f in fs]
        s, its2, rels2, sts2 = plan.solve(u2, fs, rtol=1e-10)
        assert its2 == its
        for a, b in zip(u2, us):
            assert np.array_equal(host(a), b)
