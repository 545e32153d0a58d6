"""GPU tests of the optimiser and the serving loop through the C ABI.

An analysis in the server must give the same result alone and in any mix
(the noise of step n is keyed by (seed, n), reductions have fixed order), the
same result as the one-at-a-time reference runner, and its first ELBO and a
short trajectory must match the FP64 oracle.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2501_09308_amd import workloads as W
from paper_2501_09308_amd import xrdvi as X

from gpu_common import case, context, dev, rel_l2

pytestmark = pytest.mark.gpu


def wait_all(srv, tickets, timeout=120.0):
    out, t0 = {}, time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            rc, info, res = srv.poll(t)
            if rc != X.XRDVI_PENDING:
                out[t] = (rc, info, res)
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return out


def small_case(seed, N=2000, K=12, M=15, cutoff=8.0, n_true=2):
    prob, y = case("paper50", seed, N=N, K=K, M=M, n_true=n_true)
    prob.cutoff = cutoff
    return prob, y


def test_adam_step_matches_oracle():
    ctx = context()
    rng = np.random.default_rng(5)
    n = 1000
    th, m1, m2, g = (rng.normal(size=n) for _ in range(4))
    m2 = np.abs(m2)
    ref = [a.copy() for a in (th, m1, m2)]
    for t in (1, 2, 7):
        oracle.adam(*ref, g, t, lr=0.01)
    dth, dm1, dm2, dg = (dev(a) for a in (th, m1, m2, g))
    for t in (1, 2, 7):
        X.xrdvi_adam_step(ctx, dth, dm1, dm2, dg, t, lr=0.01)
    for a, r in zip((dth, dm1, dm2), ref):
        np.testing.assert_allclose(a.cpu().numpy(), r, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("cutoff", [0.0, 8.0])
def test_server_first_elbo_and_trajectory_match_oracle(cutoff):
    prob, y = small_case(301, cutoff=cutoff, N=1500, K=6, M=10)
    S, steps, seed = 4, 5, 1234
    srv = X.Server(max_slots=4, steps_per_launch=2, arena_bytes=1 << 28)
    t = srv.submit(prob, y, S, steps, seed, lr=0.01)
    rc, info, res = wait_all(srv, [t])[t]
    srv.close()
    assert rc == X.XRDVI_OK
    # oracle SVI loop with the same noise and optimiser
    loc, ls = W.init_params(prob.K, float((y - prob.bg).max()))
    m = [np.zeros((4, prob.K)) for _ in range(4)]
    trace = []
    for n in range(steps):
        eps = oracle.eps_philox(S, prob.K, seed, n)
        e, _, gl, gs = oracle.elbo(prob, y, loc, ls, eps)
        trace.append(e)
        oracle.adam(loc, m[0], m[1], gl, n + 1, lr=0.01)
        oracle.adam(ls, m[2], m[3], gs, n + 1, lr=0.01)
    np.testing.assert_allclose(res["trace"], trace, rtol=1e-6)
    np.testing.assert_allclose(res["loc"], loc, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(res["logscale"], ls, rtol=1e-6, atol=1e-6)


def _mix(seed0, n):
    cases = []
    for i in range(n):
        p, y = small_case(seed0 + i, N=1000 + 397 * i, K=5 + 3 * i, M=8 + i,
                          cutoff=(0.0 if i % 3 == 0 else 8.0))
        cases.append((p, y, 2 + (i % 3) * 3, 6 + i, 77 + i))
    return cases


def test_result_is_the_same_alone_and_in_the_mix():
    target = small_case(400, N=2500, K=14, M=12, cutoff=8.0)
    S, steps, seed = 8, 12, 99
    srv = X.Server(max_slots=8, steps_per_launch=3, arena_bytes=1 << 28)
    t = srv.submit(*target, S, steps, seed)
    alone = wait_all(srv, [t])[t]
    # the same request among others, admitted into a different slot
    others = [srv.submit(p, y, s, st, sd) for p, y, s, st, sd in _mix(410, 6)]
    t2 = srv.submit(*target, S, steps, seed)
    more = [srv.submit(p, y, s, st, sd) for p, y, s, st, sd in _mix(430, 3)]
    res = wait_all(srv, others + [t2] + more)
    srv.close()
    assert alone[0] == X.XRDVI_OK and res[t2][0] == X.XRDVI_OK
    assert all(r[0] == X.XRDVI_OK for r in res.values())
    for k in ("loc", "logscale", "trace"):
        assert np.array_equal(alone[2][k], res[t2][2][k]), k


def test_server_matches_plain_runner_and_graph_matches_direct():
    prob, y = small_case(500, N=3000, K=10, M=20, cutoff=8.0)
    dense, yd = small_case(501, N=1800, K=7, M=9, cutoff=0.0)
    S, steps, seed = 6, 9, 4242
    ctx = context()
    plain = X.xrdvi_plain_run(ctx, prob, y, S, steps, seed)
    plain_d = X.xrdvi_plain_run(ctx, dense, yd, S, steps, seed)
    outs = {}
    for graph in (True, False):
        srv = X.Server(max_slots=4, steps_per_launch=4, use_graph=graph,
                       arena_bytes=1 << 28)
        a = srv.submit(prob, y, S, steps, seed)
        b = srv.submit(dense, yd, S, steps, seed)
        r = wait_all(srv, [a, b])
        srv.close()
        outs[graph] = (r[a][2], r[b][2])
    for k in ("loc", "logscale", "trace"):
        assert np.array_equal(outs[True][0][k], outs[False][0][k])
        assert np.array_equal(outs[True][1][k], outs[False][1][k])
        np.testing.assert_allclose(outs[True][0][k], plain[k], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(outs[True][1][k], plain_d[k], rtol=1e-12, atol=1e-12)


def test_crowded_tiles_give_the_same_bits_served_and_alone():
    """More peaks reach each tile than the forward stages in LDS at once
    (K=256 x 80 peaks on a 40 deg grid: over 1024 peak centres inside a
    128-point tile), so some phases of each chunk take the global-memory
    path.  The batched and the single-analysis forwards must split the
    phases alike: the served result equals its one-at-a-time run bit for
    bit, symmetric and asymmetric."""
    ctx = context()
    prob, y = small_case(905, N=2000, K=256, M=80, cutoff=8.0)
    per_tile = np.histogram(prob.peak_pos, bins=np.append(
        prob.x[::128], prob.x[-1]))[0]
    assert per_tile.max() > 1024
    S, steps = 4, 4
    ref = {a: X.xrdvi_plain_run(ctx, prob, y, S, steps, 21 + a, asymmetric=a)
           for a in (False, True)}
    srv = X.Server(max_slots=4, steps_per_launch=2, arena_bytes=1 << 29)
    small, ys = small_case(906, N=1500, K=8, M=12, cutoff=8.0)
    tk = {a: srv.submit(prob, y, S, steps, 21 + a, asymmetric=a) for a in (False, True)}
    other = srv.submit(small, ys, 3, 5, 7)
    res = wait_all(srv, list(tk.values()) + [other])
    srv.close()
    for a, t in tk.items():
        assert res[t][0] == X.XRDVI_OK
        for k in ("loc", "logscale", "trace"):
            assert np.array_equal(res[t][2][k], ref[a][k]), (a, k)


def test_every_variant_class_comes_and_goes():
    """Analyses of all eight variants (dense or windowed, symmetric or
    asymmetric peaks, constant or sec-law width), with different step
    counts, pass through a three-slot server, so that the set of resident
    variants, and with it the launched kernels and the replayed graph,
    changes many times.  Each result equals its one-at-a-time run bit for
    bit."""
    ctx = context()
    prob, y = small_case(910, N=1400, K=6, M=10, cutoff=8.0)
    S = 3
    cases = []
    for i, (cut, asym, law) in enumerate(
            [(c, a, w) for w in (0, "sec") for a in (False, True)
             for c in (0.0, 8.0)]):
        p = W.Problem(x=prob.x, bg=prob.bg, peak_off=prob.peak_off,
                      peak_pos=prob.peak_pos, peak_int=prob.peak_int, cutoff=cut,
                      true_idx=prob.true_idx, phi_true=prob.phi_true)
        cases.append((p, dict(asymmetric=asym, width_law=law), 3 + 2 * i, 60 + i))
    refs = [X.xrdvi_plain_run(ctx, p, y, S, steps, seed, **kw)
            for p, kw, steps, seed in cases]
    srv = X.Server(max_slots=3, steps_per_launch=2, arena_bytes=1 << 28)
    tickets = [srv.submit(p, y, S, steps, seed, **kw) for p, kw, steps, seed in cases]
    res = wait_all(srv, tickets)
    srv.close()
    for t, ref, (_, kw, _, _) in zip(tickets, refs, cases):
        assert res[t][0] == X.XRDVI_OK
        for k in ("loc", "logscale", "trace"):
            assert np.array_equal(res[t][2][k], ref[k]), (kw, k)


def test_server_errors_and_cancel():
    prob, y = small_case(600, N=1200, K=6, M=8)
    srv = X.Server(max_slots=1, steps_per_launch=1, arena_bytes=1 << 26)
    # invalid request
    bad = W.Problem(x=prob.x[::-1].copy(), bg=prob.bg, peak_off=prob.peak_off,
                    peak_pos=prob.peak_pos, peak_int=prob.peak_int, cutoff=8.0,
                    true_idx=prob.true_idx, phi_true=prob.phi_true)
    with pytest.raises(X.XrdviError) as ei:
        srv.submit(bad, y, 4, 5, 1)
    assert ei.value.code == X.XRDVI_EINVAL
    # never fits a 64 MiB arena
    huge = W.make_problem("paper50", 601, N=12000, K=300, M=60, step=0.01)
    yh = huge.bg + 10.0
    with pytest.raises(X.XrdviError) as ei:
        srv.submit(huge, yh, 128, 5, 1)
    assert ei.value.code == X.XRDVI_ENOMEM
    # cancel a long-running request and a queued one
    run = srv.submit(prob, y, 4, 100000, 1)
    queued = srv.submit(prob, y, 4, 5, 2)
    time.sleep(0.2)
    srv.cancel(queued)
    srv.cancel(run)
    res = wait_all(srv, [run, queued])
    assert res[run][0] == X.XRDVI_ECANCELED and res[queued][0] == X.XRDVI_ECANCELED
    ok = srv.submit(prob, y, 4, 3, 3)
    assert wait_all(srv, [ok])[ok][0] == X.XRDVI_OK
    with pytest.raises(X.XrdviError):
        srv.poll(ok)
    srv.close()


def test_slot_reuse_by_analyses_of_other_shapes():
    """One slot, several queued analyses of different K, N and S: each is
    admitted into the slot its predecessor left, and must still match its
    one-at-a-time run (regression: the batched work prefix must follow the
    slot's new occupant)."""
    ctx = context()
    shapes = [(3000, 30, 10, 8), (1200, 6, 8, 2), (2200, 12, 15, 4),
              (900, 4, 5, 3)]
    cases = [(small_case(700 + i, N=N, K=K, M=M), S)
             for i, (N, K, M, S) in enumerate(shapes)]
    srv = X.Server(max_slots=1, steps_per_launch=2, arena_bytes=1 << 28)
    tickets = [srv.submit(p, y, S, 6, 50 + i) for i, ((p, y), S) in enumerate(cases)]
    res = wait_all(srv, tickets)
    srv.close()
    for i, ((p, y), S) in enumerate(cases):
        rc, info, out = res[tickets[i]]
        assert rc == X.XRDVI_OK
        ref = X.xrdvi_plain_run(ctx, p, y, S, 6, 50 + i)
        for k in ("loc", "logscale", "trace"):
            np.testing.assert_allclose(out[k], ref[k], rtol=1e-12, atol=1e-12)


def test_many_phase_windowed_analyses_in_the_server():
    """Windowed analyses with K >= 128 (their batched forward stages peak
    lists in LDS), symmetric and asymmetric, served beside small ones, must
    match their one-at-a-time runs."""
    ctx = context()
    big, yb = small_case(900, N=3000, K=160, M=25, cutoff=8.0)
    small, ys = small_case(901, N=1500, K=8, M=12, cutoff=8.0)
    S, steps = 4, 6
    ref = {
        "sym": X.xrdvi_plain_run(ctx, big, yb, S, steps, 11),
        "asym": X.xrdvi_plain_run(ctx, big, yb, S, steps, 12, asymmetric=True),
    }
    srv = X.Server(max_slots=6, steps_per_launch=2, arena_bytes=1 << 29)
    others = [srv.submit(small, ys, 3, 5, 40 + i) for i in range(3)]
    t_sym = srv.submit(big, yb, S, steps, 11)
    t_asym = srv.submit(big, yb, S, steps, 12, asymmetric=True)
    res = wait_all(srv, others + [t_sym, t_asym])
    srv.close()
    assert all(r[0] == X.XRDVI_OK for r in res.values())
    for name, t in (("sym", t_sym), ("asym", t_asym)):
        for k in ("loc", "logscale", "trace"):
            np.testing.assert_allclose(res[t][2][k], ref[name][k], rtol=1e-12,
                                       atol=1e-12)
