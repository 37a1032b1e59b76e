"""GPU tests of the serving loop (chainhull_server_*): every request's hull,
computed in a mix of requests that arrive while others run, equals the hull
of the same request alone (hull2d), and the small ones equal the oracle's;
admission follows the memory budget.  Each case prints its name before its
GPU calls."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1508_05488_amd as ch  # noqa: E402
from oracle import hull as oracle  # noqa: E402
from paper_1508_05488_amd import workloads as wl  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def request_mix(count, seed, hi=3_000_000):
    rng = np.random.default_rng(seed)
    names = ("square", "disk", "gaussian", "adversarial")
    out = []
    for k in range(count):
        n = int(np.exp(rng.uniform(np.log(1_000), np.log(hi))))
        d = names[k % 4]
        out.append(wl.generate(d, n, seed * 1000 + k))
    # tiny and degenerate requests
    out.append(np.zeros((0, 2), np.float32))
    out.append(np.array([[5, 5]], np.float32))
    out.append(np.full((300, 2), 77, np.float32))
    out.append(np.stack([np.arange(500) % 31, np.arange(500) % 31], 1).astype(np.float32))
    return out


def test_mix_equals_alone():
    reqs = request_mix(40, seed=21)
    dev = [torch.from_numpy(p).cuda() for p in reqs]
    say(f"  server: {len(reqs)} requests, {sum(p.shape[0] for p in reqs)} points")
    alone = [ch.hull2d(p).cpu().numpy() for p in dev]
    with ch.Server(workers=4) as srv:
        tickets = []
        for k, p in enumerate(dev):
            tickets.append(srv.submit(p))
            if k % 7 == 3:
                time.sleep(0.0005)  # arrivals spread over the run
        got = [srv.wait(t) for t in tickets]
        st = srv.stats()
    say(f"  server stats {st}")
    assert st["completed"] == len(reqs)
    assert st["batched_requests"] > 0 and st["single_requests"] > 0
    for k, ((h, ms), a) in enumerate(zip(got, alone)):
        assert ms >= 0.0
        assert np.array_equal(h.cpu().numpy(), a), f"request {k} (n={reqs[k].shape[0]}) differs from hull2d alone"
        if reqs[k].shape[0] <= 200_000:
            assert np.array_equal(a, oracle.hull(reqs[k])), f"request {k} differs from the oracle"


def test_budget_admits_one_at_a_time():
    reqs = [wl.generate("disk", 600_000 + 10_000 * k, 31 + k) for k in range(5)]
    dev = [torch.from_numpy(p).cuda() for p in reqs]
    need = max(ch.workspace_bytes(p.shape[0]) for p in reqs)
    say("  server: budget for one request")
    with ch.Server(workers=4, mem_budget=need) as srv:
        tickets = [srv.submit(p) for p in dev]
        got = [srv.wait(t)[0].cpu().numpy() for t in tickets]
        st = srv.stats()
    assert st["max_inflight"] == 1
    for p, g in zip(dev, got):
        assert np.array_equal(g, ch.hull2d(p).cpu().numpy())


def test_request_beyond_budget_is_refused():
    p = torch.from_numpy(wl.generate("square", 400_000, 41)).cuda()
    say("  server: request beyond the budget")
    with ch.Server(workers=1, mem_budget=1 << 20) as srv:
        with pytest.raises(ch.ChainHullError) as e:
            srv.submit(p)
        assert e.value.status == ch.CH_EADMIT
        small = torch.from_numpy(wl.generate("square", 10_000, 42)).cuda()
        h, _ = srv.wait(srv.submit(small))
        assert np.array_equal(h.cpu().numpy(), oracle.hull(small.cpu().numpy()))


def test_domain_error_stays_in_its_request():
    good = [wl.generate("gaussian", 20_000, 51 + k) for k in range(3)]
    bad = wl.generate("square", 20_000, 55)
    bad[123, 0] = np.nan
    big_bad = wl.generate("disk", 400_000, 56)
    big_bad[7, 1] = 1 << 23
    say("  server: domain errors in one small and one large request")
    with ch.Server(workers=2) as srv:
        t_good = [srv.submit(torch.from_numpy(p).cuda()) for p in good]
        t_bad = srv.submit(torch.from_numpy(bad).cuda())
        t_big = srv.submit(torch.from_numpy(big_bad).cuda())
        for p, t in zip(good, t_good):
            assert np.array_equal(srv.wait(t)[0].cpu().numpy(), oracle.hull(p))
        outs = {}
        for t in (t_bad, t_big):
            outs[t] = srv._live[t][2]
            with pytest.raises(ch.ChainHullError) as e:
                srv.wait(t)
            assert e.value.status == ch.CH_EDOMAIN
    # a failed request's count is 0 whichever path served it, as hull2d
    # leaves it
    torch.cuda.synchronize()
    for t, cnt in outs.items():
        assert int(cnt.item()) == 0, t


def test_server_memory_stays_within_budget():
    # large requests (each alone on a worker's stream, with its own
    # workspace) on four workers under a budget of about two workspaces: the
    # memory the workers keep between requests counts against the budget
    n = 1_000_000
    reqs = [torch.from_numpy(wl.generate(("square", "disk")[k % 2], n, 91 + k)).cuda() for k in range(12)]
    outs = [(torch.empty(n, dtype=torch.int32, device="cuda"), torch.zeros(1, dtype=torch.int32, device="cuda"))
            for _ in reqs]
    alone = [ch.hull2d(p).cpu().numpy() for p in reqs]
    ch.release()  # no workspace of this process's own calls stays behind
    budget = int(2.5 * ch.workspace_bytes(n))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    say(f"  server: 12 requests of {n} points, budget {budget >> 20} MiB")
    low = free0
    with ch.Server(workers=4, mem_budget=budget) as srv:
        tickets = [srv.submit(p, o, c) for p, (o, c) in zip(reqs, outs)]
        got = []
        for t in tickets:
            got.append(srv.wait(t)[0].cpu().numpy())
            low = min(low, torch.cuda.mem_get_info()[0])
    used = free0 - low
    say(f"  server: most device memory in use {used >> 20} MiB")
    assert used <= budget + (64 << 20), (used, budget)
    for g, a in zip(got, alone):
        assert np.array_equal(g, a)


def test_poisson_arrivals():
    reqs = request_mix(60, seed=61, hi=1_000_000)
    dev = [torch.from_numpy(p).cuda() for p in reqs]
    alone = [ch.hull2d(p).cpu().numpy() for p in dev]
    rng = np.random.default_rng(62)
    gaps = rng.exponential(1.0 / 5000.0, size=len(dev))
    say(f"  server: {len(dev)} Poisson arrivals at 5000/s")
    with ch.Server(workers=4) as srv:
        tickets = []
        t0 = time.perf_counter()
        due = t0
        for p, g in zip(dev, gaps):
            due += g
            while time.perf_counter() < due:
                pass
            tickets.append(srv.submit(p))
        res = [srv.wait(t) for t in tickets]
    lat = np.array([ms for _, ms in res])
    assert np.all(lat > 0)
    for (h, _), a in zip(res, alone):
        assert np.array_equal(h.cpu().numpy(), a)
