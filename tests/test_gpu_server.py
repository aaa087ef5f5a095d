"""Continuous-batching server: every query's result in a concurrent mix
equals the same query made alone (bit for bit), and the rounds really mix
windows of several queries.  Also with a conditioned (child) model, whose
queries first sample the parent model."""
import numpy as np
import pytest

from gpu_common import require_gpu

pytestmark = pytest.mark.gpu

QUERIES = [  # (seed, x0, y0, w, h, level): uneven sizes, overlaps, repeats, two seeds
    (3, 0, 0, 64, 64, 0), (3, 40, -20, 96, 48, 0), (3, 0, 0, 64, 64, 0), (7, -1000003, 999983, 33, 70, 0),
    (3, 500, 500, 128, 17, 0), (3, 30, 10, 20, 20, 2), (7, -1000003, 999990, 64, 64, 0), (3, -64, 0, 64, 64, 0),
    (3, 1000, -3000, 160, 96, 0), (7, 5, 5, 9, 9, 0), (3, 47, -13, 31, 77, 1), (3, 600, 450, 64, 64, 0),
]


def context(td, wpath, ppath):
    c = td.Context(0).load_weights(wpath)
    if ppath:
        c.set_conditioning(td.Context(0).load_weights(ppath))
    return c


def run_alone(td, torch, wpath, ppath, q):
    with context(td, wpath, ppath) as c:
        C = c.info("channels")
        out = torch.empty((C, q[4], q[3]), device="cuda")
        c.sample_region_async(*q, out)
        torch.cuda.synchronize()
        return out.cpu().numpy()


@pytest.mark.parametrize("config,inflight,budget,parent", [("c1", 6, 64 << 30, None), ("c1", 2, 200 << 20, None),
                                                           ("c1t2", 12, 64 << 30, None), ("lg", 4, 64 << 30, None),
                                                           ("c1h", 6, 64 << 30, "cc"), ("lgh", 3, 64 << 30, "lgc"),
                                                           ("lgs", 5, 64 << 30, None)])
def test_mix_equals_alone(weights, config, inflight, budget, parent):
    require_gpu()
    import torch
    from paper_2512_08309_amd import td
    wpath = weights(config)
    ppath = weights(parent) if parent else None
    with td.Context(0) as c:
        c.load_weights(wpath)
        T = c.info("levels")
    queries = [q[:5] + (min(q[5], T - 1),) for q in QUERIES]
    alone = [run_alone(td, torch, wpath, ppath, q) for q in queries]
    with context(td, wpath, ppath) as c:
        C = c.info("channels")
        with td.Server(c, budget, inflight) as srv:
            outs, tickets = [], []
            # submit in two waves: the second arrives while the first is in flight
            for i, q in enumerate(queries):
                outs.append(torch.full((C, q[4], q[3]), float("nan"), device="cuda"))
                tickets.append(srv.submit(*q, outs[-1]))
                if i == 5:
                    srv.progress(3)
            done = {}
            for _ in range(100000):
                n = srv.progress(1)
                for t in tickets:
                    if t not in done:
                        ok, lat = srv.poll(t)
                        if ok:
                            done[t] = lat
                if len(done) == len(tickets):
                    break
            torch.cuda.synchronize()
            st = srv.stats()
        assert len(done) == len(queries) and n == 0
        assert st["completed"] == len(queries) and st["rounds"] > 0
        for q, o, a in zip(queries, outs, alone):
            assert np.array_equal(o.cpu().numpy(), a), q
        cs = c.cache_stats()
        # shared windows are evaluated once: fewer evaluations than the sum of cold cones
        from oracle import windows as wn
        H, S, T = c.info("window"), c.info("stride"), c.info("levels")
        cold = sum(wn.cone_window_count(q[1:5], q[5], T, H, S) for q in queries)
        assert cs["misses"] < cold
        print(config, "inflight", inflight, "rounds", st["rounds"], "windows", st["batched_windows"],
              "cold-sum", cold, "mean batch %.1f" % (st["batched_windows"] / st["rounds"]))


def test_failed_round_stops_the_server_and_drops_the_cache(weights):
    """A round that throws part-way (here the parent model is replaced while
    a child query is in flight, which the next admission rejects) leaves the
    server refusing further rounds; destroying it drops the child's cache,
    and the context then answers like a fresh one."""
    require_gpu()
    import torch
    from paper_2512_08309_amd import td
    with td.Context(0) as p, td.Context(0) as c:
        p.load_weights(weights("lgc"))
        c.load_weights(weights("lgh")).set_conditioning(p)
        C = c.info("channels")
        outs = [torch.empty((C, 40, 40), device="cuda") for _ in range(2)]
        srv = td.Server(c, 64 << 30, 4)
        try:
            srv.submit(5, 0, 0, 40, 40, 0, outs[0])
            assert srv.progress(1) == 1                      # 8 levels: still in flight
            srv.submit(5, 100, 0, 40, 40, 0, outs[1])
            p.load_weights(weights("lgc", seed=1))
            with pytest.raises(td.TDError) as e:
                srv.progress(1)
            assert e.value.status == td.TD_E_STATE, str(e.value)
            with pytest.raises(td.TDError) as e:
                srv.progress(1)
            assert e.value.status == td.TD_E_STATE and "earlier round" in str(e.value)
        finally:
            srv.close()
        assert c.cache_stats()["bytes_used"] == 0
        got = c.sample_region(5, 0, 0, 40, 40, 0)
    with td.Context(0) as p2, td.Context(0) as c2:
        p2.load_weights(weights("lgc", seed=1))
        c2.load_weights(weights("lgh")).set_conditioning(p2)
        want = c2.sample_region(5, 0, 0, 40, 40, 0)
    assert np.array_equal(got, want)
