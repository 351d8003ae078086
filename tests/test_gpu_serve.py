"""The serving runtime (tnrg_server_*): continuous batching of requests with
different N, chi, M, K and R, admitted by workspace footprint.

  * every request of a 20-request mix gives the same F and gradient in the
    mix as alone (bit for bit when it ran in the same capacity bucket, else
    to 1e-10 relative);
  * an arena that holds two workspaces never runs more than two requests;
  * a request whose bonds outgrow its bucket is regrown inside the server,
    up to the server's largest admitted bucket;
  * a request too large for the arena fails alone with TNRG_ENOMEM;
  * queued requests can be cancelled.
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import workloads as W  # noqa: E402

from gpu_helpers import device_problem  # noqa: E402


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_03639_amd as P
    return P


def say(*a):
    print(*a, flush=True)


def small_mix(n, seed=7):
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        task = ("x", "cnot", "ghz")[i % 3]
        specs.append(dict(task=task, N=int(rng.choice([6, 8, 10])), M=int(rng.integers(12, 30)),
                          T=3.0, chi=int(rng.choice([4, 8, 16])), K=int(rng.choice([2, 4, 8])),
                          R=2 if task != "ghz" else 1, sigma=0.3, seed=100 + i))
    return specs


def make_request(P, spec, dcap=0):
    p = W.make_problem(**spec)
    d = device_problem(p)
    return P.serve.Request(d["model"], d["ux"], d["uy"], d["uzz"], d["J"], d["inputs"],
                           d["targets"], dcap=dcap)


def test_same_result_alone_and_in_the_mix(P):
    specs = small_mix(20)
    say(f"serving mix: {len(specs)} requests")
    alone = []
    for sp in specs:
        p = W.make_problem(**sp)
        d = device_problem(p)
        r = P.grape_fidelity_grad(d["model"], d["ux"], d["uy"], d["uzz"], d["J"], d["inputs"],
                                  d["targets"])
        alone.append(r)
    torch.cuda.synchronize()
    reqs = [make_request(P, sp) for sp in specs]
    with P.serve.Server(arena_bytes=1 << 30, n_streams=4) as srv:
        tickets = [srv.submit(q) for q in reqs]
        done = srv.drain()
        info = srv.info()
    assert info["completed"] == len(specs) and info["queued"] == 0 and info["running"] == 0
    by_ticket = {c["ticket"]: c for c in done}
    assert sorted(by_ticket) == sorted(tickets)
    bitwise = 0
    for t, q, a in zip(tickets, reqs, alone):
        c = by_ticket[t]
        assert c["status"] == 0, c
        same_bucket = c["dcap"] == a["dcap"]
        for nm in ("F", "g_ux", "g_uy", "g_uzz"):
            x, y = getattr(q, nm), a[nm]
            if same_bucket:
                assert torch.equal(x, y), (t, nm)
            else:
                scale = float(y.abs().max())
                assert float((x - y).abs().max()) <= 1e-10 * scale, (t, nm)
        bitwise += same_bucket
    say(f"  {bitwise} of {len(specs)} ran in the same bucket (bitwise equal)")


def test_admission_by_footprint(P):
    specs = [dict(task="cnot", N=8, M=20, T=3.0, chi=8, K=4, R=2, sigma=0.3, seed=200 + i)
             for i in range(6)]
    reqs = [make_request(P, sp, dcap=8) for sp in specs]
    need = reqs[0].workspace_bytes(8)
    say(f"admission: 6 requests of {need} workspace bytes, arena for 2")
    arena = 2 * ((need + 255) // 256 * 256) + 1024
    with P.serve.Server(arena_bytes=arena, n_streams=4) as srv:
        for q in reqs:
            srv.submit(q)
        done, peak = [], 0
        deadline = time.time() + 60
        while len(done) < len(reqs) and time.time() < deadline:
            done += srv.progress()
            peak = max(peak, srv.info()["running"])
        assert len(done) == len(reqs)
    assert 1 <= peak <= 2
    assert all(c["status"] == 0 for c in done)


def test_bucket_regrowth_in_the_server(P):
    # GHZ at N = 8 reaches bond dimension 16: buckets 4 and 8 overflow
    spec = dict(task="ghz", N=8, M=10, T=4.0, chi=16, K=2, R=1, sigma=0.5, seed=8)
    p = W.make_problem(**spec)
    d = device_problem(p)
    ref = P.grape_fidelity_grad(d["model"], d["ux"], d["uy"], d["uzz"], d["J"], d["inputs"],
                                d["targets"], dcap=16)
    q = make_request(P, spec)
    with P.serve.Server(arena_bytes=1 << 28, n_streams=2) as srv:
        srv.submit(q)
        done = srv.drain()
        info = srv.info()
    say(f"regrowth: {done[0]['launches']} launches, bucket {done[0]['dcap']}")
    assert done[0]["status"] == 0 and done[0]["dcap"] == 16
    assert done[0]["launches"] >= 2 and info["regrown"] >= 1
    assert torch.equal(q.F, ref["F"]) and torch.equal(q.g_ux, ref["g_ux"])
    # a server that admits buckets up to 8 refuses the same request
    q2 = make_request(P, dict(spec, seed=9))
    with P.serve.Server(arena_bytes=1 << 28, n_streams=1, max_dcap=8) as srv:
        srv.submit(q2)
        done = srv.drain()
    assert done[0]["status"] == P.tnrg.EUNSUPPORTED and done[0]["dcap"] <= 8


def test_too_large_and_cancel(P):
    big = make_request(P, dict(task="x", N=10, M=20, T=3.0, chi=8, K=8, R=2, sigma=0.3, seed=1),
                       dcap=8)
    small = [make_request(P, dict(task="x", N=6, M=10, T=3.0, chi=4, K=2, R=1, sigma=0.3,
                                  seed=2 + i), dcap=4) for i in range(5)]
    need_small = small[0].workspace_bytes(4)
    assert big.workspace_bytes(8) > 4 * need_small
    say("too large / cancel")
    with P.serve.Server(arena_bytes=2 * need_small + 4096, n_streams=1) as srv:
        tb = srv.submit(big)
        ts = [srv.submit(q) for q in small]
        done = srv.progress()
        # the big request fails at once; one small one runs, the rest wait
        assert any(c["ticket"] == tb and c["status"] == P.tnrg.ENOMEM for c in done)
        cancelled = srv.cancel_queued()
        done += srv.drain()
    assert len(cancelled) >= 1
    assert set(cancelled) | {c["ticket"] for c in done} == set(ts) | {tb}
    for c in done:
        if c["ticket"] != tb:
            assert c["status"] == 0
