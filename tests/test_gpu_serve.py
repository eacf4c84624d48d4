"""The request server on the GPU: every served request is bit-identical to a
direct call on the same inputs, whatever it was batched with, and one served
request is checked against the oracle."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_02640_amd import inputs as I

from . import parity as PM

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"
WAIT_S = 60.0


def _say(*a):
    print("[gpu-serve]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kx():
    from paper_2411_02640_amd import kx as K
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    K.lib()
    return K


@pytest.fixture(scope="module")
def mechs(kx, mech9, mech53):
    ms = {"syn9": (kx.Mechanism(mech9, 0), mech9), "syn53": (kx.Mechanism(mech53, 0), mech53)}
    yield ms
    for dm, _ in ms.values():
        dm.close()


def _inputs(ns, n, seed):
    spec = I.StateSpec(n_points=n, seed=seed, T_range=(300.0, 2800.0), p_atm_range=(1.0, 40.0),
                       dirichlet_alpha=0.3)
    T, p, Y = I.make_states(ns, spec)
    return [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (T, p, Y)], (T, p, Y)


def _direct(kx, dm, Td, pd, Yd, transport, precision):
    w = kx.production_rates(dm, Td, pd, Yd, precision=precision)
    tr = kx.transport(dm, Td, pd, Yd, precision=precision) if transport else (None,) * 3
    torch.cuda.synchronize()
    return (w,) + tuple(tr)


def _same(a, b):
    return (a is None and b is None) or torch.equal(a, b)


def _footprint(ns, n, transport):
    d = ns + ((ns + 2) if transport else 0)
    return (n * 8 * d + 255) // 256 * 256


def _resident(*dms):
    """Arena bytes the resident tables of these mechanisms take."""
    return sum((dm.device_bytes + 255) // 256 * 256 for dm in dms)


def test_served_equals_direct_mixed_batches(kx, mechs):
    """24 requests over two mechanisms, both precisions, both op sets and
    ragged sizes are queued behind a finished request that holds the arena;
    releasing it admits them all in one pass, so they run as a few mixed
    batches.  Each output must equal the direct call bit for bit."""
    rng = np.random.default_rng(11)
    cases = []
    sizes = [1, 63, 64, 65, 1000, 4097, 20000, 70001]
    for i in range(24):
        name = "syn9" if i % 3 == 0 else "syn53"
        n = int(sizes[i % len(sizes)])
        tr = bool(rng.integers(2))
        prec = "fp64" if rng.integers(2) else "mixed"
        dm, mech = mechs[name]
        (Td, pd, Yd), _ = _inputs(mech["n_species"], n, 100 + i)
        cases.append((name, n, tr, prec, Td, pd, Yd))
    ns53 = mechs["syn53"][1]["n_species"]
    total = sum(_footprint(mechs[c[0]][1]["n_species"], c[1], c[2]) for c in cases)
    first = _footprint(mechs[cases[0][0]][1]["n_species"], cases[0][1], cases[0][2])
    n_blk = -(-(total - first + 256) // (8 * ns53))
    budget = max(total, _footprint(ns53, n_blk, False))
    assert budget - _footprint(ns53, n_blk, False) < first
    (Tb, pb, Yb), _ = _inputs(ns53, n_blk, 99)
    res = _resident(mechs["syn9"][0], mechs["syn53"][0])
    srv = kx.Server(0, hbm_budget=budget + res, max_slots=64)
    try:
        srv.add_mech(mechs["syn9"][0])
        srv.add_mech(mechs["syn53"][0])
        assert srv.stats()["resident_bytes"] == res
        blocker = srv.submit(mechs["syn53"][0], Tb, pb, Yb)
        assert srv.wait(blocker, WAIT_S)["state"] == "done"
        reqs = [(srv.submit(mechs[c[0]][0], *c[4:], transport=c[2], precision=c[3]), c)
                for c in cases]
        assert srv.stats()["queued"] == len(cases)
        srv.release(blocker)
        for t, (name, n, tr, prec, Td, pd, Yd) in reqs:
            _say("request", t, name, "n =", n, "transport" if tr else "rates", prec)
            r = srv.wait(t, WAIT_S)
            assert r["state"] == "done", r
            got = srv.outputs(t)
            ref = _direct(kx, mechs[name][0], Td, pd, Yd, tr, prec)
            for g, e, what in zip(got, ref, ("wdot", "mu", "lambda", "Dmix")):
                assert _same(g, e), (name, n, prec, what)
            srv.release(t)
        st = srv.stats()
        _say(st)
        assert st["completed"] == len(cases) + 1 and st["failed"] == 0
        # one batch per (mechanism, precision) group after the blocker
        assert st["batches"] <= 1 + 4
        assert st["arena_in_use"] == res
    finally:
        srv.close()


def test_served_matches_oracle(kx, mechs):
    dm, mech = mechs["syn53"]
    (Td, pd, Yd), (T, p, Y) = _inputs(mech["n_species"], 3001, 7)
    srv = kx.Server(0, hbm_budget=256 << 20, max_slots=8)
    try:
        t = srv.submit(dm, Td, pd, Yd, transport=True)
        assert srv.wait(t, WAIT_S)["state"] == "done"
        w, mu, lam, Dm = [x.cpu().numpy() for x in srv.outputs(t)]
        srv.release(t)
    finally:
        srv.close()
    om = O.OracleMech(mech)
    ref, s = om.production_rates(T, p, Y)
    rep = PM.wdot_report(w, ref, s)
    _say(rep)
    assert rep["ok"], rep
    rmu, rlam, rDm = om.transport(T, p, Y)
    for name, g, r in (("mu", mu, rmu), ("lambda", lam, rlam), ("Dmix", Dm, rDm)):
        rep = PM.rel_report(g, r, PM.REL_FP64)
        assert rep["ok"], (name, rep)


def test_budget_pressure_and_cancel(kx, mechs):
    dm, mech = mechs["syn53"]
    ns, n = mech["n_species"], 30000
    fp = (n * 8 * ns + 255) // 256 * 256
    srv = kx.Server(0, hbm_budget=2 * fp + _resident(dm), max_slots=16)
    try:
        (Td, pd, Yd), _ = _inputs(ns, n, 21)
        ref = _direct(kx, dm, Td, pd, Yd, False, "fp64")[0]
        a = srv.submit(dm, Td, pd, Yd)
        b = srv.submit(dm, Td, pd, Yd)
        assert srv.wait(a, WAIT_S)["state"] == "done"
        assert srv.wait(b, WAIT_S)["state"] == "done"
        c = srv.submit(dm, Td, pd, Yd)            # arena full: stays queued
        d = srv.submit(dm, Td, pd, Yd)
        with pytest.raises(kx.KxError):
            srv.wait(c, 0.2)
        srv.cancel(c)
        assert srv.poll(c)["state"] == "cancelled"
        for t in (a, b):
            assert torch.equal(srv.outputs(t)[0], ref)
            srv.release(t)
        assert srv.wait(d, WAIT_S)["state"] == "done"
        assert torch.equal(srv.outputs(d)[0], ref)
        srv.release(d)
        srv.release(c)
        st = srv.stats()
        assert st["cancelled"] == 1 and st["completed"] == 3
        assert st["arena_in_use"] == _resident(dm)
    finally:
        srv.close()


def test_graph_replay_across_batches(kx, mechs):
    """Many batches of one group replay the same graph; every replay stays
    equal to the direct result."""
    dm, mech = mechs["syn9"]
    ns = mech["n_species"]
    srv = kx.Server(0, hbm_budget=512 << 20, max_slots=4)
    try:
        for rep in range(6):
            n = 5000 + 977 * rep
            (Td, pd, Yd), _ = _inputs(ns, n, 300 + rep)
            ts = [srv.submit(dm, Td, pd, Yd, transport=True) for _ in range(3)]
            ref = _direct(kx, dm, Td, pd, Yd, True, "fp64")
            for t in ts:
                assert srv.wait(t, WAIT_S)["state"] == "done"
                got = srv.outputs(t)
                for g, e in zip(got, ref):
                    assert torch.equal(g, e)
                srv.release(t)
        st = srv.stats()
        _say(st)
        assert st["graph_launches"] == st["batches"] >= 2
    finally:
        srv.close()


def test_host_staged_client(kx, mechs):
    """A client whose data live in pinned host memory: inputs are copied in at
    arrival and outputs copied back into pinned host buffers (kx_result_copy
    with host destinations).  Every host output equals the direct call bit for
    bit, and a pageable host buffer is refused."""
    from paper_2411_02640_amd import serve_load as SL
    devs = {name: dm for name, (dm, _) in mechs.items()}
    pools, hpools = {}, {}
    for k, (name, (dm, mech)) in enumerate(sorted(mechs.items())):
        pools[name] = SL.make_pool(dm, mech["n_species"], [1000 + 777 * i for i in range(3)],
                                   40 + k)
        hpools[name] = SL.make_host_pool(pools[name], mech["n_species"])
    stream = [(name, i, i % 2 == 0, "mixed" if i == 1 else "fp64")
              for name in sorted(hpools) for i in range(3)]
    _say("host-staged stream of", len(stream), "requests")
    srv = kx.Server(0, hbm_budget=1 << 30, max_slots=8)
    try:
        rec = SL.run_stream_staged(srv, devs, hpools, stream, None, 0)
        assert len(rec) == len(stream)
        assert all(r["t_host"] >= r["t_done"] for _, r in rec)
        dm, mech = mechs["syn9"]
        n, (hT, hp, hY), _ = hpools["syn9"][0]
        t = srv.submit(dm, hT.to(DEV), hp.to(DEV), hY.to(DEV))
        assert srv.wait(t, WAIT_S)["state"] == "done"
        with pytest.raises(ValueError):
            srv.copy_outputs(t, torch.empty((mech["n_species"], n), dtype=torch.float64))
        srv.release(t)
    finally:
        srv.close()
    for name, i, tr, prec in stream:
        n, (hT, hp, hY), (w, mu, lam, Dm) = hpools[name][i]
        ref = _direct(kx, devs[name], hT.to(DEV), hp.to(DEV), hY.to(DEV), tr, prec)
        assert torch.equal(w, ref[0].cpu()), (name, i)
        if tr:
            for got, want in zip((mu, lam, Dm), ref[1:]):
                assert torch.equal(got, want.cpu()), (name, i)


def test_served_large_mechanisms_equal_direct(kx, mech100, mech200):
    """The 100- and 200-species mechanisms served (two species per lane and four
    per lane in the rates batch kernel; the 32- and 16-point matrix-core
    transport tiles), both precisions, with a ragged size, in one mixed set of
    batches: every output equals the direct call bit for bit."""
    ms = {"syn100": (kx.Mechanism(mech100, 0), mech100),
          "syn200": (kx.Mechanism(mech200, 0), mech200)}
    srv = kx.Server(0, hbm_budget=4 << 30, max_slots=16)
    try:
        cases = []
        for i, (name, n, prec) in enumerate([("syn100", 7001, "fp64"), ("syn200", 3001, "fp64"),
                                             ("syn100", 129, "mixed"), ("syn200", 40003, "mixed"),
                                             ("syn200", 1, "fp64")]):
            dm, mech = ms[name]
            (Td, pd, Yd), _ = _inputs(mech["n_species"], n, 500 + i)
            cases.append((srv.submit(dm, Td, pd, Yd, transport=True, precision=prec),
                          name, n, prec, Td, pd, Yd))
        for t, name, n, prec, Td, pd, Yd in cases:
            _say("request", t, name, "n =", n, prec)
            r = srv.wait(t, WAIT_S)
            assert r["state"] == "done", r
            got = srv.outputs(t)
            ref = _direct(kx, ms[name][0], Td, pd, Yd, True, prec)
            for g, e, what in zip(got, ref, ("wdot", "mu", "lambda", "Dmix")):
                assert _same(g, e), (name, n, prec, what)
            srv.release(t)
    finally:
        srv.close()
        for dm, _ in ms.values():
            dm.close()


def test_served_other_fit_order_equals_direct(kx):
    """A mechanism with 4-coefficient transport fits (the batch and one-tile
    kernels' forms for any fit order) served in small batches (graph replay)
    and then in big ones (one workgroup per tile), both precisions: every
    output equals the direct call bit for bit."""
    import dataclasses
    mech = I.make_mechanism(dataclasses.replace(I.MECH_53, fit_order=4, name="syn53_fit4"))
    dm = kx.Mechanism(mech, 0)
    srv = kx.Server(0, hbm_budget=4 << 30, max_slots=16)
    try:
        for group in ([(3001, "fp64"), (129, "mixed")], [(150001, "fp64"), (140003, "mixed")]):
            cases = []
            for i, (n, prec) in enumerate(group):
                (Td, pd, Yd), _ = _inputs(53, n, 700 + n % 97 + i)
                cases.append((srv.submit(dm, Td, pd, Yd, transport=True, precision=prec),
                              n, prec, Td, pd, Yd))
            for t, n, prec, Td, pd, Yd in cases:
                _say("request", t, "syn53_fit4 n =", n, prec)
                r = srv.wait(t, WAIT_S)
                assert r["state"] == "done", r
                got = srv.outputs(t)
                ref = _direct(kx, dm, Td, pd, Yd, True, prec)
                for g, e, what in zip(got, ref, ("wdot", "mu", "lambda", "Dmix")):
                    assert _same(g, e), (n, prec, what)
                srv.release(t)
    finally:
        srv.close()
        dm.close()


def test_inputs_ready_event(kx, mechs):
    """A request whose inputs are still being written on another stream when it
    is submitted: the server waits for the event recorded after that work, and
    the outputs equal the direct call on the finished inputs."""
    dm, mech = mechs["syn53"]
    ns, n = mech["n_species"], 200_000
    (Td, pd, Yd), _ = _inputs(ns, n, 77)
    ref = _direct(kx, dm, Td, pd, Yd, True, "fp64")
    T2, p2, Y2 = torch.empty_like(Td), torch.empty_like(pd), torch.empty_like(Yd)
    side = torch.cuda.Stream()
    ready = torch.cuda.Event()
    srv = kx.Server(0, hbm_budget=1 << 30, max_slots=8)
    try:
        srv.add_mech(dm)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            # slow enough that the server would read unfinished inputs
            for _ in range(20):
                Y2.copy_(Yd)
            T2.copy_(Td)
            p2.copy_(pd)
            ready.record(side)
        t = srv.submit(dm, T2, p2, Y2, transport=True, inputs_ready=ready)
        assert srv.wait(t, WAIT_S)["state"] == "done"
        got = srv.outputs(t)
        for g, e in zip(got, ref):
            assert torch.equal(g, e)
        srv.release(t)
    finally:
        srv.close()


def test_big_batches_one_tile_kernels(kx, mechs):
    """Batches of 2^17 points or more run the one-workgroup-per-tile kernels
    (no graph).  Three requests per (mechanism, precision) group, 140 015 points
    in all, queued behind a request that holds the arena so that each group
    forms one batch: the 9-species mechanism (vector-ALU transport), a
    53-species mechanism with fits of D_kj (vector-ALU transport) and syn53
    (matrix-core transport), both precisions.  Every output equals the direct
    call bit for bit, and every group ran without its graph."""
    mdl = I.make_mechanism(I.MechSpec(53, 266, 30, 0, 29, seed=53325, diff_fit_kind=0,
                                      name="syn53d"))
    ms = {"syn9": mechs["syn9"], "syn53": mechs["syn53"], "syn53d": (kx.Mechanism(mdl, 0), mdl)}
    sizes = [70001, 50003, 20011]
    assert sum(sizes) >= 1 << 17
    cases = []
    for name in ms:
        for prec in ("fp64", "mixed"):
            for j, n in enumerate(sizes):
                (Td, pd, Yd), _ = _inputs(ms[name][1]["n_species"], n, 900 + 10 * len(cases) + j)
                cases.append((name, n, prec, Td, pd, Yd))
    ns53 = ms["syn53"][1]["n_species"]
    total = sum(_footprint(ms[c[0]][1]["n_species"], c[1], True) for c in cases)
    n_blk = -(-total // (8 * ns53))
    (Tb, pb, Yb), _ = _inputs(ns53, n_blk, 899)
    res = _resident(*(dm for dm, _ in ms.values()))
    budget = max(total, _footprint(ns53, n_blk, False)) + res
    srv = kx.Server(0, hbm_budget=budget, max_slots=64)
    try:
        for dm, _ in ms.values():
            srv.add_mech(dm)
        blocker = srv.submit(ms["syn53"][0], Tb, pb, Yb)
        assert srv.wait(blocker, WAIT_S)["state"] == "done"
        reqs = [(srv.submit(ms[c[0]][0], *c[3:], transport=True, precision=c[2]), c)
                for c in cases]
        assert srv.stats()["queued"] == len(cases)
        before = srv.stats()
        srv.release(blocker)
        for t, (name, n, prec, Td, pd, Yd) in reqs:
            _say("request", t, name, "n =", n, prec)
            r = srv.wait(t, WAIT_S)
            assert r["state"] == "done", r
            got = srv.outputs(t)
            ref = _direct(kx, ms[name][0], Td, pd, Yd, True, prec)
            for g, e, what in zip(got, ref, ("wdot", "mu", "lambda", "Dmix")):
                assert _same(g, e), (name, n, prec, what)
            srv.release(t)
        st = srv.stats()
        _say(st)
        batches = st["batches"] - before["batches"]
        graphs = st["graph_launches"] - before["graph_launches"]
        assert batches == 6 and graphs == 0, (batches, graphs)
    finally:
        srv.close()
        ms["syn53d"][0].close()
