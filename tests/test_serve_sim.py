"""Request server logic on the host (KX_SERVER_SIMULATE: no memory, no
kernels; a batch completes after 5 ns per point and op)."""
import pytest

from paper_2411_02640_amd import kx


@pytest.fixture(scope="module")
def m53(mech53):
    m = kx.HostMechanism(mech53)
    yield m
    m.close()


@pytest.fixture(scope="module")
def m9(mech9):
    m = kx.HostMechanism(mech9)
    yield m
    m.close()


def footprint(ns, n, transport):
    d = ns + ((ns + 2) if transport else 0)
    return (n * 8 * d + 255) // 256 * 256


def resident(*mechs):
    """Arena bytes the resident tables of these mechanisms take."""
    return sum((m.device_bytes + 255) // 256 * 256 for m in mechs)


def test_all_complete_and_release(m53):
    s = kx.Server(hbm_budget=1 << 30, max_slots=8, simulate=True)
    ts = [s.submit(m53, n=100_000, transport=(i % 2 == 0)) for i in range(20)]
    for t in ts:
        assert s.wait(t, 10.0)["state"] == "done"
        s.release(t)
    st = s.stats()
    assert st["submitted"] == 20 and st["completed"] == 20 and st["in_flight"] == 0
    assert st["arena_in_use"] == resident(m53) and 1 <= st["batches"] <= 20
    s.close()


def test_fifo_admission_under_memory_pressure(m53):
    n = 50_000
    fp = footprint(m53.n_species, n, False)
    s = kx.Server(hbm_budget=2 * fp + resident(m53), max_slots=16, simulate=True)
    ts = [s.submit(m53, n=n) for _ in range(6)]
    admits = []
    for t in ts:
        r = s.wait(t, 10.0)
        assert r["state"] == "done"
        admits.append(r["t_admit"])
        assert s.stats()["arena_in_use"] <= 2 * fp + resident(m53)
        s.release(t)
    assert admits == sorted(admits)
    s.close()


def test_blocked_queue_cancel_and_timeout(m53):
    n = 10_000
    fp = footprint(m53.n_species, n, True)
    s = kx.Server(hbm_budget=fp + resident(m53), max_slots=4, simulate=True)
    a = s.submit(m53, n=n, transport=True)
    assert s.wait(a, 10.0)["state"] == "done"          # holds the whole arena
    b = s.submit(m53, n=n, transport=True)
    c = s.submit(m53, n=n // 2)
    with pytest.raises(kx.KxError) as ei:
        s.wait(b, 0.05)
    assert ei.value.code == kx.KX_EAGAIN
    assert s.poll(b)["state"] == "queued" and s.poll(c)["state"] == "queued"
    assert s.stats()["queued"] == 2
    with pytest.raises(kx.KxError) as ei:
        s.release(b)                                     # not finished
    assert ei.value.code == kx.KX_EAGAIN
    s.cancel(b)
    assert s.poll(b)["state"] == "cancelled"
    # c still waits (strict FIFO needs memory c cannot get while a is held)
    assert s.poll(c)["state"] == "queued"
    with pytest.raises(kx.KxError) as ei:
        s.cancel(a)                                      # already done
    assert ei.value.code == kx.KX_EAGAIN
    s.release(a)
    assert s.wait(c, 10.0)["state"] == "done"
    s.release(b)
    s.release(c)
    st = s.stats()
    assert st["cancelled"] == 1 and st["completed"] == 2
    assert st["arena_in_use"] == resident(m53)
    s.close()


def test_strict_fifo_no_overtaking(m53):
    big, small = 40_000, 1_000
    fpb = footprint(m53.n_species, big, False)
    s = kx.Server(hbm_budget=fpb + footprint(m53.n_species, small, False) + resident(m53),
                  max_slots=8,
                  simulate=True)
    a = s.submit(m53, n=big)
    assert s.wait(a, 10.0)["state"] == "done"
    b = s.submit(m53, n=big)          # cannot fit while a is held
    c = s.submit(m53, n=small)        # would fit, but must not overtake b
    with pytest.raises(kx.KxError):
        s.wait(c, 0.05)
    assert s.poll(c)["state"] == "queued"
    s.release(a)
    rb, rc = s.wait(b, 10.0), s.wait(c, 10.0)
    assert rb["state"] == rc["state"] == "done"
    assert rb["t_admit"] <= rc["t_admit"]
    for t in (b, c):
        s.release(t)
    s.close()


def test_slot_limit(m53):
    s = kx.Server(hbm_budget=1 << 30, max_slots=1, simulate=True)
    ts = [s.submit(m53, n=20_000) for _ in range(5)]
    launches = []
    for t in ts:
        r = s.wait(t, 10.0)
        launches.append(r["t_launch"])
        s.release(t)
    # one request in flight at a time: every launch is a batch of its own
    assert len(set(launches)) == 5
    assert s.stats()["batches"] == 5
    s.close()


def test_batches_are_homogeneous(m53, m9):
    """60 requests of two mechanisms and both precisions queue behind a
    finished request that holds the whole arena; releasing it admits them in
    one pass, and they run as one batch per (mechanism, precision) group
    (independent of how fast the submitting thread is)."""
    n_blk = 1 << 20
    s = kx.Server(hbm_budget=footprint(m53.n_species, n_blk, False) + resident(m53, m9),
                  max_slots=64, simulate=True)
    s.add_mech(m53)
    s.add_mech(m9)
    blocker = s.submit(m53, n=n_blk)
    assert s.wait(blocker, 10.0)["state"] == "done"
    spec = [(m53 if i % 3 else m9, "fp64" if i % 2 else "mixed") for i in range(60)]
    ts = [s.submit(m, n=5_000, precision=p) for m, p in spec]
    assert s.stats()["queued"] == 60
    s.release(blocker)
    groups = {}
    for (m, p), t in zip(spec, ts):
        r = s.wait(t, 10.0)
        assert r["state"] == "done"
        groups.setdefault(r["t_launch"], set()).add((m.handle.value, p))
        s.release(t)
    assert all(len(g) == 1 for g in groups.values())
    assert s.stats()["batches"] <= 1 + 4
    s.close()


def test_zero_points_and_oversize(m53):
    s = kx.Server(hbm_budget=1 << 20, max_slots=4, simulate=True)
    t = s.submit(m53, n=0)
    assert s.poll(t)["state"] == "done"
    s.release(t)
    with pytest.raises(kx.KxError) as ei:
        s.submit(m53, n=10_000_000)
    assert ei.value.code == kx.KX_ENOMEM
    s.close()


def test_invalid_requests(m53):
    L = kx._serve_lib()
    s = kx.Server(hbm_budget=1 << 20, max_slots=4, simulate=True)
    s.add_mech(m53)
    import ctypes as C
    t = C.c_int64()

    def sub(**kw):
        r = kx._Request()
        r.mech = m53.handle.value
        r.ops, r.precision, r.n, r.arrival_s = 1, 0, 10, -1.0
        for k, v in kw.items():
            setattr(r, k, v)
        return L.kx_submit(s.handle, C.byref(r), C.byref(t))

    assert sub() == kx.KX_OK
    assert sub(ops=0) == kx.KX_EINVAL
    assert sub(ops=kx.KX_OP_TRANSPORT) == kx.KX_EINVAL
    assert sub(ops=8) == kx.KX_EINVAL
    assert sub(precision=5) == kx.KX_EINVAL
    assert sub(n=-1) == kx.KX_EINVAL
    assert sub(mech=None) == kx.KX_EINVAL
    with pytest.raises(kx.KxError):
        s.poll(123456)
    s.close()
    h = C.c_void_p()
    assert L.kx_server_create(0, 0, 4, kx.KX_SERVER_SIMULATE, C.byref(h)) == kx.KX_EINVAL
    assert L.kx_server_create(0, 1 << 20, 0, kx.KX_SERVER_SIMULATE, C.byref(h)) == kx.KX_EINVAL


def test_destroy_cancels_queued(m53):
    n = 10_000
    s = kx.Server(hbm_budget=footprint(m53.n_species, n, False) + resident(m53), max_slots=4,
                  simulate=True)
    a = s.submit(m53, n=n)
    s.wait(a, 10.0)
    ts = [s.submit(m53, n=n) for _ in range(3)]
    assert s.stats()["queued"] == 3
    s.close()   # returns although three requests could never be admitted


def test_latency_timestamps(m53):
    s = kx.Server(hbm_budget=1 << 30, max_slots=8, simulate=True)
    t0 = kx.clock()
    t = s.submit(m53, n=200_000, arrival=t0 - 0.5)
    r = s.wait(t, 10.0)
    assert r["t_arrival"] == pytest.approx(t0 - 0.5)
    assert r["t_arrival"] <= r["t_admit"] <= r["t_launch"] <= r["t_done"]
    assert r["t_done"] - r["t_launch"] >= 200_000 * 5e-9 * 0.9
    s.release(t)
    s.close()


def test_concurrent_clients(m53, m9):
    """Four client threads submit, poll, wait for, cancel and release requests
    at the same time as the scheduler runs (the ctypes calls release the GIL,
    so the library sees concurrent callers); every request ends DONE or
    CANCELLED and the arena is empty at the end."""
    import threading
    s = kx.Server(hbm_budget=64 << 20, max_slots=8, simulate=True)
    errors = []

    def client(c):
        try:
            ts = []
            for i in range(30):
                m = m53 if (i + c) % 2 else m9
                ts.append(s.submit(m, n=2_000 + 500 * i, transport=bool(i % 3 == 0),
                                   precision="mixed" if i % 4 == 0 else "fp64"))
                s.poll(ts[-1])
                if i % 7 == 3:
                    try:
                        s.cancel(ts[-1])
                    except kx.KxError:
                        pass  # already launched
            for t in ts:
                r = s.wait(t, 30.0)
                assert r["state"] in ("done", "cancelled"), r
                s.release(t)
        except Exception as e:  # noqa: BLE001 -- reported by the main thread
            errors.append(e)

    th = [threading.Thread(target=client, args=(c,)) for c in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    st = s.stats()
    assert st["submitted"] == 120 and st["completed"] + st["cancelled"] == 120
    assert st["arena_in_use"] == resident(m53, m9) and st["in_flight"] == 0
    s.close()


def test_resident_mechanisms_charge_the_budget(m53, m9):
    """kx_server_add_mech charges a mechanism's tables to the arena once; a
    request must name a resident mechanism, and its outputs must fit in what
    the resident tables leave of the budget."""
    import ctypes as C
    L = kx._serve_lib()
    r53 = resident(m53)
    n = 10_000
    budget = r53 + footprint(m53.n_species, n, False)
    s = kx.Server(hbm_budget=budget, max_slots=4, simulate=True)
    st = s.stats()
    assert st["resident_mechs"] == 0 and st["arena_in_use"] == 0
    s.add_mech(m53)
    s.add_mech(m53)                                   # a no-op the second time
    st = s.stats()
    assert st["resident_mechs"] == 1 and st["resident_bytes"] == r53
    assert st["arena_in_use"] == r53
    # a mechanism that is not resident is refused at submit
    r = kx._Request()
    r.mech, r.ops, r.precision, r.n, r.arrival_s = m9.handle.value, 1, 0, 10, -1.0
    t = C.c_int64()
    assert L.kx_submit(s.handle, C.byref(r), C.byref(t)) == kx.KX_EINVAL
    # the largest request that fits beside the tables runs and, while it holds
    # its outputs, leaves no room for another mechanism's tables
    a = s.submit(m53, n=n)
    assert s.wait(a, 10.0)["state"] == "done"
    assert L.kx_server_add_mech(s.handle, m9.handle) == kx.KX_ENOMEM
    s.release(a)
    # one more point than fits beside the tables is refused at submit
    with pytest.raises(kx.KxError) as ei:
        s.submit(m53, n=n + 64)
    assert ei.value.code == kx.KX_ENOMEM
    assert s.stats()["arena_in_use"] == r53
    s.close()
