"""kx_batch_noalloc, the entry point that allocates nothing: through the C ABI,
two calls in a row (the second with fewer and smaller items and the other
precision), every item's outputs equal, bit for bit, those of the request
server's kx_submit on the same inputs (the same batch kernels and tiles) and
of the direct calls."""
import sys

import numpy as np
import pytest

from paper_2411_02640_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _say(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


def _inputs(ns, n, seed):
    T, p, Y = I.make_states(ns, I.StateSpec(n, seed=seed, p_atm_range=(1.0, 40.0),
                                            dirichlet_alpha=0.3))
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (T, p, Y))


def _served(kx, srv, dm, items, transport, precision):
    ts = [srv.submit(dm, T, p, Y, transport=transport, precision=precision)
          for T, p, Y in items]
    out = []
    for t in ts:
        assert srv.wait(t, 60.0)["state"] == "done"
        out.append(srv.outputs(t))
        srv.release(t)
    return out


def _direct(kx, dm, items, transport, precision):
    out = []
    for T, p, Y in items:
        w = kx.production_rates(dm, T, p, Y, precision=precision)
        tr = kx.transport(dm, T, p, Y, precision=precision) if transport else (None,) * 3
        out.append((w,) + tuple(tr))
    torch.cuda.synchronize()
    return out


def _same(a, b):
    return (a is None and b is None) or torch.equal(a, b)


def test_batch_noalloc_equals_served_and_direct(mech53):
    from paper_2411_02640_amd import kx
    assert torch.cuda.is_available()
    dm = kx.Mechanism(mech53, 0)
    srv = kx.Server(0, hbm_budget=2 << 30, max_slots=64)
    try:
        calls = [([70001, 1, 4097, 20000, 63, 0, 8], True, "fp64"),
                 ([5000, 17], True, "mixed"),
                 ([300, 9], False, "fp64")]
        for c, (sizes, transport, prec) in enumerate(calls):
            _say("call", c, "sizes", sizes, "transport" if transport else "rates", prec)
            items = [_inputs(53, n, 700 + 10 * c + i) for i, n in enumerate(sizes)]
            got = kx.batch_noalloc(dm, items, transport=transport, precision=prec)
            torch.cuda.synchronize()
            served = _served(kx, srv, dm, [it for it in items if it[0].shape[0] > 0],
                             transport, prec)
            direct = _direct(kx, dm, items, transport, prec)
            si = 0
            for i, n in enumerate(sizes):
                for what, g, e in zip(("wdot", "mu", "lambda", "Dmix"), got[i], direct[i]):
                    assert _same(g, e), (c, i, n, what, "direct")
                if n > 0:
                    for what, g, e in zip(("wdot", "mu", "lambda", "Dmix"), got[i], served[si]):
                        assert _same(g, e), (c, i, n, what, "served")
                    si += 1
        # refused: too many items (host check, nothing enqueued)
        items = [_inputs(53, 4, 900)] * (kx.BATCH_MAX_ITEMS + 1)
        with pytest.raises(kx.KxError) as ei:
            kx.batch_noalloc(dm, items)
        assert ei.value.code == kx.KX_EINVAL
    finally:
        srv.close()
        dm.close()
