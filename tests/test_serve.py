"""Serving queue: admission, ordering and results alone vs in a mix.

CPU tests exercise the host-side scheduler (argument checks, HBM-budget
admission, a request that fails on a host without GPU comes back as a
finished ticket with EDEVICE instead of hanging).  GPU tests check that a
request gives the same result alone and inside a concurrent mix, and that
the served result matches the oracle.
"""
import time

import numpy as np
import pytest

import gwinputs as gi

try:
    import paper_2001_05798_amd as gw
except ImportError:  # library not built
    gw = None

needs_lib = pytest.mark.skipif(gw is None, reason="library not built")


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def _params():
    return gw.AmgParams(precision=gw.PRECISION_MIXED), gw.SolveParams(rtol=1e-8)


@needs_lib
def test_queue_argument_checks_cpu():
    q = gw.Queue(hbm_budget_bytes=1 << 30, max_slots=2)
    ap, sp = _params()
    # far larger than the budget: refused at submission
    big = gi.Problem(gi.Grid(512, 512, 256), np.ones(1))
    with pytest.raises(gw.GwError) as e:
        q.submit(big, ap, ap, sp)
    assert e.value.status == gw.ENOMEM
    bad = gi.Problem(gi.Grid(8, 8, 8), np.full(512, 1e-4), phi=0.0)
    with pytest.raises(gw.GwError) as e:
        q.submit(bad, ap, ap, sp)
    assert e.value.status == gw.EINVAL
    with pytest.raises(gw.GwError):
        q.poll(12345)
    q.close()


@needs_lib
@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_queue_without_device_finishes_with_error():
    q = gw.Queue(hbm_budget_bytes=1 << 30, max_slots=2)
    ap, sp = _params()
    p = gi.homogeneous_slab(8, 8)
    t = q.submit(p, ap, ap, sp)
    q.drain()
    res, _ = q.poll(t)
    assert res.status == gw.EDEVICE
    assert res.t_done >= res.t_start >= res.t_arrival >= 0
    q.close()


def _serve(problems, slots, budget=64 << 30, batch=None, window_us=0.0, stats=None):
    ap, sp = _params()
    tp = gw.AmgParams.travel_time(precision=gw.PRECISION_MIXED)
    q = gw.Queue(hbm_budget_bytes=budget, max_slots=slots)
    if batch is not None:
        q.set_batch(batch, window_us)
    tickets = [q.submit(p, ap, tp, sp, zone=(0, p.grid.ny, 0, max(1, p.grid.nz // 2))) for p in problems]
    q.drain()
    out = [q.poll(t) for t in tickets]
    if stats is not None:
        stats.extend(q.stats())
    q.close()
    return out


def _target():
    return gi.heterogeneous_aquifer(40, 36, 24, 2.0, 6, 101)


@pytest.fixture(scope="module")
def mix_run():
    """The target request inside a concurrent 4-slot mix of six requests."""
    if gw is None or not _has_gpu():
        pytest.skip("no GPU")
    others = [gi.heterogeneous_aquifer(s, s, s, s2, lam, seed) for s, s2, lam, seed in
              [(48, 4.0, 8, 7), (32, 1.0, 4, 8), (56, 2.0, 12, 9), (36, 4.0, 16, 10), (44, 1.0, 5, 11)]]
    return _serve(others[:3] + [_target()] + others[3:], slots=4)


@pytest.mark.gpu
def test_alone_equals_in_mix(mix_run):
    print("[case] serve alone vs mix", flush=True)
    target = _target()
    (alone_res, alone_out), = _serve([target], slots=1)
    assert alone_res.status == gw.OK, (alone_res.status, alone_res.error)
    mix = mix_run
    mix_res, mix_out = mix[3]
    assert all(r.status == gw.OK for r, _ in mix), [r.status for r, _ in mix]
    for k in ("h", "tau", "c"):
        a, b = alone_out[k], mix_out[k]
        rel = np.linalg.norm(a - b) / np.linalg.norm(a)
        print(f"  {k}: rel diff {rel:.2e} bitwise {np.array_equal(a, b)}", flush=True)
        assert rel <= 1e-6  # mixed-precision tolerance
    # requests really overlapped: some started before others finished
    starts = sorted(r.t_start for r, _ in mix)
    dones = sorted(r.t_done for r, _ in mix)
    assert starts[1] < dones[0]
    for r, _ in mix:
        assert 0 < r.bytes_used <= r.bytes_reserved, (r.bytes_used, r.bytes_reserved)


@pytest.mark.gpu
def test_shared_launches_equal_own_streams():
    # the same mix served with shared launches (every running request's solve
    # waits up to 0.5 s for the others, so solves of one phase share a batch)
    # and with each request solving on its own stream: results bit for bit
    # equal; the footprint a request held stays within its admission bytes
    if gw is None or not _has_gpu():
        pytest.skip("no GPU")
    print("[case] serve shared launches vs own streams", flush=True)
    probs = [gi.heterogeneous_aquifer(s, s - 4, s - 8, s2, lam, seed) for s, s2, lam, seed in
             [(40, 2.0, 6, 61), (32, 4.0, 4, 62), (48, 1.0, 8, 63), (36, 2.0, 5, 64)]]
    st = []
    shared = _serve(probs, slots=4, batch=16, window_us=5e5, stats=st)
    own = _serve(probs, slots=4, batch=1)
    shared_blocks, solves = st
    print(f"  {solves} solves, {shared_blocks} blocks of iterations shared by two or more", flush=True)
    assert solves == 2 * len(probs) and shared_blocks > 0
    for (ra, oa), (rb, ob) in zip(shared, own):
        assert ra.status == gw.OK and rb.status == gw.OK, (ra.error, rb.error)
        for k in ("h", "tau", "c"):
            assert np.array_equal(oa[k].view(np.uint64), ob[k].view(np.uint64)), k
        assert (ra.flow.iters, ra.tt[0].iters, ra.tt[1].iters) == (rb.flow.iters, rb.tt[0].iters, rb.tt[1].iters)
        assert 0 < ra.bytes_used <= ra.bytes_reserved, (ra.bytes_used, ra.bytes_reserved)


@pytest.mark.gpu
def test_served_result_matches_oracle(mix_run, ref):
    # the request served inside the mix against the FP64 oracle end to end:
    # flow by flexible CG on the same hierarchy settings, Darcy fluxes from
    # the oracle's own heads, then the travel-time pair by BiCGSTAB with the
    # travel-time settings; h, tau and c within the mixed-path tolerance
    print("[case] served request vs oracle", flush=True)
    p = _target()
    g = p.grid
    res, out = mix_run[3]
    assert res.status == gw.OK
    ap = gw.AmgParams()
    tp = gw.AmgParams.travel_time()
    fr = ref.solve_flow(p, ref.AmgParams(eps_strong=ap.eps_strong, npre=ap.npre, npost=ap.npost),
                        rtol=1e-8, flexible=True)
    qx, qy, qz = ref.darcy_flux(p, fr.h)
    tr = ref.solve_travel_time(g, qx, qy, qz, p.phi,
                               ref.AmgParams(eps_strong=tp.eps_strong, npre=tp.npre, npost=tp.npost),
                               rtol=1e-8, zone=(0, g.ny, 0, max(1, g.nz // 2)))
    assert fr.info.status == ref.OK and all(i.status == ref.OK for i in tr.info)
    for k, want in (("h", fr.h), ("tau", tr.tau), ("c", tr.c)):
        rel = np.linalg.norm(out[k] - want) / np.linalg.norm(want)
        print(f"  {k}: rel err vs oracle {rel:.2e}", flush=True)
        assert rel <= 1e-6, (k, rel)


@pytest.mark.gpu
def test_admission_by_budget():
    if gw is None or not _has_gpu():
        pytest.skip("no GPU")
    print("[case] serve admission", flush=True)
    probs = [gi.heterogeneous_aquifer(48, 48, 48, 2.0, 8, s) for s in range(4)]
    ap, sp = _params()
    # room for one request at a time although four slots exist
    one = 48 ** 3 * 1900 + (64 << 20)  # the queue's mixed-precision footprint
    res = _serve(probs, slots=4, budget=int(one * 1.5))
    assert all(r.status == gw.OK for r, _ in res)
    spans = sorted((r.t_start, r.t_done) for r, _ in res)
    for (s0, d0), (s1, d1) in zip(spans, spans[1:]):
        assert s1 >= d0 - 1e-6  # serialized by the budget


@needs_lib
def test_batch_argument_checks_cpu():
    q = gw.Queue(hbm_budget_bytes=1 << 30, max_slots=1)
    for bad in ((0, 0.0), (257, 0.0), (4, -1.0), (4, 0.0, 0), (4, 0.0, 17)):
        with pytest.raises(gw.GwError) as e:
            q.set_batch(*bad)
        assert e.value.status == gw.EINVAL
    q.set_batch(1)
    q.set_batch(8, 100.0, 4)
    assert q.stats() == (0, 0)
    q.close()


@needs_lib
def test_setup_cache_argument_checks_cpu():
    q = gw.Queue(hbm_budget_bytes=1 << 30, max_slots=1)
    for bad in (-1, 65):
        with pytest.raises(gw.GwError) as e:
            q.set_setup_cache(bad)
        assert e.value.status == gw.EINVAL
    q.set_setup_cache(4)
    q.set_setup_cache(0)
    q.close()


def _with_wells(p, scale):
    return gi.Problem(p.grid, p.K, p.h_west, p.h_east, [gi.Well(w.ix, w.iy, w.iz, w.q * scale) for w in p.wells],
                      p.phi, p.label)


def _serve_seq(problems, cache, budget=64 << 30):
    ap, sp = _params()
    tp = gw.AmgParams.travel_time(precision=gw.PRECISION_MIXED)
    q = gw.Queue(hbm_budget_bytes=budget, max_slots=1)
    q.set_setup_cache(cache)
    out = []
    for p in problems:  # one at a time, so the cache state is known
        t = q.submit(p, ap, tp, sp, zone=(0, p.grid.ny, 0, max(1, p.grid.nz // 2)))
        q.drain()
        out.append(q.poll(t))
    q.close()
    return out


@pytest.mark.gpu
def test_setup_cache_reuse_on_well_rates():
    if gw is None or not _has_gpu():
        pytest.skip("no GPU")
    print("[case] serve setup cache", flush=True)
    base = gi.heterogeneous_aquifer(40, 36, 24, 2.0, 6, 101)
    other = gi.heterogeneous_aquifer(40, 36, 24, 2.0, 6, 102)
    p1, p2 = _with_wells(base, 1.0), _with_wells(base, 0.5)
    res = _serve_seq([p1, p2, other, p2], cache=2)
    assert all(r.status == gw.OK for r, _ in res), [(r.status, r.error) for r, _ in res]
    assert [r.setup_reused for r, _ in res] == [0, 1, 0, 1]
    # the cached hierarchy is the one a new setup would build: same results bit for bit
    (fresh, fresh_out), = _serve_seq([p2], cache=0)
    assert fresh.setup_reused == 0
    for k in ("h", "tau", "c"):
        assert np.array_equal(res[1][1][k], fresh_out[k]), k
        assert np.array_equal(res[3][1][k], fresh_out[k]), k
    # a budget with room for one request: the cached setup gives way
    one = 40 * 36 * 24 * 1900 + (64 << 20)
    res = _serve_seq([p1, other, p2], cache=4, budget=int(one * 1.02))
    assert all(r.status == gw.OK for r, _ in res)
    assert [r.setup_reused for r, _ in res] == [0, 0, 0]
