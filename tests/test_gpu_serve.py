"""GPU tests of the continuously batched solve server.

The bar for a request's result in the mix (P16 of the scope table): the same
iterates as the request solved alone -- every kernel treats each RHS on its
own and the GCR directions are summed oldest first -- so x must agree with the
alone solve to 1e-13 relative with equal iteration counts, and every result must
reach the FP64 true residual 1e-10 against the oracle's operator.
"""
import time

import numpy as np
import pytest

import synth
from oracle.wilson import WilsonOp

pytestmark = pytest.mark.gpu

DIMS, BLOCK = [4, 4, 4, 4], [2, 2, 2, 2]
V = 256


@pytest.fixture(scope="module")
def crk():
    import paper_2502_03091_amd as m
    m.lib()
    return m


def _hier(crk, config, m0=-0.4):
    U = synth.gauge_field(DIMS, 0.3, 0, config=config)
    lat = crk.Lattice(DIMS, m0, 1.0)
    lat.load_gauge(U)
    v0 = synth.gaussian_vectors(16, V, 12, config=config, level=0)
    H = crk.Hierarchy(lat, m_prime=[16], k=[8], block=[BLOCK], n_smooth=[20], setup_form=crk.FORM_FP64,
                      init_vectors=[v0])
    return H, WilsonOp(U, DIMS, m0, 1.0)


@pytest.fixture(scope="module")
def two(crk):
    return _hier(crk, 1), _hier(crk, 11, m0=-0.3)


def _alone(H, b):
    xs, its = [], []
    for r in range(b.shape[0]):
        x, info = H.solve(b[r:r + 1], form=1)
        xs.append(x[0])
        its.append(info["iters"])
    return np.stack(xs), its


def _check_residual(op, b, x):
    D = op.dense()
    for r in range(b.shape[0]):
        if not b[r].any():
            assert not x[r].any()
            continue
        res = b[r].reshape(-1) - D @ x[r].reshape(-1)
        assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(b[r])


def test_results_alone_equal_results_in_mix(crk, two):
    (H, op), _ = two
    # request 0 fills all 7 slots, one of its RHS is zero and frees its slot
    # after the first iteration: request 1 is then admitted while the other six
    # RHS are in flight (continuous batching), request 2 waits for room.
    b0 = synth.gaussian_rhs(7, V, config=21)
    b0[3] = 0
    b1 = synth.gaussian_rhs(1, V, config=22)
    b2 = synth.gaussian_rhs(5, V, config=23)
    with crk.Server(slots_per_lane=7, max_lanes=1, form=1) as srv:
        lid = srv.add(H)
        ids = [srv.submit(lid, b) for b in (b0, b1, b2)]
        out = [srv.wait(i) for i in ids]
        st = srv.stats()
    print("stats", st, flush=True)
    print("infos", [o[1] for o in out], flush=True)
    assert st["completed"] == 3 and st["failed"] == 0
    assert out[1][1]["joined"] == 1, "request 1 should join the running lane"
    assert st["joins"] >= 1 and st["lanes_opened"] == 1
    exact = True
    for b, (x, info) in zip((b0, b1, b2), out):
        assert info["converged"] and info["true_rel_resid"] <= 1e-10
        xa, its = _alone(H, b)
        assert info["iters"] == max(its)
        nz = [r for r in range(b.shape[0]) if b[r].any()]
        err = max(np.abs(x[r] - xa[r]).max() / np.abs(xa[r]).max() for r in nz)
        exact &= all(np.array_equal(x[r], xa[r]) for r in range(b.shape[0]))
        assert err <= 1e-13, err
        _check_residual(op, b, x)
    print("bitwise equal to the alone solves:", exact, flush=True)


def test_two_lattices_run_concurrently(crk, two):
    (H1, op1), (H2, op2) = two
    bs = [synth.gaussian_rhs(n, V, config=30 + i) for i, n in enumerate([3, 2, 4, 1, 2, 3])]
    with crk.Server(slots_per_lane=4, max_lanes=2, form=1) as srv:
        l1, l2 = srv.add(H1), srv.add(H2)
        ids = [(srv.submit(l1 if i % 2 == 0 else l2, b), i) for i, b in enumerate(bs)]
        out = {i: srv.wait(rid) for rid, i in ids}
        st = srv.stats()
    print("stats", st, flush=True)
    assert st["completed"] == len(bs) and st["max_concurrent_lanes"] >= 2
    for i, b in enumerate(bs):
        H, op = ((H1, op1) if i % 2 == 0 else (H2, op2))
        x, info = out[i]
        assert info["converged"] and info["lattice"] == (0 if i % 2 == 0 else 1)
        xa, its = _alone(H, b)
        assert np.abs(x - xa).max() / np.abs(xa).max() <= 1e-13
        _check_residual(op, b, x)


def test_admission_by_footprint(crk, two):
    (H, op), _ = two
    with crk.Server(hbm_budget_bytes=1, form=1) as srv:
        with pytest.raises(crk.CrkError):
            srv.add(H)
    probe = crk.Server(slots_per_lane=4, form=1)
    lane = probe.lane_bytes(probe.add(H))
    probe.close()
    # room for exactly one lane: later requests wait for free slots in it
    bs = [synth.gaussian_rhs(n, V, config=40 + i) for i, n in enumerate([4, 3, 4, 2])]
    with crk.Server(hbm_budget_bytes=lane + lane // 2, slots_per_lane=4, max_lanes=4, form=1) as srv:
        lid = srv.add(H)
        with pytest.raises(crk.CrkError):
            srv.submit(lid, synth.gaussian_rhs(5, V, config=49))  # larger than a lane
        ids = [srv.submit(lid, b) for b in bs]
        out = [srv.wait(i) for i in ids]
        st = srv.stats()
    print("stats", st, "lane bytes", lane, flush=True)
    assert st["lanes_opened"] == 1 and st["peak_bytes"] <= lane + lane // 2
    for b, (x, info) in zip(bs, out):
        assert info["converged"]
        _check_residual(op, b, x)
    # admission order is FIFO
    assert [o[1]["t_admit"] for o in out] == sorted(o[1]["t_admit"] for o in out)


def test_idle_lanes_close(crk, two):
    (H, op), _ = two
    with crk.Server(slots_per_lane=2, max_lanes=3, idle_ms=20, form=1) as srv:
        lid = srv.add(H)
        ids = [srv.submit(lid, synth.gaussian_rhs(2, V, config=50 + i)) for i in range(4)]
        for i in ids:
            srv.wait(i)
        t0 = time.time()
        while srv.stats()["lanes_closed"] < srv.stats()["lanes_opened"] - 1 and time.time() - t0 < 10:
            time.sleep(0.02)
        st = srv.stats()
    print("stats", st, flush=True)
    assert st["lanes_opened"] >= 2
    assert st["lanes_closed"] == st["lanes_opened"] - 1  # the lattice keeps its last lane
