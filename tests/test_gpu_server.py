"""Solve server (btrt_server_*): continuous batching of requests of different sizes.

Each request's result must be bitwise the same alone and in a mix that changes while it runs,
equal to btrt_solve on a single handle with the same check interval, and the FP64 result must
match the oracle; admission must respect the device-memory budget.
"""
import sys

import numpy as np
import pytest

from paper_1902_09813_amd import btrt
from paper_1902_09813_amd import workloads as W
from tests._cases import normwise, run_oracle

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def requests(count, seed=5, side_range=(16, 120), max_steps=3000, tol=1e-7, precision=btrt.F32):
    reqs = W.c5(count, rate=1.0, seed=seed, side_range=side_range, tol=tol, max_steps=max_steps)
    return [(btrt.problem_from_workload(w, precision=precision, check_interval=200), w.phi0(), tol, ms, w)
            for _, w, tol, ms in reqs]


def drain(srv, ids, limit=10000):
    for _ in range(limit):
        if all(srv.info(i)["status"] >= btrt.REQ_DONE for i in ids):
            return
        srv.pump()
    raise AssertionError("server did not finish")


def test_result_is_the_same_alone_and_in_the_mix():
    reqs = requests(12)
    target = 5
    p, ph, tol, ms, w = reqs[target]
    say(f"[gpu] server: request {w.name} alone")
    with btrt.Server(precision=btrt.F32, check_interval=200, max_active=8) as srv:
        rid = srv.submit(p, ph, tol, ms)
        drain(srv, [rid])
        info_alone = srv.info(rid)
        alone = srv.result(rid)
    say("[gpu] server: the same request in a mix that changes while it runs")
    with btrt.Server(precision=btrt.F32, check_interval=200, max_active=8) as srv:
        ids = [srv.submit(*r[:4]) for r in reqs[:4]]
        srv.pump()
        srv.pump()
        rid = srv.submit(p, ph, tol, ms)
        for r in reqs[6:]:
            ids.append(srv.submit(*r[:4]))
            srv.pump()
        drain(srv, ids + [rid])
        info_mix = srv.info(rid)
        mixed = srv.result(rid)
    assert info_alone["steps"] == info_mix["steps"]
    assert info_alone["residual"] == info_mix["residual"]
    assert np.array_equal(alone, mixed)


def test_server_matches_single_handle_solve():
    reqs = requests(6, seed=8)
    with btrt.Server(precision=btrt.F32, check_interval=200, max_active=3) as srv:
        ids = [srv.submit(*r[:4]) for r in reqs]
        drain(srv, ids)
        for rid, (p, ph, tol, ms, w) in zip(ids, reqs):
            info = srv.info(rid)
            got = srv.result(rid)
            with btrt.Solver(btrt.problem_from_workload(w, precision=btrt.F32, check_interval=200), ph) as s:
                steps, res = s.solve(tol, ms)
                assert steps == info["steps"] and res == info["residual"], w.name
                assert np.array_equal(s.field(), got), w.name


def test_admission_respects_memory_budget():
    reqs = requests(6, seed=11, side_range=(100, 120), max_steps=1000, tol=0.0)
    need = max(r[0].workspace_size() for r in reqs)
    budget = 2 * need + 4096  # two requests fit at a time
    with btrt.Server(precision=btrt.F32, memory_bytes=budget, check_interval=200, max_active=16) as srv:
        ids = [srv.submit(*r[:4]) for r in reqs]
        srv.pump()
        st = srv.stats()
        assert st["active"] == 2 and st["queued"] == 4
        assert st["memory_in_use"] <= budget
        drain(srv, ids)
        st = srv.stats()
        assert st["completed"] == 6 and st["memory_in_use"] == 0 and st["memory_high_water"] <= budget
        for rid in ids:
            info = srv.info(rid)
            assert info["status"] == btrt.REQ_DONE and info["steps"] == 1000
            assert info["t_submit"] <= info["t_admit"] <= info["t_done"]


def test_request_larger_than_memory_is_rejected():
    p, ph, tol, ms, _ = requests(1, side_range=(120, 121))[0]
    with btrt.Server(precision=btrt.F32, memory_bytes=1 << 16, check_interval=100) as srv:
        with pytest.raises(btrt.BtrtError) as e:
            srv.submit(p, ph, tol, ms)
        assert e.value.code == btrt.E_NOMEM


def test_unstable_request_fails_alone():
    tau = 0.8
    k1 = 1 / tau
    a = (tau - 0.5) / 3.0
    bad = btrt.Problem(32, 32, precision=btrt.F32, flux_a=(0.5, 0.5), A0=(a, 0.0, a), k0=k1, k2=k1,
                       check_interval=1000)
    ph_bad = 1.0 + 0.01 * np.random.default_rng(0).random((32, 32))
    reqs = requests(3, seed=21, max_steps=8000, tol=0.0)
    with btrt.Server(precision=btrt.F32, check_interval=1000, max_active=8) as srv:
        ids = [srv.submit(*r[:4]) for r in reqs]
        rb = srv.submit(bad, ph_bad, 0.0, 20000)
        drain(srv, ids + [rb])
        assert srv.info(rb)["status"] == btrt.REQ_FAILED and srv.info(rb)["error"] == btrt.E_UNSTABLE
        for rid in ids:
            assert srv.info(rid)["status"] == btrt.REQ_DONE
        # Collecting the failed request reports its error and releases it; nothing stays resident.
        with pytest.raises(btrt.BtrtError) as e:
            srv.result(rb)
        assert e.value.code == btrt.E_UNSTABLE
        with pytest.raises(btrt.BtrtError) as e:
            srv.info(rb)
        assert e.value.code == btrt.E_INVAL
        st = srv.stats()
        assert st["active"] == 0 and st["failed"] == 1


def test_fp64_served_result_matches_oracle():
    reqs = requests(4, seed=31, side_range=(20, 60), max_steps=600, tol=0.0, precision=btrt.F64)
    with btrt.Server(precision=btrt.F64, check_interval=200, max_active=4) as srv:
        ids = [srv.submit(*r[:4]) for r in reqs]
        drain(srv, ids)
        for rid, (p, ph, tol, ms, w) in zip(ids, reqs):
            w.steps = 600
            assert normwise(srv.result(rid), run_oracle(w).phi()) <= 1e-12, w.name


@pytest.mark.parametrize("launch", [(4, 0, 0, 16), (4, 2, 0, 32), (1, 0, 0, 0)], ids=["walk16", "walk32_b2", "one_step"])
def test_server_launch_configurations_match_single_handle(launch):
    reqs = requests(5, seed=17, max_steps=1200, tol=0.0)
    with btrt.Server(precision=btrt.F32, check_interval=200, max_active=8, launch=launch) as srv:
        ids = [srv.submit(*r[:4]) for r in reqs]
        drain(srv, ids)
        for rid, (p, ph, tol, ms, w) in zip(ids, reqs):
            with btrt.Solver(btrt.problem_from_workload(w, precision=btrt.F32, check_interval=200), ph) as s:
                steps, res = s.solve(tol, ms)
                assert steps == srv.info(rid)["steps"]
                assert np.array_equal(s.field(), srv.result(rid)), (launch, w.name)


def test_automatic_launch_switches_with_the_resident_work():
    # Two large requests (together above 2^21 nodes) make the server switch to the strip walkers
    # while both are resident and back once one retires; the bits stay those of a single handle.
    big = [W.c5(1, rate=1.0, seed=s_, side_range=(1100, 1101), tol=0.0, max_steps=ms_)[0][1]
           for s_, ms_ in ((51, 600), (52, 1400))]
    small = requests(3, seed=53, max_steps=1000, tol=0.0)
    with btrt.Server(precision=btrt.F32, check_interval=200, max_active=8) as srv:
        jobs = [(srv.submit(btrt.problem_from_workload(w, precision=btrt.F32, check_interval=200), w.phi0(), 0.0,
                            w.steps), w) for w in big]
        jobs += [(srv.submit(*r[:4]), r[4]) for r in small]
        drain(srv, [j for j, _ in jobs])
        for rid, w in jobs:
            info = srv.info(rid)
            assert info["status"] == btrt.REQ_DONE
            with btrt.Solver(btrt.problem_from_workload(w, precision=btrt.F32, check_interval=200), w.phi0()) as s:
                s.step(info["steps"])
                assert np.array_equal(s.field(), srv.result(rid)), w.name


@pytest.mark.parametrize("precision", [btrt.F32, btrt.F64], ids=["f32", "f64"])
def test_large_requests_run_their_own_launches_with_the_same_bits(precision):
    # Requests of 2^20 nodes and more advance by their own single-grid launches inside each round
    # (automatic launch configuration); their results, and those of the small requests batched
    # beside them, equal btrt_solve on single handles bit for bit, periodic and walled.
    big = [W.c4(count=1, seed=41, side_range=(1024, 1024))[0], W.c4(count=1, seed=44, side_range=(1030, 1030))[0]]
    small = [w for _, w, _, _ in W.c5(5, rate=1.0, seed=47, side_range=(40, 200))]
    assert {w.bc_type[0] for w in big} == {btrt.PERIODIC, btrt.DIRICHLET}
    work = [(w, 0.0 if i % 2 else 1e-7, 1600) for i, w in enumerate(big + small)]
    say(f"[gpu] server with large requests {[w.nx for w in big]} and small ones {[w.nx for w in small]}")
    with btrt.Server(precision=precision, check_interval=400, max_active=8, memory_bytes=8 << 30) as srv:
        ids = []
        for w, tol, ms in work:
            ids.append(srv.submit(btrt.problem_from_workload(w, precision=precision, check_interval=400), w.phi0(),
                                  tol, ms))
            srv.pump()
        drain(srv, ids)
        for rid, (w, tol, ms) in zip(ids, work):
            info = srv.info(rid)
            got = srv.result(rid)
            with btrt.Solver(btrt.problem_from_workload(w, precision=precision, check_interval=400), w.phi0()) as s:
                steps, res = s.solve(tol, ms)
                assert steps == info["steps"] and res == info["residual"], w.name
                assert np.array_equal(s.field(), got), w.name
