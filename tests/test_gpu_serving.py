"""GPU tests of the continuous-batching server (hs_server_*)."""

import numpy as np
import pytest

from oracle import statevector as sv
from paper_2205_06973_amd import hisv
from paper_2205_06973_amd import serving
from paper_2205_06973_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    torch.cuda.init()
    yield


def _requests(count, seed, n_range=(8, 16), layer_range=(3, 12)):
    return wl.serving_stream(count, 1e6, seed, n_range=n_range, layer_range=layer_range)


def test_mixed_equals_alone_and_oracle():
    """Every amplitude of every request: the same in the mix as alone
    (bitwise: same kernels, same plan), and within the dtype's bars of the
    oracle (max |d| and ||d||_2)."""
    reqs = _requests(16, 3)
    print("[case] 16 requests submitted together", flush=True)
    res = serving.run_stream(reqs, read_states=True, num_streams=4)
    stats = res["stats"]
    assert stats["completed"] == len(reqs)
    assert stats["peak_inflight"] >= 2, "requests must overlap on the device"
    print("[case] the same requests one at a time", flush=True)
    alone = []
    for r in reqs:
        alone.append(serving.run_stream([r], read_states=True, num_streams=1)["states"][0])
    for r, m, a in zip(reqs, res["states"], alone):
        assert m.size == 1 << r.n
        np.testing.assert_array_equal(m, a)
        n, gates = wl.layered28(r.seed, n=r.n, layers=r.layers)
        want = sv.simulate(n, gates)
        bar_max, bar_l2 = (2e-5, 1e-4) if r.dtype == "c64" else (1e-12, 1e-11)
        assert np.max(np.abs(m - want)) <= bar_max
        assert np.linalg.norm(m - want) <= bar_l2
    assert np.all(res["latency"] > 0)
    # the four parts of each latency add up to it
    np.testing.assert_allclose(res["parts"].sum(axis=1), res["latency"], rtol=1e-9, atol=1e-9)
    assert np.all(res["parts"] >= 0)


def test_budget_is_respected():
    reqs = _requests(10, 5, n_range=(16, 16), layer_range=(4, 6))
    biggest = (1 << 16) * 16
    budget = 3 * biggest + (1 << 20)
    print("[case] budget of three 16-qubit states", flush=True)
    stats = serving.run_stream(reqs, budget_bytes=budget, num_streams=4)["stats"]
    assert stats["completed"] == len(reqs)
    assert stats["peak_bytes"] <= budget
    assert stats["cur_bytes"] == 0


def test_request_larger_than_budget_is_rejected():
    srv = hisv.Server(budget_bytes=1 << 20, num_streams=1)
    n, gates = wl.layered28(0, n=20, layers=1)
    with pytest.raises(hisv.HisvError) as e:
        srv.submit(n, gates, "c64", 0, 6)
    assert e.value.code == "HS_E_ADMISSION"
    srv.close()


def test_arrival_stamp_and_errors():
    """Latency starts at the given arrival stamp; an arrival in the future is
    refused; a request that fails during preparation reports its error."""
    srv = hisv.Server(num_streams=2)
    n, gates = wl.layered28(1, n=10, layers=3)
    with pytest.raises(hisv.HisvError) as e:
        srv.submit(n, gates, "c64", 0, 10, "greedy", arrival_s=srv.clock() + 60.0)
    assert e.value.code == "HS_E_ARG"
    t_arr = srv.clock() - 0.25  # arrived a quarter second ago
    t = srv.submit(n, gates, "c64", 0, 10, "greedy", arrival_s=t_arr)
    srv.wait(t)
    assert srv.latency(t) >= 0.25
    q, prep, adm, dev = srv.timing(t)
    assert q >= 0.25 - 1e-3 and prep > 0 and dev > 0
    srv.release(t)
    srv.close()
    # the state fits this budget but state + descriptors do not: the request
    # is accepted, fails while being prepared, and wait reports why
    srv = hisv.Server(budget_bytes=(1 << n) * 8 + 16, num_streams=1)
    t = srv.submit(n, gates, "c64", 0, 10, "greedy")
    with pytest.raises(hisv.HisvError) as e:
        srv.wait(t)
    assert e.value.code == "HS_E_ADMISSION"
    srv.release(t)
    srv.close()


def test_admission_follows_ticket_order_under_a_tight_budget():
    """Requests finish preparing out of order on the server's host threads
    (a long circuit first, short ones after).  Admission still follows
    ticket order, so a client that waits for and releases its requests in
    submission order is never left waiting on one that later, finished but
    unreleased requests keep out of the byte budget."""
    n = 14  # complex128: 256 KiB states
    big = wl.layered28(1, n=n, layers=400)[1]  # 8,400 gates: slow to partition and compile
    small = [wl.layered28(2 + i, n=n, layers=2)[1] for i in range(8)]
    # the long request and about three short ones fit together, not all nine
    srv = hisv.Server(budget_bytes=(7 << 20) // 2, num_streams=2)
    print("[case] tight budget, long request first", flush=True)
    tickets = [srv.submit(n, big, "c128", 0, 7, "greedy")]
    tickets += [srv.submit(n, g, "c128", 0, 7, "greedy") for g in small]
    for t in tickets:
        srv.wait(t, timeout_ms=60000)  # fails (HS_E_STATE) rather than hangs
        srv.release(t)
    stats = srv.stats()
    assert stats["completed"] == len(tickets)
    assert stats["cur_bytes"] == 0 and stats["peak_bytes"] <= (7 << 20) // 2
    srv.close()


def test_small_request_overtakes_a_large_one_on_the_same_stream():
    """Parts go to the device a chunk at a time, at most two chunks queued a
    request: on a single stream, a one-part request admitted right behind a
    request of some 200 parts finishes long before it, and both states
    are right."""
    srv = hisv.Server(num_streams=1)
    nb, big = wl.layered28(7, n=16, layers=150)
    ns, small = wl.layered28(8, n=10, layers=3)
    print("[case] one stream: a large request, then a small one", flush=True)
    tb = srv.submit(nb, big, "c128", 0, 6, "closure")
    ts = srv.submit(ns, small, "c128", 0, 10, "closure")
    srv.wait(tb, timeout_ms=60000)
    srv.wait(ts, timeout_ms=60000)
    q_b, prep_b, adm_b, dev_b = srv.timing(tb)
    q_s, prep_s, adm_s, dev_s = srv.timing(ts)
    assert dev_s < 0.25 * dev_b, (dev_s, dev_b)
    for t, (n, gates) in ((tb, (nb, big)), (ts, (ns, small))):
        got = srv.amplitudes(t, 0, 1 << n)
        want = sv.simulate(n, gates)
        assert np.max(np.abs(got - want)) <= 1e-12
        srv.release(t)
    srv.close()


def test_empty_circuit_request():
    """A request with no gates is its basis state (no parts to launch)."""
    srv = hisv.Server(num_streams=2)
    t = srv.submit(9, [], "c64", 5, 9, "closure")
    srv.wait(t, timeout_ms=30000)
    got = srv.amplitudes(t, 0, 1 << 9)
    want = np.zeros(1 << 9, dtype=np.complex128)
    want[5] = 1
    np.testing.assert_array_equal(got, want)
    srv.release(t)
    srv.close()


def test_release_waits_for_reads_in_flight():
    """Reads of a finished request running on other threads while it is
    released: each one either returns the whole state unchanged or fails
    with HS_E_STATE (the ticket was released first); release returns after
    the reads that had started, and later reads fail."""
    import threading
    srv = hisv.Server(num_streams=2)
    n, gates = wl.layered28(11, n=20, layers=4)
    t = srv.submit(n, gates, "c128", 0, 6, "closure")
    srv.wait(t, timeout_ms=60000)
    ref = srv.amplitudes(t, 0, 1 << n)
    want = sv.simulate(n, gates)
    assert np.max(np.abs(ref - want)) <= 1e-12
    print("[case] 20-qubit request: 2 reader threads racing a release", flush=True)
    results, errors = [], []
    start = threading.Event()

    def reader():
        start.wait()
        for _ in range(8):
            try:
                results.append(srv.amplitudes(t, 0, 1 << n))
            except hisv.HisvError as e:
                errors.append(e)

    threads = [threading.Thread(target=reader) for _ in range(2)]
    for th in threads:
        th.start()
    start.set()
    srv.release(t)
    for th in threads:
        th.join(timeout=60)
        assert not th.is_alive()
    assert len(results) + len(errors) == 16
    for got in results:
        np.testing.assert_array_equal(got, ref)
    for e in errors:
        assert e.code == "HS_E_STATE" and "released" in str(e), str(e)
    with pytest.raises(hisv.HisvError, match="released"):
        srv.amplitudes(t, 0, 16)
    srv.close()
