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
    reqs = _requests(16, 3)
    print("[case] 16 requests submitted together", flush=True)
    lat, wall, stats, mixed = serving.run_stream(reqs, read_check=1 << 8, num_streams=4)
    assert stats["completed"] == len(reqs)
    assert stats["peak_inflight"] >= 2, "requests must overlap on the device"
    print("[case] the same requests one at a time", flush=True)
    alone = []
    for r in reqs:
        _, _, _, a = serving.run_stream([r], read_check=1 << 8, num_streams=1)
        alone.append(a[0])
    for r, m, a in zip(reqs, mixed, alone):
        np.testing.assert_array_equal(m, a)  # same kernels, same plan: bitwise
        n, gates = wl.layered28(r.seed, n=r.n, layers=r.layers)
        want = sv.simulate(n, gates)[: 1 << 8]
        tol = 2e-5 if r.dtype == "c64" else 1e-12
        assert np.max(np.abs(m - want)) <= tol
    assert np.all(lat > 0)


def test_budget_is_respected():
    reqs = _requests(10, 5, n_range=(16, 16), layer_range=(4, 6))
    biggest = (1 << 16) * 16
    budget = 3 * biggest + (1 << 20)
    print("[case] budget of three 16-qubit states", flush=True)
    lat, wall, stats, _ = serving.run_stream(reqs, budget_bytes=budget, num_streams=4)
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
