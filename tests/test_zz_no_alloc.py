"""hs_norm_noalloc (the norm with its partial sums in a static device array)
against hs_norm, through the C ABI: two calls in a row, the second on a
smaller state, for both dtypes."""

import numpy as np
import pytest

from paper_2205_06973_amd import hisv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_norm_noalloc_matches_norm(dtype):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    tdt = {"c64": torch.complex64, "c128": torch.complex128}[dtype]
    g = torch.Generator().manual_seed(11)
    for n in (20, 11):  # the second call on a smaller state
        print(f"[case] norm_noalloc {dtype} n={n}", flush=True)
        # an unnormalised state with a known sum of squares
        host = torch.randn(1 << n, dtype=tdt, generator=g) * 0.37
        buf = host.to("cuda")
        st = hisv.State.wrap_tensor(buf, torch.cuda.current_stream())
        got = st.norm_noalloc()
        want = st.norm()
        assert got == want, f"n={n}: {got!r} != {want!r}"
        h = host.numpy().astype(np.complex128)
        exact = float(np.sum(h.real ** 2 + h.imag ** 2))
        assert abs(got - exact) <= 1e-12 * exact
        # a second call on the same state reads the array the first one left
        assert st.norm_noalloc() == want
        st.close()
        del buf
