"""GPU test of rst_components_noalloc, the entry point that allocates nothing
(its scratch is a fixed device array per GPU): through the C ABI, its labels
and component count must equal those of rst_components (min-id labels are
unique, so bit for bit) and the oracle's, on two calls in a row, the second
with a smaller graph (the array keeps the first call's contents); a graph
larger than the array holds is refused before any device work."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2603_11645_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rst():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_11645_amd as r
    return r


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_noalloc_equals_components_twice(rst):
    c = rst.Context(0)
    graphs = [I.random_graph(300000, 420000, seed=31, connected=False),
              I.road_mesh(200, 0.2, 0.01, seed=32)]          # the second call is smaller
    assert graphs[1].n < graphs[0].n
    for g in graphs:
        off, cols = dev(g.offsets_typed()), dev(g.cols)
        ref, k_ref = c.components(off, cols)
        label = torch.full((g.n,), -5, dtype=torch.int32, device="cuda")
        got, k = c.components_noalloc(off, cols, label=label)
        assert k == k_ref, g.name
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy()), g.name
        k_o, lab_o = oracle.components(g.n, g.offsets, g.cols)
        assert k == k_o and np.array_equal(got.cpu().numpy(), lab_o), g.name


def test_noalloc_refuses_graphs_beyond_its_scratch(rst):
    c = rst.Context(0)
    small = dev(np.zeros(2, np.int32))
    g = rst.rst_csr(1 << 25, 0, 4, ctypes.c_void_p(small.data_ptr()), None)
    lib = rst.load_library()
    k = ctypes.c_int64(0)
    rc = lib.rst_components_noalloc(c._h, ctypes.byref(g), ctypes.c_void_p(small.data_ptr()),
                                    ctypes.byref(k))
    assert rc == rst.RST_E_INVAL
