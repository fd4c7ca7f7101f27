"""GPU adjacency builder (sl_build_adjacency*) against the adjacency oracle
(paper Sec. 3.3.2, Sec. 3.3.3): integer outputs, so bit-exact."""
import ctypes

import numpy as np
import pytest

import meshgen
import oracle
from oracle.adjacency import adjacency
import paper_1502_00355_amd as sl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    sl.lib()
    yield


def same(a, b):
    return all(np.array_equal(np.asarray(x), np.asarray(y)) for x, y in zip(a, b))


CASES = {
    "one_triangle_isolated_nodes": (10, np.array([[5, 2, 9]])),
    "two_triangles": (4, np.array([[0, 1, 2], [2, 1, 3]])),
    "closed_star": (7, np.array([[0, i, i % 6 + 1] for i in range(1, 7)])),
    "edge_in_three": (7, np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4], [0, 2, 5], [0, 5, 3], [0, 4, 6]])),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_small_cases_equal_oracle(name):
    n, tris = CASES[name]
    print("adjacency", name, flush=True)
    assert same(sl.build_adjacency(n, tris), adjacency(n, tris))


@pytest.mark.parametrize("make", [
    lambda: meshgen.make_grid(13, "random", 0.3, 4),
    lambda: meshgen.make_grid(40, "unionjack", 0.2, 1),
    lambda: meshgen.make_annulus(9, 23, seed=2),
    lambda: meshgen.permute_mesh(meshgen.make_grid(31, "random", 0.4, 5), 7),
])
def test_meshes_equal_oracle(make):
    m = make()
    print("adjacency", m.name, flush=True)
    assert same(sl.build_adjacency(m.n_nodes, m.tris), adjacency(m.n_nodes, m.tris))


def test_large_permuted_grid_equals_generator_builder():
    """1024 x 1024, nodes and triangles shuffled: equals the generators'
    C builder (an implementation independent of the device one, pinned to
    the oracle on smaller meshes)."""
    m = meshgen.permute_mesh(meshgen.make_grid(1024, "random", 0.4, 2), 2)
    got = sl.build_adjacency(m.n_nodes, m.tris)
    assert same(got, (m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.boundary))


def test_device_variant_and_triangles_in_smoothing():
    """Triangles in: the device builds the adjacency and smooths; the result
    equals the oracle's on the generator's arrays."""
    import torch
    m = meshgen.make_grid(200, "random", 0.4, 21)
    tris = torch.from_numpy(np.ascontiguousarray(m.tris, dtype=np.int32)).cuda()
    nbr_ptr, nbr_idx, tri_ptr, tri_idx, bnd = sl.build_adjacency_device(tris, m.n_nodes)
    torch.cuda.synchronize()
    assert same((nbr_ptr.cpu(), nbr_idx.cpu(), tri_ptr.cpu(), tri_idx.cpu(), bnd.cpu()),
                (m.nbr_ptr, m.nbr_idx, m.tri_ptr, m.tri_idx, m.boundary))
    X = torch.from_numpy(m.coords.copy()).cuda()
    rep = sl.smooth_mesh_device(X, nbr_ptr, nbr_idx, tri_ptr, tri_idx, tris.reshape(-1), bnd, iterations=12)
    torch.cuda.synchronize()
    ref = oracle.smooth(m, 12)
    assert rep.iterations_run == 12
    assert (X.cpu().numpy() == ref.coords).all()


def test_errors_leave_outputs_untouched():
    L = sl.lib()
    n = 6
    nbr_ptr = np.full(n + 1, -7, np.int32)
    nbr_idx = np.full(64, -7, np.int32)
    tri_ptr = np.full(n + 1, -7, np.int32)
    tri_idx = np.full(64, -7, np.int32)
    bnd = np.full(n, 9, np.uint8)
    nnz = ctypes.c_int64(0)

    def call(tris, cap=64):
        t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1)
        return L.sl_build_adjacency(t.ctypes.data, t.size // 3, n, nbr_ptr.ctypes.data, nbr_idx.ctypes.data, cap,
                                    tri_ptr.ctypes.data, tri_idx.ctypes.data, bnd.ctypes.data, ctypes.byref(nnz))

    assert call([[0, 1, 6]]) == sl.SL_EINVAL
    assert call([[0, 1, -1]]) == sl.SL_EINVAL
    assert call([[0, 1, 1]]) == sl.SL_ETOPO
    assert call([[0, 1, 2], [2, 1, 3]], cap=5) == sl.SL_EINVAL
    assert nnz.value == 10 and b"10 are needed" in L.sl_last_error()
    assert (nbr_ptr == -7).all() and (nbr_idx == -7).all() and (tri_ptr == -7).all() and (tri_idx == -7).all()
    assert (bnd == 9).all()
    assert call([[0, 1, 2], [2, 1, 3]], cap=10) == sl.SL_OK
    assert nnz.value == 10 and nbr_ptr[-1] == 10 and (bnd == 1).all()
