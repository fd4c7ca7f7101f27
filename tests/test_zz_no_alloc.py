"""GPU test of smooth_mesh_device_noalloc, the entry point that allocates no
device memory: called through the C ABI, it must give what
smooth_mesh_device gives on the same inputs -- accept flags of every sweep
bit-exact, coordinates within 1e-12 (bit-exact expected and asserted) --
on two calls in a row, the second with a smaller mesh, since the calls share
one static workspace per device."""
import numpy as np
import pytest

import meshgen
import oracle
import paper_1502_00355_amd as sl

pytestmark = pytest.mark.gpu
COORD_TOL = 1e-12


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    sl.lib()
    yield


def run(fn, m, iters, tol=0.0, **opts):
    import torch
    dev = sl.to_device(m, "cuda:0")
    flags = torch.zeros(max(iters, 1) * ((m.n_nodes + 7) // 8), dtype=torch.uint8, device="cuda:0")
    rep = fn(*dev, iterations=iters, tol=tol, flags=flags, **opts)
    torch.cuda.synchronize()
    F = sl.unpack_flags(flags.cpu().numpy().reshape(max(iters, 1), -1), m.n_nodes)
    return dev[0].cpu().numpy(), rep, F[:rep.iterations_run]


def same(a, b):
    (Xa, ra, Fa), (Xb, rb, Fb) = a, b
    assert ra.iterations_run == rb.iterations_run
    assert ra.accepted_total == rb.accepted_total
    assert ra.kernel_used == rb.kernel_used
    assert (Fa == Fb).all()
    assert float(np.abs(Xa - Xb).max()) <= COORD_TOL
    assert (Xa == Xb).all()


@pytest.mark.parametrize("opts", [{}, {"form": "colored"}, {"layout": "soa", "accept": "gt"}, {"kernel": "node"},
                                  {"precision": "f32"}])
def test_noalloc_equals_the_device_entry_point(opts):
    """A 90,000-node mesh, then a 3,249-node one: each equals
    smooth_mesh_device's result, and the first also the oracle's."""
    big = meshgen.make_grid(300, "random", 0.4, 41)
    small = meshgen.make_grid(57, "random", 0.35, 42)
    for k, (m, iters) in enumerate(((big, 40), (small, 25))):
        print("noalloc %s: %d nodes, %d sweeps" % (opts, m.n_nodes, iters), flush=True)
        na = run(sl.smooth_mesh_device_noalloc, m, iters, **opts)
        same(na, run(sl.smooth_mesh_device, m, iters, **opts))
        if k == 0:
            form = "colored" if opts.get("form") == "colored" else "jacobi"
            ref = oracle.smooth(m, iters, threads=oracle.max_threads(), accept_gt=opts.get("accept") == "gt",
                                form=form, precision=opts.get("precision", "f64"))
            assert (na[2] == (ref.flags == 1)).all()
            assert (na[0] == ref.coords).all()


def test_noalloc_tolerance_then_smaller():
    """A run that stops on its tolerance, then a smaller mesh with more sweeps."""
    m1 = meshgen.make_grid(200, "random", 0.4, 43)
    m2 = meshgen.make_grid(40, "unionjack", 0.3, 44)
    same(run(sl.smooth_mesh_device_noalloc, m1, 5000, 1e-9), run(sl.smooth_mesh_device, m1, 5000, 1e-9))
    same(run(sl.smooth_mesh_device_noalloc, m2, 70), run(sl.smooth_mesh_device, m2, 70))


def test_noalloc_refuses_a_mesh_beyond_its_workspace():
    """A 2.25M-node mesh needs more than the static workspace: SL_ENOMEM before
    any work, coordinates untouched; the next call still works."""
    import torch
    m = meshgen.make_grid(1500, "random", 0.4, 45)
    dev = sl.to_device(m, "cuda:0")
    before = dev[0].clone()
    with pytest.raises(sl.SmartlapError) as e:
        sl.smooth_mesh_device_noalloc(*dev, iterations=3)
    assert e.value.status == sl.SL_ENOMEM and "workspace" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(dev[0], before)
    small = meshgen.make_grid(33, "random", 0.4, 46)
    same(run(sl.smooth_mesh_device_noalloc, small, 12), run(sl.smooth_mesh_device, small, 12))
