"""Error paths forced from the host, and the descriptor's allocator callbacks.

* PA_ERR_BREAKDOWN: CG breaks down when <p, M p> <= 0 (Sec. 3.1's PCG).
  With the field already the exact solution of its Backward Euler system
  (u = 0, zero boundary data, so b = 0 and r0 = 0) and a forced iteration
  count, the first direction is p = 0 and <p, M p> = 0: the device-side
  scalar kernel flags the breakdown and the call returns it.  The oracle
  reports the same condition.
* PA_ERR_ALLOC: an allocator callback that returns NULL, during pa_init
  (after k successful allocations, every one of them released again) and
  on a later lazy allocation (the weight of the full operator form).
* torch's caching allocator through the callbacks: the same results, bit
  for bit, as the library's own hipMalloc path, and the memory comes back
  when the context is destroyed.
"""
import gc

import numpy as np
import pytest

from paper_2403_01004_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_01004_amd import paradv
    paradv.load()
    return paradv


@pytest.mark.parametrize("op", ["aligned", "iso7"])
def test_breakdown_forced(dev, oracle_mod, op):
    prob = (inputs.conduction(7, 10, 16, seed=31) if op == "aligned"
            else inputs.viscosity(7, 10, 16, seed=32))
    prob.ub_in = np.zeros_like(prob.ub_in)
    prob.ub_out = np.zeros_like(prob.ub_out)
    zero = np.zeros_like(prob.u)
    g = dev.Operator.from_problem(prob)
    dt = 20.0 * g.dt_explicit()
    g.set_options(force_iters=2)
    u = g.bind(zero)
    st = g.advance_be(dt, 1e-10, 1, check=False)
    assert st["status"] == dev.PA_ERR_BREAKDOWN
    assert "breakdown" in dev.pa_last_error(g.ctx).lower()
    assert bool((u == 0).all())
    o = oracle_mod.Oracle.from_problem(prob)
    _, so = o.advance_be(zero, dt, 1e-10, 1, force_iters=2)
    assert so["status"] == 5
    # the context stays usable: an ordinary solve of the same system
    g.set_options()
    g.bind(zero)
    assert g.advance_be(dt, 1e-10, 1)["status"] == dev.PA_OK


class CountingAllocator:
    """torch's caching allocator that fails (returns 0) after `ok` calls."""

    def __init__(self, torch, ok):
        self.torch, self.ok = torch, ok
        self.live, self.calls, self.frees = set(), 0, 0

    def alloc(self, n):
        self.calls += 1
        if self.calls > self.ok:
            return 0
        p = self.torch.cuda.caching_allocator_alloc(n)
        self.live.add(p)
        return p

    def free(self, p):
        self.frees += 1
        self.live.remove(p)
        self.torch.cuda.caching_allocator_delete(p)


@pytest.mark.parametrize("ok", [0, 1, 7, 20])
def test_alloc_failure_at_init(dev, ok):
    import torch
    prob = inputs.conduction(6, 8, 12, seed=33)
    a = CountingAllocator(torch, ok)
    with pytest.raises(dev.PaError) as e:
        dev.Operator.from_problem(prob, allocator=(a.alloc, a.free))
    assert e.value.status == dev.PA_ERR_ALLOC
    gc.collect()
    assert a.calls > ok and not a.live and a.frees == min(ok, a.calls)


def test_alloc_failure_lazy(dev):
    import torch
    prob = inputs.viscosity(6, 8, 12, seed=34)
    a = CountingAllocator(torch, 10 ** 6)
    g = dev.Operator.from_problem(prob, allocator=(a.alloc, a.free))
    a.ok = a.calls          # every later allocation fails
    with pytest.raises(dev.PaError) as e:
        g.set_profile(w=np.ones(prob.mesh.shape))
    assert e.value.status == dev.PA_ERR_ALLOC
    del e, g    # the traceback holds the operator
    gc.collect()
    assert not a.live and a.frees == a.ok


@pytest.mark.parametrize("name", ["conduction", "viscosity"])
def test_torch_allocator(dev, name):
    import torch
    prob = (inputs.conduction(9, 14, 24, seed=35) if name == "conduction"
            else inputs.viscosity(9, 14, 24, seed=36))
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    outs = []
    for allocator in (None, "torch"):
        g = dev.Operator.from_problem(prob, allocator=allocator)
        if allocator == "torch":
            assert torch.cuda.memory_allocated() > base + 4 * 8 * prob.u.size
        dt = 40.0 * g.dt_explicit()
        u = g.bind(prob.u)
        g.advance_rkl2(dt, 0)
        g.advance_be(dt, 1e-10, 0)
        if name == "viscosity":
            g.set_options(pc=dev.PCS["bilu0"])   # allocates its pivots on first use
            g.advance_be(dt, 1e-10, 0)
        outs.append(u.cpu().numpy())
        del g, u
        gc.collect()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    assert np.array_equal(outs[0], outs[1])


def test_be_without_lazy_buffers(dev):
    """When the deferred x update's direction buffers and the row terms of
    the Jacobi diagonal cannot be allocated (every allocation after set-up
    fails), a BE advance still runs: x is updated in place every iteration
    and D is read per cell.  Its result matches the ordinary run's (same
    method, D equal up to rounding)."""
    import torch
    prob = inputs.viscosity(9, 10, 13, seed=37, vector=True)
    a = CountingAllocator(torch, 10 ** 6)
    g = dev.Operator.from_problem(prob, allocator=(a.alloc, a.free))
    a.ok = a.calls          # every later allocation fails
    dt = 30.0 * g.dt_explicit()
    u = g.bind(prob.u)
    st = g.advance_be(dt, 1e-13, 1)
    assert a.calls > a.ok   # the lazy allocations were tried
    assert not st["jacobi_rows"]
    ref = dev.Operator.from_problem(prob)
    v = ref.bind(prob.u)
    sr = ref.advance_be(dt, 1e-13, 1)
    assert sr["jacobi_rows"]
    assert abs(st["iters_total"] - sr["iters_total"]) <= 2
    x, y = u.cpu().numpy(), v.cpu().numpy()
    assert np.linalg.norm(x - y) <= 1e-12 * np.linalg.norm(y)
    del g, u, ref, v
    gc.collect()
    assert not a.live
