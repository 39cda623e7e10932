"""Device memory through a caller's provider (pqn_config_desc.dev_alloc / dev_free)."""
import numpy as np
import pytest

from paper_2604_10089_amd import binding, inputs

pytestmark = pytest.mark.gpu


def _run(ctx, c, FT):
    U, _ = ctx.mobility_apply_multi(FT)
    pairs, _ = ctx.find_contacts(0.1)
    xs, ws = inputs.planted_lcp(0, pairs.shape[0])
    b = ws - ctx.lcp_apply(pairs, xs)
    # two contacts first, then all of them: the LCP buffers grow between the calls
    x2, _ = ctx.lcp_solve(pairs[:2], b[:2], 'bi')
    x, _ = ctx.lcp_solve(pairs, b, 'bi')
    return U, x2, x


def test_torch_caching_allocator_gives_identical_results():
    """Every device buffer taken from the PyTorch caching allocator on the context's
    stream: results equal those with hipMalloc'd buffers bit for bit, the allocator
    holds the context's memory while it lives, and every block (including those
    replaced when the LCP buffers grow) is returned by pqn_destroy."""
    import torch
    c = inputs.workload('tiny', 0)['centers']
    FT = inputs.random_forces(1, c.shape[0], k=3)
    with binding.Context(c, None, 8, 16, lo=(4, 8)) as ref:
        U0, x20, x0 = _run(ref, c, FT)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    ctx = binding.Context(c, None, 8, 16, lo=(4, 8), torch_alloc=True)
    held = torch.cuda.memory_allocated() - before
    U1, x21, x1 = _run(ctx, c, FT)
    assert ctx._alloc.live > 0
    ctx.close()
    torch.cuda.synchronize()
    assert held > 0
    assert ctx._alloc.live == 0
    assert torch.cuda.memory_allocated() == before
    assert all(np.array_equal(a, b) for a, b in zip(U0, U1))
    assert np.array_equal(x20, x21) and np.array_equal(x0, x1)


def test_torch_caching_allocator_batch():
    """The same provider for a batch context: results equal the hipMalloc batch."""
    import torch
    inst = [(inputs.workload('tiny', s)['centers'], 8, 16) for s in (0, 1, 2)]
    FT = [inputs.random_forces(10 + s, 8) for s in range(3)]
    with binding.BatchContext(inst) as b0:
        U0, _ = b0.mobility_apply(FT)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    b1 = binding.BatchContext(inst, torch_alloc=True)
    U1, _ = b1.mobility_apply(FT)
    b1.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    assert all(np.array_equal(a, b) for a, b in zip(U0, U1))
