"""Side stream (config side_stream): the GEMM, near and moment work of an operator
application overlaps the far pair sum on a second stream; results must not change."""
import numpy as np
import pytest

from paper_2604_10089_amd import binding, inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_side_stream_is_bit_identical(prec):
    """K = 1, 3 and 6 densities, a GMRES solve each, an LCP solve and a time step: the
    side-stream context reproduces the one-stream context bit for bit (same kernels, same
    partial sums, the combination waits for both streams)."""
    w = inputs.workload('lattice27', 1)
    c = w['centers']
    axes = inputs.janus_axes(4, c.shape[0])
    out = {}
    for side in (False, True):
        with binding.Context(c, axes, 8, 16, lo=(4, 8), precision=prec, gmres_tol=1e-10,
                             side_stream=side) as ctx:
            r = []
            for K in (1, 3, 6):
                U, _ = ctx.mobility_apply_multi(inputs.random_forces(20 + K, c.shape[0], k=K))
                r.append(U)
            pairs, _ = ctx.find_contacts(0.1)
            if pairs.shape[0]:
                xs, ws = inputs.planted_lcp(2, pairs.shape[0])
                b = ws - ctx.lcp_apply(pairs, xs)
                r.append(ctx.lcp_solve(pairs, b, 'bi')[0])
            ctx.step(1e-3, 0.1, 'mono')
            r.append(ctx.get_state()[0])
            out[side] = r
    for a, b in zip(out[False], out[True]):
        assert np.array_equal(np.asarray(a), np.asarray(b))
