"""Host logic of the far-launch autotuner: cache keys, the recorded choice, and that the
timed configurations (216 spheres on the 12 x 24 grid, one and six densities per pass; the
32-suspension batch) are found in the shipped cache."""
import numpy as np
import pytest

from paper_2604_10089_amd import autotune, binding, inputs


def test_keys_bucket_sphere_and_node_counts_to_powers_of_two():
    assert autotune.key('mixed', 6, 216, 288) == 'mixed-K6-M256-n288'
    assert autotune.key('fp64', 1, 256, 288) == 'fp64-K1-M256-n288'
    assert autotune.key('fp64', 1, 257, 288) == 'fp64-K1-M512-n288'
    assert autotune.key('mixed', 1, 1, 128) == 'mixed-K1-M1-n128'
    c = np.zeros((10, 3))
    assert autotune.batch_key('mixed', [(c, 8, 16)]) == 'batch-mixed-I1-N2048'       # 1,280 nodes
    assert autotune.batch_key('fp64', [(c, 8, 16)] * 3) == 'batch-fp64-I4-N4096'     # 3,840 nodes


@pytest.mark.parametrize("entry", sorted(autotune.load('gfx950')))
def test_cached_choice_is_the_fastest_swept_shape(entry):
    e = autotune.load('gfx950')[entry]
    assert e['tpt'] in (1, 2) and e['chunks'] >= 0 and e.get('split', 0) in (0, 1)
    best = min(e['sweep'], key=lambda s: s['far_ms'])
    assert (e['tpt'], e['chunks'], e.get('split', 0)) == (best['tpt'], best['chunks'], best.get('split', 0))
    assert e['far_ms'] == best['far_ms']


def test_timed_configurations_hit_the_cache():
    w = inputs.workload('rsa216', 0)
    M, n = w['centers'].shape[0], w['n_theta'] * w['n_phi']
    for prec in ('mixed', 'fp64'):
        for K in (1, 6):
            hit = autotune.lookup(prec, K, M, n)
            assert hit is not None, (prec, K)
            assert binding.tuned_shape(prec, K, M, n) == hit
    inst = inputs.batched_suspensions(0)
    assert len(inst) == 32
    for prec in ('mixed', 'fp64'):
        assert autotune.lookup_batch(prec, inst) is not None, prec


def test_unknown_shapes_fall_back_to_the_library_default():
    assert autotune.lookup('mixed', 6, 4096, 288) is None
    assert binding.tuned_shape('mixed', 6, 4096, 288) == (2, 0, 0)
    assert autotune.lookup_batch('mixed', [(np.zeros((8, 3)), 8, 16)]) is None
