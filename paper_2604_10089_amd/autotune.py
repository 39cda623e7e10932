"""Autotuner for the far pair-sum launch shape.

For one workload (sphere count M, grid, precision, densities per pass K) it
times every candidate launch shape -- block layout (256 targets per block with
one or two targets per thread, or 64 targets per block whose four waves split
the sources) and number of source-sphere chunks (grid y) -- with the library's
own HIP-event timing of the far kernel over one full mobility product, and
records the fastest in a JSON cache keyed by the device architecture.
`Context` consults the cache when its caller does not fix the launch shape.

Usage (on a GPU): python -m paper_2604_10089_amd.autotune [--workload rsa216] [--K 1 6] [--prec mixed fp64]
                  python -m paper_2604_10089_amd.autotune --batch [--prec mixed fp64]
"""
import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_DIR = os.path.join(HERE, 'tuning')


def arch_name():
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(':')[0]
    except Exception:
        return 'gfx950'


def key(prec, K, M, n):
    """Cache key: precision, densities per pass, sphere count bucket (powers of 2) and nodes per sphere."""
    mb = 1 << max(0, int(np.ceil(np.log2(max(M, 1)))))
    return f'{prec}-K{K}-M{mb}-n{n}'


def cache_path(arch=None):
    return os.path.join(CACHE_DIR, f'{arch or arch_name()}.json')


def load(arch=None):
    p = cache_path(arch)
    if os.path.exists(p):
        with open(p) as f:
            return json.load(f)
    return {}


def lookup(prec, K, M, n, arch='gfx950'):
    """(tpt, chunks, split) from the cache, or None."""
    e = load(arch).get(key(prec, K, M, n))
    return None if e is None else (e['tpt'], e['chunks'], e.get('split', 0))


def batch_key(prec, instances):
    """Cache key of a batch of suspensions: precision, instance count and total nodes (powers of 2)."""
    nodes = sum(c.shape[0] * nt * nph for c, nt, nph in instances)
    nb = 1 << max(0, int(np.ceil(np.log2(max(nodes, 1)))))
    ib = 1 << max(0, int(np.ceil(np.log2(max(len(instances), 1)))))
    return f'batch-{prec}-I{ib}-N{nb}'


def lookup_batch(prec, instances, arch='gfx950'):
    """(tpt, chunks, split) of a batch of suspensions from the cache, or None."""
    e = load(arch).get(batch_key(prec, instances))
    return None if e is None else (e['tpt'], e['chunks'], e.get('split', 0))


def tune_batch(instances, prec, seed=0, verbose=True):
    """Every candidate shape of the segmented far launch of a batch context (one density per
    suspension), timed by the library's HIP events over one full batched mobility product."""
    from paper_2604_10089_amd import binding, inputs
    FT = [inputs.random_forces(seed + b, c.shape[0]) for b, (c, _, _) in enumerate(instances)]
    cands = [(t, c, 0) for t in (1, 2) for c in (0, 1, 2, 3, 4, 6, 9)]
    if prec == 'mixed':
        cands += [(1, c, 1) for c in (0, 1, 2, 3, 4, 6, 9)]
    best, rows = None, []
    for tpt, ch, sp in cands:
        with binding.BatchContext(instances, gmres_tol=1e-8, precision=prec, tpt=tpt, far_chunks=ch, far_split=sp,
                                  profile=True) as bc:
            bc.mobility_apply(FT)                       # warm-up
            _, st = bc.mobility_apply(FT)
        t = st['t_far_ms'] / max(st['n_far'], 1)
        rows.append((tpt, ch, sp, t))
        if verbose:
            print(f'  tpt={tpt} split={sp} chunks={ch or "auto"}: {t:.4f} ms per far launch', flush=True)
        if best is None or t < best[3]:
            best = (tpt, ch, sp, t)
    return best, rows


def candidates(M, K, prec):
    tpts = (1, 2) if K <= 2 else (1,)
    chunks = sorted({0} | {c for c in (2, 4, 6, 8, 12, 16, 24, 32, 48, 64) if c <= M})
    out = [(t, c, 0) for t in tpts for c in chunks]
    if prec == 'mixed':  # the split layout exists for the FP32 pair sum
        out += [(1, c, 1) for c in chunks]
    return out


def tune(centers, n_theta, n_phi, prec, K, seed=0, verbose=True):
    from paper_2604_10089_amd import binding, inputs
    M = centers.shape[0]
    FT = inputs.random_forces(seed, M, k=K)
    best = None
    rows = []
    for tpt, ch, sp in candidates(M, K, prec):
        with binding.Context(centers, None, n_theta, n_phi, gmres_tol=1e-8, precision=prec, tpt=tpt,
                             far_chunks=ch, far_split=sp, profile=True) as ctx:
            ctx.mobility_apply_multi(FT)                # warm-up
            _, st = ctx.mobility_apply_multi(FT)
        t = st['t_far_ms'] / max(st['n_far'], 1)
        rows.append((tpt, ch, sp, t))
        if verbose:
            print(f'  tpt={tpt} split={sp} chunks={ch or "auto"}: {t:.4f} ms per far launch', flush=True)
        if best is None or t < best[3]:
            best = (tpt, ch, sp, t)
    return best, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--workload', default='rsa216')
    ap.add_argument('--K', type=int, nargs='+', default=[1, 6])
    ap.add_argument('--prec', nargs='+', default=['mixed', 'fp64'])
    ap.add_argument('--batch', action='store_true',
                    help='tune the batch context of the 32 uneven suspensions instead of one workload')
    args = ap.parse_args()
    from paper_2604_10089_amd import inputs
    arch = arch_name()
    cache = load(arch)
    if args.batch:
        inst = inputs.batched_suspensions(0)
        for prec in args.prec:
            print(f'batch of {len(inst)} suspensions, {prec}', flush=True)
            (tpt, ch, sp, t), rows = tune_batch(inst, prec)
            cache[batch_key(prec, inst)] = dict(
                tpt=tpt, chunks=ch, split=sp, far_ms=round(t, 5), workload='batched_suspensions(0)',
                sweep=[dict(tpt=a, chunks=b, split=z, far_ms=round(x, 5)) for a, b, z, x in rows])
            print(f'  best tpt={tpt} split={sp} chunks={ch or "auto"} {t:.4f} ms', flush=True)
        os.makedirs(CACHE_DIR, exist_ok=True)
        with open(cache_path(arch), 'w') as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        print('wrote', cache_path(arch))
        return
    w = inputs.workload(args.workload, 0)
    c = w['centers']
    for prec in args.prec:
        for K in args.K:
            print(f'{args.workload} {prec} K={K}', flush=True)
            t0 = time.time()
            (tpt, ch, sp, t), rows = tune(c, w['n_theta'], w['n_phi'], prec, K)
            cache[key(prec, K, c.shape[0], w['n_theta'] * w['n_phi'])] = dict(
                tpt=tpt, chunks=ch, split=sp, far_ms=round(t, 5), workload=args.workload,
                sweep=[dict(tpt=a, chunks=b, split=z, far_ms=round(x, 5)) for a, b, z, x in rows])
            print(f'  best tpt={tpt} split={sp} chunks={ch or "auto"} {t:.4f} ms ({time.time() - t0:.1f} s)',
                  flush=True)
    os.makedirs(CACHE_DIR, exist_ok=True)
    with open(cache_path(arch), 'w') as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    print('wrote', cache_path(arch))


if __name__ == '__main__':
    main()
