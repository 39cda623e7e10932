"""Benchmark: mobility MVPs/s and GPair-evals/s on the 216-sphere suspension.

One timed step = one complete high-fidelity mobility product U = M F (random
forces and torques already resident in HBM, GMRES to 1e-8, mixed precision:
FP32 far pair sums, FP64 everything else) on 216 spheres of radius 1 at volume
fraction 0.3 with 12x24 nodes per sphere (62,208 nodes). The same JSON line
reports the plain FP64 path, the mixed-vs-FP64 error of every velocity block,
the far pair-sum kernel against the FP32 vector roofline (HIP events on the
library's stream), one Bi-PQN LCP solve with a planted solution on the
suspension's contact set (low fidelity 6x12), and the CPU oracle's rate on a
bounded sample of the same operator.

Usage: python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu-baseline] [--no-lcp]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3      # TFLOP/s, MI355X FP32 vector (vendor figure, packed issue)
PEAK_FP32_NONPACKED = 78.6    # TFLOP/s, 256 CU x 64 lanes x 2 flop x 2.4 GHz (no packed FP32)
FLOP_PER_PAIR = 30            # algorithmic flops of one far pair evaluation (single right-hand side)


def far_pairs(centers, n, near_gap=0.5, radius=1.0):
    c = np.asarray(centers)
    d = np.linalg.norm(c[:, None] - c[None], axis=2) - 2 * radius
    M = c.shape[0]
    near = (d < near_gap).sum() - M      # ordered near pairs (diagonal excluded)
    far = M * (M - 1) - near
    return far * n * n, near * n * (4 * n)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=10)
    ap.add_argument('--warmup', type=int, default=2)
    ap.add_argument('--seed', type=int, default=0)
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-lcp', action='store_true')
    ap.add_argument('--tpt', type=int, default=2)
    ap.add_argument('--chunks', type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f'bench.py measures one GPU: --gpus {args.gpus} is not supported (the path runs on one MI355X; '
              'multi-GPU sharding is a design note only)', file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_10089_amd import binding, inputs

    dev = torch.device('cuda:0')
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    w = inputs.workload('rsa216', args.seed)
    c = w['centers']
    M = c.shape[0]
    nt, nph = w['n_theta'], w['n_phi']
    n = nt * nph
    K, W = args.steps, args.warmup
    FTs = [torch.tensor(inputs.random_forces(100 + k, M), dtype=torch.float64, device=dev) for k in range(max(K, 1))]
    UO = torch.zeros((M, 6), dtype=torch.float64, device=dev)

    def ctx_for(prec, profile):
        return binding.Context(c, None, nt, nph, lo=w['lo'], gmres_tol=1e-8, precision=prec, tpt=args.tpt,
                               far_chunks=args.chunks, stream=stream.cuda_stream, profile=profile)

    res = {}
    for prec in ('mixed', 'fp64'):
        ctx = ctx_for(prec, True)
        for k in range(W):
            ctx.mobility_apply_dev(FTs[k % len(FTs)].data_ptr(), UO.data_ptr())
        steps = K if prec == 'mixed' else max(2, K // 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = far_ms = nfar = 0
        for k in range(steps):
            st = ctx.mobility_apply_dev(FTs[k % len(FTs)].data_ptr(), UO.data_ptr())
            its += st['gmres_iters']
            far_ms += st['t_far_ms']
            nfar += st['n_far']
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res[prec] = dict(steps=steps, sec=t1 - t0, gmres_iters=its / steps, far_ms=far_ms / max(nfar, 1),
                         matvecs_per_mvp=nfar / steps)
        print(f'[bench] {prec}: {steps} MVPs in {t1 - t0:.3f} s, {its / steps:.1f} GMRES its/MVP, '
              f'far kernel {far_ms / max(nfar, 1):.3f} ms/launch', file=sys.stderr, flush=True)
        ctx.close()

    # accuracy of mixed vs FP64 on the same forces (per velocity block)
    errs = []
    cm, cf = ctx_for('mixed', False), ctx_for('fp64', False)
    for k in range(2):
        F = FTs[k].cpu().numpy()
        Um, _ = cm.mobility_apply(F)
        Uf, _ = cf.mobility_apply(F)
        for blk in (slice(0, 3), slice(3, 6)):
            errs.append(float(np.abs(Um[:, blk] - Uf[:, blk]).max() / np.abs(Uf[:, blk]).max()))
    cf.close()

    lcp_info = None
    if not args.no_lcp:
        pairs, gaps = cm.find_contacts(0.1)
        xs, ws = inputs.planted_lcp(args.seed, pairs.shape[0])
        b = ws - cm.lcp_apply(pairs, xs)
        t0 = time.perf_counter()
        x, ls = cm.lcp_solve(pairs, b, 'bi')
        t1 = time.perf_counter()
        x2, lm = cm.lcp_solve(pairs, b, 'mono')
        lcp_info = dict(n_contacts=int(pairs.shape[0]), bi_sec=t1 - t0, bi_mvp_hi=ls['mvp_hi'],
                        bi_mvp_lo=ls['mvp_lo'], bi_emvp=round(ls['emvp'], 2),
                        lo_hi_cost_ratio=round(ls['lo_hi_cost_ratio'], 4),
                        bi_x_rel_err=float(np.abs(x - xs).max() / np.abs(xs).max()),
                        mono_mvp=lm['mvp_hi'], mono_sec=lm['t_total_ms'] / 1e3,
                        mono_x_rel_err=float(np.abs(x2 - xs).max() / np.abs(xs).max()))
        print(f'[bench] Bi-PQN planted LCP n={pairs.shape[0]}: {ls["mvp_hi"]} hi + {ls["mvp_lo"]} lo MVPs, '
              f'{t1 - t0:.3f} s', file=sys.stderr, flush=True)
    cm.close()

    pf, pn = far_pairs(c, n)
    mixed = res['mixed']
    mvps = mixed['steps'] / mixed['sec']
    pairs_per_mvp = mixed['matvecs_per_mvp'] * pf
    achieved = FLOP_PER_PAIR * pf / (mixed['far_ms'] * 1e-3) / 1e12
    fp64 = res['fp64']
    out = {
        'metric': 'mobility MVPs/s (216 spheres, mixed FP32/FP64, GMRES 1e-8)',
        'value': round(mvps, 4),
        'unit': 'MVP/s',
        'n_gpus': 1, 'steps': K, 'warmup': W,
        'ms_per_step': round(1e3 * mixed['sec'] / mixed['steps'], 3),
        'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None,
        'dtype': 'f32+f64', 'data': 'synthetic',
        'config': {'workload': 'rsa216: 216 spheres a=1, RSA phi=0.3, 12x24 nodes (62,208), near gap 0.5, '
                               'random F,T, GMRES tol 1e-8', 'n_nodes': M * n, 'far_pairs_per_matvec': int(pf)},
        'gpair_evals_per_s': round(pairs_per_mvp * mvps / 1e9, 2),
        'fp64_mvps_per_s': round(fp64['steps'] / fp64['sec'], 4),
        'speedup_mixed_vs_fp64': round(mvps / (fp64['steps'] / fp64['sec']), 3),
        'mixed_rel_err_vs_fp64': {'max_translation': max(errs[0::2]), 'max_rotation': max(errs[1::2])},
        'gmres_iters_per_mvp': {'mixed': mixed['gmres_iters'], 'fp64': fp64['gmres_iters']},
        'far_kernel_ms': {'mixed_fp32': round(mixed['far_ms'], 4), 'fp64': round(fp64['far_ms'], 4)},
        'roofline': {'bound': 'alu', 'kernel': 'k_far32', 'achieved': round(achieved, 3),
                     'peak': PEAK_FP32_VECTOR, 'unit': 'TFLOP/s', 'frac': round(achieved / PEAK_FP32_VECTOR, 4),
                     'frac_of_nonpacked_peak': round(achieved / PEAK_FP32_NONPACKED, 4), 'traffic': None},
        'lcp': lcp_info,
    }
    if not args.no_cpu_baseline:
        out['cpu_baseline'] = cpu_baseline(w, c, nt, nph, mixed)
    print(json.dumps(out), flush=True)


def cpu_baseline(w, c, nt, nph, mixed):
    """The oracle's operator rows on a bounded sample of targets, scaled to one MVP."""
    from oracle import bie
    g = bie.Geometry(c, 1.0, nt, nph)
    q = np.random.default_rng(0).standard_normal((g.N, 3))
    rng = np.random.default_rng(1)
    tg = sorted(rng.choice(g.N, size=64, replace=False).tolist())
    bie.operator_rows(g, q, tg[:2])        # warm caches of the self rows and near blocks touched
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < 15.0 and k < len(tg):
        bie.operator_rows(g, q, [tg[k]])
        k += 1
    dt = (time.perf_counter() - t0) / k
    matvec_s = dt * g.N
    mvp_s = matvec_s * mixed['matvecs_per_mvp']
    return {'value': round(1.0 / mvp_s, 8), 'unit': 'MVP/s', 'cores': 1, 'kind': 'oracle',
            'sample': f'{k} operator rows of the 216-sphere operator (one target node against all '
                      f'62,208 sources each), scaled by N = {g.N} rows per matvec and '
                      f'{mixed["matvecs_per_mvp"]:.1f} matvecs per MVP'}


if __name__ == '__main__':
    main()
