"""Benchmark: batched mobility MVPs/s and GPair-evals/s on the 216-sphere suspension.

One timed step = one batched mobility product of K = 6 independent force sets
U_r = M F_r on 216 spheres of radius 1 at volume fraction 0.3 with 12x24 nodes
per sphere (62,208 nodes): six GMRES solves (tolerance 1e-8) in lockstep whose
pair sums share one geometry pass, mixed precision (FP32 far pair sums, FP64
everything else), forces and velocities resident in HBM (the device-pointer
entry point). value = force sets per second.

The same JSON line reports: the single-force-set rate and the plain FP64 path
(both K = 1 and K = 6), the mixed-vs-FP64 error of every velocity block, the
far pair-sum kernel against the FP32 vector roofline (HIP events on the
library's stream), the 32-suspension uneven batch (one far launch per GMRES
iteration) against the same suspensions one by one, the LCP solvers on a
planted LCP of the suspension's contact set (low fidelity 6x12), ten Janus
time steps at dt 1e-3, five time steps with active contacts (axes towards the
centroid, dt 0.1) with every solver replayed on their LCPs, and the CPU
oracle's rate on a bounded sample of the same operator (one core and all
cores).

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--no-cpu-baseline] [--no-lcp] [--no-batch]
       [--no-steps] [--serial]; short runs for profilers: --counters-probe, --batch-probe, --contact-probe;
       --lcp-table for the solver comparison on three workloads.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR = 157.3      # TFLOP/s, MI355X FP32 vector FMA (256 CU x 128 lanes/clk x 2 flop x 2.4 GHz)
PEAK_FP64_VECTOR = 78.6       # TFLOP/s, MI355X FP64 vector FMA
K_RHS = 6
PROBE_BYTES = 256 << 20       # reference copy for the HBM byte counters

# HBM bytes of one far FP32 launch with six densities from rocprofv3 --pmc
# FETCH_SIZE / WRITE_SIZE (profiles/k_far32_rsa216_hbm_traffic.md), scaled by what
# the counters read for a 256 MiB copy (FETCH_SIZE x2.0, WRITE_SIZE x1.0). Valid
# only for the far-kernel source and the launch layout it was measured on:
# reported as null once either changes.
FAR_TRAFFIC = {'kernel': 'k_far32<1,6>', 'source_sha1': '1ac17695bb37f029b69c85c9b6eee64ae41547e1',
               'layout': {'tpt': 1, 'chunks': 24, 'split': 0},
               'fetch_kib': 6324.1, 'write_kib': 209952.0, 'fetch_scale': 2.0, 'write_scale': 1.0}


def far_source_sha1():
    import hashlib
    src = open(os.path.join(ROOT, 'paper_2604_10089_amd', 'csrc', 'kernels.hip')).read()
    a = src.index('// ----------------------------------------------------------- far pair sum')
    b = src.index('template <int K>\n__device__ __forceinline__ void far64_body')
    return hashlib.sha1(src[a:b].encode()).hexdigest()


def far_traffic_bytes(layout):
    t = FAR_TRAFFIC
    if t['fetch_kib'] is None or far_source_sha1() != t['source_sha1'] or layout != t['layout']:
        return None
    return int(1024 * (t['fetch_kib'] * t['fetch_scale'] + t['write_kib'] * t['write_scale']))


def far_kernel_name(layout, K):
    """Name of the far FP32 kernel a launch layout {tpt, chunks, split} runs for K densities."""
    if layout['split']:
        return f'k_far32s<{K}>'
    return f'k_far32<{layout["tpt"] if K <= 2 else 1},{K}>'


def pc_blocks(c, near_gap=0.5, radius=1.0):
    """Blocks of the preconditioner: one per sphere with a near partner (gap < near_gap) and one
    per ordered near pair."""
    d = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=2) - 2 * radius
    np.fill_diagonal(d, np.inf)
    near = d < near_gap
    return int(near.any(axis=1).sum() + near.sum())


def precond_bytes(n, L, nblocks):
    """HBM bytes of one preconditioner application: the FP16 blocks (3n x 3L each, n nodes and
    L harmonic coefficients per sphere), streamed once."""
    return int(nblocks * (3 * n) * (3 * L) * 2)


def flop_per_pair(K):
    """Algorithmic flops of one far pair with K densities (FMA = 2, rsqrt = 1): 18 shared + 12 per density."""
    return 18 + 12 * K


def far_pairs(centers, n, near_gap=0.5, radius=1.0):
    c = np.asarray(centers)
    d = np.linalg.norm(c[:, None] - c[None], axis=2) - 2 * radius
    M = c.shape[0]
    near = (d < near_gap).sum() - M      # ordered near pairs (diagonal excluded)
    far = M * (M - 1) - near
    return far * n * n


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=5)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--seed', type=int, default=0)
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-lcp', action='store_true')
    ap.add_argument('--no-batch', action='store_true')
    ap.add_argument('--no-steps', action='store_true')
    ap.add_argument('--tpt', type=int, default=None, help='targets per thread (default: autotuned)')
    ap.add_argument('--chunks', type=int, default=None, help='far source chunks (default: autotuned)')
    ap.add_argument('--split', type=int, default=None, choices=(0, 1),
                    help='far FP32 split layout, 64 targets per block (default: autotuned)')
    ap.add_argument('--no-precond', action='store_true',
                    help='plain GMRES everywhere (default: the near-patch preconditioner on every '
                         'single-suspension context; the headline is also measured without it)')
    ap.add_argument('--no-coarse', action='store_true',
                    help='one-level preconditioner (default: two levels, a coarse correction on every '
                         "sphere's degree <= 2 harmonics before the near patches, on every preconditioned "
                         'single-suspension context; the headline is also measured with one level)')
    ap.add_argument('--serial', action='store_true',
                    help='one stream everywhere (no side stream beside the far pair sum): every kernel runs '
                         'alone, as in the profiles of individual kernels')
    ap.add_argument('--counters-probe', action='store_true',
                    help='short run for rocprofv3 --pmc: a 256 MiB device copy (scale reference for FETCH_SIZE/'
                         'WRITE_SIZE) and one six-force-set product on the 216-sphere workload')
    ap.add_argument('--batch-probe', action='store_true',
                    help='short run for rocprofv3 --kernel-trace: only the 32-suspension batch, mixed precision, '
                         'preconditioned (with --no-precond: plain GMRES iterations from captured graphs); one '
                         'warm-up product and three timed ones, one JSON line')
    ap.add_argument('--contact-probe', action='store_true',
                    help='short run for rocprofv3 --kernel-trace: only the five time steps with active contacts '
                         '(FP64, then the mixed replay), one JSON line')
    ap.add_argument('--cpu-table', action='store_true',
                    help='instead of the benchmark line: the CPU oracle timed on the host cores on the 8-sphere '
                         '(full MVP and Mono-PQN LCP with the assembled operator), 27-, 64- and 216-sphere '
                         'workloads (one matvec over all cores), beside the GPU path on the same inputs')
    ap.add_argument('--lcp-table', action='store_true',
                    help='instead of the benchmark line: BB-PGD, Mono-PQN and Bi-PQN on planted LCPs of the 27-, '
                         '64- and 216-sphere workloads (three seeds each), one JSON line')
    args = ap.parse_args()
    if args.gpus != 1:
        print(f'bench.py measures one GPU: --gpus {args.gpus} is not supported (the path runs on one MI355X; '
              'multi-GPU sharding is a design note only)', file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_10089_amd import binding, inputs

    def log(*a):
        print('[bench]', *a, file=sys.stderr, flush=True)

    dev = torch.device('cuda:0')
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    w = inputs.workload('rsa216', args.seed)
    c = w['centers']
    M = c.shape[0]
    nt, nph = w['n_theta'], w['n_phi']
    n = nt * nph
    K, W = args.steps, args.warmup
    pf = far_pairs(c, n)

    PC = not args.no_precond
    # the preconditioner: built at the first solve where a configuration serves many products
    # (the MVP passes and LCP solves), when a configuration is solved a second time in the
    # time steps (a step without contacts solves once and never pays for the set-up)
    PC_FIXED = 'eager' if PC else False
    PC_COARSE = PC and not args.no_coarse

    def ctx_for(prec, kr=K_RHS, profile=True, warm_start=False, side=None, precond=None, coarse=None):
        """Context with the launch layout tuned for kr densities per pass (unless fixed on the command line).
        side: run the GEMM / near / moment work on a second stream beside the far pair sum (default: for the
        mixed path, where it measured 5-7% faster; the FP64 K = 6 pass was 2.5% slower with it). Profiled
        contexts time the far kernel alone and keep one stream. precond: right-preconditioned GMRES
        (default: on unless --no-precond); coarse: its two-level form (default: on unless --no-coarse)."""
        if side is None:
            side = prec == 'mixed' and not profile and not args.serial
        return binding.Context(c, None, nt, nph, lo=w['lo'], gmres_tol=1e-8, precision=prec, tpt=args.tpt,
                               far_chunks=args.chunks, far_split=args.split, stream=stream.cuda_stream,
                               profile=profile, tune_K=kr, warm_start=warm_start, side_stream=side,
                               precond=PC_FIXED if precond is None else precond,
                               precond_coarse=PC_COARSE if coarse is None else coarse)

    FT6 = [inputs.random_forces(100 + k, M, k=K_RHS) for k in range(max(K, 2) + W + 2)]
    # the timed products read forces from and write velocities to HBM (no host copies)
    FT6_dev = [torch.as_tensor(np.ascontiguousarray(f), dtype=torch.float64, device=dev) for f in FT6]
    UO_dev = torch.empty((K_RHS, M, 6), dtype=torch.float64, device=dev)

    if args.lcp_table:
        print(json.dumps(lcp_table(binding, inputs, stream, precond=PC_FIXED, coarse=PC_COARSE)), flush=True)
        return

    if args.cpu_table:
        print(json.dumps(cpu_table(binding, inputs, stream)), flush=True)
        return

    if args.contact_probe:
        print(json.dumps(contact_steps(binding, inputs, torch, stream, w, args, replay_solvers=False)), flush=True)
        return

    if args.batch_probe:
        inst = inputs.batched_suspensions(args.seed)
        FTb = [inputs.random_forces(500 + b, ci.shape[0]) for b, (ci, _, _) in enumerate(inst)]
        kwp = dict(tpt=args.tpt) if args.tpt else {}
        # preconditioned (eager lockstep iterations), or with --no-precond plain GMRES replayed
        # from captured graphs
        kwp.update(dict(precond='eager') if PC else dict(graphs=True))
        with binding.BatchContext(inst, gmres_tol=1e-8, precision='mixed', stream=stream.cuda_stream,
                                  side_stream=not args.serial, **kwp) as bc:
            bc.mobility_apply(FTb)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                _, bst = bc.mobility_apply(FTb)
            torch.cuda.synchronize()
            tb = (time.perf_counter() - t0) / 3
        print(json.dumps({'instances': len(inst), 'ms_per_product': round(tb * 1e3, 3),
                          'mvps_batched': round(len(inst) / tb, 2), 'lockstep_iterations': bst['n_far'],
                          'side_stream': not args.serial, 'precond': PC}), flush=True)
        return

    if args.counters_probe:
        ref = torch.empty(PROBE_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(ref)
        torch.cuda.synchronize()
        dst.copy_(ref)                      # reads and writes PROBE_BYTES once each
        torch.cuda.synchronize()
        cm = ctx_for('mixed', profile=False, side=False)  # per-dispatch counters: one kernel at a time
        _, st = cm.mobility_apply_multi(FT6[0])
        torch.cuda.synchronize()
        cm.close()
        print(json.dumps({'probe_bytes': PROBE_BYTES, 'far_launches': st['n_far'],
                          'far_pairs_per_launch': int(pf)}), flush=True)
        return

    def run_multi(ctx, steps, warm, kr):
        # the preconditioner is built in the first product after a configuration change (warm-up)
        setup_ms = 0.0
        for k in range(warm):
            st = ctx.mobility_apply_multi_dev(kr, FT6_dev[k].data_ptr(), UO_dev.data_ptr())
            setup_ms += st['t_precond_ms']
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = far_ms = nfar = mv = pc_ms = pc_n = pc_setup_timed = far_k_ms = nfar_k = 0
        for k in range(steps):
            st = ctx.mobility_apply_multi_dev(kr, FT6_dev[warm + k].data_ptr(), UO_dev.data_ptr())
            its += st['gmres_iters']
            far_ms += st['t_far_ms']
            nfar += st['n_far']
            far_k_ms += st['t_far_by_k_ms'][kr - 1]  # the launches with all kr densities
            nfar_k += st['n_far_by_k'][kr - 1]
            mv += st['matvecs']
            pc_ms += st['t_precond_apply_ms']
            pc_n += st['precond_applies']
            pc_setup_timed += st['t_precond_ms']
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        return dict(steps=steps, sec=sec, mvps=steps * kr / sec, gmres_iters=its / (steps * kr),
                    far_ms=far_k_ms / max(nfar_k, 1), far_ms_all=far_ms / max(nfar, 1), far_launches_full=nfar_k,
                    matvecs_per_mvp=mv / (steps * kr), far_launches=nfar,
                    precond_setup_ms=setup_ms, precond_setup_in_timed_ms=pc_setup_timed,
                    precond_apply_ms=pc_ms / max(pc_n, 1), precond_applies=pc_n)

    res = {}
    # headline: the library's fastest configuration (side stream on the mixed path), no event timing
    cm = ctx_for('mixed', profile=False)
    res['mixed6'] = run_multi(cm, K, W, K_RHS)
    log('mixed K=6', res['mixed6'], cm.far_shape)
    # far-kernel timing (roofline): the same launches on one stream with HIP events around each far launch
    with ctx_for('mixed', profile=True) as cp:
        prof6 = run_multi(cp, K, W, K_RHS)
    log('mixed K=6 far kernel alone', prof6)
    cm1 = ctx_for('mixed', 1, profile=False)
    res['mixed1'] = run_multi(cm1, max(2, K // 2), 1, 1)
    log('mixed K=1', res['mixed1'], cm1.far_shape)
    layout1 = cm1.far_shape
    cm1.close()
    with ctx_for('mixed', 1, profile=True) as cp1:
        prof1 = run_multi(cp1, max(2, K // 2), 1, 1)
    log('mixed K=1 far kernel alone', prof1)
    res['mixed6']['far_ms'], res['mixed1']['far_ms'] = prof6['far_ms'], prof1['far_ms']
    # the headline product with plain GMRES (no preconditioner), for comparison and for the
    # oracle's matvec count (its GMRES is unpreconditioned)
    with ctx_for('mixed', profile=False, precond=False) as cpl:
        plain6 = run_multi(cpl, K, W, K_RHS)
    log('mixed K=6 plain GMRES', plain6)
    one6 = None
    if PC_COARSE:  # and with the one-level preconditioner
        with ctx_for('mixed', profile=False, coarse=False) as cpo:
            one6 = run_multi(cpo, K, W, K_RHS)
        log('mixed K=6 one-level preconditioner', one6)
    cf = ctx_for('fp64')
    res['fp64_6'] = run_multi(cf, max(1, K // 3), 1, K_RHS)
    log('fp64 K=6', res['fp64_6'], cf.far_shape)
    cf1 = ctx_for('fp64', 1)
    res['fp64_1'] = run_multi(cf1, max(1, K // 3), 1, 1)
    log('fp64 K=1', res['fp64_1'], cf1.far_shape)
    cf1.close()

    # accuracy of mixed vs FP64 on the same six force sets (per velocity block)
    Um, _ = cm.mobility_apply_multi(FT6[0])
    Uf, _ = cf.mobility_apply_multi(FT6[0])
    errs = {}
    for name, blk in (('translation', slice(0, 3)), ('rotation', slice(3, 6))):
        errs['max_' + name] = float(max(np.abs(Um[r][:, blk] - Uf[r][:, blk]).max() / np.abs(Uf[r][:, blk]).max()
                                        for r in range(K_RHS)))
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
        t2 = time.perf_counter()
        x3, lb = cm.lcp_solve(pairs, b, 'bb')
        t2b = time.perf_counter()
        t_cold = {'bi': t1 - t0, 'mono': t2 - t1}
        # the other fidelity axis of the method: same grid, GMRES tolerance 1e-3 for the model
        # and recursive Bi-PQN over three fidelities: that model, then the coarse grid at 1e-3
        with binding.Context(c, None, nt, nph, lo=(nt, nph), gmres_tol=1e-8, gmres_tol_lo=1e-3, lo2=w['lo'],
                             gmres_tol_lo2=1e-3, precision='mixed', tpt=args.tpt, far_chunks=args.chunks,
                             far_split=args.split, stream=stream.cuda_stream, tune_K=1, precond=PC_FIXED,
                             precond_coarse=PC_COARSE) as cb:
            t3 = time.perf_counter()
            x4, lt = cb.lcp_solve(pairs, b, 'bi')
            t4 = time.perf_counter()
            x5, lr = cb.lcp_solve(pairs, b, 'birec')
            t5 = time.perf_counter()
        # Bi-PQN whose low fidelity is the same grid with far pairs from a 6x12 source grid
        # (density truncated to degree 5), at GMRES 1e-8 and at 1e-3
        cf = {}
        for tol_lo in (1e-8, 1e-3):
            with binding.Context(c, None, nt, nph, lo=(nt, nph), far_coarse_lo=6, gmres_tol=1e-8,
                                 gmres_tol_lo=tol_lo, precision='mixed', tpt=args.tpt, far_chunks=args.chunks,
                                 far_split=args.split, stream=stream.cuda_stream, tune_K=1,
                                 side_stream=not args.serial, precond=PC_FIXED,
                                 precond_coarse=PC_COARSE) as ccf:
                ccf.lcp_solve(pairs, b, 'bi')       # the coarse-grid tables and buffers warm
                torch.cuda.synchronize()
                t0c = time.perf_counter()
                xcf, scf = ccf.lcp_solve(pairs, b, 'bi')
                tcf = time.perf_counter() - t0c
            cf[f'{tol_lo:.0e}'] = dict(lo=f'{nt}x{nph}, far pairs from 6x12 (degree 5), GMRES {tol_lo:.0e}',
                                       sec=round(tcf, 3), mvp_hi=scf['mvp_hi'], mvp_lo=scf['mvp_lo'],
                                       emvp=round(scf['emvp'], 2), lo_hi_cost_ratio=round(scf['lo_hi_cost_ratio'], 4),
                                       x_rel_err=float(np.abs(xcf - xs).max() / np.abs(xs).max()),
                                       converged=scf['converged'], solves_per_s=round(1.0 / tcf, 3))
        lcp_info = dict(n_contacts=int(pairs.shape[0]), planted_active=int((xs > 0).sum()),
                        bi=dict(sec=round(t1 - t0, 3), mvp_hi=ls['mvp_hi'], mvp_lo=ls['mvp_lo'],
                                emvp=round(ls['emvp'], 2), lo_hi_cost_ratio=round(ls['lo_hi_cost_ratio'], 4),
                                x_rel_err=float(np.abs(x - xs).max() / np.abs(xs).max())),
                        mono=dict(sec=round(t2 - t1, 3), mvp=lm['mvp_hi'],
                                  x_rel_err=float(np.abs(x2 - xs).max() / np.abs(xs).max())),
                        bbpgd=dict(sec=round(t2b - t2, 3), mvp=lb['mvp_hi'],
                                   x_rel_err=float(np.abs(x3 - xs).max() / np.abs(xs).max())),
                        bi_tol_fidelity=dict(lo=f'{nt}x{nph} at GMRES 1e-3', sec=round(t4 - t3, 3),
                                             mvp_hi=lt['mvp_hi'], mvp_lo=lt['mvp_lo'], emvp=round(lt['emvp'], 2),
                                             lo_hi_cost_ratio=round(lt['lo_hi_cost_ratio'], 4),
                                             x_rel_err=float(np.abs(x4 - xs).max() / np.abs(xs).max())),
                        bi_recursive=dict(fidelities=f'{nt}x{nph} at 1e-8, {nt}x{nph} at 1e-3, '
                                                     f'{w["lo"][0]}x{w["lo"][1]} at 1e-3',
                                          sec=round(t5 - t4, 3), mvp_hi=lr['mvp_hi'], mvp_lo=lr['mvp_lo'],
                                          mvp_lo2=lr['mvp_lo2'], emvp=round(lr['emvp'], 2),
                                          cost_ratios=[round(lr['lo_hi_cost_ratio'], 4),
                                                       round(lr['lo2_hi_cost_ratio'], 4)],
                                          x_rel_err=float(np.abs(x5 - xs).max() / np.abs(xs).max())))
        for v in lcp_info.values():
            if isinstance(v, dict) and v.get('sec'):
                v['solves_per_s'] = round(1.0 / v['sec'], 3)
        lcp_info['bi_coarse_far'] = cf
        # Precision separated from tolerance: at GMRES 1e-8 every LCP product is known only to
        # ~1e-8 relative, and A's smallest eigenvalue (~8e-4) turns that into x errors of ~3e-6
        # on either path (x_rel_err above). Here b is formed with an FP64 product at GMRES 1e-12
        # and the same LCP is solved to KKT 1e-10 (absolute, eq. (kkt-error)) with GMRES 1e-10
        # inside every product, on the mixed and on the FP64 path.
        tight = dict(kkt_tol_abs=1e-10, gmres_tol=1e-10, b_from='FP64 product at GMRES 1e-12')
        xe = lambda x_: float(np.abs(x_ - xs).max() / np.abs(xs).max())
        kw_t = dict(lo=w['lo'], tpt=args.tpt, far_chunks=args.chunks, far_split=args.split,
                    stream=stream.cuda_stream, tune_K=1, precond=PC_FIXED, precond_coarse=PC_COARSE)
        with binding.Context(c, None, nt, nph, precision='fp64', gmres_tol=1e-12, **kw_t) as cref:
            b_t = ws - cref.lcp_apply(pairs, xs)
        with binding.Context(c, None, nt, nph, precision='fp64', gmres_tol=1e-10, **kw_t) as cf64, \
                binding.Context(c, None, nt, nph, precision='mixed', gmres_tol=1e-10, **kw_t) as cmt:
            for solver, key in (('bi', 'bi'), ('mono', 'mono'), ('bb', 'bbpgd')):
                t0 = time.perf_counter()
                xm, sm = cmt.lcp_solve(pairs, b_t, solver, tol_abs=1e-10, k_max=300)
                t1 = time.perf_counter()
                xf, sf = cf64.lcp_solve(pairs, b_t, solver, tol_abs=1e-10, k_max=300)
                t2 = time.perf_counter()
                tight[key] = dict(mvp_hi=sm['mvp_hi'], mvp_lo=sm['mvp_lo'], emvp=round(sm['emvp'], 2),
                                  converged=sm['converged'], x_rel_err=xe(xm), sec=round(t1 - t0, 3),
                                  fp64=dict(mvp_hi=sf['mvp_hi'], mvp_lo=sf['mvp_lo'], converged=sf['converged'],
                                            x_rel_err=xe(xf), sec=round(t2 - t1, 3)),
                                  mixed_vs_fp64_x_rel_err=float(np.abs(xm - xf).max() / np.abs(xf).max()))
        lcp_info['tight_tolerance'] = tight
        # Alg. 1 as printed (H^(0) = I throughout) against the reading's scaled metric
        pm = {}
        for solver in ('mono', 'bi'):
            t0 = time.perf_counter()
            xp, sp = cm.lcp_solve(pairs, b, solver, printed_metric=True, k_max=300)
            pm[solver] = dict(mvp_hi=sp['mvp_hi'], mvp_lo=sp['mvp_lo'], emvp=round(sp['emvp'], 2),
                              converged=sp['converged'], x_rel_err=xe(xp), sec=round(time.perf_counter() - t0, 3))
        lcp_info['printed_metric'] = pm
        # Krylov reuse across the products of one solve (recycle): GMRES iterations per
        # product and time, against the cold solves above (same LCP, same tolerance)
        rc = {}
        for solver, cold, tc in (('mono', lm, t_cold['mono']), ('bi', ls, t_cold['bi'])):
            t0r = time.perf_counter()
            xr, sr = cm.lcp_solve(pairs, b, solver, recycle=True)
            tr = time.perf_counter() - t0r
            prods = lambda st_: st_['mvp_hi'] + st_['mvp_lo']
            rc[solver] = dict(mvp_hi=sr['mvp_hi'], mvp_lo=sr['mvp_lo'], gmres_iters=sr['gmres_iters'],
                              gmres_per_product=round(sr['gmres_iters'] / max(1, prods(sr)), 2),
                              cold_gmres_iters=cold['gmres_iters'],
                              cold_gmres_per_product=round(cold['gmres_iters'] / max(1, prods(cold)), 2),
                              sec=round(tr, 3), cold_sec=round(tc, 3), speedup=round(tc / tr, 3),
                              x_rel_err=xe(xr), converged=sr['converged'])
        lcp_info['recycle'] = rc
        log('lcp', lcp_info)
    cm_layout = cm.far_shape
    cm.close()

    step_info = None
    if not args.no_steps:
        # time steps of the Janus suspension (dt 1e-3, contacts below gap 0.1, Bi-PQN, slip solves
        # warm-started from the previous step): the FP64 trajectory, and the mixed path replayed
        # from each FP64 state
        axes = inputs.janus_axes(args.seed + 7, M)
        nsteps, dt = 10, 1e-3
        states, t64, st64 = [(c, axes)], [], []
        with ctx_for('fp64', 1, profile=False, warm_start=True, precond=PC) as cs:
            cs.set_state(c, axes)
            for _ in range(nsteps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = cs.step(dt, 0.1, 'bi')
                t64.append(time.perf_counter() - t0)
                st64.append(st)
                states.append(cs.get_state())
        mixed = {}
        for name, refine in (('mixed', 0), ('mixed_refined', 1)):
            tmx, dmax = [], 0.0
            with binding.Context(c, None, nt, nph, lo=w['lo'], gmres_tol=1e-8, precision='mixed', refine=refine,
                                 tpt=args.tpt, far_chunks=args.chunks, far_split=args.split,
                                 stream=stream.cuda_stream, tune_K=1, warm_start=True,
                                 side_stream=not args.serial, precond=PC, precond_coarse=PC_COARSE) as cs:
                for k in range(nsteps):
                    cs.set_state(*states[k])
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    cs.step(dt, 0.1, 'bi')
                    tmx.append(time.perf_counter() - t0)
                    cm_k, _ = cs.get_state()
                    disp = states[k + 1][0] - states[k][0]
                    dmax = max(dmax, float(np.abs(cm_k - states[k + 1][0]).max() / np.abs(disp).max()))
            mixed[name] = (tmx, dmax)
        tmx, dmax = mixed['mixed']
        step_info = dict(steps=nsteps, dt=dt, precond='on reuse' if PC else 'off', contacts=[s_['n_contacts'] for s_ in st64],
                         active=[s_['n_active'] for s_ in st64],
                         mvp_hi=[s_['lcp']['mvp_hi'] for s_ in st64], mvp_lo=[s_['lcp']['mvp_lo'] for s_ in st64],
                         gmres_iters_nc=[s_['gmres_iters_nc'] for s_ in st64],
                         sec_per_step_fp64=round(float(np.median(t64)), 4),
                         sec_per_step_mixed=round(float(np.median(tmx)), 4),
                         speedup=round(float(np.median(t64) / np.median(tmx)), 3),
                         mixed_displacement_rel_err=dmax,
                         sec_per_step_mixed_refined=round(float(np.median(mixed['mixed_refined'][0])), 4),
                         mixed_refined_displacement_rel_err=mixed['mixed_refined'][1])
        log('steps', step_info)

    inward_info = None
    if not args.no_steps:
        inward_info = contact_steps(binding, inputs, torch, stream, w, args)
        log('steps with contacts', inward_info)

    batch_info = None
    if not args.no_batch:
        inst = inputs.batched_suspensions(args.seed)
        FTb = [inputs.random_forces(500 + b, ci.shape[0]) for b, (ci, _, _) in enumerate(inst)]
        # launch shape from the autotuner's batch entry unless fixed on the command line
        kw = dict(gmres_tol=1e-8, precision='mixed', stream=stream.cuda_stream, side_stream=not args.serial)
        if args.tpt:
            kw['tpt'] = args.tpt
        reps = 3
        # GMRES iterations replayed from captured graphs (device-side Givens), and the same
        # product with the eager lockstep loop (host Givens, one readback per iteration)
        with binding.BatchContext(inst, graphs=True, **kw) as bc:
            batch_shape = bc.far_shape
            bc.mobility_apply(FTb)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                Ubm, bst = bc.mobility_apply(FTb)
            torch.cuda.synchronize()
            tb = (time.perf_counter() - t0) / reps
        with binding.BatchContext(inst, **kw) as bc:
            bc.mobility_apply(FTb)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                bc.mobility_apply(FTb)
            torch.cuda.synchronize()
            tb_eager = (time.perf_counter() - t0) / reps
        with binding.BatchContext(inst, **dict(kw, precision='fp64')) as bc:
            bc.mobility_apply(FTb)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                Ub64, _ = bc.mobility_apply(FTb)
            torch.cuda.synchronize()
            tb64 = (time.perf_counter() - t0) / reps
        err_b = float(max(np.abs(a - b_).max() / np.abs(b_).max() for a, b_ in zip(Ubm, Ub64)))
        # every suspension with its own preconditioner (built in the warm-up product; eager
        # lockstep iterations, the preconditioners applied in segmented launches)
        bpc = None
        if PC:
            with binding.BatchContext(inst, precond='eager', **kw) as bc:
                _, bs0 = bc.mobility_apply(FTb)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    Ubp, bsp = bc.mobility_apply(FTb)
                torch.cuda.synchronize()
                tbp = (time.perf_counter() - t0) / reps
            bpc = dict(batched_sec=round(tbp, 4), mvps_batched=round(len(inst) / tbp, 2),
                       lockstep_iterations=bsp['n_far'], setup_ms=round(bs0['t_precond_ms'], 1),
                       rel_diff_vs_plain=float(max(np.abs(a - b_).max() / np.abs(b_).max()
                                                   for a, b_ in zip(Ubp, Ubm))))
        singles = [binding.Context(ci, None, nti, npi, **kw) for ci, nti, npi in inst]
        for ctx_b, F in zip(singles, FTb):
            ctx_b.mobility_apply(F)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for ctx_b, F in zip(singles, FTb):
            ctx_b.mobility_apply(F)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        for ctx_b in singles:
            ctx_b.close()
        batch_info = dict(instances=len(inst), nodes=int(sum(ci.shape[0] * nti * npi for ci, nti, npi in inst)),
                          batched_sec=round(tb, 4), mvps_batched=round(len(inst) / tb, 2),
                          graph_launches=bst['graph_launches'], eager_sec=round(tb_eager, 4),
                          mvps_batched_eager=round(len(inst) / tb_eager, 2),
                          mvps_batched_fp64=round(len(inst) / tb64, 2), mixed_rel_err_vs_fp64=err_b,
                          one_by_one_sec=round(ts, 4), mvps_one_by_one=round(len(inst) / ts, 2),
                          speedup=round(ts / tb, 3), lockstep_iterations=bst['n_far'], far_layout=batch_shape,
                          precond=bpc)
        log('batch', batch_info)

    m6 = res['mixed6']
    achieved = flop_per_pair(K_RHS) * pf / (m6['far_ms'] * 1e-3) / 1e12
    achieved1 = flop_per_pair(1) * pf / (res['mixed1']['far_ms'] * 1e-3) / 1e12
    achieved64 = flop_per_pair(K_RHS) * pf / (res['fp64_6']['far_ms'] * 1e-3) / 1e12
    out = {
        'metric': 'batched mobility MVPs/s (216 spheres, 6 force sets per pass, mixed FP32/FP64, GMRES 1e-8)',
        'value': round(m6['mvps'], 4),
        'unit': 'MVP/s',
        'n_gpus': 1, 'steps': K, 'warmup': W,
        'ms_per_step': round(1e3 * m6['sec'] / m6['steps'], 3),
        'higher_is_better': True, 'scaling': 'weak', 'vs_baseline': None,
        'dtype': 'f32+f64', 'data': 'synthetic',
        'config': {'workload': 'rsa216: 216 spheres a=1, RSA phi=0.3, 12x24 nodes (62,208), near gap 0.5, '
                               '6 random force sets per step, GMRES tol 1e-8', 'n_nodes': M * n,
                   'force_sets_per_step': K_RHS, 'far_pairs_per_matvec': int(pf)},
        'gpair_evals_per_s': round(m6['matvecs_per_mvp'] * pf * m6['mvps'] / 1e9, 2),
        # far (target, source) node-pair evaluations per second: pair-density products for the
        # six-force-set passes (geometry shared by the six), pairs for the single force set
        'gpair_evals_per_s_detail': {
            'mixed_K6_pair_density': round(m6['matvecs_per_mvp'] * pf * m6['mvps'] / 1e9, 2),
            'mixed_K1': round(res['mixed1']['matvecs_per_mvp'] * pf * res['mixed1']['mvps'] / 1e9, 2),
            'fp64_K6_pair_density': round(res['fp64_6']['matvecs_per_mvp'] * pf * res['fp64_6']['mvps'] / 1e9, 2),
            'fp64_K1': round(res['fp64_1']['matvecs_per_mvp'] * pf * res['fp64_1']['mvps'] / 1e9, 2)},
        'single_mvps_per_s': {'mixed': round(res['mixed1']['mvps'], 4), 'fp64': round(res['fp64_1']['mvps'], 4)},
        'batched_mvps_per_s': {'mixed': round(m6['mvps'], 4), 'fp64': round(res['fp64_6']['mvps'], 4)},
        'speedup_mixed_vs_fp64': {'K6': round(m6['mvps'] / res['fp64_6']['mvps'], 3),
                                  'K1': round(res['mixed1']['mvps'] / res['fp64_1']['mvps'], 3)},
        'mixed_rel_err_vs_fp64': errs,
        'gmres_iters_per_mvp': {k: round(v['gmres_iters'], 2) for k, v in res.items()},
        'far_kernel_ms': {k: round(v['far_ms'], 4) for k, v in res.items()},
        'precond': None if not PC else {
            'kind': 'near-patch Schur complements, right preconditioning (config precond)'
                    + (', with a coarse correction on degree <= 2 harmonics (precond_coarse)' if PC_COARSE else ''),
            'setup_ms': round(m6['precond_setup_ms'], 1),
            'setup_ms_in_timed_region': round(m6['precond_setup_in_timed_ms'], 1),
            'apply_ms_k6': round(prof6['precond_apply_ms'], 4),
            'apply_hbm_gbs_k6': round(precond_bytes(n, nt * nt, pc_blocks(c)) / (prof6['precond_apply_ms'] * 1e-3) / 1e9, 1)
            if prof6['precond_apply_ms'] > 0 else None,
            'block_bytes': precond_bytes(n, nt * nt, pc_blocks(c)),
            'plain_gmres': {'mvps': round(plain6['mvps'], 4), 'gmres_iters_per_mvp': round(plain6['gmres_iters'], 2),
                            'ms_per_step': round(1e3 * plain6['sec'] / plain6['steps'], 3)},
            'levels': 2 if PC_COARSE else 1,
            'one_level': None if one6 is None else {
                'mvps': round(one6['mvps'], 4), 'gmres_iters_per_mvp': round(one6['gmres_iters'], 2),
                'ms_per_step': round(1e3 * one6['sec'] / one6['steps'], 3),
                'setup_ms': round(one6['precond_setup_ms'], 1)},
            'speedup_vs_plain': round(m6['mvps'] / plain6['mvps'], 3)},
        'roofline': {'bound': 'alu', 'kernel': far_kernel_name(cm_layout, K_RHS), 'achieved': round(achieved, 3),
                     'peak': PEAK_FP32_VECTOR, 'unit': 'TFLOP/s', 'frac': round(achieved / PEAK_FP32_VECTOR, 4),
                     'flop_per_pair': flop_per_pair(K_RHS), 'layout': cm_layout,
                     'traffic': far_traffic_bytes(cm_layout),
                     'traffic_unit': 'HBM bytes per launch',
                     'k1': {'kernel': far_kernel_name(layout1, 1), 'layout': layout1, 'achieved': round(achieved1, 3),
                            'frac': round(achieved1 / PEAK_FP32_VECTOR, 4)},
                     'fp64': {'kernel': f'k_far64<{K_RHS}>', 'achieved': round(achieved64, 3),
                              'peak': PEAK_FP64_VECTOR, 'frac': round(achieved64 / PEAK_FP64_VECTOR, 4)}},
        'lcp': lcp_info,
        'batch32': batch_info,
        'time_steps': step_info,
        'time_steps_with_contacts': inward_info,
    }
    out['host'] = {'gpu': torch.cuda.get_device_name(0), 'cpu_model': cpu_model(),
                   'cpu_threads_available': len(os.sched_getaffinity(0)), 'gpu_sclk_mhz': gpu_sclk()}
    if not args.no_cpu_baseline:
        out['cpu_baseline'] = cpu_baseline(c, nt, nph, plain6)
    print(json.dumps(out), flush=True)


def contact_steps(binding, inputs, torch, stream, w, args, replay_solvers=True):
    """Five time steps with active contacts on the 216-sphere workload (FP64 trajectory, the mixed
    path replayed from each state, and optionally every solver on the same LCPs)."""
    c, nt, nph = w['centers'], w['n_theta'], w['n_phi']
    # time steps with active contacts: Janus axes towards the centroid (the paper's online runs start
    # with the amphiphilic sides facing the origin), dt 0.1, so approaching pairs enter the LCP; near
    # pairs closer than 0.02 take the 3x grid, which keeps A positive definite once gaps close below
    # ~5e-3
    ax_in = c.mean(axis=0) - c
    ax_in /= np.linalg.norm(ax_in, axis=1, keepdims=True)
    nin, dt_in = 5, 0.1
    try:
        states_in, rows = [(c, ax_in)], []
        pc = not getattr(args, 'no_precond', False)
        pcc = pc and not getattr(args, 'no_coarse', False)
        with binding.Context(c, ax_in, nt, nph, lo=w['lo'], gmres_tol=1e-8, precision='fp64', tune_K=1,
                             warm_start=True, near_close_gap=0.02, near_close_up=3,
                             stream=stream.cuda_stream, precond=pc, precond_coarse=pcc) as cs:
            for _ in range(nin):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = cs.step(dt_in, 0.1, 'bi')
                rows.append((time.perf_counter() - t0, st))
                states_in.append(cs.get_state())
        tmi, dmi = [], 0.0
        active_k = [k for k in range(nin) if rows[k][1]['n_active'] > 0]
        per_solver = {}

        def replay(cs, solver, name, ks):
            """Steps from the FP64 states ks with one solver: products and time per step."""
            out = dict(mvp_hi=[], mvp_lo=[], emvp=[], converged=[], sec=[])
            for k in ks:
                cs.set_state(*states_in[k])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st_ = cs.step(dt_in, 0.1, solver)
                out['sec'].append(round(time.perf_counter() - t0, 3))
                for key in ('mvp_hi', 'mvp_lo', 'converged'):
                    out[key].append(st_['lcp'][key])
                out['emvp'].append(round(st_['lcp']['emvp'], 2))
            per_solver[name] = out

        with binding.Context(c, ax_in, nt, nph, lo=w['lo'], gmres_tol=1e-8, precision='mixed', tune_K=1,
                             warm_start=True, near_close_gap=0.02, near_close_up=3,
                             stream=stream.cuda_stream, side_stream=not args.serial, precond=pc,
                             precond_coarse=pcc) as cs:
            for k in range(nin):
                cs.set_state(*states_in[k])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                cs.step(dt_in, 0.1, 'bi')
                tmi.append(time.perf_counter() - t0)
                cm_k, _ = cs.get_state()
                disp = states_in[k + 1][0] - states_in[k][0]
                dmi = max(dmi, float(np.abs(cm_k - states_in[k + 1][0]).max() / np.abs(disp).max()))
            # the other solvers on the same LCPs (the steps with active contacts), mixed precision
            if replay_solvers:
                replay(cs, 'bi', 'bi_pqn', active_k)
                replay(cs, 'mono', 'mono_pqn', active_k)
                replay(cs, 'bb', 'bb_pgd', active_k)
        if replay_solvers:
            # Bi-PQN whose low fidelity is the same grid solved to GMRES 1e-3, and the same grid
            # with far pairs from a 6x12 source grid (degree 5) at GMRES 1e-3
            for name, kw_lo in (('bi_pqn_tol_fidelity', {}), ('bi_pqn_coarse_far', dict(far_coarse_lo=6))):
                with binding.Context(c, ax_in, nt, nph, lo=(nt, nph), gmres_tol=1e-8, gmres_tol_lo=1e-3,
                                     precision='mixed', tune_K=1, warm_start=True, near_close_gap=0.02,
                                     near_close_up=3, stream=stream.cuda_stream, side_stream=not args.serial,
                                     precond=pc, precond_coarse=pcc, **kw_lo) as cs:
                    replay(cs, 'bi', name, active_k)
        inward_info = dict(steps=nin, dt=dt_in, near_close_gap=0.02, near_close_up=3,
                           precond='on reuse' if pc else 'off',
                           axes='towards the centroid',
                           contacts=[r[1]['n_contacts'] for r in rows], active=[r[1]['n_active'] for r in rows],
                           mvp_hi=[r[1]['lcp']['mvp_hi'] for r in rows],
                           mvp_lo=[r[1]['lcp']['mvp_lo'] for r in rows],
                           emvp=[round(r[1]['lcp']['emvp'], 2) for r in rows],
                           lcp_converged=[r[1]['lcp']['converged'] for r in rows if r[1]['n_contacts'] > 0],
                           sec_per_step_fp64=[round(r[0], 3) for r in rows],
                           sec_per_step_mixed=[round(t_, 3) for t_ in tmi],
                           speedup=round(sum(r[0] for r in rows) / sum(tmi), 3),
                           mixed_displacement_rel_err=dmi,
                           min_gap_after=round(float(inputs.min_gap(states_in[-1][0])), 6),
                           solvers_mixed=dict(steps=active_k, **per_solver))
    except Exception as e:  # a failed step is reported in the line, not a lost line
        inward_info = dict(error=f'{type(e).__name__}: {e}')
    return inward_info


def lcp_table(binding, inputs, stream, precond=False, coarse=False):
    """Products per planted LCP (about half the contacts active, KKT 1e-8) for the solvers of
    the method on the contact sets (gap < 0.1) of three workloads, mixed precision: BB-PGD,
    Mono-PQN and Bi-PQN with the coarse grid as low fidelity (each PQN solver with the scaled
    initial metric and with Alg. 1's printed H^(0) = I), Bi-PQN with the same grid at
    GMRES tolerance 1e-3 as low fidelity, and recursive Bi-PQN over both (same grid at 1e-3,
    then the coarse grid at 1e-3). E-MVP = high + low x (low-fidelity product time /
    high-fidelity product time) summed over the fidelities, all measured. The coarse-far
    variants take the same grid with far pairs from a 6x12 source grid (density truncated to
    degree 5) as the low fidelity, at GMRES 1e-8 (bi_cf) and 1e-3 (bi_cf_tol), and recursive
    Bi-PQN over that model and the coarse grid at 1e-3 (birec_cf)."""
    import torch
    rows = []
    for name in ('lattice27_contacts', 'packing64', 'rsa216'):
        for seed in (0, 1, 2):
            w = inputs.workload(name, seed)
            c, nt, nph = w['centers'], w['n_theta'], w['n_phi']
            row = dict(workload=name, seed=seed)
            with binding.Context(c, None, nt, nph, lo=w['lo'], gmres_tol=1e-8, precision='mixed',
                                 stream=stream.cuda_stream, tune_K=1, precond=precond,
                                 precond_coarse=coarse) as ctx:
                pairs, _ = ctx.find_contacts(0.1)
                if pairs.shape[0] == 0:
                    continue
                xs, ws = inputs.planted_lcp(seed, pairs.shape[0])
                b = ws - ctx.lcp_apply(pairs, xs)
                ctx.lcp_apply(pairs, xs, binding.PQN_LOFI)  # both levels' tables built before timing
                row['contacts'] = int(pairs.shape[0])
                for key, solver, printed in (('bb', 'bb', False), ('mono', 'mono', False), ('bi', 'bi', False),
                                             ('mono_printed', 'mono', True), ('bi_printed', 'bi', True)):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    x, st = ctx.lcp_solve(pairs, b, solver, printed_metric=printed, k_max=300)
                    row[key] = dict(hi=st['mvp_hi'], lo=st['mvp_lo'], emvp=round(st['emvp'], 2),
                                       sec=round(time.perf_counter() - t0, 3), conv=st['converged'],
                                       x_err=float(np.abs(x - xs).max() / np.abs(xs).max()))
            variants = (('bi_tol', 'bi', dict(gmres_tol_lo=1e-3, lo2=w['lo'], gmres_tol_lo2=1e-3)),
                        ('birec', 'birec', dict(gmres_tol_lo=1e-3, lo2=w['lo'], gmres_tol_lo2=1e-3)),
                        ('bi_cf', 'bi', dict(gmres_tol_lo=1e-8, far_coarse_lo=6)),
                        ('bi_cf_tol', 'bi', dict(gmres_tol_lo=1e-3, far_coarse_lo=6)),
                        ('birec_cf', 'birec', dict(gmres_tol_lo=1e-3, far_coarse_lo=6, lo2=w['lo'],
                                                   gmres_tol_lo2=1e-3)))
            for key, solver, kw_lo in variants:
                with binding.Context(c, None, nt, nph, lo=(nt, nph), gmres_tol=1e-8, precision='mixed',
                                     stream=stream.cuda_stream, tune_K=1, precond=precond,
                                     precond_coarse=coarse, **kw_lo) as ctx:
                    if key.startswith('bi_cf') or precond:
                        ctx.lcp_solve(pairs, b, solver)     # warm the buffers (and build the preconditioners)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    x, st = ctx.lcp_solve(pairs, b, solver)
                    row[key] = dict(hi=st['mvp_hi'], lo=st['mvp_lo'], lo2=st['mvp_lo2'], emvp=round(st['emvp'], 2),
                                    ratio=round(st['lo_hi_cost_ratio'], 3), ratio2=round(st['lo2_hi_cost_ratio'], 4),
                                    sec=round(time.perf_counter() - t0, 3), conv=st['converged'],
                                    x_err=float(np.abs(x - xs).max() / np.abs(xs).max()))
            print('[lcp-table]', row, file=sys.stderr, flush=True)
            rows.append(row)
    med = {}
    for name in ('lattice27_contacts', 'packing64', 'rsa216'):
        rs = [r for r in rows if r['workload'] == name]
        if rs:
            med[name] = {k: float(np.median([r[k]['emvp'] for r in rs]))
                         for k in ('bb', 'mono', 'bi', 'bi_tol', 'birec', 'bi_cf', 'bi_cf_tol', 'birec_cf',
                                   'mono_printed', 'bi_printed')}
            med[name + '_sec'] = {k: float(np.median([r[k]['sec'] for r in rs]))
                                  for k in ('bb', 'mono', 'bi', 'bi_tol', 'birec', 'bi_cf', 'bi_cf_tol', 'birec_cf')}
    return dict(table='planted LCPs, mixed precision, KKT 1e-8', precond=bool(precond), rows=rows,
                median_emvp=med)


def cpu_table(binding, inputs, stream):
    """The CPU oracle on the host cores against the GPU path, per workload: the 8-sphere
    workload end to end on one core (assembled operator, LU factorisation as set-up, one
    MVP and one Mono-PQN LCP on its contact set), and one matvec of the 27-, 64- and
    216-sphere operators over all cores (cpu_baseline), with the GPU path's GMRES iterations
    per MVP (mixed, 1e-8) to turn matvecs into MVPs."""
    import torch
    from oracle import bie, dynamics, lcp
    out = {}
    # 8 spheres: everything by the assembled operator, one core
    w = inputs.workload('tiny', 0)
    c = w['centers']
    g = bie.Geometry(c, 1.0, w['n_theta'], w['n_phi'])
    t0 = time.perf_counter()
    A = bie.dense_operator(g)
    FT = inputs.random_forces(1, g.M)
    bie.mobility_apply(g, FT, dense=A)        # LU factorisation (set-up)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    bie.mobility_apply(g, inputs.random_forces(2, g.M), dense=A)
    t_mvp = time.perf_counter() - t0
    pairs, _ = dynamics.find_contacts(c, 1.0, 0.1)
    Aop = lcp.lcp_operator(lambda F: bie.mobility_apply(g, F, dense=A), c, pairs)
    xs, ws = inputs.planted_lcp(0, pairs.shape[0])
    b = ws - Aop(xs)
    t0 = time.perf_counter()
    _, _, st = lcp.mono_pqn(Aop, b)
    t_lcp = time.perf_counter() - t0
    with binding.Context(c, None, w['n_theta'], w['n_phi'], gmres_tol=1e-8, precision='mixed',
                         stream=stream.cuda_stream) as ctx:
        ctx.mobility_apply(FT)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.mobility_apply(FT)
        t_gpu_mvp = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, sg = ctx.lcp_solve(pairs, b, 'mono')
        t_gpu_lcp = time.perf_counter() - t0
    out['tiny'] = dict(nodes=g.N, cores=1, setup_sec=round(t_setup, 3), mvp_sec=round(t_mvp, 5),
                       lcp_sec=round(t_lcp, 4), lcp_mvps=st['mvp'], gpu_mvp_sec=round(t_gpu_mvp, 5),
                       gpu_lcp_sec=round(t_gpu_lcp, 4), gpu_lcp_mvps=sg['mvp_hi'])
    print('[cpu-table]', 'tiny', out['tiny'], file=sys.stderr, flush=True)
    for name in ('lattice27', 'packing64', 'rsa216'):
        w = inputs.workload(name, 0)
        c, nt, nph = w['centers'], w['n_theta'], w['n_phi']
        FT = inputs.random_forces(3, c.shape[0])
        with binding.Context(c, None, nt, nph, gmres_tol=1e-8, precision='mixed', stream=stream.cuda_stream,
                             tune_K=1) as ctx:
            ctx.mobility_apply(FT)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sg = ctx.mobility_apply(FT)
            t_gpu = time.perf_counter() - t0
        cb = cpu_baseline(c, nt, nph, {'matvecs_per_mvp': float(sg['matvecs'])})
        out[name] = dict(nodes=int(c.shape[0] * nt * nph), gmres_matvecs_per_mvp=sg['matvecs'],
                         gpu_mvp_sec=round(t_gpu, 4), gpu_mvps_per_s=round(1.0 / t_gpu, 3), cpu=cb)
        print('[cpu-table]', name, out[name], file=sys.stderr, flush=True)
    return out


def gpu_sclk():
    """Engine clock levels of the GPU from sysfs after the timed region: {'levels': [MHz...], 'current': MHz},
    or None where the driver does not expose them."""
    import glob
    for path in sorted(glob.glob('/sys/class/drm/card*/device/pp_dpm_sclk')):
        try:
            levels, cur = [], None
            with open(path) as f:
                for line in f:
                    parts = line.split()
                    if len(parts) >= 2 and parts[1].lower().endswith('mhz'):
                        mhz = int(parts[1][:-3])
                        levels.append(mhz)
                        if '*' in line:
                            cur = mhz
            if levels:
                return {'levels': levels, 'current': cur}
        except (OSError, ValueError):
            continue
    return None


def cpu_model():
    try:
        with open('/proc/cpuinfo') as f:
            for line in f:
                if line.startswith('model name'):
                    return line.split(':', 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_matvec_share(job):
    """Worker of the CPU baseline (one single-threaded process): the oracle's off-sphere
    double-layer sums of one matvec for its own target spheres, and the application of its
    own sample of near-pair blocks (built first, outside the timed region, as a setup
    cost). Returns (far seconds, far pairs, near seconds, near blocks applied)."""
    c, nt, nph, spheres, near_pairs = job
    from oracle import bie
    g = bie.Geometry(c, 1.0, nt, nph)
    q = np.random.default_rng(0).standard_normal((g.N, 3))
    wq = q * g.weights[:, None]
    cls = g.pair_class()
    blocks = [(j, bie.near_block(g, i, j)) for i, j in near_pairs]
    t0 = time.perf_counter()
    for j, blk in blocks:
        np.einsum('mckd,kd->mc', blk, q[g.nodes(j)])
    t_near = time.perf_counter() - t0
    t0 = time.perf_counter()
    npairs = 0
    for i in spheres:
        xi = g.x[g.nodes(i)]
        acc = np.zeros((g.n, 3))
        for j in range(g.M):
            if cls[i, j] != 0:
                continue
            sj = g.nodes(j)
            acc += bie.dl_apply(xi, g.x[sj], g.normals[sj], wq[sj])
            npairs += g.n * g.n
    return time.perf_counter() - t0, npairs, t_near, len(blocks)


def cpu_baseline(c, nt, nph, mixed):
    """The oracle's matvec of the 216-sphere operator (numpy FP64), timed on the host cores:
    every far (target, source) pair of one matvec, split by target spheres over one
    single-threaded process per core the bench may use (at most 16), plus the self block
    and rigid projection over all spheres, plus the near-pair blocks applied on a sample
    (one block per worker, built before the timed region) scaled to all near pairs.
    All-core matvec time = the slowest worker's far share + the near and self terms
    (whose cost is below 1%); single-core time = the sum of the workers' single-threaded
    times. MVP/s = 1 / (matvec time x matvecs per MVP measured on the GPU path)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from oracle import bie
    g = bie.Geometry(c, 1.0, nt, nph)
    cls = g.pair_class()
    near = [(int(i), int(j)) for i, j in zip(*np.nonzero(cls == 1))]
    cores = min(16, len(os.sched_getaffinity(0)))
    # spheres dealt round-robin so every worker has the same mix of near-heavy spheres
    shares = [list(range(k, g.M, cores)) for k in range(cores)]
    rng = np.random.default_rng(3)
    sample = [near[k] for k in rng.choice(len(near), size=min(cores, len(near)), replace=False)]
    jobs = [(c, nt, nph, shares[k], sample[k:k + 1]) for k in range(cores)]
    saved = {v: os.environ.get(v) for v in ('OMP_NUM_THREADS', 'OPENBLAS_NUM_THREADS', 'MKL_NUM_THREADS')}
    for v in saved:
        os.environ[v] = '1'
    try:
        # a worker that dies breaks the pool (an exception), it is not restarted
        with ProcessPoolExecutor(cores, mp_context=mp.get_context('spawn')) as pool:
            res = list(pool.map(_oracle_matvec_share, jobs, timeout=600))
        # self block and rigid projection of all spheres (the self block itself is set-up)
        q = np.random.default_rng(0).standard_normal((g.N, 3))
        bie.self_block(nt, nph, 1.0)
        t0 = time.perf_counter()
        bie.self_apply(g, q)
        bie.rigid_projection(g, q)
        t_self = time.perf_counter() - t0
    finally:
        for v, x in saved.items():
            if x is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = x
    far_pairs_done = sum(r[1] for r in res)
    t_near_per_block = sum(r[2] for r in res) / max(1, sum(r[3] for r in res))
    t_near_all = t_near_per_block * len(near)
    t1 = sum(r[0] for r in res) + t_near_all + t_self
    tall = max(r[0] for r in res) + t_near_all / cores + t_self
    mpm = mixed['matvecs_per_mvp']
    detail = (f'one matvec of the {g.M}-sphere operator ({nt}x{nph}): all {far_pairs_done:,} far pairs by the '
              f'oracle\'s '
              f'double-layer sums in {cores} single-threaded processes (target spheres dealt round-robin), '
              f'self block and rigid projection of all spheres, near-pair blocks applied on {len(sample)} '
              f'of {len(near)} (built before the timed region) and scaled; x {mpm:.1f} matvecs per MVP '
              f'(the oracle\'s GMRES is unpreconditioned: the GPU path\'s plain-GMRES count)')
    return {'value': round(1.0 / (tall * mpm), 8), 'unit': 'MVP/s', 'cores': cores, 'kind': 'oracle',
            'sample': detail, 'matvec_sec': round(tall, 3),
            'single_core': {'value': round(1.0 / (t1 * mpm), 8), 'unit': 'MVP/s', 'cores': 1,
                            'matvec_sec': round(t1, 2),
                            'sample': 'the same matvec, the sum of the workers\' single-threaded times'},
            'parts_sec': {'far_max_worker': round(max(r[0] for r in res), 3), 'far_sum': round(sum(r[0] for r in res), 2),
                          'near_all_blocks': round(t_near_all, 4), 'self_and_projection': round(t_self, 4)}}


if __name__ == '__main__':
    main()
