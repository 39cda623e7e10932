"""Thin ctypes binding of libbipqn.so: argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays
to pointers and back. Names follow the C ABI in include/bipqn.h. Loading fails
loudly when the library has not been built.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, 'libbipqn.so')

PQN_OK, PQN_WARN_NOT_CONVERGED = 0, 1
PQN_FP64, PQN_MIXED = 0, 1
PQN_BBPGD, PQN_MONO, PQN_BI, PQN_BI_REC = 0, 1, 2, 3
PQN_HIFI, PQN_LOFI, PQN_LOFI2 = 0, 1, 2
SOLVERS = {'bb': PQN_BBPGD, 'mono': PQN_MONO, 'bi': PQN_BI, 'birec': PQN_BI_REC}


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class ConfigDesc(C.Structure):
    _fields_ = [('n_particles', C.c_int32), ('radius', C.c_double), ('mu', C.c_double),
                ('n_theta', C.c_int32), ('n_phi', C.c_int32), ('n_theta_lo', C.c_int32), ('n_phi_lo', C.c_int32),
                ('gmres_tol', C.c_double), ('gmres_tol_lo', C.c_double), ('gmres_restart', C.c_int32),
                ('gmres_max_iter', C.c_int32), ('near_gap', C.c_double), ('near_up', C.c_int32),
                ('slip_speed', C.c_double), ('precision', C.c_int32), ('refine_sweeps', C.c_int32),
                ('targets_per_thread', C.c_int32), ('far_chunks', C.c_int32), ('far_split', C.c_int32),
                ('device', C.c_int32),
                ('stream', C.c_void_p), ('profile', C.c_int32), ('use_graphs', C.c_int32),
                ('warm_start', C.c_int32), ('n_theta_lo2', C.c_int32), ('n_phi_lo2', C.c_int32),
                ('gmres_tol_lo2', C.c_double), ('dev_alloc', _ALLOC_FN), ('dev_free', _FREE_FN),
                ('alloc_user', C.c_void_p), ('side_stream', C.c_int32), ('near_close_gap', C.c_double),
                ('near_close_up', C.c_int32), ('far_coarse_lo', C.c_int32), ('far_coarse_lo2', C.c_int32),
                ('precond', C.c_int32), ('precond_coarse', C.c_int32)]


class TorchAllocator:
    """dev_alloc / dev_free of pqn_config_desc through the PyTorch caching allocator.

    Blocks are taken for `stream` (an int hipStream_t handle), the stream the
    context runs on. The object must outlive the context (pqn_destroy returns
    its blocks through dev_free).
    """

    def __init__(self, device, stream):
        import torch
        self.device, self.stream = int(device), int(stream)
        self.live = 0

        def _alloc(nbytes, user):
            try:
                ptr = torch.cuda.caching_allocator_alloc(max(int(nbytes), 1), self.device, self.stream)
            except Exception:  # reported to the library as NULL -> PQN_ERR_OOM
                return None
            self.live += 1
            return ptr

        def _free(ptr, user):
            torch.cuda.caching_allocator_delete(ptr)
            self.live -= 1

        self.alloc_fn = _ALLOC_FN(_alloc)
        self.free_fn = _FREE_FN(_free)

    def fill(self, d):
        d.dev_alloc, d.dev_free, d.alloc_user = self.alloc_fn, self.free_fn, None


class MvpStats(C.Structure):
    _fields_ = [('gmres_iters', C.c_int32), ('matvecs', C.c_int32), ('refine_sweeps', C.c_int32),
                ('converged', C.c_int32), ('rel_residual', C.c_double), ('t_total_ms', C.c_double),
                ('t_far_ms', C.c_double), ('n_far', C.c_int32), ('graph_launches', C.c_int32),
                ('fp64_fallback', C.c_int32), ('t_near_ms', C.c_double), ('t_gemm_ms', C.c_double),
                ('t_local_ms', C.c_double), ('t_arnoldi_ms', C.c_double), ('t_precond_ms', C.c_double),
                ('precond_fallback', C.c_int32), ('precond_applies', C.c_int32),
                ('t_precond_apply_ms', C.c_double), ('t_far_by_k_ms', C.c_double * 6),
                ('n_far_by_k', C.c_int32 * 6), ('precond_coarse_steps', C.c_int32),
                ('precond_coarse_warm', C.c_int32)]


class LcpOpts(C.Structure):
    _fields_ = [('k_max', C.c_int32), ('k_max_inner', C.c_int32), ('j_max', C.c_int32),
                ('kkt_tol_abs', C.c_double), ('kkt_tol_rel', C.c_double), ('ssn_tol', C.c_double),
                ('printed_metric', C.c_int32), ('recycle', C.c_int32)]


class LcpStats(C.Structure):
    _fields_ = [('iters', C.c_int32), ('mvp_hi', C.c_int32), ('mvp_lo', C.c_int32), ('emvp', C.c_double),
                ('lo_hi_cost_ratio', C.c_double), ('kkt_abs', C.c_double), ('converged', C.c_int32),
                ('ssn_steps', C.c_int32), ('t_total_ms', C.c_double), ('gmres_iters', C.c_int32),
                ('model_rejected', C.c_int32), ('mvp_lo2', C.c_int32), ('lo2_hi_cost_ratio', C.c_double),
                ('kkt_rel', C.c_double), ('nonpos_curvature', C.c_int32)]


class StepStats(C.Structure):
    _fields_ = [('n_contacts', C.c_int32), ('n_active', C.c_int32), ('lcp', LcpStats),
                ('gmres_iters_nc', C.c_int32), ('t_total_ms', C.c_double), ('t_contacts_ms', C.c_double),
                ('t_nc_ms', C.c_double), ('t_lcp_ms', C.c_double), ('t_update_ms', C.c_double)]


def _struct_dict(s):
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        if isinstance(v, C.Structure):
            v = _struct_dict(v)
        elif isinstance(v, C.Array):
            v = list(v)
        out[name] = v
    return out


_LIB = None
_P = C.POINTER
_D = _P(C.c_double)
_I = _P(C.c_int32)


def lib():
    """Load libbipqn.so (raises if it has not been built).

    PyTorch is imported first when it is installed: its bundled HIP runtime
    carries the same soname as the system one the library links, so the
    library then binds to the runtime already in the process and torch's
    device pointers and streams are valid in library calls. Loading the
    library first would put a second HIP runtime into the process.
    """
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f'{LIB_PATH} is missing: build it first (python -m paper_2604_10089_amd.build)')
    try:
        import torch  # noqa: F401  (loads the process's HIP runtime; no device is touched)
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    V = C.c_void_p
    sig = {
        'pqn_create': (C.c_int, [_P(ConfigDesc), _D, _D, _P(V)]),
        'pqn_destroy': (C.c_int, [V]),
        'pqn_set_state': (C.c_int, [V, _D, _D]),
        'pqn_get_state': (C.c_int, [V, _D, _D]),
        'pqn_set_precision': (C.c_int, [V, C.c_int32]),
        'pqn_mobility_apply': (C.c_int, [V, _D, _D, C.c_int32, _P(MvpStats)]),
        'pqn_mobility_apply_dev': (C.c_int, [V, V, V, C.c_int32, _P(MvpStats)]),
        'pqn_mobility_apply_multi_dev': (C.c_int, [V, C.c_int32, V, V, C.c_int32, _P(MvpStats)]),
        'pqn_nc_velocity': (C.c_int, [V, _D, C.c_int32, _P(MvpStats)]),
        'pqn_find_contacts': (C.c_int, [V, C.c_double, C.c_int32, _I, _I, _D]),
        'pqn_find_contacts_noalloc': (C.c_int, [V, C.c_double, C.c_int32, _I, _I, _D]),
        'pqn_lcp_apply': (C.c_int, [V, C.c_int32, _I, _D, _D, C.c_int32]),
        'pqn_lcp_solve': (C.c_int, [V, C.c_int32, _I, _D, _D, C.c_int32, _P(LcpOpts), _P(LcpStats)]),
        'pqn_lcp_solve_dev': (C.c_int, [V, C.c_int32, V, V, V, C.c_int32, _P(LcpOpts), _P(LcpStats)]),
        'pqn_step': (C.c_int, [V, C.c_double, C.c_double, C.c_int32, _P(LcpOpts), _P(StepStats)]),
        'pqn_bie_apply': (C.c_int, [V, C.c_int32, _D, _D]),
        'pqn_bie_apply_multi': (C.c_int, [V, C.c_int32, C.c_int32, _D, _D]),
        'pqn_get_self_block': (C.c_int, [V, C.c_int32, _D]),
        'pqn_bie_solve': (C.c_int, [V, C.c_int32, _D, _D, _P(MvpStats)]),
        'pqn_get_grid': (C.c_int, [V, C.c_int32, _I, _D, _D]),
        'pqn_host_self_block': (C.c_int, [C.c_int32, C.c_int32, C.c_double, _D, _D, _D]),
        'pqn_host_sphere_block': (C.c_int, [C.c_int32, C.c_int32, C.c_double, _D, _D]),
        'pqn_mobility_apply_multi': (C.c_int, [V, C.c_int32, _D, _D, C.c_int32, _P(MvpStats)]),
        'pqn_batch_create': (C.c_int, [C.c_int32, _P(ConfigDesc), _P(_D), _P(_D), _P(V)]),
        'pqn_batch_mobility_apply': (C.c_int, [V, _P(_D), _P(_D), _P(MvpStats), _P(MvpStats)]),
        'pqn_batch_mobility_apply_dev': (C.c_int, [V, _P(V), _P(V), _P(MvpStats), _P(MvpStats)]),
        'pqn_last_error': (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


class PqnError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f'status {status}: {msg}')
        self.status = status


def _check(status, allow_warn=True):
    if status < 0 or (status == PQN_WARN_NOT_CONVERGED and not allow_warn):
        raise PqnError(status, lib().pqn_last_error().decode())
    return status


def _dptr(a):
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def pqn_host_self_block(n_theta, n_phi, radius=1.0):
    """(offsets [n,3], weights [n], S [3n,3n]) built on the host without a device."""
    n = n_theta * n_phi
    off = np.zeros((n, 3))
    w = np.zeros(n)
    S = np.zeros((3 * n, 3 * n))
    _check(lib().pqn_host_self_block(n_theta, n_phi, radius, _dptr(off), _dptr(w), _dptr(S)))
    return off, w, S


def pqn_host_sphere_block(n_theta, n_phi, radius=1.0):
    """(D, D^{-1}), the single-sphere block 1/2 I + S + P_rigid [3n,3n] (SoA order) and its
    inverse, built on the host without a device."""
    n3 = 3 * n_theta * n_phi
    D = np.zeros((n3, n3))
    Di = np.zeros((n3, n3))
    _check(lib().pqn_host_sphere_block(n_theta, n_phi, radius, _dptr(D), _dptr(Di)))
    return D, Di


def _desc(M, n_theta, n_phi, lo=None, radius=1.0, mu=1.0, gmres_tol=1e-8, gmres_tol_lo=None, restart=50,
          max_iter=500, near_gap=0.0, near_up=2, slip=1.0, precision='fp64', refine=0, tpt=2, far_chunks=0,
          far_split=0, device=0, stream=None, profile=False, graphs=False, warm_start=False, lo2=None,
          gmres_tol_lo2=None, allocator=None, side_stream=False, near_close_gap=0.0, near_close_up=3,
          far_coarse_lo=0, far_coarse_lo2=0, precond=False, precond_coarse=False):
    d = ConfigDesc()
    d.n_particles = M
    d.radius, d.mu = radius, mu
    d.n_theta, d.n_phi = n_theta, n_phi
    if lo is not None:
        d.n_theta_lo, d.n_phi_lo = lo
    if lo2 is not None:
        d.n_theta_lo2, d.n_phi_lo2 = lo2
    d.gmres_tol = gmres_tol
    d.gmres_tol_lo = gmres_tol if gmres_tol_lo is None else gmres_tol_lo
    d.gmres_tol_lo2 = gmres_tol if gmres_tol_lo2 is None else gmres_tol_lo2
    d.gmres_restart, d.gmres_max_iter = restart, max_iter
    d.near_gap, d.near_up, d.slip_speed = near_gap, near_up, slip
    d.precision = PQN_MIXED if precision == 'mixed' else PQN_FP64
    d.refine_sweeps = refine
    d.targets_per_thread = tpt
    d.far_chunks = far_chunks
    d.far_split = 1 if far_split else 0
    d.device = device
    d.stream = stream
    d.profile = 1 if profile else 0
    d.use_graphs = 1 if graphs else 0
    d.warm_start = 1 if warm_start else 0
    if allocator is not None:
        allocator.fill(d)
    d.side_stream = 1 if side_stream else 0
    d.near_close_gap, d.near_close_up = near_close_gap, near_close_up
    d.far_coarse_lo, d.far_coarse_lo2 = far_coarse_lo, far_coarse_lo2
    # precond: False / 0 = plain GMRES, True / 1 = built when a configuration is solved a second
    # time, 'eager' / 2 = built at its first solve
    d.precond = 2 if precond in ('eager', 2) else (1 if precond else 0)
    # precond_coarse: the two-level form (a coarse correction on degree <= 2 harmonics)
    d.precond_coarse = 1 if precond_coarse else 0
    return d


def _torch_stream(device, stream):
    """(handle, owner): the given hipStream_t handle, or a new torch stream kept alive by
    the caller (a stream the library does not create, so it outlives the context's
    last dev_free)."""
    if stream is not None:
        return int(stream), None
    import torch
    st = torch.cuda.Stream(device=device)
    return int(st.cuda_stream), st


class BatchContext:
    """Independent suspensions of uneven size in one batch context (pqn_batch_*)."""

    def __init__(self, instances, torch_alloc=False, **kw):
        """instances: list of (centers [M,3], n_theta, n_phi); kw: shared settings as in Context.
        Without tpt / far_chunks / far_split the far launch shape comes from the autotuner's
        cache for this batch (else 2 targets per thread, automatic chunks)."""
        n = len(instances)
        if not any(k in kw for k in ('tpt', 'far_chunks', 'far_split')):
            hit = None
            try:
                from paper_2604_10089_amd import autotune
                hit = autotune.lookup_batch(kw.get('precision', 'fp64'),
                                            [(_f64(c).reshape(-1, 3), nt, nph) for c, nt, nph in instances])
            except Exception:
                hit = None
            if hit is not None:
                kw['tpt'], kw['far_chunks'], kw['far_split'] = hit
        self.far_shape = dict(tpt=kw.get('tpt', 2), chunks=kw.get('far_chunks', 0),
                              split=int(bool(kw.get('far_split', 0))))
        descs = (ConfigDesc * n)()
        self._centers = [_f64(c).reshape(-1, 3) for c, _, _ in instances]
        self.Ms = [c.shape[0] for c in self._centers]
        self._alloc = None
        if torch_alloc:
            kw['stream'], self._stream_obj = _torch_stream(kw.get('device', 0), kw.get('stream'))
            self._alloc = TorchAllocator(kw.get('device', 0), kw['stream'])
        for b, (c, nt, nph) in enumerate(instances):
            descs[b] = _desc(self.Ms[b], nt, nph, allocator=self._alloc, **kw)
        cp = (_D * n)(*[_dptr(c) for c in self._centers])
        h = C.c_void_p()
        _check(lib().pqn_batch_create(n, descs, cp, None, C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, 'h', None):
            lib().pqn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def mobility_apply(self, FTs, per_instance=False):
        F = [_f64(f, (m, 6)) for f, m in zip(FTs, self.Ms)]
        U = [np.zeros((m, 6)) for m in self.Ms]
        fp = (_D * len(F))(*[_dptr(f) for f in F])
        up = (_D * len(U))(*[_dptr(u) for u in U])
        st = MvpStats()
        per = (MvpStats * len(F))()
        status = _check(lib().pqn_batch_mobility_apply(self.h, fp, up, C.byref(st), per))
        out = dict(_struct_dict(st), status=status)
        if per_instance:
            out['per_instance'] = [_struct_dict(p) for p in per]
        return U, out

    def mobility_apply_dev(self, FT_ptrs, UO_ptrs):
        """Device arrays [M_b][6] per suspension (integer device pointers)."""
        n = len(self.Ms)
        fp = (C.c_void_p * n)(*FT_ptrs)
        up = (C.c_void_p * n)(*UO_ptrs)
        st = MvpStats()
        per = (MvpStats * n)()
        status = _check(lib().pqn_batch_mobility_apply_dev(self.h, fp, up, C.byref(st), per))
        return dict(_struct_dict(st), status=status, per_instance=[_struct_dict(p) for p in per])


def tuned_shape(precision, K, M, n):
    """(tpt, far_chunks, far_split) from the autotuner's cache for this shape, else the library defaults."""
    try:
        from paper_2604_10089_amd import autotune
        hit = autotune.lookup(precision, K, M, n)
    except Exception:
        hit = None
    return hit if hit is not None else (2, 0, 0)


class Context:
    """Owns one pqn_ctx. Methods carry the C ABI names without the prefix.

    tpt / far_chunks / far_split = None take the autotuned launch shape for
    (precision, densities per pass tune_K, sphere count, grid) when the cache
    has one.
    """

    def __init__(self, centers, axes=None, n_theta=8, n_phi=16, lo=None, radius=1.0, mu=1.0,
                 gmres_tol=1e-8, gmres_tol_lo=None, restart=50, max_iter=500, near_gap=0.0, near_up=2,
                 slip=1.0, precision='fp64', refine=0, tpt=None, far_chunks=None, far_split=None, device=0,
                 stream=None, profile=False, tune_K=1, graphs=False, warm_start=False, lo2=None,
                 gmres_tol_lo2=None, torch_alloc=False, side_stream=False, near_close_gap=0.0, near_close_up=3,
                 far_coarse_lo=0, far_coarse_lo2=0, precond=False, precond_coarse=False):
        c = _f64(centers).reshape(-1, 3)
        self.M = c.shape[0]
        self._alloc = None
        if torch_alloc:
            stream, self._stream_obj = _torch_stream(device, stream)
            self._alloc = TorchAllocator(device, stream)
        if tpt is None or far_chunks is None or far_split is None:
            t2, c2, s2 = tuned_shape(precision, tune_K, self.M, n_theta * n_phi)
            tpt = t2 if tpt is None else tpt
            far_chunks = c2 if far_chunks is None else far_chunks
            far_split = s2 if far_split is None else far_split
        self.far_shape = dict(tpt=tpt, chunks=far_chunks, split=int(bool(far_split)))
        d = _desc(self.M, n_theta, n_phi, lo=lo, radius=radius, mu=mu, gmres_tol=gmres_tol,
                  gmres_tol_lo=gmres_tol_lo, restart=restart, max_iter=max_iter, near_gap=near_gap,
                  near_up=near_up, slip=slip, precision=precision, refine=refine, tpt=tpt,
                  far_chunks=far_chunks, far_split=far_split, device=device, stream=stream, profile=profile,
                  graphs=graphs, warm_start=warm_start, lo2=lo2, gmres_tol_lo2=gmres_tol_lo2,
                  allocator=self._alloc, side_stream=side_stream, near_close_gap=near_close_gap,
                  near_close_up=near_close_up, far_coarse_lo=far_coarse_lo, far_coarse_lo2=far_coarse_lo2,
                  precond=precond, precond_coarse=precond_coarse)
        self.n_theta, self.n_phi, self.lo, self.lo2 = n_theta, n_phi, lo, lo2
        ax = None if axes is None else _f64(axes).reshape(-1, 3)
        h = C.c_void_p()
        _check(lib().pqn_create(C.byref(d), _dptr(c), None if ax is None else _dptr(ax), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, 'h', None):
            lib().pqn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_state(self, centers, axes=None):
        c = _f64(centers).reshape(-1, 3)
        ax = None if axes is None else _f64(axes).reshape(-1, 3)
        _check(lib().pqn_set_state(self.h, _dptr(c), None if ax is None else _dptr(ax)))

    def get_state(self):
        c = np.zeros((self.M, 3))
        ax = np.zeros((self.M, 3))
        _check(lib().pqn_get_state(self.h, _dptr(c), _dptr(ax)))
        return c, ax

    def set_precision(self, precision):
        _check(lib().pqn_set_precision(self.h, PQN_MIXED if precision == 'mixed' else PQN_FP64))

    def mobility_apply(self, FT, fidelity=PQN_HIFI):
        FT = _f64(FT, (self.M, 6))
        UO = np.zeros((self.M, 6))
        st = MvpStats()
        status = _check(lib().pqn_mobility_apply(self.h, _dptr(FT), _dptr(UO), fidelity, C.byref(st)))
        return UO, dict(_struct_dict(st), status=status)

    def mobility_apply_multi(self, FT, fidelity=PQN_HIFI):
        FT = _f64(FT).reshape(-1, self.M, 6)
        UO = np.zeros_like(FT)
        st = MvpStats()
        status = _check(lib().pqn_mobility_apply_multi(self.h, FT.shape[0], _dptr(FT), _dptr(UO), fidelity,
                                                       C.byref(st)))
        return UO, dict(_struct_dict(st), status=status)

    def mobility_apply_dev(self, FT_ptr, UO_ptr, fidelity=PQN_HIFI):
        st = MvpStats()
        status = _check(lib().pqn_mobility_apply_dev(self.h, C.c_void_p(FT_ptr), C.c_void_p(UO_ptr), fidelity,
                                                     C.byref(st)))
        return dict(_struct_dict(st), status=status)

    def mobility_apply_multi_dev(self, k_rhs, FT_ptr, UO_ptr, fidelity=PQN_HIFI):
        """K force sets in device memory: FT_ptr, UO_ptr address [K][M][6] FP64 arrays."""
        st = MvpStats()
        status = _check(lib().pqn_mobility_apply_multi_dev(self.h, k_rhs, C.c_void_p(FT_ptr), C.c_void_p(UO_ptr),
                                                           fidelity, C.byref(st)))
        return dict(_struct_dict(st), status=status)

    def nc_velocity(self, fidelity=PQN_HIFI):
        UO = np.zeros((self.M, 6))
        st = MvpStats()
        status = _check(lib().pqn_nc_velocity(self.h, _dptr(UO), fidelity, C.byref(st)))
        return UO, dict(_struct_dict(st), status=status)

    def find_contacts(self, delta):
        n = C.c_int32(0)
        L = lib()
        st = L.pqn_find_contacts(self.h, delta, 0, C.byref(n), None, None)
        if st < 0 and n.value == 0:
            _check(st)
        cap = max(n.value, 1)
        pairs = np.zeros((cap, 2), dtype=np.int32)
        gaps = np.zeros(cap)
        _check(L.pqn_find_contacts(self.h, delta, cap, C.byref(n), pairs.ctypes.data_as(_I), _dptr(gaps)))
        return pairs[:n.value].copy(), gaps[:n.value].copy()

    def lcp_apply(self, pairs, x, fidelity=PQN_HIFI):
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        x = _f64(x)
        Ax = np.zeros(pairs.shape[0])
        _check(lib().pqn_lcp_apply(self.h, pairs.shape[0], pairs.ctypes.data_as(_I), _dptr(x), _dptr(Ax),
                                   fidelity))
        return Ax

    def lcp_solve(self, pairs, b, solver='mono', k_max=0, k_max_inner=0, j_max=0, tol_abs=0.0, tol_rel=0.0,
                  x0=None, ssn_tol=0.0, printed_metric=False, recycle=False):
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        b = _f64(b)
        x = np.zeros(pairs.shape[0]) if x0 is None else _f64(x0, (pairs.shape[0],)).copy()
        o = LcpOpts(k_max, k_max_inner, j_max, tol_abs, tol_rel, ssn_tol, int(printed_metric), int(recycle))
        st = LcpStats()
        status = _check(lib().pqn_lcp_solve(self.h, pairs.shape[0], pairs.ctypes.data_as(_I), _dptr(b), _dptr(x),
                                            SOLVERS.get(solver, solver), C.byref(o), C.byref(st)))
        return x, dict(_struct_dict(st), status=status)

    def lcp_solve_dev(self, n, pairs_ptr, b_ptr, x_ptr, solver='mono', k_max=0, k_max_inner=0, j_max=0,
                      tol_abs=0.0, tol_rel=0.0, ssn_tol=0.0, printed_metric=False, recycle=False):
        """pqn_lcp_solve_dev on device pointers (ints, e.g. torch tensors' data_ptr())."""
        o = LcpOpts(k_max, k_max_inner, j_max, tol_abs, tol_rel, ssn_tol, int(printed_metric), int(recycle))
        st = LcpStats()
        status = _check(lib().pqn_lcp_solve_dev(self.h, n, C.c_void_p(pairs_ptr), C.c_void_p(b_ptr),
                                                C.c_void_p(x_ptr), SOLVERS.get(solver, solver), C.byref(o),
                                                C.byref(st)))
        return dict(_struct_dict(st), status=status)

    def step(self, dt, delta, solver='mono', k_max=0, k_max_inner=0, j_max=0, tol_abs=0.0, tol_rel=0.0,
             ssn_tol=0.0, printed_metric=False, recycle=False):
        o = LcpOpts(k_max, k_max_inner, j_max, tol_abs, tol_rel, ssn_tol, int(printed_metric), int(recycle))
        st = StepStats()
        status = _check(lib().pqn_step(self.h, dt, delta, SOLVERS.get(solver, solver), C.byref(o), C.byref(st)))
        return dict(_struct_dict(st), status=status)

    def bie_apply(self, q_soa, fidelity=PQN_HIFI):
        q = _f64(q_soa).ravel()
        y = np.zeros_like(q)
        _check(lib().pqn_bie_apply(self.h, fidelity, _dptr(q), _dptr(y)))
        return y.reshape(3, -1)

    def bie_apply_multi(self, q_soa, fidelity=PQN_HIFI):
        """q_soa [k][3][N] -> y [k][3][N], the k densities in one pass."""
        q = _f64(q_soa)
        k = q.shape[0]
        y = np.zeros_like(q)
        _check(lib().pqn_bie_apply_multi(self.h, fidelity, k, _dptr(q), _dptr(y)))
        return y

    def bie_solve(self, rhs_soa, fidelity=PQN_HIFI):
        r = _f64(rhs_soa).ravel()
        q = np.zeros_like(r)
        st = MvpStats()
        status = _check(lib().pqn_bie_solve(self.h, fidelity, _dptr(r), _dptr(q), C.byref(st)))
        return q.reshape(3, -1), dict(_struct_dict(st), status=status)

    def get_self_block(self, fidelity=PQN_HIFI):
        n = self.get_grid(fidelity)[0].shape[0]
        S = np.zeros((3 * n, 3 * n))
        _check(lib().pqn_get_self_block(self.h, fidelity, _dptr(S)))
        return S

    def get_grid(self, fidelity=PQN_HIFI):
        n = C.c_int32(0)
        _check(lib().pqn_get_grid(self.h, fidelity, C.byref(n), None, None))
        off = np.zeros((n.value, 3))
        w = np.zeros(n.value)
        _check(lib().pqn_get_grid(self.h, fidelity, C.byref(n), _dptr(off), _dptr(w)))
        return off, w
