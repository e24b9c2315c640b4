"""ctypes binding of the C ABI in include/grpic.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  Device
memory comes from PyTorch's caching allocator through the allocator
callbacks of ``grpic_config`` and work goes onto PyTorch's current HIP
stream; all computation happens in the HIP kernels of ``libgrpic.so``.
Importing this module fails loudly if the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgrpic.so")

MAX_SPECIES = 8
DEAD = 0xFF
FP64, FP32_MIXED = 0, 1
GAMMA_PAPER, GAMMA_U4 = 0, 1
DEPOSIT_CURVED, DEPOSIT_FLAT = 0, 1
RK_CLASSIC, RK_PRINTED = 0, 1
GATHER_STAGE, GATHER_STEP = 0, 1
WEIGHTS_TRILINEAR, WEIGHTS_SPATIAL = 0, 1

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("gamma_mode", ctypes.c_int32),
        ("deposit_mode", ctypes.c_int32), ("field_iters", ctypes.c_int32),
        ("sort_every", ctypes.c_int32), ("tile", ctypes.c_int32), ("fp_bits", ctypes.c_int32),
        ("nspecies", ctypes.c_int32), ("init_covariant", ctypes.c_int32),
        ("rk_mode", ctypes.c_int32), ("gather_mode", ctypes.c_int32), ("gather_weights", ctypes.c_int32),
        ("c", ctypes.c_double), ("dt", ctypes.c_double),
        ("m", ctypes.c_double), ("a", ctypes.c_double),
        ("center", ctypes.c_double * 3),
        ("r_rm", ctypes.c_double), ("r_exc", ctypes.c_double),
        ("r_damp", ctypes.c_double), ("damp_max", ctypes.c_double),
        ("outer_layer", ctypes.c_double), ("outer_damp", ctypes.c_double),
        ("B0", ctypes.c_double * 3),
        ("charge", ctypes.c_double * MAX_SPECIES), ("mass", ctypes.c_double * MAX_SPECIES),
        ("density", ctypes.c_double * MAX_SPECIES),
        ("capacity", ctypes.c_int64),
        ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", ctypes.c_void_p),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("n_alive", ctypes.c_int64 * MAX_SPECIES),
        ("n_removed_horizon", ctypes.c_int64), ("n_removed_outer", ctypes.c_int64),
        ("gamma_clamps", ctypes.c_int64), ("flags", ctypes.c_int64),
        ("charge_total", ctypes.c_double), ("energy_particles", ctypes.c_double),
        ("lz_particles", ctypes.c_double), ("energy_field", ctypes.c_double),
        ("gauss_residual_max", ctypes.c_double),
        ("mass_shell_residual_max", ctypes.c_double),
        ("deposit_blocks_lds", ctypes.c_int64), ("deposit_blocks_global", ctypes.c_int64),
        ("push_blocks_lds", ctypes.c_int64), ("push_blocks_global", ctypes.c_int64),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name == "n_alive" else v
        return out


class GrpicError(RuntimeError):
    def __init__(self, msg, code=0):
        super().__init__(msg)
        self.code = code


EINVAL = -1
EOVERFLOW = -4
ESTATE = -5
EAGAIN = -6
RUN_UNKNOWN, RUN_ACTIVE, RUN_DONE, RUN_PREEMPTED = 0, 1, 2, 3


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_U32 = ctypes.POINTER(ctypes.c_uint32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_H = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgrpic.so is not built: run `python -m paper_0904_0232_amd.build`")
        # PyTorch ships its own HIP runtime under the same soname; load it first
        # so that the library binds to that one runtime instead of a second copy.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        L.grpic_config_default.argtypes = [ctypes.POINTER(Config), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.grpic_config_default.restype = None
        L.grpic_config_size.argtypes = []
        L.grpic_config_size.restype = ctypes.c_size_t
        if L.grpic_config_size() != ctypes.sizeof(Config):
            raise GrpicError("grpic_config layout mismatch: library %d bytes, binding %d"
                             % (L.grpic_config_size(), ctypes.sizeof(Config)))
        L.grpic_config_check.argtypes = [ctypes.POINTER(Config)]
        L.grpic_config_check.restype = ctypes.c_int
        L.grpic_create.argtypes = [ctypes.POINTER(Config), ctypes.c_void_p, ctypes.POINTER(_H)]
        L.grpic_load_particles.argtypes = [_H, ctypes.c_int32, ctypes.c_int64, _D, _D, _I64]
        L.grpic_load_particles_noalloc.argtypes = [_H, ctypes.c_int32, ctypes.c_int64, _D, _D, _I64]
        L.grpic_load_particles_noalloc.restype = ctypes.c_int
        L.grpic_step.argtypes = [_H, ctypes.c_int32]
        L.grpic_push_only.argtypes = [_H, ctypes.c_int32]
        L.grpic_diagnostics.argtypes = [_H, ctypes.POINTER(Diag)]
        L.grpic_particle_count.argtypes = [_H, _I64, _I64]
        L.grpic_dump_particles.argtypes = [_H, _D, _D, _U8]
        L.grpic_restore_particles.argtypes = [_H, ctypes.c_int64, _D, _D, _U8]
        L.grpic_field_size.argtypes = [_H]
        L.grpic_field_size.restype = ctypes.c_int64
        L.grpic_dump_fields.argtypes = [_H, ctypes.c_int32, _D]
        L.grpic_restore_fields.argtypes = [_H, _D, _D]
        L.grpic_dump_nodes.argtypes = [_H, _D]
        L.grpic_state_bytes.argtypes = [_H]
        L.grpic_state_bytes.restype = ctypes.c_int64
        L.grpic_save_state.argtypes = [_H, ctypes.c_void_p, ctypes.c_int64]
        L.grpic_load_state.argtypes = [_H, ctypes.c_void_p, ctypes.c_int64]
        L.grpic_sort.argtypes = [_H, _U32, _I64]
        L.grpic_set_timing.argtypes = [_H, ctypes.c_int32]
        L.grpic_set_graphs.argtypes = [_H, ctypes.c_int32]
        L.grpic_set_graphs.restype = ctypes.c_int
        L.grpic_read_timing.argtypes = [_H, _D, _I64]
        L.grpic_particle_steps.argtypes = [_H, _I64]
        L.grpic_run_bytes.argtypes = [ctypes.POINTER(Config)]
        L.grpic_run_bytes.restype = ctypes.c_int64
        L.grpic_batch_create.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(_H)]
        L.grpic_batch_submit.argtypes = [_H, ctypes.POINTER(Config), ctypes.c_int32, ctypes.c_int32, _I64,
                                         ctypes.POINTER(_D), ctypes.POINTER(_D), _I64]
        L.grpic_batch_step.argtypes = [_H, ctypes.POINTER(ctypes.c_int32)]
        L.grpic_batch_poll.argtypes = [_H, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(Diag), _I64, _I64]
        L.grpic_batch_dump.argtypes = [_H, ctypes.c_int64, _D, _D, _U8]
        L.grpic_batch_release.argtypes = [_H, ctypes.c_int64]
        L.grpic_batch_stats.argtypes = [_H, ctypes.POINTER(ctypes.c_int32), _I64]
        L.grpic_batch_state_bytes.argtypes = [_H, ctypes.c_int64]
        L.grpic_batch_state_bytes.restype = ctypes.c_int64
        L.grpic_batch_preempt.argtypes = [_H, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64]
        L.grpic_batch_resume.argtypes = [_H, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64]
        L.grpic_batch_destroy.argtypes = [_H]
        L.grpic_batch_destroy.restype = None
        L.grpic_destroy.argtypes = [_H]
        L.grpic_destroy.restype = None
        L.grpic_strerror.argtypes = [ctypes.c_int]
        L.grpic_strerror.restype = ctypes.c_char_p
        for name in ("grpic_create", "grpic_load_particles", "grpic_step", "grpic_push_only",
                     "grpic_diagnostics", "grpic_particle_count", "grpic_dump_particles",
                     "grpic_restore_particles", "grpic_dump_fields", "grpic_restore_fields",
                     "grpic_dump_nodes", "grpic_sort", "grpic_set_timing", "grpic_read_timing",
                     "grpic_particle_steps", "grpic_batch_create", "grpic_batch_submit",
                     "grpic_batch_step", "grpic_batch_poll", "grpic_batch_dump", "grpic_batch_release",
                     "grpic_batch_stats", "grpic_batch_preempt", "grpic_batch_resume"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise GrpicError("grpic error %d: %s" % (rc, lib().grpic_strerror(rc).decode()), rc)


def _dp(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class TorchMemory:
    """Device allocator backed by torch's caching allocator (kept alive with the handle)."""

    def __init__(self):
        import torch
        self._torch = torch
        self._blocks = {}
        self.alloc_calls = 0
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        self.alloc_calls += 1
        try:
            t = self._torch.empty(int(nbytes), dtype=self._torch.uint8, device="cuda")
        except Exception:
            return None
        ptr = t.data_ptr()
        self._blocks[ptr] = t
        return ptr

    def _free(self, ptr, ctx):
        self._blocks.pop(ptr, None)

    def bytes_held(self):
        return sum(t.numel() for t in self._blocks.values())


def grpic_config_default(nx, ny=None, nz=None):
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    cfg = Config()
    lib().grpic_config_default(ctypes.byref(cfg), nx, ny, nz)
    return cfg


def grpic_create(cfg, stream=None, memory=None):
    """Returns the handle (an int).  memory: a TorchMemory (None: the library's hipMalloc)."""
    if memory is not None:
        cfg.alloc = memory.alloc
        cfg.free = memory.free
    h = _H()
    _check(lib().grpic_create(ctypes.byref(cfg), ctypes.c_void_p(stream or 0), ctypes.byref(h)))
    return h


def grpic_load_particles(h, species, x, ucov):
    x = _f64(x)
    uc = _f64(ucov)
    n = x.shape[1]
    assert x.shape == (3, n) and uc.shape == (3, n)
    kept = ctypes.c_int64()
    _check(lib().grpic_load_particles(h, int(species), n, _dp(x), _dp(uc), ctypes.byref(kept)))
    return kept.value


def grpic_load_particles_noalloc(h, species, x, ucov):
    """grpic_load_particles through the library's fixed staging array (no
    device allocation; at most 2^20 particles per call)."""
    x = _f64(x)
    uc = _f64(ucov)
    n = x.shape[1]
    assert x.shape == (3, n) and uc.shape == (3, n)
    kept = ctypes.c_int64()
    _check(lib().grpic_load_particles_noalloc(h, int(species), n, _dp(x), _dp(uc), ctypes.byref(kept)))
    return kept.value


def grpic_step(h, nsteps=1):
    _check(lib().grpic_step(h, int(nsteps)))


def grpic_push_only(h, nsteps=1):
    _check(lib().grpic_push_only(h, int(nsteps)))


def grpic_config_check(cfg):
    """0 (valid) or a negative error code; no device call."""
    return lib().grpic_config_check(ctypes.byref(cfg))


def grpic_diagnostics(h, allow_overflow=False):
    """The diagnostics as a dict.  GRPIC_EOVERFLOW raises unless
    allow_overflow (the filled diagnostics are returned then)."""
    d = Diag()
    rc = lib().grpic_diagnostics(h, ctypes.byref(d))
    if not (allow_overflow and rc == EOVERFLOW):
        _check(rc)
    return d.as_dict()


def grpic_particle_count(h):
    n = ctypes.c_int64()
    cap = ctypes.c_int64()
    _check(lib().grpic_particle_count(h, ctypes.byref(n), ctypes.byref(cap)))
    return n.value, cap.value


def grpic_dump_particles(h):
    n, _ = grpic_particle_count(h)
    x = np.zeros((3, n))
    u = np.zeros((4, n))
    sp = np.zeros(n, dtype=np.uint8)
    _check(lib().grpic_dump_particles(h, _dp(x), _dp(u), sp.ctypes.data_as(_U8)))
    return x, u, sp


def grpic_restore_particles(h, x, u, sp):
    x = _f64(x)
    u = _f64(u)
    sp = np.ascontiguousarray(sp, dtype=np.uint8)
    _check(lib().grpic_restore_particles(h, sp.shape[0], _dp(x), _dp(u), sp.ctypes.data_as(_U8)))


def grpic_save_state(h):
    """The run's full state as a uint8 array (see grpic_save_state)."""
    nb = lib().grpic_state_bytes(h)
    _check(int(nb) if nb < 0 else 0)
    buf = np.zeros((nb + 7) // 8, dtype=np.uint64)  # 8-byte aligned
    _check(lib().grpic_save_state(h, buf.ctypes.data, nb))
    return buf.view(np.uint8)[:nb]


def grpic_load_state(h, state):
    """Replace the run's state by one from grpic_save_state."""
    state = np.asarray(state, dtype=np.uint8)
    buf = np.zeros((state.size + 7) // 8, dtype=np.uint64)
    buf.view(np.uint8)[:state.size] = state
    _check(lib().grpic_load_state(h, buf.ctypes.data, state.size))


def grpic_field_size(h):
    return lib().grpic_field_size(h)


def grpic_dump_fields(h, which):
    """which: 0 D, 1 B_cov, 2 E_cov, 3 H, 4 J; returns [3][field_size]."""
    gs = grpic_field_size(h)
    out = np.zeros(3 * gs)
    _check(lib().grpic_dump_fields(h, int(which), _dp(out)))
    return out.reshape(3, gs)


def grpic_restore_fields(h, D, B):
    D = _f64(D).reshape(-1)
    B = _f64(B).reshape(-1)
    _check(lib().grpic_restore_fields(h, _dp(D), _dp(B)))


def grpic_dump_nodes(h, nnodes):
    out = np.zeros(16 * nnodes)
    _check(lib().grpic_dump_nodes(h, _dp(out)))
    return out


def grpic_sort(h, outputs=True):
    if not outputs:
        _check(lib().grpic_sort(h, None, None))
        return None
    n, _ = grpic_particle_count(h)
    keys = np.zeros(n, dtype=np.uint32)
    perm = np.zeros(n, dtype=np.int64)
    _check(lib().grpic_sort(h, keys.ctypes.data_as(_U32), perm.ctypes.data_as(_I64)))
    return keys, perm


NTIMERS = 4
TIMER_NAMES = ("push", "deposit", "fields", "sort")


def grpic_set_timing(h, enable=True):
    _check(lib().grpic_set_timing(h, 1 if enable else 0))


def grpic_set_graphs(h, enable=True):
    _check(lib().grpic_set_graphs(h, 1 if enable else 0))


def grpic_read_timing(h):
    ms = np.zeros(NTIMERS)
    n = np.zeros(NTIMERS, dtype=np.int64)
    _check(lib().grpic_read_timing(h, _dp(ms), n.ctypes.data_as(_I64)))
    return {name: (float(ms[i]), int(n[i])) for i, name in enumerate(TIMER_NAMES)}


def grpic_particle_steps(h):
    v = ctypes.c_int64()
    _check(lib().grpic_particle_steps(h, ctypes.byref(v)))
    return v.value


def grpic_destroy(h):
    if h:
        lib().grpic_destroy(h)


def grpic_run_bytes(cfg):
    return lib().grpic_run_bytes(ctypes.byref(cfg))


def grpic_batch_create(budget_bytes, max_slots):
    b = _H()
    _check(lib().grpic_batch_create(int(budget_bytes), int(max_slots), ctypes.byref(b)))
    return b


def grpic_batch_submit(b, cfg, nsteps, species_particles, keep_state=False):
    """species_particles: [(x[3][n], ucov[3][n]) per species].  Returns the run id,
    or None when the batch has no free slot or memory right now."""
    ns = len(species_particles)
    xs = [_f64(x) for x, _ in species_particles]
    us = [_f64(u) for _, u in species_particles]
    n = np.array([x.shape[1] for x in xs], dtype=np.int64)
    xp = (_D * ns)(*[_dp(x) for x in xs])
    up = (_D * ns)(*[_dp(u) for u in us])
    rid = ctypes.c_int64()
    rc = lib().grpic_batch_submit(b, ctypes.byref(cfg), int(nsteps), 1 if keep_state else 0,
                                  n.ctypes.data_as(_I64), xp, up, ctypes.byref(rid))
    if rc == EAGAIN:
        return None
    _check(rc)
    return rid.value


def grpic_batch_step(b):
    fin = ctypes.c_int32()
    _check(lib().grpic_batch_step(b, ctypes.byref(fin)))
    return fin.value


def grpic_batch_poll(b, run_id):
    st = ctypes.c_int32()
    done = ctypes.c_int32()
    d = Diag()
    ns = ctypes.c_int64()
    ps = ctypes.c_int64()
    _check(lib().grpic_batch_poll(b, int(run_id), ctypes.byref(st), ctypes.byref(done), ctypes.byref(d),
                                  ctypes.byref(ns), ctypes.byref(ps)))
    return st.value, done.value, (d.as_dict() if st.value == RUN_DONE else None), ns.value, ps.value


def grpic_batch_dump(b, run_id, n_slots):
    x = np.zeros((3, n_slots))
    u = np.zeros((4, n_slots))
    sp = np.zeros(n_slots, dtype=np.uint8)
    _check(lib().grpic_batch_dump(b, int(run_id), _dp(x), _dp(u), sp.ctypes.data_as(_U8)))
    return x, u, sp


def grpic_batch_release(b, run_id):
    _check(lib().grpic_batch_release(b, int(run_id)))


def grpic_batch_preempt(b, run_id):
    """Save an active run's state and free its slot and memory; returns the
    state as a uint8 array, the format of grpic_save_state."""
    nb = lib().grpic_batch_state_bytes(b, int(run_id))
    _check(int(nb) if nb < 0 else 0)
    buf = np.empty((nb + 7) // 8, dtype=np.uint64)  # 8-byte aligned; the save writes every byte used
    _check(lib().grpic_batch_preempt(b, int(run_id), buf.ctypes.data, nb))
    return buf.view(np.uint8)[:nb]


def grpic_batch_resume(b, run_id, state):
    """Re-admit a preempted run from its saved state; False when the batch
    has no free slot or memory right now."""
    state = np.asarray(state, dtype=np.uint8)
    if state.flags.c_contiguous and state.ctypes.data % 8 == 0:
        buf = state  # as returned by grpic_batch_preempt: no copy
    else:
        buf = np.zeros((state.size + 7) // 8, dtype=np.uint64)
        buf.view(np.uint8)[:state.size] = state
    rc = lib().grpic_batch_resume(b, int(run_id), buf.ctypes.data, state.size)
    if rc == EAGAIN:
        return False
    _check(rc)
    return True


def grpic_batch_stats(b):
    a = ctypes.c_int32()
    by = ctypes.c_int64()
    _check(lib().grpic_batch_stats(b, ctypes.byref(a), ctypes.byref(by)))
    return a.value, by.value


def grpic_batch_destroy(b):
    if b:
        lib().grpic_batch_destroy(b)
