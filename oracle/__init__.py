"""ctypes front-end to the FP64 reference oracle in ``grpic_oracle.c``.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
CPU-baseline leg of the benchmark are the only callers.  Nothing here
imports the product package, and the product package never imports this.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grpic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAXSP = 8
DEAD = 0xFF


def build(force=False):
    """Compile the oracle with gcc (single-threaded, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("gamma_mode", ctypes.c_int32), ("deposit_mode", ctypes.c_int32),
        ("nspecies", ctypes.c_int32),
        ("field_iters", ctypes.c_int32), ("rk_mode", ctypes.c_int32),
        ("gather_mode", ctypes.c_int32), ("gather_weights", ctypes.c_int32),
        ("c", ctypes.c_double), ("dt", ctypes.c_double),
        ("m", ctypes.c_double), ("a", ctypes.c_double),
        ("center", ctypes.c_double * 3),
        ("r_rm", ctypes.c_double), ("r_exc", ctypes.c_double),
        ("r_damp", ctypes.c_double), ("damp_max", ctypes.c_double),
        ("outer_layer", ctypes.c_double), ("outer_damp", ctypes.c_double),
        ("charge", ctypes.c_double * MAXSP), ("mass", ctypes.c_double * MAXSP),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("n_alive", ctypes.c_int64 * MAXSP),
        ("n_removed_horizon", ctypes.c_int64), ("n_removed_outer", ctypes.c_int64),
        ("gamma_clamps", ctypes.c_int64), ("flags", ctypes.c_int64),
        ("charge_total", ctypes.c_double), ("energy_particles", ctypes.c_double),
        ("lz_particles", ctypes.c_double), ("energy_field", ctypes.c_double),
        ("gauss_residual_max", ctypes.c_double),
        ("mass_shell_residual_max", ctypes.c_double),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name == "n_alive" else v
        return out


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_U8 = ctypes.POINTER(ctypes.c_uint8)
_U32 = ctypes.POINTER(ctypes.c_uint32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_P = ctypes.POINTER(Params)


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.or_radius.restype = ctypes.c_double
        L.or_radius.argtypes = [ctypes.c_double] * 4
        L.or_metric.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D, _D]
        L.or_metric_deriv.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
        L.or_christoffel.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
        L.or_gather.argtypes = [_P, _D, _D, _D]
        L.or_gather_weights.argtypes = [_P, ctypes.POINTER(ctypes.c_int), _D, _D]
        L.or_spatial_density.restype = ctypes.c_double
        L.or_spatial_density.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.or_mass_shell.argtypes = [_P, _D, _D, _D]
        L.or_sim_new.restype = ctypes.c_void_p
        L.or_sim_new.argtypes = [_P, ctypes.c_int64]
        L.or_sim_free.argtypes = [ctypes.c_void_p]
        L.or_sim_gsize.restype = ctypes.c_size_t
        L.or_sim_gsize.argtypes = [ctypes.c_void_p]
        L.or_sim_init_fields.argtypes = [ctypes.c_void_p, _D]
        L.or_sim_init_fields2.argtypes = [ctypes.c_void_p, _D, ctypes.c_int]
        L.or_sim_set_fields.argtypes = [ctypes.c_void_p, _D, _D]
        L.or_sim_make_reference.argtypes = [ctypes.c_void_p]
        L.or_constitutive_point.argtypes = [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D, _D, _D]
        L.or_sim_get_fields.argtypes = [ctypes.c_void_p, ctypes.c_int, _D]
        L.or_sim_node_count.restype = ctypes.c_size_t
        L.or_sim_node_count.argtypes = [ctypes.c_void_p]
        L.or_sim_compute_nodes.argtypes = [ctypes.c_void_p]
        L.or_sim_prepare_push.argtypes = [ctypes.c_void_p]
        L.or_sim_compute_derived.argtypes = [ctypes.c_void_p]
        L.or_sim_get_nodes.argtypes = [ctypes.c_void_p, _D]
        L.or_sim_set_nodes.argtypes = [ctypes.c_void_p, _D]
        L.or_sim_set_particles.restype = ctypes.c_int
        L.or_sim_set_particles.argtypes = [ctypes.c_void_p, ctypes.c_int64, _D, _D, _U8]
        L.or_sim_get_particles.argtypes = [ctypes.c_void_p, _D, _D, _U8]
        L.or_sim_count.restype = ctypes.c_int64
        L.or_sim_count.argtypes = [ctypes.c_void_p]
        L.or_sim_load.restype = ctypes.c_int64
        L.or_sim_load.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, _D, _D]
        L.or_sim_push_only.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.or_sim_deposit_moves.argtypes = [ctypes.c_void_p, ctypes.c_int64, _D, _D, _D]
        L.or_charge_density.argtypes = [_P, ctypes.c_int64, _D, _D, _D]
        L.or_sim_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.or_sort_keys.argtypes = [_P, ctypes.c_int, ctypes.c_int64, _D, _U8, _U32]
        L.or_stable_order.argtypes = [ctypes.c_int64, _U32, _I64]
        L.or_sim_diag.argtypes = [ctypes.c_void_p, ctypes.POINTER(Diag)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(nx, ny=None, nz=None, *, c=1.0, dt=0.5, m=0.0, a=0.0, center=None,
                r_rm=None, r_exc=None, gamma_mode=0, deposit_mode=0,
                field_iters=3, r_damp=None, damp_max=0.1, species=((-1.0, 1.0),),
                rk_mode=0, gather_mode=0, gather_weights=0, outer_layer=0.0, outer_damp=0.0):
    """species: sequence of (macro charge, macro mass).  rk_mode 1 takes the
    printed RK steps literally, gather_mode 1 gathers the fields once at x_n,
    gather_weights 1 weights the gather by the spatial volume (all ablations
    of the default readings).  outer_layer > 0 turns on the outer absorbing
    layer of that width with relaxation fraction outer_damp at the faces."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    p = Params()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.gamma_mode, p.deposit_mode = gamma_mode, deposit_mode
    p.field_iters = field_iters
    p.rk_mode, p.gather_mode, p.gather_weights = rk_mode, gather_mode, gather_weights
    p.c, p.dt, p.m, p.a = c, dt, m, a
    cen = (nx / 2.0, ny / 2.0, nz / 2.0) if center is None else center
    for i in range(3):
        p.center[i] = cen[i]
    rplus = m + np.sqrt(max(m * m - a * a, 0.0))
    p.r_rm = 1.1 * rplus if r_rm is None else r_rm
    p.r_exc = 0.5 * rplus if r_exc is None else r_exc
    p.r_damp = rplus if r_damp is None else r_damp
    p.damp_max = damp_max
    p.outer_layer, p.outer_damp = outer_layer, outer_damp
    p.nspecies = len(species)
    for i, (q, mass) in enumerate(species):
        p.charge[i] = q
        p.mass[i] = mass
    return p


def gather_weights(p, c, X):
    """The 8 cloud-in-cell weights (index di + 2 dj + 4 dk) of cell c at X."""
    ci = (ctypes.c_int * 3)(*[int(v) for v in c])
    W = np.zeros(8)
    lib().or_gather_weights(ctypes.byref(p), ci, _dp(np.ascontiguousarray(X, dtype=float)), _dp(W))
    return W


def spatial_density(p, x, y, z):
    return lib().or_spatial_density(ctypes.byref(p), x, y, z)


def radius(a, x, y, z):
    return lib().or_radius(a, x, y, z)


def metric(p, x, y, z):
    g = np.zeros(16)
    gi = np.zeros(16)
    r = ctypes.c_double()
    lib().or_metric(ctypes.byref(p), x, y, z, _dp(g), _dp(gi), ctypes.byref(r))
    return g.reshape(4, 4), gi.reshape(4, 4), r.value


def metric_deriv(p, x, y, z):
    dg = np.zeros(48)
    lib().or_metric_deriv(ctypes.byref(p), x, y, z, _dp(dg))
    return dg.reshape(3, 4, 4)


def christoffel(p, x, y, z):
    G = np.zeros(64)
    lib().or_christoffel(ctypes.byref(p), x, y, z, _dp(G))
    return G.reshape(4, 4, 4)


def constitutive_point(p, X, Fs_lo, Ft_up):
    """The grid's constitutive step at the point X (node coordinates): from
    (F_23, F_31, F_12) and (F^14, F^24, F^34) to (F_14, F_24, F_34) and
    (F^23, F^31, F^12)."""
    a = _f64(Fs_lo)
    b = _f64(Ft_up)
    tl = np.zeros(3)
    su = np.zeros(3)
    lib().or_constitutive_point(ctypes.byref(p), float(X[0]), float(X[1]), float(X[2]), _dp(a), _dp(b), _dp(tl),
                                _dp(su))
    return tl, su


def mass_shell(p, X, ucov):
    out = np.zeros(4)
    X = _f64(X)
    uc = _f64(ucov)
    lib().or_mass_shell(ctypes.byref(p), _dp(X), _dp(uc), _dp(out))
    return out


def charge_density(p, x, Q):
    x = _f64(x)
    Q = _f64(Q)
    n = x.shape[1]
    out = np.zeros((p.nz + 3) * (p.ny + 3) * (p.nx + 3))
    lib().or_charge_density(ctypes.byref(p), n, _dp(x), _dp(Q), _dp(out))
    return out.reshape(p.nz + 3, p.ny + 3, p.nx + 3)


def sort_keys(p, tile, x, sp):
    x = _f64(x)
    sp = np.ascontiguousarray(sp, dtype=np.uint8)
    n = sp.shape[0]
    keys = np.zeros(n, dtype=np.uint32)
    lib().or_sort_keys(ctypes.byref(p), tile, n, _dp(x), sp.ctypes.data_as(_U8),
                       keys.ctypes.data_as(_U32))
    return keys


def stable_order(keys):
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    perm = np.zeros(keys.shape[0], dtype=np.int64)
    lib().or_stable_order(keys.shape[0], keys.ctypes.data_as(_U32), perm.ctypes.data_as(_I64))
    return perm


class Sim:
    """One oracle simulation: ghosted field arrays and SoA particles."""

    def __init__(self, params, ncap=0):
        self.p = params
        self.L = lib()
        self.h = self.L.or_sim_new(ctypes.byref(params), int(ncap))
        self.gshape = (params.nz + 3, params.ny + 3, params.nx + 3)
        self.gsize = self.L.or_sim_gsize(self.h)
        self.nnodes = self.L.or_sim_node_count(self.h)

    def __del__(self):
        if getattr(self, "h", None):
            self.L.or_sim_free(self.h)
            self.h = None

    def init_fields(self, B0, covariant=False):
        b = _f64(B0)
        self.L.or_sim_init_fields2(self.h, _dp(b), 1 if covariant else 0)

    def set_fields(self, D, B):
        D = _f64(D).reshape(-1)
        B = _f64(B).reshape(-1)
        assert D.size == 3 * self.gsize and B.size == 3 * self.gsize
        self.L.or_sim_set_fields(self.h, _dp(D), _dp(B))

    def make_reference(self):
        """Take the current fields as the reference state (frozen points and
        relaxation targets)."""
        self.L.or_sim_make_reference(self.h)

    def get(self, which):
        """which: 'D', 'B', 'E', 'H', 'J' (3 comps) or 'rho_abs'."""
        idx = {"D": 0, "B": 1, "E": 2, "H": 3, "J": 4, "rho_abs": 5}[which]
        if idx == 5:
            out = np.zeros(self.gsize)
            self.L.or_sim_get_fields(self.h, 5, _dp(out))
            return out.reshape(self.gshape)
        out = np.zeros(3 * self.gsize)
        self.L.or_sim_get_fields(self.h, idx, _dp(out))
        return out.reshape((3,) + self.gshape)

    def compute_nodes(self):
        self.L.or_sim_compute_nodes(self.h)

    def prepare_push(self):
        self.L.or_sim_prepare_push(self.h)

    def compute_derived(self):
        self.L.or_sim_compute_derived(self.h)

    def nodes(self):
        out = np.zeros(16 * self.nnodes)
        self.L.or_sim_get_nodes(self.h, _dp(out))
        return out.reshape(self.p.nz + 1, self.p.ny + 1, self.p.nx + 1, 4, 4)

    def set_nodes(self, F):
        F = _f64(F).reshape(-1)
        assert F.size == 16 * self.nnodes
        self.L.or_sim_set_nodes(self.h, _dp(F))

    def set_particles(self, x, u, sp):
        x = _f64(x)
        u = _f64(u)
        sp = np.ascontiguousarray(sp, dtype=np.uint8)
        n = sp.shape[0]
        rc = self.L.or_sim_set_particles(self.h, n, _dp(x), _dp(u), sp.ctypes.data_as(_U8))
        if rc != 0:
            raise ValueError("particle capacity exceeded")

    def particles(self):
        n = self.L.or_sim_count(self.h)
        x = np.zeros((3, n))
        u = np.zeros((4, n))
        sp = np.zeros(n, dtype=np.uint8)
        self.L.or_sim_get_particles(self.h, _dp(x), _dp(u), sp.ctypes.data_as(_U8))
        return x, u, sp

    def load(self, species, x, ucov):
        x = _f64(x)
        uc = _f64(ucov)
        n = x.shape[1]
        kept = self.L.or_sim_load(self.h, species, n, _dp(x), _dp(uc))
        if kept < 0:
            raise ValueError("particle capacity exceeded")
        return kept

    def push_only(self, nsteps, use_nodes=True):
        self.L.or_sim_push_only(self.h, int(nsteps), 1 if use_nodes else 0)

    def deposit_moves(self, x1, x2, Q):
        x1 = _f64(x1)
        x2 = _f64(x2)
        Q = _f64(Q)
        self.L.or_sim_deposit_moves(self.h, x1.shape[1], _dp(x1), _dp(x2), _dp(Q))

    def step(self, nsteps=1):
        self.L.or_sim_step(self.h, int(nsteps))

    def diag(self):
        d = Diag()
        self.L.or_sim_diag(self.h, ctypes.byref(d))
        return d.as_dict()
