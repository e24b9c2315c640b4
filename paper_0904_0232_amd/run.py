"""Convenience layer over the C ABI: build a grpic_config from plain
parameters, create the run on PyTorch's current stream with PyTorch-owned
device memory, and load the seeded particles.  No computation happens here.
"""
from . import capi


def make_config(n, *, m, a, dt, B0=(0.0, 0.0, 0.0), species=((-1.0, 1.0),), c=1.0, r_rm=None,
                r_exc=None, r_damp=None, damp_max=0.1, gamma_mode=capi.GAMMA_PAPER,
                deposit_mode=capi.DEPOSIT_CURVED, field_iters=3, sort_every=0, tile=4, fp_bits=44,
                capacity=0, precision=capi.FP64, init_covariant=False, ny=None, nz=None, center=None,
                rk_mode=capi.RK_CLASSIC, gather_mode=capi.GATHER_STAGE,
                gather_weights=capi.WEIGHTS_TRILINEAR, outer_layer=0.0, outer_damp=0.0, density=None):
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    cfg = capi.grpic_config_default(n, ny, nz)
    cfg.precision = precision
    cfg.gamma_mode = gamma_mode
    cfg.deposit_mode = deposit_mode
    cfg.rk_mode = rk_mode
    cfg.gather_mode = gather_mode
    cfg.gather_weights = gather_weights
    cfg.field_iters = field_iters
    cfg.sort_every = sort_every
    cfg.tile = tile
    cfg.fp_bits = fp_bits
    cfg.c, cfg.dt, cfg.m, cfg.a = c, dt, m, a
    cen = center if center is not None else (n / 2.0, ny / 2.0, nz / 2.0)
    for i in range(3):
        cfg.center[i] = cen[i]
        cfg.B0[i] = B0[i]
    rp = m + max(m * m - a * a, 0.0) ** 0.5
    cfg.r_rm = 1.1 * rp if r_rm is None else r_rm
    cfg.r_exc = 0.5 * rp if r_exc is None else r_exc
    cfg.r_damp = rp if r_damp is None else r_damp
    cfg.damp_max = damp_max
    cfg.outer_layer, cfg.outer_damp = outer_layer, outer_damp
    cfg.init_covariant = 1 if init_covariant else 0
    cfg.nspecies = len(species)
    for i, (q, mass) in enumerate(species):
        cfg.charge[i] = q
        cfg.mass[i] = mass
        # nominal macro-particles per cell for the plasma-frequency check (0: none)
        cfg.density[i] = 0.0 if density is None else float(density[i] if hasattr(density, "__len__") else density)
    cfg.capacity = int(capacity)
    return cfg


class Run:
    """One GRPIC run on the current torch device/stream."""

    def __init__(self, cfg, torch_memory=True):
        import torch
        torch.cuda.set_device(torch.cuda.current_device())
        self.cfg = cfg
        self.memory = capi.TorchMemory() if torch_memory else None
        self.stream = torch.cuda.current_stream()
        self.h = capi.grpic_create(cfg, self.stream.cuda_stream, self.memory)
        self.nnodes = (cfg.nx + 1) * (cfg.ny + 1) * (cfg.nz + 1)
        self.gshape = (cfg.nz + 3, cfg.ny + 3, cfg.nx + 3)

    def load(self, species, x, ucov):
        return capi.grpic_load_particles(self.h, species, x, ucov)

    def step(self, n=1):
        capi.grpic_step(self.h, n)

    def push_only(self, n=1):
        capi.grpic_push_only(self.h, n)

    def diag(self, allow_overflow=False):
        return capi.grpic_diagnostics(self.h, allow_overflow)

    def particles(self):
        return capi.grpic_dump_particles(self.h)

    def save_state(self):
        """Checkpoint: the run's full state as bytes (numpy uint8)."""
        return capi.grpic_save_state(self.h)

    def load_state(self, state):
        """Resume from a checkpoint of a run with the same configuration."""
        capi.grpic_load_state(self.h, state)

    def restore_particles(self, x, u, sp):
        capi.grpic_restore_particles(self.h, x, u, sp)

    def fields(self, which):
        idx = {"D": 0, "B": 1, "E": 2, "H": 3, "J": 4}[which]
        return capi.grpic_dump_fields(self.h, idx).reshape((3,) + self.gshape)

    def restore_fields(self, D, B):
        capi.grpic_restore_fields(self.h, D, B)

    def nodes(self):
        return capi.grpic_dump_nodes(self.h, self.nnodes).reshape(
            self.cfg.nz + 1, self.cfg.ny + 1, self.cfg.nx + 1, 4, 4)

    def sort(self, outputs=True):
        return capi.grpic_sort(self.h, outputs)

    def close(self):
        if self.h:
            capi.grpic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
