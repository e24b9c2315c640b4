"""Shared helpers for the GPU parity tests: one parameter set, two configs
(the oracle's and the C ABI's), and comparison utilities."""
import numpy as np

import oracle as O


def params(n, *, m, a, dt, B0=(0.0, 0.0, 0.05), species=((-1.0, 1.0),), r_rm=None, gamma_mode=0,
           deposit_mode=0, field_iters=3, damp_max=0.1, init_covariant=False, rk_mode=0, gather_mode=0,
           gather_weights=0, c=1.0, outer_layer=0.0, outer_damp=0.0):
    return dict(n=n, m=m, a=a, dt=dt, c=c, B0=tuple(B0), species=tuple(species), r_rm=r_rm,
                gamma_mode=gamma_mode, deposit_mode=deposit_mode, field_iters=field_iters,
                damp_max=damp_max, init_covariant=init_covariant, rk_mode=rk_mode, gather_mode=gather_mode,
                gather_weights=gather_weights, outer_layer=outer_layer, outer_damp=outer_damp)


def oracle_sim(P, ncap):
    p = O.make_params(P["n"], m=P["m"], a=P["a"], dt=P["dt"], c=P.get("c", 1.0), r_rm=P["r_rm"],
                      gamma_mode=P["gamma_mode"], deposit_mode=P["deposit_mode"],
                      field_iters=P["field_iters"], damp_max=P["damp_max"], species=P["species"],
                      rk_mode=P.get("rk_mode", 0), gather_mode=P.get("gather_mode", 0),
                      gather_weights=P.get("gather_weights", 0), outer_layer=P.get("outer_layer", 0.0),
                      outer_damp=P.get("outer_damp", 0.0))
    s = O.Sim(p, ncap)
    s.init_fields(list(P["B0"]), covariant=P["init_covariant"])
    return p, s


def gpu_run(P, capacity, sort_every=0, fp_bits=44, tile=4):
    from paper_0904_0232_amd import run as R
    cfg = R.make_config(P["n"], m=P["m"], a=P["a"], dt=P["dt"], c=P.get("c", 1.0), B0=P["B0"], species=P["species"],
                        r_rm=P["r_rm"], gamma_mode=P["gamma_mode"], deposit_mode=P["deposit_mode"],
                        field_iters=P["field_iters"], damp_max=P["damp_max"], sort_every=sort_every,
                        capacity=capacity, fp_bits=fp_bits, init_covariant=P["init_covariant"], tile=tile,
                        rk_mode=P.get("rk_mode", 0), gather_mode=P.get("gather_mode", 0),
                      gather_weights=P.get("gather_weights", 0), outer_layer=P.get("outer_layer", 0.0),
                      outer_damp=P.get("outer_damp", 0.0))
    return R.Run(cfg)


def rel_err(a, b, floor):
    """max |a-b| / max(|b|, floor), elementwise."""
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor))) if a.size else 0.0


def alive(x, u, sp):
    k = sp != O.DEAD
    return x[:, k], u[:, k], sp[k]


def say(*args):
    print(*args, flush=True)
