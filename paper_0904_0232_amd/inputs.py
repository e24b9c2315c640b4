"""Seeded synthetic inputs for the GRPIC workloads (shared by tests, the
benchmark and the oracle-side checks).

This module holds no arithmetic of the method itself (no metric evaluation,
push, gather, deposit or field step): it draws positions and
covariant spatial four-velocities from counter-based Philox streams (numpy's
Philox4x32-10, keyed by seed, purpose and species) and derives the species
table from the plasma-frequency choice.  Shapes follow the workloads:

- uniform Maxwellian plasma, ppc particles per cell and species, positions
  uniform inside each cell, ions at the electrons' positions (neutral start);
- torus n ~ exp(-((rho - 24)^2 + z^2)/50) moving on circular orbits: the
  Keplerian coordinate speed v = c sqrt(m/R) (Euclidean R, prograde = along
  the frame dragging of the metric, clockwise about +z for a > 0), given as
  the covariant velocity of the non-rotating hole's circular geodesic in
  Kerr-Schild form (closed-form initial data), plus thermal spread;
- uniform plasma with an infalling shell (|R - edge/4| <= 2 gets v_r = -0.3c).

Velocities are covariant spatial components u_i (the load call completes
them on the mass shell).  Charges: |Q| = (wpe dt)^2 / (dt^2 4 pi n |q/m|_e)
with wpe dt = 0.1 and n = ppc (the nominal density), electrons q/m = -1,
ions q/m = +1/mass_ratio.
"""
import math

import numpy as np

WPE_DT = 0.1
MASS_RATIO = 20.0

PURPOSE_POS, PURPOSE_VEL, PURPOSE_ACCEPT = 1, 2, 3


def rng(seed, purpose, species=0):
    key = (int(seed) << 32) | (int(purpose) << 8) | int(species)
    return np.random.Generator(np.random.Philox(key=key))


def species_table(dt, ppc, mass_ratio=MASS_RATIO, wpe_dt=WPE_DT):
    """Two species (electron, ion): ((charge, mass), (charge, mass))."""
    wpe = wpe_dt / dt
    Q = wpe * wpe / (4.0 * math.pi * float(ppc) * 1.0)
    return ((-Q, Q), (Q, Q * mass_ratio))


def uniform_positions(seed, nx, ny, nz, ppc):
    g = rng(seed, PURPOSE_POS)
    n = nx * ny * nz * ppc
    cell = np.arange(nx * ny * nz, dtype=np.int64).repeat(ppc)
    cx = cell % nx
    cy = (cell // nx) % ny
    cz = cell // (nx * ny)
    off = g.random((3, n))
    return np.stack([cx + off[0], cy + off[1], cz + off[2]]).astype(np.float64)


def maxwellian(seed, species, n, u_th):
    g = rng(seed, PURPOSE_VEL, species)
    return g.normal(0.0, u_th, (3, n))


def uniform_plasma(seed, nx, ny, nz, ppc, u_th, mass_ratio=MASS_RATIO):
    """[(species, x[3][n], ucov[3][n]), ...] for electrons and ions."""
    x = uniform_positions(seed, nx, ny, nz, ppc)
    n = x.shape[1]
    ue = maxwellian(seed, 0, n, u_th)
    ui = maxwellian(seed, 1, n, u_th / math.sqrt(mass_ratio))
    return [(0, x, ue), (1, x.copy(), ui)]


def torus_plasma(seed, nx, ny, nz, m, spin_sign, u_th, n_per_species, center=None,
                 rho0=24.0, width2=50.0, mass_ratio=MASS_RATIO, c=1.0):
    cen = np.array(center if center is not None else (nx / 2.0, ny / 2.0, nz / 2.0))
    g = rng(seed, PURPOSE_POS)
    ga = rng(seed, PURPOSE_ACCEPT)
    # n(rho, z) ~ exp(-((rho - rho0)^2 + z^2)/width2) per unit volume is
    # rho exp(...) per d rho d phi d z: z and phi are drawn directly, rho from
    # the Gaussian by rejection against the Jacobian rho / rho_max, and
    # points outside the grid are dropped.
    sig = math.sqrt(width2 / 2.0)
    rho_max = rho0 + 8.0 * sig
    lo = np.zeros(3)
    hi = np.array([nx, ny, nz], dtype=float)
    out = np.zeros((3, 0))
    while out.shape[1] < n_per_species:
        k = max(3 * (n_per_species - out.shape[1]), 1024)
        rho = g.normal(rho0, sig, k)
        z = g.normal(0.0, sig, k)
        phi = g.random(k) * (2.0 * math.pi)
        keep = (rho > 0.0) & (ga.random(k) * rho_max < rho)
        cand = np.stack([cen[0] + rho * np.cos(phi), cen[1] + rho * np.sin(phi), cen[2] + z])[:, keep]
        inside = np.all((cand >= lo[:, None]) & (cand < hi[:, None]), axis=0)
        out = np.concatenate([out, cand[:, inside]], axis=1)
    x = out[:, :n_per_species]
    d = x - cen[:, None]
    R = np.sqrt((d ** 2).sum(0))
    rho = np.maximum(np.hypot(d[0], d[1]), 1e-12)
    # Circular geodesic of the non-rotating hole of mass m written in
    # Kerr-Schild coordinates (closed-form initial data, the spin enters only
    # as a perturbation): coordinate speed v = c sqrt(m/R) along phi_hat,
    # u^4 = 1/sqrt(1 - 3m/R), no contravariant radial motion.  Lowering the
    # index with g = eta + f k k (f = 2m/R, k = (r_hat, 1)) adds f u^4 r_hat
    # to the spatial part, so the covariant velocity the loader takes is
    # u^4 (v phi_hat + f r_hat).  Inside R = 4m (no stable orbit there) the
    # R = 4m values are used.
    Rc = np.maximum(R, 4.0 * m / c ** 2) if m > 0 else np.maximum(R, 1e-12)
    v = c * np.sqrt(m / Rc)
    u4 = 1.0 / np.sqrt(1.0 - 3.0 * m / (c * c * Rc))
    f = 2.0 * m / (c * c * Rc)
    # prograde: with the frame dragging of the metric (clockwise for spin_sign > 0)
    sgn = -1.0 if spin_sign > 0 else 1.0
    phi_hat = np.stack([-d[1] / rho, d[0] / rho, np.zeros_like(rho)]) * sgn
    r_hat = d / np.maximum(R, 1e-12)
    base = u4 * (phi_hat * v + r_hat * (f * c))
    ue = base + maxwellian(seed, 0, n_per_species, u_th)
    ui = base + maxwellian(seed, 1, n_per_species, u_th / math.sqrt(mass_ratio))
    return [(0, x, ue), (1, x.copy(), ui)]


def shell_plasma(seed, nx, ny, nz, ppc, u_th, v_r=-0.3, width=2.0, center=None, mass_ratio=MASS_RATIO, c=1.0):
    species = uniform_plasma(seed, nx, ny, nz, ppc, u_th, mass_ratio)
    cen = np.array(center if center is not None else (nx / 2.0, ny / 2.0, nz / 2.0))
    x = species[0][1]
    d = x - cen[:, None]
    R = np.sqrt((d ** 2).sum(0))
    shell = np.abs(R - nx / 4.0) <= width
    gam = 1.0 / math.sqrt(1.0 - (v_r / c) ** 2)
    rhat = d[:, shell] / np.maximum(R[shell], 1e-12)
    for _, _, u in species:
        u[:, shell] += rhat * (gam * v_r)
    return species


def horizon_radius(m, a):
    return m + math.sqrt(max(m * m - a * a, 0.0))


# The workloads: grid edge n, hole (m, a/m), field, dt, steps, plasma.
WORKLOADS = {
    "schwarzschild32": dict(n=32, m=1.5, a_frac=0.0, B0=0.05, dt=0.5, steps=10, ppc=1, u_th=0.1,
                            plasma="uniform", r_rm_factor=None, r_rm=2.2 * 1.5),
    "kerr64": dict(n=64, m=3.0, a_frac=0.95, B0=0.1, dt=0.45, steps=200, ppc=8, u_th=0.1,
                   plasma="uniform"),
    "torus128": dict(n=128, m=4.0, a_frac=0.5, B0=0.1, dt=0.45, steps=1000, ppc=8, u_th=0.05,
                     plasma="torus"),
    "shell256": dict(n=256, m=8.0, a_frac=0.99, B0=0.1, dt=0.45, steps=100, ppc=8, u_th=0.1,
                     plasma="shell"),
}


def workload_params(name):
    """Derived plain parameters of a workload (no method arithmetic)."""
    w = dict(WORKLOADS[name])
    m, a = w["m"], w["a_frac"] * w["m"]
    rp = horizon_radius(m, a)
    w["a"] = a
    w["r_plus"] = rp
    w["r_rm"] = w.get("r_rm") or 1.1 * rp
    w["r_exc"] = 0.5 * rp
    w["r_damp"] = rp
    w["damp_max"] = 0.1
    w["species"] = species_table(w["dt"], w["ppc"])
    return w


def workload_particles(name, seed=0, n_override=None):
    w = workload_params(name)
    n = w["n"]
    if w["plasma"] == "uniform":
        return uniform_plasma(seed, n, n, n, w["ppc"], w["u_th"])
    if w["plasma"] == "torus":
        nps = n_override or 8 * n ** 3
        return torus_plasma(seed, n, n, n, w["m"], 1.0 if w["a"] >= 0 else -1.0, w["u_th"], nps)
    if w["plasma"] == "shell":
        return shell_plasma(seed, n, n, n, w["ppc"], w["u_th"])
    raise KeyError(w["plasma"])
