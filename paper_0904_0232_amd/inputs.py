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
- uniform plasma with an infalling shell (|R - edge/4| <= 2 gets v_r = -0.3c);
- the paper's application (a Keplerian disk and an infalling corona, c =
  0.05; its readings are listed at jet_params).

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


# The paper's application (Sec. 6): a Keplerian disk and an infalling
# corona around a spinning hole on a 64 x 64 x 128 grid with c = 0.05,
# dt = 1, contravariant B^z = 30 and q/m = 1e-3 (electrons and positrons),
# 500 steps.  Readings where the text is silent or garbled:
#  - the unit charge is unspecified; q = 1 makes the hole's mass length
#    m = G M_c / c^2 = (dx c^2)^2 M_c / c^2 = 0.75 cells for M_c = 300;
#  - r_S is the Schwarzschild radius 2m, so the disk's inner edge is
#    r_d = 3 r_S = 6m and v_K = c sqrt(r_S / 2r) = c sqrt(m/r) is Keplerian;
#  - the disk (|cos theta| < 1/8, r > r_d) runs out to the grid, with 800,000
#    particles in all (half of each species), cold, on circular orbits;
#  - the corona fills the rest outside r_rm at 1/100 of the disk density and
#    falls in from rest at infinity (radial, the non-rotating hole's
#    free-fall velocity);
#  - the macro charge gives wp dt = 0.1 at the disk density (as for the
#    other workloads), and the electrons and positrons start at the same
#    positions with the same velocities (neutral start).
JET = dict(nx=64, ny=64, nz=128, c=0.05, dt=1.0, steps=500, M_c=300.0, unit_charge=1.0, a_frac=0.95,
           B0=30.0, qm=1e-3, n_disk=800000, corona_fraction=0.01, disk_cos=1.0 / 8.0)


def jet_params():
    """Plain parameters of the jet workload (no method arithmetic)."""
    w = dict(JET)
    G = (1.0 * w["c"] ** 2 / w["unit_charge"]) ** 2  # dimensionless G with dx = 1
    m = G * w["M_c"] / w["c"] ** 2
    a = w["a_frac"] * m
    rp = horizon_radius(m, a)
    w.update(m=m, a=a, r_plus=rp, r_rm=1.1 * rp, r_s=2.0 * m, r_d=6.0 * m,
             center=(w["nx"] / 2.0, w["ny"] / 2.0, w["nz"] / 2.0))
    # disk volume (counted on a fine lattice) sets the disk density
    cen = np.array(w["center"])
    h = 0.25
    g = [np.arange(h / 2, n, h) - c0 for n, c0 in zip((w["nx"], w["ny"], w["nz"]), cen)]
    X, Y = np.meshgrid(g[0], g[1], indexing="ij")
    rho2 = X * X + Y * Y
    vol = 0.0
    for z in g[2]:
        r2 = rho2 + z * z
        vol += np.count_nonzero((r2 > w["r_d"] ** 2) & (z * z < w["disk_cos"] ** 2 * r2)) * h ** 3
    w["disk_volume"] = vol
    n_disk_species = w["n_disk"] / 2.0 / vol  # particles per cell and species in the disk
    wp = 0.1 / w["dt"]
    Q = wp * wp / (4.0 * math.pi * n_disk_species * w["qm"])
    w["species"] = ((-Q, Q / w["qm"]), (Q, Q / w["qm"]))
    return w


def jet_particles(seed=0, n_disk=None):
    """[(species, x[3][n], ucov[3][n])] for electrons and positrons."""
    w = jet_params()
    nx, ny, nz, c, m = w["nx"], w["ny"], w["nz"], w["c"], w["m"]
    cen = np.array(w["center"])
    nd = (n_disk or w["n_disk"]) // 2
    g = rng(seed, PURPOSE_POS)
    box = np.array([nx, ny, nz], dtype=float)

    def draw(n, want_disk):
        out = np.zeros((3, 0))
        while out.shape[1] < n:
            cand = g.random((3, max(4 * (n - out.shape[1]), 4096))) * box[:, None]
            d = cand - cen[:, None]
            r2 = (d * d).sum(0)
            disk = (r2 > w["r_d"] ** 2) & (d[2] ** 2 < w["disk_cos"] ** 2 * r2)
            keep = disk if want_disk else (~disk & (r2 > w["r_rm"] ** 2))
            out = np.concatenate([out, cand[:, keep]], axis=1)
        return out[:, :n]

    corona_volume = nx * ny * nz - w["disk_volume"] - 4.0 / 3.0 * math.pi * w["r_rm"] ** 3
    nc = int(round(w["corona_fraction"] * nd / w["disk_volume"] * corona_volume))
    xd, xc = draw(nd, True), draw(nc, False)
    # disk: circular geodesic of the non-rotating hole (coordinate speed
    # c sqrt(m/R) along phi_hat, prograde = along the frame dragging,
    # clockwise for a > 0; dx^4/dtau = c / sqrt(1 - 3m/R)); lowering with
    # g = eta + f k k (f = 2m/R, k = (r_hat, 1)) gives the covariant
    # u_i = u^4 (v/c phi_hat + f r_hat)
    d = xd - cen[:, None]
    R = np.sqrt((d * d).sum(0))
    rho = np.maximum(np.hypot(d[0], d[1]), 1e-12)
    phi_hat = -np.stack([-d[1] / rho, d[0] / rho, np.zeros_like(rho)])
    u4 = c / np.sqrt(1.0 - 3.0 * m / R)
    f = 2.0 * m / R
    ud = u4 * (phi_hat * np.sqrt(m / R) + (d / R) * f)
    # corona: free fall from rest at infinity, radial; in Kerr-Schild form
    # (u_4 = -c) the covariant radial component is -c sqrt(f) / (1 + sqrt(f))
    d = xc - cen[:, None]
    R = np.sqrt((d * d).sum(0))
    sf = np.sqrt(2.0 * m / R)
    uc = (d / R) * (-c * sf / (1.0 + sf))
    x = np.concatenate([xd, xc], axis=1)
    u = np.concatenate([ud, uc], axis=1)
    return [(0, x, u), (1, x.copy(), u.copy())]


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
