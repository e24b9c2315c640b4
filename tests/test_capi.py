"""Host-side checks of the C ABI library (no GPU needed): it loads and exports
every function declared in include/grpic.h, and the binding's structure
layouts agree with the header's field lists."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grpic.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(grpic_[a-z_0-9]+)\s*\(", src)))


def _lib():
    from paper_0904_0232_amd import capi
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("libgrpic.so not built")
    return ctypes.CDLL(capi.LIB_PATH)


def test_library_exports_every_declared_symbol():
    L = _lib()
    names = _declared_functions()
    assert "grpic_create" in names and "grpic_step" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def _struct_fields(name):
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + ";", src)
    body = m.group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        decl = re.sub(r"\[[^\]]*\]", "", decl)
        toks = decl.replace("*", " ").split()
        for part in " ".join(toks[1:]).split(","):
            out.append(part.strip().split()[-1])
    return out


def test_binding_struct_layouts_follow_header():
    from paper_0904_0232_amd import capi
    assert [f for f, _ in capi.Config._fields_] == _struct_fields("grpic_config")
    assert [f for f, _ in capi.Diag._fields_] == _struct_fields("grpic_diag")
    L = _lib()
    cfg = capi.Config()
    L.grpic_config_default(ctypes.byref(cfg), 16, 20, 24)
    assert (cfg.nx, cfg.ny, cfg.nz) == (16, 20, 24)
    assert cfg.field_iters == 3 and cfg.fp_bits == 44 and cfg.c == 1.0
    assert list(cfg.center) == [8.0, 10.0, 12.0]
    assert cfg.rk_mode == capi.RK_CLASSIC and cfg.gather_mode == capi.GATHER_STAGE
    L.grpic_config_size.restype = ctypes.c_size_t
    assert L.grpic_config_size() == ctypes.sizeof(capi.Config)


def test_strerror_codes():
    L = _lib()
    L.grpic_strerror.restype = ctypes.c_char_p
    assert L.grpic_strerror(0) == b"ok"
    assert L.grpic_strerror(-1) == b"invalid argument"


def test_config_check_plasma_frequency():
    """grpic_config_check (host only) applies the plasma-frequency criterion
    of Sec. 5.1, omega_p dt < 2 with omega_p^2 = 4 pi n q^2 / m, per species
    with a nominal density set, besides the other limits."""
    import math
    from paper_0904_0232_amd import capi
    _lib()
    cfg = capi.grpic_config_default(16)
    cfg.dt = 0.5
    cfg.nspecies = 2
    cfg.charge[0], cfg.mass[0] = -0.02, 0.02
    cfg.charge[1], cfg.mass[1] = 0.02, 0.4
    assert capi.grpic_config_check(cfg) == 0  # no density: not checked

    def density_for(wdt, q, m):
        w = wdt / cfg.dt
        return w * w * m / (4.0 * math.pi * q * q)

    for s, (q, m) in enumerate(((-0.02, 0.02), (0.02, 0.4))):
        cfg.density[0] = cfg.density[1] = 0.0
        cfg.density[s] = density_for(1.99, q, m)
        assert capi.grpic_config_check(cfg) == 0, s
        cfg.density[s] = density_for(2.01, q, m)
        assert capi.grpic_config_check(cfg) == capi.EINVAL, s
    cfg.density[0], cfg.density[1] = -1.0, 0.0
    assert capi.grpic_config_check(cfg) == capi.EINVAL
    cfg.density[0] = float("nan")
    assert capi.grpic_config_check(cfg) == capi.EINVAL
    # the workloads' own species tables sit at omega_pe dt = 0.1
    from paper_0904_0232_amd import inputs
    sp = inputs.species_table(0.45, 8)
    cfg = capi.grpic_config_default(32)
    cfg.dt, cfg.nspecies = 0.45, 2
    for s, (q, m) in enumerate(sp):
        cfg.charge[s], cfg.mass[s], cfg.density[s] = q, m, 8.0
    assert capi.grpic_config_check(cfg) == 0
    cfg.density[0] = 8.0 * 401.0  # omega_pe dt = 0.1 sqrt(401) > 2
    assert capi.grpic_config_check(cfg) == capi.EINVAL
    # the Courant condition c dt < 1/sqrt(3) (Sec. 5.2)
    cfg.density[0] = 8.0
    cfg.dt = 0.58
    assert capi.grpic_config_check(cfg) == capi.EINVAL
