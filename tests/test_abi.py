"""Host-side checks of the C-ABI library that need no GPU: it loads, it exports
every function the headers under include/ declare, the Python binding declares
the same set, and configuration validation / sizing behave as documented."""
import ctypes
import glob
import os
import re

import pytest

from paper_1806_10247_amd import capi as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(lb_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["lb_create", "lb_destroy", "lb_init_equilibrium", "lb_set_force_field", "lb_set_source_field",
                 "lb_step", "lb_read_moments", "lb_read_populations", "lb_totals", "lb_residual"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(C.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert sorted(C.SIGNATURES) == declared_functions()
    for n in declared_functions():
        assert callable(getattr(C, n))


def test_config_struct_matches_header_layout():
    # int32 x4, int64 x3, int32 x3 + int32, 7 doubles, pointer, int64, int32 x4
    assert ctypes.sizeof(C.lb_config) == 4 * 4 + 8 * 3 + 4 * 4 + 8 * 7 + 8 + 8 + 4 * 4


def test_validate_config():
    ok = C.lb_config_default(lattice=C.LB_D3Q27, nx=8, ny=8, nz=8)
    assert C.lb_validate_config(ok)[0] == C.LB_OK
    bad = [
        dict(nu=0.0), dict(nu=-1.0), dict(nx=0), dict(lattice=7), dict(storage=3), dict(abi_version=99),
        dict(lattice=C.LB_D2Q9, nz=0), dict(omega_bulk=2.0), dict(omega_third=0.0), dict(rho0=0.0),
        dict(block_x=96), dict(block_x=512), dict(residual_interval=-1), dict(flags=16),
        dict(rows_per_thread=3), dict(rows_per_thread=-1), dict(x_pairs=3), dict(x_pairs=-1),
        dict(x_pairs=2), dict(x_pairs=2, storage=C.LB_STORE_F16_DEV, nx=7),
        dict(x_pairs=2, storage=C.LB_STORE_F16_DEV, rows_per_thread=2),
        dict(x_pairs=2, storage=C.LB_STORE_F16_DEV, plane_pad=1),
        dict(lattice=C.LB_D2Q9_D2Q5, nz=1, D_phi=0.0), dict(bc=(0, 5, 0)),
        dict(nx=1 << 11, ny=1 << 11, nz=1 << 10),
        # the product nx*ny*nz wraps around int64 here; the check must not form it
        dict(nx=(1 << 21) + 1, ny=(1 << 21) + 1, nz=(1 << 21) + 1),
        dict(nx=1 << 30, ny=1 << 30, nz=1 << 30),
    ]
    for kw in bad:
        cfg = C.lb_config_default(lattice=kw.pop("lattice", C.LB_D3Q27), nx=8, ny=8, nz=8)
        if cfg.lattice != C.LB_D3Q27:
            cfg.nz = 1
        for k, v in kw.items():
            if k == "bc":
                for i in range(3):
                    cfg.bc[i] = v[i]
            else:
                setattr(cfg, k, v)
        rc, msg = C.lb_validate_config(cfg)
        assert rc == C.LB_EINVAL and msg, kw
    # a 2D lattice with nz > 1 is a stack of independent 2D lattices
    stack = C.lb_config_default(lattice=C.LB_D2Q9_D2Q5, nx=8, ny=8, nz=4, D_phi=0.1)
    assert C.lb_validate_config(stack)[0] == C.LB_OK


def test_required_bytes():
    cfg = C.lb_config_default(lattice=C.LB_D3Q27, storage=C.LB_STORE_F32_DEV, nx=256, ny=256, nz=256)
    n = 256**3
    b = C.lb_required_bytes(cfg)
    assert b >= 27 * n * 4
    assert b < 27 * (n + 8192) * 4
    cfg.plane_pad = 0
    assert C.lb_required_bytes(cfg) == 27 * n * 4
    cfg2 = C.lb_config_default(lattice=C.LB_D2Q9_D2Q5, storage=C.LB_STORE_F64, nx=10, ny=3, nz=1, plane_pad=2)
    assert C.lb_required_bytes(cfg2) == 14 * 32 * 8
    cfg2.nu = -1
    assert C.lb_required_bytes(cfg2) == 0


def test_create_rejects_bad_config_before_touching_the_gpu():
    cfg = C.lb_config_default(nu=-1.0)
    with pytest.raises(C.LbError) as e:
        C.lb_create(cfg)
    assert e.value.code == C.LB_EINVAL
    assert "nu" in C.lb_last_error(None)


def test_null_context_calls_fail_cleanly():
    assert C.lib().lb_step(None, 1) == C.LB_EINVAL
    assert C.lib().lb_get_step(None) == -1
    C.lb_destroy(None)


def test_unet_config_validation():
    """lb_unet_create rejects bad shapes before touching a device."""
    for kw in [dict(levels=0), dict(levels=7), dict(channels=(24, 32, 48, 96)), dict(in_channels=17),
               dict(out_channels=0), dict(height=200), dict(width=8), dict(max_batch=0), dict(abi_version=5)]:
        cfg = C.lb_unet_config_default(**kw)
        with pytest.raises(C.LbError) as e:
            C.lb_unet_create(cfg)
        assert e.value.code == C.LB_EINVAL, kw
