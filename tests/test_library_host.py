"""Host-side checks of librlbm.so that need no GPU: it loads, exports every symbol
include/rlbm.h declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rl():
    from paper_1709_09073_amd import rlbm
    # test_sanitized_host.py reruns this module against an instrumented build
    if os.environ.get("RLBM_TEST_LIBRARY"):
        rlbm.LIB_PATH = os.environ["RLBM_TEST_LIBRARY"]
    rlbm.lib()
    return rlbm


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rlbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rlbm_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(rl):
    names = declared_functions()
    assert "rlbm_init" in names and "rlbm_step" in names and "rlbm_moments" in names
    L = rl.lib()
    for nm in names:
        assert hasattr(L, nm), nm


def test_strerror(rl):
    L = rl.lib()
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert isinstance(L.rlbm_strerror(code), bytes)


def _params(**kw):
    from paper_1709_09073_amd import rlbm
    p = rlbm.Params(nx=16, ny=8, stats=0, order=5, precision=0, tau_mode=0, tau=1.0, tau_a=2.0, tau_b=0.25,
                    guess=0, mlp=None, f_a=ctypes.c_void_p(0x1000), f_b=ctypes.c_void_p(0x2000), stream=None)
    p.bc[:] = [0, 0, 0, 0]
    p.theta_wall[:] = [1.0, 1.0]
    for k, v in kw.items():
        if k == "bc":
            p.bc[:] = v
        elif k == "force":
            p.force[:] = v
        else:
            setattr(p, k, v)
    return p


INVALID = [
    dict(nx=1), dict(ny=0), dict(stats=3), dict(order=7), dict(order=1), dict(precision=5), dict(tau=0.0),
    dict(tau=0.5),   # gamma (1 + |u|)/2 >= 1/2 for every state: the relaxation would over-shoot
    dict(tau_mode=1, tau_b=0.0), dict(tau_mode=2), dict(bc=[0, 1, 0, 0]), dict(bc=[0, 0, 2, 2]),
    dict(bc=[2, 2, 0, 0], nx=3), dict(f_a=ctypes.c_void_p(0)), dict(f_b=ctypes.c_void_p(0x1000)),
    dict(tile_x=48, tile_y=5), dict(tile_x=8, tile_y=32), dict(tile_x=64, tile_y=2),
    # non-equilibrium walls: y sides only, ny >= 3, positive imposed state; finite force
    dict(bc=[3, 3, 0, 0], wall_n=1.0, wall_theta=1.0), dict(bc=[0, 0, 3, 3], ny=2, wall_n=1.0, wall_theta=1.0),
    dict(bc=[0, 0, 3, 3], wall_n=0.0, wall_theta=1.0), dict(bc=[0, 0, 3, 3], wall_n=1.0, wall_theta=-1.0),
    dict(force=(float("nan"), 0.0)),
]


@pytest.mark.parametrize("kw", INVALID)
def test_invalid_params_rejected(rl, kw):
    L = rl.lib()
    p = _params(**kw)
    fi = rl.InitFields(n=ctypes.c_void_p(0x10), z=None, theta=ctypes.c_void_p(0x10), ux=ctypes.c_void_p(0x10),
                       uy=ctypes.c_void_p(0x10), given_z=0)
    ctx = ctypes.c_void_p()
    assert L.rlbm_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.byref(fi)) == rl.RLBM_EINVAL
    assert not ctx.value


def test_lower_orders_only_for_maxwell_juttner(rl):
    L = rl.lib()
    p = _params(order=3, stats=1)
    fi = rl.InitFields(n=ctypes.c_void_p(0x10), z=None, theta=ctypes.c_void_p(0x10), ux=ctypes.c_void_p(0x10),
                       uy=ctypes.c_void_p(0x10), given_z=0)
    ctx = ctypes.c_void_p()
    assert L.rlbm_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.byref(fi)) == rl.RLBM_ENOTIMPL


@pytest.mark.parametrize("kw", [dict(force=(1e-6, 0.0), precision=2), dict(force=(1e-6, 0.0), order=3),
                                dict(bc=[0, 0, 3, 3], wall_n=1.0, wall_theta=1.0, precision=2)])
def test_forced_variant_limits(rl, kw):
    """Forced flow and non-equilibrium walls run at order 5 with FP64/FP32 populations."""
    L = rl.lib()
    p = _params(**kw)
    fi = rl.InitFields(n=ctypes.c_void_p(0x10), z=None, theta=ctypes.c_void_p(0x10), ux=ctypes.c_void_p(0x10),
                       uy=ctypes.c_void_p(0x10), given_z=0)
    ctx = ctypes.c_void_p()
    assert L.rlbm_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.byref(fi)) == rl.RLBM_ENOTIMPL


def test_missing_init_fields_rejected(rl):
    L = rl.lib()
    p = _params()
    fi = rl.InitFields(n=None, z=None, theta=ctypes.c_void_p(0x10), ux=ctypes.c_void_p(0x10),
                       uy=ctypes.c_void_p(0x10), given_z=0)
    ctx = ctypes.c_void_p()
    assert L.rlbm_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.byref(fi)) == rl.RLBM_EINVAL


def test_null_context_calls(rl):
    L = rl.lib()
    assert L.rlbm_step(None, 1) == rl.RLBM_EINVAL
    assert L.rlbm_sync(None) == rl.RLBM_EINVAL
    assert L.rlbm_state_index(None) == -1
    assert L.rlbm_noneq_tensors(None, 0, None, None, None, None) == rl.RLBM_EINVAL
    L.rlbm_free(None)


def test_struct_layouts_follow_the_header(rl):
    """The binding's structures carry every member of the header's, in order (the
    check flag of rlbm_params, the raw-moment outputs of rlbm_out_fields)."""
    src = open(os.path.join(ROOT, "include", "rlbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    for struct, cls in (("rlbm_params", rl.Params), ("rlbm_out_fields", rl.OutFields),
                        ("rlbm_init_fields", rl.InitFields)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (struct, struct), src, flags=re.S).group(1)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            decl = re.sub(r"^(const\s+)?\w+\s*", "", decl)
            for nm in decl.split(","):
                names.append(re.sub(r"[\s*]|\[\d+\]", "", nm))
        assert [f[0] for f in cls._fields_] == names, struct
