"""The C-ABI library builds, loads and exports every declared symbol; host
argument checks reject bad calls before anything reaches a GPU (no GPU
needed: invalid calls return before the context is used)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def declared_functions():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", text, flags=re.M):
            name = m.group(1)
            if name not in ("if", "defined") and not text[m.start():m.end()].startswith("#"):
                names.append(name)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_2007_15385_amd as P
    if not os.path.exists(P.lib_path()):
        from paper_2007_15385_amd import build
        build.build()
    return P.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("pip_create", "pip_destroy", "pip_status_str", "pip_last_error",
                 "polygon_to_generators", "pip_voronoi", "pip_sign_of_offset",
                 "pip_ray_crossing", "pip_voronoi_fp32_plain", "pip_voronoi_max_margin"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"


def test_status_strings_and_version(lib):
    for code, name in [(0, b"PIP_OK"), (1, b"PIP_EINVAL"), (2, b"PIP_EDEGENERATE"),
                       (3, b"PIP_ENONCONVEX"), (4, b"PIP_EHIP"), (5, b"PIP_ENOMEM"),
                       (6, b"PIP_EUNSUPPORTED")]:
        assert lib.pip_status_str(code) == name
    assert lib.pip_version() >= 100


def test_null_context_and_null_out(lib):
    assert lib.pip_create(0, None) == 1
    assert lib.pip_voronoi(None, 8, 4, 16, 0, 10, 32, None, None) == 1
    assert b"ctx" in lib.pip_last_error(None)


@pytest.fixture
def fake_ctx():
    # Never dereferenced by a call whose arguments fail the host checks.
    buf = ctypes.create_string_buffer(4096)
    return ctypes.addressof(buf), buf


@pytest.mark.parametrize("fn", ["pip_voronoi", "pip_sign_of_offset", "pip_ray_crossing",
                                "pip_voronoi_fp32_plain", "pip_voronoi_max_margin"])
def test_argument_checks(lib, fake_ctx, fn):
    ctx, _keep = fake_ctx
    f = getattr(lib, fn)
    A = 1 << 20  # an aligned fake address; never dereferenced on these paths
    # V NULL, V misaligned
    assert f(ctx, None, 4, A, 0, 10, A, None, None) == 1
    assert f(ctx, A + 4, 4, A, 0, 10, A, None, None) == 1
    # n < 3 and n > 64
    assert f(ctx, A, 2, A, 0, 10, A, None, None) == 1
    assert f(ctx, A, 65, A, 0, 10, A, None, None) == 6
    # bad dtype, negative m, NULL / misaligned points
    assert f(ctx, A, 4, A, 7, 10, A, None, None) == 1
    assert f(ctx, A, 4, A, 0, -1, A, None, None) == 1
    assert f(ctx, A, 4, None, 0, 10, A, None, None) == 1
    assert f(ctx, A, 4, A + 4, 0, 10, A, None, None) == 1
    assert f(ctx, A, 4, A + 8, 1, 10, A, None, None) == 1   # float64 needs 16 bytes
    # NULL / misaligned output, misaligned status
    assert f(ctx, A, 4, A, 0, 10, None, None, None) == 1
    assert f(ctx, A, 4, A, 0, 10, A + 2, None, None) == 1
    assert f(ctx, A, 4, A, 0, 10, A, A + 2, None) == 1
    # m == 0 with no status: nothing to do
    assert f(ctx, A, 4, None, 0, 0, None, None, None) == 0
    assert len(lib.pip_last_error(None)) > 0


def test_generators_argument_checks(lib, fake_ctx):
    ctx, _keep = fake_ctx
    A = 1 << 20
    assert lib.polygon_to_generators(ctx, A, 4, None, None, None) == 1
    assert lib.polygon_to_generators(ctx, A, 4, A + 4, None, None) == 1
    assert lib.polygon_to_generators(ctx, A, 1, A, None, None) == 1
    assert lib.polygon_to_generators(None, A, 4, A, None, None) == 1


def test_library_has_no_cpu_fallback_symbols(lib):
    # the product library must not contain the oracle
    for name in ("oracle_voronoi", "oracle_generators", "oracle_cost"):
        assert not hasattr(lib, name)


def test_plan_create_rejects_null_arguments(lib):
    """pip_plan_create checks its pointers before it touches a context."""
    import ctypes
    h = ctypes.c_void_p()
    desc = ctypes.create_string_buffer(128)
    assert lib.pip_plan_create(None, 0, desc, ctypes.byref(h)) == 1
