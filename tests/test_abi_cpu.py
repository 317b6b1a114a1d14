"""The C-ABI library without a GPU: it loads, exports every symbol declared in
include/lb.h, and rejects bad configurations before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lb.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1505_02037_amd import build, lb

    if not os.path.exists(lb.LIB_PATH):
        build.build()
    return lb.load_library()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("lb_create", "lb_init_fields", "lb_step", "lb_moments", "lb_destroy"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header(lib):
    from paper_1505_02037_amd import lb

    assert set(lb.EXPORTS) == set(_declared())


def test_bad_configs_are_rejected_without_a_device(lib):
    from paper_1505_02037_amd import lb

    bad = [
        lb.make_config(8, 8, 8, 0.5),          # tau must exceed 1/2
        lb.make_config(8, 8, 8, float("nan")),
        lb.make_config(0, 8, 8, 0.6),          # empty extent
        lb.make_config(8, -1, 8, 0.6),
        lb.make_config(8, 8, 8, 0.6, slicing=7),
        lb.make_config(8, 8, 8, 0.6, precision=9),
        lb.make_config(2048, 2048, 2048, 0.6),  # more than 2^32 sites
    ]
    for cfg in bad:
        h = ctypes.c_void_p(1234)
        rc = lib.lb_create(ctypes.byref(cfg), ctypes.byref(h))
        assert rc == lb.LB_EINVAL
        assert not h.value
        assert lib.lb_device_bytes(ctypes.byref(cfg)) == 0
    cfg = lb.make_config(8, 8, 8, 0.6)
    cfg.lattice = 9
    assert lib.lb_create(ctypes.byref(cfg), None) == lb.LB_EINVAL


def test_null_handle_calls_fail_cleanly(lib):
    from paper_1505_02037_amd import lb

    assert lib.lb_step(None, 1) == lb.LB_EINVAL
    assert lib.lb_moments(None, None, 0) == lb.LB_EINVAL
    assert lib.lb_init_fields(None, None, 0) == lb.LB_EINVAL
    assert lib.lb_steps_done(None) == -1
    lib.lb_destroy(None)
    assert lib.lb_strerror(lb.LB_EINVAL) == b"invalid argument"


def test_device_bytes_matches_layout(lib):
    from paper_1505_02037_amd import lb

    n = 100 * 30 * 7
    ps = (n + 63) // 64 * 64
    assert lb.device_bytes(100, 30, 7) == (2 * 16 * 19 + 16 + 7) * ps * 8
