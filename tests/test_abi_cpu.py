"""The C-ABI library without a GPU: it loads, exports every symbol declared in
include/lb.h, and rejects bad configurations before touching a device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("lb.h", "lb_serve.h")]
PROBE_HEADER = os.path.join(ROOT, "include", "hbm_probe.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1505_02037_amd import build, lb

    if not os.path.exists(lb.LIB_PATH):
        build.build()
    return lb.load_library()


def _declared(headers=None, prefix="lb_"):
    names = set()
    for h in headers or HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(%s[a-z_0-9]+)\s*\(" % prefix, text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("lb_create", "lb_init_fields", "lb_step", "lb_moments", "lb_destroy"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header(lib):
    from paper_1505_02037_amd import lb, serve

    assert set(lb.EXPORTS) | set(serve.EXPORTS) == set(_declared())


def test_probe_library_exports_its_header():
    import ctypes as C

    from paper_1505_02037_amd import build

    if not os.path.exists(build.PROBE_LIB):
        build.build()
    probe = C.CDLL(build.PROBE_LIB)
    names = _declared([PROBE_HEADER], prefix="hbm_")
    assert names == ["hbm_copy_probe", "hbm_read_probe", "hbm_reread_probe"]
    assert all(hasattr(probe, n) for n in names)
    ms = C.c_double()
    assert probe.hbm_copy_probe(C.c_size_t(100), 1, C.byref(ms)) == -1  # not a multiple of 64


def test_server_rejects_bad_configs(lib):
    import ctypes as C

    from paper_1505_02037_amd import serve

    serve._lib()
    for budget, prec, slots, k in [(0, 0, 4, 8), (1 << 30, 5, 4, 8), (1 << 30, 0, 0, 8), (1 << 30, 0, 4, 0)]:
        cfg = serve.ServerConfig(budget, prec, slots, k, -1, None)
        h = C.c_void_p()
        assert lib.lb_server_create(C.byref(cfg), C.byref(h)) == -1
        assert not h.value
    assert lib.lb_server_advance(None, None) == -1
    lib.lb_server_destroy(None)


def test_bad_configs_are_rejected_without_a_device(lib):
    from paper_1505_02037_amd import lb

    bad = [
        lb.make_config(8, 8, 8, 0.5),          # tau must exceed 1/2
        lb.make_config(8, 8, 8, float("nan")),
        lb.make_config(0, 8, 8, 0.6),          # empty extent
        lb.make_config(8, -1, 8, 0.6),
        lb.make_config(8, 8, 8, 0.6, slicing=3),
        lb.make_config(8, 8, 8, 0.6, precision=9),
        lb.make_config(2048, 2048, 2048, 0.6),  # more than 2^32 sites
        lb.make_config(8, 8, 8, 0.6, path=3),
        lb.make_config(8, 8, 8, 0.6, lattice=7),                      # unknown lattice
        lb.make_config(8, 8, 2, 0.6, lattice=lb.D2Q9),                # D2Q9 is one site thick
        lb.make_config(8, 8, 1, 0.6, lattice=lb.D2Q9, path=lb.PATH_FUSED),  # split path only
        lb.make_config(8, 8, 8, 0.6, collision=2),                    # unknown collision
        lb.make_config(8, 8, 8, 0.6, collision=lb.COLLISION_REGULARIZED, path=lb.PATH_FUSED),
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
    assert lib.lb_set_matter(None, 0, None, 0, 0) == lb.LB_EINVAL
    lib.lb_destroy(None)
    assert lib.lb_strerror(lb.LB_EINVAL) == b"invalid argument"


def test_device_bytes_matches_layout(lib):
    from paper_1505_02037_amd import lb

    n = 100 * 30 * 7
    ps = (n + 63) // 64 * 64 + 320  # planes padded by 320 elements
    assert lb.device_bytes(100, 30, 7) == (2 * 16 * 19 + 16 + 7) * ps * 8
    assert lb.device_bytes(100, 30, 7, precision=lb.FP32_DEV) == (16 * 19 + 16 + 7) * ps * 8
    assert lb.device_bytes(100, 30, 7, path=lb.PATH_FUSED) == (2 * 16 * 19 + 16 + 16 + 7) * ps * 8
    n2 = 100 * 30
    ps2 = (n2 + 63) // 64 * 64 + 320
    assert lb.device_bytes(100, 30, 1, lattice=lb.D2Q9) == (2 * 16 * 9 + 16 + 7) * ps2 * 8
    assert lb.device_bytes(100, 30, 1, precision=lb.FP32_DEV, lattice=lb.D2Q9) == (16 * 9 + 16 + 7) * ps2 * 8


def test_build_entry_reaches_both_build_steps(monkeypatch):
    """__graft_entry__.build() calls the HIP build and the oracle build (the
    compilers are replaced by recorders here; the real build runs outside
    the test suite)."""
    import importlib

    import __graft_entry__

    calls = []
    hip_build = importlib.import_module("paper_1505_02037_amd.build")
    oracle_build = importlib.import_module("oracle.build")
    monkeypatch.setattr(hip_build, "build", lambda verbose=False: calls.append("hip"))
    monkeypatch.setattr(oracle_build, "build", lambda verbose=False: calls.append("oracle"))
    __graft_entry__.build()
    assert calls == ["hip", "oracle"]


def test_config_layout_matches_header(tmp_path):
    """The binding's lb_config has the header's size and field offsets (a C
    program built with gcc against include/lb.h prints them)."""
    import subprocess

    from paper_1505_02037_amd import lb

    names = [f for f, _ in lb.LBConfig._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"lb.h\"\nint main(void) {\n"
                   + "".join(f'  printf("%zu\\n", offsetof(lb_config, {n}));\n' for n in names)
                   + '  printf("%zu\\n", sizeof(lb_config));\n  return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert out[:-1] == [getattr(lb.LBConfig, n).offset for n in names]
    assert out[-1] == ctypes.sizeof(lb.LBConfig)


def test_allocator_hooks_must_come_in_pairs(lib):
    from paper_1505_02037_amd import lb

    class Never(lb.DeviceAllocator):
        def alloc(self, nbytes):
            return None

        def free(self, ptr):
            pass

    hooks = Never().hooks()
    cfg = lb.make_config(10, 10, 10, 0.8, hooks=hooks)
    assert lib.lb_device_bytes(ctypes.byref(cfg)) > 0
    cfg.dev_free = lb.DEV_FREE_FN()  # NULL
    assert lib.lb_device_bytes(ctypes.byref(cfg)) == 0
    cfg = lb.make_config(10, 10, 10, 0.8)
    cfg.dev_free = hooks[1]
    assert lib.lb_device_bytes(ctypes.byref(cfg)) == 0

