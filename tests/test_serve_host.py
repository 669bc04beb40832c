"""CPU checks of the request server: the arena allocator and admission policy (hrlb_sched.h, through
a small C++ check program), and request validation at submit time (host-only calls; the arena
pointer is never dereferenced before a scheduling round, so no device is needed)."""
import ctypes as C
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_and_admission_policy(tmp_path):
    exe = tmp_path / "sched_check"
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "paper_1810_07803_amd", "csrc"),
                    os.path.join(ROOT, "tests", "sched_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr


def _server(arena_bytes, precision=1, check_every=100):
    from paper_1810_07803_amd import hrlb

    lib = hrlb.load()
    cfg = hrlb.ServerConfig(4, check_every, 2, precision)
    h = C.c_void_p()
    fake_arena = C.c_void_p(1 << 20)  # aligned, never touched by submit
    hrlb._check(lib.hrlb_server_create(C.byref(cfg), fake_arena, arena_bytes, None, C.byref(h)))
    return lib, h


def _req(hrlb, **kw):
    p = hrlb.make_params(delta=1.0, uw=0.1, ncell=kw.pop("ncell", 64), precision=kw.pop("precision", 1))
    r = hrlb.SolveRequest(kw.pop("Qx", 4), 3, kw.pop("Qy", 4), 3, p, kw.pop("tol", 1e-6), 1,
                          kw.pop("max_steps", 1000), -1.0)
    assert not kw
    return r


def test_submit_validates_requests():
    from paper_1810_07803_amd import hrlb

    lib, h = _server(64 << 20)
    rid = C.c_long()
    assert lib.hrlb_server_submit(h, C.byref(_req(hrlb)), C.byref(rid)) == hrlb.HRLB_OK
    assert rid.value == 1
    info = hrlb.RequestInfo()
    assert lib.hrlb_server_request(h, rid.value, C.byref(info), None, None, 1) == hrlb.HRLB_OK
    assert info.state == hrlb.HRLB_REQ_WAITING and info.t_admit == -1.0 and info.bytes > 0
    # a waiting request is not released
    assert lib.hrlb_server_request(h, rid.value, C.byref(info), None, None, 0) == hrlb.HRLB_OK
    bad = [
        (_req(hrlb, precision=0), hrlb.HRLB_E_INVALID),          # precision differs from the server's
        (_req(hrlb, max_steps=150), hrlb.HRLB_E_INVALID),        # not a multiple of check_every
        (_req(hrlb, max_steps=0), hrlb.HRLB_E_INVALID),
        (_req(hrlb, tol=0.0), hrlb.HRLB_E_INVALID),
        (_req(hrlb, ncell=30), hrlb.HRLB_E_INVALID),             # not a multiple of 4
        (_req(hrlb, Qx=2), hrlb.HRLB_E_INVALID),                 # velocity set
        (_req(hrlb, Qx=32, Qy=12, ncell=4096), hrlb.HRLB_E_NOMEM),  # never fits the arena
    ]
    for r, want in bad:
        assert lib.hrlb_server_submit(h, C.byref(r), C.byref(rid)) == want
        assert len(lib.hrlb_last_error()) > 0
    assert lib.hrlb_server_request(h, 99, C.byref(info), None, None, 0) == hrlb.HRLB_E_INVALID
    lib.hrlb_server_free(h)


def test_server_config_is_validated():
    from paper_1810_07803_amd import hrlb

    lib = hrlb.load()
    h = C.c_void_p()
    for cfg, arena in ((hrlb.ServerConfig(0, 100, 0, 1), 1 << 20), (hrlb.ServerConfig(4, 0, 0, 1), 1 << 20),
                       (hrlb.ServerConfig(4, 100, -1, 1), 1 << 20), (hrlb.ServerConfig(4, 100, 0, 7), 1 << 20)):
        assert lib.hrlb_server_create(C.byref(cfg), C.c_void_p(1 << 20), arena, None, C.byref(h)) == hrlb.HRLB_E_INVALID
    cfg = hrlb.ServerConfig(4, 100, 0, 1)
    assert lib.hrlb_server_create(C.byref(cfg), C.c_void_p(1000), 1 << 20, None, C.byref(h)) == hrlb.HRLB_E_INVALID


@pytest.mark.parametrize("n", [1, 5])
def test_server_clock_is_monotonic(n):
    from paper_1810_07803_amd import hrlb

    lib, h = _server(1 << 20)
    t = [lib.hrlb_server_clock(h) for _ in range(n + 1)]
    assert all(b >= a for a, b in zip(t, t[1:])) and t[0] >= 0.0
    lib.hrlb_server_free(h)
