"""Host-side checks of the serving layer (no GPU): the first-fit device
arena against a unit-map model, request packing and footprints, and the
server's argument checks that precede any device call."""
import ctypes as ct
import os
import subprocess

import numpy as np
import pytest

from paper_2003_02547_amd import binding as B
from paper_2003_02547_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("seed", [1, 2])
def test_arena_first_fit_model(tmp_path, seed):
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), os.path.join(HERE, "native", "arena_check.cpp")],
                   check=True)
    res = subprocess.run([str(exe), str(seed)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok")


def test_pack_sizes_and_variant():
    L = B.lib()
    qps = [W.mass_spring_chain4(1), W.mass_spring_chain8(0), W.random_uneven(3)]
    for qp in qps:
        p = B.Packed(qp)
        assert p.nbytes % 64 == 0 and p.footprint % 256 == 0
        dims = B.Dims.of(qp)
        arr = (ct.c_void_p * 1)(dims.h)
        hb, db = ct.c_size_t(), ct.c_size_t()
        assert L.oqp_batch_bytes(arr, 1, ct.byref(B.default_arg()), ct.byref(hb), ct.byref(db)) == B.OK
        # a batch of one holds at least the request footprint plus its descriptors
        assert db.value >= p.footprint
    # footprint grows with the horizon at fixed stage sizes
    a = B.Packed(W.mass_spring(4, 10, 0.5, 1.0, np.zeros(8)))
    b = B.Packed(W.mass_spring(4, 20, 0.5, 1.0, np.zeros(8)))
    assert a.variant == b.variant and b.footprint > a.footprint


def test_pack_errors():
    L = B.lib()
    q = B.Qp(W.mass_spring_chain4(1))
    nb = ct.c_size_t()
    assert L.oqp_pack_bytes(q.h, ct.byref(nb)) == B.OK
    mem = B._aligned(nb.value + 64, 64)
    assert L.oqp_pack(q.h, mem.ctypes.data, nb.value - 64) == B.ENOMEM
    assert L.oqp_pack(q.h, mem.ctypes.data + 8, nb.value) == B.EINVAL
    assert L.oqp_pack(q.h, mem.ctypes.data, nb.value) == B.OK
    fb, v = ct.c_size_t(), ct.c_int()
    assert L.oqp_pack_footprint(mem.ctypes.data, ct.byref(fb), ct.byref(v)) == B.OK
    junk = B._aligned(256, 64)
    assert L.oqp_pack_footprint(junk.ctypes.data, ct.byref(fb), ct.byref(v)) == B.EINVAL
    # stage sizes beyond every compiled variant
    d = B.Dims(2, [300, 300, 300], [2, 2, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0])
    qb = ct.c_void_p()
    qmem = B._aligned(L.oqp_qp_bytes(d.h))
    assert L.oqp_qp_init(d.h, qmem.ctypes.data, qmem.nbytes, ct.byref(qb)) == B.OK
    assert L.oqp_pack_bytes(qb, ct.byref(nb)) == B.EINVAL


def test_server_bytes_and_init_errors():
    L = B.lib()
    c = B.ServerCfg()
    L.oqp_server_cfg_default(ct.byref(c))
    hb, fb = ct.c_size_t(), ct.c_size_t()
    assert L.oqp_server_bytes(ct.byref(c), ct.byref(hb), ct.byref(fb)) == B.OK
    h1 = hb.value
    c.max_requests *= 2
    assert L.oqp_server_bytes(ct.byref(c), ct.byref(hb), ct.byref(fb)) == B.OK
    assert hb.value > h1
    c.max_launch = 0
    assert L.oqp_server_bytes(ct.byref(c), ct.byref(hb), ct.byref(fb)) == B.EINVAL
    L.oqp_server_cfg_default(ct.byref(c))
    assert L.oqp_server_bytes(ct.byref(c), ct.byref(hb), ct.byref(fb)) == B.OK
    host = B._aligned(hb.value, 64)
    dev = ct.c_void_p(1 << 20)  # never dereferenced: every check below fails first
    streams = (ct.c_void_p * 2)(None, None)
    out = ct.c_void_p()
    arg = B.default_arg()
    # too few streams
    assert L.oqp_server_init(ct.byref(c), ct.byref(arg), host.ctypes.data, hb.value, dev, fb.value + (1 << 20),
                             streams, 1, ct.byref(out)) == B.EINVAL
    # host buffer too small
    assert L.oqp_server_init(ct.byref(c), ct.byref(arg), host.ctypes.data, 64, dev, fb.value + (1 << 20),
                             streams, 2, ct.byref(out)) == B.ENOMEM
    # no room for an arena
    assert L.oqp_server_init(ct.byref(c), ct.byref(arg), host.ctypes.data, hb.value, dev, fb.value,
                             streams, 2, ct.byref(out)) == B.ENOMEM
    # pageable host memory is refused
    assert L.oqp_server_init(ct.byref(c), ct.byref(arg), host.ctypes.data, hb.value, dev, fb.value + (1 << 20),
                             streams, 2, ct.byref(out)) == B.EINVAL
    assert b"page-locked" in L.oqp_last_error()
