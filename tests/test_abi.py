"""The C-ABI library loads on a machine without a GPU, exports every symbol
include/pic.h declares, its ctypes mirror matches the C layout, and the
allocation-free calls (pic_query, pic_strerror) validate configurations."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


def _lib():
    from paper_2501_14795_amd import _lib
    if not os.path.exists(_lib.SO_PATH):
        pytest.skip("libpic.so not built")
    return _lib


def test_exports_every_declared_symbol():
    L = _lib()
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char \*|pic_sim \*)\s*(pic_\w+)\s*\(", text, re.M))
    assert declared == set(L.EXPORTS)
    lib = L.load()
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.SO_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (pic_\w+)$", out, re.M))
    assert declared <= exported


def test_struct_layout_matches_header(tmp_path):
    L = _lib()
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "pic.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(pic_config), sizeof(pic_buffers), sizeof(pic_sizes),
         sizeof(pic_diag_out), sizeof(pic_timing_out), sizeof(pic_species), sizeof(pic_particles));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(pic_config, species), offsetof(pic_config, tile),
         offsetof(pic_buffers, sp), offsetof(pic_diag_out, leavers), offsetof(pic_sizes, work_bytes));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(src), "-o", str(exe)])
    got = subprocess.check_output([str(exe)], text=True).split()
    c = ctypes
    want = [c.sizeof(L.pic_config), c.sizeof(L.pic_buffers), c.sizeof(L.pic_sizes),
            c.sizeof(L.pic_diag_out), c.sizeof(L.pic_timing_out), c.sizeof(L.pic_species),
            c.sizeof(L.pic_particles),
            L.pic_config.species.offset, L.pic_config.tile.offset, L.pic_buffers.sp.offset,
            L.pic_diag_out.leavers.offset, L.pic_sizes.work_bytes.offset]
    assert [int(v) for v in got] == want


def _cfg(L, nx=64, ny=64, dx=0.1, dy=0.1, dt=0.07, tile=16, n=1000, ns=1, reps=0, flags=0, filt=0, every=0,
         ppl=0):
    c = L.pic_config()
    c.nx, c.ny, c.dx, c.dy, c.dt, c.tile, c.j_replicas, c.n_species, c.flags = nx, ny, dx, dy, dt, tile, reps, ns, flags
    c.j_filter = filt
    c.sort_every = every
    c.ppl = ppl
    for k in range(ns):
        c.species[k].qm = -1.0
        c.species[k].q = -1.0 / 16
        c.species[k].n = n
    return c


def test_query_sizes_and_validation():
    L = _lib()
    s = L.pic_query(_cfg(L))
    assert s.n_tiles == 16 and s.field_bytes == 9 * 64 * 64 * 4 and s.work_bytes > 0
    big = L.pic_query(_cfg(L, nx=2048, ny=2048, n=2048 * 2048 * 16))
    assert big.n_tiles == 128 * 128
    # workspace grows linearly with particles (the 16-bit tile-relative cells 2 B, leaver
    # entries 4 B + 32-B leaver records, holes 4 B, 32-B mover staging records: 74 B/particle)
    s2 = L.pic_query(_cfg(L, n=2000))
    assert 74 * 1000 <= s2.work_bytes - s.work_bytes <= 74 * 1000 + 16 * 256
    cases = [
        (dict(dt=0.0708), L.PIC_ECFL),          # Eq. (1): limit 0.070711 at dx = dy = 0.1
        (dict(dt=0.08), L.PIC_ECFL),
        (dict(tile=12), L.PIC_ETILE),
        (dict(nx=72), L.PIC_ETILE),
        (dict(nx=8, tile=16), L.PIC_EINVAL),
        (dict(nx=32768 + 16), L.PIC_EINVAL),
        (dict(ns=0), L.PIC_EINVAL),
        (dict(ns=5), L.PIC_EINVAL),
        (dict(reps=3), L.PIC_EINVAL),
        (dict(flags=32), L.PIC_EINVAL),
        # the quadratic shape: one sort per step, fixed-point current, one LDS
        # copy, two particles per lane, no moving window
        (dict(flags=16, every=2), L.PIC_EINVAL),
        (dict(flags=16 | 1), L.PIC_EINVAL),
        (dict(flags=16, reps=2), L.PIC_EINVAL),
        (dict(flags=16 | 4), L.PIC_EINVAL),
        (dict(flags=16, ppl=1), L.PIC_EINVAL),
        (dict(flags=3), L.PIC_EINVAL),          # Esirkepov needs the fixed-point current
        (dict(n=-1), L.PIC_EINVAL),
        (dict(n=2 ** 31), L.PIC_EINVAL),
        (dict(filt=-1), L.PIC_EINVAL),
        (dict(filt=L.PIC_MAX_FILTER + 1), L.PIC_EINVAL),
        # sort cadence: 1, 2 or 4; above 1 only with the fixed-point current and
        # one LDS copy, without the moving window, where the halo fits the tile
        (dict(every=3), L.PIC_EINVAL),
        (dict(every=-1), L.PIC_EINVAL),
        (dict(every=2, flags=1), L.PIC_EINVAL),             # PIC_FLAG_J_FLOAT
        (dict(every=2, reps=2), L.PIC_EINVAL),
        (dict(every=2, flags=4), L.PIC_EINVAL),             # PIC_FLAG_MOVING_WINDOW
        (dict(tile=8, every=4), L.PIC_ETILE),               # 2k + 1 > tile
        # particles per lane: 1, 2 or 4; other than 2 with the fixed-point
        # current, the default deposit and one LDS copy
        (dict(ppl=3), L.PIC_EINVAL),
        (dict(ppl=-1), L.PIC_EINVAL),
        (dict(ppl=4, flags=1), L.PIC_EINVAL),
        (dict(ppl=1, flags=2), L.PIC_EINVAL),
        (dict(ppl=4, reps=2), L.PIC_EINVAL),
    ]
    for kw, code in cases:
        ns = kw.pop("ns", 1)
        c = _cfg(L, ns=min(max(ns, 0), 4), **kw)
        if ns == 0 or ns == 5:
            c.n_species = ns
        with pytest.raises(L.PicError) as e:
            L.pic_query(c)
        assert e.value.code == code, (kw, e.value.code)
    assert L.pic_query(_cfg(L, dt=0.0707)).n_tiles == 16
    for ppl in (1, 2, 4):
        assert L.pic_query(_cfg(L, ppl=ppl, every=2)).work_bytes == L.pic_query(_cfg(L, every=2)).work_bytes
    # 32 x 32 tiles take 70 KB of LDS with one current copy (two workgroups per
    # CU); the largest allowed configurations still fit the CU's 160 KB
    assert L.pic_query(_cfg(L, nx=64, tile=32, reps=2, flags=L.PIC_FLAG_J_FLOAT)).n_tiles == 4
    assert L.pic_query(_cfg(L, nx=64, tile=32, reps=4, flags=L.PIC_FLAG_J_FLOAT)).n_tiles == 4
    assert L.pic_query(_cfg(L, nx=64, tile=32, reps=4)).n_tiles == 4     # int64 current x 4: 158 KB
    assert L.pic_query(_cfg(L, nx=64, tile=32, every=4)).n_tiles == 4    # halo pad 4: 91 KB
    assert L.pic_query(_cfg(L, flags=L.PIC_FLAG_ESIRKEPOV)).work_bytes == s.work_bytes
    # the motion-class sort stages in six more arrays (22 B/particle: 16-bit cells); the
    # in-place sort's 32-byte records stay (the moving window's sort is the in-place one)
    m = L.pic_query(_cfg(L, flags=L.PIC_FLAG_MOTION_SORT)).work_bytes
    assert s.work_bytes + 22 * 1000 <= m <= s.work_bytes + 22 * 1000 + 16 * 256
    # capacity: per-particle scratch sized for it; below n is invalid
    c = _cfg(L)
    c.species[0].cap = 2000
    assert L.pic_query(c).work_bytes == s2.work_bytes
    c.species[0].cap = 999
    with pytest.raises(L.PicError):
        L.pic_query(c)
    # the moving window adds only the removal counters and the new particles'
    # tile offsets (17 int32), each rounded up to 256 bytes: no field copy
    sw = L.pic_query(_cfg(L, flags=L.PIC_FLAG_MOVING_WINDOW))
    assert sw.work_bytes - s.work_bytes == 2 * 256
    # a sort cadence k widens every tile's current halo to (T + 2k + 1)^2 nodes
    for every, T in ((2, 16), (4, 16), (2, 8), (2, 32)):
        base = L.pic_query(_cfg(L, tile=T))
        wide = L.pic_query(_cfg(L, tile=T, every=every))
        grow = base.n_tiles * 3 * 4 * ((T + 2 * every + 1) ** 2 - (T + 3) ** 2)
        assert grow <= wide.work_bytes - base.work_bytes <= grow + 256, (every, T)
    assert L.pic_query(_cfg(L, every=1)).work_bytes == s.work_bytes
    # the quadratic shape reaches one node further: the halo pad of a cadence of 2
    for T in (8, 16, 32):
        q = L.pic_query(_cfg(L, tile=T, flags=L.PIC_FLAG_QUADRATIC))
        assert q.work_bytes == L.pic_query(_cfg(L, tile=T, every=2)).work_bytes, T
        assert q.work_bytes == L.pic_query(_cfg(L, tile=T, flags=L.PIC_FLAG_QUADRATIC | 2, every=1)).work_bytes
    # the filter's ping-pong planes: three FP32 current planes + one FP64 density plane
    sf = L.pic_query(_cfg(L, filt=L.PIC_MAX_FILTER))
    assert 20 * 64 * 64 <= sf.work_bytes - s.work_bytes <= 20 * 64 * 64 + 2 * 256
    for code in range(0, -12, -1):
        assert L.strerror(code) != "unknown error"
    assert L.strerror(-99) == "unknown error"


def test_init_rejects_bad_buffers_without_touching_the_device():
    L = _lib()
    c = _cfg(L)
    b = L.pic_buffers()   # all NULL
    with pytest.raises(L.PicError) as e:
        L.pic_init(c, b, 0)
    assert e.value.code == L.PIC_EINVAL


def test_batch_query_validation():
    L = _lib()
    cfgs = [_cfg(L, nx=32, ny=64), _cfg(L, nx=64, ny=32, n=500)]
    nb = L.pic_batch_query(cfgs)
    assert nb > 0
    for bad in ([_cfg(L), _cfg(L, tile=8)], [_cfg(L), _cfg(L, flags=L.PIC_FLAG_J_FLOAT)],
                [_cfg(L), _cfg(L, reps=2)], [_cfg(L), _cfg(L, filt=1)],
                [_cfg(L), _cfg(L, flags=L.PIC_FLAG_ESIRKEPOV)],
                [_cfg(L, flags=L.PIC_FLAG_MOVING_WINDOW)], [_cfg(L), _cfg(L, flags=L.PIC_FLAG_MOTION_SORT)],
                [_cfg(L), _cfg(L, every=2)], [_cfg(L), _cfg(L, ppl=4)]):
        with pytest.raises(L.PicError) as e:
            L.pic_batch_query(bad)
        assert e.value.code == L.PIC_EINVAL
    # the motion-class sort is offered in batched mode
    assert L.pic_batch_query([_cfg(L, flags=L.PIC_FLAG_MOTION_SORT), _cfg(L, nx=32, flags=L.PIC_FLAG_MOTION_SORT)]) > 0
    with pytest.raises(L.PicError):
        L.pic_batch_query([])
    with pytest.raises(L.PicError) as e:
        L.pic_batch_query([_cfg(L), _cfg(L, dt=0.08)])
    assert e.value.code == L.PIC_ECFL
