"""CPU checks of the C ABI: the library loads, exports every declared symbol, and rejects bad arguments
before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2010_14258_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", "", txt)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", txt, re.M):
            names.add(m.group(1))
    return sorted(names)


def test_library_loads_and_exports_every_declared_symbol():
    lib = N.load()
    declared = _declared_functions()
    assert "ldbp_forward" in declared
    for name in declared:
        assert hasattr(lib, name), name
    # every declared function has a Python signature and vice versa
    assert set(declared) == set(N.SIGNATURES), set(declared) ^ set(N.SIGNATURES)


def test_status_strings():
    lib = N.load()
    assert lib.ldbp_status_string(0) == b"ok"
    assert lib.ldbp_status_string(-2) == b"workspace too small"
    assert lib.ldbp_version().startswith(b"ldbp-gfx950")


def _ws(dtype=0, npol=1, nwave=2, n=100, ntap=(15, 3), ckpt=None, every=0, plan=None):
    lib = N.load()
    out = ctypes.c_size_t(123)
    nt = N.i32_array(ntap)
    st = lib.ldbp_forward_workspace_size(dtype, npol, nwave, n, len(ntap), nt, ckpt, every,
                                         ctypes.byref(plan) if plan else None, ctypes.byref(out))
    return st, out.value


def test_workspace_size_and_validation():
    st, b = _ws(ntap=[15] * 3)
    assert st == 0 and b == 0                          # one pass, no workspace
    st, b = _ws(ntap=[15] * 50, nwave=4, n=1000)
    assert st == 0 and b == 4 * 1000 * 8               # several passes ping-pong through one buffer
    st, b = _ws(ntap=[15] * 50, nwave=4, n=1000, ckpt=ctypes.c_void_p(16), every=5)
    assert st == 0 and b == 0                          # checkpoints serve as pass buffers
    assert _ws(ntap=[4])[0] == N.LDBP_EINVAL          # even length
    assert _ws(ntap=[65])[0] == N.LDBP_EINVAL         # too long
    assert _ws(npol=3)[0] == N.LDBP_EUNSUPPORTED
    assert _ws(dtype=7)[0] == N.LDBP_EINVAL
    assert _ws(n=0)[0] == N.LDBP_EINVAL
    assert _ws(nwave=0)[0] == N.LDBP_EINVAL
    assert _ws(plan=N.LdbpPlan(65, 1, 0, 0))[0] == N.LDBP_EINVAL
    assert _ws(plan=N.LdbpPlan(3, 1000, 0, 0))[0] == N.LDBP_EINVAL
    assert b"odd" in N.load().ldbp_last_error() or True


def _fwd(**kw):
    lib = N.load()
    a = dict(dtype=0, npol=1, nwave=2, n=64, ntap=(5, 3), taps=16, c=16, x=4096, y=8192, ckpt=0, every=0,
             ws=0, wsb=0)
    a.update(kw)
    nt = N.i32_array(a["ntap"])
    return lib.ldbp_forward(a["dtype"], a["npol"], a["nwave"], a["n"], len(a["ntap"]), nt, a["taps"], a["c"],
                            a["x"], a["y"], a["ckpt"], a["every"], None, a["ws"], a["wsb"], None)


def test_forward_rejects_bad_arguments_before_any_gpu_work():
    # Fake (never dereferenced) addresses: every case fails validation on the host.
    assert _fwd(x=0) == N.LDBP_EINVAL
    assert _fwd(x=4100) == N.LDBP_EINVAL                 # misaligned
    assert _fwd(y=4096 + 512) == N.LDBP_EINVAL           # overlaps x (2*64*8 = 1024 bytes)
    assert _fwd(ntap=(5, 2)) == N.LDBP_EINVAL
    assert _fwd(ntap=[5] * 100, n=100000, x=1 << 30, y=1 << 31) == N.LDBP_EWORKSPACE   # multi-pass needs ws
    assert _fwd(ckpt=1 << 20, every=0) == N.LDBP_EINVAL
    assert _fwd(ckpt=4096 + 512, every=1, y=1 << 24) == N.LDBP_EINVAL  # ckpt overlaps x


def _bwd(flags=0, x=1 << 20, gy=1 << 24, gx=None, ws=None, ws_bytes=0, ntap=(15, 3), n=64, nwave=2):
    lib = N.load()
    pl = N.LdbpPlan(0, 0, 0, flags)
    nt = N.i32_array(ntap)
    return lib.ldbp_backward(0, 1, nwave, n, len(ntap), nt, 1 << 12, 1 << 13, x, None, 0, gy, gx, 1 << 14, 1 << 15,
                             ctypes.byref(pl), ws, ws_bytes, None)


def test_backward_rejects_bad_arguments_before_any_gpu_work():
    # Fake (never dereferenced) addresses: every case fails validation on the host.
    assert _bwd(flags=4) == N.LDBP_EINVAL                               # undefined plan flag
    assert _bwd(flags=N.LDBP_PLAN_SYMMETRIC) == N.LDBP_EWORKSPACE       # valid flag, missing workspace
    assert _bwd(ntap=(15, 4)) == N.LDBP_EINVAL                          # even length
    assert _bwd(x=(1 << 20) + 8) == N.LDBP_EINVAL                       # misaligned
    assert _bwd(gx=(1 << 24) + 512, ws=1 << 28, ws_bytes=1 << 30) == N.LDBP_EINVAL   # gx overlaps gy


def test_batch_plan_rejects_bad_tables_before_any_gpu_work():
    lib = N.load()
    h = ctypes.c_void_p(0)
    lens = (ctypes.c_int64 * 2)(100, 200)
    ns = N.i32_array([2, 1])
    assert lib.ldbp_batch_plan_create(0, 1, 2, lens, ns, N.i32_array([3, 4, 5]), None, ctypes.byref(h)) == N.LDBP_EINVAL
    assert lib.ldbp_batch_plan_create(0, 1, 0, lens, ns, N.i32_array([3, 5, 5]), None, ctypes.byref(h)) == N.LDBP_EINVAL
    assert lib.ldbp_batch_plan_create(0, 3, 2, lens, ns, N.i32_array([3, 5, 5]), None, ctypes.byref(h)) == N.LDBP_EUNSUPPORTED
    bad = (ctypes.c_int64 * 2)(100, 0)
    assert lib.ldbp_batch_plan_create(0, 1, 2, bad, ns, N.i32_array([3, 5, 5]), None, ctypes.byref(h)) == N.LDBP_EINVAL
    assert h.value in (None, 0)
    # total halo larger than any LDS work size: planned as several passes (the tables are valid; without
    # a GPU the device allocation fails)
    st = lib.ldbp_batch_plan_create(0, 1, 1, lens, N.i32_array([200]), N.i32_array([63] * 200), None, ctypes.byref(h))
    assert st in (N.LDBP_OK, N.LDBP_EHIP)
    if st == N.LDBP_OK:
        lib.ldbp_batch_plan_destroy(h)
    assert lib.ldbp_batch_forward(None, 16, 16, 16, 32, None) == N.LDBP_EINVAL


def test_default_plan_chunks_and_even_passes():
    from paper_2010_14258_amd import ldbp as L
    # complex64, two polarisations, 3 outputs per thread: 2 chunks of 768 samples (three workgroups of
    # 48 KiB fit a compute unit's 160 KiB of LDS, three of 72 KiB do not); 64 steps of 5 taps in 2
    # passes of 32 (halo 64): tile 1536 - 128
    assert L.ldbp_forward_plan_query(0, 2, 8, 1 << 20, [5] * 64) == (2, 1408, 32)
    # one chunk asked for: 3 passes (the halo rule allows 24 steps), spread 22, 21, 21
    assert L.ldbp_forward_plan_query(0, 2, 8, 1 << 20, [5] * 64, plan=(0, 1, 3, 1)) == (3, 680, 22)
    # complex64, one polarisation, 7 outputs per thread: 1 chunk (three of 56 KiB exceed 160 KiB);
    # 50 steps of 15 taps, at most 16 per pass by the halo rule, spread 13, 13, 12, 12: tile 1792 - 182
    assert L.ldbp_forward_plan_query(0, 1, 64, 65536, [15] * 50) == (4, 1610, 13)
    # complex128, two polarisations, 1 output per thread: 3 chunks of 256 samples
    assert L.ldbp_forward_plan_query(1, 2, 8, 1 << 20, [5] * 64) == (3, 680, 22)


def test_checkpointed_forward_groups_whole_blocks():
    from paper_2010_14258_amd import ldbp as L
    # 50 steps of 15 taps, checkpoints every 2 steps: passes of whole blocks (halo rule: at most 8
    # blocks), not 25 passes; the 25 blocks spread evenly over the 4 passes (7, 7, 7, 4)
    npass, _, maxs = L.ldbp_forward_plan_query(0, 1, 64, 65536, [15] * 50, ckpt_every=2)
    assert npass == 4 and maxs == 14
    # steps_per_pass is rounded down to whole blocks
    npass, _, maxs = L.ldbp_forward_plan_query(0, 1, 64, 65536, [15] * 50, ckpt_every=2, plan=(7, 0))
    assert maxs == 6 and npass == 9
    # a pass never splits a block, whatever the plan asks for
    npass, _, maxs = L.ldbp_forward_plan_query(0, 1, 64, 65536, [15] * 50, ckpt_every=5, plan=(3, 0))
    assert maxs == 5 and npass == 10


def _aws(n=1000, ntap=(15, 15), nl=None, edge=1, nwave=2, plan=None):
    lib = N.load()
    out = ctypes.c_size_t(123)
    st = lib.ldbp_forward_aperiodic_workspace_size(0, 1, nwave, n, len(ntap), N.i32_array(ntap),
                                                   N.i32_array(nl) if nl else None, edge,
                                                   ctypes.byref(plan) if plan else None, ctypes.byref(out))
    return st, out.value


def test_aperiodic_workspace_and_validation():
    # one pass: no workspace; zero edge works on n + 2P samples, valid edge on n
    st, b = _aws(ntap=[15] * 3)
    assert st == 0 and b == 0
    P = 7 * 50
    st, b = _aws(ntap=[15] * 50, n=1000, nwave=4, edge=N.LDBP_EDGE_ZERO)
    buf = (4 * (1000 + 2 * P) * 8 + 255) // 256 * 256
    assert st == 0 and b == 2 * buf                   # several passes: two intermediate buffers
    st, b = _aws(ntap=[15] * 50, n=1000, nwave=4, edge=N.LDBP_EDGE_VALID, plan=N.LdbpPlan(25, 0, 0, 0))
    assert st == 0 and b == (4 * 1000 * 8 + 255) // 256 * 256   # two passes: one buffer
    assert _aws(ntap=[15] * 50, n=2 * P, edge=N.LDBP_EDGE_VALID)[0] == N.LDBP_EINVAL   # no valid output
    assert _aws(ntap=[15, 15], n=1000, nl=[41, 3], edge=N.LDBP_EDGE_VALID)[0] == 0
    assert _aws(ntap=[15, 15], n=2 * (14 + 21), nl=[41, 3], edge=N.LDBP_EDGE_VALID)[0] == N.LDBP_EINVAL
    assert _aws(edge=3)[0] == N.LDBP_EINVAL
    # the call itself rejects the same before any GPU work
    lib = N.load()
    st = lib.ldbp_forward_aperiodic(0, 1, 1, 8, 2, N.i32_array([5, 5]), None, ctypes.c_void_p(16),
                                    ctypes.c_void_p(16), None, ctypes.c_void_p(1024), ctypes.c_void_p(4096),
                                    N.LDBP_EDGE_VALID, None, None, 0, None)
    assert st == N.LDBP_EINVAL


def test_tx_shape_symbols_validation():
    lib = N.load()
    args = (0, 1, 2, 64, 2, 10.7e9, 0.1)
    assert lib.tx_shape_symbols(*args, None, ctypes.c_void_p(16), ctypes.c_void_p(4096), None, 0,
                                None) == N.LDBP_EINVAL                       # no symbols
    assert lib.tx_shape_symbols(0, 1, 2, 64, 7, 10.7e9, 0.1, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                ctypes.c_void_p(4096), None, 0, None) == N.LDBP_EUNSUPPORTED   # rho 7
    assert lib.tx_shape_symbols(0, 1, 2, 64, 3, 10.7e9, 0.1, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                ctypes.c_void_p(4096), None, 0, None) == N.LDBP_EWORKSPACE     # rho 3 is valid
    assert lib.tx_shape_symbols(*args, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(4096), None, 0,
                                None) == N.LDBP_EWORKSPACE


def test_guard_workspace_and_status():
    """LDBP_PLAN_GUARD adds 256 bytes for the non-finite flag (after the 256-aligned intermediate buffer of a
    multi-pass forward, or alone); LDBP_ENONFINITE has its status text; the aperiodic forward rejects it."""
    lib = N.load()
    g = N.LdbpPlan(0, 0, 0, N.LDBP_PLAN_GUARD)
    st, b = _ws(ntap=[15] * 3, plan=g)
    assert st == 0 and b == 256
    st, b = _ws(ntap=[15] * 50, nwave=4, n=1001, plan=g)
    assert st == 0 and b == ((4 * 1001 * 8 + 255) // 256) * 256 + 256
    st, b = _ws(ntap=[15] * 50, nwave=4, n=1000, ckpt=ctypes.c_void_p(16), every=5, plan=g)
    assert st == 0 and b == 256
    assert lib.ldbp_status_string(N.LDBP_ENONFINITE) == b"non-finite output"
    out = ctypes.c_size_t(0)
    st = lib.ldbp_forward_aperiodic_workspace_size(0, 1, 1, 1000, 2, N.i32_array([3, 3]), None, N.LDBP_EDGE_ZERO,
                                                   ctypes.byref(g), ctypes.byref(out))
    assert st == 0   # sizing ignores flags; the call itself rejects unknown bits
    bad = N.LdbpPlan(0, 0, 0, N.LDBP_PLAN_GUARD)
    st = lib.ldbp_forward_aperiodic(0, 1, 1, 1000, 2, N.i32_array([3, 3]), None, ctypes.c_void_p(256),
                                    ctypes.c_void_p(512), None, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21),
                                    N.LDBP_EDGE_ZERO, ctypes.byref(bad), None, 0, None)
    assert st == N.LDBP_EINVAL


def test_guarded_forward_checks_workspace_before_any_launch():
    """A guarded forward without room for its flag fails with LDBP_EWORKSPACE before any GPU work."""
    lib = N.load()
    g = N.LdbpPlan(0, 0, 0, N.LDBP_PLAN_GUARD)
    st = lib.ldbp_forward(0, 1, 2, 100, 2, N.i32_array([3, 3]), ctypes.c_void_p(256), ctypes.c_void_p(512),
                          ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21), None, 0, ctypes.byref(g), None, 0, None)
    assert st == N.LDBP_EWORKSPACE
    st = lib.ldbp_forward(0, 1, 2, 100, 2, N.i32_array([3, 3]), ctypes.c_void_p(256), ctypes.c_void_p(512),
                          ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21), None, 0, ctypes.byref(g),
                          ctypes.c_void_p(1 << 22), 128, None)
    assert st == N.LDBP_EWORKSPACE


def test_noalloc_forward_rejects_batches_beyond_its_scratch_before_any_gpu_work():
    """The forward without allocation checks its scratch need on the host: a multi-pass forward whose
    intermediate signal exceeds LDBP_NOALLOC_SCRATCH_BYTES returns LDBP_EWORKSPACE (no GPU here, so a
    HIP call would have failed with LDBP_EHIP instead)."""
    lib = N.load()
    ntap = N.i32_array([15] * 50)
    n = N.LDBP_NOALLOC_SCRATCH_BYTES // 8 // 4 + 1            # 4 waveforms: one sample more than fits
    st = lib.ldbp_forward_noalloc(0, 1, 4, n, 50, ntap, 16, 16, 4096, 8192, None, 0, None, None)
    assert st == N.LDBP_EWORKSPACE
    assert b"LDBP_NOALLOC_SCRATCH_BYTES" in lib.ldbp_last_error()
    # argument errors come first, as for ldbp_forward
    assert lib.ldbp_forward_noalloc(0, 1, 4, 64, 1, N.i32_array([4]), 16, 16, 4096, 8192, None, 0, None,
                                    None) == N.LDBP_EINVAL
    assert lib.ldbp_forward_noalloc(0, 3, 4, 64, 1, N.i32_array([5]), 16, 16, 4096, 8192, None, 0, None,
                                    None) == N.LDBP_EUNSUPPORTED


def test_ssm_batch_plan_validation_before_any_gpu_work():
    lib = N.load()
    link = N.SsmLink(21.4e9, 4.6e-5, -2.17e-26, 1.3e-3, 1e5, 1.0, 0.0, 1, 2, None, 1, 0)
    out = ctypes.c_void_p(0)

    def create(lens, spans, dbp=1, dtype=0, npol=1):
        return lib.ssm_batch_plan_create(dtype, npol, len(lens), (ctypes.c_int64 * len(lens))(*lens),
                                         N.i32_array(spans), ctypes.byref(link), dbp, ctypes.byref(out))

    assert create([4096, 4097], [1, 1]) == N.LDBP_EUNSUPPORTED      # 4097 = 17 x 241
    assert create([4096, 7 * 1024], [1, 1]) == N.LDBP_EUNSUPPORTED  # factor 7
    assert create([4096], [0]) == N.LDBP_EINVAL                     # no span
    assert create([4096], [1], dbp=2) == N.LDBP_EINVAL
    assert create([4096], [1], npol=3) == N.LDBP_EUNSUPPORTED
    assert create([1 << 25], [1]) == N.LDBP_EUNSUPPORTED            # beyond 2^24
    assert out.value is None
    # lengths 2^a 3^b 5^c pass validation; without a GPU the plan's allocation then fails
    assert create([4500, 6000], [2, 3]) == N.LDBP_EHIP


def test_ssm_accepts_5_smooth_lengths_and_rejects_others():
    lib = N.load()
    link = N.SsmLink(21.4e9, 4.6e-5, -2.17e-26, 1.3e-3, 1e5, 1.0, 0.0, 2, 2, None, 1, 0)
    b = ctypes.c_size_t(0)
    for n in (3000, 4050, 6000, 162000, 259200):
        assert lib.ssm_workspace_size(0, 1, 2, n, ctypes.byref(link), ctypes.byref(b)) == N.LDBP_OK, n
        assert b.value > 0
    for n in (4097, 7000, 3 * 11 * 256):
        assert lib.ssm_workspace_size(0, 1, 2, n, ctypes.byref(link), ctypes.byref(b)) == N.LDBP_EUNSUPPORTED, n
