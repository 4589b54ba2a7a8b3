"""The C ABI without a GPU: exported symbols, host-side planning and argument checks.

Nothing here launches a kernel: every estimation call below is rejected by the host-side
argument checks before anything is enqueued (fake non-null pointers are never dereferenced).
"""
import ctypes
import json
import os
import re

import pytest

import bruteforce as bf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fge.h")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def fge():
    from paper_2006_14970_amd import fge as mod
    mod.load()
    return mod


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fge_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported(fge):
    names = declared_functions()
    assert len(names) >= 10
    lib = fge.load()
    for name in names:
        assert hasattr(lib, name), f"{name} declared in fge.h but not exported"


def test_params_layout_and_defaults(fge):
    p = fge.default_params()
    assert p.size == ctypes.sizeof(fge.Params) == 48
    assert abs(p.omega - 0.1) < 1e-7 and abs(p.eps_r - 5e-3) < 1e-9
    assert (p.small_size, p.iters_small, p.iters_big) == (32, 10, 2)
    assert (p.storage, p.order, p.kernel, p.strip_rows, p.coarse_max_px, p.tile_max_px) == (0,) * 6
    assert fge.load().fge_version() == 9


def test_plan_matches_golden(fge):
    gold = json.load(open(os.path.join(GOLDEN, "level_plans.json")))
    for case in gold["plans"]:
        info = fge.plan(case["H"], case["W"])
        assert [list(x) for x in info.levels] == case["levels"], case


def test_level_size_exact_exhaustive_to_4096(fge):
    for full in range(1, 4097):
        n = bf.num_levels_exact(full, 1)
        assert fge.num_levels(1, full) == n
        for lv in range(1, n + 1):
            assert fge.level_size(full, lv, n) == bf.level_size_exact(full, lv, n)


@pytest.mark.slow
def test_level_size_exact_all_sides(fge):
    """Every side up to 32767 at every level count it can meet (its own and larger ones)."""
    for full in range(4097, 32768, 7):
        for n in range(bf.num_levels_exact(full, 1), 16):
            for lv in range(1, n + 1):
                assert fge.level_size(full, lv, n) == bf.level_size_exact(full, lv, n), (full, lv, n)


def test_bad_sizes(fge):
    lib = fge.load()
    assert lib.fge_num_levels(5, 0) == 0 and lib.fge_num_levels(1, 32768) == 0
    assert lib.fge_level_size(5, 0, 3) == 0 and lib.fge_level_size(5, 4, 3) == 0
    assert fge.workspace_bytes(10, 0) == 0
    with pytest.raises(fge.FgeError):
        fge.plan(10, 40000)


def test_coarse_split(fge):
    info = fge.plan(3072, 4096)
    assert info.n_coarse == 5            # the automatic limit: up to 32x28 (<= 1024 px)
    assert fge.plan(64, 64).n_coarse == 5
    assert fge.plan(3072, 4096, fge.default_params(coarse_max_px=-1)).n_coarse == 0
    assert fge.plan(3072, 4096, fge.default_params(coarse_max_px=4096)).n_coarse == 6
    assert fge.plan(3072, 4096, fge.default_params(coarse_max_px=1024)).n_coarse == 5
    assert fge.plan(64, 64, fge.default_params(coarse_max_px=4096)).n_coarse == 6
    # with a larger low-resolution threshold the 10-sweep levels stay in the block (to 4096 px)
    big = fge.plan(3072, 4096, fge.default_params(small_size=64))
    assert big.n_coarse == 6 and big.levels[5][2] == 10


def test_workspace_sizes(fge):
    for (W, H) in ((4096, 3072), (1024, 768), (300, 7), (65, 65)):
        info = fge.plan(H, W)
        lv = info.levels
        need32 = fge.workspace_bytes(H, W)
        need16 = fge.workspace_bytes(H, W, fge.default_params(storage=fge.F16))
        if len(lv) >= 2 and info.n_coarse < len(lv):
            px = [w * h for (w, h, _) in lv]
            # the coarse block's last level is always stored (levels inside a pyramid run of
            # tile levels may stay in LDS, so the level before the finest need not be)
            assert need32 >= 6 * 4 * px[info.n_coarse - 1]
            assert need16 >= 6 * 2 * px[info.n_coarse - 1]
            # two ping-pong state buffers plus the compact copies of the small levels' inputs
            small = sum(q for q in px if q <= 65536) if W * H > 65536 else 0
            assert need32 <= 6 * 4 * (px[-2] + px[-3]) + 16 * small + 256 * (len(px) + 2)
    assert fge.workspace_bytes(64, 64, fge.default_params(coarse_max_px=4096)) == 0   # all coarse


# Fake device addresses for calls the host-side checks reject before any launch: 4 GiB apart, so
# that no buffer of any size used here overlaps another (overlaps are rejected too).
I0, A0, F0, B0, WS0 = 1 << 32, 2 << 32, 3 << 32, 4 << 32, 8 << 32


def _call(fge, W, H, p, I=I0, A=A0, F=F0, B=B0, ws=None, ws_len=0):
    lib = fge.load()
    return lib.fge_estimate_foreground(I, A, H, W, ctypes.byref(p) if p is not None else None,
                                       F, B, ws, ws_len, None)


def test_argument_errors_before_launch(fge):
    p = fge.default_params()
    assert _call(fge, 0, 10, p) == fge.FGE_EINVAL
    assert _call(fge, 10, 40000, p) == fge.FGE_EINVAL
    assert _call(fge, 64, 64, p, I=None) == fge.FGE_EINVAL
    assert _call(fge, 64, 64, p, F=5 << 32, B=5 << 32) == fge.FGE_EINVAL
    for field, bad in (("size", 12), ("storage", 7), ("order", 3), ("kernel", 9),
                       ("eps_r", 0.0), ("omega", -1.0), ("iters_big", -2), ("strip_rows", -1),
                       ("coarse_max_px", 5000), ("tile_max_px", -2)):
        q = fge.default_params()
        setattr(q, field, bad)
        assert _call(fge, 64, 64, q) == fge.FGE_EINVAL, field
    q = fge.default_params(kernel=fge.KERNEL_FUSED, iters_big=3)
    assert _call(fge, 1024, 768, q, ws=WS0, ws_len=1 << 30) == fge.FGE_EUNSUPPORTED
    need = fge.workspace_bytes(768, 1024, p)
    assert _call(fge, 1024, 768, p) == fge.FGE_EWORKSPACE
    assert _call(fge, 1024, 768, p, ws=WS0, ws_len=need - 1) == fge.FGE_EWORKSPACE
    assert _call(fge, 1024, 768, p, ws=WS0 + 16, ws_len=need) == fge.FGE_EWORKSPACE
    assert fge.load().fge_status_string(fge.FGE_EWORKSPACE).startswith(b"FGE_EWORKSPACE")


def test_batch_planning_host_only(fge):
    from paper_2006_14970_amd import synth
    sizes = synth.batch_sizes()
    p16 = fge.default_params(storage=fge.F16)
    b = fge.Batch([(h, w) for w, h in sizes], p16)
    n_levels = [len(fge.plan(h, w, p16).levels) for w, h in sizes]
    n_coarse = [fge.plan(h, w, p16).n_coarse for w, h in sizes]
    assert b.steps == max(n - c for n, c in zip(n_levels, n_coarse))
    assert 4 <= b.launch_count <= 2 + 2 + 2 * b.steps
    # the batch needs at least every image's own workspace
    assert b.workspace_bytes >= sum(fge.workspace_bytes(h, w, p16) for w, h in sizes)
    lib = fge.load()
    n = len(sizes)
    W = (ctypes.c_int32 * n)(*[w for w, _ in sizes])
    H = (ctypes.c_int32 * n)(*[h for _, h in sizes])
    assert lib.fge_batch_workspace_bytes_for(n, H, W, ctypes.byref(p16)) == b.workspace_bytes
    b.close()


def test_batch_argument_errors(fge):
    with pytest.raises(fge.FgeError) as e:
        fge.Batch([(10, 10), (5, 0)])
    assert e.value.status == fge.FGE_EINVAL
    with pytest.raises(fge.FgeError) as e:
        fge.Batch([(200, 300)], fge.default_params(kernel=fge.KERNEL_NAIVE))
    assert e.value.status == fge.FGE_EUNSUPPORTED
    with pytest.raises(fge.FgeError) as e:
        fge.Batch([(200, 300)], fge.default_params(coarse_max_px=-1))
    assert e.value.status == fge.FGE_EUNSUPPORTED
    b = fge.Batch([(200, 300), (50, 40)])
    lib = fge.load()
    null = (ctypes.c_void_p * 2)()
    assert lib.fge_batch_run(b._h, null, null, null, null, None, 0, None) == fge.FGE_EINVAL
    b.close()


def test_server_host_functions(fge):
    """Server configuration, footprints and argument errors (no device call is reached)."""
    assert ctypes.sizeof(fge.ServerConfig) == 32
    assert ctypes.sizeof(fge.ServerResult) == 48
    assert ctypes.sizeof(fge.ServerStats) == 96
    c = fge.server_config()
    assert (c.size, c.max_active, c.pipeline_depth, c.budget_bytes, c.tick_table_bytes) == \
        (32, 1024, 2, 0, 16 << 20)
    assert fge.server_reserved_bytes(c) == 2 * (16 << 20)
    assert fge.server_reserved_bytes(fge.server_config(pipeline_depth=3)) == 3 * (16 << 20)
    p16 = fge.default_params(storage=fge.F16)
    # The footprint is I, alpha, F, B plus the served plan's workspace.  For images above
    # 64K px the single-image plan keeps its compact input copies in F instead of the workspace,
    # so the served workspace exceeds fge_workspace_bytes by the small levels' copies (levels of
    # at most 64K px: 4 planes of fewer than 2^17 px in all).
    for (W, H), staged in (((4096, 3072), True), ((300, 7), False), ((1, 1), False),
                           ((1920, 1080), True)):
        for p, elem in ((p16, 2), (None, 4)):
            ws = fge.workspace_bytes(H, W, p) if p else fge.workspace_bytes(H, W)
            got = fge.server_request_bytes(H, W, p) if p else fge.server_request_bytes(H, W)
            extra = got - (10 * elem * W * H + (ws + 255) // 256 * 256)
            if staged:
                assert 0 < extra <= 4 * elem * (1 << 17) + 16 * 256, (W, H, elem, extra)
            else:
                assert extra == 0, (W, H, elem, extra)
    assert fge.server_request_bytes(5, 0) == 0
    lib = fge.load()
    h = ctypes.c_void_p()
    big = 1 << 30

    def create(p=None, cfg=None, arena=0x100000, nbytes=big, stream=0x10):
        return lib.fge_server_create(ctypes.byref(p) if p else None,
                                     ctypes.byref(cfg) if cfg else None, arena, nbytes, stream,
                                     ctypes.byref(h))

    assert create(arena=None) == fge.FGE_EINVAL
    assert create(stream=None) == fge.FGE_EINVAL
    assert create(arena=0x100010) == fge.FGE_EINVAL
    assert create(nbytes=32 << 20) == fge.FGE_EWORKSPACE
    assert create(cfg=fge.server_config(pipeline_depth=9)) == fge.FGE_EINVAL
    assert create(cfg=fge.server_config(max_active=-1)) == fge.FGE_EINVAL
    assert create(cfg=fge.server_config(tick_table_bytes=1024)) == fge.FGE_EINVAL
    bad = fge.server_config()
    bad.size = 8
    assert create(cfg=bad) == fge.FGE_EINVAL
    assert create(p=fge.default_params(kernel=fge.KERNEL_NAIVE)) == fge.FGE_EUNSUPPORTED
    assert create(p=fge.default_params(coarse_max_px=-1)) == fge.FGE_EUNSUPPORTED
    assert create(p=fge.default_params(eps_r=0.0)) == fge.FGE_EINVAL
    assert not h.value
    assert fge.load().fge_status_string(fge.FGE_EBUDGET).startswith(b"FGE_EBUDGET")


def test_autotuner_host_side(fge):
    lib = fge.load()
    assert lib.fge_tune_candidates() == 21
    for (W, H) in ((4096, 3072), (1024, 768), (300, 7)):
        need = lib.fge_tune_workspace_bytes(H, W, None)
        assert need >= fge.workspace_bytes(H, W)
        for t in (0, 1 << 16, 1 << 18, 1 << 20):
            assert need >= fge.workspace_bytes(H, W, fge.default_params(tile_max_px=t))
    sizes = [(300, 200), (1024, 768), (77, 900)]
    W = (ctypes.c_int32 * 3)(*[w for w, _ in sizes])
    H = (ctypes.c_int32 * 3)(*[h for _, h in sizes])
    assert lib.fge_batch_tune_workspace_bytes(3, H, W, None) >= \
        lib.fge_batch_workspace_bytes_for(3, H, W, None)
    best = fge.Params()
    # argument errors are reported before anything touches the device
    assert lib.fge_autotune(None, A0, 64, 64, None, F0, B0, None, 0, None, 3,
                            ctypes.byref(best), None, 0, None) == fge.FGE_EINVAL
    assert lib.fge_autotune(I0, A0, 64, 64, None, F0, B0, None, 0, None, 3,
                            None, None, 0, None) == fge.FGE_EINVAL
    assert lib.fge_autotune(I0, A0, 768, 1024, None, F0, B0, None, 0, None, 3,
                            ctypes.byref(best), None, 0, None) == fge.FGE_EWORKSPACE
    null = (ctypes.c_void_p * 3)()
    assert lib.fge_batch_autotune(3, null, null, H, W, None, null, null, None, 0, None, 3,
                                  ctypes.byref(best), None, 0, None) == fge.FGE_EWORKSPACE


def test_reporting_and_layout_argument_errors(fge):
    lib = fge.load()
    assert lib.fge_energy_workspace_bytes(3072, 4096) == 2048 * 5 * 8
    assert lib.fge_energy_workspace_bytes(10, 10) == 256
    assert lib.fge_energy_workspace_bytes(10, 0) == 0
    a = 0x100000
    assert lib.fge_energy(a, a, a, a, 64, 64, None, None, a, 256, None) == fge.FGE_EINVAL
    assert lib.fge_energy(a, a, a, a, 64, 64, None, a, None, 0, None) == fge.FGE_EWORKSPACE
    assert lib.fge_energy(a, a, a, a, 64, 64, None, a, a + 16, 256, None) == fge.FGE_EWORKSPACE
    assert lib.fge_energy(a, a, a, a, 64, 0, None, a, a, 256, None) == fge.FGE_EINVAL
    assert lib.fge_hwc_to_planar(a, fge.U8, 5, 8, 8, a, a, fge.F32, None) == fge.FGE_EINVAL
    assert lib.fge_hwc_to_planar(a, fge.U8, 4, 8, 8, a, None, fge.F32, None) == fge.FGE_EINVAL
    assert lib.fge_hwc_to_planar(a, 7, 3, 8, 8, a, None, fge.F32, None) == fge.FGE_EINVAL
    assert lib.fge_planar_to_hwc(a, fge.F32, 8, 8, a, 9, None) == fge.FGE_EINVAL
    assert lib.fge_planar_to_hwc(None, fge.F32, 8, 8, a, fge.U8, None) == fge.FGE_EINVAL


def test_jacobi_and_converge_host_side(fge):
    lib = fge.load()
    pj = fge.default_params(order=fge.JACOBI)
    info = fge.plan(768, 1024, pj)
    assert info.n_coarse == 0 and [it for _, _, it in info.levels] == \
        [it for _, _, it in fge.plan(768, 1024).levels]
    need = lib.fge_converge_workspace_bytes(768, 1024, ctypes.byref(pj))
    # Jacobi temporary (6 planes at full size) on top of the level buffers
    assert need >= 6 * 4 * 1024 * 768 and fge.workspace_bytes(768, 1024, pj) == need
    with pytest.raises(fge.FgeError) as e:
        fge.plan(768, 1024, fge.default_params(order=fge.JACOBI, kernel=fge.KERNEL_FUSED))
    assert e.value.status == fge.FGE_EUNSUPPORTED
    with pytest.raises(fge.FgeError) as e:
        fge.Batch([(200, 300)], pj)
    assert e.value.status == fge.FGE_EUNSUPPORTED
    a = 0x100000
    p = fge.default_params()
    nw = lib.fge_converge_workspace_bytes(64, 64, ctypes.byref(p))

    def conv(tol, ms, ws=WS0, nbytes=nw, I=I0):
        return lib.fge_estimate_foreground_converge(I, A0, 64, 64, ctypes.byref(p), tol, ms,
                                                    F0, B0, None, ws, nbytes, None)
    assert conv(1e-4, 0) == fge.FGE_EINVAL
    assert conv(1e-4, 100001) == fge.FGE_EINVAL
    assert conv(float("nan"), 10) == fge.FGE_EINVAL
    assert conv(1e-4, 10, I=None) == fge.FGE_EINVAL
    assert conv(1e-4, 10, nbytes=nw - 1) == fge.FGE_EWORKSPACE
    assert conv(1e-4, 10, ws=None) == fge.FGE_EWORKSPACE
    h = ctypes.c_void_p()
    assert lib.fge_server_create(ctypes.byref(pj), None, 0x100000, 1 << 30, 0x10,
                                 ctypes.byref(h)) == fge.FGE_EUNSUPPORTED


def test_quality_argument_errors(fge):
    lib = fge.load()
    a = 0x100000
    nw = lib.fge_quality_workspace_bytes(64, 64)
    assert nw == 16 * 4 * 8          # 16 blocks of 256 pixels, 4 partial sums each
    assert lib.fge_quality(a, a, a, 64, 64, fge.U8, 1.4, a, a, nw, None) == fge.FGE_EINVAL
    assert lib.fge_quality(a, a, a, 64, 64, fge.F32, 0.0, a, a, nw, None) == fge.FGE_EINVAL
    assert lib.fge_quality(a, a, a, 64, 64, fge.F32, 5.0, a, a, nw, None) == fge.FGE_EINVAL
    assert lib.fge_quality(a, a, a, 64, 64, fge.F32, 1.4, a, None, 0, None) == fge.FGE_EWORKSPACE
    assert lib.fge_quality(None, a, a, 64, 64, fge.F32, 1.4, a, a, nw, None) == fge.FGE_EINVAL
    assert lib.fge_composite(a, a, a, 64, 64, fge.U8, a, None) == fge.FGE_EINVAL
    assert lib.fge_composite(a, a, a, 64, 0, fge.F32, a, None) == fge.FGE_EINVAL


def test_level_options_host_side(fge):
    lib = fge.load()
    assert ctypes.sizeof(fge.LevelOptions) == 24
    p = fge.default_params()
    near = fge.level_options("nearest")
    smooth = fge.level_options("smooth")
    wn = lib.fge_levels_workspace_bytes(768, 1024, ctypes.byref(p), ctypes.byref(near))
    wsm = lib.fge_levels_workspace_bytes(768, 1024, ctypes.byref(p), ctypes.byref(smooth))
    assert wn == lib.fge_converge_workspace_bytes(768, 1024, ctypes.byref(p))
    # level copies (4 float planes of 512x384) and the row pass (4 planes of 512x768) on top
    assert wsm >= wn + 16 * 512 * 384 + 16 * 512 * 768
    bad = fge.level_options("smooth")
    bad.size = 16
    assert lib.fge_levels_workspace_bytes(64, 64, ctypes.byref(p), ctypes.byref(bad)) == 0
    a = 0x100000
    nw = lib.fge_levels_workspace_bytes(64, 64, ctypes.byref(p), ctypes.byref(smooth))

    def run(o, ws=WS0):
        return lib.fge_estimate_foreground_levels(I0, A0, 64, 64, ctypes.byref(p),
                                                  ctypes.byref(o), F0, B0, None, ws, nw, None)
    assert run(bad) == fge.FGE_EINVAL
    odd = fge.level_options("smooth")
    odd.resize = 7
    assert run(odd) == fge.FGE_EINVAL
    assert run(fge.level_options("smooth", tol=1e-4, max_sweeps=0)) == fge.FGE_EINVAL
    assert run(smooth, ws=None) == fge.FGE_EWORKSPACE
    # passes = 1: the layout of the fused passes (the smooth one adds its row pass), errors
    pn = fge.level_options("nearest", tol=1e-4, passes=True)
    ps = fge.level_options("smooth", tol=1e-4, passes=True)
    wpn = lib.fge_levels_workspace_bytes(768, 1024, ctypes.byref(p), ctypes.byref(pn))
    wps = lib.fge_levels_workspace_bytes(768, 1024, ctypes.byref(p), ctypes.byref(ps))
    assert wpn == lib.fge_converge_passes_workspace_bytes(768, 1024, ctypes.byref(p))
    assert wps >= wpn + 16 * 512 * 768
    nps = lib.fge_levels_workspace_bytes(64, 64, ctypes.byref(p), ctypes.byref(ps))
    assert run(fge.level_options("smooth", tol=-1.0, passes=True), ws=WS0) == fge.FGE_EINVAL
    assert run(fge.level_options("smooth", tol=1e-4, max_sweeps=0, passes=True)) == fge.FGE_EINVAL
    two = fge.level_options("smooth", tol=1e-4, passes=True)
    two.passes = 2
    assert run(two) == fge.FGE_EINVAL
    assert lib.fge_estimate_foreground_levels(I0, A0, 64, 64, ctypes.byref(p), ctypes.byref(ps),
                                              F0, B0, None, WS0, nps - 1, None) == fge.FGE_EWORKSPACE


def test_staged_inputs_do_not_grow_workspace(fge):
    """A large single image stages the compact inputs of its intermediate levels in F's memory
    (F is written only by the finest level), so its workspace is the two ping-pong state
    buffers alone: level 11 (2048x1573) in one, level 10 (1024x806) in the other."""
    def a256(x):
        return (x + 255) // 256 * 256
    for elem, p in ((4, None), (2, fge.default_params(storage=fge.F16))):
        want = a256(6 * 2048 * 1573 * elem) + a256(6 * 1024 * 806 * elem)
        got = fge.workspace_bytes(3072, 4096, p) if p else fge.workspace_bytes(3072, 4096)
        assert got == want, (elem, got, want)


def test_outputs_overlapping_inputs_rejected(fge):
    """F and B may not share a byte with I, alpha, each other or the workspace: the single-image,
    converge and batch entry points compare the byte ranges before anything is enqueued."""
    p = fge.default_params()
    H, W = 300, 700
    plane = H * W * 4
    need = fge.workspace_bytes(H, W, p)
    ok = dict(ws=WS0, ws_len=need)
    # a valid layout passes the checks and would launch: use a plan that fails later instead
    # (FGE_EWORKSPACE with one byte too few), so nothing is enqueued
    assert _call(fge, W, H, p, ws=WS0, ws_len=need - 1) == fge.FGE_EWORKSPACE
    bad = [dict(F=I0 + 3 * plane - 1),                # last byte of I
           dict(F=A0 - 3 * plane + 1),                # F's last byte on alpha's first
           dict(B=A0 + plane - 4),
           dict(B=F0 + 3 * plane - 1),                # F and B share a byte
           dict(F=WS0 + need - 1),                    # F starts inside the workspace
           dict(B=WS0 - 3 * plane + 1)]
    for kw in bad:
        assert _call(fge, W, H, p, **kw, **ok) == fge.FGE_EINVAL, kw
    # touching ranges are fine (one byte apart)
    assert _call(fge, W, H, p, F=I0 + 3 * plane, B=I0 + 6 * plane, ws=WS0, ws_len=need - 1) == \
        fge.FGE_EWORKSPACE
    lib = fge.load()
    nw = lib.fge_converge_workspace_bytes(H, W, ctypes.byref(p))
    assert lib.fge_estimate_foreground_converge(I0, A0, H, W, ctypes.byref(p), 1e-4, 10, I0 + 8,
                                                B0, None, WS0, nw, None) == fge.FGE_EINVAL
    b = fge.Batch([(H, W)], p)
    arr = lambda v: (ctypes.c_void_p * 1)(v)   # noqa: E731
    assert lib.fge_batch_run(b._h, arr(I0), arr(A0), arr(A0 + 16), arr(B0), WS0,
                             b.workspace_bytes, None) == fge.FGE_EINVAL
    b.close()


def _header_params(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"\b" + name + r"\s*\(([^)]*)\)", text)
    assert m, name
    return [re.sub(r"[^A-Za-z0-9_]", " ", a).split()[-1] for a in m.group(1).split(",")]


def test_header_sizes_are_height_first():
    """Every size pair of the C ABI is (H, W): the header's parameter names, checked for every
    declaration that takes both."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(fge_[a-z_0-9]+)\s*\(", text)))
    seen = 0
    for name in names:
        args = _header_params(name)
        if "H" in args and "W" in args:
            assert args.index("H") + 1 == args.index("W"), (name, args)
            seen += 1
    assert seen >= 20
    assert _header_params("fge_estimate_foreground")[:4] == ["I", "alpha", "H", "W"]
    assert _header_params("fge_workspace_bytes") == ["H", "W", "p"]
    assert _header_params("fge_batch_create")[:3] == ["n", "H", "W"]


def test_non_square_plan_order(fge):
    """A non-square size in the ABI's order plans the image the caller means: 301 rows of 700
    pixels give level sizes whose widths are the larger ones."""
    info = fge.plan(301, 700)
    w, h, _ = info.levels[-1]
    assert (w, h) == (700, 301)
    lib = fge.load()
    arr = ctypes.c_int32 * 16
    wo, ho, it = arr(), arr(), arr()
    n, nc = ctypes.c_int32(), ctypes.c_int32()
    assert lib.fge_plan(301, 700, None, 16, wo, ho, it, ctypes.byref(n), ctypes.byref(nc)) == 0
    assert (wo[n.value - 1], ho[n.value - 1]) == (700, 301)


def test_closed_form_params_and_argument_errors(fge):
    """fge_closed_form: the parameter block's layout and defaults (omega 1 as eq. 2 prints it,
    the eps regulariser, the 1e-6 residual of the remark after eq. 2), the workspace size, and
    every argument error returned before anything is enqueued."""
    p = fge.cf_default_params()
    assert p.size == ctypes.sizeof(fge.CfParams) == 40
    assert (p.omega, p.eps, p.tol, p.max_iter, p.storage, p.warm_start) == (1.0, 5e-3, 1e-6,
                                                                            20000, fge.F32, 0)
    assert ctypes.sizeof(fge.CfInfo) == 80
    lib = fge.load()
    H, W = 300, 700
    need = fge.cf_workspace_bytes(H, W)
    assert need >= 5 * 6 * 8 * H * W and need % 256 == 0
    assert fge.cf_workspace_bytes(0, 5) == 0 and fge.cf_workspace_bytes(5, 40000) == 0

    def call(H=H, W=W, p=p, I=I0, A=A0, F=F0, B=B0, ws=WS0, ws_len=None):
        info = fge.CfInfo()
        return lib.fge_closed_form(I, A, H, W, ctypes.byref(p) if p is not None else None, F, B,
                                   ws, need if ws_len is None else ws_len, None,
                                   ctypes.byref(info))

    assert call(ws_len=need - 1) == fge.FGE_EWORKSPACE            # passes every other check
    assert call(ws=None) == fge.FGE_EWORKSPACE
    assert call(ws=WS0 + 8) == fge.FGE_EWORKSPACE                 # unaligned
    assert call(H=1, W=1, ws_len=0) == fge.FGE_EINVAL             # one pixel: no edge, singular
    assert call(H=0) == fge.FGE_EINVAL
    assert call(I=None) == fge.FGE_EINVAL
    assert call(F=I0 + 8) == fge.FGE_EINVAL                       # output overlaps the input
    assert call(B=F0) == fge.FGE_EINVAL
    for field, bad in (("eps", 0.0), ("eps", float("nan")), ("omega", -1.0), ("tol", 0.0),
                       ("tol", float("inf")), ("max_iter", -1), ("storage", fge.U8), ("size", 8)):
        q = fge.cf_default_params()
        setattr(q, field, bad)
        assert call(p=q) == fge.FGE_EINVAL, field
    # the estimation entry points do not take float64 storage
    assert _call(fge, 64, 64, fge.default_params(storage=fge.F64)) == fge.FGE_EINVAL
