"""CPU checks of the C ABI: the library loads, exports every entry point include/megs.h declares,
and rejects bad arguments before any GPU work (no compute call needs a GPU here)."""
import ctypes
import os
import re

import pytest

from paper_2509_07021_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "megs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(megs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(L.EXPORTED) == set(names)


def test_flag_values_match_the_header():
    text = open(os.path.join(ROOT, "include", "megs.h")).read()
    flags = dict((name, int(val)) for name, val in re.findall(r"#define (MEGS_FLAG_[A-Z_]+) (\d+)u", text))
    assert set(flags) == {"MEGS_FLAG_ONE_STAGE_SORT", "MEGS_FLAG_PERSISTENT", "MEGS_FLAG_STATS",
                          "MEGS_FLAG_DETERMINISTIC", "MEGS_FLAG_RECORD_PLANES"}
    for name, val in flags.items():
        assert getattr(L, name) == val, name
    assert len(set(flags.values())) == len(flags) and all(v & (v - 1) == 0 for v in flags.values())


def test_version_and_empty_error():
    lib = L.load()
    assert lib.megs_version().startswith(b"megs")
    assert isinstance(lib.megs_last_error(), bytes)


def _args(tile=16, batch=64, flags=0, nv=1, k=0, width=32, height=32, n=0, dt=0, cap=0, waves=0, subtile=0):
    sc = L.MegsScene()
    sc.n, sc.k, sc.dt_geom, sc.dt_color, sc.dt_amp = n, k, dt, 0, 0
    cams = (L.MegsCamera * max(nv, 1))()
    for c in cams:
        c.width, c.height, c.fx, c.fy, c.znear = width, height, 20.0, 20.0, 0.2
    cfg = L.MegsConfig(tile, batch, flags, waves, cap, subtile, 0)
    return sc, cams, cfg


def _forward(sc, cams, nv, cfg):
    lib = L.load()
    st = L.MegsState()
    noop = L.ALLOC_FN(lambda ctx, n: None)
    status = lib.megs_render_forward(ctypes.byref(sc), cams, nv, ctypes.byref(cfg), noop, None,
                                     ctypes.c_void_p(16), ctypes.byref(st), None)
    return status, lib.megs_last_error().decode()


@pytest.mark.parametrize("kw,needle", [
    (dict(tile=12), "tile"),
    (dict(batch=100), "batch"),
    (dict(batch=16), "batch"),
    (dict(flags=64), "flags"),
    (dict(nv=0), "n_views"),
    (dict(nv=65), "n_views"),
    (dict(k=9), "k ="),
    (dict(width=0), "image size"),
    (dict(dt=7), "dtype"),
    (dict(n=-1), "n ="),
    (dict(n=10), "null geometry"),
    (dict(cap=-5), "pair_capacity"),
    (dict(waves=3), "waves"),
    (dict(tile=8, waves=2), "one wave"),
    (dict(subtile=4), "subtile"),
    (dict(tile=8, subtile=8), "subtile"),
])
def test_forward_rejects_bad_arguments(kw, needle):
    nv = kw.pop("nv", 1)
    sc, cams, cfg = _args(nv=nv, **kw)
    status, msg = _forward(sc, cams, nv, cfg)
    assert status == L.MEGS_ERR_ARG, (status, msg)
    assert needle in msg


def test_backward_and_graph_reject_bad_state():
    lib = L.load()
    sc, cams, cfg = _args()
    st = L.MegsState()
    g = L.MegsSceneGrad()
    noop = L.ALLOC_FN(lambda ctx, n: None)
    status = lib.megs_render_backward(ctypes.byref(sc), cams, 1, ctypes.byref(cfg), ctypes.byref(st),
                                      ctypes.c_void_p(16), noop, None, ctypes.byref(g), None)
    assert status == L.MEGS_ERR_ARG
    assert "state" in lib.megs_last_error().decode()
    h = ctypes.c_void_p()
    status = lib.megs_graph_create(ctypes.byref(sc), cams, 1, ctypes.byref(cfg), noop, None, ctypes.c_void_p(16),
                                   None, None, 0, ctypes.c_void_p(1), ctypes.byref(h))
    assert status == L.MEGS_ERR_ARG and "pair_capacity" in lib.megs_last_error().decode()


def test_mask_gradient_planes_must_match_scene():
    lib = L.load()
    sc, cams, cfg = _args(n=4)
    for p in L.PLANES:
        if p not in ("pmask_logit", "lmask_logit", "axis", "sharp", "amp"):
            setattr(sc, p, 16)
    sc.pmask_logit = 16
    g = L.MegsSceneGrad()
    for p in ("pos", "logscale", "quat", "op_logit", "base"):
        setattr(g, p, 16)
    st = L.MegsState()
    st.n_records, st.n_views, st.tile, st.internal = 4, 1, 16, 16
    noop = L.ALLOC_FN(lambda ctx, n: None)
    status = lib.megs_render_backward(ctypes.byref(sc), cams, 1, ctypes.byref(cfg), ctypes.byref(st),
                                      ctypes.c_void_p(16), noop, None, ctypes.byref(g), None)
    assert status == L.MEGS_ERR_ARG and "pmask_logit" in lib.megs_last_error().decode()


def test_profile_calls_without_work():
    lib = L.load()
    assert lib.megs_profile_begin() == L.MEGS_OK
    p = L.MegsProfile()
    assert lib.megs_profile_end(ctypes.byref(p)) == L.MEGS_OK
    assert all(c == 0 for c in p.count)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libmegs.so"))
    with pytest.raises(RuntimeError, match="not built"):
        L.load()


def test_compact_and_compressed_rows_reject_bad_arguments():
    lib = L.load()
    noop = L.ALLOC_FN(lambda ctx, n: None)
    out = L.MegsCompacted()
    sc, cams, cfg = _args()
    status = lib.megs_compact(ctypes.byref(sc), float("nan"), 1.0, noop, None, None, ctypes.byref(out))
    assert status == L.MEGS_ERR_ARG and "NaN" in lib.megs_last_error().decode()
    status = lib.megs_compact(ctypes.byref(sc), 0.01, 1.0, ctypes.cast(None, L.ALLOC_FN), None, None,
                              ctypes.byref(out))
    assert status == L.MEGS_ERR_ARG
    # dense scenes carry no lobe count; compressed rows need 0 <= n_lobes <= n k
    sc, cams, cfg = _args(n=0, k=3)
    sc.n_lobes = 5
    status, msg = _forward(sc, cams, 1, cfg)
    assert status == L.MEGS_ERR_ARG and "n_lobes" in msg
    sc.lobe_off = 16
    sc.n_lobes = 1
    status, msg = _forward(sc, cams, 1, cfg)
    assert status == L.MEGS_ERR_ARG and "exceeds" in msg
    sc.n_lobes = -1
    status, msg = _forward(sc, cams, 1, cfg)
    assert status == L.MEGS_ERR_ARG and "n_lobes" in msg


def test_loss_and_adam_reject_bad_arguments():
    lib = L.load()
    noop = L.ALLOC_FN(lambda ctx, n: None)
    sizes = (ctypes.c_int32 * 2)(16, 16)
    st = lib.megs_photometric_loss(ctypes.c_void_p(16), ctypes.c_void_p(16), 0, sizes, 0.2, noop, None,
                                   ctypes.c_void_p(16), None, None)
    assert st == L.MEGS_ERR_ARG and "n_views" in lib.megs_last_error().decode()
    st = lib.megs_photometric_loss(ctypes.c_void_p(16), ctypes.c_void_p(16), 1, sizes, 1.5, noop, None,
                                   ctypes.c_void_p(16), None, None)
    assert st == L.MEGS_ERR_ARG and "lambda" in lib.megs_last_error().decode()
    bad = (ctypes.c_int32 * 2)(0, 16)
    st = lib.megs_photometric_loss(ctypes.c_void_p(16), ctypes.c_void_p(16), 1, bad, 0.2, noop, None,
                                   ctypes.c_void_p(16), None, None)
    assert st == L.MEGS_ERR_ARG and "size" in lib.megs_last_error().decode()
    st = lib.megs_photometric_loss(ctypes.c_void_p(16), ctypes.c_void_p(16), 1, sizes, 0.2, noop, None,
                                   ctypes.c_void_p(16), None, None)
    assert st == L.MEGS_ERR_ALLOC
    v = ctypes.c_void_p(16)
    assert lib.megs_adam_step(4, v, 7, v, v, v, 1e-3, 0.9, 0.999, 1e-15, 1, None) == L.MEGS_ERR_ARG
    assert lib.megs_adam_step(4, v, 0, v, v, v, 1e-3, 0.9, 0.999, 1e-15, 0, None) == L.MEGS_ERR_ARG
    assert lib.megs_adam_step(4, v, 0, v, v, v, 1e-3, 1.0, 0.999, 1e-15, 1, None) == L.MEGS_ERR_ARG
    assert lib.megs_adam_step(0, None, 0, None, None, None, 1e-3, 0.9, 0.999, 1e-15, 1, None) == L.MEGS_OK


def test_noalloc_forward_rejects_what_does_not_fit():
    """The no-allocation forward refuses, before any launch, work whose memory exceeds its static
    scratch: here the per-pixel state of one 4096 x 4096 view alone."""
    lib = L.load()
    sc, cams, cfg = _args(width=4096, height=4096)
    st = L.MegsState()
    status = lib.megs_render_forward_noalloc(ctypes.byref(sc), cams, 1, ctypes.byref(cfg), ctypes.c_void_p(16),
                                             ctypes.byref(st), None)
    assert status == L.MEGS_ERR_CAPACITY
    msg = lib.megs_last_error().decode()
    assert "static scratch" in msg and str(L.MEGS_NOALLOC_SCRATCH_BYTES) in msg
    sc, cams, cfg = _args(cap=8 << 20)  # a fixed pair table of 8M pairs does not fit either
    status = lib.megs_render_forward_noalloc(ctypes.byref(sc), cams, 1, ctypes.byref(cfg), ctypes.c_void_p(16),
                                             ctypes.byref(st), None)
    assert status == L.MEGS_ERR_CAPACITY
    sc, cams, cfg = _args(tile=12)  # argument checks come first, as in megs_render_forward
    status = lib.megs_render_forward_noalloc(ctypes.byref(sc), cams, 1, ctypes.byref(cfg), ctypes.c_void_p(16),
                                             ctypes.byref(st), None)
    assert status == L.MEGS_ERR_ARG


def _sized(n, nv, w, h, tile, sub, flags, cap, n_pairs):
    """megs_state_bytes for a scene of n Gaussians (plane pointers are placeholders: nothing is
    launched or read)."""
    lib = L.load()
    sc, cams, cfg = _args(tile=tile, nv=nv, width=w, height=h, n=n, k=4, flags=flags, cap=cap, subtile=sub)
    for p in L.PLANES:
        setattr(sc, p, 1 << 20)
    mem = L.MegsMemory()
    status = lib.megs_state_bytes(ctypes.byref(sc), cams, nv, ctypes.byref(cfg), n_pairs, ctypes.byref(mem))
    assert status == L.MEGS_OK, lib.megs_last_error().decode()
    return mem


def test_state_bytes_sizes_the_forward_and_backward():
    """The memory of a forward and backward (host only). The backward's per-record sums (36 bytes per
    record) and, when they fit, the pair sort's alternate buffers (8 bytes per pair) live in the
    forward's work space, which is free after the key emission; the deterministic mode keeps its
    work space and allocates both."""
    n, nv, P = 1_000_000, 8, 32_000_000
    nr = n * nv
    npix = nv * 1920 * 1080
    m = _sized(n, nv, 1920, 1080, 32, 8, 0, 0, P)
    assert m.backward == 0 and m.work >= 36 * nr
    assert 48 * nr + 8 * npix + m.work <= m.frame <= 48 * nr + 8 * npix + m.work + (1 << 20)
    assert 8 * P <= m.pairs <= 8 * P + (1 << 20)            # sorted keys and values only
    few = _sized(n, nv, 1920, 1080, 32, 8, 0, 0, 4_000_000)  # the alternates fit with room to spare
    assert few.work == m.work and few.pairs <= 8 * 4_000_000 + (1 << 20)
    many = _sized(n, nv, 1920, 1080, 32, 8, 0, 0, 60_000_000)  # they do not fit: the pair block holds them
    assert many.work == m.work and many.pairs >= 16 * 60_000_000
    fixed = _sized(n, nv, 1920, 1080, 32, 8, 0, 60_000_000, 0)  # a known capacity sizes the work space for them
    assert fixed.work >= 8 * 60_000_000 and fixed.pairs <= 8 * 60_000_000 + (1 << 20) and fixed.backward == 0
    det = _sized(n, nv, 1920, 1080, 32, 0, L.MEGS_FLAG_DETERMINISTIC, 0, P)
    assert det.work < 36 * nr and det.pairs >= 24 * P and det.backward >= 36 * nr + 36 * P
    lib = L.load()
    sc, cams, cfg = _args()
    assert lib.megs_state_bytes(ctypes.byref(sc), cams, 1, ctypes.byref(cfg), -1, ctypes.byref(L.MegsMemory())) \
        == L.MEGS_ERR_ARG


def test_stages_are_roctx_ranges():
    """Every stage's enqueue is a named ROCTX range (for rocprofv3 --marker-trace): the library imports
    the range calls and holds one name per stage."""
    import subprocess
    syms = subprocess.run(["nm", "-D", L.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert "roctxRangePushA" in syms and "roctxRangePop" in syms
    data = open(L.LIB_PATH, "rb").read()
    for stage in L.STAGES:
        assert f"megs:{stage}".encode() + b"\0" in data, stage
