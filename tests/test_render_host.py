"""CPU tests of the binding's host logic: the autotuner cache (its key and the JSON file it keeps)."""
import json



from paper_2509_07021_amd import render as R
from paper_2509_07021_amd import scenes as S


class _FakeScene:
    """The fields autotune_key reads, without device memory."""

    def __init__(self, n=1000, k=4, dt=("f16", "f16", "bf16"), pmask=True, lmask=False, ragged=False):
        self.n, self.k, self.dt = n, k, dt
        self.has_pmask, self.has_lmask, self.ragged = pmask, lmask, ragged
        self.planes = {}
        self.sh_degree = 0


def test_autotune_key_separates_what_the_timings_depend_on():
    cams = [S.look_at((0, -4, 0), 640, 360), S.look_at((0, 4, 0), 1920, 1080)]
    base = R.autotune_key(_FakeScene(), cams, R.Config(16, 64), "gfx950")
    assert base == R.autotune_key(_FakeScene(), cams, R.Config(32, 128), "gfx950")  # the tuned fields are not in it
    others = [R.autotune_key(_FakeScene(n=1001), cams, R.Config(16, 64), "gfx950"),
              R.autotune_key(_FakeScene(k=3), cams, R.Config(16, 64), "gfx950"),
              R.autotune_key(_FakeScene(dt=("f32", "f32", "f32")), cams, R.Config(16, 64), "gfx950"),
              R.autotune_key(_FakeScene(lmask=True), cams, R.Config(16, 64), "gfx950"),
              R.autotune_key(_FakeScene(ragged=True), cams, R.Config(16, 64), "gfx950"),
              R.autotune_key(_FakeScene(), cams[:1], R.Config(16, 64), "gfx950"),
              R.autotune_key(_FakeScene(), cams[::-1], R.Config(16, 64), "gfx950"),
              R.autotune_key(_FakeScene(), cams, R.Config(16, 64, flags=1), "gfx950"),
              R.autotune_key(_FakeScene(), cams, R.Config(16, 64), "gfx942")]
    assert len(set(others + [base])) == len(others) + 1


def test_autotune_cache_file_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert R._load_cache(path) == {}
    R._store_cache(path, "a", {"tile": 32, "batch": 64, "waves": 1, "subtile": 8, "ms": 1.5})
    R._store_cache(path, "b", {"tile": 16, "batch": 128, "waves": 4, "subtile": 0, "ms": 2.5})
    d = R._load_cache(path)
    assert d["a"]["tile"] == 32 and d["b"]["waves"] == 4
    with open(path) as f:
        assert set(json.load(f)) == {"a", "b"}
    # a damaged file is ignored rather than trusted
    with open(path, "w") as f:
        f.write("{not json")
    assert R._load_cache(path) == {}
