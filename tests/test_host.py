"""Host-side logic that needs no GPU: the schedule cache and the bench's
command-line contract."""
import json
import os
import subprocess
import sys

from paper_1907_07774_amd import autotune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_schedule_cache_key_classes():
    assert autotune.key("gfx950", 256, "fp32", 1) == "gfx950/n256/fp32/b1"
    assert autotune.key("gfx950", 64, "fp64", 5) == "gfx950/n64/fp64/b8"
    assert autotune.key("gfx950", 128, "fp32", 48) == "gfx950/n128/fp32/b64"


def test_schedule_cache_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "sched.json"
    monkeypatch.setenv("TUMORGRAD_SCHEDULES", str(path))
    assert autotune.lookup("gfx950", 256, "fp32", 1) is None  # no file yet
    autotune.store({autotune.key("gfx950", 256, "fp32", 1): {
        "pencils": 32, "z_waves": 2, "slabs": 1, "waves_per_simd": 1, "ms": 1.0,
        "passes": {"x_fwd_div": [16, 1], "z_matvec": [0, 4]}}})
    autotune.store({autotune.key("gfx950", 64, "fp64", 1): {
        "pencils": 16, "z_waves": 1}})  # older entry without slabs/occupancy/passes
    sch, passes = autotune.lookup("gfx950", 256, "fp32", 1)
    assert sch == (32, 2, 1, 1)
    assert passes == {"x_fwd_div": (16, 1), "z_matvec": (0, 4)}
    assert autotune.lookup("gfx950", 64, "fp64", 1) == ((16, 1, 1, 1), {})
    assert autotune.lookup("gfx942", 256, "fp32", 1) is None
    tab = json.loads(path.read_text())
    assert len(tab) == 2  # store merges
    path.write_text("not json")
    assert autotune.lookup("gfx950", 256, "fp32", 1) is None  # unreadable cache ignored


def test_shipped_schedule_cache_is_valid():
    tab = autotune.load(autotune.DEFAULT_CACHE)
    assert tab
    for k, ent in tab.items():
        arch, n, prec, b = k.split("/")
        assert prec in ("fp32", "fp64") and b in ("b1", "b8", "b64")
        assert ent["pencils"] in autotune.PENCILS
        assert ent["z_waves"] in autotune.Z_WAVES
        assert ent.get("slabs", 1) in autotune.SLABS
        assert ent.get("waves_per_simd", 1) in autotune.OCCUPANCY
        for name, (c, o) in ent.get("passes", {}).items():
            assert name in autotune.PASSES and o in autotune.OCCUPANCY
            assert c in (0, 8, 16) if name == "z_matvec" else c in autotune.PENCILS


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


class _FakePlan:
    """Stands in for api.Plan in the schedule search: passes as a dict, and
    the wide z matvec (z_waves 8) accepting only its own shape, as the
    library does."""

    def __init__(self, zw):
        self.zw = zw
        self.passes = {k: (32, 1) for k in autotune.PASSES}
        self.passes["z_matvec"] = (8, 1)

    def get_schedule(self):
        return (32, self.zw, 1, 1)

    def get_pass(self, k):
        return self.passes[k]

    def set_pass(self, k, c, o):
        if k == "z_matvec" and self.zw == 8 and (c, o) != self.passes[k]:
            raise RuntimeError("the wide z matvec has no per-pass variant")
        self.passes[k] = (c, o)


def test_pass_search_with_and_without_the_wide_z_matvec(monkeypatch):
    # forward time: 100 ms, 5 less with x_inv_grad at (16, 4), 2 less with
    # the z matvec in pairs
    def fake_time(plan, args, reps):
        return (100.0 - (5.0 if plan.passes["x_inv_grad"] == (16, 4) else 0.0)
                - (2.0 if plan.passes["z_matvec"] == (16, 1) else 0.0))
    monkeypatch.setattr(autotune, "_median_forward", fake_time)
    for zw in (2, 8):
        plan = _FakePlan(zw)
        passes, before, after = autotune.tune_passes(plan, None, None, None, None)
        assert before == 100.0
        assert passes["x_inv_grad"] == (16, 4)
        if zw == 8:
            assert "z_matvec" not in passes and after == 95.0
            assert plan.passes["z_matvec"] == (8, 1)
        else:
            assert passes["z_matvec"] == (16, 1) and after == 93.0
