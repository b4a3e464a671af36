"""Schedule table (bpm_schedule_set/get/save/load): host logic, no device."""
import pytest

from paper_2601_06340_amd import bpm as B


@pytest.fixture(autouse=True)
def clean_table():
    keys = [("f32", 4096, 0), ("f32", 4096, 1), ("f64", 32768, 2), ("f32", 16384, 1)]
    yield
    for prec, nx, kind in keys:
        B.schedule_set(prec, nx, kind, "default")


def test_set_get_and_strain_classes():
    assert B.schedule_get("f32", 4096, 0) == "default"
    B.schedule_set("f32", 4096, 0, "mixed")
    assert B.schedule_get("f32", 4096, 0) == "mixed"
    assert B.schedule_get("f32", 4096, 1) == "default"      # another strain class
    assert B.schedule_get("f64", 4096, 0) == "default"      # another precision
    B.schedule_set("f64", 32768, 2, "any")
    assert B.schedule_get("f64", 32768, 3) == "any"         # dislocation and table share a class
    B.schedule_set("f32", 4096, 0, "default")
    assert B.schedule_get("f32", 4096, 0) == "default"


def test_save_and_load_round_trip(tmp_path):
    B.schedule_set("f32", 4096, 0, "mixed")
    B.schedule_set("f64", 32768, 2, "any")
    path = tmp_path / "schedules.txt"
    B.schedule_save(path)
    B.schedule_set("f32", 4096, 0, "default")
    B.schedule_set("f64", 32768, 2, "default")
    B.schedule_load(path)
    assert B.schedule_get("f32", 4096, 0) == "mixed"
    assert B.schedule_get("f64", 32768, 2) == "any"
    lines = [l for l in path.read_text().splitlines() if not l.startswith("#")]
    assert sorted(lines) == sorted(["1 12 0 2", "0 15 2 3"])


@pytest.mark.parametrize("prec,nx,kind,sched", [
    ("f32", 32768, 0, "mixed"),    # a staged size: the mixed kernel does not take it
    ("f32", 512, 0, "any"),        # below the any-size kernel's range
    ("f64", 16384, 0, "mixed"),    # FP64 mixed range ends at 8192
    ("f32", 3000, 0, "uniform"),   # not a power of two
    ("f32", 1 << 17, 0, "uniform"),
    ("f32", 4096, 7, "uniform"),   # no such strain kind
])
def test_set_rejects_what_a_family_cannot_march(prec, nx, kind, sched):
    with pytest.raises(B.BpmError):
        B.schedule_set(prec, nx, kind, sched)


def test_get_rejects_bad_keys():
    with pytest.raises(B.BpmError):
        B.schedule_get("f32", 1000, 0)


def test_load_checks_every_line_before_changing_the_table(tmp_path):
    path = tmp_path / "bad.txt"
    path.write_text("# comment\n1 12 0 2\n1 15 0 2\n")   # second entry: mixed at a staged size
    with pytest.raises(B.BpmError):
        B.schedule_load(path)
    assert B.schedule_get("f32", 4096, 0) == "default"
    path.write_text("1 12 0\n")
    with pytest.raises(B.BpmError):
        B.schedule_load(path)
    with pytest.raises(B.BpmError):
        B.schedule_load(tmp_path / "missing.txt")
