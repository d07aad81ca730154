"""Host logic of the intersection-threshold autotuner (no GPU): the coordinate descent,
the validity rule, the cache keys and the cache file."""
import pytest

from paper_2403_02997_amd import autotune as at


def test_valid_matches_the_library_range():
    assert at.valid((16, 512, 4096, 1024))
    assert not at.valid((32, 16, 4096, 1024))   # lane_max > wave_max
    assert not at.valid((16, 1024, 4096, 1024))  # wave_max > 512
    assert not at.valid((16, 512, 0, 1024))
    assert not at.valid((16, 512, 32768, 1024))
    assert not at.valid((16, 512, 4096, 2048))


def test_descent_reaches_the_best_grid_point_of_a_separable_cost():
    target = (8, 256, 8192, 512)
    seen = []

    def measure(p):
        seen.append(p)
        return 42, sum(abs(a - b) / b for a, b in zip(p, target))

    best, t, n = at.descend(measure, (16, 512, 4096, 1024))
    assert best == target and t == 0
    assert n == len(seen) == len(set(seen))          # each setting measured once
    assert all(at.valid(p) for p in seen)


def test_descent_tunes_the_hub_count_when_given():
    seen = []

    def measure(p):
        seen.append(p)
        return 0, abs(p[4] - 128) + 0.001 * p[0]

    best, _, _ = at.descend(measure, (16, 512, 4096, 1024, 256))
    assert best[4] == 128 and all(len(p) == 5 for p in seen)
    assert {p[4] for p in seen} == set(at.CANDIDATES["max_hubs"])
    assert not at.valid((16, 512, 4096, 1024, 257))


def test_descent_keeps_the_start_against_noise_sized_gains():
    def measure(p):  # every other setting 1 % faster: within the margin
        return 0, 1.0 if p == (16, 512, 4096, 1024) else 0.99

    best, t, _ = at.descend(measure, (16, 512, 4096, 1024))
    assert best == (16, 512, 4096, 1024) and t == 1.0


def test_descent_never_measures_an_invalid_setting():
    seen = []

    def measure(p):
        seen.append(p)
        return 0, 1.0

    at.descend(measure, (32, 128, 4096, 1024))
    assert all(p[0] <= p[1] for p in seen)


def test_descent_rejects_a_setting_that_changes_the_result():
    def measure(p):
        return (7 if p[2] != 2048 else 8), 1.0

    with pytest.raises(RuntimeError):
        at.descend(measure, (16, 512, 4096, 1024))


def test_workload_key_groups_by_size_class():
    assert at.workload_key("single", 4194304, 128308020) == at.workload_key("single", 4194305,
                                                                             130000000)
    assert at.workload_key("single", 1024, 20000) != at.workload_key("batch", 1024, 20000, 16)
    assert at.workload_key("single", 0, 0) == "single:g0:n-1:m-1"


def test_cache_file_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "autotune.json")
    assert at.load_cache(path) == {}
    at.store_cache(path, {"k": {"params": [8, 256, 4096, 512], "ms": 1.5}})
    assert at.load_cache(path) == {"k": {"params": [8, 256, 4096, 512], "ms": 1.5}}
    (tmp_path / "bad.json").write_text("not json")
    assert at.load_cache(str(tmp_path / "bad.json")) == {}
