"""The batch autotuner's persistent cache (host only: no GPU).

rt_tune_cache_put / rt_tune_cache_get through the C ABI, the JSON file they
share with other processes, and the file's tolerance of damage.  The GPU
side (rt_batch_create storing what it timed, and a second batch of the same
signature taking the stored shape) is in tests/test_gpu_batch.py.
"""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def rt(tmp_path, monkeypatch):
    import paper_2305_07450_amd as rt
    path = tmp_path / "tune.json"
    monkeypatch.setenv("RT_TUNE_CACHE", str(path))
    rt.rt_tune_cache_forget()
    yield rt
    rt.rt_tune_cache_forget()


def _path():
    return os.environ["RT_TUNE_CACHE"]


def test_put_then_get_in_memory_and_from_the_file(rt):
    key = "gfx950:256cu:2:64x36d2n8l1:1920x1080d4n64l2s"
    assert rt.rt_tune_cache_get(key) is None
    rt.rt_tune_cache_put(key, 2048, 16, 16)
    assert rt.rt_tune_cache_get(key) == (2048, 16, 16)
    rt.rt_tune_cache_forget()
    assert rt.rt_tune_cache_get(key) == (2048, 16, 16)   # read back from the file
    doc = json.load(open(_path()))
    assert doc["format"] == "rtmi-tune-cache-1"
    assert list(doc["entries"].values()) == [{"workgroups": 2048, "wave_w": 16, "waves": 4}]


def test_another_process_reads_the_stored_shape(rt):
    keys = {f"gfx950:256cu:1:{w}x{h}d1n4l1": (512 * (i + 1), tw, th)
            for i, (w, h, tw, th) in enumerate([(320, 180, 8, 8), (640, 360, 64, 2),
                                                 (1280, 720, 16, 8)])}
    for k, s in keys.items():
        rt.rt_tune_cache_put(k, *s)
    code = ("import json, sys, paper_2305_07450_amd as rt; "
            "keys = json.loads(sys.argv[1]); "
            "print(json.dumps({k: rt.rt_tune_cache_get(k) for k in keys}))")
    out = subprocess.run([sys.executable, "-c", code, json.dumps(list(keys))], cwd=ROOT,
                         env=dict(os.environ), capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    got = json.loads(out.stdout.strip().splitlines()[-1])
    assert {k: tuple(v) for k, v in got.items()} == keys


def test_keys_are_distinct_and_a_miss_stays_a_miss(rt):
    rt.rt_tune_cache_put("a", 256, 8, 8)
    rt.rt_tune_cache_put("b", 1024, 64, 4)
    rt.rt_tune_cache_forget()
    assert rt.rt_tune_cache_get("a") == (256, 8, 8)
    assert rt.rt_tune_cache_get("b") == (1024, 64, 4)
    assert rt.rt_tune_cache_get("ab") is None
    rt.rt_tune_cache_put("a", 512, 16, 4)   # replaced
    rt.rt_tune_cache_forget()
    assert rt.rt_tune_cache_get("a") == (512, 16, 4)
    assert len(json.load(open(_path()))["entries"]) == 2


@pytest.mark.parametrize("shape", [(0, 8, 8), (2 ** 20 + 1, 8, 8), (256, 32, 2), (256, 8, 4),
                                   (256, 16, 32), (256, 64, 3), (-5, 16, 4)])
def test_shapes_the_tuner_cannot_pick_are_refused(rt, shape):
    with pytest.raises(rt.RtError) as e:
        rt.rt_tune_cache_put("k", *shape)
    assert e.value.status == rt.RT_ERR_INVALID_ARG
    assert rt.rt_tune_cache_get("k") is None
    assert not os.path.exists(_path())


def test_a_damaged_file_is_ignored_and_rewritten(rt):
    with open(_path(), "w") as f:
        f.write('{"format": "rtmi-tune-cache-1", "entries": {\n'
                ' "00000000000000aa:1": {"workgroups": 999, "wave_w": 12, "waves": 4},\n'
                ' garbage line\n'
                ' "not a digest": {"workgroups": 1, "wave_w": 8, "waves": 1}\n')
    assert rt.rt_tune_cache_get("a") is None
    rt.rt_tune_cache_put("a", 256, 8, 8)
    doc = json.load(open(_path()))
    assert list(doc["entries"].values()) == [{"workgroups": 256, "wave_w": 8, "waves": 1}]
    with open(_path(), "w") as f:
        f.write("not json at all\n")
    rt.rt_tune_cache_forget()
    assert rt.rt_tune_cache_get("a") is None


def test_empty_path_keeps_the_cache_in_memory(rt, monkeypatch, tmp_path):
    monkeypatch.setenv("RT_TUNE_CACHE", "")
    rt.rt_tune_cache_put("m", 256, 8, 8)
    assert rt.rt_tune_cache_get("m") == (256, 8, 8)
    rt.rt_tune_cache_forget()
    assert rt.rt_tune_cache_get("m") is None
    assert list(tmp_path.iterdir()) == []


def test_missing_directories_are_created(rt, monkeypatch, tmp_path):
    path = tmp_path / "x" / "y" / "tune.json"
    monkeypatch.setenv("RT_TUNE_CACHE", str(path))
    rt.rt_tune_cache_put("d", 512, 64, 1)
    assert json.load(open(path))["entries"]
