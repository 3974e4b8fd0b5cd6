"""The committed counter records that bench.py reads: their machine-readable lines
parse, name the headline launch shapes and hold values in range."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _fields(name, tag):
    text = open(os.path.join(ROOT, "profiles", name)).read()
    m = re.search(tag + r" sources_sha256=([0-9a-f]{64}) (.*?)-->", text)
    assert m, f"{name}: no {tag} line"
    return dict(kv.split("=", 1) for kv in m.group(2).split())


def test_traffic_record_parses():
    f = _fields("hbm_traffic_batch128_512.md", "traffic-record")
    assert "forward:1,8,8,1,11" in f and "backprojection:1,64,4,1" in f
    for k, v in f.items():
        direction, shape = k.split(":")
        assert direction in ("forward", "backprojection")
        # variant, images, angles, staging, and for the forward the slab rows
        assert len(shape.split(",")) == (5 if direction == "forward" else 4)
        # at least the algorithmic bytes of one direction (0.40 GB) move per launch
        assert int(v) > 4.0e8


def test_counter_record_parses():
    f = _fields("cache_hit_rates_batch128_512_f32.md", "counter-record")
    assert "forward:1,8,8,1,11" in f and "backprojection:1,64,4,1" in f
    for v in f.values():
        c = {k: float(x) for k, x in (kv.split(":") for kv in v.split(","))}
        assert set(c) == {"l2_hit", "l1_hit", "lds_conflict"}
        assert all(0.0 <= x <= 1.0 for x in c.values())
