"""The benchmark's command line and the tuning tables it reads (no device):
more than one GPU is refused with a message, and the tuned launch shapes and
plane paddings are well formed."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_tuning_table_is_well_formed():
    from paper_2510_18688_amd import autotune
    with open(autotune.DB) as f:
        db = json.load(f)
    for key, v in db.items():
        if "tile" in v:
            tx, ty = v["tile"]
            assert tx in (64, 128, 256) and 1 <= ty <= 256, key
        if "pad" in v:
            assert v["pad"] % 64 == 0 and 0 <= v["pad"] <= 65536, key
    # the benchmark's workloads have tuned entries
    assert autotune.lookup(2048, 2048) is not None
    for size in ((2048, 2048), (4096, 2048), (256, 128, 30), (256, 256, 256)):
        assert autotune.lookup_pad(*size) % 64 == 0
    # untuned sizes: no padding, and the nearest 2D size for the tile
    assert autotune.lookup_pad(123, 45) == 0
    assert autotune.lookup_pad(7, 8, 9) == 0
    # state layout (rows per block, pad): tuned, else 4-row blocks without pad
    for size in ((2048, 2048), (4096, 2048)):
        rb, pad = autotune.lookup_layout(*size)
        assert rb in (0, 1, 2, 4, 8, 16, 32) and pad % 64 == 0
    assert autotune.lookup_layout(123, 45) == (1, 0)
    assert autotune.lookup_layout(1000, 45) == (4, 0)
    for size in ((256, 128, 30), (256, 256, 256)):
        rb, pad = autotune.lookup_layout3(*size)
        assert rb in (0, 1, 2, 4, 8, 16, 32, 64) and pad % 64 == 0
    assert autotune.lookup_layout3(7, 8, 9) == (32, 0)
    assert autotune.lookup_strip3(256, 256, 256) in (8, 16, 32, 64)
    assert autotune.lookup_strip3(7, 8, 9) == 16
    assert autotune.lookup(2000, 2000) == autotune.lookup(2048, 2048)
