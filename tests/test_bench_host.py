"""Host logic of bench.py (no GPU): the digest that keys the committed
traffic counters to the kernel sources, and the single-GPU contract."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_text_drops_comments_and_keeps_literals():
    src = ('int a = 1; // one\n/* two\n lines */ int b = 2;\n'
           'const char *s = "// not a comment"; char q = \'"\'; char e = \'\\\'\';\n')
    assert bench.code_text(src) == ('int a = 1; int b = 2; const char *s = "// not a comment"; '
                                    'char q = \'"\'; char e = \'\\\'\';')


def test_digest_follows_code_not_comments():
    csrc = os.path.join(ROOT, "paper_2305_07545_amd", "csrc")
    for name in bench.KERNEL_SOURCES:
        src = open(os.path.join(csrc, name), encoding="utf-8").read()
        text = bench.code_text(src)
        assert text, name
        assert bench.code_text(src + "\n// a note\n/* another */\n") == text
        assert bench.code_text(src.replace("\n", "\n  ")) == text  # indentation
        assert bench.code_text(src + "\nint x;\n") != text


def test_traffic_records_name_their_sources():
    for w in ("large", "bacterial", "batched"):
        rec = json.load(open(os.path.join(ROOT, "profiles", f"traffic_{w}.json")))
        assert len(rec["source_sha256"]) == 64
        assert rec["phases"] and all(p["bytes_per_launch"] > 0 for p in rec["phases"].values())


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "--gpus must be 1" in r.stdout
