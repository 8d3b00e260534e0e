"""The tuner's cache file (PCOP_TUNE_CACHE): a tuned context appends its
choice, a later process reads it back instead of tuning, and an entry that
does not fit the context (here a block count beyond the partial-sum buffer)
is ignored and the shape tuned afresh.  Each step runs in a child process,
since the choices are also cached inside a process."""
import json
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHILD = """
import json, sys
sys.path.insert(0, {root!r})
from paper_2410_22686_amd import Solver
s = Solver(2, 15, 16, [1e-4, 1e-6], tune=True, device="cuda:0")
print("KERNELS " + json.dumps(s.kernels), flush=True)
"""


def child(cache):
    env = dict(os.environ, PCOP_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [l for l in r.stdout.splitlines() if l.startswith("KERNELS ")][-1]
    return json.loads(line[len("KERNELS "):])


def lines(cache):
    return [l.split() for l in open(cache).read().splitlines() if l.startswith("pcop-tune ")]


def test_tune_cache_roundtrip(tmp_path):
    cache = tmp_path / "tune.txt"
    k1 = child(cache)
    rows = lines(cache)
    assert len(rows) == 1, rows
    row = rows[0]
    # pcop-tune <version> <device> <14 key ints> <time_cols> <dst_variant> <jchunk> <ms> <3 x 41 ints>
    assert len(row) == 3 + 14 + 4 + 3 * 41, len(row)
    assert row[2].startswith("gfx"), row[2]
    assert int(row[19]) == k1["kkt_jchunk"] and abs(float(row[20]) - k1["tuned_ms"]) <= 1e-5 * k1["tuned_ms"]
    # a process reading an edited entry takes the file's choice without tuning
    row[19] = "3"            # matvec: one thread per point marching 3 levels
    row[20] = "0.123456"     # the recorded apply time
    cache.write_text(" ".join(row) + "\n")
    k2 = child(cache)
    assert k2["kkt_jchunk"] == 3 and abs(k2["tuned_ms"] - 0.123456) < 1e-9, k2
    assert len(lines(cache)) == 1  # nothing tuned, nothing appended
    # an entry whose multi-dot block count exceeds the context's buffer is
    # ignored: the shape is tuned again and a new line appended
    row[21] = "100000"
    cache.write_text(" ".join(row) + "\n")
    k3 = child(cache)
    assert len(lines(cache)) == 2
    assert abs(k3["tuned_ms"] - 0.123456) > 1e-9
