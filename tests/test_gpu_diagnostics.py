"""Diagnostics of the device path: with RTROM_LOG=3 the library prints a line
when a problem is created, one per time step (sweeps, phase, convergence,
residual, ranks), one per ROM phase change within a march, and one when the
problem is destroyed.  Run in a child process so the level is read fresh."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

CODE = """
from paper_2603_19647_amd import rtrom, workloads as W
s = W.random_slab(3, 64, 8, method='rom', precision='mixed', dt=0.01, tol=1e-10, nsteps=40)
p = rtrom.Problem(s)
for _ in range(4):
    p.march(10)
h = p.history()
st = p.stats()
print('phases', ' '.join(map(str, h['phase'].tolist())))
print('iters', ' '.join(map(str, h['iters'].tolist())))
print('n0n1', st['n0'], st['n1'])
p.close()
"""


def test_log_level_three_traces_a_rom_march():
    print("diagnostics: RTROM_LOG=3 child march", flush=True)
    env = dict(os.environ, RTROM_LOG="3")
    r = subprocess.run([sys.executable, "-c", CODE], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    out = dict(line.split(" ", 1) for line in r.stdout.strip().splitlines())
    phases = list(map(int, out["phases"].split()))
    iters = list(map(int, out["iters"].split()))
    n0, n1 = map(int, out["n0n1"].split())
    err = r.stderr
    m = re.search(r"rtrom: problem (\d+) created: 1D, 64 x 1 cells, 8 ordinates, rom, mixed precision, DSA, BE, FV",
                  err)
    assert m, err[:2000]
    pid = int(m.group(1))
    steps = re.findall(rf"rtrom: problem {pid} step (\d+): (\d+) sweeps, phase (\d+), converged", err)
    assert [int(k) for k, _, _ in steps] == list(range(1, 41))
    assert [int(i) for _, i, _ in steps] == iters
    assert [int(ph) for _, _, ph in steps] == phases
    # a phase change is reported for each march whose last step's phase
    # differs from the previous march's
    changes = re.findall(rf"rtrom: problem {pid}: ROM phase (\d+) -> (\d+) within steps (\d+)\.\.(\d+) "
                         rf"\(N0 (\d+), N1 (\d+)\)", err)
    want = [(phases[a - 2], phases[a + 8], a, a + 9) for a in (11, 21, 31) if phases[a - 2] != phases[a + 8]]
    got = [(int(a), int(b), int(c), int(d)) for a, b, c, d, _, _ in changes if int(c) > 1]
    assert got == want and len(want) >= 1, (changes, phases)
    assert int(changes[-1][4]) == n0 and int(changes[-1][5]) == n1
    assert f"rtrom: problem {pid} destroyed after 40 steps" in err


TUNE_CODE = """
import sys
import numpy as np
from paper_2603_19647_amd import rtrom, workloads as W
s = W.random_plane(3, 40, 8, 4, method='rom', precision='mixed', nsteps=4)
p = rtrom.Problem(s)
p.march(4)
np.save(sys.argv[1], p.rho())
p.close()
"""


def test_tune_cache_file_round_trip(tmp_path):
    """RTROM_TUNE_CACHE: the first process tunes the 2D sweep's prefetch
    depths and the DSA tile for the grid shape and appends them to the file;
    a later process takes the file's choice without tuning, and (neither
    choice changes any cell's arithmetic) reaches bitwise the same result."""
    cache = tmp_path / "tune.txt"
    print("diagnostics: tuning cache, first process", flush=True)
    env = dict(os.environ, RTROM_LOG="2", RTROM_TUNE_CACHE=str(cache))
    for k in ("RTROM_PLANE_PD", "RTROM_TUNE", "RTROM_DSA_TILE"):
        env.pop(k, None)
    a = tmp_path / "a.npy"
    r = subprocess.run([sys.executable, "-c", TUNE_CODE, str(a)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    assert re.search(r"plane 40x40, 16 folded ordinates: SI sweep prefetch depths \d+ \(FP32\) / \d+ \(FP64\), "
                     r"DSA tile (16|32), tuned", r.stderr), r.stderr[-2000:]
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and re.fullmatch(r"plane_tune 40 40 16 (2|4|8|16) (2|4|8|16) (16|32)", lines[0]), lines
    tuned_tile = int(lines[0].split()[-1])
    other = 48 - tuned_tile
    # a cached choice other than the tuned one is taken as it is
    cache.write_text(f"not a cache line\nplane_tune 40 40 16 2 16 {other}\n")
    print("diagnostics: tuning cache, second process", flush=True)
    b = tmp_path / "b.npy"
    r = subprocess.run([sys.executable, "-c", TUNE_CODE, str(b)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    assert f"SI sweep prefetch depths 2 (FP32) / 16 (FP64), DSA tile {other}, cached" in r.stderr, r.stderr[-2000:]
    assert "tuned" not in r.stderr
    assert cache.read_text().splitlines()[-1] == f"plane_tune 40 40 16 2 16 {other}"
    import numpy as np
    np.testing.assert_array_equal(np.load(a), np.load(b))
