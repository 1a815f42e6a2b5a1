"""CPU checks of bench.py's contract that need no GPU: a request for more
than one GPU is refused with a JSON message and exit status 2 before any
device work, and the committed half-sweep counter summaries were taken on
the kernel sources in the tree (their recorded source hash is the current
one), so that the benchmark's `traffic` field reports them rather than
null."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_halfsweep_counter_summaries_match_the_sources():
    import bench
    khash = bench.kernel_hash()
    for prec in ("f32", "f64"):
        for reals in (18, 12, 8):
            name = f"halfsweep_48x48x48x48_{prec}_{reals}real_pmc.txt"
            traffic = bench.measured_traffic(name, khash)
            assert traffic is not None, name
            # HBM bytes of one half-sweep: within a few percent of the
            # algorithmic 16 links x stored reals per site update
            alg = 16 * reals * (4 if prec == "f32" else 8) * (48 ** 4 // 2)
            assert 0.99 < traffic / alg < 1.05, (name, traffic / alg)
