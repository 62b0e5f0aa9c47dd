"""The benchmark measures one GPU: asking for more exits at once with a message saying so (no GPU
needed; the check runs before anything touches a device)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "--gpus 2" in r.stderr and "one GPU" in r.stderr
    assert r.stdout == ""


def test_morton_order_of_the_query_record():
    """The query record's coherent order: points sorted by the Morton code of their cell, the code
    interleaving the bits of x, y, z (x lowest), checked against the interleave written bit by bit."""
    import numpy as np

    sys.path.insert(0, ROOT)
    import bench

    rng = np.random.default_rng(7)
    p = rng.uniform(-3.0, 5.0, size=(2000, 3))
    perm = bench.morton_order(np, p, 0.01)
    assert sorted(perm.tolist()) == list(range(len(p)))
    c = np.floor((p - p.min(axis=0)) / 0.01).astype(np.int64)

    def code(x, y, z):
        r = 0
        for b in range(21):
            r |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
        return r

    codes = [code(*map(int, row)) for row in c]
    assert [codes[i] for i in perm] == sorted(codes)
    # neighbouring cells of one 2x2x2 cube are consecutive codes
    assert code(0, 0, 0) + 1 == code(1, 0, 0) and code(1, 1, 1) == 7
