"""CPU checks of host-side pieces: seeded generators and the bench contract."""
import os
import subprocess
import sys

import numpy as np

from paper_2604_15796_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_generators_are_seeded_and_shaped():
    a, b = W.config1(), W.config1()
    assert np.array_equal(a.c, b.c) and np.array_equal(a.extra["c_obs"], b.extra["c_obs"])
    assert a.c.shape == (256, 256) and a.nf == 8 and a.ne == 64
    assert np.all((a.c >= 1480) & (a.c <= 1600)) and np.all(a.alpha >= 0)
    # elements on the top face, centred, at 0.3 mm pitch
    assert np.allclose(a.elems[:, 2], 0) and np.allclose(np.diff(a.elems[:, 0]), 0.3e-3)
    assert abs(a.elems[:, 0].mean() - a.nx * a.dx / 2) < 1e-12
    p3 = W.config3()
    assert p3.c.shape == (384, 384) and p3.nf == 12 and p3.ne == 128
    assert set(np.unique(p3.c)) == {1500.0, 1540.0, 1580.0}
    p4 = W.config4()
    assert p4.c.shape == (96, 128, 128) and p4.dim == 3 and np.allclose(p4.elems[:, 1], p4.ny * p4.dx / 2)
    insts = W.config2()
    assert len(insts) == 32 and {p.nx for p in insts} <= {128, 192, 256, 384, 512}
    assert all(32 <= p.ne <= 128 and 1 <= p.nf <= 4 for p in insts)
    assert all(np.all(np.diff(p.freqs) >= 0) for p in insts)
    # compressed pitch keeps the aperture within 90% of the width
    for p in insts:
        assert p.elems[:, 0].max() - p.elems[:, 0].min() <= 0.9 * p.nx * p.dx


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
