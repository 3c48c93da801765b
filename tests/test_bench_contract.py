"""CPU checks of bench.py's command-line contract: one GPU only (larger
--gpus values exit with a message before any GPU work), and the measured
HBM traffic is reported only for the stencil sources it was taken on."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_measurement_options():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--stencil-only", "--stencil27-only", "--c5-only", "--sweep"):
        assert opt in r.stdout


def test_traffic_is_tied_to_the_stencil_sources():
    import bench
    digest = bench.stencil_source_digest()
    assert re.fullmatch(r"[0-9a-f]{64}", digest)
    t = bench.measured_traffic()
    assert t is None or (isinstance(t, int) and t > 0)
    # the committed summary names the digest it was taken on
    text = open(bench.TRAFFIC_FILE).read()
    recorded = re.search(r'"stencil_source_sha256": "([0-9a-f]{64})"', text).group(1)
    assert (t is not None) == (recorded == digest)


def test_host_pool_helpers():
    """The host-side pools: worker count within one GPU's share of the host,
    the uneven-draw members built in spawned workers equal the ones built
    here, and one oracle step on a small grid runs in a worker."""
    import numpy as np
    import bench
    import workloads
    assert 1 <= bench._pool_workers() <= 16
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
    params = [dict(n=(20, 22, 18), freq=5.0, h=37.5, npml=3, seed=11),
              dict(n=(17, 19, 21), freq=6.0, h=31.25, npml=3, seed=12)]
    got = bench.c4_members(params)
    for p, (n, h, npml, vref, omega, src, m32) in zip(params, got):
        w = workloads.c4_problem(p)
        assert n == tuple(w.n) and h == w.h and npml == w.npml and omega == w.omega
        assert src == tuple(int(v) for v in w.src[0])
        assert np.array_equal(m32, w.m.astype(np.float32))
    w = workloads.c4_problem(params[0])
    dt, setup = bench._oracle_step((tuple(w.n), w.h, w.npml, w.omega, w.v_ref, w.m, tuple(w.src[0])))
    assert dt > 0 and setup > 0
