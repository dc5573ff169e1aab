"""The batch autotuner: every tiling of the batched step gives each instance the state of a single
grid run with the same tiling (bit for bit), timing a tiling runs real steps, and the tuned choice
is cached so that a later batch of the same mix of shapes starts on it."""
import numpy as np
import pytest

from paper_2206_02145_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2206_02145_amd import lbcg
    lbcg.lib()
    lbcg.tune_cache_clear()
    yield lbcg
    lbcg.tune_cache_clear()


def plist_2d():
    draws = W.sweep_draws(4, seed=3)
    sides = (64, 96, 128, 72)  # 72: a row shorter than two 64-wide tiles
    return [W.sweep_instance(sd, *d[1:]) for sd, d in zip(sides, draws)]


def plist_3d():
    return [W.scaled(W.config3(), 70, 20, 18, seed_R=5.0), W.scaled(W.config3(), 64, 24, 16, seed_R=6.0)]


@pytest.mark.parametrize("dim,prec", [(2, "fp32"), (2, "fp64"), (2, "fp16shift"), (3, "fp32"), (3, "fp64")])
def test_every_batch_tiling_matches_single_grids(lb, dim, prec):
    plist = plist_2d() if dim == 2 else plist_3d()
    b0 = lb.Batch(plist, prec)
    names = b0.variants()
    b0.close()
    print(f"[tuning] batch tilings dim {dim} {prec}: {names}", flush=True)
    assert len(names) >= 2
    fields = ("raw_h", "raw_g", "raw_f", "phi_prev")
    for k, name in enumerate(names):
        b = lb.Batch(plist, prec)
        b.select_variant(k)
        assert b.variant == k
        b.run(30)
        for i, p in enumerate(plist):
            s = lb.Solver(p, prec)
            s.select_variant(s.variants().index(name))
            s.step(30)
            for f in fields:
                dt = np.float64 if prec == "fp64" else np.float32
                assert np.array_equal(s.read(f, dt), b.read(i, f, dt)), (name, i, f)
            s.close()
        b.close()


def test_batch_variant_timer_runs_real_steps_and_tuning_is_cached(lb):
    lb.tune_cache_clear()
    plist = plist_2d()
    a, c = lb.Batch(plist, "fp32"), lb.Batch(plist, "fp32")
    k = len(a.variants()) - 1
    a.run(3)
    us = a.time_variant(k, 4)
    assert us > 0 and a.nstep == 8 and a.variant == 0
    c.run(3)
    c.select_variant(k)
    c.run(5, use_graph=False)
    for i in range(len(plist)):
        for f in ("raw_h", "raw_g", "raw_f", "phi_prev"):
            assert np.array_equal(a.read(i, f, np.float32), c.read(i, f, np.float32)), (i, f)
    best, best_us, all_us = a.autotune(3)
    assert a.variant == best and best_us > 0 and best_us == all_us.min() and len(all_us) == len(a.variants())
    assert a.nstep == 8 + 2 * 4 * len(a.variants())  # two timing rounds of launches + 1 steps
    # a new batch with the same mix of shapes starts on the tuned tiling; another mix does not
    d = lb.Batch(plist, "fp32")
    assert d.variant == best
    e = lb.Batch(plist[:2], "fp32")
    assert e.variant == 0
    # graph replay after a selection uses the new tiling
    d.select_variant(0)
    d.run(20, use_graph=True)
    f = lb.Batch(plist, "fp32")
    f.select_variant(0)
    f.run(20, use_graph=False)
    for i in range(len(plist)):
        assert np.array_equal(d.read(i, "raw_f", np.float32), f.read(i, "raw_f", np.float32))
    for x in (a, c, d, e, f):
        x.close()
    lb.tune_cache_clear()
    g = lb.Batch(plist, "fp32")
    assert g.variant == 0
    g.close()


def test_tuning_cache_file_carries_the_choice_to_another_process(lb, tmp_path):
    """With LBCG_TUNE_CACHE naming a file, a choice made in one process is read back by the next:
    its first batch of the same mix of shapes starts on the tuned tiling."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    prog = (
        "import sys; sys.path.insert(0, {root!r})\n"
        "from paper_2206_02145_amd import lbcg, workloads as W\n"
        "draws = W.sweep_draws(3, seed=3)\n"
        "b = lbcg.Batch([W.sweep_instance(96, *d[1:]) for d in draws], 'fp32')\n"
        "if sys.argv[1] == 'tune':\n"
        "    best, us, _ = b.autotune(2)\n"
        "    print('CHOICE', b.variants()[best])\n"
        "else:\n"
        "    print('CHOICE', b.variants()[b.variant])\n"
        "b.close()\n").format(root=root)
    env = dict(os.environ, LBCG_TUNE_CACHE=str(cache))
    out = []
    for mode in ("tune", "use"):
        r = subprocess.run([sys.executable, "-c", prog, mode], env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        out.append([l for l in r.stdout.splitlines() if l.startswith("CHOICE")][-1])
    print("[tuning]", out, cache.read_text().strip(), flush=True)
    assert out[0] == out[1]
    assert "batch gfx" in cache.read_text() and out[0].split(" ", 1)[1] in cache.read_text()
