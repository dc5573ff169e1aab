"""Write the oracle's state of a seeded subset of the batched sweep's instances after the sweep's
4000 steps, sampled, for the binary32 batch parity test (tests/test_gpu_sweep_parity.py).

    python tests/golden/make_sweep.py            # the sweep's eps 0.05: sweep_c4.npz
    python tests/golden/make_sweep.py 0.02       # the same draws at eps 0.02: sweep_c4_eps0.02.npz
                                                 # (about a minute each on 8 cores)

The instances are drawn from the sweep's own 256 draws (numpy default_rng(2206), see
paper_2206_02145_amd.workloads.sweep_draws): the first instance of every side length and the one
with the largest inflow velocity. Only the oracle (binary64) and the seeded draws are used.
Stored per instance: the crystal extents along 16 directions every 100 steps, and per field (phi,
U, rho, ux, uy) the values on the row y = ny/2 and the column x = nx/2 and at 4096 nodes drawn
with default_rng(22060 + instance index), plus each field's maximum |value| over the whole grid.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2206_02145_amd import workloads as W  # noqa: E402

STEPS, EVERY, N_RANDOM = 4000, 100, 4096


def chosen():
    """Indices into the 256 sweep draws: the first of each side, then the largest inflow velocity."""
    draws = W.sweep_draws(256)
    idx = []
    for side in W.SIDES:
        idx.append(next(i for i, d in enumerate(draws) if d[0] == side))
    fast = int(np.argmax([d[3] for d in draws]))
    if fast not in idx:
        idx.append(fast)
    return idx, draws


def main(eps=None):
    idx, draws = chosen()
    out = {"indices": np.array(idx, dtype=np.int32)}
    dirs = W.directions(16)
    t0 = time.time()
    for i in idx:
        p = W.sweep_instance(*draws[i])
        if eps is not None:
            p["eps"] = eps
        sim = O.Sim(p)
        L = []
        for _ in range(STEPS // EVERY):
            sim.step(EVERY)
            L.append(sim.measure(dirs)[0])
        f = sim.fields()
        nx, ny = p["nx"], p["ny"]
        rng = np.random.default_rng(22060 + i)
        ys = np.concatenate([np.full(nx, ny // 2), np.arange(ny), rng.integers(0, ny, N_RANDOM)])
        xs = np.concatenate([np.arange(nx), np.full(ny, nx // 2), rng.integers(0, nx, N_RANDOM)])
        out[f"{i}_nodes"] = np.stack([ys, xs], 1).astype(np.int32)
        out[f"{i}_L"] = np.array(L)
        for k in ("phi", "U", "rho", "ux", "uy"):
            out[f"{i}_{k}"] = f[k][0, ys, xs]
            out[f"{i}_absmax_{k}"] = np.array(np.abs(f[k]).max())
        print(f"instance {i} {draws[i]}: {time.time() - t0:.0f} s", flush=True)
    out["meta"] = np.array(json.dumps(dict(steps=STEPS, every=EVERY, draws=[list(draws[i]) for i in idx],
                                           eps=W.BASE["eps"] if eps is None else eps,
                                           oracle_threads=O.num_threads(), seconds=round(time.time() - t0, 1))))
    path = os.path.join(HERE, "sweep_c4.npz" if eps is None else f"sweep_c4_eps{eps}.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path}: {os.path.getsize(path) / 1e6:.2f} MB", flush=True)


if __name__ == "__main__":
    main(float(sys.argv[1]) if len(sys.argv) > 1 else None)
