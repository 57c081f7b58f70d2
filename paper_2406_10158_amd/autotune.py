"""Autotuner for the engine's launch shape.

The paper tunes two launch parameters by grid search -- working threads per
warp and warps per block -- and finds the best point moves with contention
(Section 4.2, Exp-3 to Exp-5 and Insight 2).  On gfx950 the analogous knobs
are lanes per transaction (1, 4, 16, 64), wavefronts per workgroup (1..16),
the number of workgroups and the run mode (plain in-kernel retry, or
graph-replayed epochs).  ``tune`` measures each feasible point on the real
batch and returns the fastest; ``TuneCache`` keeps the winners in a JSON file
keyed by workload, contention and batch size.
"""
from __future__ import annotations

import json
import os
import time

from . import binding as b

LANES = (1, 4, 16, 64)
WAVES = (1, 2, 4, 8, 16)
MODES = (("plain", b.CC_MODE_PLAIN), ("epoch", b.CC_MODE_EPOCH))


def candidates(lanes=LANES, waves=WAVES, modes=MODES, grids=(0,), epoch_attempts=(1, 8)):
    """Launch points to try; epoch mode also varies the attempts each transaction gets per epoch."""
    for mname, mode in modes:
        for L in lanes:
            for W in waves:
                for G in grids:
                    for d in (epoch_attempts if mode == b.CC_MODE_EPOCH else (0,)):
                        yield {"mode_name": mname, "mode": mode, "lanes_per_txn": L, "waves_per_wg": W, "grid": G,
                               "defer_after": d}


def tune(engine, batch_id: int, n_txns: int, points=None, repeats: int = 1, reset=None, log=None):
    """Run every launch point on the submitted batch; returns (best, results).

    ``reset`` (optional) is called before each run to restore the tables.
    A point the library rejects (register slots or workgroup size not
    available for that lanes-per-transaction) is recorded as infeasible.
    """
    results = []
    for pt in (points if points is not None else candidates()):
        params = {k: v for k, v in pt.items() if k != "mode_name"}
        times = []
        err = None
        for _ in range(repeats):
            if reset is not None:
                reset()
            try:
                st = engine.run(batch_id, **params)
            except b.CCError as e:
                err = e
                break
            times.append(st["run_ns"])
        rec = dict(pt)
        if err is not None:
            rec.update(feasible=False, error=str(err))
        else:
            t = min(times)
            rec.update(feasible=True, run_ms=t / 1e6, txn_per_s=n_txns / (t * 1e-9), attempts=st["attempts"],
                       epochs=st["epochs"], passes=st["passes"], p99_ms=st["lat_p99_ns"] / 1e6)
        results.append(rec)
        if log:
            log(rec)
    ok = [r for r in results if r["feasible"]]
    best = max(ok, key=lambda r: r["txn_per_s"]) if ok else None
    return best, results


class TuneCache:
    """Winning launch points, keyed by (workload, contention, batch size, scheme)."""

    def __init__(self, path: str):
        self.path = path
        self.data = {}
        if os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    @staticmethod
    def key(workload: str, theta: float, n_txns: int, scheme: str) -> str:
        return f"{workload}|theta={theta}|txns={n_txns}|{scheme}"

    def get(self, key: str):
        return self.data.get(key)

    def put(self, key: str, best: dict):
        self.data[key] = dict(best, tuned_at=time.strftime("%Y-%m-%d %H:%M:%S"))

    def save(self):
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
