"""Shared helpers for the engine tests: run a batch through the C-ABI and check it with the oracle."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402

SCHEMES = ["occ", "2pl_nw", "to", "mvcc", "tictoc", "2pl_wd"]


def binding():
    """The C-ABI binding; a missing library is an error, never a skip."""
    from paper_2406_10158_amd import binding as b
    return b


def run_batch(tables, batch, scheme="occ", engine=None, **params):
    """Run ``batch`` on fresh copies of ``tables``; returns (outcomes, reads, final_tables, stats)."""
    b = binding()
    own = engine is None
    eng = b.Engine(tables) if own else engine
    if not own:
        eng.load(tables)
    try:
        bid = eng.submit(batch, scheme)
        err = None
        try:
            stats = eng.run(bid, **params)
        except b.CCError as e:
            err = e
            stats = b.cc_stats(eng.ctx, bid)
        out, reads = eng.outcomes(bid, batch.n_txns, batch.total_ops)
        final = eng.tables()
        eng.release(bid)
    finally:
        if own:
            eng.close()
    if err is not None:
        stats["error"] = err
    return out, reads, final, stats


def check(tables, batch, out, reads, final, require_all_committed=True):
    return oracle.check_run(tables, batch, out["status"], out["serial_hi"], out["serial_lo"], reads, final,
                            require_all_committed=require_all_committed)


def run_and_check(tables, batch, scheme="occ", engine=None, **params):
    out, reads, final, stats = run_batch(tables, batch, scheme, engine, **params)
    assert "error" not in stats, stats["error"]
    rep = check(tables, batch, out, reads, final)
    assert rep.ok, f"{scheme} {params}: {rep}"
    assert stats["committed"] == batch.n_txns
    assert stats["attempts"] == int(out["attempts"].astype(np.int64).sum())
    return out, reads, final, stats
