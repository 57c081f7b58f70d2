"""Random batches that mix every operation kind, on small contended tables.

Each case runs ``workload.mixed_workload`` (two tables of 40 x 3 and 300 x 5
cells, Zipf 0.8, reads, adds, conditional adds and slot writes in row groups
of 1-3 fields) under one scheme and one team width.  The width chooses the
kernel variant: L=1 with up to 16 operations (16 register slots per lane),
L=4 with up to 64 (16 slots), L=16 with up to 64 (4 slots), L=64 with up to
256 (4 slots).  The ticketed schemes are checked by the oracle's serial
replay in the reported order. GaccO, GaccO with shared reads, and GPUTx are
compared element by element with the id-order replay.
"""
import numpy as np
import pytest

import oracle
from helpers import SCHEMES, binding, run_and_check, run_batch
from paper_2406_10158_amd import workload as wl

pytestmark = pytest.mark.gpu

DETERMINISTIC = ["gacco", "gacco_shared", "gputx"]
WIDTHS = {1: ((1, 16), 1_500), 4: ((1, 64), 600), 16: ((1, 64), 600), 64: ((1, 256), 200)}


@pytest.fixture(scope="module", autouse=True)
def _announce(request):
    print(f"\n[gpu] module {request.module.__name__}", flush=True)


def _run(scheme, lanes, seed, **params):
    ops, n = WIDTHS[lanes]
    tabs, b = wl.mixed_workload(n_txns=n, ops=ops, theta=0.8, seed=seed)
    print(f"[gpu] mixed {scheme} L={lanes} seed={seed} params={params}", flush=True)
    if scheme in DETERMINISTIC:
        b_ = binding()
        flags = params.pop("flags", 0) | (b_.CC_RUN_SHARED_READS if scheme == "gacco_shared" else 0)
        out, reads, final, st = run_batch(tabs, b, "gputx" if scheme == "gputx" else "gacco",
                                          lanes_per_txn=lanes, flags=flags, **params)
        assert "error" not in st, st["error"]
        assert np.all(out["status"] == oracle.COMMITTED)
        exp_fin, exp_reads = oracle.id_order_expected(tabs, b)
        bad = np.nonzero(np.asarray(reads, np.int64) != exp_reads)[0]
        assert len(bad) == 0, f"{len(bad)} read values differ, first ops {bad[:5].tolist()}"
        for t, (g, e) in enumerate(zip(final, exp_fin)):
            assert np.array_equal(np.asarray(g, np.int64), e), f"table {t} differs"
    else:
        run_and_check(tabs, b, scheme, lanes_per_txn=lanes, **params)
    return b


@pytest.mark.parametrize("lanes", sorted(WIDTHS))
@pytest.mark.parametrize("scheme", SCHEMES + DETERMINISTIC)
def test_mixed_kinds(scheme, lanes):
    b = _run(scheme, lanes, seed=1000 + 10 * lanes + (SCHEMES + DETERMINISTIC).index(scheme))
    assert b.n_ops.max() > WIDTHS[lanes][0][1] // 2  # the wide variants really were needed


@pytest.mark.parametrize("scheme", SCHEMES)
def test_mixed_kinds_latch_and_strict(scheme):
    b_ = binding()
    _run(scheme, 16, seed=2000, flags=b_.CC_RUN_LATCH)
    _run(scheme, 4, seed=2001, flags=b_.CC_RUN_STRICT_FENCES, waves_per_wg=4)


@pytest.mark.parametrize("scheme", ["occ", "tictoc", "gacco"])
def test_mixed_kinds_more_seeds(scheme):
    for seed in range(3000, 3004):
        _run(scheme, 16, seed=seed)


@pytest.mark.parametrize("scheme", SCHEMES + DETERMINISTIC)
def test_mixed_kinds_sixteen_tables_and_256_fields(scheme):
    # the table and field limits: 16 tables, one of them 256 fields wide
    shapes = tuple((int(r), int(f)) for r, f in zip((5, 9, 17, 33, 64, 100, 7, 300, 50, 2, 400, 13, 80, 3, 256, 60),
                                                   (1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 1, 2, 3, 256, 4, 5)))
    tabs, b = wl.mixed_workload(shapes=shapes, n_txns=1_000, ops=(1, 16), theta=0.8, seed=4000)
    assert len(tabs) == 16 and int(b.table.max()) == 15
    wide = b.table == 13
    assert wide.any() and int(b.field[wide].max()) > 200
    print(f"[gpu] mixed 16 tables {scheme}", flush=True)
    if scheme in DETERMINISTIC:
        b_ = binding()
        flags = b_.CC_RUN_SHARED_READS if scheme == "gacco_shared" else 0
        out, reads, final, st = run_batch(tabs, b, "gputx" if scheme == "gputx" else "gacco", flags=flags)
        assert "error" not in st, st["error"]
        exp_fin, exp_reads = oracle.id_order_expected(tabs, b)
        assert np.array_equal(np.asarray(reads, np.int64), exp_reads)
        assert all(np.array_equal(np.asarray(g, np.int64), x) for g, x in zip(final, exp_fin))
    else:
        run_and_check(tabs, b, scheme)
