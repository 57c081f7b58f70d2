"""Batches submitted from device memory (cc_submit_batch / cc_submit_batch_keyed with on_device = 1).

The library validates and packs the caller's device arrays with its ingest
kernels.  Checked here, in a child process that initialises torch first (see
test_gpu_device_buffers.py for why):
* runs of device-submitted batches pass the oracle's replay (OCC, MVCC,
  GaccO's id-order execution, a keyed batch), and equal the host-submitted
  batch's run where the outcome is unique (one team, or GaccO);
* every malformed batch of the host-only validation cases gets the status
  cc_check_batch gives for it on the host;
* arrays that are not device memory of the context's device, or shorter than
  the counts say, are refused with CC_E_INVAL before any kernel reads them.
"""
import subprocess
import sys

import pytest

from helpers import ROOT

pytestmark = pytest.mark.gpu

CHILD = r'''
import sys
import torch
torch.cuda.init()
sys.path.insert(0, ROOT)
sys.path.insert(0, ROOT + "/tests")
import numpy as np
from paper_2406_10158_amd import binding as B, workload as wl
import oracle
from test_abi import CHECK_CASES, SHAPES, _batch

def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.uint8)).to("cuda")

print("[child] kv batch, device-submitted, occ / mvcc / gacco", flush=True)
tabs, b = wl.kv_workload(n_rows=20_000, n_fields=4, n_txns=20_000, ops=(1, 24), theta=0.9, seed=61)
with B.Engine(tabs) as eng:
    for scheme in ("occ", "mvcc", "gacco"):
        eng.load(tabs)
        bid = eng.submit_device(b, scheme)
        eng.run(bid)
        out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
        fin = eng.tables()
        if scheme == "gacco":
            exp_fin, exp_reads = oracle.id_order_expected(tabs, b)
            assert np.array_equal(reads, exp_reads) and np.array_equal(fin[0], exp_fin[0]), scheme
        rep = oracle.check_run(tabs, b, out["status"], out["serial_hi"], out["serial_lo"], reads, fin)
        assert rep.ok, (scheme, rep)
        eng.release(bid)
    # one 64-lane team in one wavefront runs the batch serially in id order: host- and
    # device-submitted batches must give identical outcomes
    res = []
    for how in ("host", "device"):
        eng.load(tabs)
        bid = eng.submit(b, "occ") if how == "host" else eng.submit_device(b, "occ")
        eng.run(bid, lanes_per_txn=64, waves_per_wg=1, grid=1)
        res.append((eng.outcomes(bid, b.n_txns, b.total_ops), eng.tables()))
        eng.release(bid)
    (o1, r1), f1 = res[0]
    (o2, r2), f2 = res[1]
    assert np.array_equal(r1, r2) and np.array_equal(f1[0], f2[0])
    assert np.array_equal(o1["serial_lo"], o2["serial_lo"]) and np.array_equal(o1["attempts"], o2["attempts"])

print("[child] order-entry batch, device-submitted, tictoc", flush=True)
tabs, b = wl.order_entry_workload(8, 3_000, seed=62)
with B.Engine(tabs) as eng:
    bid = eng.submit_device(b, "tictoc")
    eng.run(bid)
    out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
    fin = eng.tables()
    assert oracle.check_run(tabs, b, out["status"], out["serial_hi"], out["serial_lo"], reads, fin).ok
    assert oracle.order_entry_invariants(tabs, fin, b, out["status"] == 1) == []

print("[child] keyed batch, device-submitted keys", flush=True)
tabs, b = wl.kv_workload(n_rows=30_000, n_fields=4, n_txns=8_000, ops=16, theta=0.6, seed=63)
keys = wl.index_keys(30_000, seed=63)
op_keys = wl.keyed_ops(b, [keys])
with B.Engine(tabs) as eng:
    eng.create_index(0, keys)
    bid = eng.submit_device(b, "occ", keys=op_keys)
    eng.run(bid)
    rows = eng.rows(bid, b.total_ops)
    exp_rows = oracle.resolve_keys([keys], b, op_keys)
    assert np.array_equal(rows.astype(np.int64), exp_rows)
    out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
    rb = oracle.with_rows(b, exp_rows)
    assert oracle.check_run(tabs, rb, out["status"], out["serial_hi"], out["serial_lo"], reads, eng.tables()).ok

print("[child] malformed batches: device status == host status", flush=True)
tabs = [np.zeros(s, np.int64) for s in SHAPES]
with B.Engine(tabs) as eng:
    n = 0
    for case, status in CHECK_CASES:
        txns, ops = _batch(**case)
        host = B.cc_check_batch(SHAPES, txns, ops, 0)
        assert host == status
        try:
            bid = B.cc_submit_batch(eng.ctx, dev(txns), dev(ops), 0)
            got = 0
            B.cc_release_batch(eng.ctx, bid)
        except B.CCError as e:
            got = e.status
        assert got == host, (case, got, host)
        n += 1
    txns, ops = _batch(rows=[1, 2, 3])
    bad = []
    t2 = txns.copy(); t2["n_ops"] = 4; bad.append((t2, ops))                       # op range past the end
    bad.append((np.concatenate([txns, txns]), ops))                              # two txns share ops
    t4 = txns.copy(); t4["reserved"] = 1; bad.append((t4, ops))
    big = np.zeros(300, B.OP_DTYPE); big["row"] = np.arange(300) % 100; big["field"] = np.arange(300) // 100
    t5 = np.zeros(1, B.TXN_DTYPE); t5["n_ops"] = 300; bad.append((t5, big))     # more than 256 ops
    for t_, o_ in bad:
        host = B.cc_check_batch(SHAPES, t_, o_, 0)
        assert host == B.CC_E_INVAL
        try:
            B.cc_submit_batch(eng.ctx, dev(t_), dev(o_), 0)
            got = 0
        except B.CCError as e:
            got = e.status
        assert got == host
    # GaccO needs transactions in op order
    txns, ops = _batch(rows=[1, 2, 3, 4])
    two = np.zeros(2, B.TXN_DTYPE); two["first_op"] = [2, 0]; two["n_ops"] = [2, 2]
    try:
        B.cc_submit_batch(eng.ctx, dev(two), dev(ops), B.CC_GACCO)
        got = 0
    except B.CCError as e:
        got = e.status
    assert got == B.CC_E_INVAL
    bid = B.cc_submit_batch(eng.ctx, dev(two), dev(ops), B.CC_OCC)
    B.cc_release_batch(eng.ctx, bid)
    # not device memory, or shorter than the counts: refused before any kernel reads it
    lib = B.lib
    import ctypes
    u64 = ctypes.c_uint64()
    st = lib.cc_submit_batch(eng.ctx, txns.ctypes.data, 1, ops.ctypes.data, 4, 0, 1, ctypes.byref(u64))
    assert st == B.CC_E_INVAL
    dt, do = dev(txns[:1]), dev(ops)
    st = lib.cc_submit_batch(eng.ctx, dt.data_ptr(), 1, do.data_ptr(), 1 << 20, 0, 1, ctypes.byref(u64))
    assert st == B.CC_E_INVAL
    print(f"[child] {n} malformed cases agree", flush=True)
print("DEVICE_SUBMIT_OK", flush=True)
'''


def test_device_submitted_batches():
    print("\n[gpu] device-submitted batches (child process)", flush=True)
    r = subprocess.run([sys.executable, "-c", f"ROOT = {ROOT!r}\n" + CHILD], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-4000:]
    assert "DEVICE_SUBMIT_OK" in r.stdout
