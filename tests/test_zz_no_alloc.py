"""The allocation-free entry point (cc_run_static) against the batch entry points it stands for.

cc_run_static validates, packs and runs a device-resident batch with every
buffer beyond the caller's inputs and outputs in the library's static device
array.  Its results are checked against cc_submit_batch (on_device = 1) +
cc_run + cc_fetch_outcomes on the same tables, in a child process that
initialises torch first (torch carries its own HIP runtime; see
test_gpu_device_buffers.py):
* what is unique in a run matches exactly: every transaction commits, and
  the final table is the add-only closed form, identical for both entry
  points; everything else (reads, serial keys) passes the oracle's replay;
* one 64-lane team in one wavefront runs the batch serially in id order, so
  there the outcomes and read values of both entry points are bit-identical;
* two calls in a row, the second with a smaller batch, each agree with the
  batch entry points (nothing of the first call leaks into the second);
* a batch above the static limits, a scheme or mode that needs per-batch
  buffers, and a malformed batch are refused with the documented status.
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
import numpy as np
from paper_2406_10158_amd import binding as B, workload as wl
import oracle

def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.uint8)).to("cuda")

def static_run(eng, b, scheme, **kw):
    txns, ops = B.pack_batch(b)
    out = torch.zeros(b.n_txns * B.OUTCOME_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    reads = torch.full((b.total_ops,), -7, dtype=torch.int64, device="cuda")  # cleared by the call
    st = B.cc_run_static(eng.ctx, dev(txns), dev(ops), B.SCHEMES[scheme], B.run_params(**kw), out, reads)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(B.OUTCOME_DTYPE), reads.cpu().numpy(), eng.tables(), st

def batch_run(eng, b, scheme, **kw):
    bid = eng.submit_device(b, scheme)
    st = eng.run(bid, **kw)
    out, reads = eng.outcomes(bid, b.n_txns, b.total_ops)
    fin = eng.tables()
    eng.release(bid)
    return out, reads, fin, st

def ok(tabs, b, out, reads, fin):
    rep = oracle.check_run(tabs, b, out["status"], out["serial_hi"], out["serial_lo"], reads, fin)
    assert rep.ok, rep

tabs, big = wl.kv_workload(n_rows=60_000, n_fields=4, n_txns=30_000, ops=16, theta=0.9, seed=71)
_, small = wl.kv_workload(n_rows=60_000, n_fields=4, n_txns=4_000, ops=(2, 12), theta=0.6, seed=72)
with B.Engine(tabs) as eng:
    for scheme in ("occ", "2pl_nw", "2pl_wd", "to", "tictoc"):
        for name, b in (("30k x 16 ops", big), ("4k x 2-12 ops", small)):
            print(f"[child] {scheme} {name}", flush=True)
            eng.load(tabs)
            o1, r1, f1, s1 = batch_run(eng, b, scheme)
            eng.load(tabs)
            o2, r2, f2, s2 = static_run(eng, b, scheme)
            closed = oracle.final_add_only(tabs, b)
            assert np.all(o1["status"] == B.CC_COMMITTED) and np.all(o2["status"] == B.CC_COMMITTED)
            assert s2["committed"] == b.n_txns and s2["attempts"] == int(o2["attempts"].astype(np.int64).sum())
            assert np.array_equal(f1[0], f2[0]) and np.array_equal(f2[0], closed[0])
            ok(tabs, b, o1, r1, f1)
            ok(tabs, b, o2, r2, f2)
    print("[child] one team: bit-identical outcomes", flush=True)
    for b in (big, small):
        eng.load(tabs)
        # (without the hot-row engine, which runs the hottest rows' writers first)
        o1, r1, f1, _ = batch_run(eng, b, "occ", lanes_per_txn=64, waves_per_wg=1, grid=1,
                                  flags=B.CC_RUN_NO_HOT_ENGINE)
        eng.load(tabs)
        o2, r2, f2, _ = static_run(eng, b, "occ", lanes_per_txn=64, waves_per_wg=1, grid=1)
        assert np.array_equal(r1, r2) and np.array_equal(f1[0], f2[0])
        for k in ("status", "attempts", "serial_hi", "serial_lo"):
            assert np.array_equal(o1[k], o2[k]), k
    print("[child] refusals", flush=True)
    txns, ops = B.pack_batch(small)
    dt, do = dev(txns), dev(ops)
    out = torch.zeros(small.n_txns * 32, dtype=torch.uint8, device="cuda")
    reads = torch.zeros(small.total_ops, dtype=torch.int64, device="cuda")
    def status(scheme, params=None, t=dt, o=do):
        try:
            B.cc_run_static(eng.ctx, t, o, scheme, params, out, reads)
            return 0
        except B.CCError as e:
            return e.status
    assert status(B.CC_MVCC) == B.CC_E_INVAL
    assert status(B.CC_GACCO) == B.CC_E_INVAL
    assert status(B.CC_OCC, B.run_params(mode=B.CC_MODE_EPOCH)) == B.CC_E_INVAL
    assert status(B.CC_OCC, B.run_params(flags=B.CC_RUN_LATCH)) == B.CC_E_INVAL
    import ctypes
    st = B.lib.cc_run_static(eng.ctx, dt.data_ptr(), B.CC_STATIC_MAX_TXNS + 1, do.data_ptr(), small.total_ops,
                             B.CC_OCC, None, out.data_ptr(), reads.data_ptr(), None, 0)
    assert st == B.CC_E_RANGE
    st = B.lib.cc_run_static(eng.ctx, dt.data_ptr(), small.n_txns, do.data_ptr(), B.CC_STATIC_MAX_OPS + 1,
                             B.CC_OCC, None, out.data_ptr(), reads.data_ptr(), None, 0)
    assert st == B.CC_E_RANGE
    bad = ops.copy()
    bad["row"][0] = 60_000  # one past the last row
    assert status(B.CC_OCC, o=dev(bad)) == B.CC_E_RANGE
    # a host array where device memory is required
    st = B.lib.cc_run_static(eng.ctx, txns.ctypes.data, small.n_txns, do.data_ptr(), small.total_ops, B.CC_OCC,
                             None, out.data_ptr(), reads.data_ptr(), None, 0)
    assert st == B.CC_E_INVAL
    # the refused calls left the context usable
    eng.load(tabs)
    o2, r2, f2, _ = static_run(eng, small, "occ")
    ok(tabs, small, o2, r2, f2)
print("NO_ALLOC_OK", flush=True)
'''


def test_run_static_matches_batch_entry_points():
    print("\n[gpu] allocation-free run (child process)", flush=True)
    r = subprocess.run([sys.executable, "-c", f"ROOT = {ROOT!r}\n" + CHILD], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-4000:]
    assert "NO_ALLOC_OK" in r.stdout
