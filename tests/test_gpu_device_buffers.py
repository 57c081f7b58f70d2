"""Device-resident buffers and a caller's stream through the C-ABI.

The library runs on a stream the caller owns (torch's), loads a table from a
device tensor, and writes the final table, the outcome records and the read
values into device tensors.  Copied back, they must pass the oracle's serial
replay.  The check runs in a child process that initialises torch before it
loads the library: torch carries its own copy of the HIP runtime, and in a
process where the library's runtime initialised first, torch finds no device.
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

print("[child] torch and the library are up", flush=True)
stream = torch.cuda.Stream()  # default priority
tabs, b = wl.kv_workload(n_rows=50_000, n_fields=4, n_txns=20_000, ops=16, theta=0.9, seed=51)
ctx = B.cc_init(0, stream.cuda_stream)
tid = B.cc_create_table(ctx, tabs[0].shape[0], tabs[0].shape[1])
dev_tab = torch.from_numpy(tabs[0]).to("cuda")
torch.cuda.synchronize()
B.cc_load(ctx, tid, dev_tab)
txns, ops = B.pack_batch(b)
bid = B.cc_submit_batch(ctx, txns, ops, B.CC_OCC)
B.cc_run(ctx, bid, B.run_params())
out_dev = torch.zeros(b.n_txns * B.OUTCOME_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
reads_dev = torch.zeros(b.total_ops, dtype=torch.int64, device="cuda")
B.cc_fetch_outcomes(ctx, bid, out_dev, reads_dev)
fin_dev = torch.empty(tabs[0].shape, dtype=torch.int64, device="cuda")
B.cc_read_table(ctx, tid, fin_dev)
stream.synchronize()
torch.cuda.synchronize()
out = out_dev.cpu().numpy().view(B.OUTCOME_DTYPE)
reads = reads_dev.cpu().numpy()
fin = fin_dev.cpu().numpy()
rep = oracle.check_run(tabs, b, out["status"], out["serial_hi"], out["serial_lo"], reads, [fin])
assert rep.ok, rep
assert (out["status"] == B.CC_COMMITTED).all()
B.cc_destroy(ctx)
print("DEVICE_BUFFERS_OK", flush=True)
'''


def test_device_buffers_and_a_callers_stream():
    print("\n[gpu] device buffers and torch's stream (child process)", flush=True)
    r = subprocess.run([sys.executable, "-c", f"ROOT = {ROOT!r}\n" + CHILD], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "DEVICE_BUFFERS_OK" in r.stdout
