"""The C-ABI library without a GPU: it loads, exports every declared entry point, and its
host-only validation rejects malformed batches with the documented status codes."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from helpers import ROOT

HEADER = os.path.join(ROOT, "include", "cc.h")
LIB = os.path.join(ROOT, "paper_2406_10158_amd", "libcc.so")


@pytest.fixture(scope="module")
def b():
    if not os.path.exists(LIB):
        from paper_2406_10158_amd import build
        build.build()
    from paper_2406_10158_amd import binding
    return binding


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(cc_[a-z_0-9]+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("cc_init", "cc_destroy", "cc_create_table", "cc_load", "cc_submit_batch", "cc_run",
              "cc_fetch_outcomes", "cc_read_table", "cc_stats", "cc_strerror", "cc_check_batch"):
        assert n in names


def test_library_exports_every_declared_symbol(b):
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing


def test_strerror_and_version(b):
    assert b.cc_strerror(0) == "ok"
    assert "duplicate" in b.cc_strerror(b.CC_E_DUPROW)
    assert b.cc_strerror(-999) == "unknown status"
    assert b.cc_version().startswith("cc-gfx950")


def test_struct_layouts_match_header(b, tmp_path):
    # compile the header with the host C compiler and compare every size and field offset
    # with the binding's numpy dtypes and ctypes structures
    layouts = [("cc_op", b.OP_DTYPE.names, None), ("cc_txn", b.TXN_DTYPE.names, None),
               ("cc_outcome", b.OUTCOME_DTYPE.names, None),
               ("cc_run_params", [f[0] for f in b.cc_run_params._fields_], None),
               ("cc_config", [f[0] for f in b.cc_config._fields_], None)]
    lines = []
    for name, fields, _ in layouts:
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"cc.h\"\nint main(void) {\n"
                   + "\n".join(lines) + "\n  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for name, dt in (("cc_op", b.OP_DTYPE), ("cc_txn", b.TXN_DTYPE), ("cc_outcome", b.OUTCOME_DTYPE)):
        assert dt.itemsize == int(got[name]), name
        for f in dt.names:
            assert dt.fields[f][1] == int(got[f"{name}.{f}"]), (name, f)
    for name, st in (("cc_run_params", b.cc_run_params), ("cc_config", b.cc_config)):
        assert ctypes.sizeof(st) == int(got[name]), name
        for f, _ in st._fields_:
            assert getattr(st, f).offset == int(got[f"{name}.{f}"]), (name, f)


def _batch(rows, tables=None, fields=None, kinds=None, args=None, txn_lens=None):
    from paper_2406_10158_amd.binding import OP_DTYPE, TXN_DTYPE
    n = len(rows)
    ops = np.zeros(n, OP_DTYPE)
    ops["row"] = rows
    ops["table"] = tables if tables is not None else 0
    ops["field"] = fields if fields is not None else 0
    ops["kind"] = kinds if kinds is not None else 0
    ops["arg"] = args if args is not None else 0
    lens = txn_lens if txn_lens is not None else [n]
    txns = np.zeros(len(lens), TXN_DTYPE)
    txns["n_ops"] = lens
    txns["first_op"] = np.concatenate([[0], np.cumsum(lens)[:-1]]) if len(lens) else []
    return txns, ops


SHAPES = [(100, 4), (10, 2)]


CHECK_CASES = [
    (dict(rows=[1, 2, 3]), 0),
    (dict(rows=[1, 100]), -2),                                   # row out of range
    (dict(rows=[1, 2], fields=[0, 4]), -2),                      # field out of range
    (dict(rows=[1, 2], tables=[0, 2]), -2),                      # table out of range
    (dict(rows=[1, 2], kinds=[0, 4]), -1),                       # unknown kind
    (dict(rows=[1, 2, 1]), -3),                                  # non-adjacent repeat of a row
    (dict(rows=[1, 1], fields=[0, 1]), 0),                       # adjacent ops on one row: one row access
    (dict(rows=[1, 1], fields=[2, 2]), -3),                      # a field repeated
    (dict(rows=[5, 5], tables=[0, 1]), 0),                       # same row id, different tables
    (dict(rows=[1, 2], kinds=[0, 3], args=[0, 0]), 0),           # WRITE_SLOT from op 0
    (dict(rows=[1, 2], kinds=[3, 0], args=[0, 0]), -1),          # WRITE_SLOT from itself
    (dict(rows=[1, 2, 3, 1], txn_lens=[2, 2]), 0),               # the same row in different txns is fine
    (dict(rows=list(range(80)) * 4, fields=[0] * 80 + [1] * 80 + [2] * 80 + [3] * 80, txn_lens=[80] * 4), 0),
    (dict(rows=[1, 2, 3, 4, 100], txn_lens=[2, 3]), -2),       # the second transaction is malformed
    (dict(rows=[1, 2, 1, 4, 100], txn_lens=[3, 2]), -3),       # both are: the first one's status wins
]


@pytest.mark.parametrize("case,status", CHECK_CASES)
def test_check_batch_statuses(b, case, status):
    txns, ops = _batch(**case)
    assert b.cc_check_batch(SHAPES, txns, ops, 0) == status


def test_check_batch_structural_errors(b):
    txns, ops = _batch(rows=[1, 2, 3])
    assert b.cc_check_batch(SHAPES, txns, ops, b.CC_GPUTX + 1) == b.CC_E_INVAL  # unknown scheme
    t2 = txns.copy(); t2["n_ops"] = 4
    assert b.cc_check_batch(SHAPES, t2, ops, 0) == b.CC_E_INVAL           # op range past the end
    t3 = np.concatenate([txns, txns])
    assert b.cc_check_batch(SHAPES, t3, ops, 0) == b.CC_E_INVAL           # two txns share ops
    t4 = txns.copy(); t4["reserved"] = 1
    assert b.cc_check_batch(SHAPES, t4, ops, 0) == b.CC_E_INVAL
    big = np.zeros(300, b.OP_DTYPE); big["row"] = np.arange(300) % 100; big["field"] = np.arange(300) // 100
    t5 = np.zeros(1, b.TXN_DTYPE); t5["n_ops"] = 300
    assert b.cc_check_batch(SHAPES, t5, big, 0) == b.CC_E_INVAL           # more than 256 ops
    empty_t, empty_o = np.zeros(0, b.TXN_DTYPE), np.zeros(0, b.OP_DTYPE)
    assert b.cc_check_batch(SHAPES, empty_t, empty_o, 0) == 0             # empty batch
    zero = np.zeros(1, b.TXN_DTYPE)
    assert b.cc_check_batch(SHAPES, zero, empty_o, 0) == 0                # a txn with no ops
    assert b.cc_check_batch([(1 << 28, 1), (1, 1)], empty_t, empty_o, 0) == b.CC_E_RANGE


def test_check_batch_gacco_needs_transactions_in_op_order(b):
    # GaccO sorts each row's accesses into transaction order by a stable sort
    # of the ops array, so transaction t's ops must come after t-1's
    txns, ops = _batch(rows=[1, 2, 3, 4])
    two = np.zeros(2, b.TXN_DTYPE)
    two["first_op"] = [2, 0]
    two["n_ops"] = [2, 2]
    assert b.cc_check_batch(SHAPES, two, ops, b.CC_GACCO) == b.CC_E_INVAL
    assert b.cc_check_batch(SHAPES, two, ops, b.CC_GPUTX) == b.CC_E_INVAL  # GPUTx has the same rule
    assert b.cc_check_batch(SHAPES, two, ops, b.CC_OCC) == 0
    two["first_op"] = [0, 2]
    assert b.cc_check_batch(SHAPES, two, ops, b.CC_GACCO) == 0
    assert b.cc_check_batch(SHAPES, two, ops, b.CC_GPUTX + 1) == b.CC_E_INVAL  # one past the last scheme


def test_check_batch_accepts_generated_workloads(b):
    from paper_2406_10158_amd import workload as wl
    tabs, bt = wl.order_entry_workload(2, 200, seed=1)
    txns, ops = b.pack_batch(bt)
    assert b.cc_check_batch([t.shape for t in tabs], txns, ops, 0) == 0
    (tab,), kb = wl.kv_workload(n_rows=1000, n_fields=10, n_txns=500, ops=(2, 64), theta=0.99)
    txns, ops = b.pack_batch(kb)
    assert b.cc_check_batch([tab.shape], txns, ops, 4) == 0
    assert b.cc_check_batch([tab.shape], txns, ops, b.CC_GACCO) == 0


def test_init_without_a_gpu_fails_cleanly(b):
    # the kernel driver's device node, not torch: in a process that loaded the library first,
    # torch's own HIP runtime can report no device while the library's sees one
    if os.path.exists("/dev/kfd"):
        pytest.skip("a GPU is present")
    with pytest.raises(b.CCError) as e:
        b.cc_init(0)
    assert e.value.status == b.CC_E_NODEV


def test_every_entry_point_rejects_a_null_context(b):
    # no GPU needed: each call returns CC_E_INVAL before touching the device (cc_destroy(NULL) is a no-op)
    lib = b.lib
    u64 = ctypes.c_uint64()
    u32 = ctypes.c_uint32()
    buf = (ctypes.c_int64 * 8)()
    params = b.run_params()
    calls = {
        "cc_create_table": lambda: lib.cc_create_table(None, 4, 1, ctypes.byref(u32)),
        "cc_load": lambda: lib.cc_load(None, 0, ctypes.addressof(buf), 4, 0),
        "cc_read_table": lambda: lib.cc_read_table(None, 0, ctypes.addressof(buf), 0),
        "cc_submit_batch": lambda: lib.cc_submit_batch(None, None, 0, None, 0, 0, 0, ctypes.byref(u64)),
        "cc_submit_batch_keyed": lambda: lib.cc_submit_batch_keyed(None, None, 0, None, 0, None, 0, 0, ctypes.byref(u64)),
        "cc_create_index": lambda: lib.cc_create_index(None, 0, None, 0),
        "cc_run": lambda: lib.cc_run(None, 1, ctypes.byref(params)),
        "cc_fetch_outcomes": lambda: lib.cc_fetch_outcomes(None, 1, None, None, 0),
        "cc_fetch_rows": lambda: lib.cc_fetch_rows(None, 1, ctypes.addressof(buf)),
        "cc_engine_plan": lambda: lib.cc_engine_plan(None, 1, ctypes.addressof(buf), ctypes.byref(u32),
                                                      ctypes.byref(u64), ctypes.byref(ctypes.c_int())),
        "cc_set_arrivals": lambda: lib.cc_set_arrivals(None, 1, None, 0),
        "cc_stats": lambda: lib.cc_stats(None, 1, None, 0),
        "cc_release_batch": lambda: lib.cc_release_batch(None, 1),
        "cc_run_static": lambda: lib.cc_run_static(None, None, 0, None, 0, 0, None, None, None, None, 0),
        "cc_device_info": lambda: lib.cc_device_info(None, None, None),
        "cc_probe": lambda: lib.cc_probe(None, 0, 1 << 20, 1, 1, None),
        "cc_probe_indices": lambda: lib.cc_probe_indices(None, 1, 1 << 20, None, 0, None),
        "cc_init": lambda: lib.cc_init(None, None),
    }
    for name, call in calls.items():
        assert call() == b.CC_E_INVAL, name
    assert lib.cc_destroy(None) == b.CC_OK
    assert isinstance(lib.cc_last_error(None), bytes)


def test_run_parameter_checks_without_a_device(b):
    ok = b.cc_check_run_params
    P = b.run_params
    # waiting for a blocking row, and hot rows last, exist for the schemes that implement them
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_WAIT_BLOCKER)) == b.CC_OK
    assert ok(b.CC_TICTOC, P(flags=b.CC_RUN_WAIT_BLOCKER)) == b.CC_OK
    for sch in (b.CC_2PL_NW, b.CC_2PL_WD, b.CC_TO, b.CC_MVCC, b.CC_GACCO, b.CC_GPUTX):
        assert ok(sch, P(flags=b.CC_RUN_WAIT_BLOCKER)) == b.CC_E_INVAL
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_HOT_LAST)) == b.CC_OK
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_HOT_LAST | b.CC_RUN_NO_HOT_LAST)) == b.CC_E_INVAL
    assert ok(b.CC_TICTOC, P(flags=b.CC_RUN_HOT_LAST)) == b.CC_E_INVAL
    # the hot-row engine: OCC, plain mode, no latches; its two flags exclude each other
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_HOT_ENGINE)) == b.CC_OK
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_NO_HOT_ENGINE)) == b.CC_OK
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_HOT_ENGINE | b.CC_RUN_NO_HOT_ENGINE)) == b.CC_E_INVAL
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_HOT_ENGINE | b.CC_RUN_LATCH)) == b.CC_E_INVAL
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_NO_HOT_ENGINE | b.CC_RUN_LATCH)) == b.CC_OK
    for mode in (b.CC_MODE_EPOCH, b.CC_MODE_SERVE):
        assert ok(b.CC_OCC, P(flags=b.CC_RUN_HOT_ENGINE, mode=mode)) == b.CC_E_INVAL
        assert ok(b.CC_OCC, P(flags=b.CC_RUN_NO_HOT_ENGINE, mode=mode)) == b.CC_OK
    for sch in (b.CC_2PL_NW, b.CC_2PL_WD, b.CC_TO, b.CC_MVCC, b.CC_TICTOC):
        for f in (b.CC_RUN_HOT_ENGINE, b.CC_RUN_NO_HOT_ENGINE):
            assert ok(sch, P(flags=f)) == b.CC_E_INVAL
    assert ok(b.CC_OCC) == b.CC_OK and ok(b.CC_OCC, P(flags=b.CC_RUN_PRECHECK | b.CC_RUN_STRICT_FENCES)) == b.CC_OK
    assert ok(b.CC_OCC, P(mode=7)) == b.CC_E_INVAL
    assert ok(b.CC_OCC, P(lanes_per_txn=8)) == b.CC_E_INVAL
    assert ok(b.CC_OCC, P(waves_per_wg=17)) == b.CC_E_INVAL
    assert ok(b.CC_OCC, P(flags=1 << 20)) == b.CC_E_INVAL
    assert ok(99) == b.CC_E_INVAL
    # the pre-check round exists for OCC, TicToc, TO and MVCC only, and its two flags exclude each other
    for name in ("occ", "tictoc", "to", "mvcc"):
        for f in (b.CC_RUN_PRECHECK, b.CC_RUN_NO_PRECHECK):
            assert ok(b.SCHEMES[name], P(flags=f)) == b.CC_OK, name
        assert ok(b.SCHEMES[name], P(flags=b.CC_RUN_PRECHECK | b.CC_RUN_NO_PRECHECK)) == b.CC_E_INVAL
    for name in ("2pl_nw", "2pl_wd", "gacco", "gputx"):
        for f in (b.CC_RUN_PRECHECK, b.CC_RUN_NO_PRECHECK):
            assert ok(b.SCHEMES[name], P(flags=f)) == b.CC_E_INVAL, name
    # eager install is an OCC option
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_EAGER_INSTALL)) == b.CC_OK
    for name in ("2pl_nw", "2pl_wd", "to", "mvcc", "tictoc", "gacco", "gputx"):
        assert ok(b.SCHEMES[name], P(flags=b.CC_RUN_EAGER_INSTALL)) == b.CC_E_INVAL, name
    # the retry-when-free flag is reserved and always rejected
    for sch in range(8):
        assert ok(sch, P(flags=b.CC_RUN_WAIT_UNLOCK)) == b.CC_E_INVAL
    # options of other schemes, and what GaccO / GPUTx do not run
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_SHARED_READS)) == b.CC_E_INVAL
    assert ok(b.CC_GACCO, P(flags=b.CC_RUN_SHARED_READS)) == b.CC_OK
    assert ok(b.CC_GPUTX, P(flags=b.CC_RUN_SHARED_READS)) == b.CC_E_INVAL
    assert ok(b.CC_OCC, P(wait_limit_us=5)) == b.CC_E_INVAL
    assert ok(b.CC_GACCO, P(wait_limit_us=5)) == b.CC_OK
    for sch in (b.CC_GACCO, b.CC_GPUTX):
        assert ok(sch, P(mode=b.CC_MODE_EPOCH)) == b.CC_E_INVAL
        assert ok(sch, P(flags=b.CC_RUN_LATCH)) == b.CC_E_INVAL
    assert ok(b.CC_OCC, P(flags=b.CC_RUN_LATCH, mode=b.CC_MODE_EPOCH)) == b.CC_OK
