"""CPU model of the transaction kernel's persistent team loop and its retry policies (no GPU).

The kernel runs passes of persistent wavefronts; each wavefront holds several
teams (one transaction each) that execute in lockstep, one attempt per loop
iteration, and every attempt releases its locks before the iteration ends.
After a failed attempt a team either backs off for a random, exponentially
growing time (the default), or -- with CC_RUN_WAIT_BLOCKER -- waits until the
row another transaction held is free and retries after a short random
jitter.  A pass defers a transaction after `defer_after` attempts to the next,
8x smaller pass; the final pass (one wavefront) never defers.

An earlier retry-when-free policy hung the GPU: two teams of one wavefront
that block each other (A writes x and reads y, B writes y and reads x) both
see their row free on the next iteration and retry together, forever, in the
final pass that never defers.  This model steps teams in exact lockstep -- the
worst case for that symmetry -- and checks the rule the kernel follows: the
wait runs only in passes that defer, so (i) a deferring pass ends after at
most defer_after attempts per transaction whatever the waits do, and (ii) the
final pass keeps the randomised back-off, which separates the pair.
"""
from __future__ import annotations

import random

import pytest

BACKOFF, WAIT, WAIT_JITTER = "backoff", "wait", "wait+jitter"


class Team:
    def __init__(self):
        self.txn = None
        self.attempts = 0        # in this pass
        self.ready_at = 0
        self.wait_row = None     # waiting for this row to be free


def run_pass(txns, pending, waves, teams_per_wave, policy, defer_after, rng, max_iters=200_000, base=1,
             wait_in_final=False):
    """One pass over `pending` (transaction ids); returns (committed, deferred, iterations).

    txns[i] = (write_rows, read_rows).  Iterations are lockstep steps of every
    team of every wavefront.  `policy` applies only when defer_after > 0; the
    final pass (defer_after == 0) always backs off, as the kernel does --
    unless wait_in_final, the rule of the earlier policy that hung.
    """
    queue = list(pending)
    teams = [[Team() for _ in range(teams_per_wave)] for _ in range(waves)]
    committed, deferred = [], []
    use_wait = policy != BACKOFF and (defer_after > 0 or wait_in_final)
    for it in range(max_iters):
        # claim transactions (in wave and team order, like the kernel's claim counter)
        for wave in teams:
            for t in wave:
                if t.txn is None and queue:
                    t.txn, t.attempts, t.ready_at, t.wait_row = queue.pop(0), 0, it, None
        if all(t.txn is None for wave in teams for t in wave) and not queue:
            return committed, deferred, it
        # waiting teams look at their row: every attempt released its locks at the end of the
        # last iteration, so a row a team waits for is always free by now
        for wave in teams:
            for t in wave:
                if t.txn is not None and t.wait_row is not None:
                    t.wait_row = None
                    t.ready_at = it + (rng.randrange(0, 4 * base) if policy == WAIT_JITTER else 0)
        # attempts of the ready teams, all at once: write locks serialise per row in a random order
        ready = [t for wave in teams for t in wave if t.txn is not None and t.ready_at <= it]
        rng.shuffle(ready)
        held = {}
        result = {}
        for t in ready:
            writes, _ = txns[t.txn]
            got = [r for r in writes if r not in held]
            for r in got:
                held[r] = t
            result[id(t)] = (len(got) == len(writes), next((r for r in writes if held[r] is not t), None))
        for t in ready:
            writes, reads = txns[t.txn]
            ok, blocker = result[id(t)]
            if ok:
                blocker = next((r for r in reads if r in held and held[r] is not t), None)
                ok = blocker is None
            t.attempts += 1
            if ok:
                committed.append(t.txn)
                t.txn = None
            elif defer_after and t.attempts >= defer_after:
                deferred.append(t.txn)
                t.txn = None
            elif use_wait:
                t.wait_row = blocker
            else:
                t.ready_at = it + 1 + rng.randrange(0, base << min(t.attempts, 12))
        # every attempt releases what it took before the iteration ends
    raise RuntimeError(f"pass did not finish in {max_iters} iterations")


def run_all(txns, waves, teams_per_wave, policy, defer_after=16, seed=0, max_iters=200_000):
    """Passes as cc_run makes them: 8x fewer wavefronts each time, the last one wavefront, never deferring."""
    rng = random.Random(seed)
    pending, passes, iters = list(range(len(txns))), 0, 0
    w = waves
    while pending:
        last = w == 1
        c, d, n = run_pass(txns, pending, w, teams_per_wave, policy, 0 if last else defer_after, rng, max_iters)
        passes += 1
        iters += n
        pending = d
        w = max(1, w // 8)
    return passes, iters


CROSSED = [({0}, {1}), ({1}, {0})]  # A writes row 0, reads row 1; B writes row 1, reads row 0


def test_model_reproduces_the_recorded_livelock():
    # the earlier rule: wait for the blocking row in the final pass too, with no jitter -> the
    # crossed pair of one wavefront retries in lockstep and never commits
    with pytest.raises(RuntimeError):
        run_pass(CROSSED, [0, 1], waves=1, teams_per_wave=2, policy=WAIT, defer_after=0, rng=random.Random(0),
                 max_iters=20_000, wait_in_final=True)


@pytest.mark.parametrize("policy", [WAIT, WAIT_JITTER])
def test_a_deferring_pass_ends_whatever_the_waits_do(policy):
    # without jitter the pair conflicts on every attempt, but each is deferred after defer_after
    # attempts, so the pass ends; the final pass (back-off) then commits both
    c, d, n = run_pass(CROSSED, [0, 1], waves=1, teams_per_wave=2, policy=policy, defer_after=16,
                       rng=random.Random(1))
    assert sorted(c + d) == [0, 1]
    if policy == WAIT:
        # lockstep: both fail on every attempt and are deferred together after defer_after attempts
        assert sorted(d) == [0, 1] and n <= 16 + 2
    passes, _ = run_all(CROSSED, waves=8, teams_per_wave=2, policy=policy)
    assert passes >= 1


@pytest.mark.parametrize("seed", range(50))
def test_final_pass_with_back_off_separates_the_pair(seed):
    c, d, n = run_pass(CROSSED, [0, 1], waves=1, teams_per_wave=2, policy=WAIT, defer_after=0,
                       rng=random.Random(seed), max_iters=5_000)
    assert sorted(c) == [0, 1] and d == []


def _zipf_txns(n, rows, ops, theta, seed):
    rng = random.Random(seed)
    weights = [1.0 / (r + 1) ** theta for r in range(rows)]
    out = []
    for _ in range(n):
        picks = set()
        while len(picks) < ops:
            picks.add(rng.choices(range(rows), weights)[0])
        picks = sorted(picks)
        w = {r for r in picks if rng.random() < 0.5}
        out.append((w, set(picks) - w))
    return out


@pytest.mark.parametrize("policy", [BACKOFF, WAIT, WAIT_JITTER])
@pytest.mark.parametrize("seed", range(4))
def test_every_transaction_commits_under_each_policy(policy, seed):
    # hot rows, many teams per wavefront, several wavefronts: every transaction commits exactly once
    txns = _zipf_txns(300, rows=40, ops=4, theta=0.9, seed=seed)
    rng_seed = 100 + seed
    pending = list(range(len(txns)))
    done = []
    w = 8
    rng = random.Random(rng_seed)
    while pending:
        c, d, _ = run_pass(txns, pending, w, 4, policy, 0 if w == 1 else 16, rng)
        done += c
        pending = d
        w = max(1, w // 8)
    assert sorted(done) == list(range(len(txns)))
