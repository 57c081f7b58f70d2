"""CPU model of the OCC hot-row engine's team loop and its waits (no GPU).

In the engine (paper_2406_10158_amd/csrc/hot_engine.h) the transactions that
write one of the batch's engine rows run in one workgroup.  Each wavefront
holds several teams that execute in lockstep, one attempt step per loop
iteration.  A step first takes the transaction's other ("cold") rows as OCC
does -- written rows locked without waiting, a held row aborts -- and then the
engine rows in decreasing engine index (the most written row, index 0, last):
a written row exclusively, a read-only row shared.  At the first engine row
that is not free the team gives back every row it took, engine and cold, and
waits, holding nothing, until that row is free; then it makes a new attempt.  A team that holds all its rows commits (or fails
validation) within the same step and releases everything.

This model steps the teams of a wavefront in exact lockstep and the
wavefronts in random order, and checks the claims the kernel's comments make:
(i) every wait ends -- no team waits while holding a row, and one that holds
all of its rows commits or fails within its step; (ii) keeping the rows taken
while waiting, without an order, deadlocks on two transactions of one
wavefront that write the same engine rows; (iii) the give-up limit releases a waiting team's rows,
and (iv) every transaction commits exactly once, also when readers and writers
of the same engine rows mix, and when waiting teams hold cold rows others need.
"""
from __future__ import annotations

import random

import pytest


class Txn:
    def __init__(self, eng_w=(), eng_r=(), cold_w=(), cold_r=()):
        self.eng_w, self.eng_r = frozenset(eng_w), frozenset(eng_r)
        self.cold_w, self.cold_r = frozenset(cold_w), frozenset(cold_r)
        assert not (self.eng_w & self.eng_r) and not (self.cold_w & self.cold_r)
        self.eng = sorted(self.eng_w | self.eng_r)


class Team:
    def __init__(self):
        self.txn = None
        self.resume = False
        self.held = set()        # engine rows held
        self.cold = set()        # cold rows locked
        self.seen = {}           # cold read row -> version seen
        self.ready_at = 0
        self.wait_since = 0
        self.attempts = 0


class Model:
    def __init__(self, txns, waves, teams_per_wave, ordered=True, wait_limit=10_000, seed=0, base=2):
        # ordered: the kernel's rule (decreasing index, rows given back to wait); otherwise
        # every missing row is tried at once and what was got is kept while waiting
        self.txns = txns
        self.ordered = ordered
        self.wait_limit = wait_limit
        self.rng = random.Random(seed)
        self.base = base
        self.queue = list(range(len(txns)))
        self.waves = [[Team() for _ in range(teams_per_wave)] for _ in range(waves)]
        self.writer = {}         # engine row -> team holding it exclusively
        self.readers = {}        # engine row -> number of shared holders
        self.cold_owner = {}     # cold row -> team
        self.cold_ver = {}       # cold row -> commits that wrote it
        self.committed = []
        self.gave_up = 0
        self.waits = 0

    # ---- engine locks --------------------------------------------------------
    def _try(self, team, j, write):
        if write:
            if j in self.writer or self.readers.get(j, 0):
                return False
            self.writer[j] = team
        else:
            if j in self.writer:
                return False
            self.readers[j] = self.readers.get(j, 0) + 1
        team.held.add(j)
        return True

    def _release_eng(self, team):
        tx = self.txns[team.txn]
        for j in team.held:
            if j in tx.eng_w:
                assert self.writer.get(j) is team
                del self.writer[j]
            else:
                self.readers[j] -= 1
                assert self.readers[j] >= 0
        team.held = set()

    def _release_cold(self, team):
        for r in team.cold:
            assert self.cold_owner.get(r) is team
            del self.cold_owner[r]
        team.cold = set()

    # ---- one lockstep step of a wavefront ---------------------------------------
    def step_wave(self, wave, it):
        active = [t for t in wave if t.txn is not None and t.ready_at <= it]
        # R1: cold rows of teams that are not resuming, all at once in a random order
        fresh = [t for t in active if not t.resume]
        self.rng.shuffle(fresh)
        ok = {}
        for t in fresh:
            tx = self.txns[t.txn]
            got = []
            good = True
            for r in sorted(tx.cold_w):
                if r in self.cold_owner:
                    good = False
                else:
                    self.cold_owner[r] = t
                    got.append(r)
            t.cold = set(got)
            for r in tx.cold_r:
                if r in self.cold_owner and self.cold_owner[r] is not t:
                    good = False
            t.seen = {r: self.cold_ver.get(r, 0) for r in tx.cold_r}
            ok[id(t)] = good
        for t in fresh:
            if not ok[id(t)]:
                self._release_cold(t)
                self._abort(t, it)
        going = [t for t in active if t.txn is not None and (t.resume or ok.get(id(t), False))]
        # R1b: engine rows, wavefront-uniform loop over the rows any team still needs
        stopped = set()
        if self.ordered:
            rows = sorted(set(j for t in going for j in self.txns[t.txn].eng if j not in t.held), reverse=True)
            for j in rows:
                cand = [t for t in going if id(t) not in stopped and j in self.txns[t.txn].eng and j not in t.held]
                self.rng.shuffle(cand)
                for t in cand:
                    if not self._try(t, j, j in self.txns[t.txn].eng_w):
                        stopped.add(id(t))
        else:
            # the rejected rule: every missing row tried at once (the lanes' atomics of one
            # wavefront land in any order), and what was got is kept
            pairs = [(t, j) for t in going for j in self.txns[t.txn].eng if j not in t.held]
            self.rng.shuffle(pairs)
            for t, j in pairs:
                if not self._try(t, j, j in self.txns[t.txn].eng_w):
                    stopped.add(id(t))
        # commit, wait, or give up
        for t in going:
            tx = self.txns[t.txn]
            if id(t) in stopped:
                if self.ordered:
                    # no one waits holding a row; the next try is a new attempt
                    self._release_eng(t)
                    self._release_cold(t)
                    t.resume = False
                    self.waits += 1
                    t.ready_at = it + 1
                    continue
                if t.resume and it - t.wait_since > self.wait_limit:
                    self._release_eng(t)
                    self._release_cold(t)
                    t.resume = False
                    self._abort(t, it)
                    continue
                if not t.resume:
                    t.wait_since = it
                t.resume = True
                self.waits += 1
                t.ready_at = it + 1
                continue
            assert set(tx.eng) <= t.held
            valid = all(self.cold_ver.get(r, 0) == v and (r not in self.cold_owner or self.cold_owner[r] is t)
                        for r, v in t.seen.items())
            if valid:
                for r in tx.cold_w:
                    self.cold_ver[r] = self.cold_ver.get(r, 0) + 1
                self.committed.append(t.txn)
            self._release_eng(t)
            self._release_cold(t)
            t.resume = False
            if valid:
                t.txn = None
            else:
                self._abort(t, it)

    def _abort(self, t, it):
        t.attempts += 1
        t.ready_at = it + 1 + self.rng.randrange(0, self.base << min(t.attempts, 8))

    def run(self, max_iters=200_000):
        for it in range(max_iters):
            for wave in self.waves:
                for t in wave:
                    if t.txn is None and self.queue:
                        t.txn, t.attempts, t.resume, t.ready_at = self.queue.pop(0), 0, False, it
            if not self.queue and all(t.txn is None for w in self.waves for t in w):
                return it
            order = list(range(len(self.waves)))
            self.rng.shuffle(order)
            for w in order:
                self.step_wave(self.waves[w], it)
        raise RuntimeError(f"no end after {max_iters} iterations: committed {len(self.committed)} of {len(self.txns)}")


# two transactions writing the same two engine rows, listed in opposite orders
CROSSED = [Txn(eng_w=(0, 1)), Txn(eng_w=(1, 0))]


@pytest.mark.parametrize("same_wave", [True, False])
@pytest.mark.parametrize("seed", range(20))
def test_ordered_acquisition_never_deadlocks_on_crossed_rows(same_wave, seed):
    txns = CROSSED * 8
    m = Model(txns, waves=1 if same_wave else 4, teams_per_wave=16 if same_wave else 4, seed=seed)
    m.run(max_iters=20_000)
    assert sorted(m.committed) == list(range(len(txns)))


def test_unordered_hold_and_wait_deadlocks():
    # the rule the kernel avoids: take every missing row at once and keep what was got; two
    # teams of one wavefront that both write rows 0-3 end up each holding rows the other
    # waits for.  A wait limit that never fires keeps them waiting.
    txns = [Txn(eng_w=(0, 1, 2, 3)), Txn(eng_w=(0, 1, 2, 3))]
    deadlocked = 0
    for seed in range(40):
        m = Model(txns, waves=1, teams_per_wave=2, ordered=False, wait_limit=10**9, seed=seed)
        try:
            m.run(max_iters=2_000)
        except RuntimeError:
            deadlocked += 1
    assert deadlocked > 0


def test_wait_limit_releases_and_every_transaction_commits():
    # unordered hold-and-wait with a small wait limit: the limit breaks each deadlock
    txns = [Txn(eng_w=(0, 1, 2, 3)), Txn(eng_w=(0, 1, 2, 3))] * 4
    m = Model(txns, waves=2, teams_per_wave=4, ordered=False, wait_limit=20, seed=3)
    m.run(max_iters=50_000)
    assert sorted(m.committed) == list(range(len(txns)))


def _random_txns(n, n_eng, n_cold, seed, p_eng=0.6):
    rng = random.Random(seed)
    out = []
    for _ in range(n):
        eng = rng.sample(range(n_eng), rng.randint(1, min(3, n_eng)))
        w = {eng[0]} | {j for j in eng[1:] if rng.random() < 0.5}   # every engine transaction writes one
        cold = rng.sample(range(n_cold), rng.randint(0, 4))
        cw = {r for r in cold if rng.random() < 0.5}
        out.append(Txn(eng_w=w, eng_r=set(eng) - w, cold_w=cw, cold_r=set(cold) - cw))
    return out


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("shape", [(1, 16), (4, 4), (16, 1)])
def test_every_transaction_commits_once_with_readers_writers_and_cold_rows(shape, seed):
    waves, tpw = shape
    txns = _random_txns(400, n_eng=4, n_cold=12, seed=seed)
    m = Model(txns, waves, tpw, seed=100 + seed)
    m.run(max_iters=100_000)
    assert sorted(m.committed) == list(range(len(txns)))
    if tpw > 1:
        # (the model steps a wavefront at once, so with one team per wavefront no one holds a
        # row between steps)
        assert m.waits > 0
    # locks are all free at the end
    assert not m.writer and not m.cold_owner and all(v == 0 for v in m.readers.values())


def test_no_team_waits_holding_an_engine_row():
    txns = _random_txns(300, n_eng=6, n_cold=8, seed=77)
    m = Model(txns, 4, 4, seed=5)
    orig = m.step_wave

    def checked(wave, it):
        orig(wave, it)
        for w in m.waves:
            for t in w:
                if t.txn is not None and t.ready_at > it:
                    # between steps a team holds rows only while it is in no attempt
                    assert not t.held and not t.cold, (m.txns[t.txn].eng, t.held)

    m.step_wave = checked
    m.run(max_iters=100_000)
    assert sorted(m.committed) == list(range(len(txns)))
