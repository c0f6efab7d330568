"""Pins of the oracle's hash table (Sec. III-B: blocks indexed by 3-D
position through an open-addressing hash table; Sec. IV: the hash-table
stress test inserts many keys at a range of load factors).

The oracle inserts keys one after another with linear probing towards
higher slots.  Pinned against what the definition and the analysis of
linear probing fix: every key is stored once and is reached from its home
slot over occupied slots only; two keys with one home slot land in adjacent
slots; the set of occupied slots and the probe sum do not depend on the
insertion order (a classical property of linear probing, Peterson 1957;
Knuth, TAOCP vol. 3, Sec. 6.4); the mean probe length follows Knuth's
asymptotic count alpha / (2 (1 - alpha)) for random keys; a full table
rejects the next key."""
import numpy as np
import pytest

import oracle as orc
import scenegen as sg


def _home(keys, cap):
    return orc.home_bucket(keys, cap)


def _slots(t, keys):
    pos = {int(k): s for s, k in enumerate(t.keys) if k != orc.HashTable.EMPTY}
    return np.array([pos[int(k)] for k in keys])


def test_keys_are_distinct_and_never_the_empty_slot():
    k = sg.hash_keys(300000)
    assert len(np.unique(k)) == len(k)
    assert not np.any(k == np.uint64(0xFFFFFFFFFFFFFFFF))
    assert np.array_equal(k[:1000], sg.hash_keys(1000))  # a prefix of the same stream


def test_every_key_is_stored_once_and_reachable_from_its_home():
    cap = 1 << 10
    keys = sg.hash_keys(800, seed=3)
    t = orc.HashTable(cap)
    probe = t.insert(keys, val_base=100)
    occ = t.occupied()
    assert occ.sum() == len(keys)
    slots = _slots(t, keys)
    home = _home(keys, cap)
    assert np.array_equal(t.vals[slots], 100 + np.arange(len(keys)))
    assert np.array_equal(probe, (slots - home) % cap)
    for h, s in zip(home, slots):
        span = (np.arange(h, h + (s - h) % cap + 1)) % cap
        assert occ[span].all()
    assert t.stats[0] == probe.max() and t.stats[1] == probe.sum() and t.stats[2] == 0


def test_keys_with_one_home_slot_fill_the_next_slots_upwards():
    cap = 16
    keys = sg.hash_keys(400, seed=5)
    home = _home(keys, cap)
    same = keys[home == 15][:3]  # home at the last slot: the probe wraps to 0, then 1
    assert len(same) == 3
    t = orc.HashTable(cap)
    assert list(t.insert(same)) == [0, 1, 2]
    assert t.keys[15] == same[0] and t.keys[0] == same[1] and t.keys[1] == same[2]


@pytest.mark.parametrize("alpha", [0.5, 0.85])
def test_occupancy_and_probe_sum_do_not_depend_on_the_order(alpha):
    cap = 1 << 12
    keys = sg.hash_keys(int(alpha * cap), seed=11)
    ref = orc.HashTable(cap)
    ref.insert(keys)
    rng = np.random.default_rng(2)
    maxes = set()
    for _ in range(6):
        t = orc.HashTable(cap)
        t.insert(keys[rng.permutation(len(keys))])
        assert np.array_equal(t.occupied(), ref.occupied())
        assert t.stats[1] == ref.stats[1]
        maxes.add(int(t.stats[0]))
    assert max(maxes) >= ref.stats[1] / len(keys)  # the longest probe is at least the mean


@pytest.mark.parametrize("alpha,tol", [(0.25, 0.03), (0.5, 0.03), (0.85, 0.10)])
def test_mean_probe_follows_the_linear_probing_analysis(alpha, tol):
    """Successful search with linear probing takes (1 + 1/(1 - alpha)) / 2
    probes on average (Knuth, Sec. 6.4), i.e. alpha / (2 (1 - alpha)) slots
    past the home slot."""
    cap = 1 << 20
    n = int(alpha * cap)
    t = orc.HashTable(cap)
    probe = t.insert(sg.hash_keys(n, seed=7))
    expect = alpha / (2 * (1 - alpha))
    assert abs(probe.mean() - expect) <= tol * expect, (probe.mean(), expect)


def test_full_table_rejects_the_next_key():
    cap = 8
    keys = sg.hash_keys(9, seed=1)
    t = orc.HashTable(cap)
    p = t.insert(keys[:8])
    assert t.occupied().all() and (p >= 0).all()
    p9 = t.insert(keys[8:])
    assert p9[0] == -1 and t.stats[2] == 1
