"""GPU parity of the hash-table stress insertion (Sec. IV hash-table stress
test; the table of Sec. III-B) through the C ABI against the oracle's
sequential linear probing.

Concurrent inserts land in slots that depend on scheduling, so slots are not
compared.  What linear probing fixes regardless of the order is compared
exactly: the set of occupied slots and the probe sum.  The rest is checked
for validity: every key is stored once with its value and is reached from
its home slot over occupied slots, and the reported longest probe is the
longest one in the GPU's own table."""
import numpy as np
import pytest

import oracle as orc
import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_21149_amd as cv
    return cv


def _table(torch, cap):
    return (torch.full((cap,), -1, dtype=torch.int64, device="cuda"),
            torch.zeros(cap, dtype=torch.int32, device="cuda"))


def _host(tk, tv):
    return tk.cpu().numpy().view(np.uint64), tv.cpu().numpy().view(np.uint32)


def _probes_of(keys_t, vals_t, keys, cap):
    """Slot and home slot of each key in a host copy of the table."""
    occ = keys_t != orc.HashTable.EMPTY
    order = np.argsort(keys_t[occ])
    sk = keys_t[occ][order]
    slot_of = np.flatnonzero(occ)[order]
    at = np.searchsorted(sk, keys)
    assert np.all(at < len(sk)) and np.array_equal(sk[at], keys), "a key is missing"
    slots = slot_of[at]
    return slots, orc.home_bucket(keys, cap)


def _check_reachable(occ, home, slots, cap):
    """Every slot from the home slot up to the key's slot is occupied."""
    free_before = np.cumsum(~occ)  # empty slots in [0, s]
    lo, hi = home, slots
    straight = hi >= lo
    nfree = np.where(straight, free_before[hi] - np.where(lo > 0, free_before[lo - 1], 0),
                     (free_before[-1] - free_before[lo - 1]) + free_before[hi])
    assert np.all(nfree == 0)


def test_small_table_matches_oracle_batch_by_batch(cv):
    """2^16 slots filled to 85 % in batches of 4096 keys (ragged last batch)."""
    import torch
    cap = 1 << 16
    n = int(0.85 * cap)
    keys = sg.hash_keys(n, seed=7)
    ctx = cv.Context(block_capacity=64)
    tk, tv = _table(torch, cap)
    kd = torch.from_numpy(keys.view(np.int64)).cuda()
    ref = orc.HashTable(cap)
    stats = torch.zeros(3, dtype=torch.int64, device="cuda")
    for b0 in range(0, n, 4096):
        b1 = min(n, b0 + 4096)
        stats.zero_()
        ref_sum0 = int(ref.stats[1])
        ctx.hash_insert(tk, tv, b0, kd[b0:b1], stats, val_base=b0)
        ref.insert(keys[b0:b1], val_base=b0)
        st = stats.cpu().numpy()
        hk, hv = _host(tk, tv)
        occ = hk != orc.HashTable.EMPTY
        assert np.array_equal(occ, ref.occupied()), b0
        assert st[1] == ref.stats[1] - ref_sum0 and st[2] == 0, (b0, st)
        slots, home = _probes_of(hk, hv, keys[b0:b1], cap)
        assert np.array_equal(hv[slots], np.arange(b0, b1, dtype=np.uint32))
        assert st[0] == ((slots - home) % cap).max()
        _check_reachable(occ, home, slots, cap)
    ctx.close()


def test_full_size_table_matches_oracle(cv):
    """The benchmark's largest case: 2^26 slots, 85 % load (57 M keys) in
    batches of 2^20 keys.  Occupancy and probe sum against the oracle; every
    key present with its value; the longest probe against the GPU table."""
    import torch
    cap = 1 << 26
    n = int(0.85 * cap)
    keys = sg.hash_keys(n, seed=7)
    ctx = cv.Context(block_capacity=64)
    tk, tv = _table(torch, cap)
    kd = torch.from_numpy(keys.view(np.int64)).cuda()
    stats = torch.zeros((n + (1 << 20) - 1) >> 20, 3, dtype=torch.int64, device="cuda")
    for j, b0 in enumerate(range(0, n, 1 << 20)):
        ctx.hash_insert(tk, tv, b0, kd[b0:b0 + (1 << 20)], stats[j], val_base=b0)
    st = stats.cpu().numpy()
    hk, hv = _host(tk, tv)
    del tk, tv, kd
    ref = orc.HashTable(cap)
    probe = ref.insert(keys)
    occ = hk != orc.HashTable.EMPTY
    assert np.array_equal(occ, ref.occupied())
    assert st[:, 1].sum() == ref.stats[1] and st[:, 2].sum() == 0
    # the value of a slot is its key's index (val_base = batch start): every
    # slot holds the key its value names, and the values are all distinct
    S = np.flatnonzero(occ)
    i_gpu = hv[S].astype(np.int64)
    assert np.array_equal(hk[S], keys[i_gpu])
    assert len(np.unique(i_gpu)) == n
    # home slots from the oracle's table: slot - probe length of its key
    R = np.flatnonzero(ref.occupied())
    i_ref = ref.vals[R].astype(np.int64)
    home = np.empty(n, np.int64)
    home[i_ref] = (R - probe[i_ref]) % cap
    disp = (S - home[i_gpu]) % cap
    assert st[:, 0].max() == disp.max()
    _check_reachable(occ, home[i_gpu], S, cap)
    ctx.close()


def test_rejects_bad_input_and_stops_on_an_understated_load(cv):
    import torch
    ctx = cv.Context(block_capacity=64)
    st = torch.zeros(3, dtype=torch.int64, device="cuda")
    keys = torch.from_numpy(sg.hash_keys(8, seed=2).view(np.int64)).cuda()
    tk, tv = _table(torch, 1000)  # not a power of two
    with pytest.raises(cv.CovoxError):
        ctx.hash_insert(tk, tv, 0, keys, st)
    tk, tv = _table(torch, 1024)
    with pytest.raises(cv.CovoxError):  # 1020 + 8 > 15/16 of 1024
        ctx.hash_insert(tk, tv, 1020, keys, st)
    with pytest.raises(ValueError):
        ctx.hash_insert(tk, tv[:512], 0, keys, st)
    ctx.hash_insert(tk, tv, 0, keys[:0], st)  # no keys: nothing runs
    assert st.cpu().tolist() == [0, 0, 0]
    # every slot holds a key (the caller did not clear the table but claims
    # it is empty): each probe stops after 1024 slots and is counted
    tk.fill_(5)
    ctx.hash_insert(tk, tv, 0, keys, st)
    assert st.cpu().tolist()[2] == 8
    assert bool((tk == 5).all())
    ctx.close()
