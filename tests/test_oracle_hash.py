"""Pins for the oracle's hash function and hash-table structure (Sec. 3.2, 3.3)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hash_values.txt")


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append([int(t) for t in line.split()])
    return rows


def test_hash_golden_values(oracle_mod):
    rows = _golden_rows()
    assert len(rows) == 8
    for x, y, z, h16, h20, h22 in rows:
        assert oracle_mod.hash_index(x, y, z, (1 << 16) - 1) == h16
        assert oracle_mod.hash_index(x, y, z, (1 << 20) - 1) == h20
        assert oracle_mod.hash_index(x, y, z, (1 << 22) - 1) == h22


def _check_structure(vol, inserted):
    """Invariants of a bucket + excess-list table (Sec. 3.2): every inserted
    key is retrievable; keys unique; chains acyclic and reach only excess
    slots; used excess slots == allocated entries not in a bucket; free +
    used == capacity; block pointers unique."""
    pos, off, ptr = vol.entries()
    nb = vol.n_buckets
    for key in inserted:
        i = vol.lookup(*key)
        assert i >= 0 and tuple(pos[i]) == tuple(key)
    alloc = np.flatnonzero(ptr >= 0)
    keys = {tuple(p) for p in pos[alloc]}
    assert len(keys) == alloc.size
    assert len(set(ptr[alloc].tolist())) == alloc.size
    assert keys == {tuple(k) for k in inserted}
    # chains: each bucket chain is acyclic and every excess slot is reached once
    reached = np.zeros(vol.n_excess, np.int32)
    for b in range(nb):
        seen = set()
        i = b
        while off[i] >= 1:
            j = nb + off[i] - 1
            assert j not in seen, "cycle in chain"
            seen.add(j)
            reached[j - nb] += 1
            i = j
    assert reached.max(initial=0) <= 1
    used_excess = int(reached.sum())
    in_excess = int((alloc >= nb).sum())
    assert used_excess == in_excess
    # an entry in a chain hashes to the chain's bucket
    for i in alloc[alloc >= nb]:
        h = oracle_hash_of(pos[i], nb)
        j = h
        found = False
        while off[j] >= 1:
            j = nb + off[j] - 1
            if j == i:
                found = True
                break
        assert found
    assert vol.n_free_excess + used_excess == vol.n_excess
    assert vol.n_free_blocks + alloc.size == vol.n_blocks


def oracle_hash_of(p, nb):
    from oracle import oracle as O
    return O.hash_index(int(p[0]), int(p[1]), int(p[2]), nb - 1)


def test_tiny_table_adversarial_collisions(oracle_mod):
    vol = oracle_mod.Volume(0.01, 0.04, 100, 1 << 4, 1 << 8, 1 << 9)
    rng = np.random.default_rng(7)
    keys = set()
    while len(keys) < 200:
        keys.add(tuple(int(t) for t in rng.integers(-40, 40, size=3)))
    keys = sorted(keys)
    for k in keys:
        assert vol.insert(*k) >= 0
        assert vol.insert(*k) >= 0          # idempotent
    assert vol.flags == 0
    _check_structure(vol, keys)
    # 200 keys in 16 buckets: at most 16 sit in buckets, the rest are chained
    pos, off, ptr = vol.entries()
    assert int((ptr[:16] >= 0).sum()) <= 16
    assert int((ptr[16:] >= 0).sum()) >= 184


def test_absent_keys_not_found(oracle_mod):
    vol = oracle_mod.Volume(0.01, 0.04, 100, 1 << 4, 1 << 8, 1 << 9)
    for k in [(0, 0, 0), (1, 2, 3), (-5, 4, 2)]:
        vol.insert(*k)
    for k in [(0, 0, 1), (3, 2, 1), (-5, 4, 3), (16, 0, 0)]:
        assert vol.lookup(*k) == -1


@pytest.mark.parametrize("which", ["blocks", "excess"])
def test_capacity_exhaustion_flags(oracle_mod, which):
    if which == "blocks":
        vol = oracle_mod.Volume(0.01, 0.04, 100, 1 << 10, 1 << 8, 50)
        flag = 1
    else:
        vol = oracle_mod.Volume(0.01, 0.04, 100, 1 << 2, 10, 1 << 9)
        flag = 2
    keys = [(x, y, 0) for x in range(12) for y in range(12)]
    ok = [k for k in keys if vol.insert(*k) >= 0]
    assert vol.flags & flag
    pos, off, ptr = vol.entries()
    alloc = {tuple(p) for p in pos[ptr >= 0]}
    assert alloc == set(ok) and alloc <= set(keys)
    if which == "blocks":
        assert len(alloc) == 50 and vol.n_free_blocks == 0
    else:
        assert vol.n_free_excess == 0 and len(alloc) <= 4 + 10
    _check_structure(vol, ok)
