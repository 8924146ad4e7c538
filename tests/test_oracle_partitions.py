"""Pins of the oracle's partition-aware ML helpers (the per-partition P_ML
comparison proposed with the results of Sec. IV-C; partitions as the static
nnz-balanced row partitioning of Sec. IV-A, taken over row blocks)."""
import numpy as np

import oracle


def rp_of(lengths):
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)


def test_uniform_rows_split_evenly():
    # 64 rows of 5 nonzeros, 4 rows per block -> 16 blocks of 20; Q = 8
    # partitions of exactly 2 blocks each (closed form q * 16 / 8).
    b = oracle.ml_partition_bounds(rp_of([5] * 64), 4, 8)
    assert b.tolist() == [2 * q for q in range(9)]


def test_one_heavy_block_leaves_empty_partitions():
    # block 0 holds 700 of 1,000 nonzeros (rows of 175), blocks 1..3 hold 100
    # each; Q = 10 targets 0, 100, ..., 900: targets 100..700 all land on
    # block 1 (first nonzero 700), 800 on block 2, 900 on block 3.
    lengths = [175] * 4 + [25] * 12
    b = oracle.ml_partition_bounds(rp_of(lengths), 4, 10)
    assert b.tolist() == [0, 1, 1, 1, 1, 1, 1, 1, 2, 3, 4]
    nonempty = int(np.sum(np.diff(b) > 0))
    assert nonempty == 4


def test_no_nonzeros_is_one_partition():
    b = oracle.ml_partition_bounds(np.zeros(11, dtype=np.int32), 4, 5)
    assert b.tolist() == [0, 0, 0, 0, 0, 3]


def test_ragged_last_block_and_trailing_empty_rows():
    # 10 rows, 4 per block -> 3 blocks (4, 4, 2 rows); all nonzeros in rows 0..3
    b = oracle.ml_partition_bounds(rp_of([3, 3, 3, 3] + [0] * 6), 4, 3)
    assert b.tolist() == [0, 1, 1, 3]


def test_partition_nonzeros_are_balanced():
    # invariants on a random matrix: monotone, first/last fixed, and every
    # partition starts at the first block reaching its share of nonzeros
    rng = np.random.default_rng(7)
    lengths = rng.integers(0, 40, size=1000)
    rp = rp_of(lengths)
    NG, Q = 8, 16
    b = oracle.ml_partition_bounds(rp, NG, Q)
    nblk = -(-1000 // NG)
    assert b[0] == 0 and b[-1] == nblk and np.all(np.diff(b) >= 0)
    firsts = np.array([rp[min(k * NG, 1000)] for k in range(nblk + 1)])
    nnz = int(rp[-1])
    for q in range(1, Q):
        t = q * nnz // Q
        assert firsts[b[q]] >= t
        assert b[q] == 0 or firsts[b[q] - 1] < t
    # each partition's nonzeros stay within nnz/Q plus one block's worth
    blk = np.diff(firsts)
    for q in range(Q):
        assert blk[b[q]:b[q + 1]].sum() <= nnz / Q + blk.max() + 1


def test_ratios_by_hand():
    bounds = np.array([0, 2, 2, 5])
    base = np.array([10, 30, 5, 5, 10])
    probe = np.array([5, 15, 10, 10, 0])
    r = oracle.ml_partition_ratios(base, probe, bounds)
    assert r.tolist() == [2.0, 0.0, 1.0]
    assert oracle.ml_partition_ratios(base, np.zeros(5), bounds).tolist() == [0.0, 0.0, 0.0]
