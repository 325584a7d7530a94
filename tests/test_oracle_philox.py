"""Pins of the oracle's Philox4x32 (Salmon et al., SC'11, Sec. 4) against
values fixed outside this repository: the published known-answer vectors and
rocRAND's independent engine."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_kat.txt")


def _kat_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            rounds = int(tok[0])
            vals = [int(x, 16) for x in tok[1:]]
            rows.append((rounds, vals[0:4], vals[4:6], vals[6:10]))
    return rows


@pytest.mark.parametrize("rounds,ctr,key,expect", _kat_rows())
def test_philox_known_answers(rounds, ctr, key, expect):
    assert list(O.philox4x32(ctr, key, rounds)) == expect


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox_probe.cpp")
    exe = str(tmp_path_factory.mktemp("rr") / "probe")
    subprocess.check_call([hipcc, "-O1", src, "-o", exe])
    return exe


def test_philox_matches_rocrand_engine(rocrand_probe):
    rng = np.random.default_rng(12345)
    for i in range(24):
        key = int(rng.integers(0, 2**63)) * (1 + (i & 1))
        ctr = [int(rng.integers(0, 2**32)), int(rng.integers(0, 2**30)),
               int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))]
        out = subprocess.check_output(
            [rocrand_probe, hex(key)] + [hex(c) for c in ctr]).decode().split()
        ref = [int(x, 16) for x in out]
        mine = O.philox4x32(ctr, [key & 0xFFFFFFFF, key >> 32], 10)
        assert list(mine) == ref, (key, ctr)


def test_philox_words_uniform():
    # Output bits of consecutive counters are balanced (a dropped round or a
    # swapped multiplier keeps this, but a wrong word order/xor often not).
    words = np.array([O.philox4x32([i, 7, 3 << 8, 0], [1, 0], 10)
                      for i in range(4096)], dtype=np.uint64).reshape(-1)
    bits = ((words[:, None] >> np.arange(32, dtype=np.uint64)) & 1).mean(0)
    assert np.all(np.abs(bits - 0.5) < 0.02)


def test_schedule_round_count_has_published_vectors():
    # the block schedule draws Philox4x32 with O.SCHEDULE_ROUNDS rounds: the
    # published known-answer file covers that round count, so the
    # generator the schedule uses is pinned, not only the 10-round default
    assert O.SCHEDULE_ROUNDS in {r for r, _, _, _ in _kat_rows()}
    assert O.Job(2, 1, np.zeros((1, 1), np.uint8), 1.0).rounds == \
        O.SCHEDULE_ROUNDS
