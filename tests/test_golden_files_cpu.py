"""The full-length oracle references under tests/golden/ (written by
tests/golden/make_full_length.py from the oracle only): their shape, that
every count row sums to the number of sites, and that their first rows are
what the oracle gives now (init counts and the first MCS), so a stale file
is caught on the CPU before the GPU tests compare against it."""
import numpy as np
import pytest

import oracle as O
from paper_2508_16639_amd.workloads import RPS512, RPSLS3200
from tests.golden import make_full_length as golden


@pytest.mark.parametrize("w,fname,n_check", [
    (RPS512, "rps_L512_10000mcs.txt", 5),
    (RPSLS3200, "rpsls_L3200_1000mcs.txt", 1)])
def test_golden_full_length_file(w, fname, n_check):
    rows, sha, hdr = golden.read(fname)
    assert rows.shape == (w.mcs + 1, w.S + 1)
    assert (rows.sum(1, dtype=np.uint64) == w.L * w.L).all()
    assert sha is not None and len(sha) == 64
    job = O.Job(w.L, w.S, O.circulant_matrix(w.S, w.K), w.ex, w.sel, w.rep,
                seed=w.seed, replica=w.replica)
    assert hdr["rounds"] == job.rounds
    g = job.init()
    c = O.o2_run(job, g, 0, n_check)
    assert np.array_equal(rows[:n_check + 1], c)
