"""Random-number artefact screen of the HIP path (GPU twin of
tests/test_rng_artefacts.py).

With selection and reproduction off, every action is an exchange whose swap
does not look at the species, so the lattice stays i.i.d. uniform over
{0..S} at every MCS (the init draw included).  The screen runs at the
benchmark's lattice side on the persistent kernel and on a whole-lattice
LDS job, where tile seams, quad boundaries or per-workgroup streams would
show up as stripes or excess equal-neighbour pairs."""
import numpy as np
import pytest

from paper_2508_16639_amd import escg
from tests.gpu_util import host, pair
from tests.lattice_stats import screen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("L,S,route,moore", [(3200, 5, "persistent", False),
                                              (3200, 3, "persistent", True),
                                              (256, 3, "lds", False)])
def test_exchange_only_stays_iid(L, S, route, moore):
    K = [1, 3] if S == 5 else [1]
    p, _ = pair(L, S, K, 5.0, 0.0, 0.0, seed=21, replica=4, moore=moore,
                route=route)
    lat = torch.empty(L * L, dtype=torch.uint8, device="cuda:0")
    escg.init(p, lat)
    g = host(lat).reshape(L, L)
    assert screen(g, S + 1) == []
    t = 0
    for n in (1, 7, 24):
        escg.step_mcs(p, lat, t, n, None)
        t += n
        assert escg.last_route() == route
        g = host(lat).reshape(L, L)
        assert screen(g, S + 1) == [], (t, screen(g, S + 1))
