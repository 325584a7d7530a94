"""Every launch choice in the autotuner's cache for this device gives the
same bytes as the library's default choice (and, for a short run, as the
oracle): tuning changes speed, never results."""
import numpy as np
import pytest

import oracle as O
from paper_2508_16639_amd import autotune, escg
from paper_2508_16639_amd.workloads import random_lattice
from tests.gpu_util import dev, host, pair

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _records():
    if not torch.cuda.is_available():
        return []
    dk = autotune.device_key(torch)
    return sorted((k, v) for k, v in autotune.load_cache().items()
                  if k.startswith(dk + "|"))


def _parse(k):
    _, _, kernel, side, scls = k.split("|")
    return kernel, side[2:], scls.endswith("=1")


def test_cache_has_entries_for_this_device():
    kinds = {_parse(k)[0] for k, _ in _records()}
    assert {"persistent", "multi", "batch"} <= kinds, kinds


@pytest.mark.parametrize("k,rec", _records(), ids=[k for k, _ in _records()])
def test_tuned_choice_gives_default_bytes(k, rec):
    kernel, side, small = _parse(k)
    kw = autotune.launch_choice(rec)
    S, K = (3, [1]) if small else (9, [1, 2, 4])
    if kernel == "batch":
        sides = [int(x) for x in side.split(",")]
        specs = [(sides[i % len(sides)], i) for i in range(12)]
        ps, offs, off = [], [], 0
        for L, i in specs:
            ps.append(escg.Params(L=L, S=S, dom=escg.circulant_dom(S, K),
                                  ex=float(escg.eps_from_mobility(1e-3, L)),
                                  seed=5, replica=i))
            offs.append(off)
            off += L * L
        outs = []
        for first in (ps[0], ps[0].with_launch(**kw)):
            buf = torch.zeros(off, dtype=torch.uint8, device="cuda:0")
            res = torch.empty(len(ps) * escg.BATCH_RESULT_WORDS,
                              dtype=torch.int32, device="cuda:0")
            escg.batch_run([first] + ps[1:], offs, buf, [40] * len(ps),
                           escg.STOP_NONE, True, res)
            outs.append((host(buf), host(res)))
        assert np.array_equal(outs[0][0], outs[1][0])
        assert np.array_equal(outs[0][1], outs[1][1])
        return
    L = int(side)
    n = 3
    p, j = pair(L, S, K, float(escg.eps_from_mobility(1e-4, L)), seed=L,
                replica=1)
    g0 = random_lattice(L, S, seed=L + 3, domain=3)
    ref = g0.copy()
    O.o2_run(j, ref, 5, n, want_counts=False)
    if kernel == "multi":
        lats = [dev(g0), dev(g0)]
        escg.step_batch([p.with_launch(**kw)], [lats[0]], [5], [n])
        assert escg.last_route() == "persistent"
        escg.step_batch([p.with_launch(route="tiled")], [lats[1]], [5], [n])
        got = [host(t) for t in lats]
    else:
        route = "persistent" if kernel == "persistent" else "tiled"
        got = []
        for q in (p.with_launch(route=route, **kw), p.with_launch(route=route)):
            lat = dev(g0)
            escg.step_mcs(q, lat, 5, n, None)
            assert escg.last_route() == route
            got.append(host(lat))
    assert np.array_equal(got[0], got[1])
    assert np.array_equal(got[0], ref)
    escg.async_status()
