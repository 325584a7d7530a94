"""Helpers shared by the GPU tests: build matching (library, oracle) jobs from
one description, and move arrays between numpy and the device."""
import numpy as np

import oracle as O
from paper_2508_16639_amd import escg


# The kernel path the next pair() jobs ask for ("auto", "lds", "tiled" or
# "persistent"; set by the tests' route_to).  It travels in each job's
# launch choices, per call: the library holds no routing state.
ROUTE = ["auto"]


def launch_route(L, route):
    """The route a job of side L is given for a test route: the persistent
    kernel needs L % 8 == 0, so such tests run other sides per MCS."""
    if route == "persistent" and (L % 8 or L < 16):
        return "tiled"
    return route


def pair(L, S, K, ex, sel=1.0, rep=1.0, seed=1, replica=0, D=None,
         moore=False, P=None, route=None):
    """The same job for the HIP library (escg.Params) and the oracle."""
    if D is None:
        D = O.circulant_matrix(S, K) if K else np.zeros((S, S), np.uint8)
    p = escg.Params(L=L, S=S, dom=escg.dom_from_matrix(D), ex=ex, sel=sel,
                    rep=rep, seed=seed, replica=replica, moore=moore, prob=P,
                    route=launch_route(L, route or ROUTE[0]))
    j = O.Job(L, S, D, ex, sel, rep, seed=seed, replica=replica,
              nbhd=8 if moore else 4, P=P)
    return p, j


def probabilities(D, seed=0):
    """Seeded dominance probabilities on the edges of D (zeros elsewhere),
    some at the ends 0 and 1."""
    rng = np.random.default_rng(seed)
    P = rng.uniform(0.05, 0.95, size=D.shape) * (D != 0)
    P[(D != 0) & (rng.random(D.shape) < 0.15)] = 1.0
    P[(D != 0) & (rng.random(D.shape) < 0.1)] = 0.0
    return P


def dev(a, device="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def host(t):
    import torch
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a.view(np.uint32) if a.dtype == np.int32 else a
