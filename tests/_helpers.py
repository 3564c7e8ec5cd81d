"""Small helpers shared by the tests (no method arithmetic)."""
import numpy as np

from paper_1701_07452_amd import inputs as I


def oracle_sim(G, q, b, **kw):
    from oracle import OracleSim, default_params
    P = default_params(**kw)
    sim = OracleSim(P, G.descs)
    for ip, (qp, bp) in enumerate(I.split(G, q, b)):
        sim.set_state(ip, qp, bp)
    return sim


def oracle_gather(G, sim):
    return I.gather(G, [sim.get_state(i) for i in range(G.npatch)])


def l1_norm(err):
    e = np.abs(err).mean(axis=tuple(range(1, err.ndim)))
    return float(np.sqrt((e ** 2).sum()))
