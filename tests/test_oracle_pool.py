"""The reference's worker pool (used by the GPU tests of many models) gives
the same moments as in-process runs, bit for bit."""
import numpy as np

from paper_2003_02845_amd import workloads as W


def test_pool_matches_in_process(oracle_mod):
    from oracle import pool
    ws = W.batch_models(n_models=3, size_scale=0.04)
    dts = []
    ref = []
    for w in ws:
        o = oracle_mod.Oracle(w)
        dt = o.max_dt(0.4)
        dts.append(dt)
        o.step(dt, 3)
        ref.append(o.moments())
    got = pool.moments_after(ws, dts, 3, processes=2)
    for (zg, tg), (zr, tr) in zip(got, ref):
        assert np.array_equal(zg, zr) and np.array_equal(tg, tr)
