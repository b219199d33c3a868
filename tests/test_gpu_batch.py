"""Batches of independent spherically symmetric models (btx_batch_*).

Each model of a batch is checked against the FP64 reference (FP64 batches to
1e-12; mixed batches to 1e-5 in the per-zone number and energy moments) and
against the same model stepped alone with btx_step.  Graph replay is checked
against direct launches of the same steps, with host work and
synchronisations between the replays.  The full 64-model batch of uneven
sizes (100-600 radial zones, 12-24 groups, 16-48 directions) runs with the
autotuner and its cache file.
"""
import sys

import numpy as np
import pytest

from paper_2003_02845_amd import workloads as W

pytestmark = pytest.mark.gpu


def _btx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2003_02845_amd import btx
    return btx


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _models(n, scale, precision, seed):
    rng = np.random.default_rng(seed)
    ws = W.batch_models(n_models=n, size_scale=scale)
    for w in ws:
        w.precision = precision
        w.f0 = w.f0 * (1.0 + 0.3 * rng.random(w.f0.shape)) + 1e-3 * rng.random(w.f0.shape)
    return ws


def _batch(btx, ws, precision, **kw):
    import torch
    b = btx.Batch(ws, precision=precision, stream=torch.cuda.current_stream().cuda_stream, **kw)
    for m, w in enumerate(ws):
        b.set_background(m)
        b.set_state(m, w.f0)
    return b


def _single_shape(w):
    """the face shape a single context takes (8 work items per direction, the
    fewest groups per item of 3, 4, 5, 6, 8 covering the groups and three
    guard rows)"""
    return 8, min(c for c in (3, 4, 5, 6, 8) if 8 * c >= w.n_eps + 3)


def _moments_close(zg, zr, tol):
    for k in (0, 1):
        mask = np.abs(zr[..., 1]) > 1e-8 * np.abs(zr[..., 1]).max()
        rel = np.max(np.abs(zg[..., k] - zr[..., k])[mask] / np.abs(zr[..., k][mask]))
        assert rel <= tol, (k, rel)


def test_batch_fp64_matches_reference(oracle_mod):
    btx = _btx()
    ws = _models(5, 0.03, W.PREC_FP64, 21)
    _say(f"[gpu] fp64 batch of {len(ws)} models: " + ", ".join(f"{w.n_zones}x{w.block}" for w in ws))
    b = _batch(btx, ws, W.PREC_FP64)
    dts = [b.max_dt(m, 0.4) for m in range(len(ws))]
    b.step(dts, 3)
    for m, w in enumerate(ws):
        o = oracle_mod.Oracle(w)
        assert abs(o.max_dt(0.4) - dts[m]) <= 1e-13 * dts[m]
        o.step(dts[m], 3)
        ref, got = o.state(), b.get_state(m)
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        _say(f"[gpu]   model {m}: rel err {err:.3e}")
        assert err <= 1e-12
        zg, tg = b.moments(m)
        zr, tr = o.moments()
        assert np.allclose(tg, tr, rtol=1e-12, atol=1e-12 * np.abs(tr).max())
    b.close()


def test_batch_mixed_matches_single_contexts(oracle_mod):
    btx = _btx()
    import torch
    ws = _models(6, 0.05, W.PREC_MIXED, 22)
    _say(f"[gpu] mixed batch of {len(ws)} models vs single contexts")
    b = _batch(btx, ws, W.PREC_MIXED)
    dts = [b.max_dt(m, 0.4) for m in range(len(ws))]
    b.step(dts, 5)
    for m, w in enumerate(ws):
        c = btx.Context(w, precision=W.PREC_MIXED, stream=torch.cuda.current_stream().cuda_stream)
        c.set_background()
        c.set_state(w.f0)
        c.step(dts[m], 5)
        single, batched = c.get_state(), b.get_state(m)
        nch, ce = b.shape(m)
        err = float(np.max(np.abs(batched - single)) / np.max(np.abs(single)))
        _say(f"[gpu]   model {m}: shape {nch}x{ce}, batch vs single {err:.3e}")
        if (nch, ce) == _single_shape(w):  # the single context's own shape: same arithmetic
            assert err == 0.0
        else:
            assert err <= 1e-5
        o = oracle_mod.Oracle(w)
        o.step(dts[m], 5)
        zr, _ = o.moments()
        zg, _ = b.moments(m)
        _moments_close(zg, zr, 1e-5)
        c.close()
    b.close()


def test_batch_graph_replays_match_direct_launches(tmp_path):
    btx = _btx()
    ws = _models(4, 0.04, W.PREC_MIXED, 23)
    _say("[gpu] batch graph replays vs direct launches")
    cache = tmp_path / "tune.json"             # the second batch adopts the first one's tuning
    a = _batch(btx, ws, W.PREC_MIXED, tune_cache=cache)
    d = _batch(btx, ws, W.PREC_MIXED, tune_cache=cache)
    d.use_graph(False)
    dts = [a.max_dt(m, 0.4) for m in range(len(ws))]
    for rep in range(4):                    # one step per call, host reads in between
        a.step(dts, 1)
        d.step(dts, 1)
        for m in range(len(ws)):
            assert a.shape(m) == d.shape(m)
            assert np.array_equal(a.get_state(m), d.get_state(m)), (rep, m)
    a.step(dts, 3)
    d.step(dts, 3)
    for m in range(len(ws)):
        assert np.array_equal(a.get_state(m), d.get_state(m))
        _, ta = a.moments(m)
        _, td = d.moments(m)
        assert np.array_equal(ta, td)
    a.close()
    d.close()


def test_batch_time_level_graph_matches_direct_launches(tmp_path):
    """The time-level step replayed as a captured graph equals the same
    substeps launched directly, bit for bit, over several replays with host
    reads in between; new levels for a model make the graph be captured
    again, and it still agrees."""
    btx = _btx()
    ws = _models(4, 0.04, W.PREC_MIXED, 41)
    _say("[gpu] batch time-level graph vs direct launches")
    cache = tmp_path / "tune.json"
    a = _batch(btx, ws, W.PREC_MIXED, tune_cache=cache)
    d = _batch(btx, ws, W.PREC_MIXED, tune_cache=cache)
    d.use_graph(False)
    dts = [a.max_dt(m, 0.4) for m in range(len(ws))]
    for x in (a, d):
        x.set_time_levels(0, a.time_levels(0, 3))
        x.set_time_levels(2, a.time_levels(2, 1))
    for rep in range(3):
        a.step(dts, 1)
        d.step(dts, 1)
        for m in range(len(ws)):
            assert np.array_equal(a.get_state(m), d.get_state(m)), (rep, m)
    for x in (a, d):                            # the level lists change: a new graph
        x.set_time_levels(1, a.time_levels(1, 2))
        x.set_time_levels(0, None)
    a.step(dts, 2)
    d.step(dts, 2)
    for m in range(len(ws)):
        assert np.array_equal(a.get_state(m), d.get_state(m)), m
        _, ta = a.moments(m)
        _, td = d.moments(m)
        assert np.array_equal(ta, td)
    a.close()
    d.close()


def test_full_batch_100_steps(oracle_mod, tmp_path):
    """The whole 64-model batch for its 100 steps, tuned with the cache file:
    every model against the reference (per-zone number and energy moments,
    1e-5; number with the boundary outflow, 1e-5) and against the same model
    stepped alone (bit for bit where the tuner kept the single context's
    shape, else 1e-5 in the moments); a second batch reads the tuner's cache."""
    import torch
    from oracle import pool
    btx = _btx()
    ws = _models(64, 1.0, W.PREC_MIXED, 24)
    total = sum(w.n_values for w in ws)
    _say(f"[gpu] 64-model batch, {total:.3g} values, 100 steps")
    cache = tmp_path / "tune.json"
    b = _batch(btx, ws, W.PREC_MIXED, tune_cache=cache)
    dts = [b.max_dt(m, 0.4) for m in range(len(ws))]
    b.step(dts, 100)
    torch.cuda.synchronize()
    assert cache.exists()
    shapes = [b.shape(m) for m in range(len(ws))]
    _say(f"[gpu]   shapes {sorted(set(shapes))}; the reference in a pool of workers")
    ref = pool.moments_after(ws, dts, 100)
    worst = 0.0
    for m, w in enumerate(ws):
        zg, tg = b.moments(m)
        zr, tr = ref[m]
        _moments_close(zg, zr, 1e-5)
        assert abs(tg[0, 0] + tg[0, 1] - tr[0, 0] - tr[0, 1]) <= 1e-5 * tr[0, 0]
        c = btx.Context(w, precision=W.PREC_MIXED, stream=torch.cuda.current_stream().cuda_stream)
        c.set_background()
        c.set_state(w.f0)
        c.step(dts[m], 100)
        single = c.get_state()
        if tuple(shapes[m]) == _single_shape(w):
            assert np.array_equal(b.get_state(m), single), m
        else:
            zs, _ = c.moments()
            _moments_close(zg, zs, 1e-5)
        c.close()
        J = zr[..., 1]
        mask = np.abs(J) > 1e-8 * np.abs(J).max()
        worst = max(worst, float(np.max(np.abs(zg[..., 1] - J)[mask] / np.abs(J[mask]))))
    _say(f"[gpu]   all 64 models within {worst:.2e} of the reference in J")
    b.close()
    again = _batch(btx, ws, W.PREC_MIXED, tune_cache=cache)
    again.step(dts, 1)
    assert [again.shape(m) for m in range(len(ws))] == shapes
    again.close()


def test_batch_time_levels(oracle_mod):
    """Time levels in a batch: models with different highest levels (2, 1 and
    none) step 2^L substeps of their own dt per batch step; each model's state
    equals a single context stepping the same levels as many level-stepped
    steps (bit for bit where the batch kept the context's face shape, else to
    1e-12), and the first matches the reference (1e-12)."""
    import torch
    btx = _btx()
    ws = _models(3, 0.03, W.PREC_FP64, 31)
    b = _batch(btx, ws, W.PREC_FP64)
    dts = [b.max_dt(m, 0.4) for m in range(len(ws))]
    levs = [b.time_levels(0, 2), b.time_levels(1, 1), None]
    _say(f"[gpu] batch time levels: highest {[int(l.max()) if l is not None else 0 for l in levs]}")
    b.set_time_levels(0, levs[0])
    b.set_time_levels(1, levs[1])
    L = max(int(l.max()) for l in levs if l is not None)
    b.step(dts, 2)
    torch.cuda.synchronize()
    for m, w in enumerate(ws):
        c = btx.Context(w, precision=W.PREC_FP64, stream=torch.cuda.current_stream().cuda_stream)
        c.set_background()
        c.set_state(w.f0)
        lm = 0 if levs[m] is None else int(levs[m].max())
        if levs[m] is not None:
            c.set_time_levels(levs[m])
        c.step(dts[m], 2 * 2 ** (L - lm))
        got, single = b.get_state(m), c.get_state()
        if tuple(b.shape(m)) == _single_shape(w):   # the same shape: the same arithmetic
            assert np.array_equal(got, single), m
        else:                                        # angle sums in another order
            assert np.max(np.abs(got - single)) <= 1e-12 * np.max(np.abs(single)), m
        c.close()
    o = oracle_mod.Oracle(ws[0])
    o.set_levels(levs[0])
    o.step(dts[0], 2 * 2 ** (L - int(levs[0].max())))
    ref = o.state()
    err = np.max(np.abs(b.get_state(0) - ref)) / np.max(np.abs(ref))
    _say(f"[gpu]   model 0 against the reference: {err:.3e}")
    assert err <= 1e-12
    b.close()


def test_batch_time_levels_after_global_steps(oracle_mod):
    """Time levels set on a batch that has already stepped (its face launches
    then grouped by shape and workgroup size, regrouped by shape alone): one
    global step, then one level-stepped step; each model equals a single
    context doing the same (bit for bit where the batch kept the context's
    face shape, else to 1e-12)."""
    import torch
    btx = _btx()
    ws = _models(5, 0.03, W.PREC_FP64, 37)           # models 0-2 and 4 share a shape, 4 a smaller workgroup
    b = _batch(btx, ws, W.PREC_FP64)
    dts = [b.max_dt(m, 0.4) for m in range(len(ws))]
    _say("[gpu] batch time levels after global steps")
    b.step(dts, 1)
    levs = [b.time_levels(0, 2), None, b.time_levels(2, 1), None, b.time_levels(4, 1)]
    for m in (0, 2, 4):
        b.set_time_levels(m, levs[m])
    L = max(int(l.max()) for l in levs if l is not None)
    b.step(dts, 1)
    torch.cuda.synchronize()
    for m, w in enumerate(ws):
        c = btx.Context(w, precision=W.PREC_FP64, stream=torch.cuda.current_stream().cuda_stream)
        c.set_background()
        c.set_state(w.f0)
        c.step(dts[m], 1)
        lm = 0 if levs[m] is None else int(levs[m].max())
        if levs[m] is not None:
            c.set_time_levels(levs[m])
        c.step(dts[m], 2 ** (L - lm))
        got, single = b.get_state(m), c.get_state()
        if tuple(b.shape(m)) == _single_shape(w):
            assert np.array_equal(got, single), m
        else:
            assert np.max(np.abs(got - single)) <= 1e-12 * np.max(np.abs(single)), m
        c.close()
    b.close()
