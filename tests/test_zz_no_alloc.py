"""btx_moments_device, the moments entry point for callers that cannot allocate
(its partial results live in a fixed device array), against btx_moments: two
calls in a row on the same GPU, the second on a smaller grid, plus the size
limit of the array."""
import numpy as np
import pytest

from paper_2003_02845_amd import btx, workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _stepped(w, precision, steps=2):
    ctx = btx.Context(w, device=0, stream=torch.cuda.current_stream().cuda_stream, precision=precision)
    ctx.set_background()
    dtype = np.float64 if precision == W.PREC_FP64 else np.float32
    ctx.set_state(np.ascontiguousarray(w.f0, dtype=dtype))
    ctx.step(ctx.max_dt(w.cfl), steps)
    return ctx


def _compare(ctx, w):
    print(f"[no_alloc] {w.name}: {w.n_zones} zones x {w.n_species} species", flush=True)
    zm_ref, tot_ref = ctx.moments()
    zm = torch.full((w.n_zones, w.n_species, 5), float("nan"), dtype=torch.float64, device="cuda")
    tot = torch.full((w.n_species, 3), float("nan"), dtype=torch.float64, device="cuda")
    ctx.moments_device(zm, tot)
    torch.cuda.synchronize()
    zm_h, tot_h = zm.cpu().numpy(), tot.cpu().numpy()
    # the zone moments come from the same kernel: bit for bit
    assert np.array_equal(zm_h, zm_ref)
    # the totals are compensated sums in another order: FP64 rounding level
    scale = np.maximum(np.abs(tot_ref), 1e-300)
    err = np.max(np.abs(tot_h - tot_ref) / scale)
    assert err <= 1e-12, err
    # totals alone (the zone moments then go to the fixed array as well)
    tot2 = torch.full((w.n_species, 3), float("nan"), dtype=torch.float64, device="cuda")
    ctx.moments_device(None, tot2)
    torch.cuda.synchronize()
    assert np.array_equal(tot2.cpu().numpy(), tot_h)
    return tot_h


def test_moments_device_matches_moments_two_calls_second_smaller():
    big = W.shock_2d(n_r=40, n_theta=16, n_eps=8, n_mu=6, n_phi=4, precision=W.PREC_FP64)
    small = W.shock_2d(n_r=12, n_theta=4, n_eps=5, n_mu=4, n_phi=4, precision=W.PREC_FP64)
    assert small.n_zones * small.n_species < big.n_zones * big.n_species
    c1 = _stepped(big, W.PREC_FP64)
    _compare(c1, big)
    c2 = _stepped(small, W.PREC_FP64)
    _compare(c2, small)
    # the first context again, after the smaller one left its values in the array
    _compare(c1, big)
    c1.close()
    c2.close()


def test_moments_device_mixed_precision_and_boundary_tally():
    w = W.shock_2d(n_r=24, n_theta=8, n_eps=6, n_mu=6, n_phi=4, precision=W.PREC_MIXED)
    ctx = _stepped(w, W.PREC_MIXED, steps=3)
    tot = _compare(ctx, w)
    assert np.all(tot[:, 1] != 0.0)            # content has left through the outer boundary
    ctx.close()


def test_moments_device_rejects_grids_beyond_the_array():
    # 1100 x 160 zones x 3 species = 528000 pairs > 524288
    w = W.shock_2d(n_r=1100, n_theta=160, n_eps=2, n_mu=2, n_phi=1, precision=W.PREC_FP64)
    w.phi_rule = W.PHI_LINEAR
    ctx = btx.Context(w, device=0, stream=torch.cuda.current_stream().cuda_stream)
    tot = torch.zeros((w.n_species, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(btx.BtxError) as e:
        ctx.moments_device(None, tot)
    assert e.value.status == btx.BTX_E_UNSUPPORTED
    ctx.close()
