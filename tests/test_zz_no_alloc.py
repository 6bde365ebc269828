"""GPU test of rbffd_weights_noalloc, the weights entry point for callers
that cannot allocate device memory: its results against rbffd_weights'
(the same kernels: bit for bit) on two calls in a row, the second with a
smaller input, and its size limit (EINVAL, nothing written)."""

import numpy as np
import pytest

from workloads import weights_config

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _outputs(nc, n_max, n_ops, fill):
    import torch
    return (torch.full((nc, n_max), -77, dtype=torch.int32, device="cuda"),
            torch.full((n_ops, nc, n_max), fill, dtype=torch.float64, device="cuda"),
            torch.full((nc,), 99, dtype=torch.int32, device="cuda"))


def test_noalloc_weights_equal_the_allocating_entry_point():
    import torch
    from paper_1509_02615_amd import rbffd as R
    ctx = R.Context(0)
    ops = [(R.DX, 0, 0), (R.DZ, 0, 0), (R.HYPERLAP, 0, 0)]
    for side, precision, given in ((48, R.SOLVE_FP64, False), (20, R.SOLVE_FP32_IR, True)):
        cfg = weights_config(side, seed=side)
        nd = cfg["nodes"]
        nc = nd.n_active
        say(f"noalloc: {side}x{side} mixed batch ({nc} stencils, n_max {cfg['n_max']}), precision {precision}, "
            f"{'given stencils' if given else 'with the search'}")
        xy = torch.from_numpy(nd.xy).cuda()
        kw = dict(n_per=torch.from_numpy(cfg["n_per"]).cuda(), m_per=torch.from_numpy(cfg["m_per"]).cuda(),
                  l_per=torch.from_numpy(cfg["l_per"]).cuda(), precision=precision)
        ref_idx, ref_w, ref_s, ref_rc = R.rbffd_weights(ctx, xy, ops, cfg["n_max"], **kw)
        if given:
            kw["idx_in"] = ref_idx
        out = _outputs(nc, cfg["n_max"], len(ops), float("nan"))
        idx, w, status, rc = R.rbffd_weights_noalloc(ctx, xy, ops, cfg["n_max"], out, **kw)
        torch.cuda.synchronize()
        assert rc == ref_rc == R.OK
        if given:   # no idx output requested: the sentinels stay
            assert bool((idx == -77).all())
        else:
            assert torch.equal(idx, ref_idx)
        assert torch.equal(status, ref_s)
        assert torch.equal(w, ref_w)        # the same kernels in the same order: bit for bit
        say(f"   equal bit for bit; status counts {torch.bincount(status).tolist()}")


def test_noalloc_limit_writes_nothing():
    import torch
    from paper_1509_02615_amd import rbffd as R
    ctx = R.Context(0)
    say(f"noalloc: {R.NOALLOC_MAX_NODES + 1} nodes -> EINVAL, outputs untouched")
    rng = np.random.default_rng(0)
    xy = torch.from_numpy(rng.uniform(0, 1, (R.NOALLOC_MAX_NODES + 1, 2))).cuda()
    out = _outputs(8, 21, 1, 5.0)
    with pytest.raises(R.RbffdError) as e:
        R.rbffd_weights_noalloc(ctx, xy, [(R.DX, 0, 0)], 21, out, m=3, l=3, n_centers=8)
    assert e.value.code == R.EINVAL
    assert bool((out[0] == -77).all()) and bool((out[1] == 5.0).all()) and bool((out[2] == 99).all())
