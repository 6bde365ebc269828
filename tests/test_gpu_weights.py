"""GPU parity of the stencil search (bit-exact) and the batched weights
(<= 1e-10 norm-wise per stencil and operator) against the CPU oracle,
called through the C ABI."""

import numpy as np
import pytest

import oracle as O
from workloads import (advection_config, density_current_config, weights_config, unit_square_cartesian,
                       channel, jittered_square)

pytestmark = pytest.mark.gpu
TOL_W = 1e-10


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1509_02615_amd import rbffd
    return rbffd


@pytest.fixture(scope="module")
def ctx(R):
    return R.Context(0)


def dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)


def _knn_case(R, ctx, xy, n, period, centers=None, n_per=None, sample=None):
    import torch
    c_t = dev(centers, torch.int32) if centers is not None else None
    np_t = dev(n_per, torch.int32) if n_per is not None else None
    got = host(R.rbffd_knn(ctx, dev(xy, torch.float64), n, period, centers=c_t, n_per=np_t,
                           n_centers=None if centers is not None else xy.shape[0]))
    cs = np.arange(got.shape[0]) if sample is None else sample
    for a in cs:
        c = int(centers[a]) if centers is not None else int(a)
        na = int(n_per[a]) if n_per is not None else n
        ref = O.knn(xy, [c], na, period)[0]
        assert np.array_equal(got[a, :na], ref), (a, got[a, :na], ref)
        assert np.all(got[a, na:] == -1)
    return got


def test_knn_bit_exact_unit_square(R, ctx):
    say("knn: 64x64 Cartesian, n=37, all centres")
    nd = unit_square_cartesian(64)
    _knn_case(R, ctx, nd.xy, 37, 0.0)


@pytest.mark.parametrize("layout", ["cartesian", "hexagonal", "scattered"])
def test_knn_bit_exact_channels(R, ctx, layout):
    say(f"knn: {layout} 400 m channel, periodic x, all centres incl. walls")
    nd = density_current_config(layout, 400.0)["nodes"]
    _knn_case(R, ctx, nd.xy, 37, nd.period_x, centers=np.arange(nd.n_active))


def test_knn_bit_exact_full_size_samples(R, ctx):
    say("knn: 100 m hexagonal channel (38,400 + ghosts), 300 sampled centres; 1M scattered, 100 samples")
    nd = density_current_config("hexagonal", 100.0)["nodes"]
    rng = np.random.default_rng(7)
    centers = np.arange(nd.n_active)
    samp = np.concatenate([rng.choice(nd.n_active, 250, replace=False), np.arange(25), nd.n_active - 1 - np.arange(25)])
    _knn_case(R, ctx, nd.xy, 37, nd.period_x, centers=centers, sample=samp)
    cfg = weights_config(1024)
    nd = cfg["nodes"]
    samp = np.concatenate([rng.choice(nd.n_active, 90, replace=False), [0, 1023, nd.n_active - 1]])
    _knn_case(R, ctx, nd.xy, cfg["n_max"], 0.0, centers=np.arange(nd.n_active), n_per=cfg["n_per"], sample=samp)


def test_knn_edge_cases(R, ctx):
    say("knn: edge cases (n = N, n = 1, ragged n_per, centre subset, duplicate distances)")
    rng = np.random.default_rng(3)
    xy = rng.uniform(0, 1, (50, 2))
    _knn_case(R, ctx, xy, 50, 0.0)                      # whole set
    _knn_case(R, ctx, xy, 1, 0.0)                       # the centre itself
    nd = channel("cartesian", 16, 5, 0.0, 16.0, 4.0)    # unit lattice, periodic: heavy ties
    n_per = rng.integers(1, 26, nd.n_active).astype(np.int32)
    _knn_case(R, ctx, nd.xy, 25, nd.period_x, centers=np.arange(nd.n_active)[::-1].copy(), n_per=n_per)
    with pytest.raises(R.RbffdError):
        R.rbffd_knn(ctx, dev(xy, __import__("torch").float64), 51, 0.0)


def _weights_parity(R, ctx, xy, ops_o, n, m, l, period, centers, sample=None, n_per=None, m_per=None,
                    l_per=None, precision=0):
    import torch
    ops = [(k, kk, mo) for (k, kk, mo) in ops_o]
    idx, W, status, rc = R.rbffd_weights(
        ctx, dev(xy, torch.float64), ops, n, m, l, period_x=period, centers=dev(centers, torch.int32),
        n_per=None if n_per is None else dev(n_per, torch.int32),
        m_per=None if m_per is None else dev(m_per, torch.int32),
        l_per=None if l_per is None else dev(l_per, torch.int32), precision=precision)
    idx, W, status = host(idx), host(W), host(status)
    # 3: solved again in FP64 after the FP32 factorisation's refinement stalled
    assert rc == R.OK and np.all((status == 0) | ((status == 3) & (precision == 1)))
    cs = range(len(centers)) if sample is None else sample
    worst = 0.0
    for a in cs:
        c = int(centers[a])
        na = int(n_per[a]) if n_per is not None else n
        ma = int(m_per[a]) if m_per is not None else m
        la = int(l_per[a]) if l_per is not None else l
        st = O.knn(xy, [c], na, period)[0]
        assert np.array_equal(idx[a, :na], st)
        Wo, so = O.stencil_weights(xy, st, c, ma, la, ops_o, period)
        assert so == 0
        for o in range(len(ops)):
            err = np.linalg.norm(W[o, a, :na] - Wo[o]) / np.linalg.norm(Wo[o])
            worst = max(worst, err)
            assert err <= TOL_W, (a, o, err)
            assert np.all(W[o, a, na:] == 0.0)
    say(f"   worst norm-wise relative weight error {worst:.2e}")
    return W


def test_weights_parity_unit_square(R, ctx):
    say("weights: 64x64 Cartesian, r^5 + deg 4 (Dx, Dy) and r^7 Lap^3, all 4096 stencils")
    cfg = advection_config(64)
    nd = cfg["nodes"]
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.HYPERLAP, 3, 7)]
    _weights_parity(R, ctx, nd.xy, ops, 37, 5, 4, 0.0, np.arange(nd.n_active))


@pytest.mark.parametrize("layout", ["cartesian", "hexagonal", "scattered"])
def test_weights_parity_channels(R, ctx, layout):
    say(f"weights: {layout} 400 m channel, r^7 + deg 4, Dx Dz Lap Lap^3 and wall Dz Dzz")
    nd = density_current_config(layout, 400.0)["nodes"]
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.LAP, 0, 0), (O.HYPERLAP, 3, 7)]
    _weights_parity(R, ctx, nd.xy, ops, 37, 7, 4, nd.period_x, np.arange(nd.n_active))
    _weights_parity(R, ctx, nd.xy, [(O.DZ, 0, 0), (O.DZZ, 0, 0)], 37, 7, 4, nd.period_x, nd.wall_nodes.ravel())


def test_empty_batch_and_largest_system(R, ctx):
    """Edge sizes: an empty batch of centres is a no-op for the search and
    the weights; the largest system the library takes (n = 100, degree 6,
    K = 128) matches the oracle on scattered nodes."""
    import torch
    say("weights: empty batch; K = 128 systems (n = 100, l = 6, r^7) on a jittered 24x24 square")
    nd = jittered_square(24, seed=6)
    xy = dev(nd.xy, torch.float64)
    idx = R.rbffd_knn(ctx, xy, 37, 0.0, centers=dev(np.zeros(0, np.int32), torch.int32))
    assert tuple(idx.shape) == (0, 37)
    idx, W, status, rc = R.rbffd_weights(ctx, xy, [(O.DX, 0, 0)], 37, 7, 4,
                                         centers=dev(np.zeros(0, np.int32), torch.int32))
    assert rc == R.OK and W.numel() == 0
    centers = np.array([0, 11, 300, 575, 290], np.int32)     # corner, edge, interior, corner, interior
    _weights_parity(R, ctx, nd.xy, [(O.DX, 0, 0), (O.LAP, 0, 0), (O.HYPERLAP, 3, 0)], 100, 7, 6, 0.0, centers)


@pytest.mark.parametrize("layout", ["cartesian", "hexagonal", "scattered"])
def test_weights_parity_box(R, ctx, layout):
    """The closed box of the rising bubble (Section 6.5): interior operators,
    and Dx, Dxx at the lateral boundary rows (corners included)."""
    from workloads import bubble_config
    say(f"weights: {layout} 400 m box, r^7 + deg 4, Dx Dz Lap Lap^3 and lateral-wall Dx Dxx")
    nd = bubble_config(layout, 400.0)["nodes"]
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.LAP, 0, 0), (O.HYPERLAP, 3, 7)]
    _weights_parity(R, ctx, nd.xy, ops, 37, 7, 4, 0.0, np.arange(nd.n_active))
    lateral = nd.bnd_nodes[nd.bnd_normal == 1]
    _weights_parity(R, ctx, nd.xy, [(O.DX, 0, 0), (O.DXX, 0, 0)], 37, 7, 4, 0.0, lateral)


@pytest.mark.parametrize("precision", [0, 1])
def test_weights_parity_mixed_batch(R, ctx, precision):
    say(f"weights: mixed n/m/l batch on 40x40 jittered square, precision {precision}")
    cfg = weights_config(40, seed=5)
    nd = cfg["nodes"]
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.HYPERLAP, 0, 0)]
    _weights_parity(R, ctx, nd.xy, ops, cfg["n_max"], 0, 0, 0.0, np.arange(nd.n_active),
                    n_per=cfg["n_per"], m_per=cfg["m_per"], l_per=cfg["l_per"], precision=precision)


def test_weights_parity_parameter_sweep(R, ctx):
    """PHS orders 3..13 with their default hyperviscosity order (Lap^((m-1)/2)),
    polynomial degrees 2..6 and stencils of 13..60 nodes mixed in one batch,
    so that every system-size bucket runs (K = 19..88: the three one-
    wavefront capacities and the block kernel); then r^1 with linear
    polynomials (Section 3, Eq. weights). Every combination is well posed by
    the oracle."""
    say("weights: m = 3..13, l = 2..6, n = 13..60 mixed in one batch; then r^1, degree 1")
    nd = jittered_square(24, seed=4)
    combos = [(3, 2, 13), (3, 3, 21), (5, 2, 16), (9, 4, 30), (9, 3, 26), (11, 5, 40), (7, 5, 43),
              (13, 6, 60), (5, 4, 49)]
    N = nd.n_active
    pick = np.arange(N) % len(combos)
    m_per = np.array([combos[p][0] for p in pick], np.int32)
    l_per = np.array([combos[p][1] for p in pick], np.int32)
    n_per = np.array([combos[p][2] for p in pick], np.int32)
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.LAP, 0, 0), (O.HYPERLAP, 0, 0)]
    _weights_parity(R, ctx, nd.xy, ops, int(n_per.max()), 0, 0, 0.0, np.arange(N), sample=np.arange(0, N, 5),
                    n_per=n_per, m_per=m_per, l_per=l_per)
    _weights_parity(R, ctx, nd.xy, ops[:3], 7, 1, 1, 0.0, np.arange(N), sample=np.arange(0, N, 11))


@pytest.mark.parametrize("precision", [0, 1])
def test_weights_parity_small_systems(R, ctx, precision):
    """The smallest systems, K = 3..21 (polynomial degree 0..3 with n from M
    to a few nodes more), odd and even K mixed in one batch: the wavefront
    kernels' elimination takes two steps per pass, and an odd K ends on a
    single step. Every combination is well posed at every centre of this
    node set (cubics on exactly n = M = 10 scattered nodes are not: near
    the edges some of those stencils are singular, so the cubic systems
    here take 11 nodes), and each operator's weights are non-zero."""
    say("weights: K = 3..21, m = 3..7, l = 0..3, mixed in one batch")
    nd = jittered_square(16, seed=7)
    combos = [(3, 0, 2), (3, 0, 3), (5, 0, 4), (3, 1, 4), (3, 1, 5), (5, 1, 6), (5, 2, 6), (5, 2, 7),
              (7, 2, 9), (7, 3, 11)]
    # interior centres: on the square's edges the nodes are collinear, and a
    # two- or three-node stencil there has exactly zero weights for one
    # derivative
    x, z = nd.xy[:nd.n_active, 0], nd.xy[:nd.n_active, 1]
    centers = np.flatnonzero((x > 0.2) & (x < 0.8) & (z > 0.2) & (z < 0.8))
    pick = np.arange(len(centers)) % len(combos)
    m_per = np.array([combos[p][0] for p in pick], np.int32)
    l_per = np.array([combos[p][1] for p in pick], np.int32)
    n_per = np.array([combos[p][2] for p in pick], np.int32)
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.LAP, 0, 0)]
    _weights_parity(R, ctx, nd.xy, ops, int(n_per.max()), 0, 0, 0.0, centers, n_per=n_per, m_per=m_per,
                    l_per=l_per, precision=precision)


def test_singular_stencils_match_the_oracle(R, ctx):
    """Cubics on exactly n = M = 10 scattered nodes: near the edges of the
    node set some of these stencils are singular (the nodes do not determine
    a cubic). The GPU flags exactly the stencils the oracle flags (status 1;
    bit-exact, integer), and the others agree with the oracle's weights."""
    import torch
    say("weights: r^7 + cubics on n = M = 10 nodes, singular stencils flagged as by the oracle")
    nd = jittered_square(12, seed=7)
    N = nd.n_active
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.LAP, 0, 0)]
    idx, W, status, rc = R.rbffd_weights(ctx, dev(nd.xy, torch.float64), ops, 10, 7, 3)
    idx, W, status = host(idx), host(W), host(status)
    want = np.zeros(N, np.int32)
    worst = 0.0
    for c in range(N):
        st = O.knn(nd.xy, [c], 10, 0.0)[0]
        assert np.array_equal(idx[c], st)
        Wo, so = O.stencil_weights(nd.xy, st, c, 7, 3, ops, 0.0)
        want[c] = so
        if so == 0:
            for o in range(len(ops)):
                err = np.linalg.norm(W[o, c] - Wo[o]) / np.linalg.norm(Wo[o])
                worst = max(worst, err)
                assert err <= TOL_W, (c, o, err)
    assert 0 < int(np.count_nonzero(want)) < N  # the node set has both kinds
    assert np.array_equal(status, want)
    assert rc == R.ESINGULAR
    say(f"   {int(np.count_nonzero(want))} singular of {N}; worst relative error of the others {worst:.2e}")


@pytest.mark.parametrize("precision", [0, 1])
def test_two_systems_per_wavefront(R, ctx, precision):
    """Systems of up to 32 unknowns run two per wavefront, and the two share
    n, m and l; a stencil whose partner has another shape is solved on its
    own afterwards. An odd count (the last wavefront holds one system), runs
    of one shape and alternating shapes (same n and l, different m
    included), against the oracle."""
    say(f"weights: K <= 32 systems two per wavefront, 4 shapes in runs and alternations, 23 stencils, "
        f"precision {precision}")
    nd = jittered_square(24, seed=8)
    shapes = [(3, 2, 13), (5, 3, 21), (3, 3, 21), (5, 2, 20)]      # (m, l, n): K = 19, 31, 31, 26
    pattern = [0, 0, 0, 0, 0, 1, 1, 0, 2, 3, 2, 3, 0, 1, 1, 1, 2, 2, 3, 0, 0, 1, 2]
    rng = np.random.default_rng(12)
    centers = rng.choice(nd.n_active, len(pattern), replace=False).astype(np.int32)
    m_per = np.array([shapes[p][0] for p in pattern], np.int32)
    l_per = np.array([shapes[p][1] for p in pattern], np.int32)
    n_per = np.array([shapes[p][2] for p in pattern], np.int32)
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.LAP, 0, 0)]
    _weights_parity(R, ctx, nd.xy, ops, int(n_per.max()), 0, 0, 0.0, centers, n_per=n_per, m_per=m_per,
                    l_per=l_per, precision=precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_weights_full_size_mixed_samples(R, ctx, precision):
    """The 1M mixed batch in both solve precisions (FP64 LU, and the FP32
    factorisation with FP64 refinement, which is accepted only at the
    oracle's accuracy: Section 3, Eq. weights), 120 sampled stencils."""
    say(f"weights: 1,048,576 scattered nodes, mixed l in {{3,4,5}}, 120 sampled stencils, precision {precision}")
    cfg = weights_config(1024)
    nd = cfg["nodes"]
    rng = np.random.default_rng(11)
    samp = np.concatenate([rng.choice(nd.n_active, 110, replace=False), [0, 1023, 5000, nd.n_active - 1]])
    samp = np.concatenate([samp, np.nonzero(cfg["n_per"] == cfg["n_max"])[0][:6]])
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.HYPERLAP, 0, 0)]
    _weights_parity(R, ctx, nd.xy, ops, cfg["n_max"], 0, 0, 0.0, np.arange(nd.n_active), sample=samp,
                    n_per=cfg["n_per"], m_per=cfg["m_per"], l_per=cfg["l_per"], precision=precision)


def test_weights_reproduce_polynomials(R, ctx):
    """Independent of the oracle: the GPU weights are exact on monomials up to
    degree l (Section 3 constraints), in physical coordinates."""
    import torch
    say("weights: polynomial reproduction of GPU weights, scattered 24x24, r^7 deg 5, n = 43")
    nd = jittered_square(24, seed=2)
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.LAP, 0, 0), (O.DZZ, 0, 0), (O.DXX, 0, 0), (O.HYPERLAP, 3, 0)]
    idx, W, status, rc = R.rbffd_weights(ctx, dev(nd.xy, torch.float64), ops, 43, 7, 5,
                                         n_centers=nd.n_active)
    idx, W = host(idx), host(W)
    for c in range(0, nd.n_active, 7):
        dx = nd.xy[idx[c], 0] - nd.xy[c, 0]
        dz = nd.xy[idx[c], 1] - nd.xy[c, 1]
        for (a, b) in O.poly_exponents(5):
            vals = dx ** a * dz ** b
            for o, (kind, k, _) in enumerate(ops):
                exact = O.poly_apply(kind, 3 if kind == O.HYPERLAP else k, a, b)
                assert abs(W[o, c] @ vals - exact) <= 1e-10 * (np.abs(W[o, c] * vals).sum() + abs(exact))


def test_fp32_factorisation_falls_back_to_fp64(R, ctx):
    """Ill-conditioned systems (r^13, degree 6, n = 34 on a jittered 8 x 8
    lattice squeezed 5x in z: condition numbers around 1e9, far beyond what
    FP32 refinement can handle) under the FP32 factorisation: the stencils
    whose refinement stalls are solved again in FP64 and marked 3. Their
    weights equal the FP64 run's bit for bit, and every stencil matches the
    oracle."""
    import torch
    say("weights: FP32 factorisation falls back to FP64 where its refinement stalls (cond ~1e9)")
    rng = np.random.default_rng(5)
    g, sq = 8, 0.2
    X, Z = np.meshgrid(np.arange(g), np.arange(g))
    xy = np.stack([X.ravel(), Z.ravel() * sq], 1).astype(np.float64)
    xy += rng.uniform(-0.2, 0.2, xy.shape) * np.array([1.0, sq])
    centers = np.arange(g * g, dtype=np.int32)
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.LAP, 0, 0)]
    runs = {}
    for prec in (0, 1):
        idx, W, status, rc = R.rbffd_weights(ctx, dev(xy, torch.float64), ops, 34, 13, 6,
                                             centers=dev(centers, torch.int32), precision=prec)
        runs[prec] = (host(idx), host(W), host(status), rc)
    idx, W64, s64, rc64 = runs[0]
    _, W32, s32, rc32 = runs[1]
    assert rc64 == R.OK and np.all(s64 == 0)
    assert rc32 == R.OK and np.all((s32 == 0) | (s32 == 3))
    fell = np.flatnonzero(s32 == 3)
    say(f"   {len(fell)} of {len(centers)} stencils solved again in FP64")
    assert len(fell) > 0
    assert np.array_equal(W32[:, fell], W64[:, fell])
    worst = 0.0
    for a, c in enumerate(centers):
        st = O.knn(xy, [int(c)], 34, 0.0)[0]
        assert np.array_equal(idx[a], st)
        Wo, so = O.stencil_weights(xy, st, int(c), 13, 6, ops, 0.0)
        assert so == 0
        for W in (W64, W32):
            for o in range(len(ops)):
                err = np.linalg.norm(W[o, a] - Wo[o]) / np.linalg.norm(Wo[o])
                worst = max(worst, err)
                assert err <= TOL_W, (a, o, err)
    say(f"   worst norm-wise relative weight error {worst:.2e}")


def test_weights_singular_and_invalid(R, ctx):
    import torch
    say("weights: singular one-sided Cartesian stencils (deg 5) flagged; invalid arguments rejected")
    nd = unit_square_cartesian(21)
    xy = dev(nd.xy, torch.float64)
    centers = np.array([10, 10 * 21 + 10], np.int32)       # edge node, interior node
    idx, W, status, rc = R.rbffd_weights(ctx, xy, [(O.DX, 0, 0)], 37, 7, 5, centers=dev(centers, torch.int32))
    assert rc == R.ESINGULAR and host(status).tolist() == [1, 0]
    for bad in (dict(m=4, l=4), dict(m=5, l=7), dict(m=5, l=4, ops=[(O.HYPERLAP, 3, 0)]),
                dict(m=5, l=6, n=20)):
        with pytest.raises(R.RbffdError) as e:
            R.rbffd_weights(ctx, xy, bad.get("ops", [(O.DX, 0, 0)]), bad.get("n", 37), bad["m"], bad["l"],
                            centers=dev(centers, torch.int32))
        assert e.value.code == R.EINVAL
    # a per-stencil degree outside 0..6: found by the device checks
    with pytest.raises(R.RbffdError) as e:
        R.rbffd_weights(ctx, xy, [(O.DX, 0, 0)], 37, 7, 0, centers=dev(centers, torch.int32),
                        l_per=dev(np.array([4, 7], np.int32), torch.int32))
    assert e.value.code == R.EINVAL


def test_invalid_arguments_write_nothing(R, ctx):
    """EINVAL leaves every output as it was (rbffd.h conventions): the
    per-stencil parameters and indices are checked on the device before the
    search or any solve writes. Outputs are filled with sentinels; one bad
    entry at a time -- a degree above 6, an even PHS order, a stencil too
    small for its polynomial terms, a centre outside the node set, a given
    stencil index outside it, Laplacian^3 of r^5 -- must leave them alone."""
    import torch
    say("weights/knn: invalid per-stencil arguments -> EINVAL with idx, w and status untouched")
    nd = jittered_square(24, seed=9)
    xy = dev(nd.xy, torch.float64)
    nc, n = 40, 37
    centers = np.arange(100, 100 + nc, dtype=np.int32)
    good = dict(n_per=np.full(nc, n, np.int32), m_per=np.full(nc, 7, np.int32), l_per=np.full(nc, 4, np.int32))
    idx_ok = R.rbffd_knn(ctx, xy, n, 0.0, centers=dev(centers, torch.int32))
    cases = []
    for key, at, val in (("l_per", 5, 7), ("m_per", 17, 6), ("n_per", 30, 12), ("centers", 39, nd.n_active),
                         ("idx_in", 3, -4), ("m_per", 0, 5)):
        cases.append((key, at, val))
    for key, at, val in cases:
        args = {k: v.copy() for k, v in good.items()}
        cen = centers.copy()
        idx_in = None
        ops = [(O.DX, 0, 0), (O.LAP, 0, 0)]
        if key == "centers":
            cen[at] = val
        elif key == "idx_in":
            idx_in = host(idx_ok).copy()
            idx_in[at, 20] = val
        else:
            args[key][at] = val
        if key == "m_per" and val == 5:
            ops = [(O.DX, 0, 0), (O.HYPERLAP, 3, 0)]          # Laplacian^3 of r^5: not continuous
        idx = torch.full((nc, n), -77, dtype=torch.int32, device="cuda")
        w = torch.full((len(ops), nc, n), 12345.0, dtype=torch.float64, device="cuda")
        status = torch.full((nc,), 99, dtype=torch.int32, device="cuda")
        with pytest.raises(R.RbffdError) as e:
            R.rbffd_weights(ctx, xy, ops, n, 0, 0, centers=dev(cen, torch.int32),
                            n_per=dev(args["n_per"], torch.int32), m_per=dev(args["m_per"], torch.int32),
                            l_per=dev(args["l_per"], torch.int32),
                            idx_in=None if idx_in is None else dev(idx_in, torch.int32), out=(idx, w, status))
        assert e.value.code == R.EINVAL, (key, e.value)
        assert f"stencil {at}" in str(e.value), (key, str(e.value))
        assert bool((idx == -77).all()) and bool((w == 12345.0).all()) and bool((status == 99).all()), key
        say(f"   {key}[{at}] = {val}: {e.value}")
    # the search alone: a bad centre or stencil size writes nothing either
    for cen, n_per in ((np.array([0, 5, nd.n_active + 3], np.int32), None),
                       (np.array([0, 5, 9], np.int32), np.array([37, 0, 37], np.int32))):
        out = torch.full((3, n), -77, dtype=torch.int32, device="cuda")
        with pytest.raises(R.RbffdError) as e:
            R.rbffd_knn(ctx, xy, n, 0.0, centers=dev(cen, torch.int32),
                        n_per=None if n_per is None else dev(n_per, torch.int32), out=out)
        assert e.value.code == R.EINVAL and bool((out == -77).all())


def test_knn_dense_cluster(R, ctx):
    """A cluster of 3,000 nodes inside one grid cell of a sparse set (more
    candidates than the search keeps in LDS): those centres, and sparse
    centres whose search block reaches the cluster, are finished by the exact
    selection kernel; bit-exact against the oracle's brute-force search,
    also with a periodic x."""
    import torch
    say("knn: 3,000-node cluster inside one cell of 400 sparse nodes (exact fallback), plain and periodic")
    rng = np.random.default_rng(21)
    sparse = rng.uniform(0.0, 1.0, (400, 2))
    cluster = np.array([0.5, 0.5]) + rng.uniform(-1e-3, 1e-3, (3000, 2))
    xy = np.concatenate([sparse, cluster])
    for period in (0.0, 1.0):
        samp = np.concatenate([np.arange(0, 400, 9), 400 + rng.choice(3000, 40, replace=False)])
        got = host(R.rbffd_knn(ctx, dev(xy, torch.float64), 37, period, centers=dev(samp.astype(np.int32), torch.int32)))
        for a, c in enumerate(samp):
            ref = O.knn(xy, [int(c)], 37, period)[0]
            assert np.array_equal(got[a], ref), (period, c)
    # a ragged n_per with the same cluster
    n_per = rng.integers(1, 61, 60).astype(np.int32)
    samp = 400 + rng.choice(3000, 60, replace=False).astype(np.int32)
    _knn_case(R, ctx, xy, 60, 0.0, centers=samp, n_per=n_per)


def test_weights_tuner_shapes_are_bit_identical(R, ctx):
    """Every launch shape of every size bucket (persistent grids of 8-24
    workgroups per compute unit or one per system; two systems per wavefront
    or one for K <= 32) gives the same idx, weights and status bit for bit,
    in both solve precisions; rbffd_weights_tune picks a shape per bucket and
    later rbffd_weights calls, which use it, give the same results again."""
    import torch
    say("weights tuner: every shape of every bucket bit-identical (mixed 40x40 batch, FP64 and FP32+IR)")
    cfg = weights_config(40, seed=5)
    nd = cfg["nodes"]
    xy = dev(nd.xy, torch.float64)
    kw = dict(n_per=dev(cfg["n_per"], torch.int32), m_per=dev(cfg["m_per"], torch.int32),
              l_per=dev(cfg["l_per"], torch.int32))
    ops = [(O.DX, 0, 0), (O.DZ, 0, 0), (O.HYPERLAP, 0, 0)]
    for prec in (R.SOLVE_FP64, R.SOLVE_FP32_IR):
        ref = R.rbffd_weights(ctx, xy, ops, cfg["n_max"], precision=prec, **kw)
        for s in range(max(R.WEIGHT_SHAPES)):
            forced = [min(s, c - 1) for c in R.WEIGHT_SHAPES]
            got = R.rbffd_weights_tune(ctx, xy, ops, cfg["n_max"], shapes=forced, precision=prec, **kw)
            assert got[4] == forced
            for a, b in zip(got[:3], ref[:3]):
                assert torch.equal(a, b), (prec, forced)
        idx, W, status, rc, chosen, ms = R.rbffd_weights_tune(ctx, xy, ops, cfg["n_max"], precision=prec, **kw)
        say(f"   precision {prec}: tuned shapes {chosen}, bucket ms {['%.3f' % t for t in ms]}")
        assert all(0 <= c < n for c, n in zip(chosen, R.WEIGHT_SHAPES))
        after = R.rbffd_weights(ctx, xy, ops, cfg["n_max"], precision=prec, **kw)
        for a, b in zip((idx, W, status) + after[:3], ref[:3] * 2):
            assert torch.equal(a, b)
    R.rbffd_weights_tune(ctx, xy, ops, cfg["n_max"], shapes=[0] * 6, **kw)   # back to the default shapes
    with pytest.raises(R.RbffdError) as e:
        R.rbffd_weights_tune(ctx, xy, ops, cfg["n_max"], shapes=[10, 0, 0, 0, 0, 0], **kw)
    assert e.value.code == R.EINVAL
