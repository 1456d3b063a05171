"""GPU parity of the k-space completion path against the FP64 oracle.

The network kernels keep weights, activations and gradients in BF16 and accumulate in FP32;
the oracle side applies the same BF16 roundings (round to nearest even) to the FP64 values at
the same places, so the comparison isolates the kernels' indexing and arithmetic.  Bars:
rel-L2 5e-3 for the network output, 3e-2 for parameter gradients (BF16 gradients through six
layers), 1e-6 for Adam and grid preparation (FP32), 1e-5 for the spectra (FP32, as RF_theta).
"""
import numpy as np
import pytest

import oracle as O
from oracle import completion as OC
from oracle.decompose import decompose_spectrum as oracle_spectrum
from paper_2603_22496_amd import configs as C
from tests import oracle_ref as OR

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def bf16(x):
    """Round to BF16 (nearest even), returned as float64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def kk():
    import torch
    from paper_2603_22496_amd import kk as K
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    K.lib()
    return K


def _params(K, seed):
    r = np.random.default_rng(seed)
    p = np.zeros(K.net_param_count(), np.float32)
    for l, (cin, wo, bo) in enumerate(K.net_layer_shapes()):
        used_in = 3 if l == 0 else 32
        W = np.zeros((9, 32, cin), np.float32)
        W[:, :, :used_in] = r.standard_normal((9, 32, used_in)) * np.sqrt(2.0 / (9 * used_in))
        if l == K.NET_LAYERS - 1:
            W[:, 2:, :] = 0.0
        p[wo:bo] = W.ravel()
        b = 0.05 * r.standard_normal(32).astype(np.float32)
        if l == K.NET_LAYERS - 1:
            b[2:] = 0.0
        p[bo:bo + 32] = b
    return p


def _unpack(K, p, rounded=True):
    layers = []
    for cin, wo, bo in K.net_layer_shapes():
        W = p[wo:bo].reshape(9, 32, cin).astype(np.float64)
        layers.append((bf16(W) if rounded else W, p[bo:bo + 32].astype(np.float64)))
    return layers


def _grid(seed, B, H, W, cols):
    r = np.random.default_rng(seed)
    g = np.zeros((B, H, W, 8))
    g[..., cols, 0] = r.standard_normal((B, H, len(cols)))
    g[..., cols, 1] = r.standard_normal((B, H, len(cols)))
    g[..., cols, 2] = 1.0
    return bf16(g)


def _to_bf16_dev(K, a):
    import torch
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).cuda()


DILATED = [(1, 1), (1, 2), (2, 4), (2, 8), (4, 16), (1, 1)]


def _emulated_forward(layers, x, dils=None):
    dils = dils or [(1, 1)] * len(layers)
    acts = [x]
    a = x
    for l, (W, b) in enumerate(layers):
        z = OC.conv3x3(a, W, b, dils[l])
        if l < len(layers) - 1:
            a = bf16(np.maximum(z, 0.0))
            acts.append(a)
        else:
            return z, acts


def _emulated_backward(layers, acts, gout, dils=None):
    dils = dils or [(1, 1)] * len(layers)
    grads = [None] * len(layers)
    g = gout
    for l in range(len(layers) - 1, -1, -1):
        if l < len(layers) - 1:
            g = g * (acts[l + 1] > 0)
        gx, gW, gb = OC.conv3x3_backward(acts[l], layers[l][0], g, dils[l])
        grads[l] = (gW, gb)
        g = bf16(gx)
    return grads


@pytest.mark.parametrize("B,H,W,dils", [(2, 5, 32, None), (1, 31, 128, None), (3, 7, 48, None),
                                         (2, 31, 128, DILATED), (1, 9, 64, DILATED)])
def test_forward_matches_oracle(kk, B, H, W, dils):
    import torch
    print("net forward B %d H %d W %d dilated %s" % (B, H, W, dils is not None), flush=True)
    p = _params(kk, 1)
    cols = sorted(np.random.default_rng(2).choice(W, size=max(2, W // 10), replace=False).tolist())
    x = _grid(3, B, H, W, cols)
    net = kk.Net(p, B, H, W, dilation=dils)
    out = torch.zeros((B, H, W, 2), dtype=torch.float32, device="cuda")
    net.forward(_to_bf16_dev(kk, x), out)
    torch.cuda.synchronize()
    ref, _ = _emulated_forward(_unpack(kk, p), x, dils)
    rel = _rel(out.cpu().numpy(), ref[..., :2])
    print("  rel-L2 %.3e" % rel, flush=True)
    assert rel <= 5e-3, rel


def test_forward_sample_index(kk):
    # batch rows read grid samples through the index table
    import torch
    B, H, W = 3, 4, 32
    p = _params(kk, 4)
    x = _grid(5, 5, H, W, [1, 7, 20])
    idx = np.array([4, 0, 2], np.int32)
    net = kk.Net(p, B, H, W)
    out = torch.zeros((B, H, W, 2), dtype=torch.float32, device="cuda")
    net.forward(_to_bf16_dev(kk, x), out, sidx=torch.from_numpy(idx).cuda())
    torch.cuda.synchronize()
    ref, _ = _emulated_forward(_unpack(kk, p), x[idx])
    assert _rel(out.cpu().numpy(), ref[..., :2]) <= 5e-3


@pytest.mark.parametrize("B,H,W,dils", [(2, 5, 32, None), (2, 31, 128, None), (2, 31, 128, DILATED)])
def test_gradients_match_oracle(kk, B, H, W, dils):
    import torch
    print("net gradients B %d H %d W %d dilated %s" % (B, H, W, dils is not None), flush=True)
    p = _params(kk, 6)
    cols = list(range(0, W, 7))
    x = _grid(7, B, H, W, cols)
    tgt = np.random.default_rng(8).standard_normal((B, H, W, 2)).astype(np.float32).astype(np.float64)
    obs = x[..., 2]
    n_un = float((1 - obs).sum())
    inv = 1.0 / (2 * n_un)
    net = kk.Net(p, B, H, W, dilation=dils)
    loss = net.backward(_to_bf16_dev(kk, x), torch.from_numpy(tgt.astype(np.float32)).cuda(), inv)
    torch.cuda.synchronize()
    g_gpu = net.read(kk.NET_GRADS)
    layers = _unpack(kk, p)
    out, acts = _emulated_forward(layers, x, dils)
    l_ref, gout = OC.masked_mse(out[..., :2], tgt, obs)
    assert abs(float(loss.item()) - l_ref) <= 1e-2 * l_ref
    g32 = np.zeros(out.shape)
    g32[..., :2] = bf16(gout)
    grads = _emulated_backward(layers, acts, g32, dils)
    for l, (cin, wo, bo) in enumerate(kk.net_layer_shapes()):
        gW, gb = grads[l]
        rw = _rel(g_gpu[wo:bo].reshape(9, 32, cin), gW)
        rb = _rel(g_gpu[bo:bo + 32], gb)
        print("  layer %d: dW rel %.3e  db rel %.3e" % (l, rw, rb), flush=True)
        assert rw <= 3e-2 and rb <= 3e-2, (l, rw, rb)
    # and against the plain FP64 network gradient (FP32 weights, no BF16 anywhere): the same
    # gradient up to what BF16 weights and activations change through six layers
    out64, acts64 = OC.forward(x, _unpack(kk, p, rounded=False), dils)
    _, gout64 = OC.masked_mse(out64[..., :2], tgt, obs)
    g64 = np.zeros(out64.shape)
    g64[..., :2] = gout64
    grads64 = OC.backward(_unpack(kk, p, rounded=False), acts64, g64, dils)
    for l, (cin, wo, bo) in enumerate(kk.net_layer_shapes()):
        assert _rel(g_gpu[wo:bo].reshape(9, 32, cin), grads64[l][0]) <= 0.3


def test_adam_step_matches_oracle(kk):
    import torch
    B, H, W = 2, 5, 32
    p = _params(kk, 9)
    x = _grid(10, B, H, W, [0, 9, 30])
    tgt = np.random.default_rng(11).standard_normal((B, H, W, 2)).astype(np.float32)
    net = kk.Net(p, B, H, W)
    xd, td = _to_bf16_dev(kk, x), torch.from_numpy(tgt).cuda()
    inv = 1.0 / (2 * float((1 - x[..., 2]).sum()))
    pp, m, v = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for t in (1, 2, 3):
        net.backward(xd, td, inv)
        g = net.read(kk.NET_GRADS).astype(np.float64)
        net.adam(1e-3)
        torch.cuda.synchronize()
        pp, m, v = OC.adam(pp, g, m, v, t, 1e-3)
        got = net.read(kk.NET_PARAMS).astype(np.float64)
        assert np.max(np.abs(got - pp)) <= 1e-6, t
        # 1 - b2 in FP32 is 0.99900001 short of exact: 1.3e-5 relative on the second moment
        assert _rel(net.read(kk.NET_MOMENT2), v) <= 5e-5


def test_training_reduces_loss(kk):
    import torch
    B, H, W = 4, 6, 32
    cols = [2, 9, 15, 22, 29]
    r = np.random.default_rng(12)
    # a learnable target: smooth grids (low spatial frequency), observed on a few columns
    hh, ww = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    full = np.stack([np.cos(0.2 * ww + 0.3 * hh + ph) for ph in r.uniform(0, 6.28, 2 * B)]).reshape(B, 2, H, W)
    full = np.ascontiguousarray(full.transpose(0, 2, 3, 1))
    x = np.zeros((B, H, W, 8))
    x[..., cols, 0:2] = full[..., cols, :]
    x[..., cols, 2] = 1.0
    x = bf16(x)
    net = kk.Net(_params(kk, 13), B, H, W)
    xd, td = _to_bf16_dev(kk, x), torch.from_numpy(full.astype(np.float32)).cuda()
    inv = 1.0 / (2 * float((1 - x[..., 2]).sum()))
    losses = []
    for it in range(200):
        losses.append(float(net.train_step(xd, td, inv, 2e-3).item()))
    print("loss %.4f -> %.4f" % (losses[0], losses[-1]), flush=True)
    assert losses[-1] < 0.2 * losses[0]


def test_prepare_and_merge_match_oracle(kk):
    import torch
    r = np.random.default_rng(14)
    H, W, kpad = 5, 32, 24
    spec = (r.standard_normal((H, W, kpad)) + 1j * r.standard_normal((H, W, kpad))).astype(np.complex64)
    cols = [1, 4, 5, 17, 31]
    g2o = -np.ones(W, np.int32)
    g2o[cols] = np.arange(len(cols))
    bins = np.array([3, 0, 22, 11], np.int32)
    B = len(bins)
    sd = torch.from_numpy(spec).cuda()
    grid = torch.zeros((B, H, W, 8), dtype=torch.bfloat16, device="cuda")
    tgt = torch.zeros((B, H, W, 2), dtype=torch.float32, device="cuda")
    sc = torch.zeros(B, dtype=torch.float32, device="cuda")
    obs_src = torch.from_numpy(np.array(cols, np.int32)).cuda()
    g2o_d = torch.from_numpy(g2o).cuda()
    kk.net_prepare(sd, obs_src, g2o_d, grid, sc, bins=torch.from_numpy(bins).cuda(), target=tgt)
    torch.cuda.synchronize()
    gg, tt, ss = grid.float().cpu().numpy(), tgt.cpu().numpy(), sc.cpu().numpy()
    for b, k in enumerate(bins):
        inp, target, obs, scale = OC.prepare(spec[:, :, k].astype(np.complex128), cols)
        assert abs(ss[b] - scale) <= 1e-6 * scale
        np.testing.assert_allclose(gg[b, ..., :3], bf16(inp), rtol=0, atol=0)
        assert not gg[b, ..., 3:].any()
        assert _rel(tt[b], target) <= 1e-6
    # merge: observed pairs copied, the rest out * scale; other bins untouched
    out = torch.from_numpy(tt).cuda()
    dst = torch.full((H, W, kpad), 7.0 + 0j, dtype=torch.complex64, device="cuda")
    kk.net_merge(out, sc, sd, obs_src, g2o_d, dst, bins=torch.from_numpy(bins).cuda())
    torch.cuda.synchronize()
    d = dst.cpu().numpy()
    for b, k in enumerate(bins):
        _, target, obs, scale = OC.prepare(spec[:, :, k].astype(np.complex128), cols)
        ref = OC.merge(spec[:, :, k].astype(np.complex128), target, obs, scale)
        np.testing.assert_array_equal(d[:, cols, k], spec[:, cols, k])
        assert _rel(d[:, :, k], ref) <= 1e-6
    untouched = np.setdiff1d(np.arange(kpad), bins)
    assert np.all(d[:, :, untouched] == 7.0)


def test_spectrum_and_inverse_match_oracle(kk):
    import torch
    ds = C.tiny_dataset(1)
    su = kk.make_setup(C.TINY)
    spec = kk.decompose_spectrum(kk.to_device(ds.rf), su.geom, kk.to_device(su.luts["shift"]), su.M, su.tpad)
    torch.cuda.synchronize()
    ot = OR.tables(su, C.TINY)
    Y = oracle_spectrum(ds.rf, ot.luts["shift"], ot.luts["tpad"])     # [N][M][K]
    kpad = kk.spectrum_bins(su.tpad)
    got = spec.cpu().numpy()
    half = su.tpad // 2
    assert got.shape[-1] == kpad
    assert _rel(got[..., :half], Y[..., :half]) <= 1e-5
    assert not got[..., half:].any()
    # inverse of the (Nyquist-free) spectrum against the oracle's inverse of the same bins
    rt = kk.spectrum_inverse(spec, su.tpad, C.TINY.T)
    torch.cuda.synchronize()
    Yz = Y.copy()
    Yz[..., half:] = 0
    ref = O.inverse_bins(Yz, su.tpad, C.TINY.T)
    assert _rel(rt.cpu().numpy(), ref) <= 1e-5


def test_net_errors(kk):
    import ctypes
    L = kk.lib()
    assert L.kk_net_workspace_bytes(2, 5, 40) == 0       # W not a multiple of 16
    assert L.kk_net_workspace_bytes(2, 5, 208) == 0      # wider than the staging limit
    assert L.kk_net_workspace_bytes(0, 5, 32) == 0
    assert L.kk_net_read(None, 0, None, None) == kk.KK_E_NULL
    assert L.kk_spectrum_bins(100) == 0 and L.kk_spectrum_bins(4096) == 2056
    bad = kk.Net(_params(kk, 15), 2, 5, 32)
    bad._dil[3] = 0
    import torch
    with pytest.raises(kk.KKError):
        bad.forward(torch.zeros((2, 5, 32, 8), dtype=torch.bfloat16, device="cuda"),
                    torch.zeros((2, 5, 32, 2), dtype=torch.float32, device="cuda"))
    net = kk.Net(_params(kk, 15), 2, 5, 32)
    buf = np.zeros(8, np.float32)
    assert L.kk_net_read(kk._dev(net.state), 9, buf.ctypes.data, None) == kk.KK_E_ARG
    assert L.kk_net_adam(kk._dev(net.state), 0, ctypes.c_float(1e-3), None) == kk.KK_E_ARG
    assert L.kk_clear(kk._dev(net.ws), 7, None) == kk.KK_E_ARG


@pytest.fixture(scope="module")
def pipeline(kk):
    from paper_2603_22496_amd import completion as CP
    cs = CP.setup()
    return CP, cs, CP.Device(cs)


def test_observed_spectrum_is_the_full_banks_columns(kk, pipeline):
    import torch
    CP, cs, d = pipeline
    su = cs.full
    rf = kk.to_device(CP.phantom(cs, 12000, 300).rf)
    full = kk.decompose_spectrum(rf, su.geom, d.shift_full, len(su.sel["rx_theta"]), su.tpad, ws=d.ws)
    obs = kk.decompose_spectrum(rf, su.geom, d.shift_obs, len(cs.cols), su.tpad, ws=d.ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(obs.cpu().numpy(), full.cpu().numpy()[:, cs.cols, :])


def test_perfect_prediction_reproduces_the_full_image(kk, pipeline):
    # completing every band bin (DC to 9.75 MHz) with the true grid leaves only the unobserved
    # bins above the band and the Nyquist bin out of the fully sampled image
    import torch
    CP, cs, d = pipeline
    su = cs.full
    W = len(su.sel["rx_theta"])
    rf = kk.to_device(CP.phantom(cs, 12001, 300).rf)
    ref = CP.full_image(cs, d, rf).cpu().numpy()
    full = kk.decompose_spectrum(rf, su.geom, d.shift_full, W, su.tpad, ws=d.ws)
    obs = kk.decompose_spectrum(rf, su.geom, d.shift_obs, len(cs.cols), su.tpad, ws=d.ws)
    tgt = torch.zeros((CP.BATCH, cs.w.N, W, 2), dtype=torch.float32, device="cuda")
    kk.clear(d.out)
    for k0 in range(0, cs.kpad, CP.BATCH):
        B = min(CP.BATCH, cs.kpad - k0)
        kk.net_merge(d.out, d.scale, obs, d.cols_obs, d.g2o, d.spec_done, k_first=k0, B=B)
    for k0 in range(cs.k_lo, cs.k_hi, CP.BATCH):
        B = min(CP.BATCH, cs.k_hi - k0)
        kk.net_prepare(full, d.cols_full, d.g2o, d.grid, d.scale, k_first=k0, B=B, target=tgt)
        kk.net_merge(tgt, d.scale, obs, d.cols_obs, d.g2o, d.spec_done, k_first=k0, B=B)
    kk.spectrum_inverse(d.spec_done, su.tpad, cs.w.T, out=d.rt_full)
    img = kk.beamform(d.rt_full, su.plan, d.plan_full, image=d.img, ws=d.bws).cpu().numpy()
    rel = _rel(img, ref)
    print("perfect completion rel-L2 %.3e" % rel, flush=True)
    assert rel <= 1e-3


def test_complete_image_paths_run(kk, pipeline):
    import torch
    CP, cs, d = pipeline
    rf = kk.to_device(CP.phantom(cs, 12002, 300).rf)
    ref = CP.full_image(cs, d, rf).cpu().numpy()
    plain = CP.complete_image(cs, d, rf, None).cpu().numpy()
    net = kk.Net(CP.init_params(0), CP.BATCH, cs.w.N, len(cs.full.sel["rx_theta"]))
    done = CP.complete_image(cs, d, rf, net).cpu().numpy()
    assert np.isfinite(plain).all() and np.isfinite(done).all()
    e_plain = CP.scaled_error(plain, ref)
    print("untrained: compressed rel-L2 %.3f (best gain %.3f), completed %.3f" % (e_plain[0], e_plain[1],
                                                                                 CP.scaled_error(done, ref)[0]))
    assert e_plain[1] < 1.0
