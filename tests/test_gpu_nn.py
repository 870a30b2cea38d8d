"""GPU: the learned surrogate's matrix-core kernels against the FP64 oracle on
identical BF16 operands (forward, data gradient, weight gradient), its loss
and optimiser kernels, the plain-flow label context, and a training smoke
test."""
import ctypes as C
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2308_09209_amd import surrogate as S  # noqa: E402
from paper_2308_09209_amd import vstitch as V  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_bf16(x):
    """float -> BF16 bits (round to nearest even), as int16"""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16).view(np.int16)


def from_bf16(b):
    return (np.ascontiguousarray(b).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


SIZES = [(13, 37), (20, 9), (1, 5)]


def split_images(flat, c):
    out, off = [], 0
    for (h, w) in SIZES:
        out.append(flat[off:off + h * w].reshape(1, h, w, c))
        off += h * w
    return out


def test_mfma_fragment_layout():
    rng = np.random.default_rng(0)
    a = to_bf16(rng.normal(size=(16, 16)))
    b = to_bf16(rng.normal(size=(16, 16)))
    out = torch.zeros(256, dtype=torch.float32, device="cuda:0")
    da, db = dev(a), dev(b)          # held until the kernel has run
    V.check(V.lib().vs_nn_mfma_probe(C.c_void_p(da.data_ptr()), C.c_void_p(db.data_ptr()),
                                     C.c_void_p(out.data_ptr()), None), "probe")
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(64, 4)
    D = from_bf16(a) @ from_bf16(b)
    for l in range(64):
        for i in range(4):
            assert abs(got[l, i] - D[4 * (l // 16) + i, l % 16]) <= 1e-5 * (1 + abs(D[4 * (l // 16) + i, l % 16]))


def test_mfma_k32_fragment_layout():
    rng = np.random.default_rng(1)
    a = to_bf16(rng.normal(size=(16, 32)))
    b = to_bf16(rng.normal(size=(32, 16)))
    out = torch.zeros(256, dtype=torch.float32, device="cuda:0")
    da, db = dev(a), dev(b)
    V.check(V.lib().vs_nn_mfma_probe_k32(C.c_void_p(da.data_ptr()), C.c_void_p(db.data_ptr()),
                                         C.c_void_p(out.data_ptr()), None), "probe k32")
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(64, 4)
    D = from_bf16(a) @ from_bf16(b)
    for l in range(64):
        for i in range(4):
            assert abs(got[l, i] - D[4 * (l // 16) + i, l % 16]) <= 1e-5 * (1 + abs(D[4 * (l // 16) + i, l % 16]))


def conv_call(x, cin, w, b, y, cout, imgs, mode):
    return V.lib().vs_nn_conv3x3(C.c_void_p(x.data_ptr()), cin, C.c_void_p(w.data_ptr()),
                                 None if b is None else C.c_void_p(b.data_ptr()), C.c_void_p(y.data_ptr()), cout,
                                 C.byref(imgs), mode, 0.1, None)


@pytest.mark.parametrize("cin,cout", [(32, 32), (16, 32), (32, 16)])
def test_conv_many_tiles_per_block_elementwise(cin, cout):
    """more 16x16 tiles than the persistent grid holds blocks (each block walks
    several tiles), ragged edges, a 1x1 image: every FP32 output within the
    worst-case bound of an FP32 sum of 9 cin + 1 terms, |y - ref| <= n u / (1 - n u)
    * (sum |w x| + |b|); the BF16 leaky-ReLU output and the flow output are the
    FP32 output's own activation (rounded to nearest even) and channels 0-1, bit
    for bit"""
    sizes = [(600, 600), (37, 250), (1, 1)]
    rng = np.random.default_rng(7 * cin + cout)
    P = sum(h * w for h, w in sizes)
    x = to_bf16(rng.normal(size=(P, cin)))
    w = to_bf16(rng.normal(size=(cout, 9, cin)) * 0.2)
    b = rng.normal(size=cout).astype(np.float32)
    imgs = V.nn_images(sizes)
    xd, wd, bd = dev(x), dev(w), dev(b)
    y32 = torch.empty((P, cout), dtype=torch.float32, device="cuda:0")
    y16 = torch.empty((P, cout), dtype=torch.int16, device="cuda:0")
    yf = torch.empty((P, 2), dtype=torch.float32, device="cuda:0")
    say(f"[conv {cin}->{cout}] {len(sizes)} images, {P} pixels")
    V.check(conv_call(xd, cin, wd, bd, y32, cout, imgs, V.CONV_F32), "conv f32")
    V.check(conv_call(xd, cin, wd, bd, y16, cout, imgs, V.CONV_LRELU), "conv lrelu")
    V.check(conv_call(xd, cin, wd, bd, yf, cout, imgs, V.CONV_FLOW2), "conv flow2")
    xs, off = [], 0
    for (h, ww) in sizes:
        xs.append(from_bf16(x)[off:off + h * ww].reshape(1, h, ww, cin))
        off += h * ww
    ref = np.concatenate([O.conv3x3(xi, from_bf16(w), b.astype(np.float64)).reshape(-1, cout) for xi in xs])
    mag = np.concatenate([O.conv3x3(np.abs(xi), np.abs(from_bf16(w))).reshape(-1, cout) for xi in xs])
    mag += np.abs(b.astype(np.float64))
    n = 9 * cin + 1
    u = 2.0 ** -24
    bound = n * u / (1 - n * u) * mag
    got = y32.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref)
    say(f"[conv {cin}->{cout}] max |err| / bound = {float((err / np.maximum(bound, 1e-300)).max()):.3f}")
    assert (err <= bound).all()
    lre = np.where(got > 0, got, np.float32(0.1) * got.astype(np.float32))
    np.testing.assert_array_equal(y16.cpu().numpy(), to_bf16(lre))
    np.testing.assert_array_equal(yf.cpu().numpy(), y32.cpu().numpy()[:, :2])


def test_conv_rejects_misaligned_pointers():
    imgs = V.nn_images([(16, 16)])
    x = torch.zeros(16 * 16 * 32 + 8, dtype=torch.int16, device="cuda:0")
    w = torch.zeros(32 * 9 * 32, dtype=torch.int16, device="cuda:0")
    y = torch.zeros(16 * 16 * 32 + 8, dtype=torch.int16, device="cuda:0")
    xv = x[1:]                                      # 2 bytes past a 16-byte boundary
    assert V.STATUS[conv_call(xv, 32, w, None, y, 32, imgs, V.CONV_LINEAR)] == "VS_E_INVAL"
    assert V.STATUS[conv_call(x, 32, w, None, y[4:], 32, imgs, V.CONV_LINEAR)] == "VS_E_INVAL"
    V.check(conv_call(x, 32, w, None, y[8:], 32, imgs, V.CONV_LINEAR), "aligned")
    torch.cuda.synchronize()


@pytest.mark.parametrize("cin,cout", [(16, 32), (32, 32), (32, 16)])
def test_conv_forward_matches_oracle(cin, cout):
    rng = np.random.default_rng(cin * 100 + cout)
    P = sum(h * w for h, w in SIZES)
    x = to_bf16(rng.normal(size=(P, cin)))
    w = to_bf16(rng.normal(size=(cout, 9, cin)) * 0.2)
    b = rng.normal(size=cout).astype(np.float32)
    imgs = V.nn_images(SIZES)
    xd, wd, bd = dev(x), dev(w), dev(b)
    y32 = torch.empty((P, cout), dtype=torch.float32, device="cuda:0")
    y16 = torch.empty((P, cout), dtype=torch.int16, device="cuda:0")
    V.check(V.lib().vs_nn_conv3x3(C.c_void_p(xd.data_ptr()), cin, C.c_void_p(wd.data_ptr()),
                                  C.c_void_p(bd.data_ptr()), C.c_void_p(y32.data_ptr()), cout, C.byref(imgs),
                                  V.CONV_F32, 0.1, None), "conv")
    V.check(V.lib().vs_nn_conv3x3(C.c_void_p(xd.data_ptr()), cin, C.c_void_p(wd.data_ptr()),
                                  C.c_void_p(bd.data_ptr()), C.c_void_p(y16.data_ptr()), cout, C.byref(imgs),
                                  V.CONV_LRELU, 0.1, None), "conv")
    ref = np.concatenate([O.conv3x3(xi, from_bf16(w), b.astype(np.float64)).reshape(-1, cout)
                          for xi in split_images(from_bf16(x), cin)])
    e32 = rel_l2(y32.cpu().numpy().astype(np.float64), ref)
    lre = np.where(ref > 0, ref, 0.1 * ref)
    e16 = rel_l2(from_bf16(y16.cpu().numpy()), lre)
    say(f"[conv {cin}->{cout}] rel L2: FP32 out {e32:.2e}, BF16 leaky-ReLU out {e16:.2e}")
    assert e32 <= 1e-5 and e16 <= 4e-3


@pytest.mark.parametrize("cin,cout", [(16, 32), (32, 32), (32, 16)])
def test_conv_backward_matches_oracle(cin, cout):
    rng = np.random.default_rng(cin * 7 + cout)
    P = sum(h * w for h, w in SIZES)
    x = to_bf16(rng.normal(size=(P, cin)))
    w = to_bf16(rng.normal(size=(cout, 9, cin)) * 0.2)
    dz = to_bf16(rng.normal(size=(P, cout)))
    imgs = V.nn_images(SIZES)
    xd, wd, dzd = dev(x), dev(w), dev(dz)
    # data gradient: the forward kernel on flipped weights
    wf = torch.empty((cin, 9, cout), dtype=torch.int16, device="cuda:0")
    V.check(V.lib().vs_nn_flip_weights(C.c_void_p(wd.data_ptr()), C.c_void_p(wf.data_ptr()), cin, cout, None), "flip")
    dx = torch.empty((P, cin), dtype=torch.float32, device="cuda:0")
    V.check(V.lib().vs_nn_conv3x3(C.c_void_p(dzd.data_ptr()), cout, C.c_void_p(wf.data_ptr()), None,
                                  C.c_void_p(dx.data_ptr()), cin, C.byref(imgs), V.CONV_F32, 0.1, None), "dgrad")
    ref_dx = np.concatenate([O.conv3x3_bwd_data(g, from_bf16(w)).reshape(-1, cin)
                             for g in split_images(from_bf16(dz), cout)])
    # weight gradient
    nbytes = V.lib().vs_nn_wgrad_scratch_bytes(cin, cout, C.byref(imgs))
    scratch = torch.empty(nbytes // 4 + 1, dtype=torch.float32, device="cuda:0")
    dwb = torch.empty(cout * 9 * cin + cout, dtype=torch.float32, device="cuda:0")
    V.check(V.lib().vs_nn_conv3x3_wgrad(C.c_void_p(xd.data_ptr()), cin, C.c_void_p(dzd.data_ptr()), cout,
                                        C.byref(imgs), C.c_void_p(scratch.data_ptr()), nbytes,
                                        C.c_void_p(dwb.data_ptr()), None), "wgrad")
    rdw = np.zeros((cout, 9, cin))
    rdb = np.zeros(cout)
    for xi, gi in zip(split_images(from_bf16(x), cin), split_images(from_bf16(dz), cout)):
        a, bb = O.conv3x3_bwd_weight(xi, gi)
        rdw += a
        rdb += bb
    got = dwb.cpu().numpy().astype(np.float64)
    e_dx = rel_l2(dx.cpu().numpy().astype(np.float64), ref_dx)
    e_dw = rel_l2(got[:cout * 9 * cin].reshape(cout, 9, cin), rdw)
    e_db = rel_l2(got[cout * 9 * cin:], rdb)
    say(f"[conv {cin}->{cout} backward] rel L2: data {e_dx:.2e} weight {e_dw:.2e} bias {e_db:.2e}")
    assert e_dx <= 1e-5 and e_dw <= 1e-5 and e_db <= 1e-5


def test_loss_lrelu_adam_kernels():
    rng = np.random.default_rng(5)
    P = 1000
    pred = rng.normal(size=(P, 16)).astype(np.float32)
    lab = rng.normal(size=(P, 2)).astype(np.float32)
    bl, dz = S.loss_and_grad(dev(pred), dev(lab))
    d = pred[:, :2].astype(np.float64) - lab
    e = np.sqrt((d ** 2).sum(1) + 1e-6)
    assert abs(float(bl.sum()) - e.sum()) < 1e-3 * e.sum()
    g = from_bf16(dz.cpu().numpy()).reshape(P, 16)
    np.testing.assert_allclose(g[:, :2], d / e[:, None] / P, rtol=1e-2, atol=1e-9)
    assert np.all(g[:, 2:] == 0)
    h = to_bf16(rng.normal(size=P))
    dh = to_bf16(rng.normal(size=P))
    out = torch.empty(P, dtype=torch.int16, device="cuda:0")
    dhd, hd = dev(dh), dev(h)
    V.check(V.lib().vs_nn_lrelu_bwd(C.c_void_p(dhd.data_ptr()), C.c_void_p(hd.data_ptr()),
                                    C.c_void_p(out.data_ptr()), P, 0.1, None), "lrelu")
    want = np.where(from_bf16(h) > 0, from_bf16(dh), 0.1 * from_bf16(dh))
    np.testing.assert_allclose(from_bf16(out.cpu().numpy()), want, rtol=1e-2, atol=0)
    w = rng.normal(size=64).astype(np.float32)
    gr = rng.normal(size=64).astype(np.float32)
    wd, md, vd = dev(w), torch.zeros(64, device="cuda:0"), torch.zeros(64, device="cuda:0")
    grd = dev(gr)
    for step in (1, 2):
        V.check(V.lib().vs_nn_adam(C.c_void_p(wd.data_ptr()), C.c_void_p(md.data_ptr()), C.c_void_p(vd.data_ptr()),
                                   C.c_void_p(grd.data_ptr()), None, 64, 1e-2, 0.9, 0.999, 1e-8, step, None), "adam")
    m = v = 0
    ww = w.astype(np.float64)
    for step in (1, 2):
        m = 0.9 * m + 0.1 * gr
        v = 0.999 * v + 0.001 * gr.astype(np.float64) ** 2
        ww = ww - 1e-2 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
    np.testing.assert_allclose(wd.cpu().numpy(), ww, rtol=1e-5, atol=1e-6)


def test_plain_flow_context_matches_oracle():
    from tests.test_oracle_flow import _pyr, texture
    T = texture(96, 200, 3, sigma=2.0)
    rng = np.random.default_rng(3)
    M = np.roll(T, (1, 2), axis=(0, 1)) + rng.normal(size=T.shape).astype(np.float32)
    M = np.clip(np.round(M), 0, 255).astype(np.float32)
    T = np.round(T).astype(np.float32)
    pf = V.PlainFlow(200, 96)
    ftm, fmt = pf(dev(T), dev(M))
    lam = V.default_params().lk_lambda
    want_tm = O.pyramid_flow(_pyr(T), _pyr(M), lam=lam)
    want_mt = O.pyramid_flow(_pyr(M), _pyr(T), lam=lam)
    np.testing.assert_array_equal(ftm.cpu().numpy(), want_tm)
    np.testing.assert_array_equal(fmt.cpu().numpy(), want_mt)
    yt2, ym2 = pf.level(2)
    np.testing.assert_array_equal(yt2.cpu().numpy(), _pyr(T)[2])


def test_training_reduces_the_loss():
    from paper_2308_09209_amd import train_surrogate as TS
    data = TS.build_dataset(96, H=256, W=128, max_disp=6.0, seed=3, chunk=32, log=say)
    net = S.Net(seed=0)
    n_tr, n = TS.split(data, 16)
    before = TS.evaluate(net, data, n_tr, n)
    hist, after = TS.train(net, data, steps=200, batch=8, lr=2e-3, log=say, val=16)
    say(f"[training] held-out EPE {before:.4f} -> {after:.4f} level-2 px; training EPE "
        f"{hist[0][1]:.4f} -> {hist[-1][1]:.4f}")
    assert after < 0.8 * before
    # weights survive a save / load round trip bit for bit
    net2 = S.Net.from_blob(net.blob())
    for a, b in zip(net.w16, net2.w16):
        assert torch.equal(a, b)
