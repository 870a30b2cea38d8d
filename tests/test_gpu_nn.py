"""GPU: the learned surrogate's matrix-core kernels against the FP64 oracle on
identical BF16 operands (forward, data gradient, weight gradient), its loss
and optimiser kernels, the network object (vs_nn_*: forward, backward, Adam,
save / load) against the oracle's FP64 training step, the label pooling, the
plain-flow label context, and a training smoke test."""
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
    blob = net.blob()
    net2 = S.Net.from_blob(blob)
    assert net2.blob() == blob


def test_training_on_variational_labels_reduces_the_loss():
    """The variational estimator as the label source (flow = 2 in the
    library's plain-flow context): its labels differ from the Lucas-Kanade
    ones, and a network trained on them learns them."""
    from paper_2308_09209_amd import train_surrogate as TS
    lk = TS.build_dataset(16, H=256, W=128, max_disp=6.0, seed=5, chunk=16, log=say)
    data = TS.build_dataset(96, H=256, W=128, max_disp=6.0, seed=5, chunk=16, log=say, label_flow=2)
    d = (data[2][:16] - lk[2]).norm(dim=-1).mean().item()
    say(f"[variational labels] mean difference to the Lucas-Kanade labels {d:.4f} level-2 px")
    assert 0.0 < d < 1.0
    net = S.Net(seed=0)
    n_tr, n = TS.split(data, 16)
    before = TS.evaluate(net, data, n_tr, n)
    _, after = TS.train(net, data, steps=200, batch=8, lr=2e-3, log=say, val=16)
    say(f"[variational labels] held-out EPE {before:.4f} -> {after:.4f} level-2 px")
    assert after < 0.8 * before


NET_LAYERS = ((16, 32), (32, 32), (32, 16))
NET_SIZES = [(23, 41), (16, 16), (5, 70)]


def _net_state(h):
    """master parameters and gradients of network object h, FP64 per layer:
    ([w], [b], [dw], [db])"""
    n = C.c_size_t()
    V.check(V.lib().vs_nn_params(h, None, None, C.byref(n), None), "params count")
    tp = torch.empty(n.value, dtype=torch.float32, device="cuda:0")
    tg = torch.empty_like(tp)
    V.check(V.lib().vs_nn_params(h, C.c_void_p(tp.data_ptr()), C.c_void_p(tg.data_ptr()), None, None), "params")
    torch.cuda.synchronize()
    flat_p, flat_g = tp.cpu().numpy().astype(np.float64), tg.cpu().numpy().astype(np.float64)
    ws, bs, dws, dbs, off = [], [], [], [], 0
    for ci, co in NET_LAYERS:
        nw = co * 9 * ci
        ws.append(flat_p[off:off + nw].reshape(co, 9, ci))
        dws.append(flat_g[off:off + nw].reshape(co, 9, ci))
        bs.append(flat_p[off + nw:off + nw + co])
        dbs.append(flat_g[off + nw:off + nw + co])
        off += nw + co
    assert off == n.value
    return ws, bs, dws, dbs


def _make_net(seed=3):
    spec = V.nn_spec(NET_LAYERS, in_live=16, alpha=0.1, max_pixels=4096)
    h = C.c_void_p()
    V.check(V.lib().vs_nn_create(C.byref(spec), seed, C.byref(h)), "vs_nn_create")
    return h


def test_network_forward_backward_matches_oracle_step():
    """One training step through the C ABI (vs_nn_forward + vs_nn_backward)
    against the oracle's FP64 step on the same BF16 weights, FP32 biases and
    inputs: prediction, loss and every layer's gradients.  The kernels keep
    hidden activations and back-propagated gradients in BF16 (unit roundoff
    2^-9), the oracle in FP64, so the bars are relative L2 errors a few such
    roundings allow: 1e-2 on the prediction and the loss, 3e-2 on gradients."""
    h = _make_net()
    rng = np.random.default_rng(8)
    P = sum(a * b for a, b in NET_SIZES)
    x = to_bf16(rng.normal(size=(P, 16)))
    lab = rng.normal(size=(P, 2)).astype(np.float32) * 0.3
    imgs = V.nn_images(NET_SIZES)
    xd, ld = dev(x), dev(lab)
    pred = torch.empty((P, 16), dtype=torch.float32, device="cuda:0")
    loss = torch.zeros((), dtype=torch.float32, device="cuda:0")
    V.check(V.lib().vs_nn_forward(h, C.c_void_p(xd.data_ptr()), C.byref(imgs), C.c_void_p(pred.data_ptr()), None), "fwd")
    V.check(V.lib().vs_nn_backward(h, C.c_void_p(ld.data_ptr()), C.c_void_p(loss.data_ptr()), None), "bwd")
    torch.cuda.synchronize()
    ws, bs, dws, dbs = _net_state(h)
    wq = [from_bf16(to_bf16(w)).reshape(w.shape) for w in ws]   # the kernels multiply BF16 weights
    r_loss, r_pred, r_dw, r_db = O.nn_train_step(wq, bs, from_bf16(x).reshape(P, 16), lab, NET_SIZES, 0.1)
    e_pred = rel_l2(pred.cpu().numpy().astype(np.float64), r_pred)
    e_loss = abs(float(loss.cpu()) / P - r_loss) / r_loss
    say(f"[network step] rel L2 prediction {e_pred:.2e}, loss {e_loss:.2e}")
    assert e_pred <= 1e-2 and e_loss <= 1e-2
    for li in range(len(NET_LAYERS)):
        e_w, e_b = rel_l2(dws[li], r_dw[li]), rel_l2(dbs[li], r_db[li])
        say(f"  layer {li}: rel L2 weight gradient {e_w:.2e}, bias gradient {e_b:.2e}")
        assert e_w <= 3e-2 and e_b <= 3e-2, li
    V.lib().vs_nn_destroy(h)


def test_network_adam_save_load():
    """vs_nn_adam_step against Adam written out in numpy on the object's own
    gradients; the weight file survives vs_nn_save / vs_nn_load byte for byte
    and gives the same prediction bit for bit; a file of another layer list is
    refused."""
    h = _make_net(4)
    rng = np.random.default_rng(9)
    P = 16 * 16
    imgs = V.nn_images([(16, 16)])
    x = dev(to_bf16(rng.normal(size=(P, 16))))
    lab = dev(rng.normal(size=(P, 2)).astype(np.float32))
    m = v = None
    for step in (1, 2):
        V.check(V.lib().vs_nn_forward(h, C.c_void_p(x.data_ptr()), C.byref(imgs), None, None), "fwd")
        V.check(V.lib().vs_nn_backward(h, C.c_void_p(lab.data_ptr()), None, None), "bwd")
        torch.cuda.synchronize()
        ws, bs, dws, dbs = _net_state(h)
        p0 = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in zip(ws, bs)])
        g = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in zip(dws, dbs)])
        m = 0.1 * g if m is None else 0.9 * m + 0.1 * g
        v = 0.001 * g ** 2 if v is None else 0.999 * v + 0.001 * g ** 2
        want = p0 - 1e-2 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
        V.check(V.lib().vs_nn_adam_step(h, 1e-2, 0.9, 0.999, 1e-8, None), "adam")
        torch.cuda.synchronize()
        ws2, bs2, _, _ = _net_state(h)
        got = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in zip(ws2, bs2)])
        np.testing.assert_allclose(got, want, rtol=1e-5, atol=1e-6)
    n = C.c_size_t()
    V.check(V.lib().vs_nn_save(h, None, 0, C.byref(n)), "size")
    buf = C.create_string_buffer(n.value)
    V.check(V.lib().vs_nn_save(h, buf, n.value, C.byref(n)), "save")
    blob = buf.raw
    h2 = _make_net(99)
    V.check(V.lib().vs_nn_load(h2, blob, len(blob)), "load")
    buf2 = C.create_string_buffer(n.value)
    V.check(V.lib().vs_nn_save(h2, buf2, n.value, C.byref(n)), "save 2")
    assert buf2.raw == blob
    p1 = torch.empty((P, 16), dtype=torch.float32, device="cuda:0")
    p2 = torch.empty_like(p1)
    V.check(V.lib().vs_nn_forward(h, C.c_void_p(x.data_ptr()), C.byref(imgs), C.c_void_p(p1.data_ptr()), None), "f1")
    V.check(V.lib().vs_nn_forward(h2, C.c_void_p(x.data_ptr()), C.byref(imgs), C.c_void_p(p2.data_ptr()), None), "f2")
    torch.cuda.synchronize()
    assert torch.equal(p1, p2)
    # the surrogate's production network: another layer list, refused
    prod = S.Net(seed=1, max_pixels=4096)
    assert V.lib().vs_nn_load(h2, prod.blob(), len(prod.blob())) == -1
    prod.close()
    V.lib().vs_nn_destroy(h)
    V.lib().vs_nn_destroy(h2)


def test_pool_flow_block_means():
    """vs_nn_pool_flow against block means written out in numpy (ragged last
    block row and column) for factors 1, 3 and 4."""
    rng = np.random.default_rng(10)
    h, w = 37, 50
    flow = rng.normal(size=(h, w, 2)).astype(np.float32) * 4
    fd = dev(flow)
    for f in (1, 3, 4):
        ho, wo = -(-h // f), -(-w // f)
        out = torch.empty((ho, wo, 2), dtype=torch.float32, device="cuda:0")
        V.check(V.lib().vs_nn_pool_flow(C.c_void_p(fd.data_ptr()), w, h, f, C.c_void_p(out.data_ptr()), None), "pool")
        torch.cuda.synchronize()
        want = np.zeros((ho, wo, 2))
        for Y in range(ho):
            for X in range(wo):
                want[Y, X] = flow[Y * f:(Y + 1) * f, X * f:(X + 1) * f].reshape(-1, 2).astype(np.float64).mean(0) / f
        np.testing.assert_allclose(out.cpu().numpy(), want, rtol=1e-5, atol=1e-6)


def test_flow_only_on_caller_strips_matches_oracle():
    """vs_flow_only (steps a5-a6 on a caller RGB strip pair, identity colour
    matrix) against the oracle: per-pixel luma, then its pyramidal flow in both
    directions, bit for bit; a second size re-plans the context's workspace."""
    from tests.test_oracle_flow import _pyr, texture
    from paper_2308_09209_amd.scenes import small_scene
    sc = small_scene(n_cams=2, W=200, H=110, overlap=0.35, ring=False, seed_config=5)
    st = V.Stitcher(sc.rig())
    lam = V.default_params().lk_lambda
    rng = np.random.default_rng(11)
    for h, w in ((96, 200), (64, 130)):
        chans = [texture(h, w, 20 + c, sigma=2.0) for c in range(3)]
        sj = np.stack(chans, -1)
        si = np.roll(sj, (1, 2), axis=(0, 1)) + rng.normal(scale=2.0, size=sj.shape)
        sj = np.clip(np.round(sj), 0, 255).astype(np.uint8)
        si = np.clip(np.round(si), 0, 255).astype(np.uint8)
        fij, fji = st.flow_only(torch.from_numpy(si).cuda(), torch.from_numpy(sj).cuda())
        yl = [np.array([[O.luma(*s[y, x]) for x in range(w)] for y in range(h)], np.float32) for s in (sj, si)]
        want_ij = O.pyramid_flow(_pyr(yl[0]), _pyr(yl[1]), lam=lam)
        want_ji = O.pyramid_flow(_pyr(yl[1]), _pyr(yl[0]), lam=lam)
        np.testing.assert_array_equal(fij.cpu().numpy(), want_ij)
        np.testing.assert_array_equal(fji.cpu().numpy(), want_ji)
        say(f"[flow_only {w}x{h}] median flow_ij {np.median(want_ij[8:-8, 8:-8], axis=(0, 1))}")
    st.close()
