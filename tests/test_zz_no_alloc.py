"""The allocation-free plain flow (vs_flow_run_noalloc) through the C ABI
against the context-owning entry point (vs_flow_create + vs_flow_run) on the
same seeded luma pairs: bit for bit, on consecutive calls whose shapes shrink
and grow again (the static workspace keeps the previous call's contents), and
once against the oracle's pyramidal flow."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2308_09209_amd import vstitch as V  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def luma_pair(h, w, seed):
    from tests.test_oracle_flow import texture
    T = texture(h, w, seed, sigma=2.0)
    rng = np.random.default_rng(seed + 100)
    M = np.roll(T, (1, -2), axis=(0, 1)) + rng.normal(size=T.shape).astype(np.float32)
    return np.round(T).astype(np.float32), np.clip(np.round(M), 0, 255).astype(np.float32)


def test_noalloc_flow_matches_context_flow_on_shrinking_and_growing_calls():
    # ragged tails: neither width is a multiple of the 64-px flow tile, nor
    # height of its rows; the second call is smaller, the third grows again
    shapes = [(200, 328, 5), (120, 200, 6), (260, 452, 7)]
    for h, w, seed in shapes:
        say(f"[noalloc] {w}x{h} seed {seed}")
        T, M = luma_pair(h, w, seed)
        yt, ym = dev(T), dev(M)
        pf = V.PlainFlow(w, h)
        want_tm, want_mt = pf(yt, ym)
        got_tm, got_mt = V.flow_run_noalloc(yt, ym)
        torch.cuda.synchronize()
        assert torch.equal(got_tm, want_tm), (w, h)
        assert torch.equal(got_mt, want_mt), (w, h)
        # one direction only, into caller tensors
        out = torch.full((h, w, 2), 7.0, dtype=torch.float32, device="cuda:0")
        V.flow_run_noalloc(yt, ym, flow_tm=out, flow_mt=False)
        torch.cuda.synchronize()
        assert torch.equal(out, want_tm)
        pf.close()


def test_noalloc_flow_matches_oracle():
    from tests.test_oracle_flow import _pyr
    T, M = luma_pair(96, 200, 3)
    got_tm, got_mt = V.flow_run_noalloc(dev(T), dev(M))
    lam = V.default_params().lk_lambda
    np.testing.assert_array_equal(got_tm.cpu().numpy(), O.pyramid_flow(_pyr(T), _pyr(M), lam=lam))
    np.testing.assert_array_equal(got_mt.cpu().numpy(), O.pyramid_flow(_pyr(M), _pyr(T), lam=lam))


def test_noalloc_flow_rejects_pairs_beyond_its_workspace():
    yt = torch.zeros((1000, 1000), dtype=torch.float32, device="cuda:0")
    with pytest.raises(V.VSError) as e:
        V.flow_run_noalloc(yt, yt.clone())
    assert e.value.status == -1
    # the library is still usable afterwards
    T, M = luma_pair(64, 96, 9)
    pf = V.PlainFlow(96, 64)
    want, _ = pf(dev(T), dev(M))
    got, _ = V.flow_run_noalloc(dev(T), dev(M), flow_mt=False)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    pf.close()
