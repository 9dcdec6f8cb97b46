"""The no-allocation classifier (lbm_classify_series_noalloc) against the
allocating one (lbm_classify_series), through the C ABI: the same series,
the same records bit for bit, on two calls in a row (the second smaller, so
it reuses the first call's work memory), on a non-default stream; and the
size limit of its fixed work array is enforced before anything is issued."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    from paper_2211_05009_amd import lbm as mod
    return mod


def mixed_series(ns, n, seed):
    """Steady, periodic, modulated, drifting and noisy rows (seeded)."""
    rng = np.random.default_rng(seed)
    k = np.arange(n, dtype=np.float64)
    rows = []
    for i in range(ns):
        kind = i % 5
        if kind == 0:
            r = np.full(n, 0.3) + 1e-9 * rng.standard_normal(n)
        elif kind == 1:
            r = np.sin(2 * np.pi * k / (40 + 3 * i)) + 1e-3 * rng.standard_normal(n)
        elif kind == 2:
            r = np.sin(2 * np.pi * k / 57) * (1 + 0.3 * np.sin(2 * np.pi * k / 403))
        elif kind == 3:
            r = np.exp(-k / (n / 2)) + 1e-6 * rng.standard_normal(n)
        else:
            r = np.cumsum(rng.standard_normal(n))
        rows.append(r)
    return np.stack(rows)


def same(a, b):
    for key in a:
        x, y = a[key], b[key]
        if isinstance(x, float) and math.isnan(x):
            assert math.isnan(y), key
        else:
            assert x == y, (key, x, y)


def test_noalloc_matches_the_allocating_classifier(lbm):
    import torch
    stream = torch.cuda.Stream()
    rec = lbm.ct.sizeof(lbm.FlowState)
    # second call smaller: fewer, shorter series in a wider row stride
    for ns, n, ld, seed in ((60, 6000, 6000, 0), (9, 700, 1000, 1)):
        host = np.zeros((ns, ld))
        host[:, :n] = mixed_series(ns, n, seed)
        full = torch.tensor(host, dtype=torch.float64, device="cuda")
        dev = full[:, :n]
        ref = lbm.lbm_classify_series(dev, 1e-6, 0.05)
        out = torch.full((ns * rec,), 0xAB, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        lbm.lbm_classify_series_noalloc(dev, 1e-6, 0.05, out, stream=stream)
        stream.synchronize()
        got = lbm.flow_states_from_bytes(out.cpu().numpy().tobytes(), ns)
        assert len(got) == len(ref) == ns
        for a, b in zip(got, ref):
            same(a, b)
        states = {r["state"] for r in ref}
        assert {"steady", "periodic"} <= states, states


def test_noalloc_rejects_work_beyond_its_array(lbm):
    import torch
    n = 10_000
    limit = (4 << 20) // (2 * n + 8)           # 209 series of 10,000 samples
    dev = torch.zeros((limit + 1, n), dtype=torch.float64, device="cuda")
    out = torch.empty(((limit + 1) * lbm.ct.sizeof(lbm.FlowState),), dtype=torch.uint8,
                      device="cuda")
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_classify_series_noalloc(dev, 1e-6, 0.05, out)
    assert e.value.code == lbm.LBM_EINVAL
    assert "32 MiB" in str(e.value)
    # exactly at the limit it runs
    lbm.lbm_classify_series_noalloc(dev[:limit], 1e-6, 0.05, out)
    torch.cuda.synchronize()
    got = lbm.flow_states_from_bytes(out.cpu().numpy().tobytes(), limit)
    assert all(r["state"] == "steady" for r in got)
