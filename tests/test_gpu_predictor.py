"""The size predictor's device kernels (forward, gradient, Adam) against the
fp64 reference perceptron, and what the trained predictor gains the request
server over reserving one result pair per input byte."""
import math

import numpy as np
import pytest

import mlp_ref
import paper_2505_04431_amd as kc
import synth
from gpu_util import assert_same, to_device
from paper_2505_04431_amd import predictor

pytestmark = pytest.mark.gpu


def dev():
    import torch
    return torch.device("cuda:0")


@pytest.mark.parametrize("F,H,B", [(7, 16, 257), (10, 32, 1000), (1, 1, 3)])
def test_forward_and_gradient_match_reference(F, H, B):
    import torch
    rng = np.random.Generator(np.random.PCG64(F * 100 + H))
    net = kc.Predictor(F, H, seed=5)
    p = net.params().astype(np.float64)
    p += rng.normal(0, 0.1, size=p.size)  # biases away from zero too
    net.set_params(p.astype(np.float32))
    p32 = net.params().astype(np.float64)
    X = rng.normal(size=(B, F)).astype(np.float32)
    t = rng.normal(size=B).astype(np.float32)
    xt, tt = torch.from_numpy(X).to(dev()), torch.from_numpy(t).to(dev())
    y = net.forward(xt).cpu().numpy()
    np.testing.assert_allclose(y, mlp_ref.forward(p32, X, F, H), rtol=1e-4, atol=1e-5)
    loss = net.gradient(xt, tt)
    assert loss == pytest.approx(mlp_ref.loss(p32, X, t, F, H), rel=1e-4)
    g = net.grads()
    want = mlp_ref.grad(p32, X, t, F, H)
    np.testing.assert_allclose(g, want, rtol=1e-3, atol=1e-5 * max(1.0, np.abs(want).max()))
    # deterministic: the same batch gives the same bits
    net.gradient(xt, tt)
    assert np.array_equal(net.grads(), g)
    net.close()


def test_adam_training_fits_a_smooth_function():
    import torch
    rng = np.random.Generator(np.random.PCG64(9))
    X = rng.uniform(-2, 2, size=(2000, 3)).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2 - 0.3 * X[:, 2]).astype(np.float32)
    net = kc.Predictor(3, 32, seed=1)
    xt, tt = torch.from_numpy(X).to(dev()), torch.from_numpy(t).to(dev())
    first = net.gradient(xt, tt)
    for s in range(1500):
        net.gradient(xt, tt, want_loss=False)
        net.adam_step(1e-2)
    last = net.gradient(xt, tt)
    assert last < first / 20, (first, last)
    p = net.params().astype(np.float64)
    np.testing.assert_allclose(net.forward(xt).cpu().numpy(), mlp_ref.forward(p, X, 3, 32),
                               rtol=1e-4, atol=1e-4)
    net.close()


def served_jobs(seed, n, max_genome=400_000):
    specs = synth.c5_jobs(n, seed=synth.CONFIG_SEED_BASE + 5 + seed)
    out = []
    for sp in specs:
        sp = dict(sp)
        sp["genome_len"] = int(min(max_genome, max(2_000, sp["genome_len"] // 100)))
        sp["read_len"] = min(sp["read_len"], max(150, sp["genome_len"] // 4))
        r, o = synth.c5_job_reads(sp, seed=synth.CONFIG_SEED_BASE + 5 + seed, threads=8)
        out.append((r, o, sp["k"]))
    return out


def featurise(jobs):
    import torch
    X, lnd, dev_in = [], [], []
    for r, o, k in jobs:
        rt, ot = to_device(r, o)
        f, _ = predictor.job_features(rt, ot, k)
        keys, cnts = kc.count(rt, ot, k)
        X.append(f)
        lnd.append(math.log(max(1, cnts.numel())))
        dev_in.append((rt, ot, k, int(cnts.numel())))
    torch.cuda.synchronize()
    return np.array(X), np.array(lnd), dev_in


def test_predictor_gain_in_the_server():
    """Trained on jobs of the served recipe counted in full, evaluated on other
    jobs: its reservations are far closer to the true result size than one pair
    per input byte, and the server's results are unchanged by the hints."""
    import torch
    train = [j for s in range(11, 19) for j in served_jobs(s, 40)]
    test = served_jobs(40, 40)
    Xtr, ytr, _ = featurise(train)
    Xte, yte, dev_te = featurise(test)
    sp = predictor.SizePredictor(hidden=16, seed=3)
    hist = sp.fit(Xtr, ytr, steps=3000, lr=3e-3)
    assert hist[-1] < hist[0]
    err = np.abs(sp.predict_ln(Xte) - yte)
    assert np.median(err) < 0.2, np.median(err)
    hints = [sp.hint(x) for x in Xte]
    pair = lambda k: 20 if k > 32 else 12
    actual = sum(d * pair(k) for (_, _, k, d) in dev_te)
    bound = sum(int(rt.numel()) * pair(k) for (rt, _, k, _) in dev_te)
    hinted = sum(min(h, int(rt.numel())) * pair(k) for h, (rt, _, k, _) in zip(hints, dev_te))
    over_bound, over_hint = bound - actual, max(0, hinted - actual)
    print("result bytes: actual %d, reserved by bound %d, by predictor %d; median |ln err| %.3f"
          % (actual, bound, hinted, np.median(err)), flush=True)
    assert over_hint < over_bound / 4
    misses = sum(h < d for h, (_, _, _, d) in zip(hints, dev_te))
    assert misses <= len(hints) // 10
    # served with and without hints: identical results
    results = {}
    for use in (False, True):
        srv = kc.Server(budget_bytes=8 << 30, workers=4)
        ids = [srv.submit(rt, ot, k, P=16, distinct_hint=(h if use else 0))
               for h, (rt, ot, k, _) in zip(hints, dev_te)]
        out = []
        for j in ids:
            assert srv.wait(j) == "done"
            kk, cc = srv.result(j)
            out.append((kk.cpu().numpy().view(np.uint64), cc.cpu().numpy().view(np.uint32)))
            srv.release(j)
        st = srv.stats()
        assert st["result_bytes_actual"] == actual
        results[use] = out
        srv.close()
    for a, b in zip(results[False], results[True]):
        assert_same(a, b, "hinted vs unhinted")
    sp.close()
