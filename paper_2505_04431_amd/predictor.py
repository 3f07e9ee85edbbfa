"""Estimate of a counting job's number of distinct keys, for the request
server's result reservation (``distinct_hint``).

Features of a job (all cheap): its size (bytes, reads, mean read length, k)
and the distinct/valid window counts of two prefixes of its reads (about 1%
and 3% of the bytes), counted by the library itself. Reads are sampled
uniformly from the genome, so a prefix is a random sample; how the distinct
fraction of the samples extrapolates to the whole job depends on coverage,
error rate and repeats, and that mapping is what the perceptron learns from
jobs counted in full. The network predicts the correction to a plain
extrapolation (the larger sample's distinct keys scaled by the read count:
exact when every window is distinct, too high when k-mers repeat), so it
only has to learn how far below that line a job falls. Training and
inference run in the library's own kernels (kc_pred_*). The estimate never
changes a count: a low one only makes the server account the result late.
"""
from __future__ import annotations

import math

import numpy as np

from . import kc

N_FEATURES = 10
SAMPLE_FRACS = (0.01, 0.03)


def job_features(reads, offsets, k: int, P: int = 1) -> tuple[np.ndarray, dict]:
    """Features of one job (device tensors as for kc.count). Returns the
    feature vector and the raw sample counts."""
    import torch
    n_reads = int(offsets.numel()) - 1
    ends = offsets[[0, n_reads]].cpu().numpy().view(np.uint64) if n_reads >= 0 else None
    n_bytes = int(ends[1] - ends[0]) if n_reads > 0 else 0
    raw = {"n_bytes": n_bytes, "n_reads": n_reads, "k": k}
    samples = []
    for frac in SAMPLE_FRACS:
        m = max(1, min(n_reads, int(math.ceil(n_reads * frac)))) if n_reads else 0
        if m:
            keys, cnts = kc.count(reads, offsets[:m + 1], k, P)
            d = int(cnts.numel())
            w = int(cnts.to(torch.int64).sum().item()) if d else 0
        else:
            d = w = 0
        samples.append((w, d))
    raw["samples"] = samples
    lg = lambda v: math.log(max(v, 1))
    mean_len = n_bytes / max(n_reads, 1)
    (w1, d1), (w2, d2) = samples
    f = [lg(n_bytes), lg(n_reads), lg(mean_len), k / 64.0, lg(w1), lg(d1), lg(w2), lg(d2),
         lg(d1) - lg(w1) if w1 else 0.0, lg(d2) - lg(w2) if w2 else 0.0]
    return np.array(f, dtype=np.float32), raw


def baseline_ln(features) -> np.ndarray:
    """ln of the plain extrapolation d2 * n_reads / m2 from the features."""
    F = np.atleast_2d(np.asarray(features, np.float64))
    n = np.exp(F[:, 1])
    m2 = np.maximum(1.0, np.ceil(n * SAMPLE_FRACS[1]))
    return F[:, 7] + np.log(n / m2)


class SizePredictor:
    """ln(distinct keys) from job features, trained on jobs counted in full."""

    def __init__(self, hidden: int = 16, seed: int = 7):
        self.net = kc.Predictor(N_FEATURES, hidden, seed)
        self.mu = np.zeros(N_FEATURES, np.float32)
        self.sd = np.ones(N_FEATURES, np.float32)
        self.t_mu, self.t_sd = 0.0, 1.0
        self.resid_sd = 1.0

    def _norm(self, X):
        return ((np.asarray(X, np.float32) - self.mu) / self.sd).astype(np.float32)

    def fit(self, X, ln_d, steps: int = 3000, lr: float = 3e-3, val_frac: float = 0.2,
            device=None) -> list[float]:
        """Full-batch Adam on the device over all but a seeded val_frac of the
        jobs; the spread of the errors on those held-out jobs sets the margin
        of hint(). Returns the training loss every 100 steps."""
        import torch
        X_all = np.asarray(X, np.float32)
        ln_all = np.asarray(ln_d, np.float64)
        perm = np.random.Generator(np.random.PCG64(len(ln_all))).permutation(len(ln_all))
        n_val = int(len(ln_all) * val_frac) if len(ln_all) >= 10 else 0
        val, tr = perm[:n_val], perm[n_val:]
        X = X_all[tr]
        y = (ln_all[tr] - baseline_ln(X)).astype(np.float32)
        self.mu = X.mean(axis=0)
        self.sd = np.maximum(X.std(axis=0), 1e-3).astype(np.float32)
        self.t_mu, self.t_sd = float(y.mean()), float(max(y.std(), 1e-3))
        dev = device or torch.device("cuda", torch.cuda.current_device())
        xt = torch.from_numpy(self._norm(X)).to(dev)
        tt = torch.from_numpy(((y - self.t_mu) / self.t_sd).astype(np.float32)).to(dev)
        hist = []
        for s in range(steps):
            loss = self.net.gradient(xt, tt, want_loss=(s % 100 == 0))
            if loss is not None:
                hist.append(loss)
            self.net.adam_step(lr)
        chk = val if n_val else tr
        err = self.predict_ln(X_all[chk], device=dev) - ln_all[chk]
        self.resid_sd = float(max(np.sqrt(np.mean(err * err)), 1e-3))
        return hist

    def predict_ln(self, X, device=None) -> np.ndarray:
        import torch
        dev = device or torch.device("cuda", torch.cuda.current_device())
        xt = torch.from_numpy(self._norm(np.atleast_2d(X))).to(dev)
        y = self.net.forward(xt).cpu().numpy().astype(np.float64)
        return y * self.t_sd + self.t_mu + baseline_ln(X)

    def hint(self, features, margin_sd: float = 2.0) -> int:
        """Distinct-key reservation for one job: the estimate raised by
        margin_sd residual standard deviations of the training fit."""
        ln = float(self.predict_ln(features)[0]) + margin_sd * self.resid_sd
        return max(1, int(math.ceil(math.exp(min(ln, 60.0)))))

    def close(self):
        self.net.close()
