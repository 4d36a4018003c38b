"""Training driver of the output-size predictor (argument marshalling and
orchestration only; features, targets, training and inference run in the
library's kernels).

Training rows come from the symbolic pass of each training product
(msp_training_rows); mini-batch indices are drawn on the host from a seeded
generator and uploaded once; the capacity margin delta is the 0.99 quantile
of the training residuals.
"""
from __future__ import annotations

import numpy as np

from . import binding, gen


def training_set(h: binding.Handle, products):
    """Concatenated (features, targets) device tensors of all rows of the
    given (A, B) device-matrix pairs."""
    import torch
    rows = sum(A.nrows for A, _ in products)
    feats = torch.empty((max(rows, 1), 8), dtype=torch.float32, device=f"cuda:{h.device}")
    targets = torch.empty(max(rows, 1), dtype=torch.float32, device=f"cuda:{h.device}")
    o = 0
    for A, B in products:
        h.training_rows(A, B, feats[o:o + A.nrows], targets[o:o + A.nrows])
        o += A.nrows
    return feats[:rows], targets[:rows]


def train(h: binding.Handle, feats, targets, steps=2000, batch=4096, seed=0, lr=1e-3,
          init_seed=0, quantile=0.99):
    """Train a fresh predictor; returns (predictor, losses, delta)."""
    import torch
    pred = binding.Predictor(h, gen.mlp_init(init_seed).astype(np.float32))
    idx = gen.minibatch_indices(feats.shape[0], batch, steps, seed)
    didx = torch.from_numpy(idx).to(feats.device)
    losses = pred.train(feats, targets, didx, lr=lr)
    delta = pred.calibrate(feats, targets, quantile)
    return pred, losses, delta


def fixed_capacity_params(b3: float) -> np.ndarray:
    """A network that outputs the constant b3 (all weights zero): b3 = +8
    makes every capacity the upper bound min(prod, n); b3 = -8 the lower
    bound max nnz(B(k,:))."""
    p = np.zeros(binding.NPARAM, dtype=np.float32)
    p[-1] = b3
    return p


def linear_fit_params(feats_host: np.ndarray, targets_host: np.ndarray) -> np.ndarray:
    """A network computing y = a + b * x1 (x1 = log2(1+prod)/16), the least
    squares fit on the training rows: h1_0 = relu(x1) = x1, h2_0 = h1_0,
    y = W3_0 h2_0 + b3."""
    x1 = feats_host[:, 1].astype(np.float64)
    t = targets_host.astype(np.float64)
    A = np.stack([np.ones_like(x1), x1], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, t, rcond=None)
    p = np.zeros(binding.NPARAM, dtype=np.float32)
    p[0 * 8 + 1] = 1.0                      # W1[0][1]
    p[576 + 0 * 64 + 0] = 1.0               # W2[0][0]
    p[4736 + 0] = b                         # W3[0]
    p[4800] = a                             # b3
    return p


def main(argv=None):
    """Train the predictor on training members of the mixed suite (by default
    the full-size members of the held-out member's family), then time that
    held-out member's one-pass product against the plain product and print
    the learned-path statistics."""
    import argparse
    import time
    import torch
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--member", type=int, default=23, help="held-out suite index (index = 3 mod 4)")
    ap.add_argument("--train-members", type=int, default=12, help="first N training members")
    ap.add_argument("--any-family", action="store_true", help="train on members of every family")
    ap.add_argument("--scale", type=int, default=0, help="training members built 2^-scale smaller")
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    suite = gen.learned_suite()
    test = [m for m in suite if m.index == a.member and m.held_out]
    if not test:
        raise SystemExit(f"member {a.member} is not a held-out member")
    h = binding.Handle(0)
    prods = []
    pool = [m for m in suite if not m.held_out and (a.any_family or m.family == test[0].family)]
    for m in pool[:a.train_members]:
        d = binding.DeviceCSR.from_host(m.build(scale_down=a.scale), "cuda:0")
        prods.append((d, d))
    feats, targets = training_set(h, prods)
    del prods
    pred, losses, delta = train(h, feats, targets, steps=a.steps, seed=0)
    print(f"trained on {int(feats.shape[0])} rows: loss {losses[0]:.4f} -> {float(np.mean(losses[-20:])):.5f}, "
          f"delta {delta:.4f}", flush=True)
    del feats, targets
    M = test[0].build()
    dM = binding.DeviceCSR.from_host(M, "cuda:0")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(a.reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)) * 1e3

    t_plain = timed(lambda: h.spgemm(dM, dM))
    t_learn = timed(lambda: h.spgemm_learned(pred, dM, dM))
    _, st = h.spgemm_learned(pred, dM, dM)
    print(f"member {a.member} ({test[0].family}, {M.nrows} rows, nnz(A) {M.nnz}): plain {t_plain:.3f} ms, "
          f"learned {t_learn:.3f} ms ({t_plain / t_learn:.3f}x); overflow rows {st['overflow_rows']}, "
          f"sum cap / nnz {st['sum_cap'] / max(st['nnz'], 1):.3f}", flush=True)
    pred.close()
    h.close()


if __name__ == "__main__":
    main()
