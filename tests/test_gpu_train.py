"""rb_mlp_train (whole Adam steps inside the library) against the
layer-by-layer calls it replaces: input gather, rb_mlp_forward,
rb_mlp_loss, rb_mlp_backward and rb_mlp_adam in turn.

The fused step forms every intermediate from the same operands with the same
matrix-core sequence and element arithmetic, so the weights, the Adam moments
and the BF16 copy must agree bit for bit after several steps; only the loss
value, whose partial sums are added in another order, is compared to a
relative 1e-5.  Shapes cover the benchmark's surrogate (2 + 2 x 141 phase
inputs, 256 hidden, 282 outputs, batch 4,096), a ragged batch (not a
multiple of the 16-sample row blocks), narrow layers, and the shapes that
run the layer-by-layer path inside rb_mlp_train (two plain inputs; a
hidden width that is not a multiple of 64)."""
import numpy as np
import pytest
import torch

import rb_inputs as ri

pytestmark = pytest.mark.gpu


def _features(F, N, flo, fhi, seed):
    from paper_1805_06124_amd import _check, _ptr, load
    table = torch.empty(3 * N, dtype=torch.float64, device="cuda")
    _check("rb_chirp_table", load().rb_chirp_table(float(flo), float(fhi), N, _ptr(table), None))
    rows = np.sort(np.random.default_rng(seed).choice(N, F, replace=False)).astype(np.int64)
    return {"rows": torch.from_numpy(rows).cuda(), "table": table, "din": 2 + 2 * F}


def _pair(k, h, F, B, seed):
    from paper_1805_06124_amd import surrogate as sg
    w = ri.WORKLOADS["chirp_small_c128"]
    feats = _features(F, w.N, w.flo, w.fhi, seed) if F else None
    din = feats["din"] if feats else 2
    dout = 2 * k
    p = ri.mlp_init(seed, din, h, dout)
    ranges = (w.mlo, w.mhi, w.qlo, w.qhi)
    a = sg.Surrogate(k, p, ranges=ranges, hidden=h, batch=B, features=feats)
    b = sg.Surrogate(k, p, ranges=ranges, hidden=h, batch=B, features=feats)
    M = 3000
    params = torch.from_numpy(w.params(M=M)).cuda()
    targets = torch.from_numpy((0.2 * np.random.default_rng(seed + 1).standard_normal((M, dout))).astype(np.float32))
    return a, b, params, targets.cuda(), M


@pytest.mark.parametrize("k,h,F,B,steps", [(141, 256, 141, 4096, 3), (15, 64, 10, 1000, 4), (20, 128, 40, 512, 2),
                                           (20, 128, 40, 2056, 2), (47, 256, 0, 300, 2), (30, 100, 5, 257, 2)])
def test_train_matches_layer_by_layer(rb, k, h, F, B, steps):
    """Batches 4,096 and 512 give the row kernel a multiple of 8 workgroups
    (sample blocks handed out by XCD); 4,096 and 2,056 give the weight
    gradients 8 splits (one per XCD; at 2,056 the last split holds 40 rows
    and the row blocks keep their order); the others take neither."""
    a, b, params, targets, M = _pair(k, h, F, B, seed=11 + k)
    idx = torch.from_numpy(np.random.default_rng(k).integers(0, M, (steps, B))).cuda()
    lr = (1e-3 * (1.0 + np.arange(steps))).astype(np.float32)
    X = torch.empty((B, a.din), dtype=torch.float32, device="cuda")
    T = torch.empty((B, a.dout), dtype=torch.float32, device="cuda")
    Y = torch.empty((B, a.dout), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    la = []
    for s in range(steps):
        a.gather(params, targets, idx[s], X, T)
        a.forward(X, Y)
        a.loss_backward(X, Y, T, loss)
        a.adam(float(lr[s]))
        la.append(float(loss.item()))
    lb = torch.zeros(steps, dtype=torch.float32, device="cuda")
    b.train_steps(params, targets, idx, lr, lb)
    torch.cuda.synchronize()
    assert a.step == b.step == steps
    for name in ("p32", "m", "v", "p16"):
        ta, tb = getattr(a, name), getattr(b, name)
        assert torch.equal(ta, tb), (name, int((ta != tb).sum()))
    np.testing.assert_allclose(lb.cpu().numpy(), la, rtol=1e-5)
    # the trained weights serve predictions as before
    Ya = a.forward(X)
    Yb = b.forward(X)
    assert torch.equal(Ya, Yb)


def test_train_in_chunks_continues_adam(rb):
    """Two calls of 2 steps equal one call of 4 (the Adam step count and the
    moments carry over)."""
    a, b, params, targets, M = _pair(15, 64, 10, 1000, seed=5)
    idx = torch.from_numpy(np.random.default_rng(9).integers(0, M, (4, 1000))).cuda()
    lr = np.full(4, 2e-3, dtype=np.float32)
    a.train_steps(params, targets, idx, lr)
    b.train_steps(params, targets, idx[:2].contiguous(), lr[:2])
    b.train_steps(params, targets, idx[2:].contiguous(), lr[2:])
    torch.cuda.synchronize()
    for name in ("p32", "m", "v", "p16"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name


def test_pipelined_train_equals_plain_chunks(rb):
    """Surrogate.train (indices uploaded and losses read back through pinned
    double buffers while the device trains) gives the same weights and
    losses as a plain loop of rb_mlp_train calls over the same chunks, with
    a ragged last chunk."""
    a, b, params, targets, M = _pair(15, 64, 10, 1000, seed=6)
    steps, lr0 = 1234, 1e-3

    def index_fn(s0, c):
        return ri.batch_indices(77, M, 1000, c, s0)

    hist = a.train(params, targets, steps, index_fn, lr0=lr0, log_every=100)
    ref = []
    loss = torch.zeros(500, dtype=torch.float32, device="cuda")
    for s in range(0, steps, 500):
        c = min(500, steps - s)
        lr = 0.5 * lr0 * (1.0 + np.cos(np.pi * (s + np.arange(c)) / steps))
        b.train_steps(params, targets, torch.from_numpy(index_fn(s, c)).cuda(), lr, loss)
        lv = loss[:c].cpu().numpy()
        ref += [(s + j, float(lv[j])) for j in range(c) if (s + j) % 100 == 0 or s + j == steps - 1]
    torch.cuda.synchronize()
    assert hist == ref
    for name in ("p32", "m", "v", "p16"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
