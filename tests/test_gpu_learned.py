"""Learned initial guess: device network vs the FP64 reference (BF16 rounding at the same
points), training, and the residual-check fallback."""
import numpy as np
import pytest

import inputs
from oracle import nn_ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1305_4452_amd as iga  # noqa: E402
from paper_1305_4452_amd import learned  # noqa: E402


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-30)


def test_forward_and_gradients_match_reference():
    net = iga.GuessNet(batch_max=4)
    w = learned.init_weights(seed=3)
    net.set_weights(w)
    x = inputs.normal(7, 0, 3 * 2 * 32 * 32).reshape(3, 2, 32, 32).astype(np.float32)
    t = inputs.normal(8, 0, 3 * 65 * 65).reshape(3, -1).astype(np.float32)
    y = net.forward(torch.as_tensor(x, device="cuda")).cpu().numpy()
    yr, _ = nn_ref.forward(w.astype(np.float64), x.astype(np.float64), bf=True)
    assert rel(y, yr) < 2e-3
    for lw in (0.0, 0.5):
        net.set_loss(lw)
        loss, g = net.gradients(torch.as_tensor(x, device="cuda"), torch.as_tensor(t, device="cuda"))
        lr_, gr = nn_ref.loss_and_grad(w.astype(np.float64), x.astype(np.float64), t.astype(np.float64), bf=True,
                                       lap_weight=lw)
        assert abs(loss - lr_) < 1e-3 * lr_
        k = 0
        for name, shp in nn_ref.SHAPES:
            n = int(np.prod(shp))
            assert rel(g[k:k + n], gr[k:k + n]) < 5e-3, (lw, name)
            k += n
    assert np.array_equal(net.get_weights(), w)


def test_training_reduces_loss():
    net = iga.GuessNet(batch_max=32)
    net.set_weights(learned.init_weights(seed=4))
    x = inputs.normal(9, 0, 32 * 2 * 32 * 32).reshape(32, 2, 32, 32).astype(np.float32)
    tgt = np.tanh(x[:, 0, :, :].mean(axis=(1, 2)))[:, None] * np.ones((1, 65 * 65))
    xd, td = torch.as_tensor(x, device="cuda"), torch.as_tensor(tgt.astype(np.float32), device="cuda")
    first = net.train_step(xd, td, 1e-3)
    for _ in range(60):
        last = net.train_step(xd, td, 1e-3)
    assert last < 0.3 * first


def test_learned_pipeline_small_with_fallback():
    """Trained as the default benchmark trains it (2,000 instances, 12 epochs), the guess must remove at
    least half of the zero guess's error: mean relative L2 error < 0.5, against 1.0 for the zero guess
    (0.25 measured at this size)."""
    summary, net, std = learned.run(n_train=2000, n_test=100, epochs=12, log=None)
    assert summary["train_instances"] > 1700
    for key in ("zero", "learned_raw", "learned_checked"):
        assert summary[key]["wrong"] == 0, key
    assert summary["guess_rel_error_mean"] < 0.5
    assert summary["learned_checked"]["newton_iters_mean"] <= summary["zero"]["newton_iters_mean"]
    # a corrupted network output must fall back to the zero guess and still give the same answer
    test = learned.instances(range(20000, 20012))
    sols, reps, tz = learned.solve_zero([w for _, _, w in test])
    keep = [i for i, r in enumerate(reps) if r["converged"]]
    tk = [test[i] for i in keep]
    for bad in (lambda g: g * 100.0, lambda g: g * np.nan):
        ev = learned.evaluate(net, std, tk, [sols[i] for i in keep], corrupt=bad)
        assert ev["fallbacks"] == len(tk)
        assert ev["learned_checked"]["wrong"] == 0
        assert ev["learned_checked"]["newton_iters_mean"] == ev["zero"]["newton_iters_mean"]
