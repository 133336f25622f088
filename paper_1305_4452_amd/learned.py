"""Learned initial guess for -div(kappa grad u) = lambda e^u on a 64x64-element, degree-3 mesh.

Pipeline (every numerical step runs in libiga's HIP kernels; this module only orchestrates):
  1. instances: log kappa on 32x32 cells and lambda (seeded, from `inputs.learned_instance`);
  2. targets: plain Newton solutions from the zero guess by the batched solver; instances where
     it fails (no solution near the fold for that kappa) are rejected and counted;
  3. training: the device network (igann_*) on standardised inputs and targets with Adam;
  4. use: guess = network output (interior coefficients, zero boundary); if its error estimate
     ||P^{-1} R(guess)|| (P the fast-diagonalisation preconditioner, iga_batch_error_estimates)
     is larger than that of the zero guess, the zero guess is used instead, and plain Newton from
     the zero guess is the judge of the converged answer.
"""
from __future__ import annotations

import math
import time

import numpy as np

import inputs

from . import IGABatch, GuessNet, IGA_FP64

NEL, P, NCELL, NIN = 64, 3, 32, 65


def instances(indices, seed=5, log=None):
    out = []
    for k, i in enumerate(indices):
        logk, lam, w = inputs.learned_instance(int(i), seed=seed, nel=NEL, p=P, ncell=NCELL)
        out.append((logk, lam, w))
        if log and (k + 1) % 5000 == 0:
            log(f"drew {k + 1} instances")
    return out


def interior(U):
    return np.asarray(U).reshape(NEL + P, NEL + P)[1:-1, 1:-1].reshape(-1)


def full_from_interior(v):
    U = np.zeros((NEL + P, NEL + P))
    U[1:-1, 1:-1] = np.asarray(v).reshape(NIN, NIN)
    return U.reshape(-1)


def solve_zero(ws, chunk=1000, atol=1e-10, max_newton=50, log=None):
    """Plain Newton from the zero guess for every workload (batched).  Returns the solutions,
    the per-instance reports and the total solve time."""
    import torch
    sols, reps, t_solve = [], [], 0.0
    for s in range(0, len(ws), chunk):
        part = ws[s:s + chunk]
        b = IGABatch(part)
        U = torch.zeros(b.N, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t = time.perf_counter()
        per, _ = b.newton_solve(U, atol=atol, max_newton=max_newton, raise_on_fail=False)
        torch.cuda.synchronize()
        t_solve += time.perf_counter() - t
        sols += b.unpack(U.cpu().numpy())
        reps += per
        b.close()
        if log:
            log(f"solved {min(s + chunk, len(ws))}/{len(ws)} from the zero guess ({t_solve:.1f} s)")
    return sols, reps, t_solve


class Standardiser:
    def __init__(self, logk, lam, tgt):
        self.k_mu, self.k_sd = float(np.mean(logk)), float(np.std(logk)) + 1e-12
        self.l_mu, self.l_sd = float(np.mean(lam)), float(np.std(lam)) + 1e-12
        self.t_mu = np.mean(tgt, axis=0)
        self.t_sd = float(np.std(tgt - self.t_mu)) + 1e-12

    def x(self, logk, lam):
        logk = np.asarray(logk).reshape(-1, NCELL, NCELL)
        lam = np.asarray(lam).reshape(-1)
        X = np.empty((len(lam), 2, NCELL, NCELL), dtype=np.float32)
        X[:, 0] = (logk - self.k_mu) / self.k_sd
        X[:, 1] = ((lam - self.l_mu) / self.l_sd)[:, None, None]
        return X

    def t(self, tgt):
        return ((np.asarray(tgt) - self.t_mu) / self.t_sd).astype(np.float32)

    def inv(self, y):
        return np.asarray(y, dtype=np.float64) * self.t_sd + self.t_mu

    def state(self):
        return dict(k_mu=self.k_mu, k_sd=self.k_sd, l_mu=self.l_mu, l_sd=self.l_sd, t_mu=self.t_mu.tolist(),
                    t_sd=self.t_sd)


def init_weights(seed=11):
    """He-uniform weights and small biases from the seeded generator (flat igann layout)."""
    shapes = [("W0", (64, 2, 3, 3), 2 * 9), ("b0", (64,), 0), ("W1", (64, 64, 3, 3), 64 * 9), ("b1", (64,), 0),
              ("W2", (64, 64, 4, 4), 64), ("b2", (64,), 0), ("W3", (64, 1, 2, 2), 64 * 4), ("b3", (1,), 0)]
    out = []
    for k, (name, shp, fan) in enumerate(shapes):
        n = int(np.prod(shp))
        if fan:
            bound = math.sqrt(6.0 / fan)
            out.append(inputs.uniform(seed, 100 + k, n, -bound, bound))
        else:
            out.append(np.zeros(n))
    return np.concatenate(out).astype(np.float32)


def train(net, X, T, epochs=20, batch=128, lr=2e-3, seed=12, log=None):
    """Adam with a cosine learning-rate decay over all steps; minibatches in seeded order."""
    import torch
    n = len(X)
    Xd = torch.as_tensor(X, device="cuda")
    Td = torch.as_tensor(T, device="cuda")
    steps = epochs * max(1, n // batch)
    k = 0
    hist = []
    for ep in range(epochs):
        order = np.argsort(inputs.uniform(seed, ep, n))
        tot, cnt = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            idx = torch.as_tensor(order[s:s + batch], device="cuda")
            xb = Xd.index_select(0, idx).contiguous()
            tb = Td.index_select(0, idx).contiguous()
            cur = lr * 0.5 * (1 + math.cos(math.pi * k / steps))
            want = (s + batch > n - batch)
            loss = net.train_step(xb, tb, cur, want_loss=True)
            tot += loss
            cnt += 1
            k += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4e}")
    return hist


def predict(net, std, logk, lam, batch=None, smooth=0):
    """Network output -> interior coefficients: the network predicts the standardised U/lambda
    (which removes the lambda scale, u ~ lambda v for small lambda); libiga un-standardises and
    multiplies by lambda.  Batches of `batch` instances (default: as many as the network was
    created for); the guesses are copied back once."""
    import torch
    batch = batch or net.bmax
    X = torch.as_tensor(std.x(logk, lam), device="cuda")
    lam = torch.as_tensor(np.asarray(lam, dtype=np.float32).reshape(-1), device="cuda")
    mu = torch.as_tensor(std.t_mu, dtype=torch.float32, device="cuda")
    out = []
    for s in range(0, len(X), batch):
        y = net.forward(X[s:s + batch])
        net.postprocess(y, mu, std.t_sd, lam[s:s + batch], smooth)
        out.append(y)
    return torch.cat(out).cpu().numpy().astype(np.float64)


def _solve_from(b, starts, atol, max_newton=50, U=None):
    """Newton on an existing batch from the given starts; returns solutions, reports, seconds.  With a
    device buffer U (reused across calls) the batch's captured step graph is reused too."""
    import torch
    if U is None:
        U = torch.as_tensor(b.pack(starts), device="cuda")
    else:
        U.copy_(torch.as_tensor(b.pack(starts)))
    torch.cuda.synchronize()
    t = time.perf_counter()
    per, _ = b.newton_solve(U, atol=atol, max_newton=max_newton, raise_on_fail=False)
    torch.cuda.synchronize()
    return b.unpack(U.cpu().numpy()), per, time.perf_counter() - t


def _residual_norms(b, starts):
    """||R(U)|| of every start (a Newton call with no steps evaluates the residual only)."""
    import torch
    U = torch.as_tensor(b.pack(starts), device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    per, _ = b.newton_solve(U, atol=0.0, max_newton=0, raise_on_fail=False)
    torch.cuda.synchronize()
    return np.array([p["res_norm0"] for p in per]), time.perf_counter() - t


def _error_estimates(b, starts):
    """||P^{-1} R(U)|| of every start (the fast-diagonalisation estimate of its error)."""
    import torch
    U = torch.as_tensor(b.pack(starts), device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    est = b.error_estimates(U)
    return est, time.perf_counter() - t


def evaluate(net, std, test, sols_ref, atol=1e-10, chunk=1000, corrupt=None):
    """Newton from the zero guess, from the raw learned guess, and from the learned guess with
    the check (fall back to zero when the guess's error estimate ||P^{-1} R(guess)|| exceeds
    that of the zero guess, or is not finite), all on the same instances and to the same absolute
    tolerance.  A run counts as wrong when it does not converge or lands on a different solution
    than Newton from zero (e.g. the upper Bratu branch).  `fallbacks_residual_norm` counts the
    guesses the plain residual-norm test ||R(guess)|| > ||R(0)|| would have rejected.
    `corrupt(guesses)` (tests only) perturbs the guesses to exercise the fallback."""
    import torch
    ws = [w for _, _, w in test]
    predict(net, std, [test[0][0]], [test[0][1]])   # untimed: first launches load the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    guesses = predict(net, std, [l for l, _, _ in test], [lam for _, lam, _ in test])
    if corrupt is not None:
        guesses = corrupt(guesses)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    Ug = [full_from_interior(g) for g in guesses]
    res = {"zero": dict(iters=[], time=0.0, wrong=0), "learned_raw": dict(iters=[], time=t_infer, wrong=0),
           "learned_checked": dict(iters=[], time=t_infer, wrong=0)}
    fallbacks = fallbacks_res = 0
    for s in range(0, len(ws), chunk):
        part = ws[s:s + chunk]
        zeros = [np.zeros_like(u) for u in Ug[s:s + chunk]]
        raw = [np.nan_to_num(u, nan=0.0, posinf=0.0, neginf=0.0) for u in Ug[s:s + chunk]]
        b = IGABatch(part)                 # set-up (untimed), shared by every start
        rg, _ = _residual_norms(b, Ug[s:s + chunk])
        rz, _ = _residual_norms(b, zeros)
        fallbacks_res += int((~np.isfinite(rg) | (rg > rz)).sum())
        eg, t1 = _error_estimates(b, Ug[s:s + chunk])
        ez, t2 = _error_estimates(b, zeros)
        t_check = t1 + t2
        bad = ~np.isfinite(eg) | (eg > ez)
        fallbacks += int(bad.sum())
        checked = [zeros[i] if bad[i] else Ug[s + i] for i in range(len(part))]
        Ubuf = torch.empty(b.N, dtype=torch.float64, device="cuda")
        _solve_from(b, zeros, atol, U=Ubuf)   # untimed: captures the step graph the timed solves replay
        for key, starts, extra in (("zero", zeros, 0.0), ("learned_raw", raw, 0.0), ("learned_checked", checked, t_check)):
            out, per, dt = _solve_from(b, starts, atol, U=Ubuf)
            r = res[key]
            r["time"] += dt + extra
            for i in range(len(part)):
                ref = sols_ref[s + i]
                ok = per[i]["converged"] and np.abs(out[i] - ref).max() <= 1e-6 * max(np.abs(ref).max(), 1e-30)
                r["wrong"] += int(not ok)
                r["iters"].append(per[i]["newton_iters"])
        b.close()
    summ = dict(instances=len(ws), inference_s=t_infer, fallbacks=fallbacks, fallbacks_residual_norm=fallbacks_res,
                guess_rel_error_mean=float(np.mean([np.linalg.norm(full_from_interior(g) - u) / np.linalg.norm(u)
                                                    for g, u in zip(guesses, sols_ref)])))
    for key, r in res.items():
        summ[key] = dict(newton_iters_mean=float(np.mean(r["iters"])), time_s=r["time"], wrong=r["wrong"])
    return summ


LAP_WEIGHT = 0.0

# Algorithmic multiply-adds x 2 per sample (stride and padding zeros not counted): forward = conv 3x3
# 2->64 on 32^2 + conv 3x3 s2 64->64 to 16^2 + transposed conv 4x4 s4 64->64 to 64^2 + transposed conv 2x2
# 64->1 to 65^2; a training step adds both gradients of the three inner layers and the weight gradient
# of the first.
FWD_FLOP = 2.0 * (64 * 2 * 9 * 32 * 32 + 64 * 64 * 9 * 16 * 16 + 64 * 64 * 16 * 16 * 16 + 64 * 4 * 64 * 64)
TRAIN_FLOP = FWD_FLOP + 2.0 * (2 * 64 * 4 * 64 * 64 + 2 * 64 * 64 * 16 * 16 * 16 + 2 * 64 * 64 * 9 * 16 * 16
                               + 64 * 2 * 9 * 32 * 32)
BF16_PEAK_TFLOPS = 2500.0


def run(n_train=20000, n_test=2000, epochs=40, batch=128, lr=2e-3, log=print, lap_weight=LAP_WEIGHT):
    """Generate, train and evaluate; returns a summary dict."""
    t = time.perf_counter()
    tr = instances(range(n_train), log=log)
    te = instances(range(20000, 20000 + n_test), log=log)
    t_inst = time.perf_counter() - t
    if log:
        log(f"{len(tr)} + {len(te)} instances drawn ({t_inst:.1f} s)")
    sols_tr, reps_tr, t_gen = solve_zero([w for _, _, w in tr], log=log, max_newton=20)
    keep = [i for i, r in enumerate(reps_tr) if r["converged"]]
    rej_tr = len(tr) - len(keep)
    logk = np.array([tr[i][0] for i in keep])
    lam = np.array([tr[i][1] for i in keep])
    tgt = np.array([interior(sols_tr[i]) / tr[i][1] for i in keep])     # U / lambda
    std = Standardiser(logk, lam, tgt)
    net = GuessNet(batch_max=max(batch, 512))   # the held-out set is predicted in batches of 512
    net.set_weights(init_weights())
    net.set_loss(lap_weight)
    t = time.perf_counter()
    hist = train(net, std.x(logk, lam), std.t(tgt), epochs=epochs, batch=batch, lr=lr, log=log)
    t_train = time.perf_counter() - t
    sols_te, reps_te, t_zero = solve_zero([w for _, _, w in te], log=log, max_newton=20)
    keep_te = [i for i, r in enumerate(reps_te) if r["converged"]]
    te_k = [te[i] for i in keep_te]
    if log:
        log("evaluating the learned guess")
    ev = evaluate(net, std, te_k, [sols_te[i] for i in keep_te])
    steps = epochs * (len(keep) // batch)
    train_tf = TRAIN_FLOP * steps * batch / t_train / 1e12
    infer_tf = FWD_FLOP * len(te_k) / ev["inference_s"] / 1e12
    ev.update(train_instances=len(keep), train_rejected=rej_tr, test_rejected=len(te) - len(keep_te),
              epochs=epochs, lap_weight=lap_weight, loss_first=hist[0], loss_last=hist[-1], train_s=t_train,
              datagen_s=t_gen,
              instance_setup_s=t_inst,
              train_tflop_per_s=train_tf, train_frac_bf16_peak=train_tf / BF16_PEAK_TFLOPS,
              inference_tflop_per_s=infer_tf, inference_frac_bf16_peak=infer_tf / BF16_PEAK_TFLOPS,
              flop_note="algorithmic flops per sample: forward %.3g, training step %.3g; inference time includes "
                        "the host-side input preparation and the copy of the guesses back" % (FWD_FLOP, TRAIN_FLOP))
    return ev, net, std


if __name__ == "__main__":
    # python -m paper_1305_4452_amd.learned [n_train n_test epochs]: the learned-guess workload
    # (defaults: 20,000 training and 2,000 held-out instances, 40 epochs); prints the summary
    import json
    import sys

    args = [int(a) for a in sys.argv[1:4]]
    n_train, n_test, epochs = (args + [20000, 2000, 40][len(args):])[:3]
    t0 = time.perf_counter()
    summary, _, _ = run(n_train=n_train, n_test=n_test, epochs=epochs, log=lambda m: print(m, flush=True))
    summary["total_s"] = time.perf_counter() - t0
    print(json.dumps(summary), flush=True)
