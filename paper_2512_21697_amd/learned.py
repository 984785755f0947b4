"""Training and use of the learned initial guess (include/tdde_mlp.h) on solver-generated data.

Pipeline:
  1. ``collect_samples``: propagate a batch of pulse instances with the library's batched solver and
     draw random state entries every few steps: each training row holds psi_{n-3..n+1} at that entry,
     the field at t_n +- dt/2 and the spinor component.
  2. ``train``: minibatch Adam on the GPU with the library's forward / backward kernels.
  3. ``propagate``: run instances with a given guess mode ("zero", "prev", "mlp") and return the
     BiCGSTAB iterations of every instance-step; the solve tolerance is the same in every mode, so
     the states agree to the solver tolerance and only the iteration counts differ.
Host code here only moves data (sampling indices, copies); all arithmetic runs in the library.
"""
from __future__ import annotations

import math
import time

import numpy as np

from ._lib import GUESS_GIVEN, GUESS_PREV, GUESS_ZERO, STATS_DTYPE, Net, Solver, solve_opts

HIDDEN, N_FEAT = 256, 32


def init_params(seed: int, n_params: int) -> np.ndarray:
    """Uniform fan-in initialisation of W1, W2 and a zero last layer (the network starts as the
    fitted skip alone)."""
    rng = np.random.default_rng(seed)
    p = []
    p.append(rng.uniform(-1, 1, (HIDDEN, N_FEAT)) * math.sqrt(3.0 / 11.0))  # W1 (11 live features)
    p.append(np.zeros(HIDDEN))  # b1
    p.append(rng.uniform(-1, 1, (HIDDEN, HIDDEN)) * math.sqrt(3.0 / HIDDEN))  # W2
    p.append(np.zeros(HIDDEN))  # b2
    p.append(np.zeros((2, HIDDEN)))  # W3
    p.append(np.zeros(2))  # b3
    flat = np.concatenate([a.ravel() for a in p]).astype(np.float32)
    assert flat.size == n_params
    return flat


def collect_samples(torch, op, pulses, n_steps, psi0, dt, t0=0.0, every=20, rows_per_instance=256, seed=0,
                    guess=GUESS_PREV, chunk_log=None):
    """Propagate every instance to its own n_steps and sample training rows. Returns float64 [M][16]."""
    B = len(pulses)
    E = op.n_unknowns
    s = Solver(op, B)
    s.set_dt(dt)
    s.set_pulses(pulses)
    opts = solve_opts(tol=1e-12, max_iter=300, guess=guess)
    dev = "cuda:0"
    psi = torch.from_numpy(np.ascontiguousarray(psi0.reshape(-1))).to(dev)
    hist = [psi.clone() for _ in range(4)]  # psi_n, psi_{n-1}, psi_{n-2}, psi_{n-3}
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    ns = np.asarray(n_steps, dtype=np.int32)
    # the field at the midpoint of every step, evaluated by the library's device pulses (the values the
    # solver and the guess kernel use): fv[b][n] = f(t_n + dt/2)
    fv = s.eval_pulses(t0, 0, int(ns.max()))[:, :, 0]
    rows = []
    comp = torch.arange(E, device=dev)
    s_of = ((comp // op.nr) % 2).to(torch.float64)
    for n in range(int(ns.max())):
        s.run_batched(psi, t0, n, 1, ns, opts)
        if n >= 3 and n % every == 0:
            active = [b for b in range(B) if n < ns[b]]
            for b in active:
                idx = torch.randint(0, E, (rows_per_instance,), generator=gen, device=dev)
                gi = idx + b * E
                raw = torch.zeros(rows_per_instance, 16, dtype=torch.float64, device=dev)
                for k, h in enumerate(hist):
                    v = h[gi]
                    raw[:, 2 * k] = v.real
                    raw[:, 2 * k + 1] = v.imag
                nxt = psi[gi]
                raw[:, 8] = nxt.real
                raw[:, 9] = nxt.imag
                raw[:, 10] = float(fv[b, n])
                raw[:, 11] = float(fv[b, n - 1])
                raw[:, 12] = s_of[idx]
                rows.append(raw)
        # rotate the history: the oldest buffer receives psi_{n+1}
        last = hist.pop()
        last.copy_(psi)
        hist.insert(0, last)
        if chunk_log and n % 200 == 0:
            chunk_log(f"collect: step {n}")
    s.close()
    return torch.cat(rows, 0)


def train(torch, net: Net, raw, n_iter=1500, batch_rows=8192, lr=1e-3, seed=0, log=None):
    """Least-squares skip on all rows, then minibatch Adam on the GPU; returns the loss history
    (in units of the skip's residual)."""
    net.fit_skip(raw)
    gen = torch.Generator(device=raw.device)
    gen.manual_seed(seed)
    M = raw.shape[0]
    losses = []
    for it in range(n_iter):
        idx = torch.randint(0, M, (min(batch_rows, M),), generator=gen, device=raw.device)
        mb = raw[idx].contiguous()
        losses.append(net.backward(mb))
        lr_it = lr * (0.1 if it > 0.8 * n_iter else 1.0)
        net.adam(lr_it)
        if log and it % 250 == 0:
            log(f"train: iter {it} loss {losses[-1]:.3e}")
    return np.array(losses)


def propagate(torch, op, pulses, n_steps, psi0, dt, mode, net: Net | None = None, t0=0.0, chunk=32, wg_per_cu=0):
    """Run every instance to its own length with guess mode "zero", "prev", "skip" (the network's
    fitted linear part alone) or "mlp" (the whole network). wg_per_cu: launch shape of the
    persistent grid (0 = library default).

    Returns (final states [B*E] tensor, per-step stats array [steps][B], elapsed seconds)."""
    B = len(pulses)
    E = op.n_unknowns
    s = Solver(op, B)
    s.set_dt(dt)
    s.set_pulses(pulses)
    s.set_launch(wg_per_cu)
    dev = "cuda:0"
    ns = np.asarray(n_steps, dtype=np.int32)
    total = int(ns.max())
    psi = torch.from_numpy(np.ascontiguousarray(psi0.reshape(-1))).to(dev)
    stats = torch.zeros(total * B * STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    sz = B * STATS_DTYPE.itemsize
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    if mode in ("zero", "prev"):
        opts = solve_opts(tol=1e-12, max_iter=300, guess=GUESS_ZERO if mode == "zero" else GUESS_PREV)
        n = 0
        while n < total:
            k = min(chunk, total - n)
            s.run_batched(psi, t0, n, k, ns, opts, stats[n * sz:(n + k) * sz])
            n += k
    elif mode in ("mlp", "skip"):
        assert net is not None
        net.set_pulses(pulses)
        c_saved, sig_saved = net.get_skip()
        if mode == "skip":
            net.set_skip(c_saved, 0.0)
        opts = solve_opts(tol=1e-12, max_iter=300, guess=GUESS_GIVEN)
        hist = [psi.clone() for _ in range(4)]
        guess = torch.empty_like(psi)
        for n in range(total):
            net.guess(hist, E, op.nr, t0 + n * dt, dt, guess)
            s.run_batched(psi, t0, n, 1, ns, opts, stats[n * sz:(n + 1) * sz], guess=guess)
            last = hist.pop()
            last.copy_(psi)
            hist.insert(0, last)
        if mode == "skip":
            net.set_skip(c_saved, sig_saved)
    else:
        raise ValueError(mode)
    torch.cuda.synchronize()
    el = time.perf_counter() - t_start
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=STATS_DTYPE).reshape(total, B)
    s.close()
    return psi, st, el


def active_mask(n_steps, total):
    ns = np.asarray(n_steps)
    return np.arange(total)[:, None] < ns[None, :]
