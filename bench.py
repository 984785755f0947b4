"""Benchmark of the Crank-Nicolson / BiCGSTAB time step on one MI355X.

Headline workload: the beyond-dipole single-GPU share (Nr = 4000 order-7 radial functions per
component, 770 angular channels with l <= 40 and |mu| <= 9/2, six coupling terms with |dl| <= 2,
mu' = mu +- 1; N = 6.16e6 complex128 unknowns), sin^2 pulses at omega and omega +- 2 pi / T
(E0 = 0.05, T = 20, dt = 1e-3), started mid-pulse at t = T/4 so the coupling is switched on,
FP64 BiCGSTAB to a relative residual of 1e-12, right-preconditioned by the block LU of
M = S + i dt/2 H0 (the paper's setting), previous-state guess. One "step" is one full time step of
the hot path: field evaluation at the midpoint, right-hand side, initial guess, BiCGSTAB with the
preconditioner, true-residual check. Steps run in persistent launches of up to 64 steps; the
timed region starts with every input resident in HBM.

Sub-lines (same JSON line): the same workload without the preconditioner, its standalone operator
apply, the hydrogen dipole case (ground state at t = 0, and mid-pulse with E0 = 0.5), the small
block-banded case (from t = 0 and from t = T/4), mixed precision on the hydrogen operator, the
64-instance batched sweep with zero / previous / fitted-skip / learned guesses, and the oracle on
the host cores.

Prints one JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
DEFAULT_WG_PER_CU = 4  # the library's default launch shape (work-groups per CU of the persistent grid)
DEFAULT_SEGMENT = 24   # the library's default least rows per preconditioner segment
SECTIONS = ("c3plain", "apply", "c2", "c2d", "c1", "mixed", "batched", "spectrum", "beyond", "cpu")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


# ------------------------------------------------------------------------------ algorithmic counts

def operator_bytes(op):
    """Operator data a matrix-free apply reads at least once: the kappa-polynomial H0 / S bands, the
    coupling bands and angular values (8-byte value + 4-byte column), the per-channel complex bands."""
    n = op.h_poly.size * 8 + op.s_poly.size * 8 + sum(t.r_band.size * 8 + t.a_val.size * 12 for t in op.terms)
    if op.h_chan is not None:
        n += op.h_chan.size * 16
    return n


def apply_bytes(op):
    """One apply: x read, y written, operator data read."""
    return 2 * op.n_unknowns * 16 + operator_bytes(op)


def apply_flops(op):
    """Real floating-point operations of one apply y = a_S S x + a_H H x (FMA = 2), per element:
    every H0 / S tap block (real taps: 4 flop, complex: 8), for every coupling term the angular
    combination over its row (real value x complex: 4 flop per entry) and its radial taps
    (4 flop per tap and nonzero (s, s') block), the complex term prefactor (8) and the final
    combination (16)."""
    nb = 2 * op.hb + 1
    E = op.n_unknowns
    blk_h = sum(int(np.any(op.h_poly[:, s, s2] != 0)) for s in range(2) for s2 in range(2)) / 2.0
    blk_s = sum(int(np.any(op.s_poly[:, s, s2] != 0)) for s in range(2) for s2 in range(2)) / 2.0
    per = nb * 4 * (blk_h + blk_s)
    if op.h_chan is not None:
        per += nb * 8 * sum(int(np.any(op.h_chan[:, s, s2] != 0)) for s in range(2) for s2 in range(2)) / 2.0
    for t in op.terms:
        nnz_row = len(t.a_col) / op.nang
        blk = sum(int(np.any(t.r_band[s, s2] != 0)) for s in range(2) for s2 in range(2)) / 2.0
        per += nnz_row * 4 * max(blk, 1.0) + nb * 4 * blk + 8
    return (per + 16) * E


def factor_blocks(op):
    """Distinct diagonal blocks of M = S + i dt/2 H0: one per channel with its own complex band,
    else one per distinct kappa."""
    return op.nang if op.h_chan is not None else len(np.unique(op.kappa))


def prec_bytes(op):
    """One block-preconditioner solve: the banded L and U factors (2 w + 1 complex values per row,
    w = 2 hb + 1) of every distinct block read once, input read, output written."""
    w = 2 * op.hb + 1
    return factor_blocks(op) * 2 * op.nr * (2 * w + 1) * 16 + 2 * op.n_unknowns * 16


def algorithmic_bytes_per_step(op, matvecs, precs, iters):
    """Minimal HBM bytes of one time step as the solver runs it: every operator apply counted in
    `matvecs` (Krylov products, the true-residual check, which also forms the next step's right-hand
    side), every preconditioner solve counted in `precs`, and 4 + 12 * iters plain vector passes
    (right-hand side, guess and residual set-up; the BiCGSTAB vector updates and dot products of
    every iteration)."""
    E = op.n_unknowns
    return matvecs * apply_bytes(op) + precs * prec_bytes(op) + (4 + 12 * iters) * E * 16


def source_hash():
    """Hash of the kernel sources: measured counters are only reported for the kernels they were
    taken from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2512_21697_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name, launch_key, kernel="persistent_kernel"):
    """HBM counters of a kernel from the committed rocprofv3 counter summary
    ``profiles/<kernel>_<name>_counters.json``, or None when it is missing, was taken from other
    kernel sources or under another launch shape."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{name}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash() or d.get("launch") != launch_key:
        return None
    return d


# ------------------------------------------------------------------------------ GPU runs

def run_gpu_steps(P, torch, w, steps, warmup, precond, guess, chunk=64, precision=0, launch=0, info=None,
                  segment=None, form=None, prec_bits=64):
    """Run warmup + timed steps of one instance in chunks of steps (one library call each).

    launch: work-groups per CU of the persistent grid (1..4, 0 = library default), or "auto" to
    let the autotuner time one chunk of steps (on a scratch copy of the state, before the warmup)
    under every shape and keep the fastest. segment: least rows per preconditioner segment (None =
    library default), or "auto" to tune it the same way (preconditioned runs only). form: solver form,
    "persistent" (None: the library default), "split" (one kernel per window of the iteration; FP64
    previous-state-guess steps only) or "auto" to time both on the tuning chunk. prec_bits: storage
    of the preconditioner factors read by the kernel-per-window form (64, or 32). ``info`` (a dict)
    receives the choices, the timings, the grid actually launched and, in the split form, the
    durations of the timed region's apply kernel v = A p^ (HIP events on the library's stream).
    Returns (ms_per_step, stats array, [(kernel ms, steps) per launch], wall seconds, final state)."""
    from paper_2512_21697_amd.autotune import tune_form, tune_launch, tune_segment
    s = P.Solver(w.op, 1)
    try:
        if segment not in (None, "auto"):
            s.set_prec_segment(int(segment))
        s.set_dt(w.dt)
        s.set_pulses(w.pulses)
        s.set_prec_storage(prec_bits)
        opts = P.solve_opts(tol=1e-12, max_iter=300, guess=guess, precond=precond, precision=precision,
                            inner_tol=1e-5, max_outer=20)
        psi = torch.from_numpy(w.psi0.reshape(-1)).to("cuda:0")
        stream = torch.cuda.current_stream()
        tune_chunk = min(chunk, 20)
        scratch = torch.empty_like(psi)
        tune_stats = torch.zeros(tune_chunk * 40, dtype=torch.uint8, device="cuda:0")
        tune_n = np.array([tune_chunk], dtype=np.int32)

        def one_chunk():
            scratch.copy_(psi)
            s.run_batched(scratch, w.t0, 0, tune_chunk, tune_n, opts, tune_stats)

        if launch == "auto":
            best, times, grids = tune_launch(s, one_chunk, prefer=DEFAULT_WG_PER_CU)
            if info is not None:
                info["wg_per_cu"] = best
                info["ms_per_chunk"] = {str(k): round(v * 1e3, 3) for k, v in times.items()}
                info["grid_per_shape"] = {str(k): g for k, g in grids.items()}
                info["chunk_steps"] = tune_chunk
        else:
            s.set_launch(int(launch))
            if info is not None:
                info["wg_per_cu"] = int(launch) or DEFAULT_WG_PER_CU
        split_ok = guess == P.GUESS_PREV and precision == 0
        if form == "auto" and split_ok:
            best_f, ftimes = tune_form(s, one_chunk)
            if info is not None:
                info["form"] = best_f
                info["ms_per_chunk_by_form"] = {k: round(v * 1e3, 3) for k, v in ftimes.items()}
        else:
            s.set_split(form == "split" and split_ok)
            if info is not None:
                info["form"] = "split" if (form == "split" and split_ok) else "persistent"
        is_split = info is not None and info.get("form") == "split"
        if segment == "auto" and precond:
            best_m, mtimes = tune_segment(s, w.dt, one_chunk, prefer=DEFAULT_SEGMENT)
            if info is not None:
                info["segment_rows"] = best_m
                info["ms_per_chunk_by_segment"] = {str(k): round(v * 1e3, 3) for k, v in mtimes.items()}
        elif info is not None and precond:
            info["segment_rows"] = int(segment) if segment not in (None, "auto") else DEFAULT_SEGMENT
        one_chunk()
        torch.cuda.synchronize()
        del scratch, tune_stats
        if info is not None:
            info["n_wg"], info["wg_per_instance"] = s.launch_info()  # the grid of the launches that follow
        total = warmup + steps
        n_steps = np.array([total], dtype=np.int32)
        stats = torch.zeros(total * 40, dtype=torch.uint8, device="cuda:0")
        k = 0
        while k < warmup:
            n = min(chunk, warmup - k)
            s.run_batched(psi, w.t0, k, n, n_steps, opts, stats[k * 40:(k + n) * 40])
            k += n
        torch.cuda.synchronize()
        if is_split:
            s.split_timing(8 * steps + 16)
        evs = []
        t0 = time.perf_counter()
        start = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        while k < total:
            n = min(chunk, total - k)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            s.run_batched(psi, w.t0, k, n, n_steps, opts, stats[k * 40:(k + n) * 40])
            e1.record(stream)
            evs.append((e0, e1, n))
            k += n
        end = torch.cuda.Event(enable_timing=True)
        end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = start.elapsed_time(end)
        launches = [(a.elapsed_time(b), n) for a, b, n in evs]
        if is_split:
            d = s.read_split_timing()
            s.split_timing(0)
            # launches in blocks past the last step find no work and end at once
            act = [x for x in d if x > 0.1 * max(d)] if d else []
            info["apply_v_launches"] = len(d)
            info["apply_v_active_launches"] = len(act)
            info["apply_v_ms"] = float(np.mean(act)) if act else None
        st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
    finally:
        s.close()
    return ms / steps, st[warmup:], launches, wall, psi


def step_summary(w, ms, st, launches):
    iters = st["iters"].astype(float)
    mv = st["matvecs"].astype(float)
    pc = st["precs"].astype(float)
    kern_ms = sum(t for t, _ in launches) / max(1, len(launches))
    per_launch = sum(n for _, n in launches) / max(1, len(launches))
    bytes_step = algorithmic_bytes_per_step(w.op, float(mv.mean()), float(pc.mean()), float(iters.mean()))
    return {"steps_per_s": 1000.0 / ms, "ms_per_step": ms, "iters_per_step": float(iters.mean()),
            "matvecs_per_step": float(mv.mean()), "precond_solves_per_step": float(pc.mean()),
            "all_converged": bool(np.all(st["status"] == 0)), "max_true_rel_res": float(st["true_rel_res"].max()),
            "kernel_ms_per_launch": kern_ms, "steps_per_launch": per_launch, "alg_bytes_per_step": bytes_step,
            "alg_GBps": bytes_step * per_launch / (kern_ms * 1e-3) / 1e9}


def step_section(P, torch, w, steps, warmup, precond, guess=None, launch=0, label="", form="auto"):
    guess = P.GUESS_PREV if guess is None else guess
    info = {}
    ms, st, launches, wall, psi = run_gpu_steps(P, torch, w, steps, warmup, precond, guess, launch=launch, info=info,
                                                form=form)
    out = step_summary(w, ms, st, launches)
    out.update({"workload": label, "steps": steps, "precond": bool(precond),
                "guess": {0: "zero", 1: "previous", 2: "given"}[guess], "launch": info})
    del psi
    return out


def s_norm(P, torch, op, psi):
    """psi^H S psi with the library's apply (S x: a_s = 1, a_h = 0)."""
    s = P.Solver(op, 1)
    try:
        s.set_field(np.zeros((1, op.n_fields)))
        y = torch.empty_like(psi)
        s.apply(psi, y, 1.0, 0.0)
        torch.cuda.synchronize()
        v = float(torch.vdot(psi, y).real.item())
    finally:
        s.close()
    return v


def mixed_section(P, torch, w, steps, warmup):
    """FP32-inner / FP64-refinement solve on the hydrogen operator vs the FP64 path (same steps)."""
    ms64, st64, _, _, psi64 = run_gpu_steps(P, torch, w, steps, warmup, precond=1, guess=P.GUESS_PREV)
    ms, st, launches, wall, psi = run_gpu_steps(P, torch, w, steps, warmup, precond=1, guess=P.GUESS_PREV,
                                                precision=P.PREC_MIXED)
    diff = float(torch.linalg.vector_norm(psi - psi64).item() / torch.linalg.vector_norm(psi64).item())
    n0 = s_norm(P, torch, w.op, torch.from_numpy(w.psi0.reshape(-1)).to("cuda:0"))
    n1 = s_norm(P, torch, w.op, psi)
    return {"steps": steps, "ms_per_step": ms, "steps_per_s": 1000.0 / ms, "fp64_steps_per_s": 1000.0 / ms64,
            "speedup_vs_fp64": ms64 / ms, "outer_iters_per_step": float(st["outer_iters"].mean()),
            "inner_iters_per_step": float(st["iters"].mean()), "all_converged": bool(np.all(st["status"] == 0)),
            "max_true_rel_res": float(st["true_rel_res"].max()),
            "state_rel_diff_vs_fp64_after_steps": diff, "s_norm_drift": abs(n1 - n0)}


def tune_batched(P, torch, w5, steps=8):
    """Autotune the persistent launch shape of the batched sweep: one launch of ``steps`` zero-guess
    steps of every instance, on a scratch copy of the states, per shape."""
    from paper_2512_21697_amd.autotune import tune_launch
    s = P.Solver(w5.op, w5.batch)
    try:
        s.set_dt(w5.dt)
        s.set_pulses(w5.pulses)
        psi = torch.from_numpy(np.ascontiguousarray(w5.psi0.reshape(-1))).to("cuda:0")
        scratch = torch.empty_like(psi)
        stats = torch.zeros(steps * w5.batch * P.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
        ns = np.full(w5.batch, steps, dtype=np.int32)
        opts = P.solve_opts(tol=1e-12, max_iter=300, guess=P.GUESS_ZERO)

        def one_launch():
            scratch.copy_(psi)
            s.run_batched(scratch, w5.t0, 0, steps, ns, opts, stats)

        best, times, grids = tune_launch(s, one_launch, prefer=DEFAULT_WG_PER_CU)
        n_wg, per_inst = s.launch_info()
        del psi, scratch, stats
    finally:
        s.close()
    return {"wg_per_cu": best, "ms_per_launch": {str(k): round(v * 1e3, 3) for k, v in times.items()},
            "grid_per_shape": {str(k): g for k, g in grids.items()},
            "launch_steps": steps, "n_wg": n_wg, "wg_per_instance": per_inst}


def batched_learned_section(P, torch, train_steps, eval_steps, n_train=200, train_batch=50, log=None):
    """Batched sweep (64 instances of the block-banded recipe at Nr = 2000, Nang = 41) with zero,
    previous-state, fitted-skip and full-network guesses; the network is trained on solver
    trajectories of n_train other pulses."""
    from paper_2512_21697_amd import learned
    from workloads import synthetic
    w5 = synthetic.config5()
    op = w5.op
    psi0 = w5.psi0[0]
    rows = []
    t0 = time.perf_counter()
    for k in range(0, n_train, train_batch):
        seeds = list(range(1 + k, 1 + min(n_train, k + train_batch)))
        tp, tn = synthetic.batched_pulses(seeds)
        tn = np.minimum(tn, train_steps)
        rows.append(learned.collect_samples(torch, op, tp, tn, np.repeat(psi0[None], len(seeds), 0), w5.dt, every=10,
                                            rows_per_instance=128, seed=k))
        if log:
            log(f"bench: collected trajectories {k + len(seeds)}/{n_train}")
    raw = torch.cat(rows, 0)
    del rows
    t_collect = time.perf_counter() - t0
    net = P.Net(16384, 1e-6)
    try:
        net.set_params(learned.init_params(0, net.n_params))
        t0 = time.perf_counter()
        losses = learned.train(torch, net, raw, n_iter=800, batch_rows=16384, lr=1e-3)
        t_train = time.perf_counter() - t0
        ns = w5.n_steps.copy() if eval_steps <= 0 else np.minimum(w5.n_steps, eval_steps)
        launch = tune_batched(P, torch, w5)
        if log:
            log(f"bench: batched launch shape {launch}")
        out = {"instances": int(w5.batch), "steps_per_instance": [int(ns.min()), int(ns.max())],
               "train_rows": int(raw.shape[0]), "collect_s": t_collect, "train_s": t_train,
               "loss_first": float(losses[:10].mean()), "loss_last": float(losses[-50:].mean()),
               "skip_sigma": float(net.get_skip()[1]), "launch": launch}
        del raw
        ref = None
        for mode in ("zero", "prev", "skip", "mlp"):
            fin, st, el = learned.propagate(torch, op, w5.pulses, ns, w5.psi0, w5.dt, mode, net=net,
                                            wg_per_cu=launch["wg_per_cu"])
            act = learned.active_mask(ns, st.shape[0])
            if ref is None:
                ref = fin
            d = float(torch.linalg.vector_norm(fin - ref).item() / torch.linalg.vector_norm(ref).item())
            out[mode] = {"iters_per_step": float(st["iters"][act].mean()),
                         "instance_steps_per_s": float(act.sum() / el),
                         "batched_steps_per_s": float(st.shape[0] / el),
                         "all_converged": bool(np.all(st["status"][act] == 0)), "rel_diff_vs_zero_guess": d}
            if log:
                log(f"bench: batched {mode}: {out[mode]}")
            del fin
        del ref
    finally:
        net.close()
    return out


def apply_section(P, torch, w, reps=20):
    """Standalone operator apply y = S x + i dt/2 H x at the step's fields: average kernel time
    (HIP events on the library's stream), algorithmic GB/s and GFLOP/s."""
    from oracle.fields import field_values, midpoint_time
    s = P.Solver(w.op, w.batch)
    try:
        s.set_field(np.array([field_values(w.pulses[0], midpoint_time(w.t0, w.dt))]))
        x = torch.from_numpy(w.psi0.reshape(-1)).to("cuda:0")
        y = torch.empty_like(x)
        stream = torch.cuda.current_stream()
        for _ in range(3):
            s.apply(x, y, 1.0, 0.5j * w.dt)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            s.apply(x, y, 1.0, 0.5j * w.dt)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        del x, y
    finally:
        s.close()
    b = apply_bytes(w.op)
    fl = apply_flops(w.op)
    return {"kernel": "apply_kernel<double>", "ms": ms, "alg_bytes": b, "alg_GBps": b / (ms * 1e-3) / 1e9,
            "frac_hbm": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "alg_flop": fl,
            "GFLOPs": fl / (ms * 1e-3) / 1e9, "frac_fp64": fl / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}


def spectrum_section(P, torch, reps=20):
    """Photoelectron spectrum of ionised hydrogen (eq. dPdE): propagate the ground state through a
    4-cycle pulse (w = 1, E0 = 1) at dt = 8e-3 and 4e-3 on the GPU, then time tdde_spectrum (projection onto
    the 848 field-free levels of 21 kappa blocks inside (0.02, 3) a.u., density, grid of 300 energies)
    and report the spectral error between the two time resolutions (the paper's convergence metric)."""
    from workloads import spectrum as wspec
    out = {}
    spectra = []
    inp = None
    for dt in (8e-3, 4e-3):
        w, inp = wspec.hydrogen_case(dt=dt)
        n = int(w.n_steps[0])
        s = P.Solver(w.op, 1)
        try:
            s.set_dt(dt)
            s.set_pulses(w.pulses)
            psi = torch.from_numpy(w.psi0.reshape(-1)).to("cuda:0")
            opts = P.solve_opts(tol=1e-12, max_iter=300, guess=P.GUESS_PREV, precond=1)
            stats = torch.zeros(n * P.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda:0")
            ns = np.array([n], dtype=np.int32)
            t0 = time.perf_counter()
            k = 0
            while k < n:
                m = min(64, n - k)
                s.run_batched(psi, w.t0, k, m, ns, opts, stats[k * 40:(k + m) * 40])
                k += m
            torch.cuda.synchronize()
            t_prop = time.perf_counter() - t0
            st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
            s.spectrum_setup(inp.blk_of, inp.n_lev, inp.levels, inp.edges, inp.vecs, inp.grid)
            dp = torch.zeros(inp.grid.size, dtype=torch.float64, device="cuda:0")
            stream = torch.cuda.current_stream()
            s.spectrum(psi, dp)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                s.spectrum(psi, dp)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            spectra.append(dp.clone())
            pr = dp.cpu().numpy()
            out[f"dt_{dt:g}"] = {"steps": n, "propagation_s": t_prop, "steps_per_s": n / t_prop,
                                  "all_converged": bool(np.all(st["status"] == 0)),
                                  "iters_per_step": float(st["iters"].mean()),
                                  "ionisation_in_window": float(np.sum(0.5 * (pr[1:] + pr[:-1]) * np.diff(inp.grid))),
                                  "spectrum_ms": ms}
            if dt == 4e-3:
                err = s.spectrum_error(spectra[1], spectra[0])
                out["spectral_error_dt_vs_dt2"] = float(err[0])
            del psi, stats
        finally:
            s.close()
    nr, lev = 600, int(inp.levels.size)
    b = lev * 2 * nr * 8 + 21 * 2 * nr * 16 + inp.grid.size * 8
    out["spectrum"] = {"kernels": "spec_project_kernel + spec_grid_kernel", "levels": lev, "grid": int(inp.grid.size),
                       "ms": out["dt_0.004"]["spectrum_ms"], "alg_bytes": b,
                       "alg_GBps": b / (out["dt_0.004"]["spectrum_ms"] * 1e-3) / 1e9}
    return out


# ------------------------------------------------------------------------------ CPU oracle baseline

def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"os_cpu_count": os.cpu_count(), "cpu_model": model}


def cpu_baseline_extrapolated(w, matvecs, precs, iters, n_channels=4):
    """The oracle's step cost on the host, extrapolated from timed pieces (the assembled operator of
    this workload does not fit in host memory): the CSR matvec of a row slice of n_channels channels
    (scaled by nang / n_channels), one channel block's sparse-LU preconditioner solve (scaled by the
    channel count) and one vector update over all unknowns (scaled by the step's vector passes),
    combined with the GPU run's matvecs, preconditioner solves and iterations per step."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    from oracle.assemble import channel_rows, kappa_poly_block
    from oracle.fields import field_values, midpoint_time
    op = w.op
    f = field_values(w.pulses[0], midpoint_time(w.t0, w.dt))
    j0 = op.nang // 2
    t_build = time.perf_counter()
    rows = channel_rows(op, f, 1.0, 0.5j * w.dt, j0, j0 + n_channels)
    t_build = time.perf_counter() - t_build
    x = w.psi0.reshape(-1)
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        rows @ x
    t_mv = (time.perf_counter() - t0) / reps * op.nang / n_channels
    kap = float(op.kappa[j0])
    blk = kappa_poly_block(op.h_poly, kap, op.nr, op.hb).astype(np.complex128)
    sblk = kappa_poly_block(op.s_poly, kap, op.nr, op.hb) if op.s_poly.shape[0] else sp.identity(2 * op.nr)
    M = (sblk + 0.5j * w.dt * blk).tocsc()
    lu = spla.splu(M)
    v = x[:2 * op.nr].copy()
    t0 = time.perf_counter()
    for _ in range(reps):
        lu.solve(v)
    t_pc = (time.perf_counter() - t0) / reps * op.nang
    y = np.empty_like(x)
    t0 = time.perf_counter()
    for _ in range(reps):
        np.add(x, 0.3 * x, out=y)
    t_vec = (time.perf_counter() - t0) / reps
    t_step = matvecs * t_mv + precs * t_pc + (4 + 12 * iters) * t_vec
    info = host_info()
    return {"value": 1.0 / t_step, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": (f"extrapolated: CSR matvec of the rows of {n_channels} of {op.nang} channels "
                       f"({rows.nnz} nonzeros, {t_mv / op.nang * n_channels * 1e3:.1f} ms, x {op.nang / n_channels:.1f}), "
                       f"one channel block's sparse-LU solve (x {op.nang}), one vector update (x "
                       f"{4 + 12 * iters:.0f}); combined with the GPU run's {matvecs:.2f} matvecs, "
                       f"{precs:.2f} preconditioner solves, {iters:.2f} iterations per step; "
                       f"scipy CSR matvec and SuperLU solve are single-threaded"),
            "s_per_matvec": t_mv, "s_per_precond": t_pc, "s_per_vector_pass": t_vec, "s_per_step": t_step,
            "slice_assembly_s": t_build, **info}


def cpu_baseline_steps(w, precond, budget_s=20.0):
    """The oracle (CSR assembly once, preconditioned textbook BiCGSTAB per step) on the host cores,
    whole steps of the same workload. Returns (steps/s, steps, seconds, threads used)."""
    from oracle.assemble import Assembled
    from oracle.step import BlockPreconditioner, cn_step
    asm = Assembled(w.op)
    M = BlockPreconditioner(asm, w.dt) if precond else None
    psi = w.psi0[0]
    t0 = time.perf_counter()
    c0 = time.process_time()
    n = 0
    while True:
        psi, st = cn_step(asm, w.pulses[0], w.t0 + n * w.dt, w.dt, psi, guess="prev", precond=M)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 50:
            break
    el = time.perf_counter() - t0
    cpu = time.process_time() - c0
    return n / el, n, el, max(1, round(cpu / el))


# ------------------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma list of sub-lines to run beside the headline: " + ",".join(SECTIONS) + " (or none)")
    ap.add_argument("--sub-steps", type=int, default=200, help="steps of the hydrogen / small-case sub-lines")
    ap.add_argument("--batched-steps", type=int, default=0,
                    help="cap on the steps per instance in the batched section (0: every instance's own length, "
                         "400-1200 steps)")
    ap.add_argument("--train-steps", type=int, default=200, help="steps per training trajectory of the learned guess")
    ap.add_argument("--wg-per-cu", default="auto", help="persistent work-groups per CU (1..4, 0 = default), or auto")
    ap.add_argument("--segment", default="auto", help="least rows per preconditioner segment, or auto")
    ap.add_argument("--form", default="auto", choices=("auto", "persistent", "split"),
                    help="solver form of the headline: one persistent launch per chunk, one kernel per window of "
                         "the iteration, or auto (time both)")
    ap.add_argument("--no-headline", action="store_true",
                    help="skip the headline run (profiling runs of a sub-line's kernel only; no value)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB once (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; runs on several GPUs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    sections = set() if args.sections in ("", "none") else set(args.sections.split(","))

    import torch

    import paper_2512_21697_amd as P
    from workloads import dkb, synthetic

    _log("bench: building the beyond-dipole workload (Nr=4000, 770 channels, six terms, N=6.16e6)")
    w3 = synthetic.config3(driven=True)
    launch = args.wg_per_cu if args.wg_per_cu == "auto" else int(args.wg_per_cu)
    tuning = {}
    _log(f"bench: gpu steps={args.steps} warmup={args.warmup}")
    if args.no_headline:
        head = {"steps_per_s": None, "ms_per_step": None, "iters_per_step": None, "matvecs_per_step": None,
                "precond_solves_per_step": None, "all_converged": None, "max_true_rel_res": None,
                "kernel_ms_per_launch": None, "steps_per_launch": 0, "alg_bytes_per_step": 0.0, "alg_GBps": 0.0}
        ms_step = None
    else:
        seg = args.segment if args.segment == "auto" else int(args.segment)
        ms_step, st, launches, wall, psi = run_gpu_steps(P, torch, w3, args.steps, args.warmup, precond=1,
                                                         guess=P.GUESS_PREV, launch=launch, info=tuning, segment=seg,
                                                         form=args.form)
        del psi
        head = step_summary(w3, ms_step, st, launches)
    _log(f"bench: headline {head}")
    split_form = tuning.get("form") == "split"
    traffic = None
    passes = None
    E3 = w3.op.n_unknowns
    if split_form:
        # dominant kernel: the operator apply v = A p^ fused with <r^, v> (one of three applies a step)
        rk = "sp_apply_v_kernel"
        rk_bytes = apply_bytes(w3.op) + E3 * 16
        rk_ms = tuning.get("apply_v_ms")
        achieved = rk_bytes / (rk_ms * 1e-3) / 1e9 if rk_ms else None
        tr = measured_traffic("beyond_dipole", f"grid{tuning.get('n_wg')}", kernel=rk)
        if tr is not None and not args.no_headline:
            traffic = (tr["fetch_kib_per_launch"] * tr["fetch_scale"] + tr["write_kib_per_launch"] * tr["write_scale"]) * 1024.0
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic, "kernel": rk,
                "kernel_ms_per_launch": rk_ms, "launches_timed": tuning.get("apply_v_active_launches"),
                "alg_bytes_per_launch": rk_bytes,
                "step_alg_bytes": head["alg_bytes_per_step"],
                "step_alg_GBps": head["alg_bytes_per_step"] / (ms_step * 1e-3) / 1e9 if ms_step else None,
                "source_hash": source_hash()}
    else:
        key = f"grid{tuning.get('n_wg')}_seg{tuning.get('segment_rows')}"
        tr = measured_traffic("beyond_dipole", key)
        if tr is not None and not args.no_headline:
            per_step = (tr["fetch_kib_per_step"] * tr["fetch_scale"] + tr["write_kib_per_step"] * tr["write_scale"]) * 1024.0
            traffic = per_step * head["steps_per_launch"]
            passes = per_step / max(1.0, head["iters_per_step"]) / (E3 * 16)
        roof = {"bound": "hbm", "achieved": head["alg_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": head["alg_GBps"] / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "persistent_kernel", "kernel_ms_per_launch": head["kernel_ms_per_launch"],
                "steps_per_launch": head["steps_per_launch"],
                "alg_bytes_per_launch": head["alg_bytes_per_step"] * head["steps_per_launch"],
                "alg_bytes_per_step": head["alg_bytes_per_step"],
                "hbm_passes_per_iteration": passes, "source_hash": source_hash()}
    res = {
        "metric": "TDDE steps/s (beyond-dipole operator, preconditioned FP64 BiCGSTAB to 1e-12)",
        "value": head["steps_per_s"],
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic (seeded generator of the beyond-dipole recipe; no dataset)",
        "config": {"workload": "beyond-dipole single-GPU share: Nr=4000 (order 7), Nang=770 (l<=40, |mu|<=9/2), "
                               "six coupling terms |dl|<=2 mu'=mu+-1, N=6.16e6 complex128, dt=1e-3, "
                               "E0=0.05 sin^2 pulses at w=0.057 and w+-2pi/T (T=20) from t=T/4, tol 1e-12, "
                               "block-LU preconditioner, previous-state guess; solver form and launch autotuned",
                   "batch": 1, "seq_len": None, "parallelism": "single GPU", "launch": tuning},
        "iters_per_step": head["iters_per_step"],
        "matvecs_per_step": head["matvecs_per_step"],
        "precond_solves_per_step": head["precond_solves_per_step"],
        "all_converged": head["all_converged"],
        "max_true_rel_res": head["max_true_rel_res"],
        "roofline": roof,
    }
    sub = {}
    if not args.no_headline and split_form:
        _log("bench: beyond-dipole, FP32 preconditioner factors (same form, launch and segment)")
        info32 = {}
        f32_form = tuning.get("form")
        ms32, st32, _, _, psi32 = run_gpu_steps(P, torch, w3, args.steps, args.warmup, precond=1, guess=P.GUESS_PREV,
                                                launch=int(tuning.get("wg_per_cu", 0)), info=info32,
                                                segment=tuning.get("segment_rows"), form=f32_form, prec_bits=32)
        del psi32
        sub["beyond_dipole_fp32_factors"] = {
            "steps_per_s": 1000.0 / ms32, "ms_per_step": ms32, "iters_per_step": float(st32["iters"].mean()),
            "all_converged": bool(np.all(st32["status"] == 0)), "max_true_rel_res": float(st32["true_rel_res"].max()),
            "note": "preconditioner factors stored in FP32 (tdde_set_prec_storage(32)); iteration, residuals and "
                    "states FP64 to the same 1e-12 tolerance", "launch": info32}
    if "c3plain" in sections:
        _log("bench: beyond-dipole without preconditioner")
        sub["beyond_dipole_plain"] = step_section(P, torch, w3, args.steps, args.warmup, 0, label="c3 driven, no M")
    if "apply" in sections:
        _log("bench: beyond-dipole standalone apply")
        sub["beyond_dipole_apply"] = apply_section(P, torch, w3)
    if "c2" in sections or "c2d" in sections or "mixed" in sections:
        _log("bench: building the hydrogen workload (Nr=2000, 41 channels)")
        w2 = dkb.config2()
        if "c2" in sections:
            sub["hydrogen"] = step_section(P, torch, w2, args.sub_steps, 5, 1, label="hydrogen from the ground state, t=0")
        if "c2d" in sections:
            w2d = dkb.config2(E0=0.5, driven=True)
            sub["hydrogen_driven"] = step_section(P, torch, w2d, args.sub_steps, 5, 1,
                                                  label="hydrogen mid-pulse t=T/2+pi/(2w), E0=0.5")
            del w2d
        if "mixed" in sections:
            _log("bench: mixed precision on the hydrogen operator")
            sub["mixed_precision"] = mixed_section(P, torch, w2, args.sub_steps, 5)
        del w2
    if "c1" in sections:
        for drv in (False, True):
            w1 = synthetic.config1(driven=drv)
            for g, gn in ((P.GUESS_PREV, "prev"), (P.GUESS_ZERO, "zero")):
                sub[f"small_{'driven_' if drv else ''}{gn}"] = step_section(
                    P, torch, w1, 20, 5, 0, guess=g, label=f"N=3200 {'t0=T/4' if drv else 't0=0'}")
    if "batched" in sections:
        _log("bench: batched sweep, learned vs plain guesses")
        sub["batched_learned"] = batched_learned_section(P, torch, args.train_steps, args.batched_steps, log=_log)
    if "beyond" in sections:
        _log("bench: physical beyond-dipole hydrogen operator")
        from workloads import beyond
        wb = beyond.workload(nr=600, kappa_max=6, mu2_max=5, l_max=3)
        sb = step_section(P, torch, wb, args.sub_steps, 5, 1,
                          label="hydrogen in the beyond-dipole pulse (eq. bdpA): nr=600, |kappa|<=6, |mu|<=5/2 "
                                "(60 channels), l<=3 (96 terms), E0=1, w=1, from T/4")
        sb["apply"] = apply_section(P, torch, wb)
        sub["beyond_dipole_physical"] = sb
        del wb
    if "spectrum" in sections:
        _log("bench: photoelectron spectrum of ionised hydrogen")
        sub["spectrum"] = spectrum_section(P, torch)
    res["sub"] = sub
    if "cpu" in sections and not args.no_headline:
        _log("bench: cpu oracle baseline (extrapolated from timed pieces)")
        res["cpu_baseline"] = cpu_baseline_extrapolated(w3, head["matvecs_per_step"], head["precond_solves_per_step"],
                                                        head["iters_per_step"])
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 16
        a = torch.ones(n, dtype=torch.complex128, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = 2 * n * 16
        del a, b
    # Release every device buffer before the interpreter exits: library contexts are closed where
    # they are used; drop the remaining tensors and the caching allocator's blocks while the HIP
    # runtime is still up (finalisers that free device memory after a profiler's own exit-time
    # teardown have crashed the process).
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
