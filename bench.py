"""Benchmark of the Crank-Nicolson / BiCGSTAB time step on one MI355X.

Default workload: the hydrogen dipole case (DKB B-splines, Nr = 2000 radial pairs on [0, 200],
41 kappa channels at mu = 1/2, N = 164000 complex128 unknowns, dt = 2e-4, ground state start,
sin^2 pulse with 8 cycles at omega = 0.057, E0 = 0.05), preconditioned FP64 BiCGSTAB to a relative
residual of 1e-12. One "step" is one full time step of the hot path: field evaluation at the
midpoint, right-hand side, initial guess, BiCGSTAB with the block LU preconditioner, true-residual
check. Steps run in persistent launches of up to 64 steps; the timed region starts with the
inputs resident in HBM.

Prints one JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DEFAULT_WG_PER_CU = 4  # the library's default launch shape (work-groups per CU of the persistent grid)
FP64_PEAK_TFLOPS = 78.6


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def operator_bytes(op):
    """Operator data a matrix-free apply reads at least once: the kappa-polynomial H0 / S bands, the
    coupling bands and angular values, the per-channel complex bands."""
    n = op.h_poly.size * 8 + op.s_poly.size * 8 + sum(t.r_band.size * 8 + t.a_val.size * 12 for t in op.terms)
    if op.h_chan is not None:
        n += op.h_chan.size * 16
    return n


def apply_bytes(op):
    """One apply: x read, y written, operator data read."""
    return 2 * op.n_unknowns * 16 + operator_bytes(op)


def prec_bytes(op):
    """One block preconditioner solve: every channel's banded L and U factors (2 w + 1 complex
    values per row) read once, input read and output written."""
    w = 2 * op.hb + 1
    return op.nang * 2 * op.nr * (2 * w + 1) * 16 + 2 * op.n_unknowns * 16


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


def measured_traffic(wg_per_cu):
    """HBM bytes per launch of the persistent kernel from the committed rocprofv3 counter summary,
    or None when it is missing, was taken from other kernel sources or under another launch
    shape (work-groups per CU)."""
    path = os.path.join(ROOT, "profiles", "persistent_kernel_hydrogen_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash() or d.get("wg_per_cu") != wg_per_cu:
        return None
    return d


def run_gpu_steps(P, torch, w, steps, warmup, precond, guess, chunk=64, precision=0, launch=0, info=None):
    """Run warmup + timed steps in persistent chunks.

    launch: work-groups per CU of the persistent grid (1..4, 0 = library default), or "auto" to
    let the autotuner time one chunk of steps (on a scratch copy of the state, before the warmup)
    under every shape and keep the fastest; ``info`` (a dict) receives the choice and the timings.
    Returns (ms_per_step, stats array, [(kernel ms, steps) per launch], wall seconds, final state)."""
    from paper_2512_21697_amd.autotune import tune_launch
    s = P.Solver(w.op, 1)
    s.set_dt(w.dt)
    s.set_pulses(w.pulses)
    opts = P.solve_opts(tol=1e-12, max_iter=200, guess=guess, precond=precond, precision=precision, inner_tol=1e-5,
                        max_outer=20)
    psi = torch.from_numpy(w.psi0.reshape(-1)).to("cuda:0")
    stream = torch.cuda.current_stream()
    if launch == "auto":
        scratch = torch.empty_like(psi)
        tune_stats = torch.zeros(chunk * 40, dtype=torch.uint8, device="cuda:0")
        tune_n = np.array([chunk], dtype=np.int32)

        def one_chunk():
            scratch.copy_(psi)
            s.run_batched(scratch, w.t0, 0, chunk, tune_n, opts, tune_stats)

        best, times = tune_launch(s, one_chunk, prefer=DEFAULT_WG_PER_CU)
        del scratch, tune_stats
        if info is not None:
            info["wg_per_cu"] = best
            info["ms_per_chunk"] = {str(k): round(v * 1e3, 3) for k, v in times.items()}
            info["chunk_steps"] = chunk
    else:
        s.set_launch(int(launch))
        if info is not None:
            info["wg_per_cu"] = int(launch) or DEFAULT_WG_PER_CU
    if info is not None:
        info["n_wg"], info["wg_per_instance"] = s.launch_info()
    total = warmup + steps
    n_steps = np.array([total], dtype=np.int32)
    stats = torch.zeros(total * 40, dtype=torch.uint8, device="cuda:0")
    # warmup
    k = 0
    while k < warmup:
        n = min(chunk, warmup - k)
        s.run_batched(psi, w.t0, k, n, n_steps, opts, stats[k * 40:(k + n) * 40])
        k += n
    torch.cuda.synchronize()
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
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
    s.close()
    return ms / steps, st[warmup:], launches, wall, psi


def s_norm(P, torch, op, psi):
    """psi^H S psi with the library's apply (S x: a_s = 1, a_h = 0)."""
    s = P.Solver(op, 1)
    s.set_field(np.zeros((1, op.n_fields)))
    y = torch.empty_like(psi)
    s.apply(psi, y, 1.0, 0.0)
    torch.cuda.synchronize()
    s.close()
    return float(torch.vdot(psi, y).real.item())


def mixed_section(P, torch, w, steps, warmup, psi64):
    """FP32-inner / FP64-refinement solve on the hydrogen operator vs the FP64 path (same steps)."""
    ms, st, launches, wall, psi = run_gpu_steps(P, torch, w, steps, warmup, precond=1, guess=P.GUESS_PREV,
                                                precision=P.PREC_MIXED)
    diff = float(torch.linalg.vector_norm(psi - psi64).item() / torch.linalg.vector_norm(psi64).item())
    n0 = s_norm(P, torch, w.op, torch.from_numpy(w.psi0.reshape(-1)).to("cuda:0"))
    n1 = s_norm(P, torch, w.op, psi)
    return {"ms_per_step": ms, "steps_per_s": 1000.0 / ms, "outer_iters_per_step": float(st["outer_iters"].mean()),
            "inner_iters_per_step": float(st["iters"].mean()), "all_converged": bool(np.all(st["status"] == 0)),
            "max_true_rel_res": float(st["true_rel_res"].max()),
            "state_rel_diff_vs_fp64_after_steps": diff, "s_norm_drift": abs(n1 - n0)}


def tune_batched(P, torch, w5, steps=8):
    """Autotune the persistent launch shape of the batched sweep: one launch of ``steps`` zero-guess
    steps of every instance, on a scratch copy of the states, per shape."""
    from paper_2512_21697_amd.autotune import tune_launch
    s = P.Solver(w5.op, w5.batch)
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

    best, times = tune_launch(s, one_launch, prefer=DEFAULT_WG_PER_CU)
    n_wg, per_inst = s.launch_info()
    s.close()
    del psi, scratch, stats
    return {"wg_per_cu": best, "ms_per_launch": {str(k): round(v * 1e3, 3) for k, v in times.items()},
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
    t_collect = time.perf_counter() - t0
    net = P.Net(16384, 1e-6)
    net.set_params(learned.init_params(0, net.n_params))
    t0 = time.perf_counter()
    losses = learned.train(torch, net, raw, n_iter=800, batch_rows=16384, lr=1e-3)
    t_train = time.perf_counter() - t0
    ns = np.minimum(w5.n_steps, eval_steps)
    launch = tune_batched(P, torch, w5)
    if log:
        log(f"bench: batched launch shape {launch}")
    out = {"instances": int(w5.batch), "train_rows": int(raw.shape[0]), "collect_s": t_collect, "train_s": t_train,
           "loss_first": float(losses[:10].mean()), "loss_last": float(losses[-50:].mean()),
           "skip_sigma": float(net.get_skip()[1]), "launch": launch}
    ref = None
    for mode in ("zero", "prev", "skip", "mlp"):
        fin, st, el = learned.propagate(torch, op, w5.pulses, ns, w5.psi0, w5.dt, mode, net=net,
                                        wg_per_cu=launch["wg_per_cu"])
        act = learned.active_mask(ns, st.shape[0])
        if ref is None:
            ref = fin
        d = float(torch.linalg.vector_norm(fin - ref).item() / torch.linalg.vector_norm(ref).item())
        out[mode] = {"iters_per_step": float(st["iters"][act].mean()), "instance_steps_per_s": float(act.sum() / el),
                     "batched_steps_per_s": float(st.shape[0] / el), "all_converged": bool(np.all(st["status"][act] == 0)),
                     "rel_diff_vs_zero_guess": d}
        if log:
            log(f"bench: batched {mode}: {out[mode]}")
    net.close()
    return out


def spmv_measure(P, torch, w, reps=20):
    """Standalone operator apply y = S x + i dt/2 H x: average kernel time (HIP events)."""
    s = P.Solver(w.op, w.batch)
    s.set_field(np.ones((w.batch, w.op.n_fields)) * 0.01)
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
    s.close()
    return ms


def cpu_baseline(w, precond, budget_s=20.0):
    """The oracle (CSR assembly once, preconditioned textbook BiCGSTAB per step) on the host cores.
    Returns (steps/s, steps, seconds, threads used = process CPU time / wall time)."""
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the beyond-dipole apply measurement")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched learned-guess comparison")
    ap.add_argument("--batched-steps", type=int, default=200, help="steps per instance in the batched sections")
    ap.add_argument("--wg-per-cu", default="auto",
                    help="persistent work-groups per CU (1..4), or 'auto' to autotune before the warmup")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the run, copy MIB MiB once (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import paper_2512_21697_amd as P
    from workloads import dkb, synthetic

    _log("bench: building hydrogen workload (Nr=2000, 41 channels)")
    w = dkb.config2()
    E = w.op.n_unknowns
    _log(f"bench: gpu steps={args.steps} warmup={args.warmup}")
    launch = args.wg_per_cu if args.wg_per_cu == "auto" else int(args.wg_per_cu)
    tuning = {}
    ms_step, st, launches, wall, psi64 = run_gpu_steps(P, torch, w, args.steps, args.warmup, precond=1,
                                                       guess=P.GUESS_PREV, launch=launch, info=tuning)
    _log(f"bench: launch shape {tuning}")
    iters = st["iters"].astype(float)
    mv = st["matvecs"].astype(float)
    ok = bool(np.all(st["status"] == 0))
    # roofline of the persistent solver kernel (the only kernel of the timed region)
    kern_ms = sum(t for t, _ in launches) / max(1, len(launches))
    steps_per_launch = sum(n for _, n in launches) / max(1, len(launches))
    it_mean = float(iters.mean())
    bytes_step = algorithmic_bytes_per_step(w.op, float(mv.mean()), float(st["precs"].mean()), it_mean)
    achieved = bytes_step * steps_per_launch / (kern_ms * 1e-3) / 1e9
    tr = measured_traffic(tuning.get("wg_per_cu"))
    traffic = None
    if tr is not None:
        traffic = (tr["fetch_kib_per_step"] * tr["fetch_scale"] + tr["write_kib_per_step"] * tr["write_scale"]) * 1024.0 \
            * steps_per_launch
    res = {
        "metric": "TDDE steps/s (hydrogen dipole, preconditioned FP64 BiCGSTAB to 1e-12)",
        "value": 1000.0 / ms_step,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic (seeded generator; DKB hydrogen operator computed on the host)",
        "config": {"workload": "hydrogen dipole: Nr=2000, Nang=41 (l<=20, mu=1/2), N=164000, dt=2e-4, "
                               "E0=0.05, w=0.057, 8-cycle sin^2, ground-state start, tol 1e-12, "
                               "block-LU preconditioner, previous-state guess",
                   "batch": 1, "seq_len": None, "parallelism": "single GPU", "launch": tuning},
        "iters_per_step": it_mean,
        "matvecs_per_step": float(mv.mean()),
        "precond_solves_per_step": float(st["precs"].mean()),
        "all_converged": ok,
        "max_true_rel_res": float(st["true_rel_res"].max()),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "persistent_kernel", "kernel_ms_per_launch": kern_ms,
                     "steps_per_launch": steps_per_launch, "alg_bytes_per_launch": bytes_step * steps_per_launch,
                     "alg_bytes_per_step": bytes_step, "source_hash": source_hash()},
    }
    if not args.no_mixed:
        _log("bench: mixed precision on the hydrogen operator")
        res["mixed_precision"] = mixed_section(P, torch, w, args.steps, args.warmup, psi64)
    if not args.no_batched:
        _log("bench: batched sweep, learned vs plain guesses")
        res["batched_learned"] = batched_learned_section(P, torch, args.batched_steps, args.batched_steps, log=_log)
    if not args.no_extra:
        _log("bench: beyond-dipole apply (Nr=4000, Nang=770, N=6.16e6)")
        w3 = synthetic.config3()
        ms3 = spmv_measure(P, torch, w3)
        E3 = w3.op.n_unknowns
        b3 = apply_bytes(w3.op)
        res["spmv_beyond_dipole"] = {"ms": ms3, "alg_GBps": b3 / (ms3 * 1e-3) / 1e9,
                                     "frac_hbm": b3 / (ms3 * 1e-3) / 1e9 / HBM_PEAK_GBS, "alg_bytes": b3,
                                     "N": E3}
        del w3
    if not args.no_cpu:
        _log("bench: cpu oracle baseline")
        rate, n, el, threads = cpu_baseline(w, True, args.cpu_budget)
        res["cpu_baseline"] = {"value": rate, "unit": "steps/s", "cores": threads, "kind": "oracle",
                               "sample": f"{n} steps of the same workload from the ground state "
                                         f"({el:.1f} s; CSR assembly and LU factorisation excluded; "
                                         f"cores = process CPU time / wall time)"}
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 16
        a = torch.ones(n, dtype=torch.complex128, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        res["copy_probe_bytes"] = 2 * n * 16
    print(json.dumps(res))


if __name__ == "__main__":
    main()
