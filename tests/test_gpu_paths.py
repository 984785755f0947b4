"""Parity of every path the benchmark times, at sizes that reach it (marked gpu).

References are the oracle's own solves (BiCGSTAB to 1e-14, with the block-LU preconditioner where
the operator has a non-identity overlap), forward error <= cond(A) * 1e-14; per-step tolerance
1e-10, accumulated over chained steps.

* beyond-dipole recipe (six terms sharing one angular pattern, |dl| <= 2, mu' = mu +- 1) at
  Nr = 300 (two full radial tiles and a ragged one) and l <= 12 (210 channels, 630 tiles, more than
  the persistent grid's work-groups): one step and a chained three-step launch, with and without
  the preconditioner, from a mid-pulse start.
* beyond-dipole at full size (N = 6.16e6): two single-step launches as the benchmark runs them;
  residual of the second step's equation on sampled rows from the element-wise definition,
  apply parity of the result on the same rows.
* hydrogen at full size: chained launches of 62, 63 and 64 steps; steps 63 and 64 compared with
  oracle steps fed the GPU's previous state (each chained step takes its right-hand side from the
  previous step's residual check).
* batched sweep at full size with instances retiring inside one launch.
* mixed precision at full hydrogen size.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.assemble import Assembled  # noqa: E402
from oracle.fields import field_values, midpoint_time  # noqa: E402
from oracle.rows import apply_rows  # noqa: E402
from oracle.step import BlockPreconditioner, cn_step  # noqa: E402
from workloads import dkb, synthetic  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


def _say(msg):
    print(msg, flush=True)


def _run(P, w, psi, step0, n, opts, n_total=None, batch=1):
    s = P.Solver(w.op, batch)
    try:
        s.set_dt(w.dt)
        s.set_pulses(w.pulses)
        stats = torch.zeros(n * batch * 40, dtype=torch.uint8, device=DEV)
        ns = np.full(batch, n_total if n_total is not None else step0 + n, dtype=np.int32)
        s.run_batched(psi, w.t0, step0, n, ns, opts, stats)
        torch.cuda.synchronize()
        st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
    finally:
        s.close()
    return st


@pytest.fixture(scope="module")
def c3_small():
    w = synthetic.config3(nr=300, lmax=12, driven=True)
    assert w.op.nang * 3 > 512
    _say(f"c3 recipe: nang {w.op.nang}, N {w.op.n_unknowns}; oracle assembly")
    asm = Assembled(w.op)
    M = BlockPreconditioner(asm, w.dt)
    refs = [w.psi0[0]]
    for k in range(3):
        r, st = cn_step(asm, w.pulses[0], w.t0 + k * w.dt, w.dt, refs[-1], guess="prev", tol=1e-14, precond=M)
        assert st.converged
        refs.append(r)
    return w, refs


@pytest.mark.parametrize("precond", [0, 1])
def test_beyond_dipole_recipe_steps_match_oracle(gpu, c3_small, precond):
    import paper_2512_21697_amd as P
    w, refs = c3_small
    op = w.op
    opts = P.solve_opts(tol=1e-12, max_iter=200, guess=P.GUESS_PREV, precond=precond)
    psi = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
    _say(f"c3 recipe precond={precond}: one step")
    st = _run(P, w, psi, 0, 1, opts)
    assert st["status"][0] == 0 and st["true_rel_res"][0] <= 1e-12
    got = psi.cpu().numpy().reshape(op.nang, 2, op.nr)
    err = np.linalg.norm(got - refs[1]) / np.linalg.norm(refs[1])
    _say(f"  step 1 rel err {err:.2e} iters {st['iters'][0]}")
    assert err < 1e-10
    _say(f"c3 recipe precond={precond}: chained three-step launch")
    psi = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
    st = _run(P, w, psi, 0, 3, opts)
    assert np.all(st["status"] == 0) and st["true_rel_res"].max() <= 1e-12
    got = psi.cpu().numpy().reshape(op.nang, 2, op.nr)
    err = np.linalg.norm(got - refs[3]) / np.linalg.norm(refs[3])
    _say(f"  after 3 chained steps rel err {err:.2e}")
    assert err < 3e-10


def test_beyond_dipole_full_size_step_residual_on_rows(gpu):
    import paper_2512_21697_amd as P
    w = synthetic.config3(driven=True)
    op = w.op
    E, nr = op.n_unknowns, op.nr
    opts = P.solve_opts(tol=1e-12, max_iter=200, guess=P.GUESS_PREV, precond=1)
    s = P.Solver(op, 1)
    try:
        s.set_dt(w.dt)
        s.set_pulses(w.pulses)
        psi = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        stats = torch.zeros(2 * 40, dtype=torch.uint8, device=DEV)
        ns = np.array([10], dtype=np.int32)
        _say("c3 full size: step 1")
        s.run_batched(psi, w.t0, 0, 1, ns, opts, stats[:40])
        torch.cuda.synchronize()
        psi1 = psi.cpu().numpy().reshape(op.nang, 2, nr).copy()
        _say("c3 full size: step 2")
        s.run_batched(psi, w.t0, 1, 1, ns, opts, stats[40:])
        torch.cuda.synchronize()
        psi2 = psi.cpu().numpy().reshape(op.nang, 2, nr).copy()
        st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
        _say(f"  stats {st[['status', 'iters', 'matvecs', 'precs']].tolist()} true res {st['true_rel_res'].tolist()}")
        assert np.all(st["status"] == 0) and st["true_rel_res"].max() <= 1e-12
        f = np.array(field_values(w.pulses[0], midpoint_time(w.t0 + w.dt, w.dt)))
        s.set_field(f[None])
        bvec = torch.empty_like(psi)
        s.apply(torch.from_numpy(psi1.reshape(-1)).to(DEV), bvec, 1.0, -0.5j * w.dt)
        yvec = torch.empty_like(psi)
        s.apply(psi, yvec, 1.0, 0.5j * w.dt)
        torch.cuda.synchronize()
        bnorm = float(torch.linalg.vector_norm(bvec).item())
        y_gpu = yvec.cpu().numpy()
    finally:
        s.close()
    rng = np.random.default_rng(21)
    special = [j * 2 * nr + sc * nr + i for j in (0, op.nang // 3, op.nang - 1) for sc in (0, 1)
               for i in (0, 127, 128, nr - 33, nr - 1)]
    rows = np.unique(np.concatenate([rng.integers(0, E, 300), special]))
    _say(f"  oracle rows: {len(rows)}")
    a = apply_rows(op, list(f), 1.0, 0.5j * w.dt, psi2, rows)
    b = apply_rows(op, list(f), 1.0, -0.5j * w.dt, psi1, rows)
    res = np.abs(b - a)
    _say(f"  max |b - A psi2| on rows / ||b|| = {res.max() / bnorm:.2e}; rms * sqrt(N) / ||b|| = "
         f"{np.sqrt(np.mean(res ** 2) * E) / bnorm:.2e}")
    assert res.max() <= 2e-12 * bnorm
    assert np.sqrt(np.mean(res ** 2) * E) <= 5e-12 * bnorm
    assert np.max(np.abs(y_gpu[rows] - a)) <= 1e-13 * np.max(np.abs(a))


def test_hydrogen_chained_launch_full_size(gpu):
    import paper_2512_21697_amd as P
    w = dkb.config2(driven=True, E0=0.5)
    op = w.op
    opts = P.solve_opts(tol=1e-12, max_iter=200, guess=P.GUESS_PREV, precond=1)
    states = {}
    for n in (62, 63, 64):
        psi = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        _say(f"hydrogen: chained launch of {n} steps")
        st = _run(P, w, psi, 0, n, opts)
        assert np.all(st["status"] == 0) and st["true_rel_res"].max() <= 1e-12
        states[n] = psi.cpu().numpy().reshape(op.nang, 2, op.nr)
    asm = Assembled(op)
    M = BlockPreconditioner(asm, w.dt)
    for n in (63, 64):
        ref, rst = cn_step(asm, w.pulses[0], w.t0 + (n - 1) * w.dt, w.dt, states[n - 1], guess="prev", tol=1e-14,
                           precond=M)
        assert rst.converged
        err = np.linalg.norm(states[n] - ref) / np.linalg.norm(ref)
        _say(f"  step {n} rel err {err:.2e}")
        assert err < 1e-10


def test_batched_full_size_instances_retire_inside_launch(gpu):
    import paper_2512_21697_amd as P
    w = synthetic.config5()
    B = w.batch
    step0, n = 396, 8
    ns = (400 + np.arange(B) % 6).astype(np.int32)  # instances retire after 4..9 steps of the launch
    s = P.Solver(w.op, B)
    try:
        s.set_dt(w.dt)
        s.set_pulses(w.pulses)
        psi = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        stats = torch.zeros(n * B * 40, dtype=torch.uint8, device=DEV)
        _say("batched: 8-step launch, instances retiring at steps 400..405")
        s.run_batched(psi, w.t0, step0, n, ns, P.solve_opts(tol=1e-12, max_iter=300, guess=P.GUESS_ZERO), stats)
        torch.cuda.synchronize()
        st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE).reshape(n, B)
        got = psi.cpu().numpy().reshape(B, w.op.nang, 2, w.op.nr)
    finally:
        s.close()
    for k in range(n):
        live = step0 + k < ns
        assert np.all(st["status"][k][live] == 0)
    asm = Assembled(w.op)
    for b in (0, 5, 17):
        ref = w.psi0[b]
        for step in range(step0, min(int(ns[b]), step0 + n)):
            ref, rst = cn_step(asm, w.pulses[b], w.t0 + step * w.dt, w.dt, ref, guess="zero", tol=1e-14)
            assert rst.converged
        err = np.linalg.norm(got[b] - ref) / np.linalg.norm(ref)
        _say(f"  instance {b} (retires at step {ns[b]}): rel err {err:.2e}")
        assert err < 1e-10 * (min(int(ns[b]), step0 + n) - step0)


def test_mixed_precision_full_size_hydrogen(gpu):
    import paper_2512_21697_amd as P
    w = dkb.config2(driven=True, E0=0.5)
    op = w.op
    opts = P.solve_opts(tol=1e-12, max_iter=200, guess=P.GUESS_PREV, precond=1, precision=P.PREC_MIXED,
                        inner_tol=1e-5, max_outer=20)
    psi = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
    states = [w.psi0[0]]
    for k in range(2):
        _say(f"mixed precision: step {k + 1}")
        st = _run(P, w, psi, k, 1, opts, n_total=10)
        assert st["status"][0] == 0 and st["true_rel_res"][0] <= 1e-12
        states.append(psi.cpu().numpy().reshape(op.nang, 2, op.nr).copy())
    asm = Assembled(op)
    M = BlockPreconditioner(asm, w.dt)
    for k in range(2):
        ref, rst = cn_step(asm, w.pulses[0], w.t0 + k * w.dt, w.dt, states[k], guess="prev", tol=1e-14, precond=M)
        err = np.linalg.norm(states[k + 1] - ref) / np.linalg.norm(ref)
        _say(f"  step {k + 1} rel err {err:.2e}")
        assert err < 1e-10
