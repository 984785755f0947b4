"""GPU parity of the HIP library against the FP64 oracle (marked gpu).

Every case feeds the same seeded inputs to libtdde.so (through the C ABI) and to the oracle and
compares element by element. Tolerances:
  * apply FP64: 1e-13 relative (max-norm) -- different summation order only;
  * apply FP32: 2e-6 relative (FP32 accumulation over at most ~60 taps of mixed sign);
  * time step FP64: 1e-10 relative state error per step (the solves stop at 1e-12 relative residual;
    cond(A) <= ~20 for the S = I operators, and the preconditioned hydrogen runs are compared with a
    direct solve of the same step);
  * mixed precision: 1e-10 per step (FP64 refinement to the same 1e-12 residual).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.assemble import Assembled  # noqa: E402
from oracle.fields import field_values, midpoint_time  # noqa: E402
from oracle.step import BlockPreconditioner, cn_step, step_matrices  # noqa: E402
from workloads import dkb, synthetic  # noqa: E402
from workloads.desc import Pulse, replace  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _lib():
    import paper_2512_21697_amd as P
    return P


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(DEV)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


def _rand_state(op, batch, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((batch, op.nang, 2, op.nr)) + 1j * rng.standard_normal((batch, op.nang, 2, op.nr))
    return x


CASES = {
    "tiny_pq_s": lambda: synthetic.tiny(s_identity=False),
    "tiny_ident": lambda: synthetic.tiny(nr=150, nang=4, s_identity=True),
    "c1": lambda: synthetic.config1(),
    "h_small": lambda: dkb.config2(nr=300, r_max=60.0, lmax=3, driven=True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_apply_fp64_matches_oracle(gpu, name):
    P = _lib()
    w = CASES[name]()
    op = w.op
    batch = 2
    s = P.Solver(op, batch)
    rng = np.random.default_rng(5)
    f = rng.standard_normal((batch, op.n_fields))
    s.set_field(f)
    x = _rand_state(op, batch, 11)
    a_s, a_h = complex(0.8, -0.3), complex(0.1, 0.45)
    y = torch.zeros(batch * op.n_unknowns, dtype=torch.complex128, device=DEV)
    s.apply(_dev(x).reshape(-1), y, a_s, a_h)
    torch.cuda.synchronize()
    yg = y.cpu().numpy().reshape(batch, -1)
    asm = Assembled(op)
    for b in range(batch):
        ref = asm.operator(list(f[b]), a_s, a_h) @ x[b].ravel()
        assert _rel(yg[b], ref) < 1e-13, name


@pytest.mark.parametrize("name", ["tiny_pq_s", "h_small"])
def test_apply_fp32_matches_oracle(gpu, name):
    P = _lib()
    w = CASES[name]()
    op = w.op
    s = P.Solver(op, 1)
    f = np.array([[0.3, -0.7][: op.n_fields]])
    s.set_field(f)
    x = _rand_state(op, 1, 3)
    xd = torch.from_numpy(x.astype(np.complex64).reshape(-1)).to(DEV)
    y = torch.zeros_like(xd)
    s.apply(xd, y, 1.0, 0.5j * 0.01, c64=True)
    torch.cuda.synchronize()
    ref = Assembled(op).operator(list(f[0]), 1.0, 0.5j * 0.01) @ x.astype(np.complex64).astype(np.complex128).ravel()
    assert _rel(y.cpu().numpy().astype(np.complex128), ref) < 2e-6


@pytest.mark.parametrize("name", ["tiny_pq_s", "tiny_ident", "c1", "h_small"])
def test_preconditioner_matches_direct_solve(gpu, name):
    """z = M^-1 v with M = S + i dt/2 H0 (eq. matrixM) against a sparse LU solve of M."""
    P = _lib()
    w = CASES[name]()
    op = w.op
    s = P.Solver(op, 2)
    s.set_dt(w.dt)
    v = _rand_state(op, 2, 9)
    z = torch.zeros(2 * op.n_unknowns, dtype=torch.complex128, device=DEV)
    s.precond_apply(_dev(v).reshape(-1), z)
    torch.cuda.synchronize()
    zg = z.cpu().numpy().reshape(2, -1)
    M = BlockPreconditioner(Assembled(op), w.dt)
    for b in range(2):
        ref = M(v[b].ravel())
        assert _rel(zg[b], ref) < 1e-11, name


def _opts(P, **kw):
    return P.solve_opts(**kw)


@pytest.mark.parametrize("precond", [0, 1])
def test_solve_matches_dense_lu(gpu, precond):
    P = _lib()
    w = synthetic.tiny(s_identity=False)
    op = w.op
    s = P.Solver(op, 1)
    s.set_dt(w.dt)
    f = np.array([[0.4, -0.2]])
    s.set_field(f)
    asm = Assembled(op)
    A = asm.operator(list(f[0]), 1.0, 0.5j * w.dt)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(op.n_unknowns) + 1j * rng.standard_normal(op.n_unknowns)
    x = torch.zeros(op.n_unknowns, dtype=torch.complex128, device=DEV)
    st, stats = s.solve(_dev(b), x, _opts(P, tol=1e-13, guess=P.GUESS_ZERO, precond=precond))
    xd = np.linalg.solve(A.toarray(), b)
    assert st == 0, stats
    assert _rel(x.cpu().numpy(), xd) < 1e-10
    assert stats[0]["true_rel_res"] <= 1e-13


def _run_steps(P, w, n, precond=0, guess=None, precision=0, batch_pulses=None):
    op = w.op
    s = P.Solver(op, 1)
    s.set_dt(w.dt)
    s.set_pulses(w.pulses)
    g = P.GUESS_PREV if guess is None else guess
    psi = _dev(w.psi0).reshape(-1).clone()
    states, stats = [], []
    for k in range(n):
        st, sts = s.step(psi, w.t0 + k * w.dt, _opts(P, tol=1e-12, guess=g, precond=precond, precision=precision,
                                                      max_iter=300))
        assert st == 0, (k, sts)
        stats.append(sts[0])
        states.append(psi.cpu().numpy().reshape(op.nang, 2, op.nr).copy())
    return states, stats


@pytest.mark.parametrize("guess", [0, 1])
def test_c1_steps_match_oracle(gpu, guess):
    """Config 1 (N = 3200), 20 steps: each GPU step fed the same psi_n as the oracle's dense solve."""
    P = _lib()
    w = synthetic.config1(driven=True)
    states, stats = _run_steps(P, w, 20, guess=guess)
    asm = Assembled(w.op)
    psi = w.psi0[0]
    worst = 0.0
    for k in range(20):
        ref, _ = cn_step(asm, w.pulses[0], w.t0 + k * w.dt, w.dt, psi, solver="dense")
        gpu_next = states[k]
        err = np.linalg.norm(gpu_next - ref) / np.linalg.norm(ref)
        worst = max(worst, err)
        psi = gpu_next  # the next step starts from the GPU state: per-step error, not accumulated
    assert worst < 1e-10, worst
    assert all(s["true_rel_res"] <= 1e-12 for s in stats)


def test_hydrogen_steps_match_direct_solve(gpu):
    """Hydrogen (nr = 300, l <= 3), driven, preconditioned BiCGSTAB vs sparse LU per step."""
    P = _lib()
    w = dkb.config2(nr=300, r_max=60.0, lmax=3, driven=True, E0=0.5)
    states, stats = _run_steps(P, w, 5, precond=1)
    asm = Assembled(w.op)
    psi = w.psi0[0]
    for k in range(5):
        ref, _ = cn_step(asm, w.pulses[0], w.t0 + k * w.dt, w.dt, psi, solver="splu")
        err = np.linalg.norm(states[k] - ref) / np.linalg.norm(ref)
        assert err < 1e-10, (k, err, stats[k])
        psi = states[k]
    assert max(s["iters"] for s in stats) <= 10


def test_mixed_precision_step(gpu):
    P = _lib()
    w = dkb.config2(nr=300, r_max=60.0, lmax=3, driven=True, E0=0.5)
    states, stats = _run_steps(P, w, 3, precond=1, precision=P.PREC_MIXED)
    asm = Assembled(w.op)
    psi = w.psi0[0]
    for k in range(3):
        ref, _ = cn_step(asm, w.pulses[0], w.t0 + k * w.dt, w.dt, psi, solver="splu")
        err = np.linalg.norm(states[k] - ref) / np.linalg.norm(ref)
        assert err < 1e-10, (k, err, stats[k])
        assert stats[k]["outer_iters"] >= 1
        psi = states[k]


def test_batched_matches_per_instance_oracle(gpu):
    """Three instances with different pulses and lengths advanced in one persistent launch."""
    P = _lib()
    w = synthetic.config5(batch=3, nr=200, nang=6, seeds=[10001, 10002, 10003])
    n_steps = np.array([5, 3, 4], dtype=np.int32)
    s = P.Solver(w.op, 3)
    s.set_dt(w.dt)
    s.set_pulses(w.pulses)
    psi = _dev(w.psi0).reshape(-1).clone()
    stats = torch.zeros(5 * 3 * 40, dtype=torch.uint8, device=DEV)
    s.run_batched(psi, w.t0, 0, 5, n_steps, P.solve_opts(tol=1e-12, guess=P.GUESS_ZERO), stats)
    torch.cuda.synchronize()
    got = psi.cpu().numpy().reshape(3, w.op.nang, 2, w.op.nr)
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE).reshape(5, 3)
    asm = Assembled(w.op)
    for b in range(3):
        ref = w.psi0[b]
        for k in range(int(n_steps[b])):
            ref, _ = cn_step(asm, w.pulses[b], w.t0 + k * w.dt, w.dt, ref, solver="splu")
            assert st[k, b]["status"] == 0
        err = np.linalg.norm(got[b] - ref) / np.linalg.norm(ref)
        assert err < 1e-10 * n_steps[b], (b, err)


def test_not_converged_status_and_context_reuse(gpu):
    P = _lib()
    w = synthetic.config1(driven=True)
    s = P.Solver(w.op, 1)
    s.set_dt(w.dt)
    s.set_pulses(w.pulses)
    psi = _dev(w.psi0).reshape(-1).clone()
    st, stats = s.step(psi, w.t0, P.solve_opts(tol=1e-12, max_iter=1, guess=P.GUESS_ZERO))
    assert st == 1 and stats[0]["status"] == 1 and stats[0]["iters"] == 1
    psi = _dev(w.psi0).reshape(-1).clone()
    st, stats = s.step(psi, w.t0, P.solve_opts(tol=1e-12, guess=P.GUESS_ZERO))
    assert st == 0 and stats[0]["true_rel_res"] <= 1e-12


def test_bad_buffer_rejected_before_launch(gpu):
    P = _lib()
    w = synthetic.tiny()
    s = P.Solver(w.op, 1)
    s.set_field(np.zeros((1, 2)))
    x = torch.zeros(10, dtype=torch.complex128, device=DEV)
    with pytest.raises(ValueError):
        s.apply(x, x.clone())


@pytest.mark.parametrize("case", ["h_prev", "c1_prev", "c1_zero", "c1_tight"])
def test_multistep_launch_matches_oracle(gpu, case):
    """Several steps in one persistent launch: every step after the first takes its right-hand side
    from the previous step's residual check (one shared operator pass). The final state is compared
    with the oracle's chain of steps (errors accumulate over the steps). "c1_tight" asks for a
    relative residual of 1e-16, below what FP64 reaches, so checks fail and restart: the launch must
    still end, with every step converged or NOT_CONVERGED and the state close to the oracle's."""
    P = _lib()
    if case == "h_prev":
        w = dkb.config2(nr=300, r_max=60.0, lmax=3, driven=True, E0=0.5)
        precond, guess, n, tol, max_iter = 1, P.GUESS_PREV, 6, 1e-12, 100
    else:
        w = synthetic.config1(driven=True)
        precond, guess, n = 0, (P.GUESS_ZERO if case == "c1_zero" else P.GUESS_PREV), 8
        tol, max_iter = (1e-16, 25) if case == "c1_tight" else (1e-12, 300)
    s = P.Solver(w.op, 1)
    s.set_dt(w.dt)
    s.set_pulses(w.pulses)
    psi = _dev(w.psi0).reshape(-1).clone()
    stats = torch.zeros(n * 40, dtype=torch.uint8, device=DEV)
    s.run_batched(psi, w.t0, 0, n, np.array([n], dtype=np.int32),
                  P.solve_opts(tol=tol, max_iter=max_iter, guess=guess, precond=precond), stats)
    torch.cuda.synchronize()
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
    got = psi.cpu().numpy().reshape(w.op.nang, 2, w.op.nr)
    assert np.all(np.isfinite(got))
    asm = Assembled(w.op)
    ref = w.psi0[0]
    for k in range(n):
        ref, _ = cn_step(asm, w.pulses[0], w.t0 + k * w.dt, w.dt, ref, solver="splu" if precond else "dense")
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    if case == "c1_tight":
        assert set(st["status"].tolist()) <= {0, 1}, st["status"]
        assert err < 1e-10 * n, err
    else:
        assert np.all(st["status"] == 0), st
        assert np.all(st["true_rel_res"] <= tol), st["true_rel_res"]
        assert err < 1e-10 * n, err


@pytest.mark.parametrize("wg_per_cu", [1, 2, 3, 4])
def test_launch_shapes_match_oracle(gpu, wg_per_cu):
    """Every persistent launch shape gives the oracle's states: the preconditioned hydrogen case
    (one instance spread over the whole grid) and three uneven instances in one launch."""
    P = _lib()
    w = dkb.config2(nr=300, r_max=60.0, lmax=3, driven=True, E0=0.5)
    n = 4
    s = P.Solver(w.op, 1)
    s.set_dt(w.dt)
    s.set_pulses(w.pulses)
    n_wg_default, _ = s.launch_info()
    s.set_launch(wg_per_cu)
    n_wg, per_inst = s.launch_info()
    assert 1 <= per_inst <= n_wg <= n_wg_default
    psi = _dev(w.psi0).reshape(-1).clone()
    stats = torch.zeros(n * 40, dtype=torch.uint8, device=DEV)
    s.run_batched(psi, w.t0, 0, n, np.array([n], dtype=np.int32),
                  P.solve_opts(tol=1e-12, max_iter=100, guess=P.GUESS_PREV, precond=1), stats)
    torch.cuda.synchronize()
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
    assert np.all(st["status"] == 0), st
    got = psi.cpu().numpy().reshape(w.op.nang, 2, w.op.nr)
    asm = Assembled(w.op)
    ref = w.psi0[0]
    for k in range(n):
        ref, _ = cn_step(asm, w.pulses[0], w.t0 + k * w.dt, w.dt, ref, solver="splu")
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-10 * n, err
    s.close()

    wb = synthetic.config5(batch=3, nr=200, nang=6, seeds=[10001, 10002, 10003])
    n_steps = np.array([5, 3, 4], dtype=np.int32)
    sb = P.Solver(wb.op, 3)
    sb.set_dt(wb.dt)
    sb.set_pulses(wb.pulses)
    sb.set_launch(wg_per_cu)
    psi = _dev(wb.psi0).reshape(-1).clone()
    stats = torch.zeros(5 * 3 * 40, dtype=torch.uint8, device=DEV)
    sb.run_batched(psi, wb.t0, 0, 5, n_steps, P.solve_opts(tol=1e-12, guess=P.GUESS_ZERO), stats)
    torch.cuda.synchronize()
    got = psi.cpu().numpy().reshape(3, wb.op.nang, 2, wb.op.nr)
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE).reshape(5, 3)
    asm = Assembled(wb.op)
    for b in range(3):
        ref = wb.psi0[b]
        for k in range(int(n_steps[b])):
            ref, _ = cn_step(asm, wb.pulses[b], wb.t0 + k * wb.dt, wb.dt, ref, solver="splu")
            assert st[k, b]["status"] == 0
        err = np.linalg.norm(got[b] - ref) / np.linalg.norm(ref)
        assert err < 1e-10 * n_steps[b], (b, err)
    sb.close()


def test_launch_shape_errors_and_autotune(gpu):
    """Out-of-range shapes are rejected and leave the grid unchanged; the autotuner leaves the
    solver on the shape it reports as fastest."""
    from paper_2512_21697_amd.autotune import tune_launch
    P = _lib()
    w = synthetic.config1(driven=True)
    s = P.Solver(w.op, 1)
    s.set_dt(w.dt)
    s.set_pulses(w.pulses)
    before = s.launch_info()
    for bad in (-1, 5):
        with pytest.raises(P.TddeError):
            s.set_launch(bad)
    assert s.launch_info() == before
    s.set_launch(1)
    s.set_launch(0)
    assert s.launch_info() == before
    psi0 = _dev(w.psi0).reshape(-1)
    scratch = torch.empty_like(psi0)
    stats = torch.zeros(8 * 40, dtype=torch.uint8, device=DEV)
    opts = P.solve_opts(tol=1e-12, guess=P.GUESS_PREV)

    def run():
        scratch.copy_(psi0)
        s.run_batched(scratch, w.t0, 0, 8, np.array([8], dtype=np.int32), opts, stats)

    best, times, grids = tune_launch(s, run, reps=2)
    assert set(times) == {1, 2, 3, 4} and times[best] == min(times.values())
    assert s.launch_info()[0] == grids[best]
    torch.cuda.synchronize()
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
    assert np.all(st["status"] == 0)
    s.close()


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("seg", [16, 48])
def test_prec_segment_lengths_match_oracle(gpu, seg, split):
    """Other least segment lengths of the preconditioner (refactored at set_dt) give the same steps, in
    the persistent and the kernel-per-window solver. 600 rows: 16-row segments put 4 channels in a chain
    work-group, 48-row segments 8, and the blocks with fewer channels leave channel slots empty."""
    P = _lib()
    w = dkb.config2(nr=300, r_max=60.0, lmax=3, driven=True)
    s = P.Solver(w.op, 1)
    try:
        with pytest.raises(P.TddeError):
            s.set_prec_segment(5)
        s.set_split(split)
        s.set_prec_segment(seg)
        s.set_dt(w.dt)
        s.set_pulses(w.pulses)
        psi = _dev(w.psi0).reshape(-1)
        st = torch.zeros(3 * 40, dtype=torch.uint8, device=DEV)
        s.run_batched(psi, w.t0, 0, 3, np.array([3], dtype=np.int32),
                      P.solve_opts(tol=1e-12, guess=P.GUESS_PREV, precond=1), st)
        torch.cuda.synchronize()
        got = psi.cpu().numpy().reshape(w.psi0[0].shape)
    finally:
        s.close()
    asm = Assembled(w.op)
    ref = w.psi0[0]
    for k in range(3):
        ref, _ = cn_step(asm, w.pulses[0], w.t0 + k * w.dt, w.dt, ref, solver="splu")
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-10
