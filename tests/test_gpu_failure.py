"""Failure and resume paths of the GPU solver, forced from the host (marked gpu).

* A NaN in the right-hand side stops the solve at its first reduction with TDDE_NONFINITE, and
  the context stays usable.
* A shadow residual orthogonal to r0 (exact zeros: b lives on channel 0, r^ on channel 1, so
  <r^, r0> = 0 exactly) makes rho vanish in the first window: the solver restarts with r^ = r and
  still reaches the dense solution; the oracle's BiCGSTAB, given the same shadow, restarts too.
* Checkpoint / resume: 2k steps in one persistent launch equal k + k steps in two launches (the
  state saved between them, as at the paper's checkpoints, Sec. 3.1) bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.assemble import Assembled  # noqa: E402
from oracle.bicgstab import bicgstab  # noqa: E402
from oracle.fields import field_values, midpoint_time  # noqa: E402
from oracle.step import step_matrices  # noqa: E402
from workloads import dkb, synthetic  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


def _fields(w):
    return np.array([field_values(w.pulses[0], midpoint_time(w.t0, w.dt))])


def test_nonfinite_rhs_stops_with_status(gpu):
    import paper_2512_21697_amd as P
    w = synthetic.config1(driven=True)
    s = P.Solver(w.op, 1)
    try:
        s.set_dt(w.dt)
        s.set_field(_fields(w))
        rng = np.random.default_rng(5)
        n = w.op.n_unknowns
        bh = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        bad = bh.copy()
        bad[1234] = complex(np.nan, 0.0)
        for precond in (0, 1):
            x = torch.zeros(n, dtype=torch.complex128, device=DEV)
            st, stats = s.solve(torch.from_numpy(bad).to(DEV), x,
                                P.solve_opts(tol=1e-12, max_iter=300, guess=P.GUESS_ZERO, precond=precond))
            print(f"precond={precond}: status {st}, {stats[0]}", flush=True)
            assert st == P.TDDE_NONFINITE and stats[0]["status"] == P.TDDE_NONFINITE
            assert stats[0]["iters"] == 0
            # the context stays usable
            x = torch.zeros(n, dtype=torch.complex128, device=DEV)
            st, stats = s.solve(torch.from_numpy(bh).to(DEV), x,
                                P.solve_opts(tol=1e-12, max_iter=300, guess=P.GUESS_ZERO, precond=precond))
            assert st == 0 and stats[0]["true_rel_res"] <= 1e-12
    finally:
        s.close()


@pytest.mark.parametrize("precond", [0, 1])
def test_forced_breakdown_restarts_and_converges(gpu, precond):
    import paper_2512_21697_amd as P
    w = synthetic.config1(driven=True)
    op = w.op
    nr = op.nr
    n = op.n_unknowns
    rng = np.random.default_rng(6)
    b = np.zeros(n, dtype=np.complex128)
    b[:2 * nr] = rng.standard_normal(2 * nr) + 1j * rng.standard_normal(2 * nr)       # channel 0
    shadow = np.zeros(n, dtype=np.complex128)
    shadow[2 * nr:4 * nr] = rng.standard_normal(2 * nr) + 1j * rng.standard_normal(2 * nr)  # channel 1
    assert np.vdot(shadow, b) == 0
    f = _fields(w)
    s = P.Solver(op, 1)
    try:
        s.set_dt(w.dt)
        s.set_field(f)
        sh = torch.from_numpy(shadow).to(DEV)
        s.set_shadow(sh)
        x = torch.zeros(n, dtype=torch.complex128, device=DEV)
        st, stats = s.solve(torch.from_numpy(b).to(DEV), x,
                            P.solve_opts(tol=1e-12, max_iter=300, guess=P.GUESS_ZERO, precond=precond))
        s.set_shadow(None)
        got = x.cpu().numpy()
    finally:
        s.close()
    print(f"precond={precond}: status {st}, {stats[0]}", flush=True)
    assert st == 0 and stats[0]["restarts"] >= 1
    A, _ = step_matrices(Assembled(op), f[0], w.dt)
    Ad = A.toarray()
    ref = np.linalg.solve(Ad, b)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-10, err
    # the oracle takes the same branch on the same shadow
    xo, so = bicgstab(A, b, None, tol=1e-12, rhat0=shadow)
    assert so.converged and so.restarts >= 1


@pytest.mark.parametrize("case", ["c1_prev", "c1_zero", "h_small_prec"])
def test_chunked_resume_is_bitwise(gpu, case):
    import paper_2512_21697_amd as P
    if case.startswith("c1"):
        w = synthetic.config1(driven=True)
        precond = 0
        guess = P.GUESS_PREV if case == "c1_prev" else P.GUESS_ZERO
    else:
        w = dkb.config2(nr=300, r_max=60.0, lmax=3, driven=True)
        precond = 1
        guess = P.GUESS_PREV
    k = 3
    opts = P.solve_opts(tol=1e-12, max_iter=300, guess=guess, precond=precond)
    s = P.Solver(w.op, 1)
    try:
        s.set_dt(w.dt)
        s.set_pulses(w.pulses)
        ns = np.array([100], dtype=np.int32)
        one = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        st1 = torch.zeros(2 * k * 40, dtype=torch.uint8, device=DEV)
        s.run_batched(one, w.t0, 0, 2 * k, ns, opts, st1)
        two = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        st2 = torch.zeros(2 * k * 40, dtype=torch.uint8, device=DEV)
        s.run_batched(two, w.t0, 0, k, ns, opts, st2[:k * 40])
        saved = two.cpu().numpy().copy()   # the checkpoint
        two = torch.from_numpy(saved).to(DEV)
        s.run_batched(two, w.t0, k, k, ns, opts, st2[k * 40:])
        torch.cuda.synchronize()
        a1 = np.frombuffer(st1.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
        a2 = np.frombuffer(st2.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
        g1, g2 = one.cpu().numpy(), two.cpu().numpy()
    finally:
        s.close()
    print(f"{case}: iters one launch {a1['iters'].tolist()}, two {a2['iters'].tolist()}; "
          f"max |diff| {np.max(np.abs(g1 - g2)):.3e}", flush=True)
    assert np.all(a1["status"] == 0) and np.all(a2["status"] == 0)
    assert np.array_equal(a1["iters"], a2["iters"])
    assert np.array_equal(g1, g2)
