"""The allocation-free solve against the context-workspace solve (marked gpu).

tdde_solve_static runs the solver with its scratch in the library's static device array instead of
the context's workspace; everything else (kernels, launch shape, reduction order) is the same, so
its results must equal tdde_solve's bit for bit. Two calls in a row on one GPU, the second on a
smaller problem (the array keeps the first call's contents), then a third on a different operator;
a solve larger than the array is rejected before any launch.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.fields import field_values, midpoint_time  # noqa: E402
from workloads import dkb, synthetic  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


def _solve_both(P, w, batch, precond, guess, seed):
    op = w.op
    s = P.Solver(op, batch)
    try:
        s.set_dt(w.dt)
        f = np.array([field_values(w.pulses[0], midpoint_time(w.t0, w.dt))] * batch)
        s.set_field(f)
        rng = np.random.default_rng(seed)
        shape = (batch * op.n_unknowns,)
        b = torch.from_numpy(rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).to(DEV)
        x0 = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        if guess == P.GUESS_ZERO:
            x0[:] = 0
        opts = P.solve_opts(tol=1e-12, max_iter=400, guess=guess, precond=precond)
        x_ref = torch.from_numpy(x0.copy()).to(DEV)
        st_ref, stats_ref = s.solve(b, x_ref, opts)
        x_st = torch.from_numpy(x0.copy()).to(DEV)
        st, stats = s.solve(b, x_st, opts, static=True)
        torch.cuda.synchronize()
        got, ref = x_st.cpu().numpy(), x_ref.cpu().numpy()
        print(f"N={op.n_unknowns} batch={batch} precond={precond}: status {st}/{st_ref}, iters "
              f"{[d['iters'] for d in stats]} / {[d['iters'] for d in stats_ref]}", flush=True)
        assert st == st_ref == 0
        assert np.array_equal(got, ref)
        assert stats == stats_ref
    finally:
        s.close()


def test_static_solve_matches_workspace_solve_two_calls(gpu):
    import paper_2512_21697_amd as P
    # first call: hydrogen operator, N = 164000, preconditioned, given guess
    _solve_both(P, dkb.config2(driven=True), 1, 1, P.GUESS_GIVEN, 1)
    # second call, smaller: N = 3200 block-banded operator, two instances, unpreconditioned, zero guess
    _solve_both(P, synthetic.config1(driven=True), 2, 0, P.GUESS_ZERO, 2)
    # third: tiny general operator (S != I, P-Q coupling, several terms), preconditioned
    _solve_both(P, synthetic.tiny(s_identity=False), 1, 1, P.GUESS_GIVEN, 3)


def test_static_solve_rejects_oversize(gpu):
    import paper_2512_21697_amd as P
    w = synthetic.config1()
    batch = 160  # 160 * 3200 complex unknowns: 10 vectors of 8.2 MB exceed the 64 MiB array
    s = P.Solver(w.op, batch)
    try:
        s.set_dt(w.dt)
        s.set_field(np.zeros((batch, w.op.n_fields)))
        n = batch * w.op.n_unknowns
        b = torch.ones(n, dtype=torch.complex128, device=DEV)
        x = torch.zeros_like(b)
        with pytest.raises(P.TddeError, match="static"):
            s.solve(b, x, P.solve_opts(tol=1e-12, guess=P.GUESS_ZERO), static=True)
        # the context stays usable: the workspace solve runs
        st, _ = s.solve(b, x, P.solve_opts(tol=1e-12, guess=P.GUESS_ZERO, max_iter=400))
        assert st == 0
    finally:
        s.close()
