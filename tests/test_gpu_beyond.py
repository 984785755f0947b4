"""The physical beyond-dipole operator (hydrogen, six time functions, H^theta_l for l <= 3) through the
GPU library vs the oracle (marked gpu).

* apply y = S x + i dt/2 H(t) x at random fields: 1e-13 relative (max norm) against the oracle's
  CSR assembly of the same description;
* preconditioned Crank-Nicolson steps from the ground state mid-pulse: a chained launch of four
  steps, each step compared with the oracle's step (BiCGSTAB to 1e-14 with the same block LU) fed the
  previous oracle state, 1e-10 relative after four steps.
Sizes: nr = 300 (two full radial tiles and a ragged one), 28 channels (|kappa| <= 4, |mu| <= 3/2),
96 coupling terms; and the benchmark's 60 channels (|kappa| <= 6, |mu| <= 5/2) at nr = 600.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.assemble import Assembled  # noqa: E402
from oracle.step import BlockPreconditioner, cn_step  # noqa: E402
from workloads import beyond  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


CASES = {"small": dict(nr=300, kappa_max=4, mu2_max=3, l_max=3),
         "bench": dict(nr=600, kappa_max=6, mu2_max=5, l_max=3)}


@pytest.mark.parametrize("size", ["small", "bench"])
def test_beyond_apply_matches_oracle(gpu, size):
    import paper_2512_21697_amd as P
    w = beyond.workload(**CASES[size])
    op = w.op
    rng = np.random.default_rng(8)
    f = rng.standard_normal(op.n_fields)
    x = rng.standard_normal(op.n_unknowns) + 1j * rng.standard_normal(op.n_unknowns)
    s = P.Solver(op, 1)
    try:
        s.set_field(f[None])
        xd = torch.from_numpy(x).to(DEV)
        y = torch.empty_like(xd)
        s.apply(xd, y, 1.0, 0.5j * w.dt)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
    finally:
        s.close()
    ref = Assembled(op).operator(f, 1.0, 0.5j * w.dt) @ x
    rel = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"{size}: {op.nang} channels, {len(op.terms)} terms, apply rel diff {rel:.2e}", flush=True)
    assert rel < 1e-13


@pytest.mark.parametrize("size", ["small", "bench"])
def test_beyond_steps_match_oracle(gpu, size):
    import paper_2512_21697_amd as P
    w = beyond.workload(**CASES[size])
    op = w.op
    n = 4
    s = P.Solver(op, 1)
    try:
        s.set_dt(w.dt)
        s.set_pulses(w.pulses)
        psi = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        st = torch.zeros(n * 40, dtype=torch.uint8, device=DEV)
        s.run_batched(psi, w.t0, 0, n, np.array([n], dtype=np.int32),
                      P.solve_opts(tol=1e-12, max_iter=300, guess=P.GUESS_PREV, precond=1), st)
        torch.cuda.synchronize()
        stats = np.frombuffer(st.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE)
        got = psi.cpu().numpy().reshape(op.nang, 2, op.nr)
    finally:
        s.close()
    assert np.all(stats["status"] == 0) and stats["true_rel_res"].max() <= 1e-12
    asm = Assembled(op)
    M = BlockPreconditioner(asm, w.dt)
    ref = w.psi0[0]
    for k in range(n):
        ref, rst = cn_step(asm, w.pulses[0], w.t0 + k * w.dt, w.dt, ref, guess="prev", tol=1e-14, precond=M)
        assert rst.converged
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    # the pulse moves probability out of the initial channel
    moved = 1.0 - np.linalg.norm(ref[beyond.channels(CASES[size]["kappa_max"], CASES[size]["mu2_max"]).index((-1, 1))]) ** 2
    print(f"{size}: iters {stats['iters'].tolist()}, rel err {err:.2e}, weight outside the initial channel {moved:.2e}",
          flush=True)
    assert err < 1e-10
