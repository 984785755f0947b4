"""Field table and device pulse evaluation through the C ABI (marked gpu).

* The device's pulse values (tdde_eval_pulses) agree with the oracle's pulse at the step midpoints
  (same formula, different sine implementations: 1e-14 relative to the amplitude).
* Steps driven by a field table tabulated from the device's own pulse values equal the
  pulse-driven steps bit for bit (one launch of several chained steps, and single steps).
* Steps driven by a table that is not a sin^2 pulse (the pulse values times a ramp) match the
  oracle's steps with the same explicit field values (1e-10 per step).
* A launch whose steps run past the table is rejected before any launch.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.assemble import Assembled  # noqa: E402
from oracle.bicgstab import bicgstab  # noqa: E402
from oracle.fields import field_values, midpoint_time  # noqa: E402
from oracle.step import step_matrices  # noqa: E402
from workloads import synthetic  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


@pytest.mark.parametrize("case", ["c1d", "tiny"])
def test_device_pulses_match_oracle(gpu, case):
    import paper_2512_21697_amd as P
    w = synthetic.config1(driven=True) if case == "c1d" else synthetic.tiny()
    s = P.Solver(w.op, w.batch)
    try:
        s.set_dt(w.dt)
        s.set_pulses(w.pulses)
        n = 40
        got = s.eval_pulses(w.t0, 3, n)
    finally:
        s.close()
    for b in range(w.batch):
        for k in range(n):
            t = midpoint_time(w.t0 + (3 + k) * w.dt, w.dt)
            ref = np.array(field_values(w.pulses[b], t))
            amp = np.array([p.amp for p in w.pulses[b]])
            assert np.all(np.abs(got[b, k] - ref) <= 1e-14 * amp), (b, k, got[b, k], ref)


@pytest.mark.parametrize("precond", [0, 1])
def test_table_steps_equal_pulse_steps_bitwise(gpu, precond):
    import paper_2512_21697_amd as P
    w = synthetic.config1(driven=True)
    n = 6
    opts = P.solve_opts(tol=1e-12, max_iter=300, guess=P.GUESS_PREV, precond=precond)
    s = P.Solver(w.op, 1)
    try:
        s.set_dt(w.dt)
        s.set_pulses(w.pulses)
        tab = s.eval_pulses(w.t0, 0, n)
        ns = np.array([n], dtype=np.int32)
        a = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        s.run_batched(a, w.t0, 0, n, ns, opts)
        s.set_field_table(tab)
        b = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        s.run_batched(b, w.t0, 0, n, ns, opts)
        # single steps through tdde_step take row 0
        s.set_field_table(tab[:, :1])
        c = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        s.step(c, w.t0, opts)
        s.set_pulses(w.pulses)
        d = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        s.step(d, w.t0, opts)
        torch.cuda.synchronize()
    finally:
        s.close()
    assert torch.equal(a, b)
    assert torch.equal(c, d)


def test_table_not_a_pulse_matches_oracle(gpu):
    import paper_2512_21697_amd as P
    w = synthetic.tiny()
    op = w.op
    n = 4
    rows = np.array([[field_values(w.pulses[0], midpoint_time(w.t0 + k * w.dt, w.dt)) for k in range(n)]])
    ramp = np.linspace(0.5, 2.0, n)[None, :, None] * np.array([1.0, -0.7])[None, None, :]
    tab = rows * ramp + 0.01
    opts = P.solve_opts(tol=1e-13, max_iter=400, guess=P.GUESS_PREV, precond=1)
    s = P.Solver(op, 1)
    try:
        s.set_dt(w.dt)
        s.set_field_table(tab)
        psi = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
        st = torch.zeros(n * 40, dtype=torch.uint8, device=DEV)
        s.run_batched(psi, w.t0, 0, n, np.array([n], dtype=np.int32), opts, st)
        with pytest.raises(P.TddeError, match="field table"):
            s.run_batched(psi, w.t0, n - 1, 2, np.array([n + 1], dtype=np.int32), opts)
        got = psi.cpu().numpy().reshape(op.nang, 2, op.nr)
    finally:
        s.close()
    asm = Assembled(op)
    ref = w.psi0[0]
    for k in range(n):
        A, B = step_matrices(asm, tab[0, k], w.dt)
        ref = np.linalg.solve(A.toarray(), B @ ref.ravel()).reshape(ref.shape)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-10, err
