"""Pins of the FP64 oracle against what the paper and the mathematics fix (no GPU).

Each test names the passage it checks. The oracle is compared with things that are
not itself: dense LAPACK solves, closed-form phases of the Cayley step, conservation
laws, the Dirac-Coulomb spectrum, the velocity-form dipole sum rule, brute force on
tiny inputs. A few tests plant a plausible mistake in the oracle and check that a pin
catches it.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fields
from oracle.assemble import Assembled
from oracle.bicgstab import bicgstab
from oracle.rows import apply_rows
from oracle.step import BlockPreconditioner, cn_step, propagate
from workloads import dkb, synthetic
from workloads.desc import Pulse, replace

C = 137.036
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_energies():
    out = {}
    for line in open(os.path.join(GOLD, "dirac_coulomb_hydrogen.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, k, lab, e = line.split()
        out[(int(n), int(k))] = float(e)
    return out


@pytest.fixture(scope="module")
def tiny_w():
    return synthetic.tiny(s_identity=False)


@pytest.fixture(scope="module")
def small_h():
    """Hydrogen on a short grid (nr=300, r_max=60, l <= 3): fast enough for dense checks."""
    op, basis, th = dkb.hydrogen_operator(nr=300, r_max=60.0, lmax=3)
    return op


# ---------------------------------------------------------------- assembly (eq. fullH)

@pytest.mark.parametrize("s_identity", [True, False])
def test_csr_assembly_equals_elementwise_definition(s_identity):
    """eq. fullH: the kron/block-diag CSR assembly equals the entry-by-entry definition."""
    w = synthetic.tiny(s_identity=s_identity)
    asm = Assembled(w.op)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((w.op.nang, 2, w.op.nr)) + 1j * rng.standard_normal((w.op.nang, 2, w.op.nr))
    f = [0.7, -1.3]
    a_s, a_h = complex(1.0, 0.2), complex(-0.1, 0.4)
    y = asm.operator(f, a_s, a_h) @ x.ravel()
    rows = np.arange(w.op.n_unknowns)
    y2 = apply_rows(w.op, f, a_s, a_h, x, rows)
    assert np.max(np.abs(y - y2)) <= 1e-13 * np.max(np.abs(y))


def test_hamiltonian_hermitian_and_overlap_spd(tiny_w, small_h):
    """H0 and every coupling combination are Hermitian (Sec. 2.1); S is SPD (B-spline Gram)."""
    for op in (tiny_w.op, small_h, synthetic.config1().op):
        asm = Assembled(op)
        H = asm.hamiltonian([0.9, -0.4][: op.n_fields]).toarray()
        assert np.max(np.abs(H - H.conj().T)) <= 1e-12 * np.max(np.abs(H))
        if op.s_poly.shape[0]:
            S = asm.S.toarray()
            assert np.allclose(S, S.conj().T, atol=0)
            assert np.linalg.eigvalsh(S).min() > 0


# ---------------------------------------------------------------- BiCGSTAB vs LAPACK

def test_bicgstab_matches_dense_lu_tiny(tiny_w):
    """BiCGSTAB (van der Vorst 1992) reaches the LAPACK solution of the step system."""
    asm = Assembled(tiny_w.op)
    f = fields.field_values(tiny_w.pulses[0], 3.1)
    A = asm.operator(f, 1.0, 0.5j * 0.05)
    rng = np.random.default_rng(3)
    b = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    x, st = bicgstab(A, b, None, tol=1e-13, max_iter=500)
    xd = np.linalg.solve(A.toarray(), b)
    assert st.converged
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-11


def test_bicgstab_c1_step_matches_dense_lu():
    """Config 1 (N = 3200): every one of 3 steps agrees with the dense LU solve to 1e-11."""
    w = synthetic.config1(driven=True)
    asm = Assembled(w.op)
    psi = w.psi0[0]
    for n in range(3):
        t = w.t0 + n * w.dt
        x, st = cn_step(asm, w.pulses[0], t, w.dt, psi, guess="zero")
        xd, _ = cn_step(asm, w.pulses[0], t, w.dt, psi, solver="dense")
        assert st.converged and st.true_rel_res <= 1e-12
        # forward error bound: cond(A) * tol, cond(A) = 18.8 for this operator
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 2.5e-11
        psi = xd


def test_preconditioned_bicgstab_hydrogen(small_h):
    """With M = S + i dt/2 H0 (eq. matrixM) BiCGSTAB converges in a few iterations and matches LU."""
    w = dkb.config2(nr=300, r_max=60.0, lmax=3, driven=True)
    asm = Assembled(w.op)
    M = BlockPreconditioner(asm, w.dt)
    x, st = cn_step(asm, w.pulses[0], w.t0, w.dt, w.psi0[0], guess="zero", precond=M)
    xd, _ = cn_step(asm, w.pulses[0], w.t0, w.dt, w.psi0[0], solver="dense")
    assert st.converged and st.iters <= 6
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-11


# ---------------------------------------------------------------- Cayley step invariants (eq. solPsi)

def _c1_free():
    w = synthetic.config1()
    return replace(w, pulses=[[Pulse(0.0, 20.0, 0.057, 0.0, True)]])


def test_field_free_eigenstate_phase_closed_form():
    """H0 v = E v  =>  one step multiplies v by z = (1 - i E dt/2) / (1 + i E dt/2) (eq. solPsi)."""
    w = _c1_free()
    op = w.op
    asm = Assembled(op)
    H0 = asm.H0.toarray()
    nblk = 2 * op.nr
    for j, s, which in [(0, 0, 0), (3, 1, 5), (7, 0, 199)]:
        off = j * nblk + s * op.nr
        E, V = np.linalg.eigh(H0[off:off + op.nr, off:off + op.nr])
        psi = np.zeros(op.n_unknowns, dtype=complex)
        psi[off:off + op.nr] = V[:, which]
        x, st = cn_step(asm, w.pulses[0], 0.0, w.dt, psi.reshape(op.nang, 2, op.nr), guess="zero")
        z = (1 - 0.5j * E[which] * w.dt) / (1 + 0.5j * E[which] * w.dt)
        assert np.linalg.norm(x.ravel() - z * psi) < 1e-11
    # small-component phase at E ~ -2c^2 is about 3.035 rad per step
    assert abs(abs(np.angle((1 + 0.5j * 2 * C * C * 1e-3) / (1 - 0.5j * 2 * C * C * 1e-3))) - 3.0352) < 1e-3


def test_hydrogen_ground_state_is_stationary():
    """Field-free: the 1s state only acquires the phase z(E_1s) per step (generalised eigenproblem)."""
    w = dkb.config2(nr=300, r_max=60.0, lmax=3)
    asm = Assembled(w.op)
    M = BlockPreconditioner(asm, w.dt)
    free = [[Pulse(0.0, 1.0, 1.0, 0.0, True)]]
    x, st = cn_step(asm, free[0], 0.0, w.dt, w.psi0[0], guess="zero", precond=M)
    E = w.meta["E_ground"]
    z = (1 - 0.5j * E * w.dt) / (1 + 0.5j * E * w.dt)
    assert np.linalg.norm(x - z * w.psi0[0]) < 1e-11
    assert abs(np.angle(z) - 1.000013e-4) < 1e-9  # -E dt for E = -0.50000666


def test_norm_conservation_driven():
    """Hermitian H: psi^H S psi is conserved by the Cayley step for any field."""
    w = synthetic.config1(driven=True)
    w = replace(w, pulses=[[Pulse(5.0, 20.0, 0.057, 0.3, True)]])
    asm = Assembled(w.op)
    psi, stats = propagate(asm, w.pulses[0], w.t0, w.dt, w.psi0[0], 4, solver="splu")
    assert abs(np.linalg.norm(psi) - 1.0) < 1e-13


def test_hydrogen_s_norm_conservation():
    w = dkb.config2(nr=300, r_max=60.0, lmax=3, driven=True, E0=5.0)
    asm = Assembled(w.op)
    psi, _ = propagate(asm, w.pulses[0], w.t0, w.dt, w.psi0[0], 5, solver="splu")
    v = psi.ravel()
    assert abs(np.vdot(v, asm.S @ v).real - 1.0) < 1e-12


def test_time_reversal():
    """U(-dt) U(dt) = I at a fixed midpoint time (the Cayley transform is exactly reversible)."""
    w = synthetic.tiny()
    asm = Assembled(w.op)
    f = fields.field_values(w.pulses[0], 3.0)
    from oracle.step import step_matrices
    A, B = step_matrices(asm, f, w.dt)
    psi = w.psi0[0].ravel()
    fwd = np.linalg.solve(A.toarray(), B @ psi)
    A2, B2 = step_matrices(asm, f, -w.dt)
    back = np.linalg.solve(A2.toarray(), B2 @ fwd)
    assert np.linalg.norm(back - psi) < 1e-12


def _order_errors(midpoint):
    """Errors after t = 0.4 of a strongly driven tiny operator at dt = T/16, T/32, T/64 vs T/512."""
    w = synthetic.tiny()
    asm = Assembled(w.op)
    pulses = [Pulse(3.0, 1e9, 4.0, 0.3, False), Pulse(2.0, 1e9, 3.0, 1.0, False)]
    T = 0.4
    import oracle.step as ostep
    orig = ostep.midpoint_time
    if not midpoint:  # planted mistake: evaluate H at the end of the step
        ostep.midpoint_time = lambda t, dt: t + dt
    try:
        def run(n):
            psi, _ = propagate(asm, pulses, 3.0, T / n, w.psi0[0], n, solver="dense")
            return psi
        ref = run(512)
        errs = [np.linalg.norm(run(n) - ref) for n in (16, 32, 64)]
    finally:
        ostep.midpoint_time = orig
    return errs


def test_second_order_in_dt_with_midpoint_rule():
    """Midpoint rule (Sec. 2.4) gives O(dt^2): halving dt divides the error by about 4."""
    e = _order_errors(True)
    assert 3.7 < e[0] / e[1] < 4.3 and 3.7 < e[1] / e[2] < 4.3


def test_planted_endpoint_time_breaks_order():
    """Planted mistake: H(t + dt) instead of the midpoint drops the order to 1 (ratio about 2)."""
    e = _order_errors(False)
    assert e[0] / e[1] < 2.5 and e[1] / e[2] < 2.5


# ---------------------------------------------------------------- DKB hydrogen physics

def test_dirac_coulomb_energies(small_h):
    """DKB B-spline H0 reproduces the closed-form Dirac-Coulomb levels (Sec. 2.2-2.3)."""
    gold = _golden_energies()
    op = small_h
    for kap in (-1, 1, -2, 2, -3):
        ns = sorted(n for (n, k) in gold if k == kap)
        w, _ = dkb.bound_states(op.h_poly, op.s_poly, float(kap), op.nr, op.hb, n_states=len(ns))
        for n, e in zip(ns, w):
            assert abs(e - gold[(n, kap)]) < 1e-9, (n, kap, e, gold[(n, kap)])


def test_no_spurious_states(small_h):
    """Dual kinetic balance (eq. dualkinetic): the lowest level above -c^2 of every kappa block is the
    physical n = l+1 state; no spurious level lies below it. 2s1/2 and 2p1/2 stay degenerate."""
    gold = _golden_energies()
    op = small_h
    lowest = {-1: (1, -1), 1: (2, 1), -2: (2, -2), 2: (3, 2), -3: (3, -3)}
    for kap, key in lowest.items():
        w, _ = dkb.bound_states(op.h_poly, op.s_poly, float(kap), op.nr, op.hb, n_states=1)
        assert abs(w[0] - gold[key]) < 1e-9
    e2s = dkb.bound_states(op.h_poly, op.s_poly, -1.0, op.nr, op.hb, n_states=2)[0][1]
    e2p = dkb.bound_states(op.h_poly, op.s_poly, 1.0, op.nr, op.hb, n_states=1)[0][0]
    assert abs(e2s - e2p) < 1e-9


def _racah_cg(j1, m1, j2, m2, J, M):
    """Clebsch-Gordan coefficient from the Racah formula (independent of the spin-1/2 closed forms)."""
    if abs(m1 + m2 - M) > 1e-12:
        return 0.0
    f = math.factorial

    def fi(x):
        return f(int(round(x)))
    pre = math.sqrt((2 * J + 1) * fi(J + j1 - j2) * fi(J - j1 + j2) * fi(j1 + j2 - J) / fi(j1 + j2 + J + 1))
    pre *= math.sqrt(fi(J + M) * fi(J - M) * fi(j1 - m1) * fi(j1 + m1) * fi(j2 - m2) * fi(j2 + m2))
    s = 0.0
    for k in range(0, 100):
        args = [k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k]
        if any(a < -1e-9 for a in args):
            continue
        if k > j1 + j2 + J + 5:
            break
        s += (-1) ** k / np.prod([fi(a) for a in args])
    return pre * s


def test_clebsch_gordan_closed_forms_match_racah():
    for l in range(0, 5):
        for j2 in (2 * l - 1, 2 * l + 1):
            if j2 < 0:
                continue
            for mu2 in range(-j2, j2 + 1, 2):
                c1, c2 = dkb.clebsch_spin_half(l, j2, mu2)
                mu = mu2 / 2
                r1 = _racah_cg(l, mu - 0.5, 0.5, 0.5, j2 / 2, mu) if abs(mu - 0.5) <= l else 0.0
                r2 = _racah_cg(l, mu + 0.5, 0.5, -0.5, j2 / 2, mu) if abs(mu + 0.5) <= l else 0.0
                assert abs(c1 - r1) < 1e-12 and abs(c2 - r2) < 1e-12


def test_velocity_dipole_sum_rule():
    """sum_j |<1s1/2| c alpha_z |2p_j>|^2 -> |<1s|p_z|2p0>|^2 = ((3/8) 128 sqrt2/243)^2 (nonrelativistic
    limit; O(1/c^2) corrections). Pins the dipole angular factors and the DKB radial coupling."""
    op, basis, th = dkb.hydrogen_operator(nr=300, r_max=60.0, lmax=2)
    asm = Assembled(op)
    V = asm.hamiltonian([1.0]) - asm.H0  # = -c alpha_z  (field value 1)
    ks = list(op.kappa)

    def state(kap, idx):
        w, v = dkb.bound_states(op.h_poly, op.s_poly, float(kap), op.nr, op.hb, n_states=idx + 1)
        vec = np.zeros(op.n_unknowns, dtype=complex)
        j = ks.index(kap)
        vv = v[:, idx]
        S = dkb.sparse_block(op.s_poly, float(kap), op.nr, op.hb)
        vv = vv / math.sqrt(vv @ (S @ vv))
        vec[j * 2 * op.nr:(j + 1) * 2 * op.nr] = vv
        return vec
    g1s = state(-1, 0)
    tot = 0.0
    for kap in (1, -2):
        p = state(kap, 0)
        tot += abs(np.vdot(g1s, V @ p)) ** 2
    nonrel = ((3 / 8) * 128 * math.sqrt(2) / 243) ** 2
    assert abs(tot / nonrel - 1) < 1e-3
    # dipole selection rule: 1s does not couple to 3d (kappa = 2)
    assert abs(np.vdot(g1s, V @ state(2, 0))) < 1e-14


def test_planted_transposed_coupling_breaks_hermiticity(tiny_w):
    """Planted mistake: the adjoint partner of a coupling term built without transposing R."""
    import copy
    op = copy.deepcopy(tiny_w.op)
    op.terms[1].r_band = op.terms[0].r_band.copy()
    H = Assembled(op).hamiltonian([1.0, 1.0]).toarray()
    assert np.max(np.abs(H - H.conj().T)) > 1e-3


def test_field_functions_closed_form():
    """sin^2 envelope pulse (eq. ndpPot, dipole limit): zero outside (0, T), symmetric envelope."""
    p = Pulse(2.0, 10.0, 1.3, 0.4, True)
    assert fields.pulse_value(p, -0.1) == 0.0 and fields.pulse_value(p, 10.0) == 0.0
    t = 3.7
    assert abs(fields.pulse_value(p, t) - 2.0 * math.sin(math.pi * t / 10) ** 2 * math.sin(1.3 * t + 0.4)) < 1e-15
    assert fields.midpoint_time(1.0, 0.5) == 1.25
