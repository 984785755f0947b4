"""Photoelectron spectrum (eq. dPdE) and spectral error on the GPU vs the oracle (marked gpu).

The library receives the field-free eigenpairs of every kappa block as pre-computed input (the
workload generator's dense diagonalisation); the oracle diagonalises the same blocks itself. The
density at the grid points (sum over channels of interpolated |v_n^T S psi|^2 / dE_n) must agree to
1e-10 relative to its maximum (two summation orders of the same formula), the error integral to
1e-12 relative. Sizes: a small box (nr = 200) and the benchmark's (nr = 600, l <= 10, 21 channels,
848 levels), two instances with different states each.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import spectrum as ospec  # noqa: E402
from workloads import spectrum as wspec  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


def _states(w, inp, seed):
    """Instance 0: a seeded random state; instance 1: the ground state plus eigen-components of the
    window with seeded amplitudes in the first channels."""
    op = w.op
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((op.nang, 2, op.nr)) + 1j * rng.standard_normal((op.nang, 2, op.nr))
    b = w.psi0[0].copy()
    lev0 = np.concatenate([[0], np.cumsum(inp.n_lev)])
    for j in range(min(3, op.nang)):
        blk = inp.blk_of[j]
        V = inp.vecs[lev0[blk]:lev0[blk + 1]]
        amp = rng.standard_normal(V.shape[0]) * 0.05
        b[j] += (amp @ V).reshape(2, op.nr)
    return np.stack([a, b])


@pytest.mark.parametrize("size", ["small", "bench"])
def test_spectrum_matches_oracle(gpu, size):
    import paper_2512_21697_amd as P
    if size == "small":
        w, inp = wspec.hydrogen_case(nr=200, r_max=30.0, lmax=3, e_lo=0.05, e_hi=2.0, n_grid=97)
    else:
        w, inp = wspec.hydrogen_case()
    op = w.op
    psi = _states(w, inp, 4)
    s = P.Solver(op, 2)
    try:
        s.spectrum_setup(inp.blk_of, inp.n_lev, inp.levels, inp.edges, inp.vecs, inp.grid)
        x = torch.from_numpy(psi.reshape(-1)).to(DEV)
        out = torch.zeros(2 * inp.grid.size, dtype=torch.float64, device=DEV)
        s.spectrum(x, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(2, -1)
        err_gpu = s.spectrum_error(out[:inp.grid.size].repeat(2).contiguous(), out)
    finally:
        s.close()
    ref = np.stack([ospec.spectrum(op, psi[b], inp.grid, inp.e_lo, inp.e_hi) for b in range(2)])
    for b in range(2):
        rel = np.max(np.abs(got[b] - ref[b])) / np.max(np.abs(ref[b]))
        print(f"{size} instance {b}: max density {np.max(ref[b]):.3e}, rel diff {rel:.2e}", flush=True)
        assert rel < 1e-10
    e_ref = ospec.spectral_error(ref[0], ref[1], inp.grid)
    assert err_gpu[0] == 0.0
    assert abs(err_gpu[1] - e_ref) <= 1e-10 * e_ref


def test_spectrum_setup_rejects_bad_inputs(gpu):
    import paper_2512_21697_amd as P
    w, inp = wspec.hydrogen_case(nr=200, r_max=30.0, lmax=1, e_lo=0.05, e_hi=2.0, n_grid=31)
    s = P.Solver(w.op, 1)
    try:
        bad_edges = inp.edges.copy()
        bad_edges[0, 0] = inp.levels[0] + 1.0  # the edge below above the first level
        with pytest.raises(P.TddeError, match="ascend"):
            s.spectrum_setup(inp.blk_of, inp.n_lev, inp.levels, bad_edges, inp.vecs, inp.grid)
        s.spectrum_setup(inp.blk_of, inp.n_lev, inp.levels, inp.edges, inp.vecs, inp.grid)
    finally:
        s.close()
