"""Graph mode of the persistent solver (tdde_set_graph), marked gpu.

The launch sequence of a chunk (two fill kernels and the cooperative solver launch) is captured once
on a non-default stream and replayed with each chunk's arguments. Every replay is compared bit for
bit with the same chunk run by direct launches, with eager work and synchronisations on the stream
between the replays (fill nodes and argument updates must not carry state from one replay to the
next). Cases: the small block-banded operator (unpreconditioned variant, chained chunks of five
steps) and the small hydrogen operator (preconditioned variant), and a switch back to direct mode.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import dkb, synthetic  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return True


def _chunks(P, s, w, opts, n_chunks, k, graph):
    s.set_graph(graph)
    psi = torch.from_numpy(w.psi0.reshape(-1)).to(DEV)
    ns = np.array([n_chunks * k], dtype=np.int32)
    states, stats = [], []
    junk = torch.zeros(1 << 20, dtype=torch.float64, device=DEV)
    for c in range(n_chunks):
        st = torch.zeros(k * 40, dtype=torch.uint8, device=DEV)
        s.run_batched(psi, w.t0, c * k, k, ns, opts, st)
        # eager work on the stream between replays
        junk.add_(1.0).mul_(0.5)
        s.stream.synchronize()
        states.append(psi.clone())
        stats.append(np.frombuffer(st.cpu().numpy().tobytes(), dtype=P.STATS_DTYPE).copy())
    return states, stats


@pytest.mark.parametrize("case", ["c1d", "h_small"])
def test_graph_replays_equal_direct_launches(gpu, case):
    import paper_2512_21697_amd as P
    if case == "c1d":
        w, precond = synthetic.config1(driven=True), 0
    else:
        w, precond = dkb.config2(nr=300, r_max=60.0, lmax=3, driven=True), 1
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = P.Solver(w.op, 1, stream=stream)
        try:
            s.set_dt(w.dt)
            s.set_pulses(w.pulses)
            opts = P.solve_opts(tol=1e-12, max_iter=300, guess=P.GUESS_PREV, precond=precond)
            direct, dstats = _chunks(P, s, w, opts, 4, 5, False)
            graph, gstats = _chunks(P, s, w, opts, 4, 5, True)
            again, _ = _chunks(P, s, w, opts, 2, 5, False)
        finally:
            s.close()
    for c in range(4):
        assert np.all(gstats[c]["status"] == 0)
        assert np.array_equal(gstats[c]["iters"], dstats[c]["iters"])
        assert torch.equal(graph[c], direct[c]), c
    assert torch.equal(again[1], direct[1])
