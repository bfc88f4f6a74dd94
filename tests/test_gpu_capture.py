"""GPU: the solve path allocates nothing and synchronises nothing when no
result record is asked for, so a caller can capture it in a graph.

minres_solve (want_info=False; also on the plane schedule) and batch_solve of a batch without its own
graph (want_info=False, vectors already uploaded) are captured in a torch
CUDA graph; the graph is replayed several times with eager work and
synchronisations in between, and every replay is checked bitwise against
the eager solve.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def csl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_00488_amd as C
    C.load_library()
    return C


def _crand(shape, seed):
    g = np.random.default_rng(seed)
    return torch.from_numpy(g.standard_normal(shape) + 1j * g.standard_normal(shape)).cuda()


def _coef(shape, seed):
    return torch.from_numpy(np.random.default_rng(seed).uniform(0.5, 2.0, shape)).cuda()


@pytest.mark.parametrize("shape,fp32,threads", [((63, 63), False, 0), ((15, 31, 15), True, 0),
                                               # the plane phase
                                               ((15, 31, 15), True, 1024)])
def test_minres_solve_captured(csl, shape, fp32, threads):
    p = csl.Problem(_coef(shape, 1), 10.0, 40.0, pinv_fp32=fp32, dst="fft")
    if threads:
        p.set_schedule(0, 65536, threads)
    f = _crand(shape, 2)
    z_ref, info = csl.minres_solve(p, f)
    assert info["status"] == 0
    z = torch.zeros_like(f)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        csl.minres_solve(p, f, z, want_info=False)   # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        csl.minres_solve(p, f, z, want_info=False)
    f2 = _crand(shape, 3)
    for _ in range(3):
        z.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(z, z_ref)
        # the problem's own eager work between replays
        _, i2 = csl.minres_solve(p, f2)
        assert i2["status"] == 0
    del g


def test_batch_solve_captured(csl):
    shapes = [(31, 31), (63, 63), (15, 63)]
    probs = [csl.Problem(_coef(s, 10 + j), 5.0 + j, 25.0) for j, s in enumerate(shapes)]
    fs = [_crand(s, 20 + j) for j, s in enumerate(shapes)]
    zs = [torch.zeros_like(f) for f in fs]
    b = csl.Batch(probs, use_graph=False)
    ref, infos = b.solve(fs, [torch.empty_like(f) for f in fs])
    assert all(i["status"] == 0 for i in infos)
    _, _ = b.solve(fs, zs)            # uploads these vector pointers
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.solve(fs, zs, want_info=False)
    for _ in range(3):
        for z in zs:
            z.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(z, r) for z, r in zip(zs, ref))
        csl.minres_solve(probs[0], fs[0])   # eager work between replays
    del g
    b.close()
